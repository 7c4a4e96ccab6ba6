// Internal declarations shared by the library's translation units (not part of the ABI).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <string>

#include "../../include/dmts.h"

namespace dmts {

// ------------------------------------------------------------------ error handling
void set_error(const char* fmt, ...);

#define DMTS_HIP(call)                                                              \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) {                                                         \
      ::dmts::set_error("%s:%d: %s -> %s", __FILE__, __LINE__, #call,              \
                        hipGetErrorString(e_));                                     \
      return DMTS_E_HIP;                                                            \
    }                                                                               \
  } while (0)

#define DMTS_CHECK_LAUNCH() DMTS_HIP(hipGetLastError())

#define DMTS_REQUIRE(cond, code, ...)                                               \
  do {                                                                              \
    if (!(cond)) {                                                                  \
      ::dmts::set_error(__VA_ARGS__);                                               \
      return (code);                                                                \
    }                                                                               \
  } while (0)

// Device buffer that only grows; growing waits for the stream so that no enqueued
// kernel still reads the old allocation.
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
  dmts_status reserve(size_t need, hipStream_t s);
  void release();
  template <class T> T* as() const { return static_cast<T*>(ptr); }
};

constexpr int kWave = 64;

inline int ceil_div(int64_t a, int64_t b) { return static_cast<int>((a + b - 1) / b); }

// ------------------------------------------------------------------ neighbor list
constexpr int kNlistRowCap = 256;   // most neighbors one atom may have
constexpr int kSkinRowCap = 512;    // most neighbors within cutoff + skin (skin lists)
constexpr int kSmallPairCap = 64;   // most pairs one atom may have inside the fast cutoff
struct NList {
  int32_t max_atoms = 0;
  int64_t max_pairs = 0;
  int32_t row_align = 1;
  // built state
  int32_t n_atoms = 0;
  double box = 0.0;
  double cutoff = 0.0;
  // device arrays
  int32_t* offs = nullptr;   // [max_atoms + 1]
  int32_t* nbr = nullptr;    // [max_pairs]
  int32_t* rev = nullptr;    // [max_pairs]
  float4* geo = nullptr;     // [max_pairs] (dx, dy, dz, r) at the build positions
  int32_t* cnt = nullptr;    // [max_atoms] padded row lengths
  uint32_t* flags = nullptr; // [1]
  int64_t* scan_part = nullptr;  // per-tile totals of the offset scans
  int32_t* len = nullptr;    // [max_atoms] real row lengths
  int32_t* ell = nullptr;    // [max_atoms][kNlistRowCap] sorted rows before compaction
  // cell list scratch
  int32_t* cell_of = nullptr;    // [max_atoms]
  int32_t* cell_atoms = nullptr; // [max_atoms]
  DevBuf cell_buf;               // count, start, cursor
  int32_t n_cells_cap = 0;
};

// Skin of the integrator's reference lists (A): the rows are rebuilt once some atom has
// moved half of it.
constexpr double kDefaultSkin = 1.5;

// A list kept between the evaluations of an integrator: staging rows (ell, len of `rows`) at
// cutoff + skin, rebuilt only when an atom has moved at least skin/2 since the last rebuild,
// and filtered to the cutoff at the current positions at every evaluation.
struct SkinList {
  NList* rows = nullptr;       // row lengths (len), cells and overflow flag of the rows
  int32_t* ell = nullptr;      // [n][kSkinRowCap] sorted rows at cutoff + skin
  double* x_build = nullptr;   // [3][n] positions of the last rebuild
  uint32_t* gate = nullptr;    // [2]: rebuild requested, rebuilds so far
  double skin = 0.0;
  // parameters of the current rows; a change forces a rebuild
  double cutoff = -1.0, box = -1.0;
  int32_t n = -1;
};

// pos_copy (optional, float64 [3][n]): receives the positions the list is built from.
dmts_status build_neighbors(NList* nl, const double* pos, int32_t n, double box,
                            const int32_t* sys_offsets, int32_t n_sys, double cutoff,
                            hipStream_t s, double* pos_copy = nullptr);
// The list at a cutoff <= the parent's, from the parent's rows at the current positions.
dmts_status filter_neighbors(NList* child, const NList* parent, const double* pos,
                             double cutoff, hipStream_t s);
// The list at `cutoff` for the current positions through the skin list `sk` (which must
// hold max_atoms >= n); the same rows as build_neighbors.  Falls back to build_neighbors
// when the skin is 0, the box is open or cutoff + skin reaches half the box edge.
dmts_status refresh_neighbors(NList* nl, SkinList* sk, const double* pos, int32_t n,
                              double box, double cutoff, hipStream_t s,
                              double* pos_copy = nullptr);

// ------------------------------------------------------------------ models
// Tile shape of one evaluation (see nnp_tile_shape in the ABI header).
struct TileShape {
  int32_t nw = 4;     // two-interaction pair kernels: receivers (waves) per work-group, 2/4/8
  int32_t rt = 2;     // two-interaction atom chains: 16-atom tiles per work-group, 1/2
  int32_t keep = 1;   // one-interaction model: keep the first tiles' derivatives in registers
  int32_t grid = 0;   // persistent work-groups of the grid-stride kernels (0 = natural)
};

struct Model {
  nnp_model_desc desc{};
  int32_t K = 0, F = 0, D = 0, Z = 0;
  float rc = 0.f, sigma = 0.f, escale = 0.f;
  DevBuf params;     // float32 derived tensors
  // offsets (in floats) into params
  size_t o_WbT = 0, o_Td = 0, o_Ts = 0;                  // pair block, species tables
  size_t o_W1 = 0, o_W1T = 0, o_w2 = 0;                   // kind 0 readout
  // kind 1 per-atom layers, [out][in]: U1, U2 (forward), U1T, U2T (their transposes)
  size_t o_U1T = 0, o_U1 = 0, o_U2T = 0, o_U2 = 0;        // kind 1 updates
  size_t o_W2h = 0, o_W2hs = 0;                           // kind 1 h projections
  size_t o_WoT = 0, o_Wo = 0, o_wo = 0;                   // kind 1 readout
  // BF16 form: operands rounded to bfloat16 (round to nearest even)
  bool bf16 = false;
  DevBuf params16;    // bfloat16 tensors, [out][in] (input index contiguous), both forms
  size_t h_Wb1 = 0, h_Wb2 = 0;   // kind 1 radial blocks [F][K]: one term (BF16), three (FP32)
  size_t h_U1 = 0, h_W2h = 0, h_U2 = 0, h_Wo = 0;         // forward chain layers
  size_t h_WoT = 0, h_U2T = 0, h_W2hs = 0, h_U1T = 0;     // reverse chain layers
  size_t o_WbR = 0, o_W1R = 0, o_W1TR = 0;                // kind 0: bf16-valued floats
  const __bf16* p16(size_t off) const { return params16.as<__bf16>() + off; }
  // Launch shape: the default one and the autotuner's choice per size bucket (number of
  // bits of the atom count).  No shape changes a result bit: every receiver and every atom
  // row is computed by the same arithmetic whatever work-group holds it.
  TileShape shape;
  std::map<int, TileShape> tuned;
  static int size_bucket(int32_t n) {
    int b = 0;
    while (n > 0) { ++b; n >>= 1; }
    return b;
  }
  TileShape shape_for(int32_t n) const {
    const auto it = tuned.find(size_bucket(n));
    return it == tuned.end() ? shape : it->second;
  }
  // distinct for every model created in the process (never 0): a RESPA state compares it to
  // know whether its carried forces belong to this model
  uint64_t generation = 0;
  // workspace
  DevBuf atom_ws, pair_ws, sys_ws;
  const float* p(size_t off) const { return params.as<float>() + off; }
};

// Work-groups of a grid-stride launch: grid > 0 caps it; with 0, natural (one pass over the
// receivers) unless that takes between one and two rounds of the `resident` work-groups the
// GPU holds at once, which then run as one persistent round instead of a full and a partly
// filled one.
inline int launch_grid(int grid, int natural, int resident = 0) {
  if (grid > 0) return grid < natural ? grid : natural;
  return resident > 0 && natural > resident && natural < 2 * resident ? resident : natural;
}

// ------------------------------------------------------------------ integrator program
// Kicks and drifts between two force evaluations, applied per atom in the algorithm's
// order with exactly the arithmetic of separate steps:
//   kick:  v <- v + c / m * F      (c = tau * KAPPA; F = F_small, F_large or F_large - F_small)
//   drift: x <- x + c * v          (c = tau)
// A force evaluation that is followed by such a program applies it to atom i as soon as
// F_i is final (the epilogue of its last kernel); the positions it moves are read by the
// next evaluation only.
enum IntegOp : int { kKickSlow = 0, kKickFast = 1, kKickLarge = 2, kDrift = 3, kThermo = 4 };
constexpr int kMaxOps = 8;
constexpr uint32_t kFlagStale = 0x100u;   // internal: shared list no longer complete
constexpr uint32_t kFlagFdiff = 0x200u;   // internal: |F - F_small| above the threshold

// Kick: v += c F / m.  Drift: x += c v.  Thermo: the O-step of Algorithm 1, the exact
// Ornstein-Uhlenbeck update v <- e^(-gamma h) v + sd_z xi over the inner step h, xi the
// normals of the state's O-step number ctr.
struct Prog {
  int nops;
  int op[kMaxOps];
  double c[kMaxOps];
  uint64_t ctr[kMaxOps];
};

struct Epilogue {
  Prog prog;
  double* x;                 // [3][n] float64
  double* v;                 // [3][n] float64
  const float* FL;           // [3][n] reference-model forces
  const float* Fs;           // [3][n] fast-model forces
  const int32_t* species;
  double inv_mass[8];        // per species (kernel argument: no memory round trip)
  const double* inv_mass_atom;   // [n] per-atom 1/m (repartitioned masses) or null
  const double* x_ref;       // positions of the shared list's build (displacement check) or null
  double max_disp2;
  uint32_t* flags;
  // O-step: velocity decay e^(-gamma h), per-species noise scale
  // sqrt((1 - decay^2) k_B T KAPPA / m), Philox key words
  double o_decay;
  double o_sd[8];
  double o_var;              // (1 - decay^2) k_B T KAPPA: the noise scale is sqrt(o_var / m)
  uint32_t o_key[2];
  // force-difference monitor of the slow kicks: squared threshold (0: off) and the word
  // that keeps the largest breaching |F - F_small| (float bits, eV/A)
  double fdiff_thr2;
  uint32_t* fdiff_max;
  hipEvent_t wait = nullptr;   // host side: the launch that runs the program waits for it
};

// Philox4x32 with 10 rounds (Salmon, Moraes, Dror and Shaw, SC 2011): each round maps the
// counter (c0, c1, c2, c3) to (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1,
// lo(M0 c0)) with M0 = 0xD2511F53, M1 = 0xCD9E8D57; the key is bumped by the Weyl
// constants 0x9E3779B9, 0xBB67AE85 before every round after the first.
__device__ inline void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
    const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

// Standard normal deviate d (0, 1, 2 = x, y, z) of atom i at O-step k: the Philox words
// r of counter (i, k mod 2^32, k div 2^32, 0) and the key, u_j = (r_j + 1/2) 2^-32, and
// Box-Muller: x = sqrt(-2 ln u0) cos(2 pi u1), y = sqrt(-2 ln u0) sin(2 pi u1),
// z = sqrt(-2 ln u2) cos(2 pi u3).
__device__ inline double o_normal(int i, uint64_t k, const uint32_t (&key)[2], int d) {
  uint32_t c[4] = {(uint32_t)i, (uint32_t)k, (uint32_t)(k >> 32), 0u};
  philox4x32_10(c, key[0], key[1]);
  const double ua = ((double)(d < 2 ? c[0] : c[2]) + 0.5) * 0x1p-32;
  const double ub = ((double)(d < 2 ? c[1] : c[3]) + 0.5) * 0x1p-32;
  const double rad = sqrt(-2.0 * log(ua));
  const double a = 6.283185307179586 * ub;
  return rad * (d == 1 ? sin(a) : cos(a));
}

// 1 / m of species z, from the kernel argument by selection (no dynamic indexing).
inline bool has_thermo(const Prog& p) {
  for (int k = 0; k < p.nops; ++k)
    if (p.op[k] == kThermo) return true;
  return false;
}

__device__ inline double inv_mass_of(const Epilogue& E, int z) {
  double im = E.inv_mass[0];
#pragma unroll
  for (int k = 1; k < 8; ++k) im = z == k ? E.inv_mass[k] : im;
  return im;
}
// 1 / m of atom i (species z): the per-atom table when one is set, else the species table.
__device__ inline double inv_mass_at(const Epilogue& E, int i, int z) {
  return E.inv_mass_atom ? E.inv_mass_atom[i] : inv_mass_of(E, z);
}
__device__ inline double o_sd_of(const Epilogue& E, int z) {
  double sd = E.o_sd[0];
#pragma unroll
  for (int k = 1; k < 8; ++k) sd = z == k ? E.o_sd[k] : sd;
  return sd;
}

// Slow kick of an atom with |F - F_small|^2 = df2: a breach of the threshold raises the
// internal flag and records the size (rare, so the common path has no atomics).
__device__ inline void fdiff_check(const Epilogue& E, double df2) {
  if (E.fdiff_thr2 > 0.0 && df2 > E.fdiff_thr2) {
    atomicOr(E.flags, kFlagFdiff);
    atomicMax(E.fdiff_max, __float_as_uint((float)sqrt(df2)));
  }
}

// Every input is loaded before the program runs (one memory round trip instead of one
// per op that needs a new array); x and x_ref are written or checked only if it drifts.
__device__ inline void apply_atom(const Epilogue& E, int i, int n) {
  const int z = E.species[i];
  const double im_atom = E.inv_mass_atom ? E.inv_mass_atom[i] : 0.0;
  double vv[3], xx[3], xr[3];
  float fl[3], fs[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const size_t o = (size_t)d * n + i;
    vv[d] = E.v[o];
    xx[d] = E.x[o];
    xr[d] = E.x_ref ? E.x_ref[o] : 0.0;
    fl[d] = E.FL[o];
    fs[d] = E.Fs[o];
  }
  const double im = E.inv_mass_atom ? im_atom : inv_mass_of(E, z);
  bool moved = false;
  for (int k = 0; k < E.prog.nops; ++k) {
    const int op = E.prog.op[k];
    const double c = E.prog.c[k];
    if (op == kDrift) {
      moved = true;
#pragma unroll
      for (int d = 0; d < 3; ++d) xx[d] = xx[d] + c * vv[d];
    } else if (op == kThermo) {
      const double sd = E.inv_mass_atom ? sqrt(E.o_var * im) : o_sd_of(E, z);
      for (int d = 0; d < 3; ++d)
        vv[d] = E.o_decay * vv[d] + sd * o_normal(i, E.prog.ctr[k], E.o_key, d);
    } else {
      const double ci = c * im;
      double df2 = 0.0;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        double f;
        if (op == kKickSlow) f = (double)fl[d] - (double)fs[d];
        else if (op == kKickFast) f = (double)fs[d];
        else f = (double)fl[d];
        vv[d] = vv[d] + ci * f;
        df2 += f * f;
      }
      if (op == kKickSlow) fdiff_check(E, df2);
    }
  }
  bool bad = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    E.v[(size_t)d * n + i] = vv[d];
    bad |= !isfinite(vv[d]);
  }
  uint32_t f = 0;
  if (moved) {
    double d2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      E.x[(size_t)d * n + i] = xx[d];
      bad |= !isfinite(xx[d]);
      const double u = xx[d] - xr[d];
      d2 += u * u;
    }
    if (E.x_ref && !(d2 <= E.max_disp2)) f |= kFlagStale;
  }
  if (bad) f |= DMTS_FLAG_NONFINITE;
  if (f) atomicOr(E.flags, f);
}

// The same program for one coordinate d of atom i, spread over lanes 0..2 of a wave: the
// caller loads the coordinate's inputs early (prefetch) and passes the force it has just
// computed as `fresh`; fresh_small tells whether that is the program's F_small (else
// F_large), whichever model produced it.
struct CoordIn {
  double x, v, xr, fother, im;
};

__device__ inline CoordIn prefetch_coord(const Epilogue& E, int i, int n, int d, bool fresh_small) {
  CoordIn c;
  const size_t o = (size_t)d * n + i;
  c.x = E.x[o];
  c.v = E.v[o];
  c.xr = E.x_ref ? E.x_ref[o] : 0.0;
  c.fother = fresh_small ? (double)E.FL[o] : (double)E.Fs[o];
  c.im = inv_mass_at(E, i, E.species[i]);
  return c;
}

// Runs the program on lanes 0..2 (coordinate d = lane) of the calling wave, which must all
// be active; writes x, v and raises the flags exactly as apply_atom does.  Kicks and
// drifts only: a program with an O-step runs through apply_program (has_thermo), which
// keeps the registers of the Box-Muller deviates out of the kernels that fuse this.
__device__ inline void apply_coords(const Epilogue& E, int i, int n, int lane, const CoordIn& c,
                                    float fresh, bool fresh_small) {
  double vv = c.v, xx = c.x;
  bool moved = false;
  const double im = c.im;
  const double fl = fresh_small ? c.fother : (double)fresh;
  const double fs = fresh_small ? (double)fresh : c.fother;
  for (int k = 0; k < E.prog.nops; ++k) {
    const int op = E.prog.op[k];
    const double cc = E.prog.c[k];
    if (op == kDrift) {
      moved = true;
      xx = xx + cc * vv;
    } else {
      const double ci = cc * im;
      const double f = op == kKickSlow ? fl - fs : op == kKickFast ? fs : fl;
      vv = vv + ci * f;
      if (op == kKickSlow && E.fdiff_thr2 > 0.0) {
        const double f2 = lane < 3 ? f * f : 0.0;
        const double df2 = f2 + __shfl(f2, 1, 64) + __shfl(f2, 2, 64);
        if (lane == 0) fdiff_check(E, df2);
      }
    }
  }
  const int d = lane;
  bool bad = false;
  double u2 = 0.0;
  if (d < 3) {
    E.v[(size_t)d * n + i] = vv;
    bad = !isfinite(vv);
    if (moved) {
      E.x[(size_t)d * n + i] = xx;
      bad |= !isfinite(xx);
      const double u = xx - c.xr;
      u2 = u * u;
    }
  }
  const double u2y = __shfl(u2, 1, 64), u2z = __shfl(u2, 2, 64);
  const bool any_bad = __ballot(bad) != 0;
  if (lane == 0) {
    uint32_t f = 0;
    if (moved && E.x_ref) {
      double d2 = 0.0;
      d2 += u2;
      d2 += u2y;
      d2 += u2z;
      if (!(d2 <= E.max_disp2)) f |= kFlagStale;
    }
    if (any_bad) f |= DMTS_FLAG_NONFINITE;
    if (f) atomicOr(E.flags, f);
  }
}

// The program applied to atoms 0..n-1 by a launch of its own.
dmts_status apply_program(const Epilogue& E, int32_t n, hipStream_t s);

// Work-groups of `kernel` (launched with `threads` threads each) that the current device
// holds at once, from the occupancy calculator; cached per device and kernel.
int resident_groups(const void* kernel, int threads);

// `ep` (optional, needs `forces`): integrator program applied to every atom once its force
// is final; `forces` must then be the program's F_small (fast model) or F_large.
// `ws` (optional, fast model only): a caller-provided workspace of
// small_workspace_bytes(n, nl->max_pairs) bytes used instead of the model's own (which then
// never grows).
size_t small_workspace_bytes(int32_t n, int64_t max_pairs);
dmts_status small_energy_forces(Model* m, NList* nl, const double* pos,
                                const int32_t* species, int32_t n, double box,
                                const int32_t* sys_offsets, int32_t n_sys, double* energy,
                                float* forces, float* atom_energy, hipStream_t s,
                                const Epilogue* ep = nullptr, char* ws = nullptr);
dmts_status large_energy_forces(Model* m, NList* nl, const double* pos,
                                const int32_t* species, int32_t n, double box,
                                const int32_t* sys_offsets, int32_t n_sys, double* energy,
                                float* forces, float* atom_energy, hipStream_t s,
                                const Epilogue* ep = nullptr);

dmts_status energy_forces(Model* m, NList* nl, const double* pos, const int32_t* species,
                          int32_t n, double box, const int32_t* sys_offsets, int32_t n_sys,
                          double* energy, float* forces, float* atom_energy, hipStream_t s,
                          const Epilogue* ep = nullptr, char* ws = nullptr);

// Deterministic FP64 sum of per-atom FP32 energies per system: energy[s] = sum over the
// atoms of system s (one system when sys_offsets is NULL).  `partial` (energy_partials(n)
// doubles, may be NULL) lets a single large system be summed by many work-groups; the
// result has the same bits either way.
size_t energy_partials(int32_t n);
dmts_status reduce_energy(const float* atom_e, int32_t n, const int32_t* sys_offsets,
                          int32_t n_sys, double* energy, double* partial, hipStream_t s);

// Fill kernel (used instead of hipMemsetAsync so that streams can be captured).
dmts_status fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);

// ------------------------------------------------------------------ kernel timing
// Brackets the launches issued during its lifetime with events when timing is enabled.
struct ProfScope {
  int kid;
  hipStream_t s;
  hipEvent_t a = nullptr;
  hipEvent_t b = nullptr;   // set when the launch itself records the stop event
  bool started = false;     // a is (or will be, by the dispatch) recorded
  // packet_launch: the scope holds one launch_timed launch, whose dispatch records both
  // events (no marker of its own on the stream, which would stall the queue)
  ProfScope(int kernel_class, hipStream_t stream, bool packet_launch = false);
  ~ProfScope();
  // When this class is timed: start and stop events for a launch that records them in its
  // own dispatch (the kernel's start and end), instead of around it.
  bool packet(hipEvent_t& start, hipEvent_t& stop);
};

// Launch of one kernel of a timed class: with hipExtLaunchKernelGGL when the class is being
// timed (events taken at the kernel's own start and end), a plain launch otherwise.
template <typename... KArgs, typename... Args>
void launch_timed(ProfScope& ps, void (*kernel)(KArgs...), dim3 grid, dim3 block,
                  hipStream_t s, Args... args) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ps.packet(e0, e1))
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, e0, e1, 0, static_cast<KArgs>(args)...);
  else
    hipLaunchKernelGGL(kernel, grid, block, 0, s, static_cast<KArgs>(args)...);
}

// ------------------------------------------------------------------ device helpers
// logistic(t) = 1 / (1 + e^-t) with the hardware reciprocal (v_rcp_f32, 1 ulp); for
// t -> -inf the denominator is +inf and the result 0.
__device__ __forceinline__ float logistic_f(float t) {
  return __builtin_amdgcn_rcpf(1.0f + __expf(-t));
}
__device__ __forceinline__ float silu_f(float t) { return t * logistic_f(t); }
// d/dt SiLU = s (1 + t (1 - s)) = s + SiLU(t) (1 - s), s = logistic(t)
__device__ __forceinline__ float dsilu_f(float t) {
  const float s = logistic_f(t);
  return fmaf(t * s, 1.0f - s, s);
}
__device__ __forceinline__ void silu_and_grad(float t, float& y, float& dy) {
  const float s = logistic_f(t);
  y = t * s;
  dy = fmaf(y, 1.0f - s, s);
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double minimage(double d, double box, double inv_box) {
  return box > 0.0 ? d - box * rint(d * inv_box) : d;
}

}  // namespace dmts
