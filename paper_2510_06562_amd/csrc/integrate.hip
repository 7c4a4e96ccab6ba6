// The RESPA loop of Algorithm 1 (BAOAB-RESPA with force splitting) and the
// single-time-step baseline, in float64 on the device.
//
// Kicks and drifts are per-atom streaming work (x, v float64 [3][N], forces float32).
// Consecutive kicks/drifts between two force evaluations form one program, applied to
// each atom in the algorithm's order with exactly the arithmetic of separate steps, so
// fusion never changes a bit of the trajectory.  After a two-interaction evaluation it runs
// in the epilogue of the last kernel (the force gather), as soon as the atom's force is
// final; otherwise it gets one launch of its own:
//   kick:  v <- v + (tau * KAPPA / m) * F      (F = F_small, F_large or F_large - F_small)
//   drift: x <- x + tau * v
// KAPPA converts eV/(A amu) into A/fs^2.
//
// Neighbor lists.  Each reference-model evaluation builds one list at
// r_list = max(r_c,large, r_c,small + 1 A) and records the positions it was built at.  The
// fast model of the following inner steps runs on that same list: its kernels keep only
// pairs within its own cutoff, and rows are sorted by sender, so the sums it takes are
// exactly those of a list built at its cutoff.  The list is complete for the fast model as
// long as no atom has moved more than (r_list - r_c,small)/2 since the build; every drift
// launch checks that bound on the device.  If it is ever exceeded, the call is rolled back
// to its starting state and repeated with a fresh list for every fast evaluation.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"

namespace dmts {

namespace {

// 1 eV / (A amu) in A / fs^2 from the CODATA 2018 elementary charge and atomic mass
// constant.
constexpr double kKappa = 1.602176634e-19 / (1.0e-10 * 1.66053906660e-27) * 1.0e-20;
constexpr double kBoltzmann = 8.617333262e-5;   // eV / K (CODATA 2018)

constexpr double kMinSkin = 1.0;           // A between the fast cutoff and the shared list

// Integrator ops as a launch of their own (the start of a call, or after a model whose
// kernels do not take the program as an epilogue).
__global__ void __launch_bounds__(256) k_apply(Epilogue E, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) apply_atom(E, i, n);
}

__global__ void k_copy_f64(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}

// Kinetic energy sum(m v^2)/2 / KAPPA in eV, in a fixed order: chunks of kKeChunk atoms
// (one work-group each; lane t adds atoms t + 256 j into accumulator j, the eight
// accumulators pairwise, a butterfly within each wave, the four wave sums in order), then
// the chunk sums in order, and out = {E_large, E_small, KE, E_large + KE}.
constexpr int kKeThreads = 256;
constexpr int kKeChunk = kKeThreads * 8;

__global__ void __launch_bounds__(kKeThreads)
k_ke_chunks(int n, const double* __restrict__ v, const int32_t* __restrict__ species,
            const double* __restrict__ mass, const double* __restrict__ atom_mass,
            double* __restrict__ partial) {
  __shared__ double wsum[kKeThreads / 64];
  const int base = blockIdx.x * kKeChunk;
  double a[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int i = base + (int)threadIdx.x + j * kKeThreads;
    a[j] = 0.0;
    if (i < n) {
      const double m = atom_mass ? atom_mass[i] : mass[species[i]];
      const double x = v[i], y = v[(size_t)n + i], z = v[2 * (size_t)n + i];
      a[j] = m * (x * x + y * y + z * z);
    }
  }
  double acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double e = 0.0;
    for (int w = 0; w < kKeThreads / 64; ++w) e += wsum[w];
    partial[blockIdx.x] = e;
  }
}

__global__ void k_energies(const double* __restrict__ partial, int nc,
                           const double* __restrict__ e_models, double* __restrict__ out,
                           uint32_t* __restrict__ flags) {
  if (threadIdx.x != 0) return;
  double sum = 0.0;
  for (int k = 0; k < nc; ++k) sum += partial[k];
  const double ke = 0.5 * sum / kKappa;
  const double el = e_models[0], es = e_models[1];
  if (out) {
    out[0] = el;
    out[1] = es;
    out[2] = ke;
    out[3] = el + ke;
  }
  if (!isfinite(el) || !isfinite(es) || !isfinite(ke)) atomicOr(flags, DMTS_FLAG_NONFINITE);
}

__global__ void k_merge_flags(uint32_t* dst, const uint32_t* a, const uint32_t* b) {
  if (threadIdx.x == 0) {
    uint32_t f = *a | *b;
    if (f) atomicOr(dst, f);
  }
}

}  // namespace

struct State {
  int32_t n = 0;
  double box = 0.0;
  const int32_t* species = nullptr;
  double dt = 0.0;
  int32_t n_inner = 1;
  bool first = true;
  NList* nl_small = nullptr;
  NList* nl_large = nullptr;
  NList* nl_large2 = nullptr;   // the shared list is double-buffered: nl_large / nl_large2
  SkinList skin;                // the reference evaluations' lists come from its rows
  int shared_cur = 0;           // which of the two is the fast model's current list
  hipStream_t side = nullptr;   // fast evaluations overlapped with reference evaluations
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  float* FL = nullptr;      // [3][n]
  float* Fs = nullptr;      // [3][n]
  double* x_ref = nullptr;  // [3][n] positions of the last shared-list build
  double* bak = nullptr;    // [6][n] x, v at the start of a call; then FL, Fs as [3][n] floats
  double* mass = nullptr;   // [Z]
  double* inv_mass = nullptr;
  double host_inv_mass[8] = {0, 0, 0, 0, 0, 0, 0, 0};   // the same, for kernel arguments
  double host_mass[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  // per-atom masses and their inverses (hydrogen mass repartitioning); null: species table
  double* atom_mass = nullptr;       // [n]
  double* atom_inv_mass = nullptr;   // [n]
  // Langevin O-step (gamma = 0: off, NVE); o_count numbers the state's O-steps
  double gamma = 0.0, temperature = 0.0;
  uint64_t seed = 0, o_count = 0;
  // force-difference monitor (0: off) and the calls it had redone as single-time-step runs
  double fdiff_thr = 0.0;
  int64_t n_sts_redos = 0;
  uint32_t* fdiff_max = nullptr;   // device word: largest breaching |F - F_small| (float bits)
  float last_fdiff = 0.f;
  double* e_models = nullptr;   // {E_large, E_small}
  double* ke_part = nullptr;    // per-chunk kinetic energy sums
  uint32_t* flags = nullptr;
  // generations of the models the carried forces belong to (0: none)
  uint64_t last_small = 0;
  uint64_t last_large = 0;
  int64_t n_fallbacks = 0;   // calls redone with exact lists
};

namespace {

// One call's schedule: integrator ops and force evaluations in the algorithm's order.  It
// is built first, so that every evaluation is given the ops that follow it (up to the next
// evaluation) as the epilogue of its last kernel; only ops before the first evaluation of a
// call get a launch of their own.
enum EvalKind : int { kEvalLarge = 0, kEvalSmall = 1, kEvalPlain = 2 };

struct Item {
  bool eval;
  int op_or_kind;
  double c;       // op: coefficient
  bool want_e;    // eval: sum the energies (last evaluation of its model in the call)
  uint64_t ctr;   // O-step: its number
};

struct Runner {
  State* st;
  double* x;
  double* v;
  hipStream_t s;
  // shared-list mode: the fast model runs on the reference model's list
  bool shared = false;
  double list_cut = 0.0;
  double max_disp2 = 0.0;
  Model* small = nullptr;
  Model* large = nullptr;
  std::vector<Item> sched;

  // O-step constants of this call
  double o_decay = 1.0;
  double o_sd[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  double o_var = 0.0;

  void op(int o, double c, uint64_t ctr = 0) { sched.push_back(Item{false, o, c, false, ctr}); }
  void eval(int kind, bool want_e) { sched.push_back(Item{true, kind, 0.0, want_e, 0}); }

  Epilogue epilogue(const Prog& p) const {
    Epilogue e{};
    e.prog = p;
    e.x = x;
    e.v = v;
    e.FL = st->FL;
    e.Fs = st->Fs;
    e.species = st->species;
    for (int z = 0; z < 8; ++z) e.inv_mass[z] = st->host_inv_mass[z];
    e.inv_mass_atom = st->atom_inv_mass;
    e.x_ref = shared ? st->x_ref : nullptr;
    e.max_disp2 = max_disp2;
    e.flags = st->flags;
    e.o_decay = o_decay;
    for (int z = 0; z < 8; ++z) e.o_sd[z] = o_sd[z];
    e.o_var = o_var;
    e.o_key[0] = (uint32_t)st->seed;
    e.o_key[1] = (uint32_t)(st->seed >> 32);
    e.fdiff_thr2 = st->fdiff_thr * st->fdiff_thr;
    e.fdiff_max = st->fdiff_max;
    return e;
  }
  // The model energies are only reported for the positions a call ends at, so an
  // evaluation sums them only when it is the last one of its model in the call.
  // The ops that follow an evaluation are handed to it as its epilogue (the model decides
  // whether they run inside its last kernel or right after it).
  NList* shared_list(int which) const { return which ? st->nl_large2 : st->nl_large; }
  dmts_status run_eval(const Item& it, const Prog& after, hipStream_t stream = nullptr,
                       hipEvent_t wait = nullptr) {
    hipStream_t q = stream ? stream : s;
    Epilogue E = epilogue(after);
    E.wait = wait;
    const Epilogue* ep = after.nops > 0 ? &E : nullptr;
    dmts_status r;
    if (it.op_or_kind == kEvalSmall) {
      NList* nl = shared ? shared_list(st->shared_cur) : st->nl_small;
      if (!shared) {
        r = build_neighbors(st->nl_small, x, st->n, st->box, nullptr, 1,
                            (double)small->desc.cutoff, q);
        if (r != DMTS_OK) return r;
      } else if (small->desc.kind == NNP_KIND_TWO_INTERACTION) {
        // a fast model of the reference kind sums over exact rows: the shared list's rows
        // filtered to its cutoff at the current positions (the one-interaction kernels
        // compact the rows themselves)
        r = filter_neighbors(st->nl_small, nl, x, (double)small->desc.cutoff, q);
        if (r != DMTS_OK) return r;
        nl = st->nl_small;
      }
      return energy_forces(small, nl, x, st->species, st->n, st->box, nullptr, 1,
                           it.want_e ? st->e_models + 1 : nullptr, st->Fs, nullptr, q, ep);
    }
    // reference model (Algorithm 1) or the plain single-time-step model: builds its list
    // (in shared mode at list_cut into the other buffer of the shared list, recording x_ref
    // for the fast model's displacement check, after which it becomes the current one)
    NList* nl = shared ? shared_list(st->shared_cur ^ 1) : st->nl_large;
    r = refresh_neighbors(nl, &st->skin, x, st->n, st->box,
                          shared ? list_cut : (double)large->desc.cutoff, q,
                          shared ? st->x_ref : nullptr);
    if (r != DMTS_OK) return r;
    if (shared) st->shared_cur ^= 1;
    return energy_forces(large, nl, x, st->species, st->n, st->box, nullptr, 1,
                         it.want_e ? st->e_models : nullptr, st->FL, nullptr, q, ep);
  }
  // ops [k, next evaluation) as one program
  Prog collect(size_t& k) const {
    Prog p{};
    while (k < sched.size() && !sched[k].eval) {
      if (p.nops == kMaxOps) break;
      p.op[p.nops] = sched[k].op_or_kind;
      p.c[p.nops] = sched[k].c;
      p.ctr[p.nops] = sched[k].ctr;
      ++p.nops;
      ++k;
    }
    return p;
  }
  dmts_status apply(const Prog& p) { return apply_program(epilogue(p), st->n, s); }
  dmts_status execute() {
    size_t k = 0;
    dmts_status r;
    while (k < sched.size() && !sched[k].eval) {   // ops before the first evaluation
      if ((r = apply(collect(k))) != DMTS_OK) return r;
    }
    while (k < sched.size()) {
      const Item it = sched[k++];
      size_t k_ops = k;
      Prog after = collect(k);
      // A fast evaluation followed, with kicks only in between, by a reference evaluation
      // at the same positions: the fast evaluation and its kicks run on the side stream
      // while the reference model builds its list and runs its kernels; the reference
      // model's force gather (whose epilogue reads F_small and v) waits for them.
      if (overlap_ok(it, after, k_ops, k)) {
        const Item next = sched[k++];
        Prog after2 = collect(k);
        DMTS_HIP(hipEventRecord(st->ev_fork, s));
        DMTS_HIP(hipStreamWaitEvent(st->side, st->ev_fork, 0));
        if ((r = run_eval(it, after, st->side)) != DMTS_OK) return r;
        DMTS_HIP(hipEventRecord(st->ev_join, st->side));
        if (after2.nops == 0) DMTS_HIP(hipStreamWaitEvent(s, st->ev_join, 0));
        if ((r = run_eval(next, after2, nullptr, after2.nops ? st->ev_join : nullptr)) != DMTS_OK)
          return r;
        after = after2;
      } else if ((r = run_eval(it, after)) != DMTS_OK) {
        return r;
      }
      while (k < sched.size() && !sched[k].eval) {   // more ops than one program holds
        if ((r = apply(collect(k))) != DMTS_OK) return r;
      }
    }
    sched.clear();
    return DMTS_OK;
  }
  // The overlap needs the shared list (the fast model reads the current buffer while the
  // reference model builds the other), two distinct models (separate workspaces), and no
  // drift between the two evaluations.
  bool overlap_ok(const Item& it, const Prog& after, size_t k_ops, size_t k_next) const {
    if (!shared || !st->side || small == large || it.op_or_kind != kEvalSmall) return false;
    if (k_next >= sched.size() || !sched[k_next].eval || sched[k_next].op_or_kind != kEvalLarge)
      return false;
    if (k_next - k_ops != (size_t)after.nops) return false;   // all ops fit one program
    for (int q = 0; q < after.nops; ++q)
      if (after.op[q] == kDrift) return false;
    return true;
  }
};

// Algorithm 1 (or velocity Verlet when small is NULL) for n_outer outer steps.
// The O-step over time h: decay e^(-gamma h) and the per-species noise scale
// sqrt((1 - decay^2) k_B T KAPPA / m) (Algorithm 1's thermostat, exact Ornstein-Uhlenbeck).
void o_constants(const State* st, Runner& R, double h) {
  R.o_decay = std::exp(-st->gamma * h);
  R.o_var = (1.0 - R.o_decay * R.o_decay) * kBoltzmann * st->temperature * kKappa;
  for (int z = 0; z < 8; ++z)
    R.o_sd[z] = st->host_mass[z] > 0.0
                    ? std::sqrt((1.0 - R.o_decay * R.o_decay) * kBoltzmann * st->temperature *
                                kKappa / st->host_mass[z])
                    : 0.0;
}

// n_outer steps of Algorithm 1, or with small == NULL n_outer single-time-step steps of
// length dt_sts (the state's dt when <= 0).
dmts_status run_steps(State* st, Runner& R, Model* small, Model* large, int n_outer,
                      double dt_sts = 0.0) {
  const double kappa = kKappa;
  R.small = small;
  R.large = large;
  R.sched.clear();
  const double dt = small || dt_sts <= 0.0 ? st->dt : dt_sts;
  const bool thermo = st->gamma > 0.0;
  if (!small) {
    // single-time-step baseline: BAOAB with the reference model (velocity Verlet when
    // gamma = 0)
    o_constants(st, R, dt);
    if (st->first) R.eval(kEvalPlain, n_outer == 0);
    for (int o = 0; o < n_outer; ++o) {
      R.op(kKickLarge, 0.5 * dt * kappa);
      R.op(kDrift, 0.5 * dt);
      if (thermo) R.op(kThermo, 0.0, st->o_count++);
      R.op(kDrift, 0.5 * dt);
      R.eval(kEvalPlain, o == n_outer - 1);
      R.op(kKickLarge, 0.5 * dt * kappa);
    }
  } else {
    const int n = st->n_inner;
    const double h_in = dt / n;
    o_constants(st, R, h_in);
    if (st->first) {
      R.eval(kEvalLarge, n_outer == 0);
      R.eval(kEvalSmall, n_outer == 0);
    }
    for (int o = 0; o < n_outer; ++o) {
      const bool last = o == n_outer - 1;
      R.op(kKickSlow, 0.5 * dt * kappa);
      for (int k = 0; k < n; ++k) {
        R.op(kKickFast, 0.5 * h_in * kappa);
        R.op(kDrift, 0.5 * h_in);
        if (thermo) R.op(kThermo, 0.0, st->o_count++);
        R.op(kDrift, 0.5 * h_in);
        R.eval(kEvalSmall, last && k == n - 1);
        R.op(kKickFast, 0.5 * h_in * kappa);
      }
      R.eval(kEvalLarge, last);
      R.op(kKickSlow, 0.5 * dt * kappa);
    }
  }
  st->first = false;
  return R.execute();
}

}  // namespace

dmts_status apply_program(const Epilogue& E, int32_t n, hipStream_t s) {
  if (E.prog.nops == 0 || n <= 0) return DMTS_OK;
  ProfScope ps(DMTS_K_INTEGRATE, s);
  k_apply<<<ceil_div(n, 256), 256, 0, s>>>(E, n);
  DMTS_CHECK_LAUNCH();
  return DMTS_OK;
}

}  // namespace dmts

using dmts::Model;
using dmts::NList;
using dmts::State;

extern "C" dmts_status dmts_state_create(int32_t n_atoms, double box, const int32_t* species,
                                         const double* host_mass_by_species, int32_t n_species,
                                         double dt_outer_fs, int32_t n_inner,
                                         int32_t max_nbrs_small, int32_t max_nbrs_large,
                                         dmts_state** out) {
  DMTS_REQUIRE(out && species && host_mass_by_species, DMTS_E_ARG,
               "dmts_state_create: null argument");
  *out = nullptr;
  DMTS_REQUIRE(n_atoms >= 1 && n_species >= 1 && n_species <= 8, DMTS_E_ARG,
               "dmts_state_create: bad sizes (%d atoms, %d species)", n_atoms, n_species);
  DMTS_REQUIRE(dt_outer_fs > 0.0 && n_inner >= 1, DMTS_E_ARG,
               "dmts_state_create: need dt > 0 and n_inner >= 1");
  DMTS_REQUIRE(max_nbrs_small >= 1 && max_nbrs_large >= 1, DMTS_E_ARG,
               "dmts_state_create: neighbor bounds must be positive");
  DMTS_REQUIRE(box >= 0.0, DMTS_E_ARG, "dmts_state_create: negative box");
  for (int z = 0; z < n_species; ++z)
    DMTS_REQUIRE(host_mass_by_species[z] > 0.0, DMTS_E_ARG,
                 "dmts_state_create: mass of species %d must be positive", z);
  State* st = new State();
  st->n = n_atoms;
  st->box = box;
  st->species = species;
  st->dt = dt_outer_fs;
  st->n_inner = n_inner;
  dmts_status r = nnp_nlist_create(n_atoms, (int64_t)n_atoms * (max_nbrs_small + 16), 16,
                                   reinterpret_cast<nnp_nlist**>(&st->nl_small));
  if (r == DMTS_OK)
    r = nnp_nlist_create(n_atoms, (int64_t)n_atoms * (max_nbrs_large + 16), 16,
                         reinterpret_cast<nnp_nlist**>(&st->nl_large));
  if (r == DMTS_OK)
    r = nnp_nlist_create(n_atoms, (int64_t)n_atoms * (max_nbrs_large + 16), 16,
                         reinterpret_cast<nnp_nlist**>(&st->nl_large2));
  // the skin list only uses its staging rows: no CSR capacity
  if (r == DMTS_OK)
    r = nnp_nlist_create(n_atoms, 4, 16, reinterpret_cast<nnp_nlist**>(&st->skin.rows));
  st->skin.skin = dmts::kDefaultSkin;
  double hm[16] = {0}, him[16] = {0};
  for (int z = 0; z < n_species; ++z) {
    hm[z] = host_mass_by_species[z];
    him[z] = 1.0 / host_mass_by_species[z];
    st->host_inv_mass[z] = him[z];
    if (z < 8) st->host_mass[z] = hm[z];
  }
  hipError_t e = hipSuccess;
  if (r == DMTS_OK) {
    e = hipMalloc(&st->FL, sizeof(float) * 3 * (size_t)n_atoms);
    if (e == hipSuccess) e = hipMalloc(&st->Fs, sizeof(float) * 3 * (size_t)n_atoms);
    if (e == hipSuccess) e = hipMalloc(&st->x_ref, sizeof(double) * 3 * (size_t)n_atoms);
    if (e == hipSuccess) e = hipMalloc(&st->skin.x_build, sizeof(double) * 3 * (size_t)n_atoms);
    if (e == hipSuccess)
      e = hipMalloc(&st->skin.ell, sizeof(int32_t) * dmts::kSkinRowCap * (size_t)n_atoms);
    if (e == hipSuccess) e = hipMalloc(&st->skin.gate, sizeof(uint32_t) * 2);
    if (e == hipSuccess) e = hipMemset(st->skin.gate, 0, sizeof(uint32_t) * 2);
    if (e == hipSuccess) e = hipMalloc(&st->bak, sizeof(double) * 9 * (size_t)n_atoms);
    if (e == hipSuccess) e = hipMalloc(&st->mass, sizeof(double) * 16);
    if (e == hipSuccess) e = hipMalloc(&st->inv_mass, sizeof(double) * 16);
    if (e == hipSuccess) e = hipMalloc(&st->e_models, sizeof(double) * 4);
    if (e == hipSuccess)
      e = hipMalloc(&st->ke_part, sizeof(double) * ((size_t)n_atoms / dmts::kKeChunk + 1));
    if (e == hipSuccess) e = hipMalloc(&st->flags, sizeof(uint32_t));
    if (e == hipSuccess) e = hipMalloc(&st->fdiff_max, sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemset(st->fdiff_max, 0, sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemcpy(st->mass, hm, sizeof(hm), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(st->inv_mass, him, sizeof(him), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(st->e_models, 0, sizeof(double) * 4);
    if (e == hipSuccess) e = hipMemset(st->flags, 0, sizeof(uint32_t));
    // side stream at the default priority, synchronised with the caller's stream by events.
    // The events order two streams of one device and are never read by the host, so they
    // skip the system-scope fence (a write-back of the caches that idles the recording
    // stream for several microseconds); each kernel's own completion already makes its
    // results visible device-wide.
    const unsigned ev_flags = hipEventDisableTiming | hipEventDisableSystemFence;
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&st->ev_fork, ev_flags);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&st->ev_join, ev_flags);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
      dmts::set_error("dmts_state_create: %s", hipGetErrorString(e));
      r = DMTS_E_OOM;
    }
  }
  if (r != DMTS_OK) {
    dmts_state_destroy(reinterpret_cast<dmts_state*>(st));
    return r;
  }
  *out = reinterpret_cast<dmts_state*>(st);
  return DMTS_OK;
}

extern "C" void dmts_state_destroy(dmts_state* h) {
  State* st = reinterpret_cast<State*>(h);
  if (!st) return;
  (void)hipDeviceSynchronize();
  nnp_nlist_destroy(reinterpret_cast<nnp_nlist*>(st->nl_small));
  nnp_nlist_destroy(reinterpret_cast<nnp_nlist*>(st->nl_large));
  nnp_nlist_destroy(reinterpret_cast<nnp_nlist*>(st->nl_large2));
  nnp_nlist_destroy(reinterpret_cast<nnp_nlist*>(st->skin.rows));
  (void)hipFree(st->skin.x_build);
  (void)hipFree(st->skin.ell);
  (void)hipFree(st->skin.gate);
  if (st->ev_fork) (void)hipEventDestroy(st->ev_fork);
  if (st->ev_join) (void)hipEventDestroy(st->ev_join);
  if (st->side) (void)hipStreamDestroy(st->side);
  (void)hipFree(st->FL);
  (void)hipFree(st->Fs);
  (void)hipFree(st->x_ref);
  (void)hipFree(st->bak);
  (void)hipFree(st->mass);
  (void)hipFree(st->inv_mass);
  (void)hipFree(st->atom_mass);
  (void)hipFree(st->atom_inv_mass);
  (void)hipFree(st->e_models);
  (void)hipFree(st->ke_part);
  (void)hipFree(st->fdiff_max);
  (void)hipFree(st->flags);
  delete st;
}

extern "C" dmts_status dmts_state_reset(dmts_state* h) {
  State* st = reinterpret_cast<State*>(h);
  DMTS_REQUIRE(st, DMTS_E_ARG, "dmts_state_reset: null state");
  st->first = true;
  return DMTS_OK;
}

extern "C" dmts_status dmts_state_set_thermostat(dmts_state* h, double gamma_per_fs,
                                                 double temperature_K, uint64_t seed) {
  State* st = reinterpret_cast<State*>(h);
  DMTS_REQUIRE(st, DMTS_E_ARG, "dmts_state_set_thermostat: null state");
  DMTS_REQUIRE(std::isfinite(gamma_per_fs) && gamma_per_fs >= 0.0, DMTS_E_ARG,
               "dmts_state_set_thermostat: gamma must be finite and >= 0, got %g", gamma_per_fs);
  DMTS_REQUIRE(std::isfinite(temperature_K) && temperature_K >= 0.0, DMTS_E_ARG,
               "dmts_state_set_thermostat: temperature must be finite and >= 0, got %g",
               temperature_K);
  st->gamma = gamma_per_fs;
  st->temperature = temperature_K;
  st->seed = seed;
  st->o_count = 0;
  return DMTS_OK;
}

extern "C" dmts_status dmts_state_set_atom_masses(dmts_state* h, const double* host_masses,
                                                  int32_t n_atoms) {
  State* st = reinterpret_cast<State*>(h);
  DMTS_REQUIRE(st, DMTS_E_ARG, "dmts_state_set_atom_masses: null state");
  if (!host_masses) {   // back to the species table
    (void)hipFree(st->atom_mass);
    (void)hipFree(st->atom_inv_mass);
    st->atom_mass = st->atom_inv_mass = nullptr;
    return DMTS_OK;
  }
  DMTS_REQUIRE(n_atoms == st->n, DMTS_E_ARG,
               "dmts_state_set_atom_masses: %d masses for a state of %d atoms", n_atoms, st->n);
  std::vector<double> m(2 * (size_t)n_atoms);
  for (int32_t i = 0; i < n_atoms; ++i) {
    DMTS_REQUIRE(std::isfinite(host_masses[i]) && host_masses[i] > 0.0, DMTS_E_ARG,
                 "dmts_state_set_atom_masses: mass %d is %g (must be finite and > 0)", i,
                 host_masses[i]);
    m[i] = host_masses[i];
    m[(size_t)n_atoms + i] = 1.0 / host_masses[i];
  }
  const size_t bytes = sizeof(double) * (size_t)n_atoms;
  if (!st->atom_mass) {
    DMTS_HIP(hipMalloc(&st->atom_mass, bytes));
    if (hipMalloc(&st->atom_inv_mass, bytes) != hipSuccess) {
      (void)hipFree(st->atom_mass);
      st->atom_mass = nullptr;
      DMTS_REQUIRE(false, DMTS_E_OOM, "dmts_state_set_atom_masses: out of device memory");
    }
  }
  DMTS_HIP(hipMemcpy(st->atom_mass, m.data(), bytes, hipMemcpyHostToDevice));
  DMTS_HIP(hipMemcpy(st->atom_inv_mass, m.data() + n_atoms, bytes, hipMemcpyHostToDevice));
  return DMTS_OK;
}

extern "C" dmts_status dmts_state_set_fdiff_threshold(dmts_state* h, double eV_per_A) {
  State* st = reinterpret_cast<State*>(h);
  DMTS_REQUIRE(st, DMTS_E_ARG, "dmts_state_set_fdiff_threshold: null state");
  DMTS_REQUIRE(std::isfinite(eV_per_A) && eV_per_A >= 0.0, DMTS_E_ARG,
               "dmts_state_set_fdiff_threshold: threshold must be finite and >= 0, got %g",
               eV_per_A);
  st->fdiff_thr = eV_per_A;
  return DMTS_OK;
}

extern "C" dmts_status dmts_state_fdiff(dmts_state* h, int64_t* n_sts_redos,
                                        double* last_breach) {
  State* st = reinterpret_cast<State*>(h);
  DMTS_REQUIRE(st && n_sts_redos && last_breach, DMTS_E_ARG, "dmts_state_fdiff: null argument");
  *n_sts_redos = st->n_sts_redos;
  *last_breach = st->last_fdiff;
  return DMTS_OK;
}

extern "C" dmts_status dmts_state_o_steps(dmts_state* h, uint64_t* n_o_steps) {
  State* st = reinterpret_cast<State*>(h);
  DMTS_REQUIRE(st && n_o_steps, DMTS_E_ARG, "dmts_state_o_steps: null argument");
  *n_o_steps = st->o_count;
  return DMTS_OK;
}

extern "C" dmts_status dmts_state_fallbacks(dmts_state* h, int64_t* n_calls) {
  State* st = reinterpret_cast<State*>(h);
  DMTS_REQUIRE(st && n_calls, DMTS_E_ARG, "dmts_state_fallbacks: null argument");
  *n_calls = st->n_fallbacks;
  return DMTS_OK;
}

extern "C" dmts_status dmts_state_set_skin(dmts_state* h, double skin_A) {
  State* st = reinterpret_cast<State*>(h);
  DMTS_REQUIRE(st, DMTS_E_ARG, "dmts_state_set_skin: null state");
  DMTS_REQUIRE(skin_A >= 0.0 && std::isfinite(skin_A), DMTS_E_ARG,
               "dmts_state_set_skin: skin %g must be finite and >= 0", skin_A);
  if (skin_A != st->skin.skin) {
    st->skin.skin = skin_A;
    st->skin.n = -1;   // the rows were built for another skin: rebuild at the next use
  }
  return DMTS_OK;
}

extern "C" dmts_status dmts_state_get_skin(dmts_state* h, double* skin_A) {
  State* st = reinterpret_cast<State*>(h);
  DMTS_REQUIRE(st && skin_A, DMTS_E_ARG, "dmts_state_get_skin: null argument");
  *skin_A = st->skin.skin;
  return DMTS_OK;
}

extern "C" dmts_status dmts_state_list_builds(dmts_state* h, int64_t* n_builds) {
  State* st = reinterpret_cast<State*>(h);
  DMTS_REQUIRE(st && n_builds, DMTS_E_ARG, "dmts_state_list_builds: null argument");
  uint32_t g[2] = {0u, 0u};
  DMTS_HIP(hipDeviceSynchronize());
  DMTS_HIP(hipMemcpy(g, st->skin.gate, sizeof(g), hipMemcpyDeviceToHost));
  *n_builds = g[1];
  return DMTS_OK;
}

extern "C" dmts_status dmts_state_forces(dmts_state* h, const float** f_large,
                                         const float** f_small) {
  State* st = reinterpret_cast<State*>(h);
  DMTS_REQUIRE(st, DMTS_E_ARG, "dmts_state_forces: null state");
  if (f_large) *f_large = st->FL;
  if (f_small) *f_small = st->Fs;
  return DMTS_OK;
}

extern "C" dmts_status dmts_state_flags(dmts_state* h, void* stream, uint32_t* host_flags) {
  State* st = reinterpret_cast<State*>(h);
  DMTS_REQUIRE(st && host_flags, DMTS_E_ARG, "dmts_state_flags: null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  dmts::k_merge_flags<<<1, 64, 0, s>>>(st->flags, st->nl_small->flags, st->nl_large->flags);
  dmts::k_merge_flags<<<1, 64, 0, s>>>(st->flags, st->nl_large2->flags, st->nl_large2->flags);
  DMTS_CHECK_LAUNCH();
  DMTS_HIP(hipMemcpyAsync(host_flags, st->flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  DMTS_HIP(hipStreamSynchronize(s));
  dmts_status r = dmts::fill_u32(st->flags, 0u, 1, s);
  if (r == DMTS_OK) r = dmts::fill_u32(st->nl_small->flags, 0u, 1, s);
  if (r == DMTS_OK) r = dmts::fill_u32(st->nl_large->flags, 0u, 1, s);
  if (r == DMTS_OK) r = dmts::fill_u32(st->nl_large2->flags, 0u, 1, s);
  if (r != DMTS_OK) return r;
  DMTS_HIP(hipStreamSynchronize(s));
  return DMTS_OK;
}

namespace dmts {
namespace {

// Host copy of the state a roll-back returns to: x, v (and the carried forces unless the
// next run evaluates both models afresh) go to the state's backup buffer.
dmts_status backup(State* st, const double* x, const double* v, bool forces, hipStream_t s) {
  const int64_t n3 = 3 * (int64_t)st->n;
  double* b = st->bak;
  k_copy_f64<<<ceil_div(n3, 256), 256, 0, s>>>(x, b, n3);
  k_copy_f64<<<ceil_div(n3, 256), 256, 0, s>>>(v, b + n3, n3);
  if (forces) {   // carried forces: 2 x 3n floats = 3n doubles
    DMTS_HIP(hipMemcpyAsync(b + 2 * n3, st->FL, sizeof(float) * n3, hipMemcpyDeviceToDevice, s));
    DMTS_HIP(hipMemcpyAsync(reinterpret_cast<float*>(b + 2 * n3) + n3, st->Fs,
                            sizeof(float) * n3, hipMemcpyDeviceToDevice, s));
  }
  DMTS_CHECK_LAUNCH();
  return DMTS_OK;
}

dmts_status restore(State* st, double* x, double* v, bool forces, hipStream_t s) {
  const int64_t n3 = 3 * (int64_t)st->n;
  double* b = st->bak;
  k_copy_f64<<<ceil_div(n3, 256), 256, 0, s>>>(b, x, n3);
  k_copy_f64<<<ceil_div(n3, 256), 256, 0, s>>>(b + n3, v, n3);
  if (forces) {
    DMTS_HIP(hipMemcpyAsync(st->FL, b + 2 * n3, sizeof(float) * n3, hipMemcpyDeviceToDevice, s));
    DMTS_HIP(hipMemcpyAsync(st->Fs, reinterpret_cast<float*>(b + 2 * n3) + n3,
                            sizeof(float) * n3, hipMemcpyDeviceToDevice, s));
  }
  DMTS_CHECK_LAUNCH();
  return DMTS_OK;
}

// The state's flag word and largest recorded force difference (synchronizes the stream).
dmts_status read_flags(State* st, bool monitor, hipStream_t s, uint32_t& f, float& fdiff) {
  DMTS_HIP(hipMemcpyAsync(&f, st->flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  uint32_t fm = 0;
  if (monitor)
    DMTS_HIP(hipMemcpyAsync(&fm, st->fdiff_max, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  DMTS_HIP(hipStreamSynchronize(s));
  std::memcpy(&fdiff, &fm, sizeof(fdiff));
  return DMTS_OK;
}

// n_outer outer steps of Algorithm 1 taken as one attempt that may be rolled back:
//  * an atom moved beyond the shared list's skin (shared mode): restore the starting state
//    and redo with exact lists for every evaluation;
//  * a slow kick saw |F - F_small| above the monitor's threshold (in the first attempt or
//    in the redo with exact lists): restore and redo as n_outer * n_inner single-time-step
//    steps of the inner length with the reference model (the paper's reversion).
// Either redo leaves lists or forces that are not the carried ones, so the next attempt
// evaluates both models afresh.
dmts_status checked_steps(State* st, double* x, double* v, Model* small, Model* large,
                          int n_outer, const Runner& proto, bool monitor, hipStream_t s) {
  const bool first0 = st->first;
  const uint64_t o_count0 = st->o_count;
  dmts_status r;
  if (monitor && (r = fill_u32(st->fdiff_max, 0u, 1, s)) != DMTS_OK) return r;
  if ((r = backup(st, x, v, !first0, s)) != DMTS_OK) return r;
  Runner R = proto;
  if ((r = run_steps(st, R, small, large, n_outer)) != DMTS_OK) return r;
  uint32_t f = 0;
  float fd = 0.f;
  if ((r = read_flags(st, monitor, s, f, fd)) != DMTS_OK) return r;
  constexpr uint32_t kRedo = kFlagStale | kFlagFdiff;
  if ((f & kFlagStale) && !(f & kFlagFdiff)) {
    if ((r = restore(st, x, v, !first0, s)) != DMTS_OK) return r;
    st->first = first0;
    st->o_count = o_count0;   // the same thermostat noise
    if ((r = fill_u32(st->flags, f & ~kRedo, 1, s)) != DMTS_OK) return r;
    ++st->n_fallbacks;
    Runner E{st, x, v, s};    // exact lists for every evaluation
    if ((r = run_steps(st, E, small, large, n_outer)) != DMTS_OK) return r;
    st->first = true;
    uint32_t f2 = 0;
    if ((r = read_flags(st, monitor, s, f2, fd)) != DMTS_OK) return r;
    f = (f & ~kRedo) | f2;    // a breach seen by the redo is acted on below
  }
  if (f & kFlagFdiff) {
    st->last_fdiff = std::max(st->last_fdiff, fd);
    if ((r = restore(st, x, v, !first0, s)) != DMTS_OK) return r;
    st->first = first0;
    st->o_count = o_count0;
    if ((r = fill_u32(st->flags, f & ~kRedo, 1, s)) != DMTS_OK) return r;
    ++st->n_sts_redos;
    Runner E{st, x, v, s};
    if ((r = run_steps(st, E, nullptr, large, n_outer * st->n_inner, st->dt / st->n_inner)) !=
        DMTS_OK)
      return r;
    // the single-time-step steps leave F_small behind: the next attempt evaluates both
    st->first = true;
  }
  return DMTS_OK;
}

}  // namespace
}  // namespace dmts

extern "C" dmts_status dmts_step(dmts_state* h, double* x, double* v, nnp_model* small_h,
                                 nnp_model* large_h, int32_t n_outer, double* energies_out,
                                 void* stream) {
  State* st = reinterpret_cast<State*>(h);
  Model* small = reinterpret_cast<Model*>(small_h);
  Model* large = reinterpret_cast<Model*>(large_h);
  DMTS_REQUIRE(st && x && v && large, DMTS_E_ARG, "dmts_step: null argument");
  DMTS_REQUIRE(n_outer >= 0, DMTS_E_ARG, "dmts_step: n_outer must be >= 0");
  DMTS_REQUIRE(large->desc.cutoff < 0.5 * st->box || st->box == 0.0, DMTS_E_BOX,
               "dmts_step: cutoff %g must be below half the box edge", large->desc.cutoff);
  hipStream_t s = static_cast<hipStream_t>(stream);
  // carried forces belong to the models (by identity, not address) they were computed with
  const uint64_t gs = small ? small->generation : 0, gl = large->generation;
  if (gs != st->last_small || gl != st->last_large) st->first = true;
  st->last_small = gs;
  st->last_large = gl;
  dmts::Runner R{st, x, v, s};
  dmts_status r;
  if (small) {
    const double want = std::max((double)large->desc.cutoff,
                                 (double)small->desc.cutoff + dmts::kMinSkin);
    if (st->box == 0.0 || want < 0.5 * st->box) {
      R.shared = true;
      R.list_cut = want;
      const double half_skin = 0.5 * (want - (double)small->desc.cutoff);
      R.max_disp2 = half_skin * half_skin;
    }
  }
  const bool monitor = small && st->fdiff_thr > 0.0;
  if (monitor) st->last_fdiff = 0.f;
  if (monitor) {
    // the monitor decides per outer step: one checked attempt per step
    for (int o = 0; o < n_outer; ++o)
      if ((r = dmts::checked_steps(st, x, v, small, large, 1, R, true, s)) != DMTS_OK) return r;
    if (n_outer == 0 && (r = dmts::run_steps(st, R, small, large, 0)) != DMTS_OK) return r;
  } else if (R.shared) {
    if ((r = dmts::checked_steps(st, x, v, small, large, n_outer, R, false, s)) != DMTS_OK)
      return r;
  } else if ((r = dmts::run_steps(st, R, small, large, n_outer)) != DMTS_OK) {
    return r;
  }
  {
    const int nc = (st->n + dmts::kKeChunk - 1) / dmts::kKeChunk;
    if (nc > 0)
      dmts::k_ke_chunks<<<nc, dmts::kKeThreads, 0, s>>>(st->n, v, st->species, st->mass,
                                                         st->atom_mass, st->ke_part);
    dmts::k_energies<<<1, 64, 0, s>>>(st->ke_part, nc, st->e_models, energies_out, st->flags);
  }
  DMTS_CHECK_LAUNCH();
  uint32_t f = 0;
  if ((r = dmts_state_flags(h, stream, &f)) != DMTS_OK) return r;
  DMTS_REQUIRE(!(f & DMTS_FLAG_NBR_OVERFLOW), DMTS_E_CAPACITY,
               "dmts_step: a neighbor list overflowed; raise max_nbrs");
  DMTS_REQUIRE(!(f & DMTS_FLAG_NONFINITE), DMTS_E_NONFINITE,
               "dmts_step: non-finite positions, velocities or energies");
  return DMTS_OK;
}
