// Internal declarations shared by the library's translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
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
  int32_t* len = nullptr;    // [max_atoms] real row lengths
  int32_t* ell = nullptr;    // [max_atoms][kNlistRowCap] sorted rows before compaction
  // cell list scratch
  int32_t* cell_of = nullptr;    // [max_atoms]
  int32_t* cell_atoms = nullptr; // [max_atoms]
  DevBuf cell_buf;               // count, start, cursor
  int32_t n_cells_cap = 0;
};

dmts_status build_neighbors(NList* nl, const double* pos, int32_t n, double box,
                            const int32_t* sys_offsets, int32_t n_sys, double cutoff,
                            hipStream_t s);

// ------------------------------------------------------------------ models
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
  // launch: work-groups of the pair kernels (0 = one per group of receivers); the pair
  // kernels loop over receivers in a grid-stride order, so any count gives the same bits
  int32_t grid = 0;
  // workspace
  DevBuf atom_ws, pair_ws, sys_ws;
  // natural: work-groups for one pass over the receivers; resident: how many the GPU holds
  // at once.  With the default grid, a pass that would take between one and two rounds of
  // work-groups runs as one persistent round instead of a full and a partly filled one.
  int launch_grid(int natural, int resident = 0) const {
    if (grid > 0) return grid < natural ? grid : natural;
    return resident > 0 && natural > resident && natural < 2 * resident ? resident : natural;
  }
  const float* p(size_t off) const { return params.as<float>() + off; }
};

// Work-groups of `kernel` (launched with `threads` threads each) that the current device
// holds at once, from the occupancy calculator; cached per device and kernel.
int resident_groups(const void* kernel, int threads);

dmts_status small_energy_forces(Model* m, NList* nl, const double* pos,
                                const int32_t* species, int32_t n, double box,
                                const int32_t* sys_offsets, int32_t n_sys, double* energy,
                                float* forces, float* atom_energy, hipStream_t s);
dmts_status large_energy_forces(Model* m, NList* nl, const double* pos,
                                const int32_t* species, int32_t n, double box,
                                const int32_t* sys_offsets, int32_t n_sys, double* energy,
                                float* forces, float* atom_energy, hipStream_t s);

dmts_status energy_forces(Model* m, NList* nl, const double* pos, const int32_t* species,
                          int32_t n, double box, const int32_t* sys_offsets, int32_t n_sys,
                          double* energy, float* forces, float* atom_energy, hipStream_t s);

// Deterministic FP64 sum of per-atom FP32 energies per system: energy[s] = sum over the
// atoms of system s (one system when sys_offsets is NULL).
dmts_status reduce_energy(const float* atom_e, int32_t n, const int32_t* sys_offsets,
                          int32_t n_sys, double* energy, hipStream_t s);

// Fill kernel (used instead of hipMemsetAsync so that streams can be captured).
dmts_status fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);

// ------------------------------------------------------------------ kernel timing
// Brackets the launches issued during its lifetime with events when timing is enabled.
struct ProfScope {
  int kid;
  hipStream_t s;
  hipEvent_t a = nullptr;
  ProfScope(int kernel_class, hipStream_t stream);
  ~ProfScope();
};

// ------------------------------------------------------------------ device helpers
// logistic(t) = 1 / (1 + e^-t) with the hardware reciprocal (v_rcp_f32, 1 ulp); for
// t -> -inf the denominator is +inf and the result 0.
__device__ __forceinline__ float logistic_f(float t) {
  return __builtin_amdgcn_rcpf(1.0f + __expf(-t));
}
__device__ __forceinline__ float silu_f(float t) { return t * logistic_f(t); }
// d/dt SiLU = s (1 + t (1 - s)), s = logistic(t)
__device__ __forceinline__ float dsilu_f(float t) {
  const float s = logistic_f(t);
  return s * (1.0f + t * (1.0f - s));
}
__device__ __forceinline__ void silu_and_grad(float t, float& y, float& dy) {
  const float s = logistic_f(t);
  y = t * s;
  dy = s * (1.0f + t * (1.0f - s));
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
