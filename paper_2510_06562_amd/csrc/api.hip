// Library glue: error reporting, device buffers, model creation (weight re-layout) and the
// energy/force entry point.
#include <algorithm>
#include <atomic>
#include <cstdarg>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "common.h"

namespace dmts {

namespace {
thread_local char g_err[1024] = "";
}

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
}

dmts_status DevBuf::reserve(size_t need, hipStream_t s) {
  if (need <= bytes) return DMTS_OK;
  if (ptr) {
    if (hipStreamSynchronize(s) != hipSuccess) return DMTS_E_HIP;
    (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
  }
  size_t want = need + need / 4;
  if (hipMalloc(&ptr, want) != hipSuccess) {
    ptr = nullptr;
    set_error("hipMalloc of %zu bytes failed", want);
    return DMTS_E_OOM;
  }
  bytes = want;
  return DMTS_OK;
}

void DevBuf::release() {
  if (ptr) (void)hipFree(ptr);
  ptr = nullptr;
  bytes = 0;
}

// ------------------------------------------------------------------ kernel timing
namespace {
uint32_t g_prof_mask = 0;
uint32_t g_prof_every = 1;                 // time one launch in this many of a class
uint64_t g_prof_seen[DMTS_K_COUNT] = {};   // launches of each enabled class since reset
struct ProfRec {
  hipEvent_t a, b;
};
std::vector<ProfRec> g_prof[DMTS_K_COUNT];
std::vector<hipEvent_t> g_event_pool;

hipEvent_t get_event() {
  if (!g_event_pool.empty()) {
    hipEvent_t e = g_event_pool.back();
    g_event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

ProfScope::ProfScope(int kernel_class, hipStream_t stream, bool packet_launch)
    : kid(kernel_class), s(stream) {
  if (!((g_prof_mask >> kid) & 1u)) return;
  if (g_prof_seen[kid]++ % g_prof_every != 0) return;
  a = get_event();
  if (a && !packet_launch) {
    (void)hipEventRecord(a, s);
    started = true;
  }
}

ProfScope::~ProfScope() {
  if (!a) return;
  if (!started) {   // a packet launch that could not take the events: nothing timed
    g_event_pool.push_back(a);
    return;
  }
  if (!b) {
    b = get_event();
    if (!b) return;
    (void)hipEventRecord(b, s);
  }
  g_prof[kid].push_back({a, b});
}

bool ProfScope::packet(hipEvent_t& start, hipEvent_t& stop) {
  if (!a) return false;
  b = get_event();
  if (!b) return false;
  start = a;
  stop = b;
  started = true;
  return true;
}

namespace {

constexpr int kReduceThreads = 256;
constexpr int kReduceIlp = 8;
constexpr int kEChunk = kReduceThreads * kReduceIlp;   // atoms per chunk

// FP64 sum of atom_e[base .. end) (end - base <= kEChunk) in a fixed order: lane t adds
// elements t + 256 j into accumulator j, the eight accumulators pairwise, a butterfly
// within each wave, then the four wave sums in order.  Valid in thread 0.
__device__ double chunk_sum(const float* __restrict__ atom_e, int base, int end, double* wsum) {
  double a[kReduceIlp];
#pragma unroll
  for (int j = 0; j < kReduceIlp; ++j) {
    const int k = base + (int)threadIdx.x + j * kReduceThreads;
    a[j] = k < end ? (double)atom_e[k] : 0.0;
  }
  double acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  __syncthreads();   // wsum may still be read for the previous chunk
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = acc;
  __syncthreads();
  double e = 0.0;
  for (int w = 0; w < kReduceThreads / 64; ++w) e += wsum[w];
  return e;
}

// energy[s] = sum of atom_e over system s, float64: the chunk sums of the system (chunks of
// kEChunk atoms from its first atom) added in order.  The order depends only on the
// position within the system, so a system sums to the same bits alone or inside a batch,
// and whether its chunks are summed by one work-group (here) or by one each
// (k_energy_chunks and k_energy_final).
__global__ void __launch_bounds__(kReduceThreads)
k_reduce_energy(const float* __restrict__ atom_e, int n, const int32_t* __restrict__ offs,
                double* __restrict__ energy) {
  __shared__ double wsum[kReduceThreads / 64];
  const int sys = blockIdx.x;
  const int lo = offs ? max(0, offs[sys]) : 0;
  const int hi = offs ? min(n, offs[sys + 1]) : n;
  double e = 0.0;
  for (int base = lo; base < hi; base += kEChunk) e += chunk_sum(atom_e, base, min(hi, base + kEChunk), wsum);
  if (threadIdx.x == 0) energy[sys] = e;
}

__global__ void __launch_bounds__(kReduceThreads)
k_energy_chunks(const float* __restrict__ atom_e, int n, double* __restrict__ partial) {
  __shared__ double wsum[kReduceThreads / 64];
  const int base = blockIdx.x * kEChunk;
  const double e = chunk_sum(atom_e, base, min(n, base + kEChunk), wsum);
  if (threadIdx.x == 0) partial[blockIdx.x] = e;
}

__global__ void k_energy_final(const double* __restrict__ partial, int nc,
                               double* __restrict__ energy) {
  if (threadIdx.x != 0) return;
  double e = 0.0;
  for (int k = 0; k < nc; ++k) e += partial[k];
  energy[0] = e;
}

}  // namespace

int resident_groups(const void* kernel, int threads) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, int> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find({dev, kernel});
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  const int r = per_cu * cus;
  cache[{dev, kernel}] = r;
  return r;
}

size_t energy_partials(int32_t n) { return (size_t)(n + kEChunk - 1) / kEChunk + 1; }

dmts_status reduce_energy(const float* atom_e, int32_t n, const int32_t* sys_offsets,
                          int32_t n_sys, double* energy, double* partial, hipStream_t s) {
  const int ns = sys_offsets ? n_sys : 1;
  if (ns <= 0) return DMTS_OK;
  const int nc = (n + kEChunk - 1) / kEChunk;
  if (!sys_offsets && nc > 1 && partial) {
    // one system of several chunks: a work-group per chunk, then their sum in order
    k_energy_chunks<<<nc, kReduceThreads, 0, s>>>(atom_e, n, partial);
    k_energy_final<<<1, 64, 0, s>>>(partial, nc, energy);
  } else {
    k_reduce_energy<<<ns, kReduceThreads, 0, s>>>(atom_e, n, sys_offsets, energy);
  }
  DMTS_CHECK_LAUNCH();
  return DMTS_OK;
}

}  // namespace dmts

using dmts::Model;
using dmts::NList;

namespace {

// Weight tensors of the flat blob, row-major, in the documented order.
struct Blob {
  const float* p;
  size_t o = 0;
  const float* take(size_t n) {
    const float* r = p + o;
    o += n;
    return r;
  }
};

// Round to nearest even, to bfloat16 bits (finite inputs).
uint16_t bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  return static_cast<uint16_t>(u >> 16);
}

float bf16_round(float f) {
  uint32_t u = static_cast<uint32_t>(bf16_bits(f)) << 16;
  float r;
  std::memcpy(&r, &u, 4);
  return r;
}

std::vector<float> rounded(std::vector<float> v) {
  for (auto& x : v) x = bf16_round(x);
  return v;
}

// Append a [rows][cols] float matrix as bfloat16 (rows = outputs, cols = inputs).
void append16(std::vector<uint16_t>& dst, size_t& off, const std::vector<float>& src) {
  off = dst.size();
  for (float x : src) dst.push_back(bf16_bits(x));
  while (dst.size() % 128) dst.push_back(0);
}

// Three bfloat16 terms per value, stored as three consecutive tensors: x = t1 + t2 + t3
// exactly for finite x (t1 = bf16(x), t2 = bf16(x - t1), t3 = bf16(x - t1 - t2)).
void append16_terms3(std::vector<uint16_t>& dst, size_t& off, const std::vector<float>& src) {
  off = dst.size();
  std::vector<float> r = src;
  for (int t = 0; t < 3; ++t)
    for (float& x : r) {
      const float h = bf16_round(x);
      dst.push_back(bf16_bits(x));
      x -= h;
    }
  while (dst.size() % 128) dst.push_back(0);
}

void append(std::vector<float>& dst, size_t& off, const std::vector<float>& src) {
  off = dst.size();
  dst.insert(dst.end(), src.begin(), src.end());
  while (dst.size() % 64) dst.push_back(0.f);   // keep every tensor 256-byte aligned
}

// (rows x cols) row-major -> (cols x rows) row-major, for the column range [c0, c0+nc).
std::vector<float> transpose_block(const float* W, int rows, int cols, int c0, int nc) {
  std::vector<float> t((size_t)nc * rows);
  for (int r = 0; r < rows; ++r)
    for (int c = 0; c < nc; ++c) t[(size_t)c * rows + r] = W[(size_t)r * cols + c0 + c];
  return t;
}

// Species tables: T[z][c] = scale sum_e W[c][c0 + e] emb[z][e]  (float64 accumulation)
std::vector<float> species_table(const float* W, int F, int cols, int c0, const float* emb,
                                 int Z, int D, double scale = 1.0) {
  std::vector<float> t((size_t)Z * F);
  for (int z = 0; z < Z; ++z)
    for (int c = 0; c < F; ++c) {
      double acc = 0.0;
      for (int e = 0; e < D; ++e) acc += (double)W[(size_t)c * cols + c0 + e] * emb[z * D + e];
      t[(size_t)z * F + c] = (float)(scale * acc);
    }
  return t;
}

// The two-interaction model's pair kernels take every term of the message pre-activation
// a_ij (the radial weights W_b, the species tables of interaction 1 and the [A | B]
// projection of interaction 2) multiplied by -log2(e), so that e^-a is one exp2 of what
// they accumulate; they undo the factor where SiLU(a) leaves the kernel.
constexpr double kNegLog2e = -1.4426950408889634;

std::vector<float> scaled(std::vector<float> v, double k) {
  for (auto& x : v) x = (float)(k * (double)x);
  return v;
}

}  // namespace


extern "C" const char* dmts_last_error(void) { return dmts::g_err; }

extern "C" const char* dmts_version(void) { return "dmts-mi355x 0.1 (gfx950)"; }

extern "C" dmts_status nnp_model_create(const nnp_model_desc* desc, const float* host_weights,
                                        int64_t n_weights, nnp_model** out) {
  DMTS_REQUIRE(desc && host_weights && out, DMTS_E_ARG, "nnp_model_create: null argument");
  *out = nullptr;
  const nnp_model_desc d = *desc;
  const int K = d.n_rbf, F = d.width, D = d.emb_dim, Z = d.n_species;
  DMTS_REQUIRE(d.kind == NNP_KIND_ONE_INTERACTION || d.kind == NNP_KIND_TWO_INTERACTION,
               DMTS_E_ARG, "nnp_model_create: unknown kind %d", d.kind);
  DMTS_REQUIRE(d.precision == NNP_PREC_FP32 || d.precision == NNP_PREC_BF16, DMTS_E_ARG,
               "nnp_model_create: unknown precision %d", d.precision);
  DMTS_REQUIRE(D == 16 && Z >= 1 && Z <= 8, DMTS_E_ARG,
               "nnp_model_create: need emb_dim 16 and 1..8 species (got %d, %d)", D, Z);
  if (d.kind == NNP_KIND_ONE_INTERACTION)
    DMTS_REQUIRE(K == 16 && F == 64, DMTS_E_ARG,
                 "nnp_model_create: one-interaction model supports K=16, F=64 (got %d, %d)", K, F);
  else
    DMTS_REQUIRE(K == 32 && F == 128, DMTS_E_ARG,
                 "nnp_model_create: two-interaction model supports K=32, F=128 (got %d, %d)", K, F);
  DMTS_REQUIRE(d.cutoff > 0.0 && d.cutoff < 1e3, DMTS_E_ARG, "nnp_model_create: bad cutoff");
  size_t expect;
  if (d.kind == NNP_KIND_ONE_INTERACTION)
    expect = (size_t)Z * D + (size_t)F * (K + 2 * D) + (size_t)F * F + F;
  else
    expect = (size_t)Z * D + (size_t)F * (K + 2 * D) + 2 * (size_t)F * 3 * F +
             (size_t)F * (K + 2 * F) + (size_t)F * F + F;
  DMTS_REQUIRE((size_t)n_weights == expect, DMTS_E_ARG,
               "nnp_model_create: %lld weights given, %zu expected", (long long)n_weights, expect);

  Model* m = new Model();
  static std::atomic<uint64_t> next_generation{1};
  m->generation = next_generation.fetch_add(1);
  m->desc = d;
  m->K = K;
  m->F = F;
  m->D = D;
  m->Z = Z;
  m->rc = (float)d.cutoff;
  m->sigma = (float)(d.cutoff / (K - 1));
  m->escale = (float)d.energy_scale;
  Blob b{host_weights};
  std::vector<float> P;
  const float* emb = b.take((size_t)Z * D);
  if (d.kind == NNP_KIND_ONE_INTERACTION) {
    const int cols = K + 2 * D;
    const float* Wp = b.take((size_t)F * cols);
    const float* W1 = b.take((size_t)F * F);
    const float* w2 = b.take(F);
    append(P, m->o_WbT, transpose_block(Wp, F, cols, 0, K));
    append(P, m->o_Td, species_table(Wp, F, cols, K, emb, Z, D));
    append(P, m->o_Ts, species_table(Wp, F, cols, K + D, emb, Z, D));
    append(P, m->o_W1, std::vector<float>(W1, W1 + (size_t)F * F));
    append(P, m->o_W1T, transpose_block(W1, F, F, 0, F));
    append(P, m->o_w2, std::vector<float>(w2, w2 + F));
  } else {
    const int cols1 = K + 2 * D, cols2 = K + 2 * F, Q = 3 * F;
    const float* Wp1 = b.take((size_t)F * cols1);
    const float* U1 = b.take((size_t)F * Q);
    const float* Wp2 = b.take((size_t)F * cols2);
    const float* U2 = b.take((size_t)F * Q);
    const float* Wo = b.take((size_t)F * F);
    const float* wo = b.take(F);
    append(P, m->o_Td, species_table(Wp1, F, cols1, K, emb, Z, D, kNegLog2e));
    append(P, m->o_Ts, species_table(Wp1, F, cols1, K + D, emb, Z, D, kNegLog2e));
    append(P, m->o_U1T, transpose_block(U1, F, Q, 0, Q));
    append(P, m->o_U1, std::vector<float>(U1, U1 + (size_t)F * Q));
    append(P, m->o_U2T, transpose_block(U2, F, Q, 0, Q));
    append(P, m->o_U2, std::vector<float>(U2, U2 + (size_t)F * Q));
    // [A | B] projection as [out][in]: row n < F is W_pair2[n][K+F+.] (sender), row F + n
    // is W_pair2[n][K+.] (receiver); reverse pass dh[e] = sum_c R[c] W_pair2[c][K+e] +
    // sum_c S[c] W_pair2[c][K+F+e], as [out = e][in = 2F].
    std::vector<float> W2h((size_t)2 * F * F), W2hs((size_t)F * 2 * F);
    for (int nn = 0; nn < 2 * F; ++nn)
      for (int k = 0; k < F; ++k)
        W2h[(size_t)nn * F + k] = nn < F ? Wp2[(size_t)nn * cols2 + K + F + k]
                                         : Wp2[(size_t)(nn - F) * cols2 + K + k];
    for (int e = 0; e < F; ++e)
      for (int k = 0; k < 2 * F; ++k)
        W2hs[(size_t)e * 2 * F + k] = k < F ? Wp2[(size_t)k * cols2 + K + e]
                                            : Wp2[(size_t)(k - F) * cols2 + K + F + e];
    append(P, m->o_W2h, scaled(W2h, kNegLog2e));
    append(P, m->o_W2hs, W2hs);
    append(P, m->o_WoT, transpose_block(Wo, F, F, 0, F));
    append(P, m->o_Wo, std::vector<float>(Wo, Wo + (size_t)F * F));
    append(P, m->o_wo, std::vector<float>(wo, wo + F));
  }
  std::vector<uint16_t> H;
  if (d.precision == NNP_PREC_BF16) {
    m->bf16 = true;
    if (d.kind == NNP_KIND_ONE_INTERACTION) {
      // the fast model's contractions run on the vector units with bfloat16-valued operands
      const float* Wp = host_weights + (size_t)Z * D;
      const float* W1 = Wp + (size_t)F * (K + 2 * D);
      append(P, m->o_WbR, rounded(transpose_block(Wp, F, K + 2 * D, 0, K)));
      append(P, m->o_W1R, rounded(std::vector<float>(W1, W1 + (size_t)F * F)));
      append(P, m->o_W1TR, rounded(transpose_block(W1, F, F, 0, F)));
    } else {
      const int cols1 = K + 2 * D, cols2 = K + 2 * F, Q = 3 * F;
      const float* Wp1 = host_weights + (size_t)Z * D;
      const float* U1 = Wp1 + (size_t)F * cols1;
      const float* Wp2 = U1 + (size_t)F * Q;
      const float* U2 = Wp2 + (size_t)F * cols2;
      const float* Wo = U2 + (size_t)F * Q;
      auto block = [](const float* W, int rows, int cols, int c0, int nc) {
        std::vector<float> t((size_t)rows * nc);
        for (int r = 0; r < rows; ++r)
          for (int c = 0; c < nc; ++c) t[(size_t)r * nc + c] = W[(size_t)r * cols + c0 + c];
        return t;
      };
      append16(H, m->h_Wb1, scaled(block(Wp1, F, cols1, 0, K), kNegLog2e));
      append16(H, m->h_Wb2, scaled(block(Wp2, F, cols2, 0, K), kNegLog2e));
      append16(H, m->h_U1, std::vector<float>(U1, U1 + (size_t)F * Q));            // [F][3F]
      std::vector<float> W2h((size_t)2 * F * F), W2hs((size_t)F * 2 * F);
      for (int nn = 0; nn < 2 * F; ++nn)                                              // [2F][F]
        for (int k = 0; k < F; ++k)
          W2h[(size_t)nn * F + k] = nn < F ? Wp2[(size_t)nn * cols2 + K + F + k]
                                           : Wp2[(size_t)(nn - F) * cols2 + K + k];
      for (int e = 0; e < F; ++e)                                                      // [F][2F]
        for (int k = 0; k < 2 * F; ++k)
          W2hs[(size_t)e * 2 * F + k] = k < F ? Wp2[(size_t)k * cols2 + K + e]
                                              : Wp2[(size_t)(k - F) * cols2 + K + F + e];
      append16(H, m->h_W2h, scaled(W2h, kNegLog2e));
      append16(H, m->h_U2, std::vector<float>(U2, U2 + (size_t)F * Q));
      append16(H, m->h_Wo, std::vector<float>(Wo, Wo + (size_t)F * F));
      append16(H, m->h_WoT, transpose_block(Wo, F, F, 0, F));
      append16(H, m->h_U2T, transpose_block(U2, F, Q, 0, Q));                         // [3F][F]
      append16(H, m->h_W2hs, W2hs);
      append16(H, m->h_U1T, transpose_block(U1, F, Q, 0, Q));
    }
  }
  if (d.kind == NNP_KIND_TWO_INTERACTION && d.precision == NNP_PREC_FP32) {
    // FP32 form: the radial blocks W_pair[:, :K] as three bfloat16 terms ([3][F][K])
    const int cols1 = K + 2 * D, cols2 = K + 2 * F, Q = 3 * F;
    const float* Wp1 = host_weights + (size_t)Z * D;
    const float* Wp2 = Wp1 + (size_t)F * cols1 + (size_t)F * Q;
    std::vector<float> b1((size_t)F * K), b2((size_t)F * K);
    for (int c = 0; c < F; ++c)
      for (int k = 0; k < K; ++k) {
        b1[(size_t)c * K + k] = Wp1[(size_t)c * cols1 + k];
        b2[(size_t)c * K + k] = Wp2[(size_t)c * cols2 + k];
      }
    append16_terms3(H, m->h_Wb1, scaled(b1, kNegLog2e));
    append16_terms3(H, m->h_Wb2, scaled(b2, kNegLog2e));
  }
  if (m->params.reserve(P.size() * sizeof(float), nullptr) != DMTS_OK) {
    delete m;
    return DMTS_E_OOM;
  }
  hipError_t e = hipMemcpy(m->params.ptr, P.data(), P.size() * sizeof(float),
                           hipMemcpyHostToDevice);
  if (e == hipSuccess && !H.empty()) {
    if (m->params16.reserve(H.size() * sizeof(uint16_t), nullptr) != DMTS_OK) e = hipErrorOutOfMemory;
    else e = hipMemcpy(m->params16.ptr, H.data(), H.size() * sizeof(uint16_t), hipMemcpyHostToDevice);
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    dmts::set_error("nnp_model_create: %s", hipGetErrorString(e));
    m->params.release();
    m->params16.release();
    delete m;
    return DMTS_E_HIP;
  }
  *out = reinterpret_cast<nnp_model*>(m);
  return DMTS_OK;
}

extern "C" void nnp_model_destroy(nnp_model* h) {
  Model* m = reinterpret_cast<Model*>(h);
  if (!m) return;
  (void)hipDeviceSynchronize();
  m->params.release();
  m->params16.release();
  m->atom_ws.release();
  m->pair_ws.release();
  m->sys_ws.release();
  delete m;
}

namespace dmts {
dmts_status energy_forces(Model* m, NList* nl, const double* pos, const int32_t* species,
                          int32_t n, double box, const int32_t* sys_offsets, int32_t n_sys,
                          double* energy, float* forces, float* atom_energy, hipStream_t s,
                          const Epilogue* ep, char* ws) {
  DMTS_REQUIRE(m && nl && pos && species, DMTS_E_ARG, "nnp_energy_forces: null argument");
  DMTS_REQUIRE(!ws || m->desc.kind == NNP_KIND_ONE_INTERACTION, DMTS_E_ARG,
               "energy_forces: a caller workspace is for one-interaction models");
  DMTS_REQUIRE(!ep || forces, DMTS_E_ARG, "energy_forces: an integrator epilogue needs forces");
  DMTS_REQUIRE(n == nl->n_atoms, DMTS_E_STATE,
               "nnp_energy_forces: list built for %d atoms, called with %d", nl->n_atoms, n);
  DMTS_REQUIRE(box == nl->box, DMTS_E_STATE, "nnp_energy_forces: list built for another box");
  DMTS_REQUIRE(nl->cutoff >= (double)m->desc.cutoff, DMTS_E_STATE,
               "nnp_energy_forces: list cutoff %g below the model cutoff %g", nl->cutoff,
               m->desc.cutoff);
  DMTS_REQUIRE(sys_offsets == nullptr || n_sys >= 1, DMTS_E_ARG,
               "nnp_energy_forces: n_sys must be >= 1 with sys_offsets");
  if (m->desc.kind == NNP_KIND_ONE_INTERACTION)
    return small_energy_forces(m, nl, pos, species, n, box, sys_offsets, n_sys, energy, forces,
                               atom_energy, s, ep, ws);
  return large_energy_forces(m, nl, pos, species, n, box, sys_offsets, n_sys, energy, forces,
                             atom_energy, s, ep);
}
}  // namespace dmts

extern "C" dmts_status nnp_energy_forces(nnp_model* model, nnp_nlist* nl, const double* pos,
                                         const int32_t* species, int32_t n_atoms, double box,
                                         const int32_t* sys_offsets, int32_t n_sys,
                                         double* energy, float* forces, float* atom_energy,
                                         void* stream) {
  return dmts::energy_forces(reinterpret_cast<Model*>(model), reinterpret_cast<NList*>(nl), pos,
                             species, n_atoms, box, sys_offsets, n_sys, energy, forces,
                             atom_energy, static_cast<hipStream_t>(stream));
}

extern "C" dmts_status dmts_prof_enable(uint32_t class_mask) {
  dmts::g_prof_mask = class_mask;
  return DMTS_OK;
}

extern "C" dmts_status dmts_prof_sample(uint32_t every) {
  DMTS_REQUIRE(every >= 1, DMTS_E_ARG, "dmts_prof_sample: every must be >= 1");
  dmts::g_prof_every = every;
  return DMTS_OK;
}

extern "C" dmts_status dmts_prof_reset(void) {
  for (auto& c : dmts::g_prof_seen) c = 0;
  for (auto& v : dmts::g_prof) {
    for (auto& r : v) {
      (void)hipEventSynchronize(r.b);
      dmts::g_event_pool.push_back(r.a);
      dmts::g_event_pool.push_back(r.b);
    }
    v.clear();
  }
  return DMTS_OK;
}

extern "C" dmts_status dmts_prof_read(int32_t kernel_class, double* total_ms, int64_t* launches) {
  DMTS_REQUIRE(kernel_class >= 0 && kernel_class < DMTS_K_COUNT && total_ms && launches,
               DMTS_E_ARG, "dmts_prof_read: bad argument");
  double t = 0.0;
  for (auto& r : dmts::g_prof[kernel_class]) {
    DMTS_HIP(hipEventSynchronize(r.b));
    float ms = 0.f;
    DMTS_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    t += ms;
  }
  *total_ms = t;
  *launches = (int64_t)dmts::g_prof[kernel_class].size();
  return DMTS_OK;
}

namespace {

bool valid_shape(const nnp_tile_shape& t) {
  return (t.receivers_per_group == 2 || t.receivers_per_group == 4 ||
          t.receivers_per_group == 8) &&
         (t.atom_tiles == 1 || t.atom_tiles == 2) &&
         (t.keep_derivatives == 0 || t.keep_derivatives == 1) && t.work_groups >= 0;
}

dmts::TileShape to_internal(const nnp_tile_shape& t) {
  dmts::TileShape s;
  s.nw = t.receivers_per_group;
  s.rt = t.atom_tiles;
  s.keep = t.keep_derivatives;
  s.grid = t.work_groups;
  return s;
}

nnp_tile_shape to_abi(const dmts::TileShape& s) {
  return nnp_tile_shape{s.nw, s.rt, s.keep, s.grid};
}

}  // namespace

extern "C" dmts_status nnp_model_set_grid(nnp_model* h, int32_t work_groups) {
  Model* m = reinterpret_cast<Model*>(h);
  DMTS_REQUIRE(m && work_groups >= 0, DMTS_E_ARG, "nnp_model_set_grid: bad argument");
  m->shape.grid = work_groups;
  for (auto& kv : m->tuned) kv.second.grid = work_groups;
  return DMTS_OK;
}

extern "C" dmts_status nnp_model_get_grid(nnp_model* h, int32_t* work_groups) {
  Model* m = reinterpret_cast<Model*>(h);
  DMTS_REQUIRE(m && work_groups, DMTS_E_ARG, "nnp_model_get_grid: bad argument");
  *work_groups = m->shape.grid;
  return DMTS_OK;
}

extern "C" dmts_status nnp_model_set_shape(nnp_model* h, int32_t n_atoms,
                                           const nnp_tile_shape* shape) {
  Model* m = reinterpret_cast<Model*>(h);
  DMTS_REQUIRE(m && shape, DMTS_E_ARG, "nnp_model_set_shape: null argument");
  DMTS_REQUIRE(valid_shape(*shape), DMTS_E_ARG,
               "nnp_model_set_shape: receivers_per_group must be 2, 4 or 8, atom_tiles 1 or 2, "
               "keep_derivatives 0 or 1, work_groups >= 0 (got %d, %d, %d, %d)",
               shape->receivers_per_group, shape->atom_tiles, shape->keep_derivatives,
               shape->work_groups);
  if (n_atoms <= 0) {
    m->shape = to_internal(*shape);
    m->tuned.clear();
  } else {
    m->tuned[Model::size_bucket(n_atoms)] = to_internal(*shape);
  }
  return DMTS_OK;
}

extern "C" dmts_status nnp_model_get_shape(nnp_model* h, int32_t n_atoms, nnp_tile_shape* shape) {
  Model* m = reinterpret_cast<Model*>(h);
  DMTS_REQUIRE(m && shape, DMTS_E_ARG, "nnp_model_get_shape: null argument");
  *shape = to_abi(n_atoms > 0 ? m->shape_for(n_atoms) : m->shape);
  return DMTS_OK;
}

// Times one energy+force evaluation per candidate tile shape (median of `reps` after one
// warm-up) with HIP events on `stream`, and keeps the fastest as the model's shape for the
// size bucket of n_atoms.
extern "C" dmts_status nnp_autotune(nnp_model* h, nnp_nlist* nlh, const double* pos,
                                    const int32_t* species, int32_t n_atoms, double box,
                                    const int32_t* sys_offsets, int32_t n_sys, int32_t reps,
                                    void* stream, nnp_tile_shape* chosen, double* best_ms) {
  Model* m = reinterpret_cast<Model*>(h);
  NList* nl = reinterpret_cast<NList*>(nlh);
  DMTS_REQUIRE(m && nl && reps >= 1 && reps <= 64 && n_atoms >= 1, DMTS_E_ARG,
               "nnp_autotune: bad argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  // candidates: the shapes the model's kernels take, times persistent grids (0 = natural,
  // then multiples of the 256 compute units)
  std::vector<dmts::TileShape> cands;
  const int32_t grids[] = {0, 256, 512, 1024, 2048, 4096};
  for (int32_t gsz : grids) {
    dmts::TileShape t;
    t.grid = gsz;
    if (m->desc.kind == NNP_KIND_TWO_INTERACTION) {
      for (int nw : {2, 4, 8})
        for (int rt : {1, 2}) {
          t.nw = nw;
          t.rt = rt;
          cands.push_back(t);
        }
    } else {
      for (int keep : {0, 1}) {
        t.keep = keep;
        cands.push_back(t);
      }
    }
  }
  const int ns = sys_offsets ? n_sys : 1;
  double* energy = nullptr;
  float* forces = nullptr;
  DMTS_HIP(hipMalloc(&energy, sizeof(double) * ns));
  if (hipMalloc(&forces, sizeof(float) * 3 * (size_t)n_atoms) != hipSuccess) {
    (void)hipFree(energy);
    dmts::set_error("nnp_autotune: allocation failed");
    return DMTS_E_OOM;
  }
  hipEvent_t e0, e1;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const int bucket = Model::size_bucket(n_atoms);
  const std::map<int, dmts::TileShape> saved = m->tuned;
  dmts::TileShape best = m->shape_for(n_atoms);
  double best_t = 1e300;
  dmts_status st = DMTS_OK;
  for (const dmts::TileShape& c : cands) {
    m->tuned[bucket] = c;
    std::vector<double> t;
    constexpr int kBatch = 4;   // evaluations per timing
    for (int r = 0; r <= reps && st == DMTS_OK; ++r) {
      (void)hipEventRecord(e0, s);
      for (int b = 0; b < kBatch && st == DMTS_OK; ++b)
        st = dmts::energy_forces(m, nl, pos, species, n_atoms, box, sys_offsets, n_sys,
                                 energy, forces, nullptr, s);
      (void)hipEventRecord(e1, s);
      if (st != DMTS_OK) break;
      if (hipEventSynchronize(e1) != hipSuccess) {
        st = DMTS_E_HIP;
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (r > 0) t.push_back(ms / kBatch);   // the first timing warms up
    }
    if (st != DMTS_OK) break;
    std::sort(t.begin(), t.end());
    const double med = t[t.size() / 2];
    if (med < best_t) {
      best_t = med;
      best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(energy);
  (void)hipFree(forces);
  m->tuned = saved;
  if (st != DMTS_OK) return st;
  m->tuned[bucket] = best;
  if (chosen) *chosen = to_abi(best);
  if (best_ms) *best_ms = best_t;
  return DMTS_OK;
}
