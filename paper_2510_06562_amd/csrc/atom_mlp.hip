// Per-atom dense layers of the reference potential as fused MFMA chains.
//
// Every per-atom layer is a row-local contraction [rows x K] * [K x N], so the whole chain
// of layers between two pair kernels runs in one launch: a work-group owns RT = 2 tiles of
// 16 atoms (each weight load feeds both tiles), keeps the activations of its atoms in LDS
// between layers and streams the weights (at most 384 x 384, L2-resident) from global
// memory.  The weight stream, not the products, bounds a 16-atom work-group in the FP32
// form, so both forms take 32 atoms.  Contractions use v_mfma_f32_16x16x4_f32; the
// sixteen waves of the work-group take eight 16-column blocks at a time, each block in two
// halves of K (waves w and w + 8): the second half's accumulators go through LDS and the
// first half adds them (a fixed order) and runs the layer's epilogue.  Four waves per SIMD
// hide the latency of the weight stream that two could not, and each weight is still
// loaded once per work-group.  A row's result does not depend on its tile or work-group.
//
//   chain 1 (after interaction 1):  z1 = U1 q1, h1 = SiLU(z1), [A|B] = [W_s|W_r] h1
//   chain 2 (after interaction 2):  z2 = U2 q2, h2 = h1 + SiLU(z2), y = W_o h2,
//                                   E = s_E w_o . SiLU(y), dy = s_E w_o SiLU'(y),
//                                   dh2 = W_o^T dy, dz2 = dh2 SiLU'(z2), dq2 = U2^T dz2
//   chain 3 (after the sender sums): dh1 = dh2 + W_r^T R + W_s^T S, dz1 = dh1 SiLU'(z1),
//                                   dq1 = U1^T dz1
//
// In the BF16 form (weights given as bfloat16 [out][in]) the contractions run on
// v_mfma_f32_16x16x32_bf16 with the activations rounded to bfloat16 as they are read.
//
// MFMA 16x16x4 f32 register layout:
//   A operand: lane l holds A[l % 16][k0 + l / 16]
//   B operand: lane l holds B[k0 + l / 16][l % 16]
//   D: lane l, register r holds D[4 (l / 16) + r][l % 16]
#include "atom_mlp.h"

namespace dmts {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 1024;  // sixteen waves: two K halves of eight column blocks
constexpr int kHalfWaves = kThreads / 128;
constexpr int kRT = 2;       // 16-atom tiles per work-group
constexpr int kLd = 388;     // LDS row stride (floats) for activations up to 384 wide

template <int RT>
struct AccT {
  f32x4 v[RT];   // tile t: rows 16 t .. 16 t + 15
};

// acc[16 x 16] blocks (one per row tile) = X[16 RT x K] (LDS, stride kLd) * W^T with
// W [N x K] FP32 (global, input index contiguous), columns n0 .. n0+15.  In each 32-wide
// slice of K, step s of group g takes k = 8 g + s (both operands agree), so a lane reads
// its eight X and eight W values as two 16-byte loads each.
template <int RT>
__device__ __forceinline__ AccT<RT> mfma_block(const float* X, int K, int kb, int ke,
                                               const float* __restrict__ W, int n0, int lane) {
  AccT<RT> acc;
#pragma unroll
  for (int t = 0; t < RT; ++t) acc.v[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int r = lane & 15, g = lane >> 4;
  const float* xp = X + r * kLd + 8 * g;
  const float* wp = W + (size_t)(n0 + r) * K + 8 * g;
#pragma unroll 4
  for (int k0 = kb; k0 < ke; k0 += 32) {
    const float4 w0 = *reinterpret_cast<const float4*>(wp + k0);
    const float4 w1 = *reinterpret_cast<const float4*>(wp + k0 + 4);
    const float wv[8] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const float4 x0 = *reinterpret_cast<const float4*>(xp + 16 * t * kLd + k0);
      const float4 x1 = *reinterpret_cast<const float4*>(xp + 16 * t * kLd + k0 + 4);
      const float xv[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
      for (int s = 0; s < 8; ++s)
        acc.v[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(xv[s], wv[s], acc.v[t], 0, 0, 0);
    }
  }
  return acc;
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// BF16 form: acc[16 x 16] blocks = X[16 RT x K] * W^T with W [N x K] bfloat16 (input
// index contiguous), on v_mfma_f32_16x16x32_bf16:
//   A operand: lane l holds A[l % 16][k0 + 8 (l / 16) + e], e = 0..7
//   B operand: lane l holds B[k0 + 8 (l / 16) + e][l % 16]
// X is rounded to bfloat16 (nearest even) as it is read; accumulation is FP32.
template <int RT>
__device__ __forceinline__ AccT<RT> mfma_block_bf16(const float* X, int K, int kb, int ke,
                                                    const __bf16* __restrict__ W, int n0,
                                                    int lane) {
  AccT<RT> acc;
#pragma unroll
  for (int t = 0; t < RT; ++t) acc.v[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int r = lane & 15, g = lane >> 4;
  const float* xp = X + r * kLd + 8 * g;
  const __bf16* wp = W + (size_t)(n0 + r) * K + 8 * g;
#pragma unroll 4
  for (int k0 = kb; k0 < ke; k0 += 32) {
    const bf16x8 b = *reinterpret_cast<const bf16x8*>(wp + k0);
#pragma unroll
    for (int t = 0; t < RT; ++t) {
      const float4 x0 = *reinterpret_cast<const float4*>(xp + 16 * t * kLd + k0);
      const float4 x1 = *reinterpret_cast<const float4*>(xp + 16 * t * kLd + k0 + 4);
      bf16x8 a;
      a[0] = (__bf16)x0.x; a[1] = (__bf16)x0.y; a[2] = (__bf16)x0.z; a[3] = (__bf16)x0.w;
      a[4] = (__bf16)x1.x; a[5] = (__bf16)x1.y; a[6] = (__bf16)x1.z; a[7] = (__bf16)x1.w;
      acc.v[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc.v[t], 0, 0, 0);
    }
  }
  return acc;
}

// Weights of one layer, [N][K]: FP32 or BF16.
struct LayerW {
  const float* f32;
  const __bf16* b16;
};

// Runs one layer: for every 16-column block of N, in rounds of eight blocks, the two
// waves of the block sum their K halves and the first calls epi(row, col, value) for the
// lane's four outputs.  `part` (LDS, 8 RT 64 f32x4) holds the second halves of a round.
template <int RT, class Epi>
__device__ __forceinline__ void layer(f32x4* part, const float* X, int K, LayerW Wt, int N,
                                      Epi&& epi) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int kh = wave / kHalfWaves, wl = wave % kHalfWaves;
  const int kb = kh * (K / 2), ke = kb + K / 2;
  for (int base = 0; base < N / 16; base += kHalfWaves) {   // uniform over the work-group
    const int nb = base + wl;
    AccT<RT> acc;
    if (nb < N / 16)
      acc = Wt.b16 ? mfma_block_bf16<RT>(X, K, kb, ke, Wt.b16, nb * 16, lane)
                   : mfma_block<RT>(X, K, kb, ke, Wt.f32, nb * 16, lane);
    if (kh == 1 && nb < N / 16)
#pragma unroll
      for (int t = 0; t < RT; ++t) part[(wl * RT + t) * 64 + lane] = acc.v[t];
    __syncthreads();
    if (kh == 0 && nb < N / 16) {
#pragma unroll
      for (int t = 0; t < RT; ++t) {
        const f32x4 o = part[(wl * RT + t) * 64 + lane];
#pragma unroll
        for (int r = 0; r < 4; ++r)
          epi(16 * t + 4 * (lane >> 4) + r, nb * 16 + (lane & 15), acc.v[t][r] + o[r]);
      }
    }
    __syncthreads();
  }
}

// Stage rows [m0, m0 + kRows) of a global row-major array (ld floats, K used; K and ld
// multiples of 4) into LDS with row stride `xld`, in two halves: load() issues the thread's
// 16-byte loads, store() writes them, so that the loads of several arrays are in flight
// together (one memory round trip).
template <int K, int kRows>
struct RowStage {
  static constexpr int kV = kRows * K / 4, kPer = (kV + kThreads - 1) / kThreads;
  float4 t[kPer];
  __device__ __forceinline__ void load(const float* __restrict__ G, int ld, int m0, int M) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = threadIdx.x + u * kThreads, r = e / (K / 4), k4 = e % (K / 4);
      t[u] = e < kV && (m0 + r) < M
                 ? *reinterpret_cast<const float4*>(G + (size_t)(m0 + r) * ld + 4 * k4)
                 : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }
  __device__ __forceinline__ void store(float* X, int xld) const {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = threadIdx.x + u * kThreads, r = e / (K / 4), k4 = e % (K / 4);
      if (e < kV) *reinterpret_cast<float4*>(X + r * xld + 4 * k4) = t[u];
    }
  }
};

template <int RT>
__global__ void __launch_bounds__(kThreads)
k_chain1(AtomMlpParams P, int M, const float* __restrict__ q1, float* __restrict__ z1,
         float* __restrict__ h1, float* __restrict__ P2) {
  constexpr int kRows = 16 * RT;
  __shared__ f32x4 part[kHalfWaves * RT * 64];   // K-half partial sums of a layer
  __shared__ float X[kRows * kLd];
  __shared__ float H[kRows * kLd];
  const int m0 = blockIdx.x * kRows;
  {
    RowStage<384, kRows> a;
    a.load(q1, 384, m0, M);
    a.store(X, kLd);
  }
  __syncthreads();
  layer<RT>(part, X, 384, LayerW{P.U1, P.h_U1}, 128, [&](int r, int c, float v) {
    const float h = silu_f(v);
    H[r * kLd + c] = h;
    if (m0 + r < M) {
      z1[(size_t)(m0 + r) * 128 + c] = v;
      h1[(size_t)(m0 + r) * 128 + c] = h;
    }
  });
  __syncthreads();
  layer<RT>(part, H, 128, LayerW{P.W2h, P.h_W2h}, 256, [&](int r, int c, float v) {
    if (m0 + r < M) P2[(size_t)(m0 + r) * 256 + c] = v;
  });
}

template <int RT>
__global__ void __launch_bounds__(kThreads)
k_chain2(AtomMlpParams P, int M, const float* __restrict__ q2, const float* __restrict__ h1,
         float escale, float* __restrict__ atom_e, float* __restrict__ dh2_out,
         float* __restrict__ dq2, bool backward) {
  constexpr int kRows = 16 * RT;
  __shared__ f32x4 part[kHalfWaves * RT * 64];   // K-half partial sums of a layer
  __shared__ float X[kRows * kLd];     // q2, later dz2
  __shared__ float H[kRows * kLd];     // h2, later dy
  __shared__ float Z[kRows * 128];     // z2
  __shared__ float E[kRows * 128];     // per-column energy terms of y, first h1
  const int m0 = blockIdx.x * kRows;
  {
    RowStage<384, kRows> a;
    RowStage<128, kRows> b;
    a.load(q2, 384, m0, M);
    b.load(h1, 128, m0, M);
    a.store(X, kLd);
    b.store(E, 128);
  }
  __syncthreads();
  layer<RT>(part, X, 384, LayerW{P.U2, P.h_U2}, 128, [&](int r, int c, float v) {
    Z[r * 128 + c] = v;
    H[r * kLd + c] = E[r * 128 + c] + silu_f(v);
  });
  __syncthreads();   // E (h1) is overwritten by the next layer
  __syncthreads();
  // y = W_o h2; energy terms and dy (dy overwrites the X buffer)
  layer<RT>(part, H, 128, LayerW{P.Wo, P.h_Wo}, 128, [&](int r, int c, float v) {
    float s, ds;
    silu_and_grad(v, s, ds);
    const float w = P.wo[c];
    E[r * 128 + c] = w * s;
    X[r * kLd + c] = escale * w * ds;
  });
  __syncthreads();
  // per-atom energy: fixed-order sum of 128 terms (4 lanes per row)
  if (threadIdx.x < 4 * kRows) {
    const int r = threadIdx.x >> 2, part = threadIdx.x & 3;
    float s = 0.f;
    for (int c = part * 32; c < part * 32 + 32; ++c) s += E[r * 128 + c];
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    if (part == 0 && m0 + r < M) atom_e[m0 + r] = s * escale;
  }
  if (!backward) return;
  // dh2 = W_o^T dy, dz2 = dh2 SiLU'(z2)   (dz2 goes to H)
  layer<RT>(part, X, 128, LayerW{P.WoT, P.h_WoT}, 128, [&](int r, int c, float v) {
    if (m0 + r < M) dh2_out[(size_t)(m0 + r) * 128 + c] = v;
    H[r * kLd + c] = v * dsilu_f(Z[r * 128 + c]);
  });
  __syncthreads();
  layer<RT>(part, H, 128, LayerW{P.U2T, P.h_U2T}, 384, [&](int r, int c, float v) {
    if (m0 + r < M) dq2[(size_t)(m0 + r) * 384 + c] = v;
  });
}

template <int RT>
__global__ void __launch_bounds__(kThreads)
k_chain3(AtomMlpParams P, int M, const float* __restrict__ RS, const float* __restrict__ dh2,
         const float* __restrict__ z1, float* __restrict__ dq1) {
  constexpr int kRows = 16 * RT;
  __shared__ f32x4 part[kHalfWaves * RT * 64];   // K-half partial sums of a layer
  __shared__ float X[kRows * kLd];
  __shared__ float H[kRows * kLd];
  __shared__ float D2[kRows * 128], Z1[kRows * 128];   // dh2, z1 rows
  const int m0 = blockIdx.x * kRows;
  {
    RowStage<256, kRows> a;
    RowStage<128, kRows> b, c;
    a.load(RS, 256, m0, M);
    b.load(dh2, 128, m0, M);
    c.load(z1, 128, m0, M);
    a.store(X, kLd);
    b.store(D2, 128);
    c.store(Z1, 128);
  }
  __syncthreads();
  layer<RT>(part, X, 256, LayerW{P.W2hs, P.h_W2hs}, 128, [&](int r, int c, float v) {
    const int o = r * 128 + c;
    H[r * kLd + c] = m0 + r < M ? (v + D2[o]) * dsilu_f(Z1[o]) : 0.f;
  });
  __syncthreads();
  layer<RT>(part, H, 128, LayerW{P.U1T, P.h_U1T}, 384, [&](int r, int c, float v) {
    if (m0 + r < M) dq1[(size_t)(m0 + r) * 384 + c] = v;
  });
}

}  // namespace

// rt: 16-atom tiles per work-group (1 or 2; any other value is taken as kRT).  A row's
// result does not depend on it.
dmts_status atom_chain1(const AtomMlpParams& P, int M, int rt, const float* q1, float* z1,
                        float* h1, float* P2, hipStream_t s) {
  if (M <= 0) return DMTS_OK;
  ProfScope ps(DMTS_K_ATOM_GEMM, s);
  if (rt == 1) k_chain1<1><<<ceil_div(M, 16), kThreads, 0, s>>>(P, M, q1, z1, h1, P2);
  else k_chain1<kRT><<<ceil_div(M, 16 * kRT), kThreads, 0, s>>>(P, M, q1, z1, h1, P2);
  DMTS_CHECK_LAUNCH();
  return DMTS_OK;
}

dmts_status atom_chain2(const AtomMlpParams& P, int M, int rt, const float* q2, const float* h1,
                        float escale, float* atom_e, float* dh2, float* dq2, bool backward,
                        hipStream_t s) {
  if (M <= 0) return DMTS_OK;
  ProfScope ps(DMTS_K_ATOM_GEMM, s);
  if (rt == 1)
    k_chain2<1><<<ceil_div(M, 16), kThreads, 0, s>>>(P, M, q2, h1, escale, atom_e, dh2, dq2,
                                                      backward);
  else
    k_chain2<kRT><<<ceil_div(M, 16 * kRT), kThreads, 0, s>>>(P, M, q2, h1, escale, atom_e, dh2,
                                                             dq2, backward);
  DMTS_CHECK_LAUNCH();
  return DMTS_OK;
}

dmts_status atom_chain3(const AtomMlpParams& P, int M, int rt, const float* RS, const float* dh2,
                        const float* z1, float* dq1, hipStream_t s) {
  if (M <= 0) return DMTS_OK;
  ProfScope ps(DMTS_K_ATOM_GEMM, s);
  if (rt == 1) k_chain3<1><<<ceil_div(M, 16), kThreads, 0, s>>>(P, M, RS, dh2, z1, dq1);
  else k_chain3<kRT><<<ceil_div(M, 16 * kRT), kThreads, 0, s>>>(P, M, RS, dh2, z1, dq1);
  DMTS_CHECK_LAUNCH();
  return DMTS_OK;
}

}  // namespace dmts
