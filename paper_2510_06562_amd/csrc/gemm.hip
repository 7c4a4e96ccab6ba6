// Per-atom dense layers of the potentials as MFMA GEMMs: C[M x N] = A[M x K] * B[K x N]
// (row-major), FP32 operands on v_mfma_f32_32x32x2f32, with the elementwise step that
// follows each layer fused into the store.
//
// One wavefront computes a 32-row x 64-column tile as two 32x32 MFMA blocks.  The A tile
// (32 rows x K) is staged in LDS with a padded stride; B streams from global memory
// (weights of at most 384 x 384 floats stay in L2).
//
// MFMA 32x32x2 f32 register layout (CDNA3/CDNA4):
//   A operand: lane l holds A[l % 32][k0 + l / 32]
//   B operand: lane l holds B[k0 + l / 32][l % 32]
//   D: lane l, register r holds D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32]
#include "gemm.h"

namespace dmts {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kRows = 32;
constexpr int kCols = 64;
constexpr int kMaxK = 384;

template <int EPI>
__global__ void __launch_bounds__(64)
k_gemm_f32(int M, int N, int K, const float* __restrict__ A, int lda,
           const float* __restrict__ B, int ldb, float* __restrict__ C, int ldc,
           GemmAux aux) {
  __shared__ float sA[kRows * (kMaxK + 1)];
  const int lane = threadIdx.x;
  const int m0 = blockIdx.x * kRows;
  const int n0 = blockIdx.y * kCols;
  const int stride = K + 1;
  // stage the A tile (rows beyond M are zero)
  for (int e = lane; e < kRows * K; e += 64) {
    int r = e / K, k = e - r * K;
    int row = m0 + r;
    sA[r * stride + k] = row < M ? A[(size_t)row * lda + k] : 0.0f;
  }
  __syncthreads();
  f32x16 acc0 = {0}, acc1 = {0};
  const int ar = lane & 31, ak = lane >> 5;
  const float* Bp = B + (size_t)ak * ldb + n0 + ar;
#pragma unroll 4
  for (int k0 = 0; k0 < K; k0 += 2) {
    float a = sA[ar * stride + k0 + ak];
    float b0 = Bp[(size_t)k0 * ldb];
    float b1 = Bp[(size_t)k0 * ldb + 32];
    acc0 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b0, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b1, acc1, 0, 0, 0);
  }
#pragma unroll
  for (int blk = 0; blk < 2; ++blk) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = m0 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      const int col = n0 + 32 * blk + (lane & 31);
      if (row >= M) continue;
      const float v = blk == 0 ? acc0[r] : acc1[r];
      const size_t o = (size_t)row * ldc + col;
      if constexpr (EPI == kEpiStore) {
        C[o] = v;
      } else if constexpr (EPI == kEpiSilu) {
        C[o] = v;
        aux.out[o] = silu_f(v);
      } else if constexpr (EPI == kEpiResidSilu) {
        C[o] = v;
        aux.out[o] = aux.in0[o] + silu_f(v);
      } else if constexpr (EPI == kEpiDsilu) {
        C[o] = v;
        aux.out[o] = v * dsilu_f(aux.in0[o]);
      } else if constexpr (EPI == kEpiResidDsilu) {
        aux.out[o] = (v + aux.in1[o]) * dsilu_f(aux.in0[o]);
      }
    }
  }
}

}  // namespace

dmts_status gemm_f32(int epi, int M, int N, int K, const float* A, int lda, const float* B,
                     int ldb, float* C, int ldc, GemmAux aux, hipStream_t s) {
  DMTS_REQUIRE(M >= 0 && N > 0 && K > 0 && N % kCols == 0 && K % 2 == 0 && K <= kMaxK,
               DMTS_E_ARG, "gemm_f32: unsupported shape M=%d N=%d K=%d", M, N, K);
  if (M == 0) return DMTS_OK;
  dim3 grid(ceil_div(M, kRows), N / kCols);
  ProfScope ps(DMTS_K_ATOM_GEMM, s);
  switch (epi) {
    case kEpiStore: k_gemm_f32<kEpiStore><<<grid, 64, 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, aux); break;
    case kEpiSilu: k_gemm_f32<kEpiSilu><<<grid, 64, 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, aux); break;
    case kEpiResidSilu: k_gemm_f32<kEpiResidSilu><<<grid, 64, 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, aux); break;
    case kEpiDsilu: k_gemm_f32<kEpiDsilu><<<grid, 64, 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, aux); break;
    case kEpiResidDsilu: k_gemm_f32<kEpiResidDsilu><<<grid, 64, 0, s>>>(M, N, K, A, lda, B, ldb, C, ldc, aux); break;
    default: DMTS_REQUIRE(false, DMTS_E_ARG, "gemm_f32: unknown epilogue %d", epi);
  }
  DMTS_CHECK_LAUNCH();
  return DMTS_OK;
}

}  // namespace dmts
