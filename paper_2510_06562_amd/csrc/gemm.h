// MFMA GEMM with fused elementwise epilogues (internal).
#pragma once

#include "common.h"

namespace dmts {

enum GemmEpi {
  kEpiStore = 0,       // C = acc
  kEpiSilu = 1,        // C = acc;  out = SiLU(acc)
  kEpiResidSilu = 2,   // C = acc;  out = in0 + SiLU(acc)
  kEpiDsilu = 3,       // C = acc;  out = acc * SiLU'(in0)
  kEpiResidDsilu = 4,  //           out = (acc + in1) * SiLU'(in0)   (C unused)
};

// Auxiliary row-major arrays of the epilogues; they share C's leading dimension.
struct GemmAux {
  float* out = nullptr;
  const float* in0 = nullptr;
  const float* in1 = nullptr;
};

// C[M x N] = A[M x K] * B[K x N], N a multiple of 64, K even and <= 384.
dmts_status gemm_f32(int epi, int M, int N, int K, const float* A, int lda, const float* B,
                     int ldb, float* C, int ldc, GemmAux aux, hipStream_t s);

}  // namespace dmts
