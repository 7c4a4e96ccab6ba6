// Fused per-atom MLP chains of the reference potential (internal).
#pragma once

#include "common.h"

namespace dmts {

// Weight views, row-major [out][in] (the input index contiguous).
struct AtomMlpParams {
  const float* U1;    // [128][384]  z1 = U1 q1
  const float* W2h;   // [256][128]  [A | B] = [W_s | W_r] h1
  const float* U2;    // [128][384]  z2 = U2 q2
  const float* Wo;    // [128][128]  y = W_o h2
  const float* wo;    // [128]
  const float* WoT;   // [128][128]  dh2 = W_o^T dy
  const float* U2T;   // [384][128]  dq2 = U2^T dz2
  const float* W2hs;  // [128][256]  dh1 = W_r^T R + W_s^T S
  const float* U1T;   // [384][128]  dq1 = U1^T dz1
  // BF16 form (all null for FP32): the same layers as bfloat16 [out][in]
  const __bf16* h_U1 = nullptr;    // [128][384]
  const __bf16* h_W2h = nullptr;   // [256][128]
  const __bf16* h_U2 = nullptr;    // [128][384]
  const __bf16* h_Wo = nullptr;    // [128][128]
  const __bf16* h_WoT = nullptr;   // [128][128]
  const __bf16* h_U2T = nullptr;   // [384][128]
  const __bf16* h_W2hs = nullptr;  // [128][256]
  const __bf16* h_U1T = nullptr;   // [384][128]
};

// rt: 16-atom row tiles per work-group (1 or 2), a tile shape the autotuner chooses.
dmts_status atom_chain1(const AtomMlpParams& P, int M, int rt, const float* q1, float* z1,
                        float* h1, float* P2, hipStream_t s);
dmts_status atom_chain2(const AtomMlpParams& P, int M, int rt, const float* q2, const float* h1,
                        float escale, float* atom_e, float* dh2, float* dq2, bool backward,
                        hipStream_t s);
dmts_status atom_chain3(const AtomMlpParams& P, int M, int rt, const float* RS, const float* dh2,
                        const float* z1, float* dq1, hipStream_t s);

}  // namespace dmts
