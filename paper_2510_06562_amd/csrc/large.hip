// Reference (two-interaction) potential: energy and forces.
//
// Interaction t (t = 1, 2), for a receiver i and sender j with u = d_ij / r_c:
//   a_ij = W_b b(r_ij) + S_i + R_j        t=1: S = T_d[z], R = T_s[z] (species tables)
//                                         t=2: S = B h^1 (receiver block), R = A h^1 (sender)
//   m_ij = f_c(r_ij) SiLU(a_ij)
//   M0_i = sum_j m_ij,  M1_i = sum_j m_ij u,  M2_i = sum_j m_ij (u u^T - |u|^2 I / 3)
//   q_i = [M0 ; |M1|^2 ; |M2|_F^2] (per channel)
// Atom updates h^1 = SiLU(U1 q^1), h^2 = h^1 + SiLU(U2 q^2), readout
// E_i = s_E w_o . SiLU(W_o h^2).
//
// Kernel sequence (forward, then the reverse pass):
//   pair 1 forward -> atom chain 1 (U1, SiLU, [A|B] projections) -> pair 2 forward
//   -> atom chain 2 (U2, residual, readout, E_i, and its reverse down to dE/dq^2)
//   -> pair 2 reverse (dE/da_ij per pair kept for the sender sums, v_ij = dE/dd_ij, the
//      receiver sums) -> sender gather through rev[] -> atom chain 3 (dE/dh^1 down to
//      dE/dq^1) -> pair 1 reverse (adds its v_ij) -> force gather F_i = sum_j v_ij - v_ji.
// The pair kernels recompute every pair feature from the list's geometry; only dE/da of
// interaction 2 is stored per pair, because the sender sums need it in the other row.
// No floating-point atomics: every sum has a fixed order, so results are bitwise
// reproducible.
#include <type_traits>

#include "atom_mlp.h"

namespace dmts {

namespace {

constexpr int kWaves = 4;
// Pair kernels: a work-group owns one channel half (64 channels) of kWaves receivers, one
// wave each, and keeps its half (and the staged weights of that half) over its grid-stride
// loop; which half and which receivers follow the XCD-aware walk below (XcdWalk).
constexpr int K_L = 32;
constexpr int F_L = 128;
constexpr int Z_MAX = 8;
constexpr int NMOM = 10;   // M0, M1 (x, y, z), M2 (xx, yy, zz, xy, xz, yz)

struct LargeParams {
  const __bf16* Wb;   // [NP][F][K] radial block of the interaction as NP bfloat16 terms
  const float* Td;    // [Z][F] layer 1 receiver table
  const float* Ts;    // [Z][F] layer 1 sender table
  float rc, sigma;
  int Z;
};

// ------------------------------------------------------------------ MFMA pair kernels
// One wavefront per receiver and channel half (64 channels), 16-pair row tiles (rows are
// padded to 16).  Pair geometry (d, r) comes from the neighbor list, which is built at the
// evaluation's positions.  Lane l has group g = l / 16 and column cl = l % 16.
//
// Radial contraction a = W_b b (K = 32) on v_mfma_f32_16x16x32_bf16 (A operand: lane l
// holds A[l % 16][8 g + e], B operand B[8 g + e][l % 16], e = 0..7).  The operands are
// given as NP bfloat16 terms: NP = 1 in the BF16 form (b and W_b rounded to nearest even),
// NP = 3 in the FP32 form, where x = x1 + x2 + x3 exactly (each term carries the next
// eight significant bits of x) and the six products x_i y_j with i + j <= 4 are
// accumulated in FP32, smallest first; the dropped terms are below 2^-24 |W||b|, the size
// of FP32 rounding.  The other contractions use v_mfma_f32_16x16x4f32 (A: A[cl][k0 + g],
// B: B[k0 + g][cl], D register r: D[4 g + r][cl]) in FP32.
// Forward: a = b W_b as D[pair][channel] (pair 4g + r, channel 16 blk + cl).  The moments
// M^T[y][c] = sum_p Y[p][y] m[p][c] then use that accumulator as their B operand: in step
// s the K index g stands for pair 4g + s, i.e. register s of the lane.
// Reverse pass: the transposed product a^T = W_b b^T as D[channel][pair] (channel
// 16 blk + 4g + r, pair cl): each lane owns one pair and 32 channels, so the channel sums
// of a pair are in-lane plus two cross-group shuffles; dm^T = D_i^T Y^T likewise.  The
// products of channel block b + 1 are issued before the elementwise work of block b.

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// dE/da of interaction 2 per pair slot, kept for the sender sums: FP32 in the FP32 form,
// bfloat16 (round to nearest even) in the BF16 form, where the sums feed a BF16 product
template <int NP>
using DAType = std::conditional_t<NP == 1, __bf16, float>;

constexpr int kTile = 16;
constexpr int kLdM = 68;    // LDS stride of the per-wave moment rows (64 channels)

// W_b rows [c][k] in LDS, 32 bfloat16 per row; the 16-byte chunk index k / 8 is XORed with
// bits 2..3 of the row so that the 16 rows read by one lane group fall in distinct banks.
__device__ __forceinline__ int wsw(int row, int chunk) {
  return row * K_L + 8 * (chunk ^ ((row >> 2) & 3));
}

// Per-wave adjoint rows D[y][cc] (64 channels, stride kLdH = 80): the low two bits of the
// column are XORed with bits 2..3 of the row, so that both the row-wise reads of dm^T
// (row 4 s + g in group g) and the column-wise reads of the angular sums (row cl + 1 in
// lane cl) fall in distinct banks, with addresses affine in the channel block.
constexpr int kLdH = 80;
__device__ __forceinline__ int dswz(int y, int cc) { return y * kLdH + (cc ^ ((y >> 2) & 3)); }

// The lane's bfloat16 terms of eight radial values.  NP = 1: round to nearest even.
// NP = 3: truncating split, x = t1 + t2 + t3 exactly (t1 = x with the low 16 bits cleared,
// t2 likewise of x - t1, t3 = x - t1 - t2, which has at most eight significant bits); a
// term's bfloat16 is then the high half of its FP32 bits, packed two at a time.
template <int NP>
__device__ __forceinline__ void split_terms(const float (&x)[8], bf16x8 (&t)[NP]) {
  if (NP == 1) {
#pragma unroll
    for (int e = 0; e < 8; ++e) t[0][e] = (__bf16)x[e];
    return;
  }
  uint32_t u[3][8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const uint32_t h = __float_as_uint(x[e]) & 0xffff0000u;
    const float r1 = x[e] - __uint_as_float(h);
    const uint32_t m = __float_as_uint(r1) & 0xffff0000u;
    u[0][e] = h;
    u[1][e] = m;
    u[2][e] = __float_as_uint(r1 - __uint_as_float(m));
  }
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    u32x4 w;
#pragma unroll
    for (int q = 0; q < 4; ++q)   // high halves of elements 2q (low) and 2q + 1 (high)
      w[q] = __builtin_amdgcn_perm(u[p][2 * q + 1], u[p][2 * q], 0x07060302u);
    t[p] = __builtin_bit_cast(bf16x8, w);
  }
}

// b_k(r) = exp(-(r - k sigma)^2 / (2 sigma^2)) and x_k = r - k sigma at k = k0 .. k0 + 7
// (b zero for an invalid pair).  The centres are sigma apart, so b_{k+1} = b_k rho_k with
// rho_k = exp(x_k / sigma - 1/2) = rho_{k-1} / e: two exponentials (transcendental
// instructions issue at a quarter of the vector rate) and fourteen products.  The
// relative error grows by a few units in the last place per step, to ~1e-6 at e = 7 and,
// through the rounding of the exponent x_0 / sigma - 1/2, by ~|x_0 / sigma| ulp per step;
// where that is large the b_k are tiny, so the error stays at the FP32 rounding of the
// sums over k.  With r < r_c = (K - 1) sigma the ratio stays below e^K.
__device__ __forceinline__ void radial_basis(float r, bool valid, int k0, float sigma,
                                             float inv_s2, float (&bk)[8], float (&xk)[8]) {
  const float x0 = r - sigma * k0;
  // invalid pairs: exponent -1e30 gives 0 without a branch around the exponential
  float b = __expf(valid ? -0.5f * x0 * x0 * inv_s2 : -1e30f);
  float rho = __expf(valid ? x0 * (sigma * inv_s2) - 0.5f : -1e30f);
  bk[0] = b;
#pragma unroll
  for (int e = 1; e < 8; ++e) {
    b *= rho;
    rho *= 0.36787944117144233f;   // e^-1
    bk[e] = b;
  }
#pragma unroll
  for (int e = 0; e < 8; ++e) xk[e] = r - sigma * (k0 + e);
}

// acc += W_b . b over K = 32 for one 16 x 16 block from NP-term operands; w_is_a selects
// the transposed product (W_b rows as the A operand).
template <int NP>
__device__ __forceinline__ f32x4 radial_block(const bf16x8 (&w)[NP], const bf16x8 (&b)[NP],
                                              f32x4 acc, bool w_is_a) {
  auto mf = [&](const bf16x8& wv, const bf16x8& bv, f32x4 c) {
    return w_is_a ? __builtin_amdgcn_mfma_f32_16x16x32_bf16(wv, bv, c, 0, 0, 0)
                  : __builtin_amdgcn_mfma_f32_16x16x32_bf16(bv, wv, c, 0, 0, 0);
  };
  if (NP == 3) {
    acc = mf(w[2], b[0], acc);
    acc = mf(w[1], b[1], acc);
    acc = mf(w[0], b[2], acc);
    acc = mf(w[1], b[0], acc);
    acc = mf(w[0], b[1], acc);
  }
  return mf(w[0], b[0], acc);
}

// The NP terms of W_b local row `row` (of the staged half), chunk g, from LDS.
template <int NP>
__device__ __forceinline__ void load_w(const __bf16* sW, int row, int g, bf16x8 (&w)[NP]) {
#pragma unroll
  for (int p = 0; p < NP; ++p)
    w[p] = *reinterpret_cast<const bf16x8*>(&sW[p * (F_L / 2) * K_L + wsw(row, g)]);
}

// Rows 64 h .. 64 h + 63 of the W_b terms (channel half h), as local rows 0..63.
template <int NP>
__device__ __forceinline__ void stage_w(__bf16* sW, const __bf16* __restrict__ Wb, int h) {
  constexpr int kHalf = F_L / 2;
  for (int e = threadIdx.x; e < NP * K_L * kHalf; e += blockDim.x) {
    const int p = e / (K_L * kHalf), c = (e / K_L) % kHalf, k = e % K_L;
    sW[p * kHalf * K_L + wsw(c, k / 8) + k % 8] = Wb[(size_t)p * F_L * K_L + (size_t)(kHalf * h + c) * K_L + k];
  }
}

// Y = [1, u, u u^T - |u|^2/3 (xx, yy, zz), xy, xz, yz], zero beyond the ten components.
__device__ __forceinline__ float ycomp(int y, float ux, float uy, float uz) {
  const float t3 = (ux * ux + uy * uy + uz * uz) * (1.0f / 3.0f);
  float v = 0.f;
  v = y == 0 ? 1.0f : v;
  v = y == 1 ? ux : v;
  v = y == 2 ? uy : v;
  v = y == 3 ? uz : v;
  v = y == 4 ? ux * ux - t3 : v;
  v = y == 5 ? uy * uy - t3 : v;
  v = y == 6 ? uz * uz - t3 : v;
  v = y == 7 ? ux * uy : v;
  v = y == 8 ? ux * uz : v;
  v = y == 9 ? uy * uz : v;
  return v;
}

// Component y of Y(u) as p_a p_b - d |u|^2 for a fixed row y: p_0 = 1, p_1..3 = u_x, u_y,
// u_z, and d = 1/3 on the diagonal rows 4..6 of the traceless second moment.  Rows past 9
// give 1 (any finite value will do there).  For a lane-constant row the choices of p_a, p_b
// are lane masks set once, and a component costs two selects per factor.  It is formed
// from d_ij itself (u = d_ij / r_c): `s` = r_c^-degree of the row scales it.
struct YRow {
  bool ax, ay, az, bx, by, bz;   // p_a, p_b = u_x, u_y, u_z (else 1)
  float d, s;
  __device__ YRow(int y, float irc) {
    s = y >= 1 && y <= 3 ? irc : y >= 4 && y <= 9 ? irc * irc : 1.0f;
    const int a = y >= 1 && y <= 3 ? y : y >= 4 && y <= 6 ? y - 3 : y == 7 || y == 8 ? 1 : y == 9 ? 2 : 0;
    const int b = y >= 4 && y <= 6 ? y - 3 : y == 7 ? 2 : y == 8 || y == 9 ? 3 : 0;
    ax = a == 1;
    ay = a == 2;
    az = a == 3;
    bx = b == 1;
    by = b == 2;
    bz = b == 3;
    d = y >= 4 && y <= 6 ? 1.0f / 3.0f : 0.f;
  }
  __device__ float operator()(float ux, float uy, float uz, float uu) const {
    const float pa = ax ? ux : ay ? uy : az ? uz : 1.0f;
    const float pb = bx ? ux : by ? uy : bz ? uz : 1.0f;
    return fmaf(-d, uu, pa * pb);
  }
};

// Work-groups go to the eight XCDs (each with its own L2) round-robin: work-group b runs on
// XCD b mod 8.  The pair kernels give work-group b the channel half (b >> 3) & 1 and a
// sequence of receiver groups from chunks of `chunk` consecutive groups dealt to the XCDs
// in turn, so that both halves of a receiver group, and runs of neighbouring receivers
// (which share senders), read their rows, geometry and features through one L2.  The
// chunk is kXcdChunk, or fewer where the XCD's slots would otherwise outnumber its groups
// (a small system still spreads over every XCD).  The grid is a multiple of 16; item j of
// the XCD's list is group (j / chunk * 8 + xcd) * chunk + j % chunk, visited by slot
// j mod slots.
constexpr int kXcdChunk = 8;
struct XcdWalk {
  int half, xcd, slot, slots, chunk;
  __device__ explicit XcdWalk(int n_ag) {
    const int b = blockIdx.x, k = b >> 3;
    xcd = b & 7;
    half = k & 1;
    slot = k >> 1;
    slots = gridDim.x >> 4;
    chunk = min(kXcdChunk, max(1, n_ag / (8 * slots)));
  }
  __device__ int group(int j) const { return (j / chunk * 8 + xcd) * chunk + j % chunk; }
};

// The pair kernels accumulate a' = -log2(e) a (every term of the pre-activation is stored
// with that factor), so that e^-a = 2^a' costs no product: logistic(a) = 1 / (1 + 2^a'),
// and a' logistic(a) = -log2(e) SiLU(a), whose factor the kernels undo where SiLU(a) leaves
// them (the moments M, the angular sums G and S1).
constexpr float kLn2 = 0.69314718055994531f;
__device__ __forceinline__ float silu_pre(float ap) {   // -log2(e) SiLU(a)
  return ap * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(ap));
}
__device__ __forceinline__ void silu_pre_grad(float ap, float& yp, float& dy) {
  const float s = __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(ap));
  yp = ap * s;                                 // -log2(e) SiLU(a)
  dy = fmaf(yp, fmaf(s, kLn2, -kLn2), s);      // SiLU'(a) = s + SiLU(a) (1 - s)
}

// Cosine cutoff and its derivative (zero outside); pi_rc = pi / r_c.
__device__ __forceinline__ void cutoff_fn(float r, float pi_rc, bool valid, float& fc,
                                          float& dfc) {
  float sn, cs;
  __sincosf(pi_rc * r, &sn, &cs);
  fc = valid ? 0.5f * (cs + 1.0f) : 0.f;
  dfc = valid ? -0.5f * pi_rc * sn : 0.f;
}

// The FP32 forms of both pair kernels are bound by instruction issue (FP32 MFMA, vector and
// transcendental instructions share a SIMD's issue and overlap little), the BF16 forms by
// latency at low occupancy: the registers of the forward kernel are capped so that four
// waves share a SIMD (five in the BF16 form of interaction 1, at the cost of a few spilled
// registers outside the tile loop, measured faster), those of the reverse kernel for three
// (four for the BF16 form of interaction 1, which fits 128 registers).
// NW: receivers (one wave each) per work-group, a tile shape the autotuner chooses.
template <int LAYER, int NP, int NW>
__global__ void __launch_bounds__(NW * 64)
__attribute__((amdgpu_waves_per_eu(NP == 1 && LAYER == 1 ? 5 : 4)))
k_pair_fwd_mfma(LargeParams P, const int32_t* __restrict__ offs, const int32_t* __restrict__ nbr,
                const float4* __restrict__ geo, const int32_t* __restrict__ species, int n,
                const float* __restrict__ P2, float* __restrict__ Mout, float* __restrict__ q) {
  __shared__ __bf16 sW[NP * (F_L / 2) * K_L];   // W_b [c][k] terms of the half
  __shared__ float sTs[LAYER == 1 ? Z_MAX * F_L : 1];
  __shared__ float sM[NW][16 * kLdM];   // rows 10..15 (zero moments) unused
  const int n_ag = (n + NW - 1) / NW;
  const XcdWalk xw(n_ag);
  const int half = xw.half, hb = 4 * half;   // hb: first channel block of the half
  stage_w<NP>(sW, P.Wb, half);
  if (LAYER == 1)
    for (int e = threadIdx.x; e < P.Z * F_L; e += blockDim.x) sTs[e] = P.Ts[e];
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, cl = lane & 15;
  for (int j = xw.slot, ag = xw.group(j); ag < n_ag; j += xw.slots, ag = xw.group(j)) {
  const int i = ag * NW + w;
  if (i >= n) continue;
  const int zi_s = species[i];
  float base[4];
#pragma unroll
  for (int b = 0; b < 4; ++b)
    base[b] = LAYER == 1 ? P.Td[zi_s * F_L + 16 * (hb + b) + cl]
                         : P2[(size_t)i * 2 * F_L + F_L + 16 * (hb + b) + cl];
  f32x4 Mt[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) Mt[b] = f32x4{0.f, 0.f, 0.f, 0.f};
  const float inv_s2 = 1.0f / (P.sigma * P.sigma);
  const float irc = 1.0f / P.rc;
  const float pi_rc = 3.14159265358979f * irc;
  const YRow yrow(cl, irc);   // the lane's row of M^T
  const int row0 = offs[i], row1 = offs[i + 1];
  for (int t0 = row0; t0 < row1; t0 += kTile) {
    // A operand of a = b W_b: b_k of pair cl at k = 8 g + e, as NP bfloat16 terms
    const float rp = geo[t0 + cl].w;
    const bool vp = nbr[t0 + cl] >= 0 && rp < P.rc;
    float bk[8], xk[8];
    radial_basis(rp, vp, 8 * g, P.sigma, inv_s2, bk, xk);
    bf16x8 bt[NP];
    split_terms<NP>(bk, bt);
    // f_c of pair cl; the D layout's pairs 4 g + r take theirs from lanes 4 g + r
    float fc_own, dfc_own;
    cutoff_fn(rp, pi_rc, vp, fc_own, dfc_own);
    // the lane's four pairs of the D layout: 4 g + r
    float fc[4], yop[4];
    int jj[4], zz[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      // everything computed unconditionally and selected, so that the four geometry
      // loads are issued together (a branch per pair would serialize them)
      const int p = t0 + 4 * g + r;
      const float4 gv = geo[p];
      const int j = nbr[p];
      const bool v = j >= 0 && gv.w < P.rc;
      fc[r] = __shfl(fc_own, 4 * g + r, 64);
      jj[r] = v ? j : -1;
      zz[r] = LAYER == 1 ? species[v ? j : i] : 0;
      // f_c of the pair is folded into its Y components (the A operand of M^T), so the
      // m operand below is SiLU(a) alone; an invalid pair has f_c = 0 and finite
      // (zero-padded) geometry, so its Y needs no select
      yop[r] = (fc[r] * yrow.s) * yrow(gv.x, gv.y, gv.z, gv.w * gv.w);
    }
    // sender terms of the lane's sixteen (pair, channel) values, all requested before the
    // products so that their latencies overlap
    float snd[4][4];
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int c = 16 * (hb + b) + cl;
        snd[b][r] = LAYER == 1 ? sTs[zz[r] * F_L + c]
                               : P2[(size_t)(jj[r] >= 0 ? jj[r] : i) * 2 * F_L + c];
      }
    __builtin_amdgcn_sched_barrier(0);
    f32x4 acc[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      bf16x8 wt[NP];
      load_w<NP>(sW, 16 * b + cl, g, wt);
      acc[b] = radial_block<NP>(wt, bt, f32x4{base[b], base[b], base[b], base[b]}, false);
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      f32x4 mv;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        mv[r] = silu_pre(acc[b][r] + snd[b][r]);   // f_c (0 if invalid) sits in Y
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
        Mt[b] = __builtin_amdgcn_mfma_f32_16x16x4f32(yop[s], mv[s], Mt[b], 0, 0, 0);
    }
  }
  // M^T rows y = 4 g + r -> LDS (all sixteen, without a branch; rows 10..15 are not
  // read), then moments and invariants per channel
  float* sm = sM[w];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) sm[(4 * g + r) * kLdM + 16 * b + cl] = Mt[b][r];
  wave_sync();
  float* Mi = Mout + (size_t)i * NMOM * F_L;
  float* qi = q + (size_t)i * 3 * F_L;
  {
    const int c = 16 * hb + lane;
    float mm[NMOM];
#pragma unroll
    for (int y = 0; y < NMOM; ++y) {
      mm[y] = -kLn2 * sm[y * kLdM + lane];   // undo the -log2(e) of SiLU
      Mi[y * F_L + c] = mm[y];
    }
    qi[c] = mm[0];
    qi[F_L + c] = mm[1] * mm[1] + mm[2] * mm[2] + mm[3] * mm[3];
    qi[2 * F_L + c] = mm[4] * mm[4] + mm[5] * mm[5] + mm[6] * mm[6] +
                      2.0f * (mm[7] * mm[7] + mm[8] * mm[8] + mm[9] * mm[9]);
  }
  }  // grid-stride loop over work-groups of atoms
}

// Per-pair-slot sums of dE/da (receiver sums), [slot][64 channels], stride 68.
constexpr int kLdR = 68;

constexpr bool kAhead = true;

template <int LAYER, int NP, int NW>
__global__ void __launch_bounds__(NW * 64)
__attribute__((amdgpu_waves_per_eu(NP == 1 && LAYER == 1 ? 4 : 3)))
k_pair_bwd_mfma(LargeParams P, const int32_t* __restrict__ offs, const int32_t* __restrict__ nbr,
                const float4* __restrict__ geo, const int32_t* __restrict__ species, int n,
                const float* __restrict__ P2, const float* __restrict__ Mall,
                const float* __restrict__ dq, DAType<NP>* __restrict__ dA,
                float* __restrict__ RS, float* __restrict__ v, int64_t cap) {
  __shared__ __bf16 sW[NP * (F_L / 2) * K_L];         // W_b [c][k] terms of the half
  __shared__ float sTs[LAYER == 1 ? Z_MAX * F_L : 1];
  // per wave, over its 64 channels (local index cc = c - 64 half)
  __shared__ float sD[NW][NMOM * kLdH];          // D[y][cc] of the receiver (dswz)
  __shared__ __align__(16) float sB[NW][F_L / 2];   // receiver term S_i of a_ij
  __shared__ float sR[LAYER == 2 ? NW : 1][LAYER == 2 ? kTile * kLdR : 1];
  const int n_ag = (n + NW - 1) / NW;
  const XcdWalk xw(n_ag);
  const int half = xw.half, hb = 4 * half;
  stage_w<NP>(sW, P.Wb, half);
  if (LAYER == 1)
    for (int e = threadIdx.x; e < P.Z * F_L; e += blockDim.x) sTs[e] = P.Ts[e];
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, cl = lane & 15;
  for (int j = xw.slot, ag = xw.group(j); ag < n_ag; j += xw.slots, ag = xw.group(j)) {
  const int i = ag * NW + w;
  if (i >= n) continue;
  float* sd = sD[w];
  const int zi_s = species[i];
  // D[y][c]: dE/dq folded with dq/dM, off-diagonal M2 components doubled, so that
  // dm = sum_y Y[y] D[y]
  {
    const float* Mi = Mall + (size_t)i * NMOM * F_L;
    const float* dqi = dq + (size_t)i * 3 * F_L;
    {
      const int c = 16 * hb + lane;
      const float s1 = 2.0f * dqi[F_L + c], s2 = 2.0f * dqi[2 * F_L + c];
      sd[dswz(0, lane)] = dqi[c];
#pragma unroll
      for (int y = 1; y < 4; ++y) sd[dswz(y, lane)] = s1 * Mi[y * F_L + c];
#pragma unroll
      for (int y = 4; y < 7; ++y) sd[dswz(y, lane)] = s2 * Mi[y * F_L + c];
#pragma unroll
      for (int y = 7; y < NMOM; ++y) sd[dswz(y, lane)] = 2.0f * s2 * Mi[y * F_L + c];
    }
  }
  {
    const float* src = LAYER == 1 ? P.Td + zi_s * F_L : P2 + (size_t)i * 2 * F_L + F_L;
    sB[w][lane] = src[16 * hb + lane];
    if (LAYER == 2)
      for (int e = lane; e < kTile * kLdR; e += 64) sR[w][e] = 0.f;
  }
  wave_sync();
  const float inv_s2 = 1.0f / (P.sigma * P.sigma);
  const float irc = 1.0f / P.rc;
  const float pi_rc = 3.14159265358979f * irc;
  // row of D read by lane (cl, g) for the angular sums: y = cl, clamped to row 9 for
  // cl >= 10, whose output rows are not used (an MFMA output row depends only on the A row
  // of the same index, so any finite value will do there)
  const int kr = cl < NMOM ? cl : NMOM - 1;
  const int row0 = offs[i], row1 = offs[i + 1];
  for (int t0 = row0; t0 < row1; t0 += kTile) {
    // the lane's pair
    const int p = t0 + cl;
    const float4 gv = geo[p];
    const int j0 = nbr[p];
    const bool vp = j0 >= 0 && gv.w < P.rc;
    const int j = vp ? j0 : -1;
    float fc, dfc;
    cutoff_fn(gv.w, pi_rc, vp, fc, dfc);
    const float ux = vp ? gv.x * irc : 0.f, uy = vp ? gv.y * irc : 0.f, uz = vp ? gv.z * irc : 0.f;
    // radial operands b_k(r), x_k b_k(r) at k = 8 g + e, as NP bfloat16 terms
    bf16x8 bt[NP], dbt[NP];
    {
      // b'_k = -x_k b_k / sigma^2: the operand holds x_k b_k, and the factor -1/sigma^2
      // is applied once to the pair's sum S2
      float bk[8], xk[8], dbk[8];
      radial_basis(gv.w, vp, 8 * g, P.sigma, inv_s2, bk, xk);
#pragma unroll
      for (int e = 0; e < 8; ++e) dbk[e] = xk[e] * bk[e];
      split_terms<NP>(bk, bt);
      split_terms<NP>(dbk, dbt);
    }
    // B operand of dm^T: f_c Y^T[4 s + g][pair cl].  With f_c folded in, the product is
    // f_c dm, the factor that dE/da = f_c dm SiLU'(a) needs.
    float yop[3];
#pragma unroll
    for (int s = 0; s < 3; ++s) yop[s] = fc * ycomp(4 * s + g, ux, uy, uz);
    // invalid pairs have f_c = 0, so any finite sender term will do: use the receiver's
    const float* Aj = LAYER == 2 ? P2 + (size_t)(j >= 0 ? j : i) * 2 * F_L : nullptr;
    const float* Tj = LAYER == 1 ? sTs + species[j >= 0 ? j : i] * F_L : nullptr;
    float S2 = 0.f;
    // G^T[y][pair] = sum_c D[c][y] SiLU(a)[c][pair] on MFMA: K runs over the lane group's
    // channels (index g <-> channel 16 b + 4 g + s, register s of the SiLU operand), the A
    // operand is D[16 b + 4 g + s][y] for row y = cl < 10.
    f32x4 Gt = {0.f, 0.f, 0.f, 0.f};
    // The three products of channel block bb4: a^T = W_b b^T, W_b (x b)^T (a'^T up to the
    // factor -1/sigma^2) and dm^T = D^T Y^T.  They are issued one block ahead, so that the matrix cores work on
    // block bb4 + 1 while the vector units finish bb4.
    auto issue = [&](int bb4, f32x4& ga, f32x4& gd, f32x4& dmv, float4& add) {
      // sender term of the lane's four channels 16 b + 4 g .. + 3
      const int c0 = 16 * (hb + bb4) + 4 * g;
      add = LAYER == 2 ? *reinterpret_cast<const float4*>(Aj + c0)
                       : *reinterpret_cast<const float4*>(Tj + c0);
      bf16x8 wt[NP];
      load_w<NP>(sW, 16 * bb4 + cl, g, wt);
      // the receiver term of the lane's four channels starts the accumulator
      const float4 br = *reinterpret_cast<const float4*>(&sB[w][16 * bb4 + 4 * g]);
      ga = radial_block<NP>(wt, bt, f32x4{br.x, br.y, br.z, br.w}, true);
      gd = radial_block<NP>(wt, dbt, f32x4{0.f, 0.f, 0.f, 0.f}, true);
      dmv = f32x4{0.f, 0.f, 0.f, 0.f};
      // K index 4 s + g = y runs over the ten components; rows 12..15 (s = 3) are left
      // out, and at y = 10, 11 the B operand (Y) is zero, so the A operand there may be
      // any finite value: the clamped row 9
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        const int y = 4 * s + g;
        const float dy = sd[dswz(y < NMOM ? y : NMOM - 1, 16 * bb4 + cl)];
        dmv = __builtin_amdgcn_mfma_f32_16x16x4f32(dy, yop[s], dmv, 0, 0, 0);
      }
    };
    f32x4 ga, gd, dmv;
    float4 add;
    if (kAhead) issue(0, ga, gd, dmv, add);
#pragma unroll
    for (int bb4 = 0; bb4 < 4; ++bb4) {
      f32x4 ga_n, gd_n, dmv_n;
      float4 add_n;
      if (!kAhead) issue(bb4, ga, gd, dmv, add);
      else if (bb4 < 3) issue(bb4 + 1, ga_n, gd_n, dmv_n, add_n);
      const int b = hb + bb4;
      const int c0 = 16 * b + 4 * g;   // the lane's four channels c0 .. c0+3
      const int l0 = 16 * bb4 + 4 * g;  // their index within the half
      f32x4 mv;
      float4 dav;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float addr = r == 0 ? add.x : r == 1 ? add.y : r == 2 ? add.z : add.w;
        const float a = ga[r] + addr;
        float sv, dsv;
        silu_pre_grad(a, sv, dsv);   // sv = -log2(e) SiLU(a)
        const float da = dmv[r] * dsv;   // dmv holds f_c dm
        S2 = fmaf(da, gd[r], S2);
        mv[r] = sv;
        if (r == 0) dav.x = da; else if (r == 1) dav.y = da; else if (r == 2) dav.z = da; else dav.w = da;
      }
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const float dk = sd[dswz(kr, l0 + s4)];
        Gt = __builtin_amdgcn_mfma_f32_16x16x4f32(dk, mv[s4], Gt, 0, 0, 0);
      }
      if (LAYER == 2) {
        if constexpr (NP == 1) {
          const bf16x4 h = {(__bf16)dav.x, (__bf16)dav.y, (__bf16)dav.z, (__bf16)dav.w};
          *reinterpret_cast<bf16x4*>(dA + (size_t)p * F_L + c0) = h;
        } else {
          *reinterpret_cast<float4*>(dA + (size_t)p * F_L + c0) = dav;
        }
        float4* acc = reinterpret_cast<float4*>(&sR[w][cl * kLdR + l0]);
        float4 t = *acc;
        t.x += dav.x;
        t.y += dav.y;
        t.z += dav.z;
        t.w += dav.w;
        *acc = t;
      }
      if (kAhead && bb4 < 3) {
        ga = ga_n;
        gd = gd_n;
        dmv = dmv_n;
        add = add_n;
      }
      // one region per block: the live products are those of two blocks
      __builtin_amdgcn_sched_barrier(0);
    }
    // channel sum of the pair: in-lane above, then across the four groups
    S2 += __shfl_xor(S2, 16, 64);
    S2 += __shfl_xor(S2, 32, 64);
    // Gt register r of group g holds row 4 g + r of pair cl: collect rows 0..9
    float G[NMOM];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      G[r] = Gt[r];
      G[4 + r] = __shfl_xor(Gt[r], 16, 64);
    }
    G[8] = __shfl_xor(Gt[0], 32, 64);
    G[9] = __shfl_xor(Gt[1], 32, 64);
    if (g == 0) {
      // S1 = sum_c dm_c SiLU(a_c) = sum_y Y[y] G[y]; the sums of m = f_c SiLU(a) against
      // dM1, dM2_aa and 2 dM2_ab (xy, xz, yz) are f_c G[1..3], f_c G[4..6], f_c G[7..9]
      const float t3 = (ux * ux + uy * uy + uz * uz) * (1.0f / 3.0f);
      // (G carries the -log2(e) of the SiLU operand: the -ln 2 below undoes it)
      const float S1 = -kLn2 * (G[0] + ux * G[1] + uy * G[2] + uz * G[3] + (ux * ux - t3) * G[4] +
                                (uy * uy - t3) * G[5] + (uz * uz - t3) * G[6] + ux * uy * G[7] +
                                ux * uz * G[8] + uy * uz * G[9]);
      const float t23 = (2.0f / 3.0f) * (G[4] + G[5] + G[6]);
      const float ax = G[1] + 2.0f * G[4] * ux + G[7] * uy + G[8] * uz - t23 * ux;
      const float ay = G[2] + G[7] * ux + 2.0f * G[5] * uy + G[9] * uz - t23 * uy;
      const float az = G[3] + G[8] * ux + G[9] * uy + 2.0f * G[6] * uz - t23 * uz;
      // S2 holds sum_c dE/da_c (W_b' x b)_c with the -log2(e)-scaled W_b' = -log2(e) W_b:
      // dE/dr's radial part is -S2 / (sigma^2 (-log2 e)) = ln 2 S2 / sigma^2
      const float rho = fmaf(kLn2 * inv_s2, S2, dfc * S1);
      const float ir = vp ? __builtin_amdgcn_rcpf(gv.w) : 0.f;
      const float fi = -kLn2 * irc * fc;
      const float vx = rho * gv.x * ir + fi * ax;
      const float vy = rho * gv.y * ir + fi * ay;
      const float vz = rho * gv.z * ir + fi * az;
      // this half's share of v_ij: slot [p][half] of the [cap][2] float4 array
      float4* vh = reinterpret_cast<float4*>(v) + 2 * (size_t)p + half;
      if (LAYER == 2) {
        *vh = make_float4(vx, vy, vz, 0.f);
      } else {
        float4 t = *vh;
        t.x += vx;
        t.y += vy;
        t.z += vz;
        *vh = t;
      }
    }
  }
  if (LAYER == 2) {
    // receiver sums: add the 16 pair slots in a fixed order
    wave_sync();
    float t = 0.f;
    for (int k = 0; k < kTile; ++k) t += sR[w][k * kLdR + lane];
    RS[(size_t)i * 2 * F_L + 16 * hb + lane] = t;
  }
  }  // grid-stride loop over work-groups of atoms
}

// S_j = sum over the rows of j of dA at the reverse positions (the sender sums), in FP32.
// One wave per atom; each load instruction fetches two dA rows, lanes 0-31 the first and
// lanes 32-63 the second, four channels per lane (16 or 8 bytes).  The row's reverse
// positions are read 64 at a time (one per lane) and broadcast; eight row pairs are in
// flight at once.  Each half adds its rows (even, odd positions) in row order, then the
// two halves are added.
__device__ __forceinline__ float4 load_da4(const float* dA, size_t k) {
  return *reinterpret_cast<const float4*>(dA + k);
}
__device__ __forceinline__ float4 load_da4(const __bf16* dA, size_t k) {
  const bf16x4 t = *reinterpret_cast<const bf16x4*>(dA + k);
  return make_float4((float)t[0], (float)t[1], (float)t[2], (float)t[3]);
}

template <typename T>
__global__ void __launch_bounds__(kWaves * 64)
k_sender_gather(const int32_t* __restrict__ offs, const int32_t* __restrict__ nbr,
                const int32_t* __restrict__ rev, int n, const T* __restrict__ dA,
                float* __restrict__ RS) {
  constexpr int kU = 8;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int h = lane >> 5, c0 = 4 * (lane & 31);
  const int i = blockIdx.x * kWaves + w;
  if (i >= n) return;
  float4 s = make_float4(0.f, 0.f, 0.f, 0.f);
  const int row0 = offs[i], row1 = offs[i + 1];
  for (int base = row0; base < row1; base += 64) {
    const int p = base + lane;
    const int q = (p < row1 && nbr[p] >= 0) ? rev[p] : -1;
    const int m = min(64, row1 - base);
    // k < m <= 64 steps by 16, so k + 2 u + 1 <= 63
    for (int k = 0; k < m; k += 2 * kU) {
      float4 t[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int qa = __builtin_amdgcn_readlane(q, k + 2 * u);
        const int qb = __builtin_amdgcn_readlane(q, k + 2 * u + 1);
        const int qq = h ? qb : qa;
        t[u] = qq >= 0 ? load_da4(dA, (size_t)qq * F_L + c0) : make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        s.x += t[u].x;
        s.y += t[u].y;
        s.z += t[u].z;
        s.w += t[u].w;
      }
    }
  }
  s.x += __shfl_xor(s.x, 32, 64);
  s.y += __shfl_xor(s.y, 32, 64);
  s.z += __shfl_xor(s.z, 32, 64);
  s.w += __shfl_xor(s.w, 32, 64);
  if (h == 0) *reinterpret_cast<float4*>(RS + (size_t)i * 2 * F_L + F_L + c0) = s;
}

}  // namespace

// F_i = sum_{p in row i} v[p] - v[rev[p]]  (v[p] = dE/dd_ij, d_ij = x_j - x_i), with v
// kept as two channel-half partial sums added here in a fixed order.
__global__ void __launch_bounds__(256)
k_force_gather(const int32_t* __restrict__ offs, const int32_t* __restrict__ nbr,
               const int32_t* __restrict__ rev, int n, const float* __restrict__ v, int64_t cap,
               float* __restrict__ forces, Epilogue E, bool has_ep, bool fresh_small) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + w;
  if (i >= n) return;
  CoordIn ein{};   // this atom's integrator inputs, coordinate d = lane (lanes 0..2)
  if (has_ep && lane < 3) ein = prefetch_coord(E, i, n, lane, fresh_small);
  float fx = 0.f, fy = 0.f, fz = 0.f;
  const int row0 = offs[i], row1 = offs[i + 1];
  const float4* v4 = reinterpret_cast<const float4*>(v);   // [cap][2 halves]
  for (int p = row0 + lane; p < row1; p += 64) {
    if (nbr[p] < 0) continue;
    const int q = rev[p];
    if (q < 0) continue;
    // both halves of a slot share one 32-byte sector: one random access per pair
    const float4 a0 = v4[2 * (size_t)p], a1 = v4[2 * (size_t)p + 1];
    const float4 b0 = v4[2 * (size_t)q], b1 = v4[2 * (size_t)q + 1];
    fx += (a0.x + a1.x) - (b0.x + b1.x);
    fy += (a0.y + a1.y) - (b0.y + b1.y);
    fz += (a0.z + a1.z) - (b0.z + b1.z);
  }
  fx = wave_sum(fx);
  fy = wave_sum(fy);
  fz = wave_sum(fz);
  if (lane == 0) {
    forces[i] = fx;
    forces[n + i] = fy;
    forces[2 * n + i] = fz;
  }
  if (has_ep) {   // F_i is final: the integrator step of atom i, with lane 0's sums
    const float f0x = __shfl(fx, 0, 64), f0y = __shfl(fy, 0, 64), f0z = __shfl(fz, 0, 64);
    apply_coords(E, i, n, lane, ein, lane == 0 ? f0x : lane == 1 ? f0y : f0z, fresh_small);
  }
}

dmts_status large_energy_forces(Model* m, NList* nl, const double* pos, const int32_t* species,
                                int32_t n, double box, const int32_t* sys_offsets, int32_t n_sys,
                                double* energy, float* forces, float* atom_energy, hipStream_t s,
                                const Epilogue* ep) {
  DMTS_REQUIRE(m->K == K_L && m->F == F_L, DMTS_E_ARG, "large model: unsupported shape");
  DMTS_REQUIRE(nl->row_align % kTile == 0, DMTS_E_ARG,
               "large model: the neighbor list needs row_align 16 (or a multiple), got %d",
               nl->row_align);
  const size_t F = F_L, N = (size_t)((n + 63) / 64 * 64);
  // per-atom workspace layout (floats)
  const size_t o_q1 = 0, o_M1 = o_q1 + N * 3 * F, o_z1 = o_M1 + N * NMOM * F;
  const size_t o_h1 = o_z1 + N * F, o_P2 = o_h1 + N * F, o_q2 = o_P2 + N * 2 * F;
  const size_t o_M2 = o_q2 + N * 3 * F, o_dh2 = o_M2 + N * NMOM * F;
  const size_t o_dq2 = o_dh2 + N * F, o_RS = o_dq2 + N * 3 * F;
  const size_t o_dq1 = o_RS + N * 2 * F, o_e = o_dq1 + N * 3 * F;
  const size_t o_part = o_e + N;   // FP64 partial energy sums (even offset: N % 64 == 0)
  const size_t total = o_part + 2 * energy_partials(n);
  DMTS_REQUIRE(m->atom_ws.reserve(total * sizeof(float), s) == DMTS_OK, DMTS_E_OOM,
               "large model: atom workspace");
  const int64_t cap = nl->max_pairs;
  if (forces) {
    DMTS_REQUIRE(m->pair_ws.reserve(sizeof(float) * (size_t)cap * (F + 8), s) == DMTS_OK,
                 DMTS_E_OOM, "large model: pair workspace");
  }
  float* W = m->atom_ws.as<float>();
  float* e_atom = atom_energy ? atom_energy : W + o_e;
  LargeParams P1{m->p16(m->h_Wb1), m->p(m->o_Td), m->p(m->o_Ts), m->rc, m->sigma, m->Z};
  LargeParams P2{m->p16(m->h_Wb2), nullptr, nullptr, m->rc, m->sigma, m->Z};
  AtomMlpParams A{m->p(m->o_U1),  m->p(m->o_W2h), m->p(m->o_U2),   m->p(m->o_Wo),
                  m->p(m->o_wo),  m->p(m->o_WoT), m->p(m->o_U2T),  m->p(m->o_W2hs),
                  m->p(m->o_U1T)};
  if (m->bf16) {
    A.h_U1 = m->p16(m->h_U1);
    A.h_W2h = m->p16(m->h_W2h);
    A.h_U2 = m->p16(m->h_U2);
    A.h_Wo = m->p16(m->h_Wo);
    A.h_WoT = m->p16(m->h_WoT);
    A.h_U2T = m->p16(m->h_U2T);
    A.h_W2hs = m->p16(m->h_W2hs);
    A.h_U1T = m->p16(m->h_U1T);
  }
  const int blocks = ceil_div(n, kWaves);
  const TileShape sh = m->shape_for(n);
  // the whole evaluation, instantiated for the FP32 (three-term radial operands) and the
  // BF16 form (one term), and for NW receivers per pair work-group
  auto run = [&](auto np_tag, auto nw_tag) -> dmts_status {
    constexpr int NP = decltype(np_tag)::value;
    constexpr int NW = decltype(nw_tag)::value;
    dmts_status st;
    if (n > 0) {
      // two work-groups (channel halves) per NW receivers; an even grid of at least two
      auto grid_of = [&](auto kernel) {
        const int b = launch_grid(sh.grid, 2 * ceil_div(n, NW),
                                  resident_groups(reinterpret_cast<const void*>(kernel), NW * 64));
        return dim3(b < 16 ? 16 : (b + 15) & ~15);   // whole XCD-halves quads (XcdWalk)
      };
      const dim3 wg(NW * 64);
      {
        ProfScope ps(DMTS_K_PAIR1_FORWARD, s, true);
        launch_timed(ps, &k_pair_fwd_mfma<1, NP, NW>, grid_of(&k_pair_fwd_mfma<1, NP, NW>), wg, s,
                     P1, nl->offs, nl->nbr, nl->geo, species, n, nullptr, W + o_M1, W + o_q1);
      }
      DMTS_CHECK_LAUNCH();
      if ((st = atom_chain1(A, n, sh.rt, W + o_q1, W + o_z1, W + o_h1, W + o_P2, s)) != DMTS_OK)
        return st;
      {
        ProfScope ps(DMTS_K_PAIR2_FORWARD, s, true);
        launch_timed(ps, &k_pair_fwd_mfma<2, NP, NW>, grid_of(&k_pair_fwd_mfma<2, NP, NW>), wg, s,
                     P2, nl->offs, nl->nbr, nl->geo, species, n, W + o_P2, W + o_M2, W + o_q2);
      }
      DMTS_CHECK_LAUNCH();
      if ((st = atom_chain2(A, n, sh.rt, W + o_q2, W + o_h1, m->escale, e_atom, W + o_dh2,
                            W + o_dq2, forces != nullptr, s)) != DMTS_OK)
        return st;
      if (forces) {
        // pair workspace: dA [cap][F] (FP32 or bfloat16), then v [cap][2] float4 (the
        // two channel halves' partial dE/dd_ij of a slot side by side)
        DAType<NP>* dA = m->pair_ws.as<DAType<NP>>();
        float* v = m->pair_ws.as<float>() + (size_t)cap * F;
        {
          ProfScope ps(DMTS_K_PAIR2_BACKWARD, s, true);
          launch_timed(ps, &k_pair_bwd_mfma<2, NP, NW>, grid_of(&k_pair_bwd_mfma<2, NP, NW>), wg,
                       s, P2, nl->offs, nl->nbr, nl->geo, species, n, W + o_P2, W + o_M2,
                       W + o_dq2, dA, W + o_RS, v, cap);
        }
        DMTS_CHECK_LAUNCH();
        {
          ProfScope ps(DMTS_K_GATHER, s);
          k_sender_gather<DAType<NP>><<<blocks, kWaves * 64, 0, s>>>(nl->offs, nl->nbr, nl->rev,
                                                                     n, dA, W + o_RS);
        }
        DMTS_CHECK_LAUNCH();
        if ((st = atom_chain3(A, n, sh.rt, W + o_RS, W + o_dh2, W + o_z1, W + o_dq1, s)) !=
            DMTS_OK)
          return st;
        {
          ProfScope ps(DMTS_K_PAIR1_BACKWARD, s, true);
          launch_timed(ps, &k_pair_bwd_mfma<1, NP, NW>, grid_of(&k_pair_bwd_mfma<1, NP, NW>), wg,
                       s, P1, nl->offs, nl->nbr, nl->geo, species, n, nullptr, W + o_M1,
                       W + o_dq1, static_cast<DAType<NP>*>(nullptr), nullptr, v, cap);
        }
        DMTS_CHECK_LAUNCH();
        // the integrator program runs in the force gather's epilogue, or (with an O-step)
        // as a launch of its own right after it
        const bool fuse = ep && !has_thermo(ep->prog);
        if (ep && ep->wait) DMTS_HIP(hipStreamWaitEvent(s, ep->wait, 0));
        {
          ProfScope ps(DMTS_K_GATHER, s);
          k_force_gather<<<blocks, 256, 0, s>>>(nl->offs, nl->nbr, nl->rev, n, v, cap, forces,
                                                fuse ? *ep : Epilogue{}, fuse,
                                                fuse && forces == ep->Fs);
        }
        DMTS_CHECK_LAUNCH();
        if (ep && !fuse && (st = apply_program(*ep, n, s)) != DMTS_OK) return st;
      }
    }

    return DMTS_OK;
  };
  auto run_np = [&](auto np_tag) -> dmts_status {
    switch (sh.nw) {
      case 2: return run(np_tag, std::integral_constant<int, 2>{});
      case 8: return run(np_tag, std::integral_constant<int, 8>{});
      default: return run(np_tag, std::integral_constant<int, 4>{});
    }
  };
  const dmts_status rs = m->bf16 ? run_np(std::integral_constant<int, 1>{})
                                 : run_np(std::integral_constant<int, 3>{});
  if (rs != DMTS_OK) return rs;
  if (energy)
    return reduce_energy(e_atom, n, sys_offsets, n_sys, energy,
                         reinterpret_cast<double*>(W + o_part), s);
  return DMTS_OK;
}

}  // namespace dmts
