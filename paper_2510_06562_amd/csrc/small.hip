// Fast (one-interaction) potential: energy and forces.
//
//   a_ij = W_r b(r_ij) + T_d[z_i] + T_s[z_j]      (T_d, T_s: the species-embedding blocks of
//                                                  W_pair folded with the embedding table)
//   m_ij = f_c(r_ij) SiLU(a_ij),  h_i = sum_j m_ij,  E_i = s_E w2 . SiLU(W1 h_i)
//
// Two kernels, one wavefront per receiver atom:
//   k_small_eval: walks the receiver's neighbor-list row (which may come from a longer
//     cutoff), computes the float geometry at the current positions and compacts the pairs
//     inside the cutoff with a ballot into LDS.  a = b W_r and a' = b' W_r run on MFMA
//     (16 pairs x 64 channels per tile), the messages are summed in registers, the
//     64 -> 64 -> 1 readout gives E_i and g_i = dE_i/dh_i, and then, from the tiles' values,
//     s_ij = dE_i/dr_ij = g_i . dm_ij/dr for every pair, written with the pair's unit vector
//     to its slot of the list.  Only E_i depends on r_ij through m_ij, so this is the whole
//     derivative of E_i; no neighbor's adjoint is needed.
//   k_small_force: F_i = sum_j (s_ij + s_ji) d_ij / r_ij over the row, s_ji from the reverse
//     slot.  Once F_i is final the integrator's kicks and drifts of atom i run in the same
//     wave (the program that follows the evaluation, when it has no O-step).
// Rows are sorted by sender and both kernels sum in the order of the pairs inside the
// cutoff, so the results do not depend on the list's cutoff or padding.
//
// MFMA 16x16x4 f32:  A operand lane l: A[l%16][k0 + l/16]; B: B[k0 + l/16][l%16];
//                    D register r: D[4 (l/16) + r][l%16].
// BF16 form: v_mfma_f32_16x16x16_bf16 (A: A[l%16][4 (l/16) + e], B: B[4 (l/16) + e][l%16],
// e = 0..3) with b, b' and W_r rounded to bfloat16; the readout uses bfloat16-valued W1 and
// activations with FP32 accumulation.  Geometry and elementwise math are FP32.
#include <mutex>
#include <type_traits>

#include "common.h"

namespace dmts {

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int K_S = 16;    // radial functions
constexpr int F_S = 64;    // hidden width
constexpr int Z_MAX = 8;
constexpr int kCap = kSmallPairCap;   // most pairs one receiver may have inside the cutoff
constexpr int kTile = 16;
constexpr int kLdW = 20;   // LDS stride of W_r rows [c][k]
constexpr int kLdW1 = 65;  // LDS stride of W1 rows [c][e]

struct SmallParams {
  const float* WbT;  // [K][F]  (bfloat16-valued in the BF16 form)
  const float* Td;   // [Z][F]
  const float* Ts;   // [Z][F]
  const float* W1;   // [F][F]  z_c = sum_e W1[c][e] h_e
  const float* W1T;  // [F][F]
  const float* w2;   // [F]
  float rc, sigma, escale;
  int Z;
};

__device__ __forceinline__ float bf16r(float x) { return (float)(__bf16)x; }
__device__ __forceinline__ short bf16bits(float x) { return __builtin_bit_cast(short, (__bf16)x); }

__device__ __forceinline__ float row16_sum(float v) {
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x141, 0xF, 0xF, false));
  v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x140, 0xF, 0xF, false));
  return v;
}

// Weights in LDS: W_r [c][k], the species tables and (forward kernel only) W1 [c][e].
template <bool kReadout>
struct SmallLds {
  float W[F_S * kLdW];
  float Td[Z_MAX][F_S], Ts[Z_MAX][F_S];
  // W1 [c][e] at c * (F + 1) + e (w1_at): a lane per row c (z = W1 h) or per column
  // (W1^T v) hits 64 distinct banks either way, and in both loops the address is the
  // lane's base plus a constant, so the reads need no address arithmetic
  float W1[kReadout ? F_S * kLdW1 : 1];
};

__device__ __forceinline__ int w1_at(int c, int e) { return c * kLdW1 + e; }

// Staging of the LDS weights in two halves: fetch() issues the thread's global loads into
// registers, store() writes them to LDS, so that independent work (the reverse kernel's
// first receiver loads) can overlap the loads.  The forward kernel stores them at once:
// holding them across its first receiver would raise its register peak.
template <bool kReadout>
struct Stager {
  static constexpr int kW = K_S * F_S, kT = Z_MAX * F_S, kR = kReadout ? F_S * F_S : 0;
  static constexpr int kN = kW + 2 * kT + kR;
  static constexpr int kPer = (kN + kWaves * 64 - 1) / (kWaves * 64);
  float v[kPer];
  __device__ __forceinline__ void fetch(const SmallParams& P) {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = threadIdx.x + kWaves * 64 * u;
      float x = 0.f;
      if (e < kW) x = P.WbT[e];
      else if (e < kW + kT) x = e - kW < P.Z * F_S ? P.Td[e - kW] : 0.f;
      else if (e < kW + 2 * kT) x = e - kW - kT < P.Z * F_S ? P.Ts[e - kW - kT] : 0.f;
      else if (e < kN) x = P.W1[e - kW - 2 * kT];
      v[u] = x;
    }
  }
  __device__ __forceinline__ void store(SmallLds<kReadout>& L) const {
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = threadIdx.x + kWaves * 64 * u;
      if (e < kW) L.W[(e % F_S) * kLdW + e / F_S] = v[u];
      else if (e < kW + kT) L.Td[(e - kW) / F_S][(e - kW) % F_S] = v[u];
      else if (e < kW + 2 * kT) L.Ts[(e - kW - kT) / F_S][(e - kW - kT) % F_S] = v[u];
      else if (kReadout && e < kN) {
        const int rr = (e - kW - 2 * kT) / F_S, cc = (e - kW - 2 * kT) % F_S;
        L.W1[w1_at(rr, cc)] = v[u];
      }
    }
  }
};

// 16 x 16 tile over K = 16 radial functions.  bk(e) / wk(e) give the lane's radial and
// weight operands for k = 4 e + g (FP32, e = step) or k = 4 g + e (BF16, e = element);
// b_is_a selects which of the two is the A operand; the products accumulate onto acc.
template <bool BF16, class BK, class WK>
__device__ __forceinline__ f32x4 radial_mfma(BK&& bk, WK&& wk, bool b_is_a, f32x4 acc) {
  if (BF16) {
    s16x4 x, y;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      x[e] = bf16bits(bk(e));
      y[e] = bf16bits(wk(e));
    }
    acc = b_is_a ? __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(x, y, acc, 0, 0, 0)
                 : __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(y, x, acc, 0, 0, 0);
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s)
      acc = b_is_a ? __builtin_amdgcn_mfma_f32_16x16x4f32(bk(s), wk(s), acc, 0, 0, 0)
                   : __builtin_amdgcn_mfma_f32_16x16x4f32(wk(s), bk(s), acc, 0, 0, 0);
  }
  return acc;
}

// One 16-pair tile of the receiver's compact row (pairs t0 .. t0 + 15 of the wave's LDS
// table), for the lane's channel block b (channel 16 b + cl) and D rows r (pair t0 + 4 g + r):
//   m[b][r]  = f_c SiLU(a)                                    the message
//   dm[b][r] = f_c' SiLU(a) + f_c SiLU'(a) (W_r b')_c          its derivative in r (DM only)
// with a = (W_r b)_c + T_d[z_i][c] + T_s[z_j][c].  Rows past the row give m = dm = 0 (no
// branches: they read slot 0 and are masked).  The message alone (DM false) skips the
// derivative's product; where both are computed, m has the same bits either way.
template <bool BF16, bool DM>
__device__ __forceinline__ void small_tile(const SmallLds<true>& L, const float4* sG,
                                           const int* sZ, int t0, int cnt, int zi_s, int g,
                                           int cl, float sigma, float inv_s2, float pi_rc,
                                           float (&m)[4][4], float (&dm)[4][4]) {
  const int pc = t0 + cl;   // pair of the A operand
  const bool vp = pc < cnt;
  const float rp = sG[vp ? pc : 0].w;
  float bv[4], dbv[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int kk = BF16 ? 4 * g + e : 4 * e + g;
    const float x = rp - sigma * kk;
    const float bb = __expf(vp ? -0.5f * x * x * inv_s2 : -1e30f);
    bv[e] = bb;
    dbv[e] = -x * inv_s2 * bb;
  }
  float fc[4], dfc[4];
  int zz[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int q = t0 + 4 * g + r;
    const bool v = q < cnt;
    const int qc = v ? q : 0;
    float sn, cs;
    __sincosf(pi_rc * sG[qc].w, &sn, &cs);
    fc[r] = v ? 0.5f * (cs + 1.0f) : 0.f;
    dfc[r] = v ? -0.5f * pi_rc * sn : 0.f;
    const int zq = sZ[qc];
    zz[r] = v ? zq : zi_s;
  }
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int c = 16 * b + cl;
    auto wk = [&](int e) {
      const int kk = BF16 ? 4 * g + e : 4 * e + g;
      return L.W[c * kLdW + kk];
    };
    // the receiver's table term starts the accumulator (the same for the block's rows)
    const float td = L.Td[zi_s][c];
    const f32x4 acc = radial_mfma<BF16>([&](int e) { return bv[e]; }, wk, true,
                                        f32x4{td, td, td, td});
    f32x4 accd = {0.f, 0.f, 0.f, 0.f};
    if (DM) accd = radial_mfma<BF16>([&](int e) { return dbv[e]; }, wk, true, accd);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float sv, dsv;
      silu_and_grad(acc[r] + L.Ts[zz[r]][c], sv, dsv);
      m[b][r] = fc[r] * sv;
      if (DM) dm[b][r] = fmaf(dfc[r], sv, fc[r] * dsv * accd[r]);
    }
    // one channel block at a time: the products of all four blocks in flight would hold
    // 32 more registers than the kernel can spare at three waves per SIMD
    __builtin_amdgcn_sched_barrier(0);
  }
}

// s_ij = dE_i/dr_ij = sum_c g_c dm[c] for the tile's pairs (gb[b] = g at channel 16 b + cl).
// The channel sum of pair t0 + 4 g + r is in-lane over b, then over the 16 lanes of group g;
// lane cl = r of the group writes s to the pair's list slot, spar[p], and the pair's record
// to the receiver's compact row, rec[k] = (d_ij / r_ij, p).
__device__ __forceinline__ void small_tile_store(const float (&dm)[4][4], const float (&gb)[4],
                                                 const float4* sG, const int* sP, int t0,
                                                 int cnt, int g, int cl,
                                                 float4* __restrict__ rec,
                                                 float* __restrict__ spar) {
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    float part = 0.f;
#pragma unroll
    for (int b = 0; b < 4; ++b) part = fmaf(gb[b], dm[b][r], part);
    part = row16_sum(part);
    const int q = t0 + 4 * g + r;
    if (cl == r && q < cnt) {
      const float4 gv = sG[q];
      const float ir = __builtin_amdgcn_rcpf(gv.w);
      const int p = sP[q];
      spar[p] = part;
      rec[q] = make_float4(gv.x * ir, gv.y * ir, gv.z * ir, __int_as_float(p));
    }
  }
}

// The evaluation kernel, one wavefront per receiver:
//   1. the receiver's list row (which may come from a longer cutoff) at the current
//      positions: the pairs inside the cutoff, in row order, go to an LDS table (pairs past
//      the per-atom cap raise the overflow flag and get s = 0);
//   2. the messages on MFMA tiles, summed into h_i in registers; with KEEP the derivative
//      factors dm/dr of the first two tiles stay in registers;
//   3. the readout: E_i and g_i = dE_i/dh_i;
//   4. s_ij = g_i . dm_ij/dr for every pair inside the cutoff (kept tiles from registers,
//      the others recomputed with the same arithmetic), written to the pair's list slot,
//      with the pair's record in the receiver's compact row (rec, cnt) for the force kernel.
// KEEP is a tile shape of the autotuner: registers capped at 168 (three waves per SIMD)
// with it, at 128 (four) without (asked for five, the compiler moves values into the
// accumulation registers and ends at three); 33 KiB of LDS lets four work-groups share a
// CU.
template <bool BF16, bool KEEP>
__global__ void __launch_bounds__(kWaves * 64) __attribute__((amdgpu_waves_per_eu(KEEP ? 3 : 4)))
k_small_eval(SmallParams P, const int32_t* __restrict__ offs, const int32_t* __restrict__ nbr,
             const double* __restrict__ pos, const int32_t* __restrict__ species, int n,
             double box, float* __restrict__ atom_e, float4* __restrict__ rec_all,
             float* __restrict__ spar, int32_t* __restrict__ cnt_all,
             uint32_t* __restrict__ flags) {
  __shared__ SmallLds<true> L;
  __shared__ int sZ[kWaves][kCap];
  __shared__ int sP[kWaves][kCap];
  __shared__ float4 sG[kWaves][kCap];
  __shared__ float sVec[kWaves][F_S];
  {
    Stager<true> stage;
    stage.fetch(P);
    stage.store(L);
  }
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, cl = lane & 15;
  const double inv_box = box > 0.0 ? 1.0 / box : 0.0;
  const float inv_s2 = 1.0f / (P.sigma * P.sigma);
  const float pi_rc = 3.14159265358979f / P.rc;
  const int n_wg = (n + kWaves - 1) / kWaves;
  for (int wg = blockIdx.x; wg < n_wg; wg += gridDim.x) {   // uniform over the work-group
    const int i = wg * kWaves + w;
    if (i >= n) continue;   // no work-group barrier below: waves leave independently
    // 1. pairs inside the cutoff, in row order
    int cnt = 0;
    {
      const double xi = pos[i], yi = pos[n + i], zi = pos[2 * n + i];
      const int row0 = offs[i], row1 = offs[i + 1];
      for (int base = row0; base < row1; base += 64) {
        const int p = base + lane;
        const int j = p < row1 ? nbr[p] : -1;
        // loads from the receiver itself where there is no pair: no branch, all loads of a
        // lane issue together
        const int jc = j >= 0 ? j : i;
        const int zj = species[jc];
        const float dx = static_cast<float>(minimage(pos[jc] - xi, box, inv_box));
        const float dy = static_cast<float>(minimage(pos[n + jc] - yi, box, inv_box));
        const float dz = static_cast<float>(minimage(pos[2 * n + jc] - zi, box, inv_box));
        const float r = sqrtf(dx * dx + dy * dy + dz * dz);
        const bool ok = j >= 0 && r < P.rc;
        const uint64_t mask = __ballot(ok);
        const int k = cnt + __popcll(mask & ((1ull << lane) - 1ull));
        if (ok && k < kCap) {
          sZ[w][k] = zj;
          sG[w][k] = make_float4(dx, dy, dz, r);
          sP[w][k] = p;
        } else if (ok) {
          spar[p] = 0.f;   // past the cap: left out of the sums (and flagged below)
        }
        cnt += __popcll(mask);
      }
      if (cnt > kCap) {
        if (lane == 0) atomicOr(flags, DMTS_FLAG_NBR_OVERFLOW);
        cnt = kCap;
      }
      if (lane == 0) cnt_all[i] = cnt;
    }
    wave_sync();
    float4* rec = rec_all + (size_t)i * kCap;
    // 2. messages on MFMA tiles, summed over pairs in registers
    const int zi_s = species[i];
    const float4* sg = sG[w];
    const int* sz = sZ[w];
    float hacc[4] = {0.f, 0.f, 0.f, 0.f};
    float m[4][4], dm0[4][4], dm1[4][4];
    auto add_h = [&]() {
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) hacc[b] += m[b][r];
    };
    constexpr int kKept = KEEP ? 2 : 0;   // tiles whose factors stay in registers
    if (KEEP) {
      small_tile<BF16, true>(L, sg, sz, 0, cnt, zi_s, g, cl, P.sigma, inv_s2, pi_rc, m, dm0);
      add_h();
      if (cnt > kTile) {
        small_tile<BF16, true>(L, sg, sz, kTile, cnt, zi_s, g, cl, P.sigma, inv_s2, pi_rc, m, dm1);
        add_h();
      }
    }
    for (int t0 = kKept * kTile; t0 < cnt; t0 += kTile) {
      float dmx[4][4];
      small_tile<BF16, false>(L, sg, sz, t0, cnt, zi_s, g, cl, P.sigma, inv_s2, pi_rc, m, dmx);
      add_h();
    }
    // h[c] for c = 16 b + cl: add the four pair groups
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      hacc[b] += __shfl_xor(hacc[b], 16, 64);
      hacc[b] += __shfl_xor(hacc[b], 32, 64);
    }
    if (g == 0) {
#pragma unroll
      for (int b = 0; b < 4; ++b) sVec[w][16 * b + cl] = BF16 ? bf16r(hacc[b]) : hacc[b];
    }
    wave_sync();
    // 3. readout, channel c = lane: z = W1 h, E_i = s_E w2 . SiLU(z), g = W1^T (s_E w2 SiLU'(z))
    const int c = lane;
    float z = 0.f;
#pragma unroll 16
    for (int e = 0; e < F_S; ++e) z = fmaf(L.W1[w1_at(c, e)], sVec[w][e], z);
    float y, dy;
    silu_and_grad(z, y, dy);
    const float w2 = P.w2[c];
    const float e_i = wave_sum(w2 * y) * P.escale;
    wave_sync();
    sVec[w][c] = BF16 ? bf16r(P.escale * w2 * dy) : P.escale * w2 * dy;
    wave_sync();
    float gi = 0.f;
#pragma unroll 16
    for (int k = 0; k < F_S; ++k) gi = fmaf(L.W1[w1_at(k, c)], sVec[w][k], gi);
    if (lane == 0) atom_e[i] = e_i;
    // 4. s_ij per pair into the pair's slot
    float gb[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) gb[b] = __shfl(gi, 16 * b + cl, 64);
    if (KEEP) {
      small_tile_store(dm0, gb, sg, sP[w], 0, cnt, g, cl, rec, spar);
      if (cnt > kTile) small_tile_store(dm1, gb, sg, sP[w], kTile, cnt, g, cl, rec, spar);
    }
    for (int t0 = kKept * kTile; t0 < cnt; t0 += kTile) {
      float dmx[4][4];
      small_tile<BF16, true>(L, sg, sz, t0, cnt, zi_s, g, cl, P.sigma, inv_s2, pi_rc, m, dmx);
      small_tile_store(dmx, gb, sg, sP[w], t0, cnt, g, cl, rec, spar);
    }
    wave_sync();
  }
}

// Forces F_i = sum_j (s_ij + s_ji) d_ij / r_ij over the receiver's compact row (the pairs
// inside the cutoff in row order, one per lane: the row holds at most 64), s_ji read from
// the reverse list slot rev[p].  The sum runs over the positions in the compact row, so the
// bits do not depend on the list's own cutoff or padding (a list built at the model's
// cutoff and a longer shared one give the same forces).  The kernel reads no positions, so
// the integrator program that follows the evaluation runs in its epilogue once F_i is
// final (a drift there cannot race with another wave).
__global__ void __launch_bounds__(256)
k_small_force(const int32_t* __restrict__ rev, int n, const float4* __restrict__ rec_all,
              const float* __restrict__ spar, const int32_t* __restrict__ cnt_all,
              float* __restrict__ forces, Epilogue E, bool has_ep, bool fresh_small) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + w;
  if (i >= n) return;
  CoordIn ein{};   // the atom's integrator inputs, coordinate d = lane (lanes 0..2)
  if (has_ep && lane < 3) ein = prefetch_coord(E, i, n, lane, fresh_small);
  const int cnt = cnt_all[i];
  float4 t = make_float4(0.f, 0.f, 0.f, 0.f);
  if (lane < cnt) {
    const float4 a = rec_all[(size_t)i * kCap + lane];
    const int p = __float_as_int(a.w);
    const int q = rev[p];
    // a missing reverse entry (an overflowed row) adds nothing
    const float s = spar[p] + (q >= 0 ? spar[q] : 0.f);
    t = make_float4(s * a.x, s * a.y, s * a.z, 0.f);
  }
  const float fx = wave_sum(t.x), fy = wave_sum(t.y), fz = wave_sum(t.z);
  if (lane == 0) {
    forces[i] = fx;
    forces[n + i] = fy;
    forces[2 * n + i] = fz;
  }
  if (has_ep) {   // F_i is final (every lane holds the sums): the integrator step of atom i
    apply_coords(E, i, n, lane, ein, lane == 0 ? fx : lane == 1 ? fy : fz, fresh_small);
  }
}

}  // namespace

// Workspace of one evaluation: the compact rows of pair records [n][kCap] (d/r, list slot),
// s per list slot (a list with room for max_pairs entries), the rows' lengths [n], atom
// energies [n], the energy partial sums.
size_t small_workspace_bytes(int32_t n, int64_t max_pairs) {
  const size_t N = (size_t)(n + 63) / 64 * 64;
  return sizeof(float4) * N * kCap + sizeof(float) * (size_t)max_pairs +
         sizeof(int32_t) * N + sizeof(float) * N + sizeof(double) * energy_partials(n) + 256;
}

dmts_status small_energy_forces(Model* m, NList* nl, const double* pos, const int32_t* species,
                                int32_t n, double box, const int32_t* sys_offsets, int32_t n_sys,
                                double* energy, float* forces, float* atom_energy, hipStream_t s,
                                const Epilogue* ep, char* ws) {
  DMTS_REQUIRE(m->K == K_S && m->F == F_S, DMTS_E_ARG, "small model: unsupported shape");
  const size_t N = (size_t)(n + 63) / 64 * 64;
  if (!ws) {
    DMTS_REQUIRE(m->atom_ws.reserve(small_workspace_bytes(n, nl->max_pairs), s) == DMTS_OK,
                 DMTS_E_OOM, "small model: workspace");
  }
  char* base = ws ? ws : m->atom_ws.as<char>();
  float4* rec = reinterpret_cast<float4*>(base);
  int32_t* cnt = reinterpret_cast<int32_t*>(rec + N * kCap);
  float* e_ws = reinterpret_cast<float*>(cnt + N);
  // 8-byte aligned: N % 64 == 0
  double* e_part = reinterpret_cast<double*>(e_ws + N);
  float* spar = reinterpret_cast<float*>(e_part + energy_partials(n));
  float* e_atom = atom_energy ? atom_energy : e_ws;
  SmallParams P{m->p(m->bf16 ? m->o_WbR : m->o_WbT), m->p(m->o_Td), m->p(m->o_Ts),
                m->p(m->bf16 ? m->o_W1R : m->o_W1), m->p(m->bf16 ? m->o_W1TR : m->o_W1T),
                m->p(m->o_w2), m->rc, m->sigma, m->escale, m->Z};
  if (n > 0) {
    const int natural = ceil_div(n, kWaves);
    // The integrator program (kicks and drifts) runs in the force kernel, per atom once its
    // force is final: the kernel reads no positions, so a drift cannot race with it.  The
    // forces computed here are the program's F_small or, when this model stands in for the
    // reference one (single-time-step runs), its F_large.  A program with an O-step runs as
    // a launch of its own.
    const bool fuse = ep && forces && (forces == ep->Fs || forces == ep->FL) &&
                      !has_thermo(ep->prog);
    const TileShape sh = m->shape_for(n);
    auto run = [&](auto bf_tag, auto keep_tag) {
      constexpr bool BF = decltype(bf_tag)::value;
      constexpr bool KEEP = decltype(keep_tag)::value;
      {
        ProfScope ps(DMTS_K_SMALL_FORWARD, s, true);
        const int blocks = launch_grid(
            sh.grid, natural,
            resident_groups(reinterpret_cast<const void*>(&k_small_eval<BF, KEEP>), kWaves * 64));
        launch_timed(ps, &k_small_eval<BF, KEEP>, dim3(blocks), dim3(kWaves * 64), s, P,
                     nl->offs, nl->nbr, pos, species, n, box, e_atom, rec, spar, cnt,
                     nl->flags);
      }
      if (hipPeekAtLastError() != hipSuccess || !forces) return;
      if (fuse && ep->wait) (void)hipStreamWaitEvent(s, ep->wait, 0);
      ProfScope ps(DMTS_K_SMALL_BACKWARD, s, true);
      launch_timed(ps, &k_small_force, dim3(ceil_div(n, 4)), dim3(256), s, nl->rev, n, rec,
                   spar, cnt, forces, fuse ? *ep : Epilogue{}, fuse, fuse && forces == ep->Fs);
    };
    if (m->bf16) {
      if (sh.keep) run(std::true_type{}, std::true_type{});
      else run(std::true_type{}, std::false_type{});
    } else {
      if (sh.keep) run(std::false_type{}, std::true_type{});
      else run(std::false_type{}, std::false_type{});
    }
    DMTS_CHECK_LAUNCH();
    if (ep && !fuse) {
      if (ep->wait) DMTS_HIP(hipStreamWaitEvent(s, ep->wait, 0));
      const dmts_status st = apply_program(*ep, n, s);
      if (st != DMTS_OK) return st;
    }
  }
  if (energy) return reduce_energy(e_atom, n, sys_offsets, n_sys, energy, e_part, s);
  return DMTS_OK;
}

// ------------------------------------------------------------------ allocation-free variant
// The workspace of nnp_energy_forces_noalloc: one array per device, kept for the life of the
// process, sized for kNoAllocMaxAtoms atoms on a list of at most kNoAllocMaxPairs entries.
// Host code never uses the array's name (it is a host-side stand-in for the symbol); it
// uses the device address from hipGetSymbolAddress.
constexpr int32_t kNoAllocMaxAtoms = 8192;
constexpr int64_t kNoAllocMaxPairs = int64_t(1) << 20;
constexpr size_t kNoAllocBytes = size_t(13) << 20;   // >= small_workspace_bytes(both maxima)
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch`, looked up once per device.
dmts_status scratch_address(void** out) {
  int dev = 0;
  DMTS_HIP(hipGetDevice(&dev));
  DMTS_REQUIRE(dev >= 0 && dev < kMaxDevices, DMTS_E_ARG, "noalloc: device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    DMTS_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    DMTS_REQUIRE(p != nullptr, DMTS_E_HIP, "noalloc: no device address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return DMTS_OK;
}
}  // namespace

}  // namespace dmts

extern "C" dmts_status nnp_energy_forces_noalloc(nnp_model* model, nnp_nlist* nl,
                                                 const double* pos, const int32_t* species,
                                                 int32_t n_atoms, double box,
                                                 const int32_t* sys_offsets, int32_t n_sys,
                                                 double* energy, float* forces,
                                                 float* atom_energy, void* stream) {
  using namespace dmts;
  Model* m = reinterpret_cast<Model*>(model);
  DMTS_REQUIRE(m, DMTS_E_ARG, "nnp_energy_forces_noalloc: null model");
  DMTS_REQUIRE(m->desc.kind == NNP_KIND_ONE_INTERACTION, DMTS_E_ARG,
               "nnp_energy_forces_noalloc: one-interaction models only");
  DMTS_REQUIRE(n_atoms >= 0 && n_atoms <= kNoAllocMaxAtoms, DMTS_E_CAPACITY,
               "nnp_energy_forces_noalloc: %d atoms, the fixed scratch holds at most %d",
               n_atoms, kNoAllocMaxAtoms);
  DMTS_REQUIRE(nl, DMTS_E_ARG, "nnp_energy_forces_noalloc: null list");
  const int64_t cap = reinterpret_cast<NList*>(nl)->max_pairs;
  DMTS_REQUIRE(cap <= kNoAllocMaxPairs, DMTS_E_CAPACITY,
               "nnp_energy_forces_noalloc: the list has room for %lld entries, the fixed "
               "scratch holds at most %lld", (long long)cap, (long long)kNoAllocMaxPairs);
  DMTS_REQUIRE(small_workspace_bytes(n_atoms, cap) <= kNoAllocBytes, DMTS_E_CAPACITY,
               "nnp_energy_forces_noalloc: workspace exceeds the fixed scratch");
  void* ws = nullptr;
  const dmts_status r = scratch_address(&ws);
  if (r != DMTS_OK) return r;
  return energy_forces(m, reinterpret_cast<NList*>(nl), pos, species, n_atoms, box, sys_offsets,
                       n_sys, energy, forces, atom_energy, static_cast<hipStream_t>(stream),
                       nullptr, static_cast<char*>(ws));
}
