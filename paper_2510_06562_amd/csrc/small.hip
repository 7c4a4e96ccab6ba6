// Fast (one-interaction) potential: energy and forces.
//
//   a_ij = W_r b(r_ij) + T_d[z_i] + T_s[z_j]      (T_d, T_s: the species-embedding blocks of
//                                                  W_pair folded with the embedding table)
//   m_ij = f_c(r_ij) SiLU(a_ij),  h_i = sum_j m_ij,  E_i = s_E w2 . SiLU(W1 h_i)
//
// Two kernels, one wavefront per receiver atom, one hidden channel per lane (F = 64):
//   k_small_forward:  pair messages summed into h_i, the readout, E_i and the adjoint
//                     g_i = dE/dh_i (stored, F floats per atom).
//   k_small_backward: recomputes every pair's features (nothing per pair is stored) and
//                     forms F_i = sum_j (s_ij + s_ji) d_ij / r_ij with
//                     s_ij = g_i . dm_ij/dr, where the reverse message m_ji differs from
//                     m_ij only by the swapped species tables, so one W_r b(r) serves both.
// Pair geometry (b, b', f_c, f_c', unit vector) is computed lane-per-pair for 64 pairs at
// a time and staged in LDS; the channel loop then reads it as wave-uniform broadcasts.
// Displacements are minimum-image differences of the float64 positions, rounded to float.
// BF16 form: the operands of the two contractions (W_r with b or b', W1 with h or its
// adjoint) are rounded to bfloat16 values (nearest even) and accumulated in FP32; the
// kernels run the same code with rounded weights and a rounding step on the activations.
#include "common.h"

namespace dmts {

namespace {

constexpr int kWaves = 4;
constexpr int K_S = 16;   // radial functions
constexpr int F_S = 64;   // hidden width
constexpr int Z_MAX = 8;

struct SmallParams {
  const float* WbT;  // [K][F]
  const float* Td;   // [Z][F]
  const float* Ts;   // [Z][F]
  const float* W1;   // [F][F]  z_c = sum_e W1[c][e] h_e
  const float* W1T;  // [F][F]
  const float* w2;   // [F]
  float rc, sigma, escale;
  int Z;
};

__device__ __forceinline__ float bf16r(float x) { return (float)(__bf16)x; }

struct PairStage {
  float b[64][K_S];
  float db[64][K_S];
  float fc[64], dfc[64];
  float rx[64], ry[64], rz[64];
  int z[64], j[64];
};

// Geometry of this lane's pair p (row entry) for receiver i; invalid entries get f_c = 0
// and b = 0 so that they contribute nothing.
__device__ __forceinline__ void stage_pair(PairStage& st, int lane, int p, int row1,
                                           const int32_t* nbr, const double* pos, int n,
                                           double box, double inv_box, double xi, double yi,
                                           double zi, const int32_t* species,
                                           const SmallParams& P, bool need_grad,
                                           bool bf16) {
  int j = p < row1 ? nbr[p] : -1;
  float r = 0.f, fc = 0.f, dfc = 0.f, ux = 0.f, uy = 0.f, uz = 0.f;
  bool valid = false;
  if (j >= 0) {
    float dx = static_cast<float>(minimage(pos[j] - xi, box, inv_box));
    float dy = static_cast<float>(minimage(pos[n + j] - yi, box, inv_box));
    float dz = static_cast<float>(minimage(pos[2 * n + j] - zi, box, inv_box));
    r = sqrtf(dx * dx + dy * dy + dz * dz);
    valid = r < P.rc;
    if (valid) {
      float ang = 3.14159265358979f * r / P.rc;
      float sn, cs;
      __sincosf(ang, &sn, &cs);
      fc = 0.5f * (cs + 1.0f);
      dfc = -0.5f * 3.14159265358979f / P.rc * sn;
      float inv = 1.0f / r;
      ux = dx * inv;
      uy = dy * inv;
      uz = dz * inv;
    }
  }
  const float inv_s2 = 1.0f / (P.sigma * P.sigma);
#pragma unroll
  for (int k = 0; k < K_S; ++k) {
    float x = r - P.sigma * k;   // mu_k = k r_c/(K-1) = k sigma
    float bk = valid ? __expf(-0.5f * x * x * inv_s2) : 0.f;
    const float dbk = -x * inv_s2 * bk;
    st.b[lane][k] = bf16 ? bf16r(bk) : bk;
    if (need_grad) st.db[lane][k] = bf16 ? bf16r(dbk) : dbk;
  }
  st.fc[lane] = fc;
  st.dfc[lane] = dfc;
  st.rx[lane] = ux;
  st.ry[lane] = uy;
  st.rz[lane] = uz;
  st.j[lane] = valid ? j : -1;
  st.z[lane] = valid ? species[j] : 0;
}

template <bool BF16>
__global__ void __launch_bounds__(kWaves * 64)
k_small_forward(SmallParams P, const int32_t* __restrict__ offs, const int32_t* __restrict__ nbr,
                const double* __restrict__ pos, const int32_t* __restrict__ species, int n,
                double box, float* __restrict__ atom_e, float* __restrict__ g_out) {
  __shared__ PairStage stage[kWaves];
  __shared__ float s_Ts[Z_MAX][F_S];
  __shared__ float s_vec[kWaves][F_S];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int e = threadIdx.x; e < P.Z * F_S; e += blockDim.x) s_Ts[e / F_S][e % F_S] = P.Ts[e];
  __syncthreads();
  const int n_wg = (n + kWaves - 1) / kWaves;
  for (int wg = blockIdx.x; wg < n_wg; wg += gridDim.x) {
  const int i = wg * kWaves + w;
  if (i >= n) continue;
  PairStage& st = stage[w];
  const double inv_box = box > 0.0 ? 1.0 / box : 0.0;
  const double xi = pos[i], yi = pos[n + i], zi = pos[2 * n + i];
  const int c = lane;
  float wb[K_S];
#pragma unroll
  for (int k = 0; k < K_S; ++k) wb[k] = P.WbT[k * F_S + c];
  const float td = P.Td[species[i] * F_S + c];
  float h = 0.f;
  const int row0 = offs[i], row1 = offs[i + 1];
  for (int base = row0; base < row1; base += 64) {
    stage_pair(st, lane, base + lane, row1, nbr, pos, n, box, inv_box, xi, yi, zi, species, P,
               false, BF16);
    wave_sync();
    const int nq = min(64, row1 - base);
    for (int q = 0; q < nq; ++q) {
      if (st.j[q] < 0) continue;   // wave-uniform
      float a = td + s_Ts[st.z[q]][c];
#pragma unroll
      for (int k = 0; k < K_S; ++k) a = fmaf(wb[k], st.b[q][k], a);
      h = fmaf(st.fc[q], silu_f(a), h);
    }
    wave_sync();
  }
  // readout: z = W1 h, E_i = s_E w2 . SiLU(z), and g = dE/dh = W1^T (s_E w2 * SiLU'(z))
  s_vec[w][c] = BF16 ? bf16r(h) : h;
  wave_sync();
  float z = 0.f;
  for (int e = 0; e < F_S; ++e) z = fmaf(P.W1T[e * F_S + c], s_vec[w][e], z);
  float y, dy;
  silu_and_grad(z, y, dy);
  const float w2 = P.w2[c];
  float e_i = wave_sum(w2 * y) * P.escale;
  wave_sync();
  s_vec[w][c] = BF16 ? bf16r(P.escale * w2 * dy) : P.escale * w2 * dy;
  wave_sync();
  float g = 0.f;
  for (int k = 0; k < F_S; ++k) g = fmaf(P.W1[k * F_S + c], s_vec[w][k], g);
  g_out[(size_t)i * F_S + c] = g;
  if (lane == 0) atom_e[i] = e_i;
  }  // grid-stride loop over work-groups of atoms
}

template <bool BF16>
__global__ void __launch_bounds__(kWaves * 64)
k_small_backward(SmallParams P, const int32_t* __restrict__ offs, const int32_t* __restrict__ nbr,
                 const double* __restrict__ pos, const int32_t* __restrict__ species, int n,
                 double box, const float* __restrict__ g, float* __restrict__ forces) {
  __shared__ PairStage stage[kWaves];
  __shared__ float s_Ts[Z_MAX][F_S];
  __shared__ float s_Td[Z_MAX][F_S];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int e = threadIdx.x; e < P.Z * F_S; e += blockDim.x) {
    s_Ts[e / F_S][e % F_S] = P.Ts[e];
    s_Td[e / F_S][e % F_S] = P.Td[e];
  }
  __syncthreads();
  const int n_wg = (n + kWaves - 1) / kWaves;
  for (int wg = blockIdx.x; wg < n_wg; wg += gridDim.x) {
  const int i = wg * kWaves + w;
  if (i >= n) continue;
  PairStage& st = stage[w];
  const double inv_box = box > 0.0 ? 1.0 / box : 0.0;
  const double xi = pos[i], yi = pos[n + i], zi = pos[2 * n + i];
  const int c = lane;
  float wb[K_S];
#pragma unroll
  for (int k = 0; k < K_S; ++k) wb[k] = P.WbT[k * F_S + c];
  const int zi_s = species[i];
  const float td_i = s_Td[zi_s][c], ts_i = s_Ts[zi_s][c];
  const float g_i = g[(size_t)i * F_S + c];
  float fx = 0.f, fy = 0.f, fz = 0.f;
  const int row0 = offs[i], row1 = offs[i + 1];
  for (int base = row0; base < row1; base += 64) {
    stage_pair(st, lane, base + lane, row1, nbr, pos, n, box, inv_box, xi, yi, zi, species, P,
               true, BF16);
    wave_sync();
    const int nq = min(64, row1 - base);
    for (int q = 0; q < nq; ++q) {
      const int j = st.j[q];
      if (j < 0) continue;
      const int zj = st.z[q];
      float gb = 0.f, gd = 0.f;
#pragma unroll
      for (int k = 0; k < K_S; ++k) {
        gb = fmaf(wb[k], st.b[q][k], gb);
        gd = fmaf(wb[k], st.db[q][k], gd);
      }
      const float a1 = gb + td_i + s_Ts[zj][c];   // message j -> i
      const float a2 = gb + s_Td[zj][c] + ts_i;   // message i -> j
      float s1, ds1, s2, ds2;
      silu_and_grad(a1, s1, ds1);
      silu_and_grad(a2, s2, ds2);
      const float g_j = g[(size_t)j * F_S + c];
      const float fc = st.fc[q], dfc = st.dfc[q];
      const float t = g_i * (dfc * s1 + fc * ds1 * gd) + g_j * (dfc * s2 + fc * ds2 * gd);
      fx = fmaf(t, st.rx[q], fx);
      fy = fmaf(t, st.ry[q], fy);
      fz = fmaf(t, st.rz[q], fz);
    }
    wave_sync();
  }
  fx = wave_sum(fx);
  fy = wave_sum(fy);
  fz = wave_sum(fz);
  if (lane == 0) {
    forces[i] = fx;
    forces[n + i] = fy;
    forces[2 * n + i] = fz;
  }
  }  // grid-stride loop over work-groups of atoms
}

}  // namespace

dmts_status small_energy_forces(Model* m, NList* nl, const double* pos, const int32_t* species,
                                int32_t n, double box, const int32_t* sys_offsets, int32_t n_sys,
                                double* energy, float* forces, float* atom_energy, hipStream_t s) {
  DMTS_REQUIRE(m->K == K_S && m->F == F_S, DMTS_E_ARG, "small model: unsupported shape");
  // workspace: atom energies [n] + adjoint g [n][F]
  size_t need = sizeof(float) * ((size_t)n * (1 + F_S) + 64);
  DMTS_REQUIRE(m->atom_ws.reserve(need, s) == DMTS_OK, DMTS_E_OOM, "small model: workspace");
  float* e_atom = atom_energy ? atom_energy : m->atom_ws.as<float>();
  float* g = m->atom_ws.as<float>() + ((size_t)n + 63) / 64 * 64;
  SmallParams P{m->p(m->bf16 ? m->o_WbR : m->o_WbT), m->p(m->o_Td), m->p(m->o_Ts),
                m->p(m->bf16 ? m->o_W1R : m->o_W1), m->p(m->bf16 ? m->o_W1TR : m->o_W1T),
                m->p(m->o_w2), m->rc, m->sigma, m->escale, m->Z};
  if (n > 0) {
    const int blocks = m->launch_grid(ceil_div(n, kWaves));
    { ProfScope ps(DMTS_K_SMALL_FORWARD, s);
    if (m->bf16)
      k_small_forward<true><<<blocks, kWaves * 64, 0, s>>>(P, nl->offs, nl->nbr, pos, species, n,
                                                           box, e_atom, g);
    else
      k_small_forward<false><<<blocks, kWaves * 64, 0, s>>>(P, nl->offs, nl->nbr, pos, species, n,
                                                            box, e_atom, g); }
    DMTS_CHECK_LAUNCH();
    if (forces) {
      { ProfScope ps(DMTS_K_SMALL_BACKWARD, s);
      if (m->bf16)
        k_small_backward<true><<<blocks, kWaves * 64, 0, s>>>(P, nl->offs, nl->nbr, pos, species,
                                                              n, box, g, forces);
      else
        k_small_backward<false><<<blocks, kWaves * 64, 0, s>>>(P, nl->offs, nl->nbr, pos, species,
                                                               n, box, g, forces); }
      DMTS_CHECK_LAUNCH();
    }
  }
  if (energy) return reduce_energy(e_atom, n, sys_offsets, n_sys, energy, s);
  return DMTS_OK;
}

}  // namespace dmts
