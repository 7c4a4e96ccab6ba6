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
//   pair1F -> GEMM U1 (+SiLU) -> GEMM [A|B] -> pair2F -> GEMM U2 (+residual SiLU)
//   -> GEMM W_o -> readout (E_i, dy) -> GEMM W_o^T (+SiLU') -> GEMM U2^T
//   -> pair2B (stores dE/da_ij per pair for the sender sums, v_ij = dE/dd_ij, and the
//      receiver sums) -> sender gather through rev[] -> GEMM [B;A]^T (+residual, SiLU')
//   -> GEMM U1^T -> pair1B (adds its v_ij) -> force gather F_i = sum_j v_ij - v_ji.
// The pair kernels run one wavefront per receiver, channels on lanes (two per lane);
// pair geometry is staged in LDS 64 pairs at a time and recomputed in the reverse pass.
// No floating-point atomics: every sum has a fixed order, so results are bitwise
// reproducible.
#include "atom_mlp.h"

namespace dmts {

namespace {

constexpr int kWaves = 4;
constexpr int K_L = 32;
constexpr int F_L = 128;
constexpr int Z_MAX = 8;
constexpr int NMOM = 10;   // M0, M1 (x, y, z), M2 (xx, yy, zz, xy, xz, yz)

struct LargeParams {
  const float* WbT;   // [K][F] radial block of the interaction
  const float* Td;    // [Z][F] layer 1 receiver table
  const float* Ts;    // [Z][F] layer 1 sender table
  float rc, sigma;
  int Z;
};

struct Stage {
  float b[64][K_L];
  float db[64][K_L];
  float fc[64], dfc[64];
  float ux[64], uy[64], uz[64];       // d / r_c
  float rx[64], ry[64], rz[64];       // d / r
  int z[64], j[64];
};

__device__ __forceinline__ void stage_pair(Stage& st, int lane, int p, int row1,
                                           const int32_t* nbr, const double* pos, int n,
                                           double box, double inv_box, double xi, double yi,
                                           double zi, const int32_t* species,
                                           const LargeParams& P, bool need_grad) {
  int j = p < row1 ? nbr[p] : -1;
  float r = 0.f, fc = 0.f, dfc = 0.f, dx = 0.f, dy = 0.f, dz = 0.f;
  bool valid = false;
  if (j >= 0) {
    dx = static_cast<float>(minimage(pos[j] - xi, box, inv_box));
    dy = static_cast<float>(minimage(pos[n + j] - yi, box, inv_box));
    dz = static_cast<float>(minimage(pos[2 * n + j] - zi, box, inv_box));
    r = sqrtf(dx * dx + dy * dy + dz * dz);
    valid = r < P.rc;
    if (valid) {
      float sn, cs;
      __sincosf(3.14159265358979f * r / P.rc, &sn, &cs);
      fc = 0.5f * (cs + 1.0f);
      dfc = -0.5f * 3.14159265358979f / P.rc * sn;
    }
  }
  const float inv_s2 = 1.0f / (P.sigma * P.sigma);
#pragma unroll
  for (int k = 0; k < K_L; ++k) {
    float x = r - P.sigma * k;
    float bk = valid ? __expf(-0.5f * x * x * inv_s2) : 0.f;
    st.b[lane][k] = bk;
    if (need_grad) st.db[lane][k] = -x * inv_s2 * bk;
  }
  const float irc = 1.0f / P.rc;
  const float ir = valid ? 1.0f / r : 0.f;
  st.fc[lane] = fc;
  st.dfc[lane] = dfc;
  st.ux[lane] = valid ? dx * irc : 0.f;
  st.uy[lane] = valid ? dy * irc : 0.f;
  st.uz[lane] = valid ? dz * irc : 0.f;
  st.rx[lane] = dx * ir;
  st.ry[lane] = dy * ir;
  st.rz[lane] = dz * ir;
  st.j[lane] = valid ? j : -1;
  st.z[lane] = valid ? species[j] : 0;
}

// Moments of one channel.
struct Mom {
  float m0, x, y, z, xx, yy, zz, xy, xz, yz;
  __device__ void zero() { m0 = x = y = z = xx = yy = zz = xy = xz = yz = 0.f; }
};

__device__ __forceinline__ void accumulate(Mom& M, float m, float ux, float uy, float uz,
                                           float u2) {
  const float t3 = u2 * (1.0f / 3.0f);
  M.m0 += m;
  M.x = fmaf(m, ux, M.x);
  M.y = fmaf(m, uy, M.y);
  M.z = fmaf(m, uz, M.z);
  M.xx = fmaf(m, ux * ux - t3, M.xx);
  M.yy = fmaf(m, uy * uy - t3, M.yy);
  M.zz = fmaf(m, uz * uz - t3, M.zz);
  M.xy = fmaf(m, ux * uy, M.xy);
  M.xz = fmaf(m, ux * uz, M.xz);
  M.yz = fmaf(m, uy * uz, M.yz);
}

__device__ __forceinline__ void store_moments(const Mom& M, float* Mout, float* q, int c) {
  Mout[0 * F_L + c] = M.m0;
  Mout[1 * F_L + c] = M.x;
  Mout[2 * F_L + c] = M.y;
  Mout[3 * F_L + c] = M.z;
  Mout[4 * F_L + c] = M.xx;
  Mout[5 * F_L + c] = M.yy;
  Mout[6 * F_L + c] = M.zz;
  Mout[7 * F_L + c] = M.xy;
  Mout[8 * F_L + c] = M.xz;
  Mout[9 * F_L + c] = M.yz;
  q[c] = M.m0;
  q[F_L + c] = M.x * M.x + M.y * M.y + M.z * M.z;
  q[2 * F_L + c] = M.xx * M.xx + M.yy * M.yy + M.zz * M.zz +
                   2.0f * (M.xy * M.xy + M.xz * M.xz + M.yz * M.yz);
}

// LAYER 1: species tables; LAYER 2: per-atom projections P2 = [A | B] (sender | receiver).
template <int LAYER>
__global__ void __launch_bounds__(kWaves * 64)
k_pair_forward(LargeParams P, const int32_t* __restrict__ offs, const int32_t* __restrict__ nbr,
               const double* __restrict__ pos, const int32_t* __restrict__ species, int n,
               double box, const float* __restrict__ P2, float* __restrict__ Mout,
               float* __restrict__ q) {
  __shared__ Stage stage[kWaves];
  __shared__ float s_Ts[LAYER == 1 ? Z_MAX : 1][F_L];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (LAYER == 1)
    for (int e = threadIdx.x; e < P.Z * F_L; e += blockDim.x) s_Ts[e / F_L][e % F_L] = P.Ts[e];
  __syncthreads();
  const int i = blockIdx.x * kWaves + w;
  if (i >= n) return;
  Stage& st = stage[w];
  const double inv_box = box > 0.0 ? 1.0 / box : 0.0;
  const double xi = pos[i], yi = pos[n + i], zi = pos[2 * n + i];
  const int c0 = lane, c1 = lane + 64;
  float wb0[K_L], wb1[K_L];
#pragma unroll
  for (int k = 0; k < K_L; ++k) {
    wb0[k] = P.WbT[k * F_L + c0];
    wb1[k] = P.WbT[k * F_L + c1];
  }
  float base0, base1;
  if (LAYER == 1) {
    base0 = P.Td[species[i] * F_L + c0];
    base1 = P.Td[species[i] * F_L + c1];
  } else {
    base0 = P2[(size_t)i * 2 * F_L + F_L + c0];
    base1 = P2[(size_t)i * 2 * F_L + F_L + c1];
  }
  Mom A, B;
  A.zero();
  B.zero();
  const int row0 = offs[i], row1 = offs[i + 1];
  for (int base = row0; base < row1; base += 64) {
    stage_pair(st, lane, base + lane, row1, nbr, pos, n, box, inv_box, xi, yi, zi, species, P,
               false);
    wave_sync();
    const int nq = min(64, row1 - base);
    for (int q0 = 0; q0 < nq; ++q0) {
      const int j = st.j[q0];
      if (j < 0) continue;
      float a0, a1;
      if (LAYER == 1) {
        a0 = base0 + s_Ts[st.z[q0]][c0];
        a1 = base1 + s_Ts[st.z[q0]][c1];
      } else {
        a0 = base0 + P2[(size_t)j * 2 * F_L + c0];
        a1 = base1 + P2[(size_t)j * 2 * F_L + c1];
      }
#pragma unroll
      for (int k = 0; k < K_L; ++k) {
        const float bk = st.b[q0][k];
        a0 = fmaf(wb0[k], bk, a0);
        a1 = fmaf(wb1[k], bk, a1);
      }
      const float fc = st.fc[q0];
      const float ux = st.ux[q0], uy = st.uy[q0], uz = st.uz[q0];
      const float u2 = ux * ux + uy * uy + uz * uz;
      accumulate(A, fc * silu_f(a0), ux, uy, uz, u2);
      accumulate(B, fc * silu_f(a1), ux, uy, uz, u2);
    }
    wave_sync();
  }
  float* Mi = Mout + (size_t)i * NMOM * F_L;
  float* qi = q + (size_t)i * 3 * F_L;
  store_moments(A, Mi, qi, c0);
  store_moments(B, Mi, qi, c1);
}

// Per-channel reverse-mode state of one receiver: dE/dM (M2 part as a symmetric matrix).
struct DMom {
  float m0, x, y, z, xx, yy, zz, xy, xz, yz, tr;
};

__device__ __forceinline__ DMom load_dmom(const float* Mi, const float* dqi, int c) {
  DMom d;
  d.m0 = dqi[c];
  const float s1 = 2.0f * dqi[F_L + c];
  const float s2 = 2.0f * dqi[2 * F_L + c];
  d.x = s1 * Mi[1 * F_L + c];
  d.y = s1 * Mi[2 * F_L + c];
  d.z = s1 * Mi[3 * F_L + c];
  d.xx = s2 * Mi[4 * F_L + c];
  d.yy = s2 * Mi[5 * F_L + c];
  d.zz = s2 * Mi[6 * F_L + c];
  d.xy = s2 * Mi[7 * F_L + c];
  d.xz = s2 * Mi[8 * F_L + c];
  d.yz = s2 * Mi[9 * F_L + c];
  d.tr = d.xx + d.yy + d.zz;
  return d;
}

// One channel's share of a pair's reverse pass.  Returns dE/da (for the feature sums)
// and adds the channel's contribution to v = dE/dd into (vx, vy, vz).
__device__ __forceinline__ float pair_channel_backward(const DMom& d, float a, float gd, float fc,
                                                       float dfc, float ux, float uy, float uz,
                                                       float u2, float rx, float ry, float rz,
                                                       float inv_rc, float& vx, float& vy,
                                                       float& vz) {
  float s, ds;
  silu_and_grad(a, s, ds);
  const float m = fc * s;
  const float t3 = u2 * (1.0f / 3.0f);
  const float dm = d.m0 + d.x * ux + d.y * uy + d.z * uz + d.xx * (ux * ux - t3) +
                   d.yy * (uy * uy - t3) + d.zz * (uz * uz - t3) +
                   2.0f * (d.xy * ux * uy + d.xz * ux * uz + d.yz * uy * uz);
  const float da = dm * fc * ds;
  const float rho = dm * s * dfc + da * gd;   // dE/dr through f_c and b(r)
  // dE/du through u and Y2(u): m (dM1 + 2 dM2 u - 2/3 tr(dM2) u)
  const float mr = m * inv_rc;
  const float ax = d.x + 2.0f * (d.xx * ux + d.xy * uy + d.xz * uz) - (2.0f / 3.0f) * d.tr * ux;
  const float ay = d.y + 2.0f * (d.xy * ux + d.yy * uy + d.yz * uz) - (2.0f / 3.0f) * d.tr * uy;
  const float az = d.z + 2.0f * (d.xz * ux + d.yz * uy + d.zz * uz) - (2.0f / 3.0f) * d.tr * uz;
  vx += rho * rx + mr * ax;
  vy += rho * ry + mr * ay;
  vz += rho * rz + mr * az;
  return da;
}

// LAYER 2 stores dE/da_ij per pair (dA) and the receiver sums (RS[:, 0:F]); LAYER 1 adds its
// v_ij into the per-pair vector accumulated by layer 2.
template <int LAYER>
__global__ void __launch_bounds__(kWaves * 64)
k_pair_backward(LargeParams P, const int32_t* __restrict__ offs, const int32_t* __restrict__ nbr,
                const double* __restrict__ pos, const int32_t* __restrict__ species, int n,
                double box, const float* __restrict__ P2, const float* __restrict__ Mall,
                const float* __restrict__ dq, float* __restrict__ dA, float* __restrict__ RS,
                float* __restrict__ v, int64_t cap) {
  __shared__ Stage stage[kWaves];
  __shared__ float s_Ts[LAYER == 1 ? Z_MAX : 1][F_L];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (LAYER == 1)
    for (int e = threadIdx.x; e < P.Z * F_L; e += blockDim.x) s_Ts[e / F_L][e % F_L] = P.Ts[e];
  __syncthreads();
  const int i = blockIdx.x * kWaves + w;
  if (i >= n) return;
  Stage& st = stage[w];
  const double inv_box = box > 0.0 ? 1.0 / box : 0.0;
  const double xi = pos[i], yi = pos[n + i], zi = pos[2 * n + i];
  const int c0 = lane, c1 = lane + 64;
  float wb0[K_L], wb1[K_L];
#pragma unroll
  for (int k = 0; k < K_L; ++k) {
    wb0[k] = P.WbT[k * F_L + c0];
    wb1[k] = P.WbT[k * F_L + c1];
  }
  float base0, base1;
  if (LAYER == 1) {
    base0 = P.Td[species[i] * F_L + c0];
    base1 = P.Td[species[i] * F_L + c1];
  } else {
    base0 = P2[(size_t)i * 2 * F_L + F_L + c0];
    base1 = P2[(size_t)i * 2 * F_L + F_L + c1];
  }
  const float* Mi = Mall + (size_t)i * NMOM * F_L;
  const float* dqi = dq + (size_t)i * 3 * F_L;
  const DMom d0 = load_dmom(Mi, dqi, c0);
  const DMom d1 = load_dmom(Mi, dqi, c1);
  const float inv_rc = 1.0f / P.rc;
  float R0 = 0.f, R1 = 0.f;
  const int row0 = offs[i], row1 = offs[i + 1];
  for (int base = row0; base < row1; base += 64) {
    stage_pair(st, lane, base + lane, row1, nbr, pos, n, box, inv_box, xi, yi, zi, species, P,
               true);
    wave_sync();
    const int nq = min(64, row1 - base);
    float vx_mine = 0.f, vy_mine = 0.f, vz_mine = 0.f;
    for (int q0 = 0; q0 < nq; ++q0) {
      const int j = st.j[q0];
      if (j < 0) {
        // padding, or a listed pair beyond this model's cutoff: no message, but the
        // sender gather reads dA of every listed pair
        if (LAYER == 2) {
          const size_t p = (size_t)(base + q0);
          dA[p * F_L + c0] = 0.f;
          dA[p * F_L + c1] = 0.f;
        }
        continue;
      }
      float a0, a1;
      if (LAYER == 1) {
        a0 = base0 + s_Ts[st.z[q0]][c0];
        a1 = base1 + s_Ts[st.z[q0]][c1];
      } else {
        a0 = base0 + P2[(size_t)j * 2 * F_L + c0];
        a1 = base1 + P2[(size_t)j * 2 * F_L + c1];
      }
      float gd0 = 0.f, gd1 = 0.f;
#pragma unroll
      for (int k = 0; k < K_L; ++k) {
        const float bk = st.b[q0][k], dbk = st.db[q0][k];
        a0 = fmaf(wb0[k], bk, a0);
        a1 = fmaf(wb1[k], bk, a1);
        gd0 = fmaf(wb0[k], dbk, gd0);
        gd1 = fmaf(wb1[k], dbk, gd1);
      }
      const float fc = st.fc[q0], dfc = st.dfc[q0];
      const float ux = st.ux[q0], uy = st.uy[q0], uz = st.uz[q0];
      const float rx = st.rx[q0], ry = st.ry[q0], rz = st.rz[q0];
      const float u2 = ux * ux + uy * uy + uz * uz;
      float vx = 0.f, vy = 0.f, vz = 0.f;
      const float da0 = pair_channel_backward(d0, a0, gd0, fc, dfc, ux, uy, uz, u2, rx, ry, rz,
                                              inv_rc, vx, vy, vz);
      const float da1 = pair_channel_backward(d1, a1, gd1, fc, dfc, ux, uy, uz, u2, rx, ry, rz,
                                              inv_rc, vx, vy, vz);
      if (LAYER == 2) {
        const size_t p = (size_t)(base + q0);
        dA[p * F_L + c0] = da0;
        dA[p * F_L + c1] = da1;
        R0 += da0;
        R1 += da1;
      }
      vx = wave_sum(vx);
      vy = wave_sum(vy);
      vz = wave_sum(vz);
      if (lane == q0) {
        vx_mine = vx;
        vy_mine = vy;
        vz_mine = vz;
      }
    }
    const int p = base + lane;
    if (lane < nq) {
      if (LAYER == 2) {
        v[p] = vx_mine;
        v[cap + p] = vy_mine;
        v[2 * cap + p] = vz_mine;
      } else {
        v[p] += vx_mine;
        v[cap + p] += vy_mine;
        v[2 * cap + p] += vz_mine;
      }
    }
    wave_sync();
  }
  if (LAYER == 2) {
    RS[(size_t)i * 2 * F_L + c0] = R0;
    RS[(size_t)i * 2 * F_L + c1] = R1;
  }
}

// S_j = sum over the rows of j of dA at the reverse positions (the sender sums).
__global__ void __launch_bounds__(kWaves * 64)
k_sender_gather(const int32_t* __restrict__ offs, const int32_t* __restrict__ nbr,
                const int32_t* __restrict__ rev, int n, const float* __restrict__ dA,
                float* __restrict__ RS) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * kWaves + w;
  if (i >= n) return;
  float s0 = 0.f, s1 = 0.f;
  const int row0 = offs[i], row1 = offs[i + 1];
  for (int p = row0; p < row1; ++p) {
    if (nbr[p] < 0) break;
    const int q = rev[p];
    if (q < 0) continue;
    s0 += dA[(size_t)q * F_L + lane];
    s1 += dA[(size_t)q * F_L + lane + 64];
  }
  RS[(size_t)i * 2 * F_L + F_L + lane] = s0;
  RS[(size_t)i * 2 * F_L + F_L + lane + 64] = s1;
}

}  // namespace

// F_i = sum_{p in row i} v[p] - v[rev[p]]  (v[p] = dE/dd_ij, d_ij = x_j - x_i)
__global__ void __launch_bounds__(256)
k_force_gather(const int32_t* __restrict__ offs, const int32_t* __restrict__ nbr,
               const int32_t* __restrict__ rev, int n, const float* __restrict__ v, int64_t cap,
               float* __restrict__ forces) {
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + w;
  if (i >= n) return;
  float fx = 0.f, fy = 0.f, fz = 0.f;
  const int row0 = offs[i], row1 = offs[i + 1];
  for (int p = row0 + lane; p < row1; p += 64) {
    if (nbr[p] < 0) continue;
    const int q = rev[p];
    if (q < 0) continue;
    fx += v[p] - v[q];
    fy += v[cap + p] - v[cap + q];
    fz += v[2 * cap + p] - v[2 * cap + q];
  }
  fx = wave_sum(fx);
  fy = wave_sum(fy);
  fz = wave_sum(fz);
  if (lane == 0) {
    forces[i] = fx;
    forces[n + i] = fy;
    forces[2 * n + i] = fz;
  }
}

dmts_status large_energy_forces(Model* m, NList* nl, const double* pos, const int32_t* species,
                                int32_t n, double box, const int32_t* sys_offsets, int32_t n_sys,
                                double* energy, float* forces, float* atom_energy, hipStream_t s) {
  DMTS_REQUIRE(m->K == K_L && m->F == F_L, DMTS_E_ARG, "large model: unsupported shape");
  const size_t F = F_L, N = (size_t)((n + 63) / 64 * 64);
  // per-atom workspace layout (floats)
  const size_t o_q1 = 0, o_M1 = o_q1 + N * 3 * F, o_z1 = o_M1 + N * NMOM * F;
  const size_t o_h1 = o_z1 + N * F, o_P2 = o_h1 + N * F, o_q2 = o_P2 + N * 2 * F;
  const size_t o_M2 = o_q2 + N * 3 * F, o_dh2 = o_M2 + N * NMOM * F;
  const size_t o_dq2 = o_dh2 + N * F, o_RS = o_dq2 + N * 3 * F;
  const size_t o_dq1 = o_RS + N * 2 * F, o_e = o_dq1 + N * 3 * F;
  const size_t total = o_e + N;
  DMTS_REQUIRE(m->atom_ws.reserve(total * sizeof(float), s) == DMTS_OK, DMTS_E_OOM,
               "large model: atom workspace");
  const int64_t cap = nl->max_pairs;
  if (forces) {
    DMTS_REQUIRE(m->pair_ws.reserve(sizeof(float) * (size_t)cap * (F + 3), s) == DMTS_OK,
                 DMTS_E_OOM, "large model: pair workspace");
  }
  float* W = m->atom_ws.as<float>();
  float* e_atom = atom_energy ? atom_energy : W + o_e;
  LargeParams P1{m->p(m->o_WbT), m->p(m->o_Td), m->p(m->o_Ts), m->rc, m->sigma, m->Z};
  LargeParams P2{m->p(m->o_W2bT), nullptr, nullptr, m->rc, m->sigma, m->Z};
  AtomMlpParams A{m->p(m->o_U1T), m->p(m->o_W2hT), m->p(m->o_U2T), m->p(m->o_WoT),
                  m->p(m->o_wo),  m->p(m->o_Wo),   m->p(m->o_U2),  m->p(m->o_W2hs),
                  m->p(m->o_U1)};
  const int blocks = ceil_div(n, kWaves);
  dmts_status st;
  if (n > 0) {
    { ProfScope ps(DMTS_K_PAIR1_FORWARD, s);
    k_pair_forward<1><<<blocks, kWaves * 64, 0, s>>>(P1, nl->offs, nl->nbr, pos, species, n, box,
                                                     nullptr, W + o_M1, W + o_q1); }
    DMTS_CHECK_LAUNCH();
    if ((st = atom_chain1(A, n, W + o_q1, W + o_z1, W + o_h1, W + o_P2, s)) != DMTS_OK) return st;
    { ProfScope ps(DMTS_K_PAIR2_FORWARD, s);
    k_pair_forward<2><<<blocks, kWaves * 64, 0, s>>>(P2, nl->offs, nl->nbr, pos, species, n, box,
                                                     W + o_P2, W + o_M2, W + o_q2); }
    DMTS_CHECK_LAUNCH();
    if ((st = atom_chain2(A, n, W + o_q2, W + o_h1, m->escale, e_atom, W + o_dh2, W + o_dq2,
                          forces != nullptr, s)) != DMTS_OK) return st;
    if (forces) {
      float* dA = m->pair_ws.as<float>();
      float* v = dA + (size_t)cap * F;
      { ProfScope ps(DMTS_K_PAIR2_BACKWARD, s);
      k_pair_backward<2><<<blocks, kWaves * 64, 0, s>>>(P2, nl->offs, nl->nbr, pos, species, n,
                                                        box, W + o_P2, W + o_M2, W + o_dq2, dA,
                                                        W + o_RS, v, cap); }
      DMTS_CHECK_LAUNCH();
      { ProfScope ps(DMTS_K_GATHER, s);
      k_sender_gather<<<blocks, kWaves * 64, 0, s>>>(nl->offs, nl->nbr, nl->rev, n, dA, W + o_RS); }
      DMTS_CHECK_LAUNCH();
      if ((st = atom_chain3(A, n, W + o_RS, W + o_dh2, W + o_z1, W + o_dq1, s)) != DMTS_OK)
        return st;
      { ProfScope ps(DMTS_K_PAIR1_BACKWARD, s);
      k_pair_backward<1><<<blocks, kWaves * 64, 0, s>>>(P1, nl->offs, nl->nbr, pos, species, n,
                                                        box, nullptr, W + o_M1, W + o_dq1, nullptr,
                                                        nullptr, v, cap); }
      DMTS_CHECK_LAUNCH();
      { ProfScope ps(DMTS_K_GATHER, s);
      k_force_gather<<<blocks, 256, 0, s>>>(nl->offs, nl->nbr, nl->rev, n, v, cap, forces); }
      DMTS_CHECK_LAUNCH();
    }
  }
  if (energy) return reduce_energy(e_atom, n, sys_offsets, n_sys, energy, s);
  return DMTS_OK;
}

}  // namespace dmts
