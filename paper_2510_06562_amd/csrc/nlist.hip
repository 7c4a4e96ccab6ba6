// Neighbor lists for the message-passing sums of both potentials.
//
// The pair set is {(i, j): j != i, |d_ij| < r_c} with d_ij = x_j - x_i under the
// minimum-image convention of a cube (plain difference for open boundaries, restricted
// to one molecule for a batch).  The paper leaves the search unspecified; this is a
// cell list: atoms are binned into cells of edge >= r_c, each receiver scans the 27
// surrounding cells (all atoms of its molecule, or all atoms, when there are fewer than 3
// cells per edge).  One wavefront per receiver walks the candidate stream; a ballot
// compacts the accepted senders into LDS, where they are rank-sorted by index.  Rows are
// therefore ascending in j whatever order the binning produced, so the list, and every
// floating-point sum taken along it, is bitwise reproducible.
//
// Launches per build: bin (cell id + count), scan of cells, scatter, rows (search + sort
// into a fixed-width staging table), scan of row lengths, compaction into CSR with the
// reverse index rev[p] (binary search of i in the sorted row of j).  Rows are padded with
// -1 to a multiple of the list's row alignment.
//
// The integrator's reference evaluations go through a skin list instead (a Verlet list:
// rows at r_c + skin, valid while no atom has moved skin/2 since they were built).  Per
// evaluation: the displacement test (inside the one-work-group binning, or a launch of its
// own), binning only if it failed, then one launch that rebuilds a receiver's skin row
// when asked and filters it to r_c at the current positions, then the scan and compaction
// above.  Filtering keeps the ascending order, and a row at r_c + skin holds every pair
// within r_c while the bound holds, so the list is exactly the one a fresh build gives.
#include "common.h"

namespace dmts {

namespace {

constexpr int kScanThreads = 256;
constexpr int kMaxCellsPerDim = 64;

__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Exclusive scan of in[0..n) into out[0..n] in two launches over tiles of kScanTile
// elements: k_scan_sums writes each tile's total, k_scan_tiles adds the totals of the
// tiles before its own and scans its tile.  Every load and store is coalesced (lane-
// contiguous runs) and the work per lane is a few elements, so the latency of a long
// serial loop is gone.  When the total exceeds `cap` the list would not fit: every
// offset is set to 0 (all rows empty) and the overflow flag is raised, so no consumer
// can index past the capacity.  With `zero_in`, the input is cleared after it has been
// read (the cell counters are then ready for the next build without a separate fill).
constexpr int kScanPer = 4;
constexpr int kScanTile = kScanThreads * kScanPer;

__device__ __forceinline__ int64_t block_sum_i64(int64_t v, int64_t* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();  // red may still be read by a previous call
  if (lane == 0) red[w] = v;
  __syncthreads();
  int64_t t = 0;
  for (int k = 0; k < kScanThreads / 64; ++k) t += red[k];
  return t;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_sums(const int32_t* __restrict__ in,
                                                           int32_t n,
                                                           int64_t* __restrict__ part,
                                                           const uint32_t* __restrict__ gate) {
  __shared__ int64_t red[kScanThreads / 64];
  if (gate && gate[0] == 0u) return;
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t s = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    const int64_t k = base + i * kScanThreads + threadIdx.x;
    s += k < n ? in[k] : 0;
  }
  s = block_sum_i64(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(int32_t* __restrict__ in,
                                                            int32_t* __restrict__ out,
                                                            int32_t* __restrict__ copy_to,
                                                            int32_t n, int64_t cap,
                                                            uint32_t* __restrict__ flags,
                                                            bool zero_in,
                                                            const int64_t* __restrict__ part,
                                                            int n_tiles,
                                                            const uint32_t* __restrict__ gate) {
  __shared__ int64_t red[kScanThreads / 64];
  __shared__ int64_t wsum[kScanThreads / 64];
  if (gate && gate[0] == 0u) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  // offset of this tile and the grand total
  int64_t before = 0, all = 0;
  for (int k = t; k < n_tiles; k += kScanThreads) {
    const int64_t v = part[k];
    all += v;
    before += k < (int)blockIdx.x ? v : 0;
  }
  before = block_sum_i64(before, red);
  const int64_t total = block_sum_i64(all, red);
  const bool overflow = total > cap;
  // this lane's run of kScanPer consecutive elements
  const int64_t k0 = (int64_t)blockIdx.x * kScanTile + (int64_t)t * kScanPer;
  int32_t v[kScanPer];
  int64_t run = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    v[i] = k0 + i < n ? in[k0 + i] : 0;
    run += v[i];
  }
  // inclusive scan of the lane sums within the wave, then across the waves
  int64_t incl = run;
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t u = __shfl_up(incl, off, 64);
    if (lane >= off) incl += u;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int64_t wbase = 0;
  for (int k = 0; k < w; ++k) wbase += wsum[k];
  int64_t o = before + wbase + incl - run;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    if (k0 + i < n) {
      const int32_t r = overflow ? 0 : static_cast<int32_t>(o);
      out[k0 + i] = r;
      if (copy_to) copy_to[k0 + i] = r;
      if (zero_in) in[k0 + i] = 0;
    }
    o += v[i];
  }
  if (blockIdx.x == 0 && t == 0) {
    out[n] = overflow ? 0 : static_cast<int32_t>(total);
    if (overflow && flags) atomicOr(flags, DMTS_FLAG_NBR_OVERFLOW);
  }
}

int scan_tiles(int64_t n) { return n <= 0 ? 1 : (int)((n + kScanTile - 1) / kScanTile); }

// Up to kScanOne elements: one work-group of 1,024 threads, eight consecutive elements per
// lane (one launch instead of two), the same exclusive scan, cap and flag as above.
constexpr int kScanOneThreads = 1024, kScanOnePer = 8;
constexpr int kScanOne = kScanOneThreads * kScanOnePer;

__global__ void __launch_bounds__(kScanOneThreads) k_scan_one(int32_t* __restrict__ in,
                                                             int32_t* __restrict__ out,
                                                             int32_t* __restrict__ copy_to,
                                                             int32_t n, int64_t cap,
                                                             uint32_t* __restrict__ flags,
                                                             bool zero_in,
                                                             const uint32_t* __restrict__ gate) {
  __shared__ int64_t wsum[kScanOneThreads / 64];
  if (gate && gate[0] == 0u) return;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int k0 = t * kScanOnePer;
  int32_t v[kScanOnePer];
  int64_t run = 0;
#pragma unroll
  for (int e = 0; e < kScanOnePer; ++e) {
    v[e] = k0 + e < n ? in[k0 + e] : 0;
    run += v[e];
  }
  int64_t incl = run;
  for (int off = 1; off < 64; off <<= 1) {
    const int64_t u = __shfl_up(incl, off, 64);
    if (lane >= off) incl += u;
  }
  if (lane == 63) wsum[w] = incl;
  __syncthreads();
  int64_t wbase = 0, total = 0;
  for (int k = 0; k < kScanOneThreads / 64; ++k) {
    wbase += k < w ? wsum[k] : 0;
    total += wsum[k];
  }
  const bool overflow = total > cap;
  int64_t o = wbase + incl - run;
#pragma unroll
  for (int e = 0; e < kScanOnePer; ++e) {
    if (k0 + e < n) {
      const int32_t r = overflow ? 0 : static_cast<int32_t>(o);
      out[k0 + e] = r;
      if (copy_to) copy_to[k0 + e] = r;
      if (zero_in) in[k0 + e] = 0;
    }
    o += v[e];
  }
  if (t == 0) {
    out[n] = overflow ? 0 : static_cast<int32_t>(total);
    if (overflow && flags) atomicOr(flags, DMTS_FLAG_NBR_OVERFLOW);
  }
}

// The scan: one launch up to kScanOne elements, else the two tile launches (`part` holds at
// least scan_tiles(n) values).  With `gate`, every launch returns at once unless gate[0] is
// set (the skin list's conditional rebuild).
void scan(int32_t* in, int32_t* out, int32_t* copy_to, int32_t n, int64_t cap, uint32_t* flags,
          bool zero_in, int64_t* part, hipStream_t s, const uint32_t* gate = nullptr) {
  if (n <= kScanOne) {
    k_scan_one<<<1, kScanOneThreads, 0, s>>>(in, out, copy_to, n, cap, flags, zero_in, gate);
    return;
  }
  const int tiles = scan_tiles(n);
  k_scan_sums<<<tiles, kScanThreads, 0, s>>>(in, n, part, gate);
  k_scan_tiles<<<tiles, kScanThreads, 0, s>>>(in, out, copy_to, n, cap, flags, zero_in, part,
                                              tiles, gate);
}

__device__ __forceinline__ int cell_coord(double x, double box, double inv_cell, int nc) {
  double w = x - box * floor(x / box);   // wrap into [0, box)
  if (!(w >= 0.0 && w < box)) w = 0.0;    // non-finite input: any in-range cell
  int c = static_cast<int>(w * inv_cell);
  return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

__global__ void k_cell_assign(const double* __restrict__ pos, int32_t n, double box,
                              double inv_cell, int nc, int32_t* __restrict__ cell_of,
                              int32_t* __restrict__ cell_count,
                              const uint32_t* __restrict__ gate) {
  if (gate && gate[0] == 0u) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int cx = cell_coord(pos[i], box, inv_cell, nc);
  int cy = cell_coord(pos[n + i], box, inv_cell, nc);
  int cz = cell_coord(pos[2 * n + i], box, inv_cell, nc);
  int c = (cz * nc + cy) * nc + cx;
  cell_of[i] = c;
  atomicAdd(&cell_count[c], 1);
}

__global__ void k_cell_scatter(const int32_t* __restrict__ cell_of, int32_t n,
                               int32_t* __restrict__ cursor, int32_t* __restrict__ cell_atoms,
                               const uint32_t* __restrict__ gate) {
  if (gate && gate[0] == 0u) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int slot = atomicAdd(&cursor[cell_of[i]], 1);
  cell_atoms[slot] = i;
}

// All three binning steps in one work-group, for cell grids that fit in LDS: cell ids and
// counts (LDS atomics), the exclusive scan into cell_start, then the scatter through LDS
// cursors.  The order of the atoms inside a cell is arbitrary; rows are sorted afterwards.
constexpr int kBinThreads = 1024;
constexpr int kBinCells = 4096;
constexpr int kBinAtoms = 32768;   // above this, the multi-work-group binning is faster
// With `gate` (the skin list), the work-group first decides whether the rows must be
// rebuilt: when gate[0] is already set, or some atom lies at least sqrt(half2) (half the
// skin) from x_build, its position at the last rebuild (minimum image; a non-finite
// distance counts as moved), it sets gate[0] and bins; otherwise it returns at once and
// the gated launches after it do nothing.
__global__ void __launch_bounds__(kBinThreads)
k_bin_one(const double* __restrict__ pos, int32_t n, double box, double inv_cell, int nc,
          int32_t* __restrict__ cell_of, int32_t* __restrict__ cell_start,
          int32_t* __restrict__ cell_atoms, const double* __restrict__ x_build, double half2,
          uint32_t* __restrict__ gate) {
  __shared__ int32_t cnt[kBinCells];
  __shared__ int32_t part[kBinThreads];
  __shared__ int32_t s_moved;
  const int t = threadIdx.x, n_cells = nc * nc * nc;
  if (gate) {
    if (t == 0) s_moved = 0;
    __syncthreads();
    const double inv_box = 1.0 / box;
    bool moved = false;
    for (int i = t; i < n; i += kBinThreads) {
      const double dx = minimage(pos[i] - x_build[i], box, inv_box);
      const double dy = minimage(pos[n + i] - x_build[n + i], box, inv_box);
      const double dz = minimage(pos[2 * n + i] - x_build[2 * n + i], box, inv_box);
      const double d2 = dx * dx + dy * dy + dz * dz;
      moved = moved || !(d2 < half2);
    }
    if (moved) s_moved = 1;
    __syncthreads();
    if (!s_moved && gate[0] == 0u) return;   // the same decision in every thread
    __syncthreads();                         // every thread has read gate[0]
    if (t == 0) gate[0] = 1u;
  }
  for (int c = t; c < n_cells; c += kBinThreads) cnt[c] = 0;
  __syncthreads();
  for (int i = t; i < n; i += kBinThreads) {
    const int c = (cell_coord(pos[2 * n + i], box, inv_cell, nc) * nc +
                   cell_coord(pos[n + i], box, inv_cell, nc)) * nc +
                  cell_coord(pos[i], box, inv_cell, nc);
    cell_of[i] = c;
    atomicAdd(&cnt[c], 1);
  }
  __syncthreads();
  // exclusive scan: contiguous chunks per thread, Hillis-Steele over the chunk sums
  const int per = (n_cells + kBinThreads - 1) / kBinThreads;
  const int lo = min(n_cells, t * per), hi = min(n_cells, lo + per);
  int sum = 0;
  for (int c = lo; c < hi; ++c) sum += cnt[c];
  part[t] = sum;
  __syncthreads();
  for (int off = 1; off < kBinThreads; off <<= 1) {
    const int add = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += add;
    __syncthreads();
  }
  int run = t == 0 ? 0 : part[t - 1];
  for (int c = lo; c < hi; ++c) {
    const int k = cnt[c];
    cell_start[c] = run;
    cnt[c] = run;   // becomes the cursor
    run += k;
  }
  if (t == 0) cell_start[n_cells] = n;
  __syncthreads();
  for (int i = t; i < n; i += kBinThreads) cell_atoms[atomicAdd(&cnt[cell_of[i]], 1)] = i;
}

// The displacement test of k_bin_one for the multi-work-group binning: any atom at least
// sqrt(half2) from x_build sets gate[0].
__global__ void k_skin_check(const double* __restrict__ pos, int32_t n, double box,
                             const double* __restrict__ x_build, double half2,
                             uint32_t* __restrict__ gate) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool moved = false;
  if (i < n) {
    const double inv_box = 1.0 / box;
    const double dx = minimage(pos[i] - x_build[i], box, inv_box);
    const double dy = minimage(pos[n + i] - x_build[n + i], box, inv_box);
    const double dz = minimage(pos[2 * n + i] - x_build[2 * n + i], box, inv_box);
    moved = !(dx * dx + dy * dy + dz * dz < half2);
  }
  if (__ballot(moved) != 0ull && (threadIdx.x & 63) == 0) atomicOr(gate, 1u);
}

struct Geo {
  const double* pos;
  int32_t n;
  double box, inv_box, rc2;
};

__device__ __forceinline__ bool within(const Geo& g, double xi, double yi, double zi, int j) {
  double dx = minimage(g.pos[j] - xi, g.box, g.inv_box);
  double dy = minimage(g.pos[g.n + j] - yi, g.box, g.inv_box);
  double dz = minimage(g.pos[2 * g.n + j] - zi, g.box, g.inv_box);
  return dx * dx + dy * dy + dz * dz < g.rc2;
}

// Candidate stream of receiver i.  Cell mode: the 27 cells around i's cell, in stencil
// order, each cell's members ascending.  Range mode: atoms lo..hi-1 (its molecule, or all
// atoms).  `visit(t_base, j, valid)` is called wave-uniformly once per 64 candidates
// with each lane's candidate.
struct CellCtx {
  const int32_t* cell_start;
  const int32_t* cell_atoms;
  const int32_t* cell_of;
  int nc;
};

template <bool kCells, class Visit>
__device__ __forceinline__ void walk_candidates(int i, int lo, int hi, const CellCtx& cc,
                                                int32_t* s_pref, int32_t* s_first,
                                                Visit&& visit) {
  const int lane = threadIdx.x & 63;
  if (!kCells) {
    for (int base = lo; base < hi; base += 64) {
      int j = base + lane;
      bool ok = j < hi && j != i;
      visit(ok ? j : -1, ok);
    }
    return;
  }
  // per-lane stencil cell (lanes 0..26)
  const int nc = cc.nc;
  const int ci = cc.cell_of[i];
  const int cx = ci % nc, cy = (ci / nc) % nc, cz = ci / (nc * nc);
  int count = 0, first = 0;
  if (lane < 27) {
    int dx = lane % 3 - 1, dy = (lane / 3) % 3 - 1, dz = lane / 9 - 1;
    int x = (cx + dx + nc) % nc, y = (cy + dy + nc) % nc, z = (cz + dz + nc) % nc;
    int c = (z * nc + y) * nc + x;
    first = cc.cell_start[c];
    count = cc.cell_start[c + 1] - first;
  }
  // inclusive scan of counts over lanes
  int incl = count;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    int v = __shfl_up(incl, off, 64);
    if (lane >= off) incl += v;
  }
  if (lane < 27) {
    s_pref[lane] = incl - count;
    s_first[lane] = first;
  }
  const int total = __shfl(incl, 26, 64);
  wave_sync();
  // candidate t: the last stencil cell k with s_pref[k] <= t (binary search over 27)
  auto cand = [&](int t) {
    if (t >= total) return -1;
    int a = 0, b = 27;
    while (b - a > 1) {
      const int m = (a + b) >> 1;
      if (s_pref[m] <= t) a = m; else b = m;
    }
    return cc.cell_atoms[s_first[a] + (t - s_pref[a])];
  };
  // the next batch's candidates are looked up while this batch is tested
  int jn = cand(lane);
  for (int base = 0; base < total; base += 64) {
    const int j = jn;
    if (base + 64 < total) jn = cand(base + 64 + lane);
    bool ok = j >= 0 && j != i;
    visit(j, ok);
  }
  wave_sync();
}

__device__ __forceinline__ void molecule_range(const int32_t* sys_offsets, int32_t n_sys,
                                               int i, int n, int& lo, int& hi) {
  if (!sys_offsets) {
    lo = 0;
    hi = n;
    return;
  }
  int a = 0, b = n_sys;  // find s with offs[s] <= i < offs[s+1]
  while (b - a > 1) {
    int mid = (a + b) >> 1;
    if (sys_offsets[mid] <= i) a = mid; else b = mid;
  }
  lo = max(0, sys_offsets[a]);
  hi = min(n, sys_offsets[a + 1]);
}

constexpr int kNbWaves = 4;
constexpr int kRowCap = kNlistRowCap;
constexpr int kSkinCap = kSkinRowCap;

// Search of receiver i's row: the accepted senders, in candidate order, into row[] (LDS,
// at most CAP of them).  Returns the full count, which may exceed CAP.  Whole wave.
template <bool kCells, int CAP>
__device__ __forceinline__ int search_row(const Geo& g, const CellCtx& cc,
                                          const int32_t* sys_offsets, int32_t n_sys, int i,
                                          int32_t* s_pref, int32_t* s_first, int32_t* row) {
  const int lane = threadIdx.x & 63;
  const double xi = g.pos[i], yi = g.pos[g.n + i], zi = g.pos[2 * g.n + i];
  int lo = 0, hi = 0;
  if (!kCells) molecule_range(sys_offsets, n_sys, i, g.n, lo, hi);
  int run = 0;
  walk_candidates<kCells>(i, lo, hi, cc, s_pref, s_first, [&](int j, bool ok) {
    bool acc = ok && within(g, xi, yi, zi, j);
    uint64_t mask = __ballot(acc);
    int p = run + __popcll(mask & ((1ull << lane) - 1ull));
    if (acc && p < CAP) row[p] = j;
    run += __popcll(mask);
  });
  wave_sync();
  return run;
}

// Rank sort (senders are distinct: rank = number of smaller entries) of row[0 .. run) into
// out, and into out2 when given.  Whole wave.
__device__ __forceinline__ void sort_row(const int32_t* row, int run, int32_t* out,
                                         int32_t* out2) {
  const int lane = threadIdx.x & 63;
  for (int e = lane; e < run; e += 64) {
    const int v = row[e];
    int rank = 0;
    for (int k = 0; k < run; ++k) rank += row[k] < v;
    out[rank] = v;
    if (out2) out2[rank] = v;
  }
}

// Search + sort of one receiver's row into ell[i][0 .. kRowCap); the row length goes to
// len[i] and, padded to `align`, to cnt[i].  A row longer than kRowCap raises the
// overflow flag and is cut.
template <bool kCells>
__global__ void __launch_bounds__(kNbWaves * 64)
k_rows(Geo g, CellCtx cc, const int32_t* __restrict__ sys_offsets, int32_t n_sys,
       int32_t align, int32_t* __restrict__ ell, int32_t* __restrict__ len,
       int32_t* __restrict__ cnt, uint32_t* __restrict__ flags, double* __restrict__ pos_copy) {
  __shared__ int32_t s_pref[kNbWaves][32], s_first[kNbWaves][32];
  __shared__ int32_t s_row[kNbWaves][kRowCap];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * kNbWaves + w;
  if (i >= g.n) return;
  if (pos_copy && lane < 3) pos_copy[(size_t)lane * g.n + i] = g.pos[(size_t)lane * g.n + i];
  int run = search_row<kCells, kRowCap>(g, cc, sys_offsets, n_sys, i, s_pref[w], s_first[w],
                                        s_row[w]);
  if (run > kRowCap) {
    if (lane == 0) atomicOr(flags, DMTS_FLAG_NBR_OVERFLOW);
    run = kRowCap;
  }
  sort_row(s_row[w], run, ell + (size_t)i * kRowCap, nullptr);
  if (lane == 0) {
    len[i] = run;
    cnt[i] = (run + align - 1) / align * align;
  }
}

// Row i of a list at a shorter cutoff from a parent row src[0 .. r_len) (ascending
// senders, -1 padding) filtered to |d_ij| < r_c at the current positions.  Kept entries
// stay in the parent's order, so the rows are sorted, and they are those of a list built
// at r_c whenever the parent holds every such pair.  Same outputs and overflow rule as
// k_rows.  Called by a whole wave.
__device__ __forceinline__ void filter_row(const Geo& g, int i, const int32_t* src, int r_len,
                                           int32_t align, int32_t* ell, int32_t* len,
                                           int32_t* cnt, uint32_t* flags) {
  const int lane = threadIdx.x & 63;
  const double xi = g.pos[i], yi = g.pos[g.n + i], zi = g.pos[2 * g.n + i];
  int32_t* out = ell + (size_t)i * kRowCap;
  int run = 0;
  for (int base = 0; base < r_len; base += 64) {   // wave-uniform trip count
    const int q = base + lane;
    const int j = q < r_len ? src[q] : -1;
    const bool acc = j >= 0 && within(g, xi, yi, zi, j);
    const uint64_t mask = __ballot(acc);
    const int slot = run + __popcll(mask & ((1ull << lane) - 1ull));
    if (acc && slot < kRowCap) out[slot] = j;
    run += __popcll(mask);
  }
  if (run > kRowCap) {
    if (lane == 0) atomicOr(flags, DMTS_FLAG_NBR_OVERFLOW);
    run = kRowCap;
  }
  if (lane == 0) {
    len[i] = run;
    cnt[i] = (run + align - 1) / align * align;
  }
}

// The filtered rows from a CSR parent list.
__global__ void __launch_bounds__(kNbWaves * 64)
k_sub_rows(Geo g, const int32_t* __restrict__ p_offs, const int32_t* __restrict__ p_nbr,
           int32_t align, int32_t* __restrict__ ell, int32_t* __restrict__ len,
           int32_t* __restrict__ cnt, uint32_t* __restrict__ flags) {
  const int i = blockIdx.x * kNbWaves + (threadIdx.x >> 6);
  if (i >= g.n) return;
  const int r0 = p_offs[i];
  filter_row(g, i, p_nbr + r0, p_offs[i + 1] - r0, align, ell, len, cnt, flags);
}

// One evaluation's rows from the skin list.  When gate[0] is set (the displacement test
// or a forced rebuild asked for it), each wave first rebuilds its receiver's skin row at
// cutoff + skin (g_out: search, sort, x_build) into sk_ell/sk_len, keeping the sorted row
// in LDS; a skin row longer than kSkinCap raises the overflow flag of both lists.  Then the
// row, from LDS or from the kept skin row, is filtered to the cutoff at the current
// positions (g_in) into this list's staging table, and pos_copy receives the positions.
// gate[1] counts the rebuilds.
template <bool kCells>
__global__ void __launch_bounds__(kNbWaves * 64)
k_rows_filter(Geo g_out, CellCtx cc, int32_t* __restrict__ sk_ell, int32_t* __restrict__ sk_len,
              uint32_t* __restrict__ sk_flags, double* __restrict__ x_build,
              uint32_t* __restrict__ gate, Geo g_in, int32_t align, int32_t* __restrict__ ell,
              int32_t* __restrict__ len, int32_t* __restrict__ cnt,
              uint32_t* __restrict__ flags, double* __restrict__ pos_copy) {
  __shared__ int32_t s_pref[kNbWaves][32], s_first[kNbWaves][32];
  __shared__ int32_t s_row[kNbWaves][kSkinCap];
  __shared__ int32_t s_sorted[kNbWaves][kSkinCap];
  const bool rebuild = gate[0] != 0u;
  if (rebuild && blockIdx.x == 0 && threadIdx.x == 0) gate[1] += 1u;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * kNbWaves + w;
  if (i >= g_in.n) return;
  const int32_t* src;
  int r_len;
  if (rebuild) {
    int run = search_row<kCells, kSkinCap>(g_out, cc, nullptr, 1, i, s_pref[w], s_first[w],
                                           s_row[w]);
    if (run > kSkinCap) {
      if (lane == 0) {
        atomicOr(sk_flags, DMTS_FLAG_NBR_OVERFLOW);
        atomicOr(flags, DMTS_FLAG_NBR_OVERFLOW);
      }
      run = kSkinCap;
    }
    sort_row(s_row[w], run, s_sorted[w], sk_ell + (size_t)i * kSkinCap);
    if (lane == 0) sk_len[i] = run;
    if (lane < 3) x_build[(size_t)lane * g_in.n + i] = g_in.pos[(size_t)lane * g_in.n + i];
    wave_sync();
    src = s_sorted[w];
    r_len = run;
  } else {
    src = sk_ell + (size_t)i * kSkinCap;
    r_len = sk_len[i];
  }
  filter_row(g_in, i, src, r_len, align, ell, len, cnt, flags);
  if (pos_copy && lane < 3) pos_copy[(size_t)lane * g_in.n + i] = g_in.pos[(size_t)lane * g_in.n + i];
}

// CSR rows (padded with -1) from the staging table, the reverse index
// rev[p] = offs[j] + (position of i in the sorted row of j), and the pair geometry at the
// build positions: geo[p] = (d_ij as float, |d_ij|), zero for padding.
__global__ void __launch_bounds__(kNbWaves * 64)
k_compact(Geo gm, const int32_t* __restrict__ ell, const int32_t* __restrict__ len,
          const int32_t* __restrict__ offs, int32_t* __restrict__ nbr,
          int32_t* __restrict__ rev, float4* __restrict__ geo, uint32_t* __restrict__ gate,
          uint32_t* __restrict__ sk_flags) {
  // skin list (gate given): the rows are current unless one overflowed, in which case the
  // next evaluation rebuilds them (the overflow was raised on this list already)
  if (gate && blockIdx.x == 0 && threadIdx.x == 0) {
    if (sk_flags[0] & DMTS_FLAG_NBR_OVERFLOW) sk_flags[0] = 0u;
    else gate[0] = 0u;
  }
  const int32_t n = gm.n;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int i = blockIdx.x * kNbWaves + w;
  if (i >= n) return;
  const int row0 = offs[i], row1 = offs[i + 1];
  if (row1 == row0) return;   // empty row, or the list overflowed (all offsets zero)
  const int li = len[i];
  const int32_t* src = ell + (size_t)i * kRowCap;
  for (int k = lane; k < row1 - row0; k += 64) {
    int j = k < li ? src[k] : -1;
    int r = -1;
    if (j >= 0) {
      const int32_t* rj = ell + (size_t)j * kRowCap;
      const int lj = len[j];
      // lower bound of i in rj[0 .. lj): rj[a - 1] < i <= rj[b] (bounds excluded); three
      // independent probes per round narrow the range four-fold
      int a = 0, b = lj;
      while (b - a >= 4) {
        const int q = (b - a) >> 2;
        const int m1 = a + q, m2 = a + 2 * q, m3 = a + 3 * q;
        const int v1 = rj[m1], v2 = rj[m2], v3 = rj[m3];
        if (v3 < i) a = m3 + 1;
        else if (v2 < i) { a = m2 + 1; b = m3; }
        else if (v1 < i) { a = m1 + 1; b = m2; }
        else b = m1;
      }
      while (a < b && rj[a] < i) ++a;
      r = (a < lj && rj[a] == i) ? offs[j] + a : -1;
    }
    float4 gv = make_float4(0.f, 0.f, 0.f, 0.f);
    if (j >= 0) {
      const double xi = gm.pos[i], yi = gm.pos[n + i], zi = gm.pos[2 * n + i];
      const float dx = static_cast<float>(minimage(gm.pos[j] - xi, gm.box, gm.inv_box));
      const float dy = static_cast<float>(minimage(gm.pos[n + j] - yi, gm.box, gm.inv_box));
      const float dz = static_cast<float>(minimage(gm.pos[2 * n + j] - zi, gm.box, gm.inv_box));
      gv = make_float4(dx, dy, dz, sqrtf(dx * dx + dy * dy + dz * dz));
    }
    nbr[row0 + k] = j;
    rev[row0 + k] = r;
    geo[row0 + k] = gv;
  }
}

}  // namespace

dmts_status fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return DMTS_OK;
  k_fill_u32<<<ceil_div(n, 256), 256, 0, s>>>(p, v, n);
  DMTS_CHECK_LAUNCH();
  return DMTS_OK;
}

namespace {

// Cell binning of a build at `cutoff` into nl's cell arrays; cc and cells describe the
// result (cells false: fewer than three cells per edge, rows scan all atoms).  With `gate`
// (the skin list), the displacement test against x_build runs first and every binning
// launch is conditional on its outcome.
dmts_status bin_cells(NList* nl, const double* pos, int32_t n, double box, double cutoff,
                      hipStream_t s, uint32_t* gate, const double* x_build, double half2,
                      CellCtx& cc, bool& cells) {
  cc = CellCtx{nullptr, nullptr, nullptr, 0};
  int nc = box > 0.0 ? static_cast<int>(floor(box / cutoff)) : 0;
  cells = nc >= 3;
  if (!cells) {
    if (gate) {
      k_skin_check<<<ceil_div(n, 256), 256, 0, s>>>(pos, n, box, x_build, half2, gate);
      DMTS_CHECK_LAUNCH();
    }
    return DMTS_OK;
  }
  nc = nc > kMaxCellsPerDim ? kMaxCellsPerDim : nc;
  const int n_cells = nc * nc * nc;
  if (n_cells > nl->n_cells_cap) {
    DMTS_REQUIRE(nl->cell_buf.reserve(sizeof(int32_t) * (3 * (size_t)n_cells + 2), s) == DMTS_OK,
                 DMTS_E_OOM, "build_neighbors: cell buffer allocation failed");
    // counters start at zero; every scan clears them again after reading
    dmts_status st = fill_u32(nl->cell_buf.as<uint32_t>(), 0u, n_cells, s);
    if (st != DMTS_OK) return st;
    nl->n_cells_cap = n_cells;
  }
  int32_t* cell_count = nl->cell_buf.as<int32_t>();
  int32_t* cell_start = cell_count + nl->n_cells_cap;
  int32_t* cursor = cell_start + nl->n_cells_cap + 1;
  const double inv_cell = nc / box;
  if (n_cells <= kBinCells && n <= kBinAtoms) {
    k_bin_one<<<1, kBinThreads, 0, s>>>(pos, n, box, inv_cell, nc, nl->cell_of, cell_start,
                                        nl->cell_atoms, x_build, half2, gate);
    DMTS_CHECK_LAUNCH();
  } else {
    if (gate) {
      k_skin_check<<<ceil_div(n, 256), 256, 0, s>>>(pos, n, box, x_build, half2, gate);
      DMTS_CHECK_LAUNCH();
    }
    k_cell_assign<<<ceil_div(n, 256), 256, 0, s>>>(pos, n, box, inv_cell, nc, nl->cell_of,
                                                   cell_count, gate);
    DMTS_CHECK_LAUNCH();
    scan(cell_count, cell_start, cursor, n_cells, INT64_MAX, nullptr, true, nl->scan_part, s,
         gate);
    DMTS_CHECK_LAUNCH();
    k_cell_scatter<<<ceil_div(n, 256), 256, 0, s>>>(nl->cell_of, n, cursor, nl->cell_atoms,
                                                    gate);
    DMTS_CHECK_LAUNCH();
  }
  cc = CellCtx{cell_start, nl->cell_atoms, nl->cell_of, nc};
  return DMTS_OK;
}

}  // namespace

dmts_status build_neighbors(NList* nl, const double* pos, int32_t n, double box,
                            const int32_t* sys_offsets, int32_t n_sys, double cutoff,
                            hipStream_t s, double* pos_copy) {
  DMTS_REQUIRE(nl && pos, DMTS_E_ARG, "build_neighbors: null argument");
  DMTS_REQUIRE(n >= 0 && n <= nl->max_atoms, DMTS_E_ARG,
               "build_neighbors: n_atoms %d outside [0, %d]", n, nl->max_atoms);
  DMTS_REQUIRE(cutoff > 0.0, DMTS_E_ARG, "build_neighbors: cutoff must be positive");
  DMTS_REQUIRE(box >= 0.0, DMTS_E_ARG, "build_neighbors: negative box");
  DMTS_REQUIRE(box == 0.0 || cutoff < 0.5 * box, DMTS_E_BOX,
               "build_neighbors: cutoff %g must be below half the box edge %g", cutoff, box);
  DMTS_REQUIRE(box == 0.0 || sys_offsets == nullptr, DMTS_E_ARG,
               "build_neighbors: batched molecules need open boundaries");
  DMTS_REQUIRE(sys_offsets == nullptr || n_sys >= 1, DMTS_E_ARG,
               "build_neighbors: n_sys must be >= 1 with sys_offsets");
  nl->n_atoms = n;
  nl->box = box;
  nl->cutoff = cutoff;
  ProfScope ps(DMTS_K_NEIGHBORS, s);
  if (n == 0) {
    return fill_u32(reinterpret_cast<uint32_t*>(nl->offs), 0u, 1, s);
  }
  CellCtx cc;
  bool cells;
  dmts_status r = bin_cells(nl, pos, n, box, cutoff, s, nullptr, nullptr, 0.0, cc, cells);
  if (r != DMTS_OK) return r;
  Geo g{pos, n, box, box > 0.0 ? 1.0 / box : 0.0, cutoff * cutoff};
  const int blocks = ceil_div(n, kNbWaves);
  if (cells)
    k_rows<true><<<blocks, kNbWaves * 64, 0, s>>>(g, cc, sys_offsets, n_sys, nl->row_align,
                                                   nl->ell, nl->len, nl->cnt, nl->flags,
                                                   pos_copy);
  else
    k_rows<false><<<blocks, kNbWaves * 64, 0, s>>>(g, cc, sys_offsets, n_sys, nl->row_align,
                                                    nl->ell, nl->len, nl->cnt, nl->flags,
                                                    pos_copy);
  DMTS_CHECK_LAUNCH();
  scan(nl->cnt, nl->offs, nullptr, n, nl->max_pairs, nl->flags, false, nl->scan_part, s);
  DMTS_CHECK_LAUNCH();
  k_compact<<<blocks, kNbWaves * 64, 0, s>>>(g, nl->ell, nl->len, nl->offs, nl->nbr, nl->rev,
                                             nl->geo, nullptr, nullptr);
  DMTS_CHECK_LAUNCH();
  return DMTS_OK;
}

dmts_status refresh_neighbors(NList* nl, SkinList* sk, const double* pos, int32_t n, double box,
                              double cutoff, hipStream_t s, double* pos_copy) {
  DMTS_REQUIRE(nl && sk && pos, DMTS_E_ARG, "refresh_neighbors: null argument");
  const double outer = cutoff + sk->skin;
  if (!(sk->skin > 0.0) || !(box > 0.0) || !(outer < 0.5 * box) || n < 1 || !sk->rows ||
      !sk->ell || n > sk->rows->max_atoms)
    return build_neighbors(nl, pos, n, box, nullptr, 1, cutoff, s, pos_copy);
  DMTS_REQUIRE(n <= nl->max_atoms, DMTS_E_ARG,
               "refresh_neighbors: n_atoms %d above the list's %d", n, nl->max_atoms);
  nl->n_atoms = n;
  nl->box = box;
  nl->cutoff = cutoff;
  ProfScope ps(DMTS_K_NEIGHBORS, s);
  NList* rows = sk->rows;
  if (sk->cutoff != cutoff || sk->box != box || sk->n != n) {
    // rows built for other parameters (or none yet): rebuild unconditionally
    dmts_status r = fill_u32(sk->gate, 1u, 1, s);
    if (r != DMTS_OK) return r;
    sk->cutoff = cutoff;
    sk->box = box;
    sk->n = n;
    rows->n_atoms = n;
    rows->box = box;
    rows->cutoff = outer;
  }
  // a hair below skin/2, so that rounding in the distance tests cannot lose a pair
  const double half = 0.5 * sk->skin - 1e-9;
  CellCtx cc;
  bool cells;
  dmts_status r = bin_cells(rows, pos, n, box, outer, s, sk->gate, sk->x_build, half * half, cc,
                            cells);
  if (r != DMTS_OK) return r;
  const Geo g_out{pos, n, box, 1.0 / box, outer * outer};
  const Geo g_in{pos, n, box, 1.0 / box, cutoff * cutoff};
  const int blocks = ceil_div(n, kNbWaves);
  if (cells)
    k_rows_filter<true><<<blocks, kNbWaves * 64, 0, s>>>(
        g_out, cc, sk->ell, rows->len, rows->flags, sk->x_build, sk->gate, g_in,
        nl->row_align, nl->ell, nl->len, nl->cnt, nl->flags, pos_copy);
  else
    k_rows_filter<false><<<blocks, kNbWaves * 64, 0, s>>>(
        g_out, cc, sk->ell, rows->len, rows->flags, sk->x_build, sk->gate, g_in,
        nl->row_align, nl->ell, nl->len, nl->cnt, nl->flags, pos_copy);
  DMTS_CHECK_LAUNCH();
  scan(nl->cnt, nl->offs, nullptr, n, nl->max_pairs, nl->flags, false, nl->scan_part, s);
  DMTS_CHECK_LAUNCH();
  k_compact<<<blocks, kNbWaves * 64, 0, s>>>(g_in, nl->ell, nl->len, nl->offs, nl->nbr, nl->rev,
                                             nl->geo, sk->gate, rows->flags);
  DMTS_CHECK_LAUNCH();
  return DMTS_OK;
}

dmts_status filter_neighbors(NList* child, const NList* parent, const double* pos,
                             double cutoff, hipStream_t s) {
  DMTS_REQUIRE(child && parent && pos && child != parent, DMTS_E_ARG,
               "filter_neighbors: null or aliased argument");
  DMTS_REQUIRE(cutoff > 0.0 && cutoff <= parent->cutoff, DMTS_E_ARG,
               "filter_neighbors: cutoff %g outside (0, %g] (the parent's)", cutoff,
               parent->cutoff);
  const int32_t n = parent->n_atoms;
  DMTS_REQUIRE(n <= child->max_atoms, DMTS_E_ARG,
               "filter_neighbors: the parent holds %d atoms, the child room for %d", n,
               child->max_atoms);
  child->n_atoms = n;
  child->box = parent->box;
  child->cutoff = cutoff;
  ProfScope ps(DMTS_K_NEIGHBORS, s);
  if (n == 0) return fill_u32(reinterpret_cast<uint32_t*>(child->offs), 0u, 1, s);
  const double box = parent->box;
  Geo g{pos, n, box, box > 0.0 ? 1.0 / box : 0.0, cutoff * cutoff};
  const int blocks = ceil_div(n, kNbWaves);
  k_sub_rows<<<blocks, kNbWaves * 64, 0, s>>>(g, parent->offs, parent->nbr, child->row_align,
                                              child->ell, child->len, child->cnt, child->flags);
  DMTS_CHECK_LAUNCH();
  scan(child->cnt, child->offs, nullptr, n, child->max_pairs, child->flags, false,
       child->scan_part, s);
  DMTS_CHECK_LAUNCH();
  k_compact<<<blocks, kNbWaves * 64, 0, s>>>(g, child->ell, child->len, child->offs, child->nbr,
                                             child->rev, child->geo, nullptr, nullptr);
  DMTS_CHECK_LAUNCH();
  return DMTS_OK;
}

}  // namespace dmts

// ------------------------------------------------------------------ C ABI
using dmts::NList;

extern "C" dmts_status nnp_nlist_create(int32_t max_atoms, int64_t max_pairs,
                                        int32_t row_align, nnp_nlist** out) {
  DMTS_REQUIRE(out, DMTS_E_ARG, "nnp_nlist_create: out is NULL");
  *out = nullptr;
  DMTS_REQUIRE(max_atoms >= 1 && max_pairs >= 1 && max_pairs < (int64_t(1) << 31),
               DMTS_E_ARG, "nnp_nlist_create: bad capacity (%d atoms, %lld pairs)",
               max_atoms, (long long)max_pairs);
  DMTS_REQUIRE(row_align == 4 || row_align == 16 || row_align == 32 || row_align == 64,
               DMTS_E_ARG, "nnp_nlist_create: row_align must be 4, 16, 32 or 64");
  NList* nl = new NList();
  nl->max_atoms = max_atoms;
  nl->max_pairs = (max_pairs + 3) / 4 * 4;
  nl->row_align = row_align;
  size_t a = (size_t)max_atoms;
  hipError_t e = hipSuccess;
  e = e == hipSuccess ? hipMalloc(&nl->offs, sizeof(int32_t) * (a + 1)) : e;
  e = e == hipSuccess ? hipMalloc(&nl->cnt, sizeof(int32_t) * a) : e;
  e = e == hipSuccess ? hipMalloc(&nl->cell_of, sizeof(int32_t) * a) : e;
  e = e == hipSuccess ? hipMalloc(&nl->cell_atoms, sizeof(int32_t) * a) : e;
  e = e == hipSuccess ? hipMalloc(&nl->len, sizeof(int32_t) * a) : e;
  e = e == hipSuccess ? hipMalloc(&nl->ell, sizeof(int32_t) * a * dmts::kNlistRowCap) : e;
  e = e == hipSuccess ? hipMalloc(&nl->nbr, sizeof(int32_t) * nl->max_pairs) : e;
  e = e == hipSuccess ? hipMalloc(&nl->rev, sizeof(int32_t) * nl->max_pairs) : e;
  e = e == hipSuccess ? hipMalloc(&nl->geo, sizeof(float4) * nl->max_pairs) : e;
  e = e == hipSuccess ? hipMalloc(&nl->flags, sizeof(uint32_t)) : e;
  const int tiles = std::max(dmts::scan_tiles(max_atoms),
                             dmts::scan_tiles(int64_t(dmts::kMaxCellsPerDim) *
                                              dmts::kMaxCellsPerDim * dmts::kMaxCellsPerDim));
  e = e == hipSuccess ? hipMalloc(&nl->scan_part, sizeof(int64_t) * tiles) : e;
  e = e == hipSuccess ? hipMemset(nl->flags, 0, sizeof(uint32_t)) : e;
  e = e == hipSuccess ? hipMemset(nl->offs, 0, sizeof(int32_t) * (a + 1)) : e;
  e = e == hipSuccess ? hipDeviceSynchronize() : e;
  if (e != hipSuccess) {
    dmts::set_error("nnp_nlist_create: %s", hipGetErrorString(e));
    nnp_nlist_destroy(reinterpret_cast<nnp_nlist*>(nl));
    return DMTS_E_OOM;
  }
  *out = reinterpret_cast<nnp_nlist*>(nl);
  return DMTS_OK;
}

extern "C" void nnp_nlist_destroy(nnp_nlist* h) {
  NList* nl = reinterpret_cast<NList*>(h);
  if (!nl) return;
  (void)hipDeviceSynchronize();
  (void)hipFree(nl->offs);
  (void)hipFree(nl->cnt);
  (void)hipFree(nl->cell_of);
  (void)hipFree(nl->cell_atoms);
  (void)hipFree(nl->len);
  (void)hipFree(nl->ell);
  (void)hipFree(nl->nbr);
  (void)hipFree(nl->rev);
  (void)hipFree(nl->geo);
  (void)hipFree(nl->flags);
  (void)hipFree(nl->scan_part);
  nl->cell_buf.release();
  delete nl;
}

extern "C" dmts_status nnp_filter_neighbors(nnp_nlist* child, const nnp_nlist* parent,
                                            const double* pos, double cutoff, void* stream) {
  return dmts::filter_neighbors(reinterpret_cast<NList*>(child),
                                reinterpret_cast<const NList*>(parent), pos, cutoff,
                                static_cast<hipStream_t>(stream));
}

extern "C" dmts_status nnp_build_neighbors(nnp_nlist* h, const double* pos, int32_t n_atoms,
                                           double box, const int32_t* sys_offsets,
                                           int32_t n_sys, double cutoff, void* stream) {
  return dmts::build_neighbors(reinterpret_cast<NList*>(h), pos, n_atoms, box, sys_offsets,
                               n_sys, cutoff, static_cast<hipStream_t>(stream));
}

extern "C" dmts_status nnp_nlist_flags(nnp_nlist* h, void* stream, uint32_t* host_flags) {
  NList* nl = reinterpret_cast<NList*>(h);
  DMTS_REQUIRE(nl && host_flags, DMTS_E_ARG, "nnp_nlist_flags: null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  DMTS_HIP(hipMemcpyAsync(host_flags, nl->flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  DMTS_HIP(hipStreamSynchronize(s));
  dmts_status st = dmts::fill_u32(nl->flags, 0u, 1, s);
  if (st != DMTS_OK) return st;
  DMTS_HIP(hipStreamSynchronize(s));
  return DMTS_OK;
}

extern "C" dmts_status nnp_nlist_download(nnp_nlist* h, void* stream, int32_t* host_offs,
                                          int32_t* host_nbr, int32_t* host_rev,
                                          int64_t host_cap, int64_t* n_entries) {
  NList* nl = reinterpret_cast<NList*>(h);
  DMTS_REQUIRE(nl && host_offs && n_entries, DMTS_E_ARG, "nnp_nlist_download: null argument");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = nl->n_atoms;
  DMTS_HIP(hipMemcpyAsync(host_offs, nl->offs, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, s));
  DMTS_HIP(hipStreamSynchronize(s));
  const int64_t P = host_offs[n];
  *n_entries = P;
  DMTS_REQUIRE(P <= host_cap, DMTS_E_CAPACITY, "nnp_nlist_download: %lld entries, host capacity %lld",
               (long long)P, (long long)host_cap);
  if (P > 0 && host_nbr)
    DMTS_HIP(hipMemcpyAsync(host_nbr, nl->nbr, sizeof(int32_t) * P, hipMemcpyDeviceToHost, s));
  if (P > 0 && host_rev)
    DMTS_HIP(hipMemcpyAsync(host_rev, nl->rev, sizeof(int32_t) * P, hipMemcpyDeviceToHost, s));
  DMTS_HIP(hipStreamSynchronize(s));
  return DMTS_OK;
}
