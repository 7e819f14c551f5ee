// Neighbour lists: displacement check, Hilbert cell sort, 8-atom clusters and
// per-cluster j-lists (appendix B cutoffs).
//
// A cluster lists every atom j that lies within r_list + 0.01 A (FP32
// minimum image) of at least one of its atoms i, with one bit per i; the
// margin is far above the FP32 error of d^2, so the listed pairs are a
// superset of the pairs within r_list.  The canonical list -- pairs with
// FP64 d^2 < r_list^2, d = x_j - x_i, d -= L * rint(d / L) as separate
// multiply and subtract, d^2 = (dx^2 + dy^2) + dz^2 -- is what the export
// applies to that superset; this unit is built with -ffp-contract=off so
// that sequence is exact as written.
#include "felis_internal.h"

namespace felis {
namespace {

constexpr int kCellOf = 4096;                 // candidates per table window in k_build
constexpr int kBuildWaves = 2;                // waves per list-build workgroup
constexpr int kBuildThreads = 64 * kBuildWaves;

// a wave-uniform float moved to a scalar register
__device__ __forceinline__ float scalar(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

__device__ __forceinline__ int cell_of(float v, float L, float invL, int n) {
  float u = wrapf(v, L, invL) * invL;
  int c = (int)(u * (float)n);
  return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

// Largest squared displacement since the last build that keeps a window's
// lists and cells valid: (skin/2)^2, less what volume moves have used (a
// move by s changes a pair distance r by at most |s - 1| (r + 2 r_mol) and
// an atom's place in the scaled cell grid by |s - 1| (r_mol + drift)).
__device__ __forceinline__ float skin_threshold2(const LegDev& g, int w) {
  const float used = g.skin_used[w];
  if (used == 0.f) return g.skin_half2;
  if (!(used < g.skin)) return -1.f;             // nothing left: rebuild
  const float t = 0.5f * (g.skin - used);
  return t * t;
}

// One block per window: rebuild flag = force || max displacement > skin/2;
// a window being rebuilt gets its per-cell counters zeroed.  FROM_WORD: the
// largest squared displacement was recorded by the previous step's
// integrator (same arithmetic as the scan below); either way the word is
// cleared for the next step.
template <bool FROM_WORD>
__global__ __launch_bounds__(256) void k_check(const LegDev* legs, BlockMap map, int force) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const int w = blockIdx.x - map.start[leg];
  __shared__ float red[256];
  __shared__ int s_flag;
  float m = 0.f;
  force |= g.rbforce[w];                         // a box change (barostat) since the last build
  if (FROM_WORD) {
    if (g.units < 64) {
      if (threadIdx.x == 0) m = __uint_as_float(g.maxdisp[w]);
    } else {
      // integrator waves covering this window's units
      const long long u0 = (long long)w * g.units, u1 = u0 + g.units;
      for (long long q = (u0 >> 6) + threadIdx.x; q <= ((u1 - 1) >> 6); q += blockDim.x) {
        const bool first = (q * 64) / g.units == w;         // this window is the wave's first
        m = fmaxf(m, __uint_as_float(g.wmax[2 * q + (first ? 0 : 1)]));
      }
    }
  } else if (!force) {
    const size_t o = (size_t)w * g.n;
    for (int a = threadIdx.x; a < g.n; a += blockDim.x) {
      const float dx = g.x[o + a] - g.xr[o + a], dy = g.y[o + a] - g.yr[o + a], dz = g.z[o + a] - g.zr[o + a];
      m = fmaxf(m, dx * dx + dy * dy + dz * dz);
    }
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int f = (force || !(red[0] <= skin_threshold2(g, w))) ? 1 : 0;
    g.flag[w] = f;
    g.nbuild[w] += f;
    g.maxdisp[w] = 0u;
    g.rbforce[w] = 0;
    if (f) g.skin_used[w] = 0.f;
    s_flag = f;
  }
  __syncthreads();
  if (s_flag)
    for (int c = threadIdx.x; c < g.ncell; c += blockDim.x) g.cursor[(size_t)w * g.ncell + c] = 0;
}

// items: window x atom -- Hilbert cell code, per-cell counts, reference positions
__global__ __launch_bounds__(256) void k_cells_count(const LegDev* legs, BlockMap map) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const long long i = (long long)(blockIdx.x - map.start[leg]) * blockDim.x + threadIdx.x;
  if (i >= (long long)g.W * g.n) return;
  const int w = (int)(i / g.n);
  if (!g.flag[w]) return;
  const int nf = 1 << g.nbits;
  const BoxW& B = g.box[w];
  const float x = g.x[i], y = g.y[i], z = g.z[i];
  const unsigned c = g.hcell[(cell_of(x, B.Lf[0], B.invLf[0], nf) * nf + cell_of(y, B.Lf[1], B.invLf[1], nf)) * nf +
                            cell_of(z, B.Lf[2], B.invLf[2], nf)];
  g.cellcode[i] = (int)c;
  atomicAdd(&g.cursor[(size_t)w * g.ncell + c], 1);
  g.xr[i] = x; g.yr[i] = y; g.zr[i] = z;
}

// one block per window: exclusive scan of the counts into cellstart; reset
// cursor.  The cells go through LDS 4,096 at a time, read and written with
// consecutive lanes on consecutive cells; each thread scans four neighbouring
// counts, the block scans the threads' sums (wave shuffles, then the 16 wave
// totals), and a running total carries across the pieces.
__global__ __launch_bounds__(1024) void k_cells_scan(const LegDev* legs, BlockMap map) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const int w = blockIdx.x - map.start[leg];
  if (!g.flag[w]) return;
  int* cnt = g.cursor + (size_t)w * g.ncell;
  int* st = g.cellstart + (size_t)w * (g.ncell + 1);
  constexpr int T = 1024, E = 4, TILE = T * E, NW = T / 64;
  __shared__ int s_v[TILE];
  __shared__ int s_wt[NW];
  __shared__ int s_tile;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nc = g.ncell;
  int carry = 0;                                  // counts before this piece (same in every thread)
  for (int t0 = 0; t0 < nc; t0 += TILE) {
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int c = t0 + k * T + tid;
      s_v[k * T + tid] = c < nc ? cnt[c] : 0;
    }
    __syncthreads();
    int v[E], sum = 0;
#pragma unroll
    for (int k = 0; k < E; ++k) { v[k] = s_v[tid * E + k]; sum += v[k]; }
    int inc = sum;                                // inclusive scan over the wave
    for (int o = 1; o < 64; o <<= 1) {
      const int u = __shfl_up(inc, o, 64);
      if (lane >= o) inc += u;
    }
    if (lane == 63) s_wt[wave] = inc;
    __syncthreads();
    if (wave == 0) {                              // exclusive scan of the wave totals; the piece's total
      const int t = lane < NW ? s_wt[lane] : 0;
      int ti = t;
      for (int o = 1; o < NW; o <<= 1) {
        const int u = __shfl_up(ti, o, 64);
        if (lane >= o) ti += u;
      }
      if (lane < NW) s_wt[lane] = ti - t;
      if (lane == NW - 1) s_tile = ti;
    }
    __syncthreads();
    int run = carry + s_wt[wave] + inc - sum;
#pragma unroll
    for (int k = 0; k < E; ++k) { s_v[tid * E + k] = run; run += v[k]; }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int c = t0 + k * T + tid;
      if (c < nc) { st[c] = s_v[k * T + tid]; cnt[c] = 0; }
    }
    carry += s_tile;
    __syncthreads();                              // s_v, s_wt and s_tile are rewritten next
  }
  if (tid == 0) st[nc] = carry;
}

// items: window x atom -- place each atom in its cell's range
__global__ __launch_bounds__(256) void k_cells_scatter(const LegDev* legs, BlockMap map) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const long long i = (long long)(blockIdx.x - map.start[leg]) * blockDim.x + threadIdx.x;
  if (i >= (long long)g.W * g.n) return;
  const int w = (int)(i / g.n);
  if (!g.flag[w]) return;
  const int a = (int)(i - (long long)w * g.n);
  const int c = g.cellcode[i];
  const int slot = g.cellstart[(size_t)w * (g.ncell + 1) + c] + atomicAdd(&g.cursor[(size_t)w * g.ncell + c], 1);
  g.perm[(size_t)w * g.npad + slot] = a;
}

// items: window x cell -- order atoms within a cell by index (makes the sort
// deterministic), then write the padding slots
__global__ __launch_bounds__(256) void k_cells_order(const LegDev* legs, BlockMap map) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const long long i = (long long)(blockIdx.x - map.start[leg]) * blockDim.x + threadIdx.x;
  if (i >= (long long)g.W * g.ncell) return;
  const int w = (int)(i / g.ncell);
  if (!g.flag[w]) return;
  const int c = (int)(i - (long long)w * g.ncell);
  const int* st = g.cellstart + (size_t)w * (g.ncell + 1);
  int* p = g.perm + (size_t)w * g.npad;
  const int s0 = st[c], s1 = st[c + 1];
  for (int s = s0 + 1; s < s1; ++s) {
    int v = p[s], t = s - 1;
    while (t >= s0 && p[t] > v) { p[t + 1] = p[t]; --t; }
    p[t + 1] = v;
  }
  if (c == 0)
    for (int s = g.n; s < g.npad; ++s) p[s] = -1;
}

// Legs whose cell grid and atom count fit in LDS run the check and the whole
// cell sort in one block per window: Hilbert codes and per-cell counts in
// LDS, an exclusive scan into cellstart, placement by LDS atomics, then each
// cell's atoms in index order (the same deterministic order as the grid-wide
// kernels above).
constexpr int kSortCells = 4096;
constexpr int kSortAtoms = 12288;

template <bool FROM_WORD>
__global__ __launch_bounds__(1024) void k_check_sort(const LegDev* legs, BlockMap map, int force) {
  static_assert(kSortAtoms % 1024 == 0, "one block of 1024 threads sorts a window");
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const int w = blockIdx.x - map.start[leg];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  __shared__ int s_cur[kSortCells];               // counts, then next free slot per cell
  __shared__ int s_st[kSortCells + 1];
  __shared__ unsigned short s_code[kSortAtoms];
  __shared__ int s_perm[kSortAtoms];
  __shared__ float s_red[16];
  __shared__ int s_wsum[16];
  __shared__ int s_flag;
  const size_t o = (size_t)w * g.n;
  float m = 0.f;
  force |= g.rbforce[w];                         // a box change (barostat) since the last build
  if (FROM_WORD) {
    if (g.units < 64) {
      if (tid == 0) m = __uint_as_float(g.maxdisp[w]);
    } else {
      const long long u0 = (long long)w * g.units, u1 = u0 + g.units;
      for (long long q = (u0 >> 6) + tid; q <= ((u1 - 1) >> 6); q += blockDim.x) {
        const bool first = (q * 64) / g.units == w;
        m = fmaxf(m, __uint_as_float(g.wmax[2 * q + (first ? 0 : 1)]));
      }
    }
  } else if (!force) {
    for (int a = tid; a < g.n; a += blockDim.x) {
      const float dx = g.x[o + a] - g.xr[o + a], dy = g.y[o + a] - g.yr[o + a], dz = g.z[o + a] - g.zr[o + a];
      m = fmaxf(m, dx * dx + dy * dy + dz * dz);
    }
  }
  for (int k = 32; k > 0; k >>= 1) m = fmaxf(m, __shfl_xor(m, k, 64));
  if (lane == 0) s_red[wave] = m;
  __syncthreads();
  if (tid == 0) {
    float r = s_red[0];
    for (int k = 1; k < (int)(blockDim.x >> 6); ++k) r = fmaxf(r, s_red[k]);
    const int f = (force || !(r <= skin_threshold2(g, w))) ? 1 : 0;
    g.flag[w] = f;
    g.nbuild[w] += f;
    g.maxdisp[w] = 0u;
    g.rbforce[w] = 0;
    if (f) g.skin_used[w] = 0.f;
    s_flag = f;
  }
  __syncthreads();
  if (!s_flag) return;                            // uniform over the block

  const int nc = g.ncell, n = g.n, nf = 1 << g.nbits;
  const float bL[3] = {g.box[w].Lf[0], g.box[w].Lf[1], g.box[w].Lf[2]};
  const float biL[3] = {g.box[w].invLf[0], g.box[w].invLf[1], g.box[w].invLf[2]};
  for (int c = tid; c < nc; c += blockDim.x) s_cur[c] = 0;
  // every position this thread sorts is loaded before any is used (at most
  // kSortAtoms / 1024 per thread), so the loads overlap
  constexpr int kPer = kSortAtoms / 1024;
  float px[kPer], py[kPer], pz[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int a = tid + k * 1024;
    if (a < n) { px[k] = g.x[o + a]; py[k] = g.y[o + a]; pz[k] = g.z[o + a]; }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int a = tid + k * 1024;
    if (a < n) {
      const unsigned c = g.hcell[(cell_of(px[k], bL[0], biL[0], nf) * nf + cell_of(py[k], bL[1], biL[1], nf)) *
                                     nf + cell_of(pz[k], bL[2], biL[2], nf)];
      s_code[a] = (unsigned short)c;
      atomicAdd(&s_cur[c], 1);
      g.xr[o + a] = px[k]; g.yr[o + a] = py[k]; g.zr[o + a] = pz[k];
    }
  }
  __syncthreads();
  // exclusive scan: each thread takes a run of consecutive cells
  const int per = (nc + (int)blockDim.x - 1) / (int)blockDim.x;
  const int c0 = min(nc, tid * per), c1 = min(nc, c0 + per);
  int sum = 0;
  for (int c = c0; c < c1; ++c) sum += s_cur[c];
  int inc = sum;
  for (int k = 1; k < 64; k <<= 1) {
    const int v = __shfl_up(inc, k, 64);
    if (lane >= k) inc += v;
  }
  if (lane == 63) s_wsum[wave] = inc;
  __syncthreads();
  int run = inc - sum;
  for (int k = 0; k < wave; ++k) run += s_wsum[k];
  int* cst = g.cellstart + (size_t)w * (nc + 1);
  for (int c = c0; c < c1; ++c) {
    const int cnt = s_cur[c];
    s_st[c] = run;
    cst[c] = run;
    s_cur[c] = run;
    run += cnt;
  }
  if (tid == 0) { s_st[nc] = n; cst[nc] = n; }
  __syncthreads();
  for (int a = tid; a < n; a += blockDim.x) s_perm[atomicAdd(&s_cur[s_code[a]], 1)] = a;
  __syncthreads();
  for (int c = tid; c < nc; c += blockDim.x) {    // index order within each cell
    const int b0 = s_st[c], b1 = s_st[c + 1];
    for (int q = b0 + 1; q < b1; ++q) {
      const int v = s_perm[q];
      int t = q - 1;
      while (t >= b0 && s_perm[t] > v) { s_perm[t + 1] = s_perm[t]; --t; }
      s_perm[t + 1] = v;
    }
  }
  __syncthreads();
  int* p = g.perm + (size_t)w * g.npad;
  for (int q = tid; q < g.npad; q += blockDim.x) p[q] = q < n ? s_perm[q] : -1;
}

bool sort_in_lds(const LegHost& h) { return h.ncell <= kSortCells && h.n <= kSortAtoms; }

// One workgroup per cluster: sweep the coarse blocks (aligned 2x2x2 fine
// cells) within r_list of the cluster's box, kBuildThreads blocks per round,
// each trimmed to the Hilbert span of its fine cells within r_list, and list
// every atom j with at least one i of the cluster in range.  The waves take
// consecutive 64-candidate parts of each step and append in wave order, so
// the list order is fixed (cells in sweep order, slots ascending).  Two waves
// per workgroup: every wave repeats the cluster's set-up (~700 instructions),
// so four waves spent 15 % more and one wave pays the per-round scan and
// table work twice as often.
__global__ __launch_bounds__(kBuildThreads) void k_build(const LegDev* legs, BlockMap map) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const long long item = (long long)blockIdx.x - map.start[leg];
  const int w = (int)(item / g.nclus);
  if (!g.flag[w]) return;                       // uniform over the block
  const int c = (int)(item - (long long)w * g.nclus);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;

  __shared__ int s_ai[kClus];
  __shared__ float s_xi[kClus][3];
  __shared__ int s_ex[kClus][kMaxExcl];
  __shared__ int s_nex[kClus];
  __shared__ unsigned s_bloom[64];              // 2048-bit filter of excluded atoms
  __shared__ int s_start[kBuildThreads];        // first sorted slot of each block in the round
  __shared__ int s_pre[kBuildThreads];          // exclusive prefix of candidate counts
  __shared__ int s_wsum[kBuildWaves];
  __shared__ int s_wc[2][2][kBuildWaves];
  __shared__ unsigned char s_cellof[kCellOf];   // candidate -> block of the round, one window at a time
  const size_t o = (size_t)w * g.n;
  const int* perm = g.perm + (size_t)w * g.npad;
  if (tid < 64) s_bloom[tid] = 0u;
  __syncthreads();
  if (tid < kClus) {
    const int a = perm[c * kClus + tid];
    s_ai[tid] = a;
    int ne = 0;
    // a padding slot gets defined (zero) coordinates: nothing downstream may
    // depend on what an earlier workgroup left in LDS
    s_xi[tid][0] = 0.f;
    s_xi[tid][1] = 0.f;
    s_xi[tid][2] = 0.f;
    if (a >= 0) {
      s_xi[tid][0] = g.x[o + a];
      s_xi[tid][1] = g.y[o + a];
      s_xi[tid][2] = g.z[o + a];
      const int e0 = g.excl_ptr[a], e1 = g.excl_ptr[a + 1];
      ne = e1 - e0;
      if (ne > kMaxExcl) { latch(g.err, kErrExcl, kSiteExclCount, (w << 20) | a, g.leg_index); ne = kMaxExcl; }
      for (int k = 0; k < ne; ++k) {
        const int e = g.excl_idx[e0 + k];
        s_ex[tid][k] = e;
        atomicOr(&s_bloom[(e >> 5) & 63], 1u << (e & 31));
      }
    }
    s_nex[tid] = ne;
  }
  __syncthreads();

  // box edges in scalar registers: read once, not again after every list store
  const BoxW& B = g.box[w];
  const float Lf[3] = {scalar(B.Lf[0]), scalar(B.Lf[1]), scalar(B.Lf[2])};
  const float iLf[3] = {scalar(B.invLf[0]), scalar(B.invLf[1]), scalar(B.invLf[2])};
  const int cap = __builtin_amdgcn_readfirstlane(g.cap);
  const float4 lo4 = g.bblo[item], hi4 = g.bbhi[item];
  const float lo[3] = {lo4.x, lo4.y, lo4.z}, hi[3] = {hi4.x, hi4.y, hi4.z};
  const int nf = g.ncoarse;
  const float pre = (float)g.rlist + 0.05f;
  const float pre2 = pre * pre;
  int r0[3], nC[3];
  bool full[3];
  float cen[3], half[3], csd[3];
  for (int d = 0; d < 3; ++d) {
    cen[d] = 0.5f * (lo[d] + hi[d]);
    half[d] = 0.5f * (hi[d] - lo[d]);
    if (!(half[d] >= 0.f && half[d] <= Lf[d])) { cen[d] = 0.f; half[d] = Lf[d]; }   // no valid atom
    // nf is a power of two: exact cell edge; the range ends use its inverse
    // (a rounding flip only adds or drops a cell whose nearest face lies
    // pre - r_list - 0.01 = 0.04 A beyond the list radius)
    const float cs = ldexpf(Lf[d], 1 - g.nbits);
    const float ics = ldexpf(iLf[d], g.nbits - 1);
    csd[d] = cs;
    const int a0 = (int)floorf((cen[d] - half[d] - pre) * ics);
    const int a1 = (int)floorf((cen[d] + half[d] + pre) * ics);
    full[d] = a1 - a0 + 1 >= nf;               // the range wraps onto itself: every cell, no gap test
    r0[d] = full[d] ? 0 : a0;
    nC[d] = full[d] ? nf : a1 - a0 + 1;
  }
  const float4* __restrict__ xq = g.xyzq + (size_t)w * g.npad;
  const float incl = (float)g.rlist + 0.01f;
  const float inc2 = incl * incl;
  float xi[kClus][3], ri[kClus][3];
  int ai[kClus];
  float ext[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int ii = 0; ii < kClus; ++ii) {
    ai[ii] = __builtin_amdgcn_readfirstlane(s_ai[ii]);           // uniform: scalar registers
    for (int d = 0; d < 3; ++d) {
      xi[ii][d] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(s_xi[ii][d])));
      // position relative to the cluster's first atom (always a real atom), nearest image
      const float v = xi[ii][d] - xi[0][d];
      ri[ii][d] = __fmaf_rn(-Lf[d], rintf(v * iLf[d]), v);
      if (ai[ii] >= 0) ext[d] = fmaxf(ext[d], fabsf(ri[ii][d]));
    }
  }
  // one periodic image per candidate (taken against the first atom) is the
  // nearest image for every i whenever extent + r_list + margin < L/2
  const bool shift = ext[0] + incl + 0.02f < 0.5f * Lf[0] && ext[1] + incl + 0.02f < 0.5f * Lf[1] &&
                     ext[2] + incl + 0.02f < 0.5f * Lf[2];
  // i-side terms of |r_j - r_i|^2 = |r_j|^2 - 2 r_i.r_j + |r_i|^2 in the
  // shifted frame (|r| < 25 A there, so the FP32 error of the expanded form
  // stays below 1e-3 A^2, far inside the 0.01 A margin), held in scalar
  // registers; a padding slot gets |r_i|^2 = 1e30 and never passes
  float m2[kClus][3], nc2[kClus];
#pragma unroll
  for (int ii = 0; ii < kClus; ++ii) {
    for (int d = 0; d < 3; ++d) m2[ii][d] = scalar(ai[ii] >= 0 ? -2.0f * ri[ii][d] : 0.0f);
    nc2[ii] = scalar(ai[ii] >= 0 ? -__fmaf_rn(ri[ii][0], ri[ii][0], __fmaf_rn(ri[ii][1], ri[ii][1], ri[ii][2] * ri[ii][2]))
                                 : -1.0e30f);
  }
  const int* cst = g.cellstart + (size_t)w * (g.ncell + 1);
  unsigned* outL = g.lent + (size_t)item * 2 * cap;      // partners of atoms 0-3
  unsigned* outH = outL + cap;                            // partners of atoms 4-7
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int ncells = nC[0] * nC[1] * nC[2];
  int countL = 0, countH = 0, par = 0;
  // block index ci -> (c0, c1, c2) by float-reciprocal quotients with one
  // correction (exact for ci < 2^22, with the hardware reciprocal too); a
  // block coordinate lies in (-nf, 2nf)
  // (the range is narrower than the box unless full), so one wrap suffices
  const int n12 = nC[1] * nC[2];
  const float inv12 = __builtin_amdgcn_rcpf((float)n12), inv2 = __builtin_amdgcn_rcpf((float)nC[2]);
  auto wrapc = [nf](int c) { return c < 0 ? c + nf : (c >= nf ? c - nf : c); };
  for (int cb = 0; cb < ncells; cb += kBuildThreads) {
    const int ci = cb + tid;
    int s0 = 0, cnt = 0;
    if (ci < ncells) {
      int c0 = (int)((float)ci * inv12);
      c0 += (ci - c0 * n12 < 0) ? -1 : (ci - c0 * n12 >= n12 ? 1 : 0);
      const int rem = ci - c0 * n12;
      int c1 = (int)((float)rem * inv2);
      c1 += (rem - c1 * nC[2] < 0) ? -1 : (rem - c1 * nC[2] >= nC[2] ? 1 : 0);
      const int C[3] = {r0[0] + c0, r0[1] + c1, r0[2] + rem - c1 * nC[2]};
      float gap2 = 0.f;
      for (int d = 0; d < 3; ++d) {
        if (full[d]) continue;
        const float cs = csd[d];
        const float gp = fmaxf(0.f, fmaxf((float)C[d] * cs - hi[d], lo[d] - (float)(C[d] + 1) * cs));
        gap2 += gp * gp;
      }
      if (gap2 < pre2) {
        // the block's 8 fine cells hold 8 consecutive Hilbert indices: take
        // the span from the first to the last child that passes its own gap test
        float g2c[3][2];
        for (int d = 0; d < 3; ++d)
          for (int hh = 0; hh < 2; ++hh) {
            const float cf = 0.5f * csd[d];
            const int F = 2 * C[d] + hh;
            const float gp = fmaxf(0.f, fmaxf((float)F * cf - hi[d], lo[d] - (float)(F + 1) * cf));
            g2c[d][hh] = full[d] ? 0.f : gp * gp;
          }
        const int nff = 2 * nf, W0 = 2 * wrapc(C[0]), W1 = 2 * wrapc(C[1]), W2 = 2 * wrapc(C[2]);
        unsigned hc[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
          hc[k] = g.hcell[((W0 + (k >> 2)) * nff + W1 + ((k >> 1) & 1)) * nff + W2 + (k & 1)];
        unsigned kmin = 0xffffffffu, kmax = 0u;
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (g2c[0][k >> 2] + g2c[1][(k >> 1) & 1] + g2c[2][k & 1] < pre2) {
            kmin = min(kmin, hc[k]);
            kmax = max(kmax, hc[k]);
          }
        if (kmin <= kmax) {
          s0 = cst[kmin];
          cnt = cst[kmax + 1] - s0;
        }
      }
    }
    int inc = cnt;
    for (int k = 1; k < 64; k <<= 1) {
      const int v = __shfl_up(inc, k, 64);
      if (lane >= k) inc += v;
    }
    if (lane == 63) s_wsum[wave] = inc;
    s_start[tid] = s0;
    __syncthreads();
    int woff = 0;
    for (int k = 0; k < wave; ++k) woff += s_wsum[k];
    int total = 0;
    for (int k = 0; k < kBuildWaves; ++k) total += s_wsum[k];
    const int pre_t = woff + inc - cnt;
    s_pre[tid] = pre_t;
    // candidates are taken kCellOf at a time: each block writes its index over
    // its share of the window, then a candidate finds its block in one read
    for (int T0 = 0; T0 < total; T0 += kCellOf) {
    {
      const int b0 = max(pre_t, T0), b1 = min(pre_t + cnt, T0 + kCellOf);
      for (int q = b0; q < b1; ++q) s_cellof[q - T0] = (unsigned char)tid;
    }
    __syncthreads();
    const int T1 = min(total, T0 + kCellOf);
    for (int t0 = T0; t0 < T1; t0 += kBuildThreads) {
      const int t = t0 + tid;
      unsigned mask = 0;
      int s = 0;
      if (t < T1) {
        const int l = s_cellof[t - T0];
        s = s_start[l] + (t - s_pre[l]);
        const int a = perm[s];
        const float4 rj = xq[s];
        const float xj[3] = {rj.x, rj.y, rj.z};
        {
          if (shift) {
            float rj3[3];
            for (int d = 0; d < 3; ++d) {
              const float v = xj[d] - xi[0][d];
              rj3[d] = __fmaf_rn(-Lf[d], rintf(v * iLf[d]), v);
            }
            // |r_j|^2 - 2 r_i.r_j - (r_list + 0.01)^2 < -|r_i|^2
            const float nthr = __fmaf_rn(rj3[0], rj3[0], __fmaf_rn(rj3[1], rj3[1], rj3[2] * rj3[2])) - inc2;
#pragma unroll
            for (int ii = kClus - 1; ii >= 0; --ii) {        // bit ii ends at position ii
              const float q = __fmaf_rn(m2[ii][0], rj3[0], __fmaf_rn(m2[ii][1], rj3[1], __fmaf_rn(m2[ii][2], rj3[2], nthr)));
              mask = 2u * mask + (q < nc2[ii] ? 1u : 0u);
            }
          } else {
            // rare (small boxes, spread clusters): positions from LDS and no
            // unrolling, so this path adds no registers to the common one
#pragma unroll 1
            for (int ii = 0; ii < kClus; ++ii) {
              float dx = xj[0] - s_xi[ii][0], dy = xj[1] - s_xi[ii][1], dz = xj[2] - s_xi[ii][2];
              dx -= Lf[0] * rintf(dx * iLf[0]);
              dy -= Lf[1] * rintf(dy * iLf[1]);
              dz -= Lf[2] * rintf(dz * iLf[2]);
              const float d2 = (dx * dx + dy * dy) + dz * dz;
              if (d2 < inc2 && ai[ii] >= 0) mask |= 1u << ii;
            }
          }
          const unsigned self = (unsigned)(s - c * kClus);       // the cluster's own atom: no i == j pair
          if (self < (unsigned)kClus) mask &= ~(1u << self);
          if (mask && ((s_bloom[(a >> 5) & 63] >> (a & 31)) & 1u)) {   // possibly excluded
            for (int ii = 0; ii < kClus; ++ii) {
              if (!((mask >> ii) & 1u)) continue;
              bool ex = false;
              for (int k = 0; k < s_nex[ii]; ++k) ex |= (s_ex[ii][k] == a);
              if (ex) mask &= ~(1u << ii);
            }
          }
        }
      }
      const unsigned mL = mask & 0xFu, mH = mask >> 4;
      const unsigned long long bL = __ballot(mL != 0u), bH = __ballot(mH != 0u);
      if (lane == 0) { s_wc[par][0][wave] = __popcll(bL); s_wc[par][1][wave] = __popcll(bH); }
      __syncthreads();
      int offL = countL, offH = countH;
      for (int k = 0; k < wave; ++k) { offL += s_wc[par][0][k]; offH += s_wc[par][1][k]; }
      for (int k = 0; k < kBuildWaves; ++k) { countL += s_wc[par][0][k]; countH += s_wc[par][1][k]; }
      if (mL) {
        const int pos = offL + __popcll(bL & lt);
        if (pos < cap) outL[pos] = ((unsigned)s << 8) | mL;
      }
      if (mH) {
        const int pos = offH + __popcll(bH & lt);
        if (pos < cap) outH[pos] = ((unsigned)s << 8) | mH;
      }
      par ^= 1;
    }
    __syncthreads();                            // the window's table is rewritten next
    }
    __syncthreads();                            // the round's tables are rewritten next
  }
  const int count = max(countL, countH);
  if (count > cap) {
    if (tid == 0) {
      latch(g.err, kErrListCap, kSiteList, (w << 20) | max(s_ai[0], 0), g.leg_index);
      atomicMax(g.need, count);
    }
  }
  if (tid == 0) {
    g.lcount[2 * item] = min(countL, cap);
    g.lcount[2 * item + 1] = min(countH, cap);
  }
}

// Export pairs i < j with a set list bit and FP64 distance < r (both
// half-cluster lists).
__global__ __launch_bounds__(256) void k_export(const LegDev* legs, int leg, int w, double r2,
                                                int* pairs, long long cap,
                                                unsigned long long* count) {
  const LegDev& g = legs[leg];
  const int c = blockIdx.x;
  if (c >= g.nclus) return;
  const size_t item = (size_t)w * g.nclus + c;
  const int* perm = g.perm + (size_t)w * g.npad;
  const size_t o = (size_t)w * g.n;
  for (int half = 0; half < 2; ++half) {
    const unsigned* ent = g.lent + (item * 2 + half) * g.cap;
    const int cnt = g.lcount[item * 2 + half];
    for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
      const unsigned v = ent[e];
      const unsigned m = v & 0xfu;
      if (!m) continue;
      const int aj = perm[v >> 8];
      for (int k = 0; k < 4; ++k) {
        if (!((m >> k) & 1u)) continue;
        const int ai = perm[c * kClus + 4 * half + k];
        if (ai >= aj) continue;
        double dx = (double)g.x[o + aj] - (double)g.x[o + ai];
        double dy = (double)g.y[o + aj] - (double)g.y[o + ai];
        double dz = (double)g.z[o + aj] - (double)g.z[o + ai];
        const BoxW& B = g.box[w];
        dx = dx - B.L[0] * rint(dx * B.invL[0]);
        dy = dy - B.L[1] * rint(dy * B.invL[1]);
        dz = dz - B.L[2] * rint(dz * B.invL[2]);
        const double d2 = (dx * dx + dy * dy) + dz * dz;
        if (!(d2 < r2)) continue;
        const unsigned long long k2 = atomicAdd(count, 1ull);
        if ((long long)k2 < cap) { pairs[2 * k2] = ai; pairs[2 * k2 + 1] = aj; }
      }
    }
  }
}

inline int blocks_for(long long items, int per) { return (int)((items + per - 1) / per); }

}  // namespace

void launch_check(hipStream_t s, const LegDev* d, const LegHost* h, int nl, int force, bool from_word) {
  BlockMap m;
  int nb = make_map(m, nl, [&](int i) { return sort_in_lds(h[i]) ? 0 : h[i].W; });
  if (nb) {
    if (from_word) hipLaunchKernelGGL(k_check<true>, dim3(nb), dim3(256), 0, s, d, m, force);
    else hipLaunchKernelGGL(k_check<false>, dim3(nb), dim3(256), 0, s, d, m, force);
  }
  // small legs: the check and the whole cell sort in one launch
  nb = make_map(m, nl, [&](int i) { return sort_in_lds(h[i]) ? h[i].W : 0; });
  if (nb) {
    if (from_word) hipLaunchKernelGGL(k_check_sort<true>, dim3(nb), dim3(1024), 0, s, d, m, force);
    else hipLaunchKernelGGL(k_check_sort<false>, dim3(nb), dim3(1024), 0, s, d, m, force);
  }
}

void launch_sort_pack(hipStream_t s, const LegDev* d, const LegHost* h, int nl) {
  BlockMap m;
  // grid-wide cell sort for the legs that launch_check did not sort
  auto big = [&](int i) { return !sort_in_lds(h[i]); };
  int nb = make_map(m, nl, [&](int i) { return big(i) ? blocks_for((long long)h[i].W * h[i].n, 256) : 0; });
  if (nb) hipLaunchKernelGGL(k_cells_count, dim3(nb), dim3(256), 0, s, d, m);
  nb = make_map(m, nl, [&](int i) { return big(i) ? h[i].W : 0; });
  if (nb) hipLaunchKernelGGL(k_cells_scan, dim3(nb), dim3(1024), 0, s, d, m);
  nb = make_map(m, nl, [&](int i) { return big(i) ? blocks_for((long long)h[i].W * h[i].n, 256) : 0; });
  if (nb) hipLaunchKernelGGL(k_cells_scatter, dim3(nb), dim3(256), 0, s, d, m);
  nb = make_map(m, nl, [&](int i) { return big(i) ? blocks_for((long long)h[i].W * h[i].ncell, 256) : 0; });
  if (nb) hipLaunchKernelGGL(k_cells_order, dim3(nb), dim3(256), 0, s, d, m);
  // sorted coordinates every step; sorted parameters and cluster boxes for
  // the windows being rebuilt
  launch_pack(s, d, h, nl, true);
}

void launch_lists(hipStream_t s, const LegDev* d, const LegHost* h, int nl) {
  BlockMap m;
  const int nb = make_map(m, nl, [&](int i) { return h[i].W * h[i].nclus; });
  if (nb) hipLaunchKernelGGL(k_build, dim3(nb), dim3(kBuildThreads), 0, s, d, m);
}

void launch_build(hipStream_t s, const LegDev* d, const LegHost* h, int nl) {
  launch_sort_pack(s, d, h, nl);
  launch_lists(s, d, h, nl);
}

void launch_export(hipStream_t s, const LegDev* d, const LegHost& h, int window, double r,
                   int* pairs, long long cap, unsigned long long* count) {
  if (h.nclus) hipLaunchKernelGGL(k_export, dim3(h.nclus), dim3(256), 0, s, d, 0, window, r * r, pairs, cap, count);
}

}  // namespace felis
