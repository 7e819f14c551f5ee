// Neighbour lists: displacement check, Morton cell sort, 8-atom clusters and
// per-cluster j-lists with FP64 exact inclusion bits (appendix B cutoffs).
//
// Built with -ffp-contract=off: the FP64 inclusion test d^2 < r_list^2 uses
// d = x_j - x_i, d -= L * rint(d / L) (separate multiply and subtract) and
// d^2 = (dx^2 + dy^2) + dz^2, so the set of listed pairs is a deterministic
// function of the float coordinates.
#include "felis_internal.h"

namespace felis {
namespace {

__device__ __forceinline__ unsigned morton3(unsigned x, unsigned y, unsigned z, int bits) {
  unsigned c = 0;
  for (int b = 0; b < bits; ++b) {
    c |= ((x >> b) & 1u) << (3 * b);
    c |= ((y >> b) & 1u) << (3 * b + 1);
    c |= ((z >> b) & 1u) << (3 * b + 2);
  }
  return c;
}

__device__ __forceinline__ int cell_of(float v, float L, float invL, int n) {
  float u = wrapf(v, L, invL) * invL;
  int c = (int)(u * (float)n);
  return c < 0 ? 0 : (c >= n ? n - 1 : c);
}

// One block per window: rebuild flag = force || max displacement > skin/2.
__global__ __launch_bounds__(256) void k_check(const LegDev* legs, BlockMap map, int force) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const int w = blockIdx.x - map.start[leg];
  __shared__ float red[256];
  float m = 0.f;
  if (!force) {
    const size_t o = (size_t)w * g.n;
    for (int a = threadIdx.x; a < g.n; a += blockDim.x) {
      float dx = g.x[o + a] - g.xr[o + a], dy = g.y[o + a] - g.yr[o + a], dz = g.z[o + a] - g.zr[o + a];
      m = fmaxf(m, dx * dx + dy * dy + dz * dz);
    }
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) g.flag[w] = (force || !(red[0] <= g.skin_half2)) ? 1 : 0;
}

// items: window x cell -- zero the per-cell counters of windows being rebuilt
__global__ __launch_bounds__(256) void k_cells_zero(const LegDev* legs, BlockMap map) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const long long i = (long long)(blockIdx.x - map.start[leg]) * blockDim.x + threadIdx.x;
  if (i >= (long long)g.W * g.ncell) return;
  const int w = (int)(i / g.ncell);
  if (!g.flag[w]) return;
  g.cursor[i] = 0;
}

// items: window x atom -- Morton cell code, per-cell counts, reference positions
__global__ __launch_bounds__(256) void k_cells_count(const LegDev* legs, BlockMap map) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const long long i = (long long)(blockIdx.x - map.start[leg]) * blockDim.x + threadIdx.x;
  if (i >= (long long)g.W * g.n) return;
  const int w = (int)(i / g.n);
  if (!g.flag[w]) return;
  const int nf = 1 << g.nbits;
  const float x = g.x[i], y = g.y[i], z = g.z[i];
  const unsigned c = morton3(cell_of(x, g.Lf[0], g.invLf[0], nf), cell_of(y, g.Lf[1], g.invLf[1], nf),
                             cell_of(z, g.Lf[2], g.invLf[2], nf), g.nbits);
  g.cellcode[i] = (int)c;
  atomicAdd(&g.cursor[(size_t)w * g.ncell + c], 1);
  g.xr[i] = x; g.yr[i] = y; g.zr[i] = z;
}

// one block per window: exclusive scan of the counts into cellstart; reset cursor
__global__ __launch_bounds__(1024) void k_cells_scan(const LegDev* legs, BlockMap map) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const int w = blockIdx.x - map.start[leg];
  if (!g.flag[w]) return;
  int* cnt = g.cursor + (size_t)w * g.ncell;
  int* st = g.cellstart + (size_t)w * (g.ncell + 1);
  const int T = blockDim.x;
  const int per = (g.ncell + T - 1) / T;
  const int b0 = threadIdx.x * per;
  const int b1 = min(g.ncell, b0 + per);
  int sum = 0;
  for (int c = b0; c < b1; ++c) sum += cnt[c];
  __shared__ int part[1024];
  part[threadIdx.x] = sum;
  __syncthreads();
  for (int o = 1; o < T; o <<= 1) {          // Hillis-Steele inclusive scan
    int v = threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int run = part[threadIdx.x] - sum;
  for (int c = b0; c < b1; ++c) {
    st[c] = run;
    run += cnt[c];
    cnt[c] = 0;
  }
  if (threadIdx.x == T - 1) st[g.ncell] = part[T - 1];
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

// items: window x slot -- per-slot constant parameters in sorted order
__global__ __launch_bounds__(256) void k_sorted_params(const LegDev* legs, BlockMap map) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const long long i = (long long)(blockIdx.x - map.start[leg]) * blockDim.x + threadIdx.x;
  if (i >= (long long)g.W * g.npad) return;
  const int w = (int)(i / g.npad);
  if (!g.flag[w]) return;
  const int a = g.perm[i];
  float4 p = make_float4(0.f, 0.f, 0.f, 0.f);
  if (a >= 0) p = make_float4(0.5f * g.sig[a], 2.0f * sqrtf(g.eps[a]), g.lig[a] ? 1.f : 0.f, g.q[a]);
  g.prm[i] = p;
}

// items: window x cluster -- bounding box of wrapped positions
__global__ __launch_bounds__(256) void k_bbox(const LegDev* legs, BlockMap map) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const long long i = (long long)(blockIdx.x - map.start[leg]) * blockDim.x + threadIdx.x;
  if (i >= (long long)g.W * g.nclus) return;
  const int w = (int)(i / g.nclus);
  if (!g.flag[w]) return;
  const int c = (int)(i - (long long)w * g.nclus);
  const int* p = g.perm + (size_t)w * g.npad + c * kClus;
  const size_t o = (size_t)w * g.n;
  float lo[3] = {3.0e38f, 3.0e38f, 3.0e38f}, hi[3] = {-3.0e38f, -3.0e38f, -3.0e38f};
  for (int k = 0; k < kClus; ++k) {
    const int a = p[k];
    if (a < 0) continue;
    const float v[3] = {wrapf(g.x[o + a], g.Lf[0], g.invLf[0]), wrapf(g.y[o + a], g.Lf[1], g.invLf[1]),
                        wrapf(g.z[o + a], g.Lf[2], g.invLf[2])};
    for (int d = 0; d < 3; ++d) { lo[d] = fminf(lo[d], v[d]); hi[d] = fmaxf(hi[d], v[d]); }
  }
  g.bblo[i] = make_float4(lo[0], lo[1], lo[2], 0.f);
  g.bbhi[i] = make_float4(hi[0], hi[1], hi[2], 0.f);
}

// One wave per cluster: scan the coarse cells within r_list of the cluster's
// box and list every atom j with at least one i of the cluster in range.
__global__ __launch_bounds__(256) void k_build(const LegDev* legs, BlockMap map) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long long item = (long long)(blockIdx.x - map.start[leg]) * 4 + wave;
  const long long total = (long long)g.W * g.nclus;
  const long long itm = item < total ? item : total - 1;
  const int w = (int)(itm / g.nclus);
  const bool active = item < total && g.flag[w] != 0;   // uniform per wave
  const int c = (int)(itm - (long long)w * g.nclus);

  __shared__ int s_ai[4][kClus];
  __shared__ double s_xi[4][kClus][3];
  __shared__ int s_ex[4][kClus][kMaxExcl];
  __shared__ int s_nex[4][kClus];
  const size_t o = (size_t)w * g.n;
  const int* perm = g.perm + (size_t)w * g.npad;
  if (active && lane < kClus) {
    const int a = perm[c * kClus + lane];
    s_ai[wave][lane] = a;
    int ne = 0;
    if (a >= 0) {
      s_xi[wave][lane][0] = (double)g.x[o + a];
      s_xi[wave][lane][1] = (double)g.y[o + a];
      s_xi[wave][lane][2] = (double)g.z[o + a];
      const int e0 = g.excl_ptr[a], e1 = g.excl_ptr[a + 1];
      ne = e1 - e0;
      if (ne > kMaxExcl) { atomicOr(g.err, kErrExcl); ne = kMaxExcl; }
      for (int k = 0; k < ne; ++k) s_ex[wave][lane][k] = g.excl_idx[e0 + k];
    }
    s_nex[wave][lane] = ne;
  }
  __syncthreads();            // every wave of the block reaches this barrier
  if (!active) return;

  const float4 lo4 = g.bblo[item], hi4 = g.bbhi[item];
  const float lo[3] = {lo4.x, lo4.y, lo4.z}, hi[3] = {hi4.x, hi4.y, hi4.z};
  float cen[3], half[3];
  int r0[3], r1[3];
  const int nco = g.ncoarse;
  for (int d = 0; d < 3; ++d) {
    cen[d] = 0.5f * (lo[d] + hi[d]);
    half[d] = 0.5f * (hi[d] - lo[d]);
    const float cs = g.Lf[d] / (float)nco;
    r0[d] = (int)floorf((lo[d] - (float)g.rlist) / cs) - 1;
    r1[d] = (int)floorf((hi[d] + (float)g.rlist) / cs) + 1;
    if (r1[d] - r0[d] + 1 >= nco) { r0[d] = 0; r1[d] = nco - 1; }
  }
  const float pre = (float)g.rlist + 0.05f;
  const float pre2 = pre * pre;
  const int* cst = g.cellstart + (size_t)w * (g.ncell + 1);
  unsigned* out = g.lent + (size_t)item * g.cap;
  int count = 0;
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

  for (int X = r0[0]; X <= r1[0]; ++X)
    for (int Y = r0[1]; Y <= r1[1]; ++Y)
      for (int Z = r0[2]; Z <= r1[2]; ++Z) {
        const unsigned cc = morton3((unsigned)((X % nco + nco) % nco), (unsigned)((Y % nco + nco) % nco),
                                    (unsigned)((Z % nco + nco) % nco), g.nbits - 1);
        const int s0 = cst[8 * cc], s1 = cst[8 * cc + 8];
        for (int sb = s0; sb < s1; sb += 64) {
          const int s = sb + lane;
          unsigned mask = 0;
          if (s < s1) {
            const int a = perm[s];
            const float xj[3] = {g.x[o + a], g.y[o + a], g.z[o + a]};
            float dd = 0.f;
            for (int d = 0; d < 3; ++d) {
              float v = wrapf(xj[d], g.Lf[d], g.invLf[d]) - cen[d];
              v -= g.Lf[d] * rintf(v * g.invLf[d]);
              float e = fabsf(v) - half[d];
              if (half[d] > 0.25f * g.Lf[d]) e = 0.f;
              e = fmaxf(e, 0.f);
              dd += e * e;
            }
            if (dd < pre2) {
              const double X0 = (double)xj[0], X1 = (double)xj[1], X2 = (double)xj[2];
              for (int ii = 0; ii < kClus; ++ii) {
                const int ai = s_ai[wave][ii];
                if (ai < 0 || ai == a) continue;
                double dx = X0 - s_xi[wave][ii][0];
                double dy = X1 - s_xi[wave][ii][1];
                double dz = X2 - s_xi[wave][ii][2];
                dx = dx - g.L[0] * rint(dx * g.invL[0]);
                dy = dy - g.L[1] * rint(dy * g.invL[1]);
                dz = dz - g.L[2] * rint(dz * g.invL[2]);
                const double d2 = (dx * dx + dy * dy) + dz * dz;
                if (!(d2 < g.rlist2)) continue;
                bool ex = false;
                for (int k = 0; k < s_nex[wave][ii]; ++k) ex |= (s_ex[wave][ii][k] == a);
                if (!ex) mask |= 1u << ii;
              }
            }
          }
          const unsigned long long bal = __ballot(mask != 0u);
          if (mask) {
            const int pos = count + __popcll(bal & lt);
            if (pos < g.cap) out[pos] = ((unsigned)s << 8) | mask;
          }
          count += __popcll(bal);
        }
      }
  if (count > g.cap) {
    if (lane == 0) { atomicOr(g.err, kErrListCap); atomicMax(g.need, count); }
    count = g.cap;
  }
  const int padded = min(g.cap, (count + 7) & ~7);
  for (int p = count + lane; p < padded; p += 64) out[p] = 0u;
  if (lane == 0) g.lcount[item] = padded;
}

// Export pairs i < j with a set list bit and FP64 distance < r.
__global__ __launch_bounds__(256) void k_export(const LegDev* legs, int leg, int w, double r2,
                                                int* pairs, long long cap,
                                                unsigned long long* count) {
  const LegDev& g = legs[leg];
  const int c = blockIdx.x;
  if (c >= g.nclus) return;
  const size_t item = (size_t)w * g.nclus + c;
  const int* perm = g.perm + (size_t)w * g.npad;
  const unsigned* ent = g.lent + item * g.cap;
  const int cnt = g.lcount[item];
  const size_t o = (size_t)w * g.n;
  for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
    const unsigned v = ent[e];
    const unsigned m = v & 0xffu;
    if (!m) continue;
    const int aj = perm[v >> 8];
    for (int ii = 0; ii < kClus; ++ii) {
      if (!((m >> ii) & 1u)) continue;
      const int ai = perm[c * kClus + ii];
      if (ai >= aj) continue;
      double dx = (double)g.x[o + aj] - (double)g.x[o + ai];
      double dy = (double)g.y[o + aj] - (double)g.y[o + ai];
      double dz = (double)g.z[o + aj] - (double)g.z[o + ai];
      dx = dx - g.L[0] * rint(dx * g.invL[0]);
      dy = dy - g.L[1] * rint(dy * g.invL[1]);
      dz = dz - g.L[2] * rint(dz * g.invL[2]);
      const double d2 = (dx * dx + dy * dy) + dz * dz;
      if (!(d2 < r2)) continue;
      const unsigned long long k = atomicAdd(count, 1ull);
      if ((long long)k < cap) { pairs[2 * k] = ai; pairs[2 * k + 1] = aj; }
    }
  }
}

inline int blocks_for(long long items, int per) { return (int)((items + per - 1) / per); }

}  // namespace

void launch_check(hipStream_t s, const LegDev* d, const LegHost* h, int nl, int force) {
  BlockMap m;
  const int nb = make_map(m, nl, [&](int i) { return h[i].W; });
  if (nb) hipLaunchKernelGGL(k_check, dim3(nb), dim3(256), 0, s, d, m, force);
}

void launch_build(hipStream_t s, const LegDev* d, const LegHost* h, int nl) {
  BlockMap m;
  int nb = make_map(m, nl, [&](int i) { return blocks_for((long long)h[i].W * h[i].ncell, 256); });
  if (nb) hipLaunchKernelGGL(k_cells_zero, dim3(nb), dim3(256), 0, s, d, m);
  nb = make_map(m, nl, [&](int i) { return blocks_for((long long)h[i].W * h[i].n, 256); });
  if (nb) hipLaunchKernelGGL(k_cells_count, dim3(nb), dim3(256), 0, s, d, m);
  nb = make_map(m, nl, [&](int i) { return h[i].W; });
  if (nb) hipLaunchKernelGGL(k_cells_scan, dim3(nb), dim3(1024), 0, s, d, m);
  nb = make_map(m, nl, [&](int i) { return blocks_for((long long)h[i].W * h[i].n, 256); });
  if (nb) hipLaunchKernelGGL(k_cells_scatter, dim3(nb), dim3(256), 0, s, d, m);
  nb = make_map(m, nl, [&](int i) { return blocks_for((long long)h[i].W * h[i].ncell, 256); });
  if (nb) hipLaunchKernelGGL(k_cells_order, dim3(nb), dim3(256), 0, s, d, m);
  nb = make_map(m, nl, [&](int i) { return blocks_for((long long)h[i].W * h[i].npad, 256); });
  if (nb) hipLaunchKernelGGL(k_sorted_params, dim3(nb), dim3(256), 0, s, d, m);
  nb = make_map(m, nl, [&](int i) { return blocks_for((long long)h[i].W * h[i].nclus, 256); });
  if (nb) hipLaunchKernelGGL(k_bbox, dim3(nb), dim3(256), 0, s, d, m);
  nb = make_map(m, nl, [&](int i) { return blocks_for((long long)h[i].W * h[i].nclus, 4); });
  if (nb) hipLaunchKernelGGL(k_build, dim3(nb), dim3(256), 0, s, d, m);
}

void launch_export(hipStream_t s, const LegDev* d, const LegHost& h, int window, double r,
                   int* pairs, long long cap, unsigned long long* count) {
  if (h.nclus) hipLaunchKernelGGL(k_export, dim3(h.nclus), dim3(256), 0, s, d, 0, window, r * r, pairs, cap, count);
}

}  // namespace felis
