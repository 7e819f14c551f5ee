// PME reciprocal space (smooth PME, Essmann et al. 1995; the paper names PME
// with a 1 nm real-space cutoff in appendix B and prints no PME formulas).
//
// Per window: charges q~ (ligand x lambda_elec) spread with order-4 cardinal
// B-splines into an int64 fixed-point grid (order-independent atomics, so the
// grid is bitwise reproducible).  Two windows of one leg share a complex grid
// Z = Q_a + i Q_b: with a real, even influence function G the convolution
// IDFT(G DFT(Z)) = phi_a + i phi_b, so one complex FFT pair serves two
// windows.  phi = IDFT_unnormalised(G DFT(Q)), G(m) = KE/(pi V)
// exp(-pi^2 |m|^2/alpha^2)/|m|^2 |b1 b2 b3|^2, G(0) = 0;
// E_rec = 1/2 sum_i q~_i phi(r_i); F_i = -q~_i grad(spline weights) . phi.
//
// FFT: Stockham autosort, radices 4/2/3/5, one kernel per axis; a workgroup
// holds 16 lines in LDS ([element][line] layout, coalesced loads for every
// axis).  The inverse transform is conj(DFT(conj(.))).  The z pass fuses
// forward transform, multiplication by G and inverse transform.
#include "felis_internal.h"

namespace felis {
namespace {

constexpr int kLines = 16;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }   // a * (-i)
__device__ __forceinline__ float2 conj2(float2 a) { return make_float2(a.x, -a.y); }

// forward DFT (sign -1) of size R in place
template <int R>
__device__ __forceinline__ void dft(float2* v) {
  if (R == 2) {
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b); v[1] = csub(a, b);
  } else if (R == 4) {
    const float2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    const float2 s13 = cadd(v[1], v[3]), d13 = mul_mi(csub(v[1], v[3]));
    v[0] = cadd(s02, s13); v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13); v[3] = csub(d02, d13);
  } else if (R == 3) {
    const float h = 0.86602540378443865f;               // sin(2 pi / 3)
    const float2 s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
    const float2 a = v[0];
    const float2 m = make_float2(a.x - 0.5f * s.x, a.y - 0.5f * s.y);
    const float2 t = mul_mi(make_float2(h * d.x, h * d.y));
    v[0] = cadd(a, s); v[1] = cadd(m, t); v[2] = csub(m, t);
  } else {  // R == 5
    const float c1 = 0.30901699437494742f, c2 = -0.80901699437494742f;   // cos(2pi/5), cos(4pi/5)
    const float s1 = 0.95105651629515357f, s2 = 0.58778525229247313f;    // sin(2pi/5), sin(4pi/5)
    const float2 x0 = v[0];
    const float2 a1 = cadd(v[1], v[4]), b1 = csub(v[1], v[4]);
    const float2 a2 = cadd(v[2], v[3]), b2 = csub(v[2], v[3]);
    const float2 m1 = make_float2(x0.x + c1 * a1.x + c2 * a2.x, x0.y + c1 * a1.y + c2 * a2.y);
    const float2 m2 = make_float2(x0.x + c2 * a1.x + c1 * a2.x, x0.y + c2 * a1.y + c1 * a2.y);
    const float2 t1 = mul_mi(make_float2(s1 * b1.x + s2 * b2.x, s1 * b1.y + s2 * b2.y));
    const float2 t2 = mul_mi(make_float2(s2 * b1.x - s1 * b2.x, s2 * b1.y - s1 * b2.y));
    v[0] = make_float2(x0.x + a1.x + a2.x, x0.y + a1.y + a2.y);
    v[1] = cadd(m1, t1); v[4] = csub(m1, t1);
    v[2] = cadd(m2, t2); v[3] = csub(m2, t2);
  }
}

// One Stockham stage of radix R over kLines lines (buf[e * kLines + b]).
template <int R>
__device__ __forceinline__ void stage(const float2* src, float2* dst, int n, int Ns,
                                      const float2* __restrict__ tw) {
  const int nR = n / R;
  const int step = n / (Ns * R);
  for (int t = threadIdx.x; t < nR * kLines; t += blockDim.x) {
    const int j = t / kLines, b = t - j * kLines;
    const int k = j % Ns;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      v[r] = src[(j + r * nR) * kLines + b];
      if (r) v[r] = cmul(v[r], tw[r * k * step]);       // r k step < n
    }
    dft<R>(v);
    const int o = (j / Ns) * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[(o + r * Ns) * kLines + b] = v[r];
  }
}

// Forward transform of kLines lines of length n held in src[e * kLines + b];
// returns the buffer that holds the result.
__device__ float2* fft_lines(float2* src, float2* dst, int n, const int* rad, int nrad,
                             const float2* __restrict__ tw) {
  int Ns = 1;
  for (int st = 0; st < nrad; ++st) {
    const int R = rad[st];
    switch (R) {
      case 2: stage<2>(src, dst, n, Ns, tw); break;
      case 3: stage<3>(src, dst, n, Ns, tw); break;
      case 4: stage<4>(src, dst, n, Ns, tw); break;
      default: stage<5>(src, dst, n, Ns, tw); break;
    }
    __syncthreads();
    float2* t = src; src = dst; dst = t;
    Ns *= R;
  }
  return src;
}

// MODE: 0 forward, 1 inverse, 2 forward from the int64 grids (x axis),
//       3 forward * G * inverse (z axis)
template <int AXIS, int MODE>
__global__ __launch_bounds__(256) void k_fft(const LegDev* legs, BlockMap map) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const int Kx = g.K[0], Ky = g.K[1], Kz = g.K[2];
  const int n = g.K[AXIS];
  // lines: x axis -> (z, y-chunk); y axis -> (z, x-chunk); z axis -> (y, x-chunk)
  const int inner = (AXIS == 0) ? Ky : Kx;
  const int outer = (AXIS == 2) ? Ky : Kz;
  const int nch = (inner + kLines - 1) / kLines;
  const int bl = blockIdx.x - map.start[leg];
  const int p = bl / (outer * nch);
  const int rem = bl - p * outer * nch;
  const int o = rem / nch, ch = rem - (rem / nch) * nch;
  if (p >= g.npair) return;
  __shared__ float2 bufA[kMaxFFT * kLines];
  __shared__ float2 bufB[kMaxFFT * kLines];
  float2* cg = g.cgrid + (size_t)p * g.Ktot;
  const int KxKy = Kx * Ky;
  auto offs = [&](int e, int b) -> long long {
    const int li = ch * kLines + b;
    if (li >= inner) return -1;
    if (AXIS == 0) return (long long)o * KxKy + (long long)li * Kx + e;
    if (AXIS == 1) return (long long)o * KxKy + (long long)e * Kx + li;
    return (long long)e * KxKy + (long long)o * Kx + li;
  };
  for (int idx = threadIdx.x; idx < n * kLines; idx += blockDim.x) {
    int e, b;
    if (AXIS == 0) { b = idx / n; e = idx - b * n; } else { e = idx / kLines; b = idx - e * kLines; }
    const long long off = offs(e, b);
    float2 v = make_float2(0.f, 0.f);
    if (off >= 0) {
      if (MODE == 2) {
        const int w0 = 2 * p, w1 = 2 * p + 1;
        long long* q0 = g.grid64 + (size_t)w0 * g.Ktot + off;
        v.x = (float)((double)*q0 * (1.0 / kGridScale));
        *q0 = 0;
        long long* q1 = g.grid64 + (size_t)w1 * g.Ktot + off;      // 2 npair grids exist
        v.y = (float)((double)*q1 * (1.0 / kGridScale));
        *q1 = 0;
      } else {
        v = cg[off];
        if (MODE == 1) v = conj2(v);
      }
    }
    bufA[e * kLines + b] = v;
  }
  __syncthreads();
  const float2* tw = g.tw[AXIS];
  float2* res = fft_lines(bufA, bufB, n, g.rad[AXIS], g.nrad[AXIS], tw);
  if (MODE == 3) {
    // multiply by G(kx, ky, kz): element e = kz of line (ky = o, kx = ch*kLines + b)
    const float a2 = g.alpha * g.alpha;
    for (int idx = threadIdx.x; idx < n * kLines; idx += blockDim.x) {
      const int e = idx / kLines, b = idx - e * kLines;
      const int kx = ch * kLines + b, ky = o, kz = e;
      float G = 0.f;
      if (kx < Kx) {
        const float mx = (float)(kx <= Kx / 2 ? kx : kx - Kx) * g.invLf[0];
        const float my = (float)(ky <= Ky / 2 ? ky : ky - Ky) * g.invLf[1];
        const float mz = (float)(kz <= Kz / 2 ? kz : kz - Kz) * g.invLf[2];
        const float m2 = mx * mx + my * my + mz * mz;
        if (m2 > 0.f)
          G = g.pme_pref * __expf(-9.8696044010893586f * m2 / a2) / m2 * g.bmod[0][kx] * g.bmod[1][ky] *
              g.bmod[2][kz];
      }
      const float2 v = res[idx];
      res[idx] = conj2(make_float2(v.x * G, v.y * G));     // conj for the inverse pass
    }
    __syncthreads();
    float2* other = (res == bufA) ? bufB : bufA;
    res = fft_lines(res, other, n, g.rad[AXIS], g.nrad[AXIS], tw);
  }
  for (int idx = threadIdx.x; idx < n * kLines; idx += blockDim.x) {
    int e, b;
    if (AXIS == 0) { b = idx / n; e = idx - b * n; } else { e = idx / kLines; b = idx - e * kLines; }
    const long long off = offs(e, b);
    if (off < 0) continue;
    float2 v = res[e * kLines + b];
    if (MODE == 1 || MODE == 3) v = conj2(v);
    cg[off] = v;
  }
}

__device__ __forceinline__ void bspline4(float f, float* w, float* dw) {
  const float f2 = f * f, f3 = f2 * f, g1 = 1.0f - f;
  w[0] = f3 * (1.0f / 6.0f);
  w[1] = (-3.0f * f3 + 3.0f * f2 + 3.0f * f + 1.0f) * (1.0f / 6.0f);
  w[2] = (3.0f * f3 - 6.0f * f2 + 4.0f) * (1.0f / 6.0f);
  w[3] = g1 * g1 * g1 * (1.0f / 6.0f);
  if (dw) {
    dw[0] = 0.5f * f2;
    dw[1] = 0.5f * (-3.0f * f2 + 2.0f * f + 1.0f);
    dw[2] = 0.5f * (3.0f * f2 - 4.0f * f);
    dw[3] = -0.5f * g1 * g1;
  }
}

// fractional grid coordinate in FP64: base index and offset f in [0, 1)
__device__ __forceinline__ int grid_base(float x, double invL, int K, float* f) {
  double u = (double)x * invL * (double)K;
  if (!(fabs(u) < 1.0e15)) u = 0.0;              // non-finite input -> 0 (keeps indices in range)
  const double b = floor(u);
  *f = (float)(u - b);
  long long k = (long long)b % K;
  if (k < 0) k += K;
  return (int)k;
}

// items: window x atom, 16 lanes per atom (lane = ix + 4 iy, loop over iz):
// the four x points of a grid row are adjacent lanes, so each atomic
// instruction touches 16 row segments of 32 contiguous bytes
__global__ __launch_bounds__(256) void k_spread(const LegDev* legs, BlockMap map) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const long long local = (long long)(blockIdx.x - map.start[leg]) * 16 + (threadIdx.x >> 4);
  if (local >= (long long)g.W * g.n) return;
  const int w = (int)(local / g.n);
  const int a = (int)(local - (long long)w * g.n);
  const int sub = threadIdx.x & 15, ix = sub & 3, iy = sub >> 2;
  const size_t o = (size_t)w * g.n + a;
  const float q = g.q[a] * (g.lig[a] ? g.lam[4 * w] : 1.0f);
  float fxr, fyr, fzr, wx[4], wy[4], wz[4];
  const int bx = grid_base(g.x[o], g.invL[0], g.K[0], &fxr);
  const int by = grid_base(g.y[o], g.invL[1], g.K[1], &fyr);
  const int bz = grid_base(g.z[o], g.invL[2], g.K[2], &fzr);
  bspline4(fxr, wx, nullptr);
  bspline4(fyr, wy, nullptr);
  bspline4(fzr, wz, nullptr);
  int gx = bx - ix; if (gx < 0) gx += g.K[0];
  int gy = by - iy; if (gy < 0) gy += g.K[1];
  long long* grid = g.grid64 + (size_t)w * g.Ktot + (size_t)gy * g.K[0] + gx;
  const double qxy = (double)(q * wx[ix] * wy[iy]);
#pragma unroll
  for (int iz = 0; iz < 4; ++iz) {
    int gz = bz - iz; if (gz < 0) gz += g.K[2];
    const long long v = __double2ll_rn(qxy * (double)wz[iz] * kGridScale);
    if (v) atomicAdd((unsigned long long*)&grid[(size_t)gz * g.K[0] * g.K[1]], (unsigned long long)v);
  }
}

template <bool ENERGY>
__global__ __launch_bounds__(256) void k_gather(const LegDev* legs, BlockMap map) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const long long local = (long long)(blockIdx.x - map.start[leg]) * 16 + (threadIdx.x >> 4);
  const long long tot = (long long)g.W * g.n;
  const bool valid = local < tot;
  const long long lc = valid ? local : tot - 1;
  const int w = (int)(lc / g.n);
  const int a = (int)(lc - (long long)w * g.n);
  const int sub = threadIdx.x & 15, iy = sub & 3, iz = sub >> 2;
  const size_t o = (size_t)w * g.n + a;
  const float q = g.q[a] * (g.lig[a] ? g.lam[4 * w] : 1.0f);
  float fxr, fyr, fzr, wx[4], wy[4], wz[4], dx[4], dy[4], dz[4];
  const int bx = grid_base(g.x[o], g.invL[0], g.K[0], &fxr);
  const int by = grid_base(g.y[o], g.invL[1], g.K[1], &fyr);
  const int bz = grid_base(g.z[o], g.invL[2], g.K[2], &fzr);
  bspline4(fxr, wx, dx);
  bspline4(fyr, wy, dy);
  bspline4(fzr, wz, dz);
  int gy = by - iy; if (gy < 0) gy += g.K[1];
  int gz = bz - iz; if (gz < 0) gz += g.K[2];
  const float2* cg = g.cgrid + (size_t)(w >> 1) * g.Ktot + ((size_t)gz * g.K[1] + gy) * g.K[0];
  const bool im = w & 1;
  float pot = 0.f, gxs = 0.f, gys = 0.f, gzs = 0.f;
#pragma unroll
  for (int ix = 0; ix < 4; ++ix) {
    int gx = bx - ix; if (gx < 0) gx += g.K[0];
    const float2 c = cg[gx];
    const float phi = im ? c.y : c.x;
    pot = fmaf(wx[ix], phi, pot);
    gxs = fmaf(dx[ix], phi, gxs);
  }
  const float wyz = wy[iy] * wz[iz];
  float gyz = pot * dy[iy] * wz[iz];
  float gzz = pot * wy[iy] * dz[iz];
  gxs *= wyz;
  pot *= wyz;
  gys = gyz; gzs = gzz;
  for (int off = 1; off < 16; off <<= 1) {
    pot += __shfl_xor(pot, off, 64);
    gxs += __shfl_xor(gxs, off, 64);
    gys += __shfl_xor(gys, off, 64);
    gzs += __shfl_xor(gzs, off, 64);
  }
  if (valid && sub == 0) {
    const float fx = -q * gxs * (float)g.K[0] * g.invLf[0];
    const float fy = -q * gys * (float)g.K[1] * g.invLf[1];
    const float fz = -q * gzs * (float)g.K[2] * g.invLf[2];
    const int where = (w << 20) | a;
    g.fx[o] += to_fixed((double)fx, kForceScale, g.err, kSiteGather, where, g.leg_index);
    g.fy[o] += to_fixed((double)fy, kForceScale, g.err, kSiteGather, where, g.leg_index);
    g.fz[o] += to_fixed((double)fz, kForceScale, g.err, kSiteGather, where, g.leg_index);
  }
  if (ENERGY) {
    double e = (valid && sub == 0) ? 0.5 * (double)q * (double)pot : 0.0;
    const int lane = threadIdx.x & 63;
    const int w0 = __shfl(w, 0, 64);
    const bool same = __ballot(valid && w != w0) == 0ull;
    if (same) {
      e = wave_sum(e);
      if (lane == 0)
        atomicAdd((unsigned long long*)&g.eacc[(size_t)w0 * FELIS_NE + FELIS_E_RECIP],
                  (unsigned long long)to_fixed(e, kEnergyScale, g.err));
    } else if (valid && sub == 0) {
      atomicAdd((unsigned long long*)&g.eacc[(size_t)w * FELIS_NE + FELIS_E_RECIP],
                (unsigned long long)to_fixed(e, kEnergyScale, g.err));
    }
  }
}

inline int blocks_for(long long items, int per) { return (int)((items + per - 1) / per); }

template <int AXIS, int MODE>
void fft_pass(hipStream_t s, const LegDev* d, const LegHost* h, int nl) {
  BlockMap m;
  const int nb = make_map(m, nl, [&](int i) {
    const int inner = (AXIS == 0) ? h[i].K[1] : h[i].K[0];
    const int outer = (AXIS == 2) ? h[i].K[1] : h[i].K[2];
    return h[i].npair * outer * ((inner + kLines - 1) / kLines);
  });
  if (nb) hipLaunchKernelGGL((k_fft<AXIS, MODE>), dim3(nb), dim3(256), 0, s, d, m);
}

}  // namespace

void launch_pme_fft(hipStream_t s, const LegDev* d, const LegHost* h, int nl) {
  fft_pass<0, 2>(s, d, h, nl);
  fft_pass<1, 0>(s, d, h, nl);
  fft_pass<2, 3>(s, d, h, nl);
  fft_pass<1, 1>(s, d, h, nl);
  fft_pass<0, 1>(s, d, h, nl);
}

void launch_pme(hipStream_t s, const LegDev* d, const LegHost* h, int nl, bool energy) {
  BlockMap m;
  int nb = make_map(m, nl, [&](int i) { return blocks_for((long long)h[i].W * h[i].n, 16); });
  if (!nb) return;
  hipLaunchKernelGGL(k_spread, dim3(nb), dim3(256), 0, s, d, m);
  launch_pme_fft(s, d, h, nl);
  if (energy) hipLaunchKernelGGL(k_gather<true>, dim3(nb), dim3(256), 0, s, d, m);
  else hipLaunchKernelGGL(k_gather<false>, dim3(nb), dim3(256), 0, s, d, m);
}

}  // namespace felis
