// PME reciprocal space (smooth PME, Essmann et al. 1995; the paper names PME
// with a 1 nm real-space cutoff in appendix B and prints no PME formulas).
//
// Per window: charges q~ (ligand x lambda_elec) spread with order-4 cardinal
// B-splines, summed in int64 fixed point (order-independent, so the grid is
// bitwise reproducible) by the workgroup that owns each brick of the grid.  Two windows of one leg share a complex grid
// Z = Q_a + i Q_b: with a real, even influence function G the convolution
// IDFT(G DFT(Z)) = phi_a + i phi_b, so one complex FFT pair serves two
// windows.  phi = IDFT_unnormalised(G DFT(Q)), G(m) = KE/(pi V)
// exp(-pi^2 |m|^2/alpha^2)/|m|^2 |b1 b2 b3|^2, G(0) = 0;
// E_rec = 1/2 sum_i q~_i phi(r_i); F_i = -q~_i grad(spline weights) . phi.
//
// FFT: Stockham autosort, radices 8/12/4/2/3/5.  Grids whose x-y planes fit in
// LDS twice (gfx950: 160 KB per workgroup, so up to ~100 x 100 points) are
// transformed by whole planes (x then y in one workgroup), otherwise one
// kernel per axis with 16 lines per workgroup
// ([element][line] layout, coalesced loads for every axis).  The inverse
// transform is conj(DFT(conj(.))).  The z pass fuses forward transform,
// multiplication by G and inverse transform.
#include <algorithm>

#include <climits>

#include "felis_internal.h"

namespace felis {
namespace {

constexpr float kInvSqrtKE = 0.054876864878355476f;   // 1 / sqrt(KE): packed charges carry sqrt(KE)
// Largest LDS a whole-plane x-y workgroup may take; larger planes use one
// pass per axis.  Inside an MD step the transform runs beside the pair
// kernel, which holds most wave slots: a plane workgroup needing most of a
// CU's LDS is then starved, while the per-axis passes (25 KB per workgroup
// on a 96^3 grid) run beside it (42-window complex leg: 5.54 -> 5.41 ms per
// MD step; planes up to 64 KB, e.g. 48^2, keep the whole-plane form)
constexpr size_t kXYLdsCap = 65536;
constexpr int kXYThreads = 512;               // threads per whole-plane workgroup: ~one butterfly each

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 mul_mi(float2 a) { return make_float2(a.y, -a.x); }   // a * (-i)
__device__ __forceinline__ float2 conj2(float2 a) { return make_float2(a.x, -a.y); }

// Quotient and remainder of 0 <= x < 2^22 by a block-uniform d >= 1 through a
// float reciprocal: the estimate is within 0.75 of x / d, so one correction
// in either direction makes it exact.
struct FastDiv {
  int d;
  float inv;
  __device__ explicit FastDiv(int d_) : d(d_), inv(1.0f / (float)d_) {}
  __device__ __forceinline__ int div(int x) const {
    int q = (int)((float)x * inv);               // >= 0
    const int r = x - (int)__umul24((unsigned)q, (unsigned)d);
    q += (r < 0) ? -1 : (r >= d ? 1 : 0);
    return q;
  }
};

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
  } else if (R == 12) {
    // prime-factor form 12 = 3 x 4: inputs j = (4 j1 + 3 j2) mod 12, 3-point
    // transforms over j1, then 4-point transforms over j2, outputs
    // k = (4 k1 + 9 k2) mod 12 (no twiddles between the two)
    float2 a[4][3];
#pragma unroll
    for (int j2 = 0; j2 < 4; ++j2) {
#pragma unroll
      for (int j1 = 0; j1 < 3; ++j1) a[j2][j1] = v[(4 * j1 + 3 * j2) % 12];
      dft<3>(a[j2]);
    }
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) {
      float2 b[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
      dft<4>(b);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) v[(4 * k1 + 9 * k2) % 12] = b[k2];
    }
  } else if (R == 8) {
    // two 4-point transforms of the even and odd elements, then the odd ones
    // turned by w^k, w = exp(-2 pi i / 8)
    float2 e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
    dft<4>(e);
    dft<4>(o);
    const float h = 0.70710678118654752f;               // 1 / sqrt(2)
    const float2 t1 = make_float2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));   // w o1
    const float2 t2 = mul_mi(o[2]);                                                // w^2 o2 = -i o2
    const float2 t3 = make_float2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));  // w^3 o3
    v[0] = cadd(e[0], o[0]); v[4] = csub(e[0], o[0]);
    v[1] = cadd(e[1], t1);   v[5] = csub(e[1], t1);
    v[2] = cadd(e[2], t2);   v[6] = csub(e[2], t2);
    v[3] = cadd(e[3], t3);   v[7] = csub(e[3], t3);
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

// One Stockham stage of radix R over LINES lines (buf[e * LINES + b]).
template <int R, int LINES>
__device__ __forceinline__ void stage(const float2* src, float2* dst, int n, int Ns, const float2* tw) {
  const int nR = n / R;
  const int step = n / (Ns * R);
  const int s_in = nR * LINES, s_out = Ns * LINES;
  const FastDiv dNs(Ns);
  for (int t = threadIdx.x; t < nR * LINES; t += blockDim.x) {
    // element j = t / LINES of line b = t % LINES; j = jq Ns + k
    const int j = t / LINES;
    const int jq = dNs.div(j);
    const int k = j - (int)__umul24((unsigned)jq, (unsigned)Ns);
    const int tk = (int)__umul24((unsigned)k, (unsigned)step);
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      v[r] = src[t + r * s_in];                        // element j + r nR
      if (r) v[r] = cmul(v[r], tw[r * tk]);            // r k step < n
    }
    dft<R>(v);
    const int o = t + (int)__umul24((unsigned)jq, (unsigned)((R - 1) * s_out));   // element jq Ns R + k
#pragma unroll
    for (int r = 0; r < R; ++r) dst[o + r * s_out] = v[r];
  }
}

// The first Stockham stage (Ns = 1, so no twiddles) reading its inputs
// straight from the grid: element e of line b at offs(e, b) (< 0: a line past
// the grid's edge, read as zero), conjugated for an inverse transform.  Used
// for the y and z passes, whose lines are consecutive in x, so consecutive
// threads read consecutive grid points.
template <int R, int LINES, bool CONJ, typename Off>
__device__ __forceinline__ void stage_first_global(const float2* __restrict__ cg, const Off& offs, float2* dst, int n) {
  const int nR = n / R;
  for (int t = threadIdx.x; t < nR * LINES; t += blockDim.x) {
    const int j = t / LINES, b = t - j * LINES;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const long long off = offs(j + r * nR, b);
      const float2 c = off >= 0 ? cg[off] : make_float2(0.f, 0.f);
      v[r] = CONJ ? conj2(c) : c;
    }
    dft<R>(v);
    const int o = t + j * (R - 1) * LINES;
#pragma unroll
    for (int r = 0; r < R; ++r) dst[o + r * LINES] = v[r];
  }
}

// The last Stockham stage of a line set (Ns: the product of the earlier
// radices) writing its outputs straight to the grid: output element
// jq Ns R + k + r Ns of line b goes to offs(e, b) (skipped when < 0),
// conjugated after an inverse transform.
template <int R, int LINES, bool CONJ, typename Off>
__device__ __forceinline__ void stage_last_global(const float2* src, float2* __restrict__ cg, const Off& offs, int n,
                                                  int Ns, const float2* tw) {
  const int nR = n / R;
  const int step = n / (Ns * R);
  const int s_in = nR * LINES;
  const FastDiv dNs(Ns);
  for (int t = threadIdx.x; t < nR * LINES; t += blockDim.x) {
    const int j = t / LINES, b = t - j * LINES;
    const int jq = dNs.div(j);
    const int k = j - (int)__umul24((unsigned)jq, (unsigned)Ns);
    const int tk = (int)__umul24((unsigned)k, (unsigned)step);
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      v[r] = src[t + r * s_in];
      if (r) v[r] = cmul(v[r], tw[r * tk]);
    }
    dft<R>(v);
    const int e0 = jq * Ns * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const long long off = offs(e0 + r * Ns, b);
      if (off >= 0) cg[off] = CONJ ? conj2(v[r]) : v[r];
    }
  }
}

// Forward transform of LINES lines of length n held in src[e * LINES + b],
// stages st0 .. st1 - 1 (Ns0: the product of the radices of the stages done);
// returns the buffer that holds the result.
template <int LINES>
__device__ __forceinline__ float2* fft_lines(float2* src, float2* dst, int n, const int* rad, int nrad, const float2* tw,
                                             int st0 = 0, int Ns0 = 1, int st1 = -1) {
  int Ns = Ns0;
  if (st1 < 0) st1 = nrad;
  for (int st = st0; st < st1; ++st) {
    const int R = rad[st];
    switch (R) {
      case 2: stage<2, LINES>(src, dst, n, Ns, tw); break;
      case 3: stage<3, LINES>(src, dst, n, Ns, tw); break;
      case 4: stage<4, LINES>(src, dst, n, Ns, tw); break;
      case 8: stage<8, LINES>(src, dst, n, Ns, tw); break;
      case 12: stage<12, LINES>(src, dst, n, Ns, tw); break;
      default: stage<5, LINES>(src, dst, n, Ns, tw); break;
    }
    __syncthreads();
    float2* t = src; src = dst; dst = t;
    Ns *= R;
  }
  return src;
}

// MODE: 0 forward, 1 inverse, 2 forward from the int64 grids (x axis),
//       3 forward * G * inverse (z axis)
template <int AXIS, int MODE, int LINES>
__global__ __launch_bounds__(256) void k_fft(const LegDev* legs, BlockMap map, int ukn) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const int Kx = g.K[0], Ky = g.K[1], Kz = g.K[2];
  const int n = g.K[AXIS];
  // lines: x axis -> (z, y-chunk); y axis -> (z, x-chunk); z axis -> (y, x-chunk)
  const int inner = (AXIS == 0) ? Ky : Kx;
  const int outer = (AXIS == 2) ? Ky : Kz;
  const int nch = (inner + LINES - 1) / LINES;
  const int bl = blockIdx.x - map.start[leg];
  const int p = bl / (outer * nch);
  const int rem = bl - p * outer * nch;
  const int o = rem / nch, ch = rem - (rem / nch) * nch;
  if (p >= g.npair) return;
  extern __shared__ float2 smem[];               // two buffers of n * LINES, then n twiddles
  float2* bufA = smem;
  float2* bufB = smem + (size_t)n * LINES;
  float2* tw = bufB + (size_t)n * LINES;
  for (int e = threadIdx.x; e < n; e += blockDim.x) tw[e] = g.tw[AXIS][e];
  const FastDiv dn(n);
  float2* cg = g.cgrid + (size_t)p * g.Ktot;
  const int KxKy = Kx * Ky;
  auto offs = [&](int e, int b) -> long long {
    const int li = ch * LINES + b;
    if (li >= inner) return -1;
    if (AXIS == 0) return (long long)o * KxKy + (long long)li * Kx + e;
    if (AXIS == 1) return (long long)o * KxKy + (long long)e * Kx + li;
    return (long long)e * KxKy + (long long)o * Kx + li;
  };
  float2* res;
  if (AXIS != 0 && MODE != 2) {
    // the first stage reads the grid itself (no staging pass through LDS)
    constexpr bool CJ = MODE == 1;
    switch (g.rad[AXIS][0]) {
      case 2: stage_first_global<2, LINES, CJ>(cg, offs, bufA, n); break;
      case 3: stage_first_global<3, LINES, CJ>(cg, offs, bufA, n); break;
      case 4: stage_first_global<4, LINES, CJ>(cg, offs, bufA, n); break;
      case 8: stage_first_global<8, LINES, CJ>(cg, offs, bufA, n); break;
      case 12: stage_first_global<12, LINES, CJ>(cg, offs, bufA, n); break;
      default: stage_first_global<5, LINES, CJ>(cg, offs, bufA, n); break;
    }
    __syncthreads();
    const int nrad = g.nrad[AXIS];
    if (MODE != 3 && nrad >= 2) {
      // the middle stages in LDS, the last one straight to the grid
      res = fft_lines<LINES>(bufA, bufB, n, g.rad[AXIS], nrad, tw, 1, g.rad[AXIS][0], nrad - 1);
      int Ns = 1;
      for (int st = 0; st < nrad - 1; ++st) Ns *= g.rad[AXIS][st];
      constexpr bool CO = MODE == 1;
      switch (g.rad[AXIS][nrad - 1]) {
        case 2: stage_last_global<2, LINES, CO>(res, cg, offs, n, Ns, tw); break;
        case 3: stage_last_global<3, LINES, CO>(res, cg, offs, n, Ns, tw); break;
        case 4: stage_last_global<4, LINES, CO>(res, cg, offs, n, Ns, tw); break;
        case 8: stage_last_global<8, LINES, CO>(res, cg, offs, n, Ns, tw); break;
        case 12: stage_last_global<12, LINES, CO>(res, cg, offs, n, Ns, tw); break;
        default: stage_last_global<5, LINES, CO>(res, cg, offs, n, Ns, tw); break;
      }
      return;
    }
    res = fft_lines<LINES>(bufA, bufB, n, g.rad[AXIS], nrad, tw, 1, g.rad[AXIS][0]);
  } else {
  for (int idx = threadIdx.x; idx < n * LINES; idx += blockDim.x) {
    int e, b;
    if (AXIS == 0) { b = dn.div(idx); e = idx - b * n; } else { e = idx / LINES; b = idx - e * LINES; }
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
    bufA[e * LINES + b] = v;
  }
  __syncthreads();
  res = fft_lines<LINES>(bufA, bufB, n, g.rad[AXIS], g.nrad[AXIS], tw);
  }
  if (MODE == 3) {
    // multiply by G(kx, ky, kz): element e = kz of line (ky = o, kx = ch*LINES + b),
    // in the box of the grid's window (u_kn: of its frame)
    const BoxW& B = ukn ? g.ubox[ukn == 1 ? 2 * p : p] : g.box[g.pack ? 2 * p : p];
    const float a2 = g.alpha * g.alpha;
    for (int idx = threadIdx.x; idx < n * LINES; idx += blockDim.x) {
      const int e = idx / LINES, b = idx - e * LINES;
      const int kx = ch * LINES + b, ky = o, kz = e;
      float G = 0.f;
      if (kx < Kx) {
        const float mx = (float)(kx <= Kx / 2 ? kx : kx - Kx) * B.invLf[0];
        const float my = (float)(ky <= Ky / 2 ? ky : ky - Ky) * B.invLf[1];
        const float mz = (float)(kz <= Kz / 2 ? kz : kz - Kz) * B.invLf[2];
        const float m2 = mx * mx + my * my + mz * mz;
        if (m2 > 0.f)
          G = B.pme_pref * __expf(-9.8696044010893586f * m2 / a2) / m2 * g.bmod[0][kx] * g.bmod[1][ky] *
              g.bmod[2][kz];
      }
      const float2 v = res[idx];
      res[idx] = conj2(make_float2(v.x * G, v.y * G));     // conj for the inverse pass
    }
    __syncthreads();
    float2* other = (res == bufA) ? bufB : bufA;
    const int nrad = g.nrad[AXIS];
    if (AXIS != 0) {
      // the inverse transform's last stage straight to the grid
      res = fft_lines<LINES>(res, other, n, g.rad[AXIS], nrad, tw, 0, 1, nrad - 1);
      int Ns = 1;
      for (int st = 0; st < nrad - 1; ++st) Ns *= g.rad[AXIS][st];
      switch (g.rad[AXIS][nrad - 1]) {
        case 2: stage_last_global<2, LINES, true>(res, cg, offs, n, Ns, tw); break;
        case 3: stage_last_global<3, LINES, true>(res, cg, offs, n, Ns, tw); break;
        case 4: stage_last_global<4, LINES, true>(res, cg, offs, n, Ns, tw); break;
        case 8: stage_last_global<8, LINES, true>(res, cg, offs, n, Ns, tw); break;
        case 12: stage_last_global<12, LINES, true>(res, cg, offs, n, Ns, tw); break;
        default: stage_last_global<5, LINES, true>(res, cg, offs, n, Ns, tw); break;
      }
      return;
    }
    res = fft_lines<LINES>(res, other, n, g.rad[AXIS], nrad, tw);
  }
  for (int idx = threadIdx.x; idx < n * LINES; idx += blockDim.x) {
    int e, b;
    if (AXIS == 0) { b = dn.div(idx); e = idx - b * n; } else { e = idx / LINES; b = idx - e * LINES; }
    const long long off = offs(e, b);
    if (off < 0) continue;
    float2 v = res[e * LINES + b];
    if (MODE == 1 || MODE == 3) v = conj2(v);
    cg[off] = v;
  }
}

// One Stockham stage of radix R over nl lines held as buf[e * nl + b].
template <int R>
__device__ __forceinline__ void stage_nl(const float2* src, float2* dst, int n, int Ns, const FastDiv& dnl,
                                         const float2* tw) {
  const int nl = dnl.d;
  const int nR = n / R;
  const int step = n / (Ns * R);
  const int s_in = nR * nl, s_out = Ns * nl;
  const FastDiv dNs(Ns);
  for (int t = threadIdx.x; t < nR * nl; t += blockDim.x) {
    // element j = t / nl of line t % nl; j = jq Ns + k
    const int j = dnl.div(t);
    const int jq = dNs.div(j);
    const int k = j - (int)__umul24((unsigned)jq, (unsigned)Ns);
    const int tk = (int)__umul24((unsigned)k, (unsigned)step);
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      v[r] = src[t + r * s_in];
      if (r) v[r] = cmul(v[r], tw[r * tk]);
    }
    dft<R>(v);
    const int o = t + (int)__umul24((unsigned)jq, (unsigned)((R - 1) * s_out));
#pragma unroll
    for (int r = 0; r < R; ++r) dst[o + r * s_out] = v[r];
  }
}

__device__ __forceinline__ float2* fft_lines_nl(float2* src, float2* dst, int n, const FastDiv& dnl, const int* rad, int nrad,
                                const float2* tw) {
  int Ns = 1;
  for (int st = 0; st < nrad; ++st) {
    const int R = rad[st];
    switch (R) {
      case 2: stage_nl<2>(src, dst, n, Ns, dnl, tw); break;
      case 3: stage_nl<3>(src, dst, n, Ns, dnl, tw); break;
      case 4: stage_nl<4>(src, dst, n, Ns, dnl, tw); break;
      case 8: stage_nl<8>(src, dst, n, Ns, dnl, tw); break;
      case 12: stage_nl<12>(src, dst, n, Ns, dnl, tw); break;
      default: stage_nl<5>(src, dst, n, Ns, dnl, tw); break;
    }
    __syncthreads();
    float2* t = src; src = dst; dst = t;
    Ns *= R;
  }
  return src;
}

// One workgroup per (window pair, z plane): 2D transform of the Kx x Ky
// plane in LDS -- x lines, transpose, y lines -- so a forward (or inverse)
// transform over x and y reads and writes the grid once.  INVERSE uses
// conj(DFT(conj(.))).  The line-interleaved buffers carry one extra (zero)
// line, Ky + 1 for the x lines and Kx + 1 for the y lines: with an even line
// count the scatter into line order and the transpose hit one LDS bank with
// every lane (96 lines: a stride of 192 dwords).
template <bool INVERSE>
__global__ __launch_bounds__(kXYThreads) void k_fft_xy(const LegDev* legs, BlockMap map) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const int Kx = g.K[0], Ky = g.K[1], Kz = g.K[2];
  const int bl = blockIdx.x - map.start[leg];
  const int p = bl / Kz, z = bl - p * Kz;
  if (p >= g.npair) return;
  extern __shared__ float2 smem[];                // A, B: one padded plane each; then the x and y twiddles
  const int np = Kx * Ky;
  const int nlx = Ky + 1, nly = Kx + 1;
  const int nbuf = np + max(Kx, Ky);
  float2* A = smem;
  float2* B = smem + nbuf;
  float2* twx = B + nbuf;
  float2* twy = twx + Kx;
  float2* cg = g.cgrid + (size_t)p * g.Ktot + (size_t)z * np;
  const FastDiv dKx(Kx), dKy(Ky), dlx(nlx), dly(nly);
  for (int e = threadIdx.x; e < Kx; e += blockDim.x) twx[e] = g.tw[0][e];
  for (int e = threadIdx.x; e < Ky; e += blockDim.x) twy[e] = g.tw[1][e];
  for (int x = threadIdx.x; x < Kx; x += blockDim.x) A[x * nlx + Ky] = make_float2(0.f, 0.f);
  for (int idx = threadIdx.x; idx < np; idx += blockDim.x) {       // [x][y]: lines along x
    const int y = dKx.div(idx), x = idx - y * Kx;
    float2 v = cg[idx];
    if (INVERSE) v = conj2(v);
    A[x * nlx + y] = v;
  }
  __syncthreads();
  float2* r = fft_lines_nl(A, B, Kx, dlx, g.rad[0], g.nrad[0], twx);
  float2* o = (r == A) ? B : A;
  for (int y = threadIdx.x; y < Ky; y += blockDim.x) o[y * nly + Kx] = make_float2(0.f, 0.f);
  for (int idx = threadIdx.x; idx < np; idx += blockDim.x) {       // -> [y][x]: lines along y
    const int x = dKy.div(idx), y = idx - x * Ky;
    o[y * nly + x] = r[x * nlx + y];
  }
  __syncthreads();
  r = fft_lines_nl(o, r, Ky, dly, g.rad[1], g.nrad[1], twy);
  for (int idx = threadIdx.x; idx < np; idx += blockDim.x) {
    const int y = dKx.div(idx), x = idx - y * Kx;
    float2 v = r[y * nly + x];                                      // [y][x] = grid order
    if (INVERSE) v = conj2(v);
    cg[idx] = v;
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


// spreading brick edges in grid points (x fastest).  16 x 8 x 8: against
// 8 x 8 x 8 the halo a brick must scan (3 grid spacings and the cell margin
// on every side) weighs less per owned point; reciprocal space alone on the
// 96^3 grid of 42 windows 1.73 -> 1.61 ms
constexpr int kBX = 16, kBY = 8, kBZ = 8;
constexpr int kBrickPts = kBX * kBY * kBZ;
// spreading tile: int32 fixed point, 2^26 units per e.  A grid point's charge
// stays far inside +-32 e (an atom adds at most |q| (2/3)^3), so the integer
// sum modulo 2^32 is exact and independent of the order of the adds; one
// unit (1.5e-8 e) is far below the FP32 FFT's own rounding
constexpr float kTileScale = 67108864.0f;
constexpr int kSpreadCellOf = 1024;            // candidates per table window in spreading
constexpr int kSpreadChunk = 128;              // atoms per compact task list in spreading

// Grid points of axis d that an atom with base index b touches, as a 4-bit
// mask over the stencil offsets (point b - k, k = 0..3, periodic) that fall in
// [P0, P1).
__device__ __forceinline__ unsigned brick_mask(int b, int K, int P0, int P1) {
  unsigned m = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    int p = b - k;
    if (p < 0) p += K;
    if (p >= P0 && p < P1) m |= 1u << k;
  }
  return m;
}

// One block per (window, brick of grid points, kBX x kBY x kBZ): the block owns its
// window's component of the brick (the real part of the pair's complex grid
// for the even window, the imaginary part for the odd one).  Candidate atoms
// come from the fine cells of the window's last list build that can hold an
// atom whose stencil reaches the brick (the brick's extent plus 3 grid
// spacings on the upper side, widened by skin/2 for the drift since that
// build); each contributing atom adds its stencil points inside the brick to
// an int32 fixed-point tile in LDS (integer sums: the tile does not depend on
// the order of the adds), and the block writes its component of the brick
// once, with plain stores.
__global__ __launch_bounds__(256) void k_spread(const LegDev* legs, BlockMap map) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  // grid sizes in scalar registers (otherwise reloaded from memory inside the loops)
  const int K[3] = {__builtin_amdgcn_readfirstlane(g.K[0]), __builtin_amdgcn_readfirstlane(g.K[1]),
                    __builtin_amdgcn_readfirstlane(g.K[2])};
  const int tid = threadIdx.x;
  const int nbx = (K[0] + kBX - 1) / kBX, nby = (K[1] + kBY - 1) / kBY;
  const int nbz = (K[2] + kBZ - 1) / kBZ;
  const int bl = blockIdx.x - map.start[leg];
  const int per = nbx * nby * nbz;
  const int w = bl / per;
  int r = bl - w * per;
  const int bz = r / (nbx * nby);
  r -= bz * nbx * nby;
  const int by = r / nbx, bx = r - by * nbx;
  const int P0[3] = {bx * kBX, by * kBY, bz * kBZ};
  const int P1[3] = {min(P0[0] + kBX, K[0]), min(P0[1] + kBY, K[1]), min(P0[2] + kBZ, K[2])};

  __shared__ int tile[kBrickPts];
  __shared__ int s_start[256], s_pre[256], s_wsum[4];
  __shared__ unsigned char s_cellof[kSpreadCellOf];   // candidate -> cell of the round
  __shared__ int s_n;
  __shared__ float s_q[256], s_w[256][12];
  __shared__ int s_b[256];                       // packed bases (7 bits per axis)
  __shared__ unsigned s_m[256];
  __shared__ unsigned short s_task[16 * kSpreadChunk];  // (atom << 4 | ix << 2 | iy) of the chunk
  __shared__ int s_tw[4];
  for (int e = tid; e < kBrickPts; e += 256) tile[e] = 0;
  if (tid == 0) s_n = 0;

  // candidate fine cells per axis
  const int nc = 1 << g.nbits;
  const float margin = sqrtf(g.skin_half2) + 0.05f;
  int c0[3], nspan[3];
  for (int d = 0; d < 3; ++d) {
    const float Lc = g.box[w].Lf[d] / (float)nc, hgrid = g.box[w].Lf[d] / (float)K[d];
    const int a0 = (int)floorf(((float)P0[d] * hgrid - margin) / Lc);
    const int a1 = (int)floorf(((float)(P1[d] + 3) * hgrid + margin) / Lc);
    const bool full = a1 - a0 + 1 >= nc;
    c0[d] = full ? 0 : a0;
    nspan[d] = full ? nc : a1 - a0 + 1;
  }
  const int ncells = nspan[0] * nspan[1] * nspan[2];
  const int n12 = nspan[1] * nspan[2];
  const float inv12 = 1.0f / (float)n12, inv2 = 1.0f / (float)nspan[2];
  const int wave = tid >> 6, lane = tid & 63;
  const int* cst = g.cellstart + (size_t)w * (g.ncell + 1);
  const float4* __restrict__ gs = g.gsten + (size_t)w * g.npad;
  const float4* __restrict__ xq = g.xyzq + (size_t)w * g.npad;
  __syncthreads();
  for (int cb = 0; cb < ncells; cb += 256) {
    const int ci = cb + tid;
    int s0 = 0, cnt = 0;
    if (ci < ncells) {
      // ci -> cell (float-reciprocal quotients, one correction each); a cell
      // coordinate lies in (-nc, 2nc), so one wrap suffices
      int q0 = (int)((float)ci * inv12);
      q0 += (ci - q0 * n12 < 0) ? -1 : (ci - q0 * n12 >= n12 ? 1 : 0);
      const int rem = ci - q0 * n12;
      int q1 = (int)((float)rem * inv2);
      q1 += (rem - q1 * nspan[2] < 0) ? -1 : (rem - q1 * nspan[2] >= nspan[2] ? 1 : 0);
      const int C[3] = {c0[0] + q0, c0[1] + q1, c0[2] + rem - q1 * nspan[2]};
      auto wrapc = [nc](int c) { return c < 0 ? c + nc : (c >= nc ? c - nc : c); };
      const unsigned cc = g.hcell[(wrapc(C[0]) * nc + wrapc(C[1])) * nc + wrapc(C[2])];
      s0 = cst[cc];
      cnt = cst[cc + 1] - s0;
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
    const int total = s_wsum[0] + s_wsum[1] + s_wsum[2] + s_wsum[3];
    const int pre_t = woff + inc - cnt;
    s_pre[tid] = pre_t;
    for (int T0 = 0; T0 < total; T0 += kSpreadCellOf) {
      {
        const int b0 = max(pre_t, T0), b1 = min(pre_t + cnt, T0 + kSpreadCellOf);
        for (int q = b0; q < b1; ++q) s_cellof[q - T0] = (unsigned char)tid;
      }
      __syncthreads();
      const int T1 = min(total, T0 + kSpreadCellOf);
      for (int t0 = T0; t0 < T1; t0 += 256) {
        const int t = t0 + tid;
        if (t < T1) {
          const int l = s_cellof[t - T0];
          const int s = s_start[l] + (t - s_pre[l]);
          const float4 st = gs[s];               // stencil offsets and bases (from the pack)
          int bb[3];
          unpack_bases(st.w, bb);
          const int b0 = bb[0], b1 = bb[1], b2 = bb[2];
          const float fr[3] = {st.x, st.y, st.z};
          const unsigned mx = brick_mask(b0, K[0], P0[0], P1[0]);
          const unsigned my = brick_mask(b1, K[1], P0[1], P1[1]);
          const unsigned mz = brick_mask(b2, K[2], P0[2], P1[2]);
          if (mx && my && mz) {
            const float qs = xq[s].w * kInvSqrtKE;   // the window's charge (packed times sqrt(KE))
            const int k = atomicAdd(&s_n, 1);
            s_q[k] = qs;
            bspline4(fr[0], &s_w[k][0], nullptr);
            bspline4(fr[1], &s_w[k][4], nullptr);
            bspline4(fr[2], &s_w[k][8], nullptr);
            s_b[k] = __float_as_int(st.w);
            s_m[k] = mx | (my << 4) | (mz << 8);
          }
        }
        __syncthreads();
        const int na = s_n;
        // compact task lists, kSpreadChunk atoms at a time: one (atom, ix, iy)
        // per stencil column inside the brick (about half of the 16 columns
        // of an atom near a brick face)
        for (int a0 = 0; a0 < na; a0 += kSpreadChunk) {
          {
            const unsigned m = (tid < kSpreadChunk && a0 + tid < na) ? s_m[a0 + tid] : 0u;
            const int nt = __popc(m & 0xFu) * __popc((m >> 4) & 0xFu);
            int inc = nt;
            for (int k = 1; k < 64; k <<= 1) {
              const int v = __shfl_up(inc, k, 64);
              if (lane >= k) inc += v;
            }
            if (lane == 63) s_tw[wave] = inc;
            __syncthreads();
            int pos = inc - nt;
            for (int k = 0; k < wave; ++k) pos += s_tw[k];
            for (int ix = 0; ix < 4; ++ix) {
              if (!((m >> ix) & 1u)) continue;
              for (int iy = 0; iy < 4; ++iy)
                if ((m >> (4 + iy)) & 1u) s_task[pos++] = (unsigned short)((tid << 4) | (ix << 2) | iy);
            }
          }
          __syncthreads();
          const int ntask = s_tw[0] + s_tw[1] + s_tw[2] + s_tw[3];
          for (int task = tid; task < ntask; task += 256) {   // (atom, ix, iy), loop over iz
            const unsigned word = s_task[task];
            const int k = a0 + (int)(word >> 4), ix = (int)((word >> 2) & 3u), iy = (int)(word & 3u);
            const unsigned m = s_m[k];
            int bb[3];
            unpack_bases(__int_as_float(s_b[k]), bb);
            int px = bb[0] - ix; if (px < 0) px += K[0];
            int py = bb[1] - iy; if (py < 0) py += K[1];
            const float qxy = s_q[k] * s_w[k][ix] * s_w[k][4 + iy] * kTileScale;
            const int row = ((py - P0[1]) * kBX + (px - P0[0]));
#pragma unroll
            for (int iz = 0; iz < 4; ++iz) {
              if (!((m >> (8 + iz)) & 1u)) continue;
              int pz = bb[2] - iz; if (pz < 0) pz += K[2];
              const int v = (int)rintf(qxy * s_w[k][8 + iz]);
              atomicAdd(&tile[(pz - P0[2]) * (kBX * kBY) + row], v);
            }
          }
          __syncthreads();                          // s_task and s_tw are rewritten next
        }
        __syncthreads();
        if (tid == 0) s_n = 0;
        __syncthreads();
      }
    }
    __syncthreads();                              // the round's tables are rewritten next
  }
  // this window's component of the pair's complex grid; an unpaired last
  // window, or a window with a grid of its own, also clears the imaginary part
  float* cg = reinterpret_cast<float*>(g.cgrid + (size_t)(g.pack ? w >> 1 : w) * g.Ktot);
  const int comp = g.pack ? (w & 1) : 0;
  const bool clear_im = comp == 0 && (!g.pack || w + 1 >= g.W);
  for (int e = tid; e < kBrickPts; e += 256) {
    const int lx = e % kBX, ly = (e / kBX) % kBY, lz = e / (kBX * kBY);
    const int x = P0[0] + lx, y = P0[1] + ly, z = P0[2] + lz;
    if (x >= P1[0] || y >= P1[1] || z >= P1[2]) continue;
    const size_t off = ((size_t)z * K[1] + y) * K[0] + x;
    cg[2 * off + comp] = (float)tile[e] * (1.0f / kTileScale);
    if (clear_im) cg[2 * off + 1] = 0.f;
  }
}

// Each gather block stages its 64 atoms' stencil region of the grid in LDS
// (rows read contiguously) instead of 64 scattered reads per atom; the forces
// are bitwise the same (42-window complex leg: 5.40 -> 5.34 ms per MD step)
constexpr int kGatherTile = 4096;              // grid points staged per block (16 KB)

// STEP: store the force in frx/fry/frz (the integrator adds it to the
// real-space force) instead of adding it to fx/fy/fz
template <bool ENERGY, bool STEP>
__global__ __launch_bounds__(256) void k_gather(const LegDev* legs, BlockMap map) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  // grid sizes in scalar registers (otherwise reloaded from memory inside the loops)
  const int K[3] = {__builtin_amdgcn_readfirstlane(g.K[0]), __builtin_amdgcn_readfirstlane(g.K[1]),
                    __builtin_amdgcn_readfirstlane(g.K[2])};
  // atoms in the neighbour-list sort order (spatially coherent); 4 lanes per
  // atom, lane iz sums the 16 stencil points of plane z = bz - iz
  // blocks never straddle two windows: the block's 64 atoms share one grid
  const int bpw = (g.npad + 63) >> 6;
  const int blk = blockIdx.x - map.start[leg];
  const int w = blk / bpw;
  const int s0 = (blk - w * bpw) * 64;
  if (s0 >= g.n) return;                        // padding only (uniform over the block)
  const int slot = s0 + (threadIdx.x >> 2);
  const int lc = w * g.npad + min(slot, g.npad - 1);
  const int ap = g.perm[lc];
  const bool valid = slot < g.npad && ap >= 0;
  const int a = ap >= 0 ? ap : 0;
  const int iz = threadIdx.x & 3;
  const size_t o = (size_t)w * g.n + a;
  const float q = g.xyzq[lc].w * kInvSqrtKE;    // the window's charge (packed times sqrt(KE))
  const float4 st = g.gsten[lc];               // stencil offsets and bases (from the pack)
  int bb[3];
  unpack_bases(st.w, bb);
  int bx = bb[0], by = bb[1], bz = bb[2];
  float wx[4], wy[4], wz[4], dx[4], dy[4], dz[4];
  bspline4(st.x, wx, dx);
  bspline4(st.y, wy, dy);
  bspline4(st.z, wz, dz);
  const bool im = g.pack && (w & 1);
  float p0 = 0.f, px = 0.f, py = 0.f;          // sum w phi, sum dwx phi, sum dwy phi over the plane
  // Stage the block's stencil region of the window's grid component in LDS
  // (rows read contiguously), then interpolate from LDS.  Bases are unwrapped
  // to the periodic image nearest the block's first atom's; a region larger
  // than the tile (atoms spread over the box) reads the grid directly.
  __shared__ float s_tile[kGatherTile];
  __shared__ int s_red[4][6];
  __shared__ int s_ref[3];
  if (threadIdx.x == 0) {
    int r[3];
    unpack_bases(g.gsten[(size_t)w * g.npad + s0].w, r);
    s_ref[0] = r[0]; s_ref[1] = r[1]; s_ref[2] = r[2];
  }
  __syncthreads();
  {
    const int ref[3] = {s_ref[0], s_ref[1], s_ref[2]};
    int* bp[3] = {&bx, &by, &bz};
    for (int d = 0; d < 3; ++d) {
      const int df = *bp[d] - ref[d];
      if (2 * df > K[d]) *bp[d] -= K[d];
      else if (2 * df < -K[d]) *bp[d] += K[d];
    }
  }
  int mn[3] = {valid ? bx : INT_MAX, valid ? by : INT_MAX, valid ? bz : INT_MAX};
  int mx[3] = {valid ? bx : INT_MIN, valid ? by : INT_MIN, valid ? bz : INT_MIN};
  for (int off = 1; off < 64; off <<= 1)
    for (int d = 0; d < 3; ++d) {
      mn[d] = min(mn[d], __shfl_xor(mn[d], off, 64));
      mx[d] = max(mx[d], __shfl_xor(mx[d], off, 64));
    }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
    for (int d = 0; d < 3; ++d) { s_red[wave][d] = mn[d]; s_red[wave][3 + d] = mx[d]; }
  __syncthreads();
  int lo[3], nd[3];
  for (int d = 0; d < 3; ++d) {
    int a0 = s_red[0][d], a1 = s_red[0][3 + d];
    for (int k = 1; k < 4; ++k) { a0 = min(a0, s_red[k][d]); a1 = max(a1, s_red[k][3 + d]); }
    lo[d] = a0 - 3;
    nd[d] = a1 - lo[d] + 1;
  }
  const int vol = nd[0] * nd[1] * nd[2];     // block-uniform (the first atom is valid)
  if (!valid) { bx = lo[0] + 3; by = lo[1] + 3; bz = lo[2] + 3; }   // in-tile reads, results unused
  const float* comp = reinterpret_cast<const float*>(g.cgrid + (size_t)(g.pack ? w >> 1 : w) * g.Ktot) + (im ? 1 : 0);
  if (vol <= kGatherTile) {
    for (int e = threadIdx.x; e < vol; e += 256) {
      const int x = e % nd[0], yz = e / nd[0];
      const int y = yz % nd[1], z = yz / nd[1];
      int gx = lo[0] + x, gy = lo[1] + y, gz = lo[2] + z;
      gx += gx < 0 ? K[0] : (gx >= K[0] ? -K[0] : 0);
      gy += gy < 0 ? K[1] : (gy >= K[1] ? -K[1] : 0);
      gz += gz < 0 ? K[2] : (gz >= K[2] ? -K[2] : 0);
      s_tile[e] = comp[2 * (((size_t)gz * K[1] + gy) * K[0] + gx)];
    }
    __syncthreads();
    const int zb = (bz - iz - lo[2]) * nd[1];
#pragma unroll
    for (int iy = 0; iy < 4; ++iy) {
      const float* row = s_tile + (zb + by - iy - lo[1]) * nd[0] + (bx - lo[0]);
      float s0v = 0.f, s1 = 0.f;
#pragma unroll
      for (int ix = 0; ix < 4; ++ix) {
        const float phi = row[-ix];
        s0v = fmaf(wx[ix], phi, s0v);
        s1 = fmaf(dx[ix], phi, s1);
      }
      p0 = fmaf(wy[iy], s0v, p0);
      px = fmaf(wy[iy], s1, px);
      py = fmaf(dy[iy], s0v, py);
    }
  } else {
    // wrap the unwrapped bases back into the grid and read it directly
    bx += bx < 0 ? K[0] : (bx >= K[0] ? -K[0] : 0);
    by += by < 0 ? K[1] : (by >= K[1] ? -K[1] : 0);
    bz += bz < 0 ? K[2] : (bz >= K[2] ? -K[2] : 0);
    int gz = bz - iz; if (gz < 0) gz += K[2];
    int gxv[4];
#pragma unroll
    for (int ix = 0; ix < 4; ++ix) { gxv[ix] = bx - ix; if (gxv[ix] < 0) gxv[ix] += K[0]; }
    const float2* plane = g.cgrid + (size_t)(g.pack ? w >> 1 : w) * g.Ktot + (size_t)gz * K[1] * K[0];
#pragma unroll
    for (int iy = 0; iy < 4; ++iy) {
      int gy = by - iy; if (gy < 0) gy += K[1];
      const float2* row = plane + (size_t)gy * K[0];
      float s0v = 0.f, s1 = 0.f;
#pragma unroll
      for (int ix = 0; ix < 4; ++ix) {
        const float2 c = row[gxv[ix]];
        const float phi = im ? c.y : c.x;
        s0v = fmaf(wx[ix], phi, s0v);
        s1 = fmaf(dx[ix], phi, s1);
      }
      p0 = fmaf(wy[iy], s0v, p0);
      px = fmaf(wy[iy], s1, px);
      py = fmaf(dy[iy], s0v, py);
    }
  }
  float pot = p0 * wz[iz], gxs = px * wz[iz], gys = py * wz[iz], gzs = p0 * dz[iz];
  for (int off = 1; off < 4; off <<= 1) {
    pot += __shfl_xor(pot, off, 64);
    gxs += __shfl_xor(gxs, off, 64);
    gys += __shfl_xor(gys, off, 64);
    gzs += __shfl_xor(gzs, off, 64);
  }
  const int sub = iz;
  if (valid && sub == 0) {
    const BoxW& B = g.box[w];
    const float fx = -q * gxs * (float)K[0] * B.invLf[0];
    const float fy = -q * gys * (float)K[1] * B.invLf[1];
    const float fz = -q * gzs * (float)K[2] * B.invLf[2];
    const int where = (w << 20) | a;
    const long long ix = to_fixed((double)fx, kForceScale, g.err, kSiteGather, where, g.leg_index);
    const long long iy = to_fixed((double)fy, kForceScale, g.err, kSiteGather, where, g.leg_index);
    const long long iz = to_fixed((double)fz, kForceScale, g.err, kSiteGather, where, g.leg_index);
    if (STEP && g.plain) {
      // the plain form: FP64 atomics into the leg's FP64 sums
      const size_t wn = (size_t)g.W * g.n;
      unsafeAtomicAdd(&g.fd[o], (double)fx);
      unsafeAtomicAdd(&g.fd[wn + o], (double)fy);
      unsafeAtomicAdd(&g.fd[2 * wn + o], (double)fz);
    } else if (STEP) {
      g.frx[o] = ix; g.fry[o] = iy; g.frz[o] = iz;
    } else {
      // one writer per atom; atomics without a return value let the wave
      // retire without waiting for the read-modify-write
      atomicAdd((unsigned long long*)&g.fx[o], (unsigned long long)ix);
      atomicAdd((unsigned long long*)&g.fy[o], (unsigned long long)iy);
      atomicAdd((unsigned long long*)&g.fz[o], (unsigned long long)iz);
    }
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

template <int AXIS, int MODE, int LINES>
void fft_launch(hipStream_t s, const LegDev* d, const LegHost* h, int nl, int ukn) {
  BlockMap m;
  int nmax = 0;
  const int nb = make_map(m, nl, [&](int i) {
    const int inner = (AXIS == 0) ? h[i].K[1] : h[i].K[0];
    const int outer = (AXIS == 2) ? h[i].K[1] : h[i].K[2];
    nmax = std::max(nmax, h[i].K[AXIS]);
    return h[i].npair * outer * ((inner + LINES - 1) / LINES);
  });
  const size_t lds = (2 * (size_t)nmax * LINES + nmax) * sizeof(float2);
  if (lds > 65536) {
    // above 64 KB a kernel must opt in (128-point lines of 32: 66.5 KB);
    // once per instantiation, within the device's per-workgroup limit
    static const bool opted = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft<AXIS, MODE, LINES>),
                                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                                  (int)(2 * 128 * LINES + 128) * (int)sizeof(float2)) == hipSuccess;
    if (!opted) (void)hipGetLastError();
  }
  if (nb) hipLaunchKernelGGL((k_fft<AXIS, MODE, LINES>), dim3(nb), dim3(256), lds, s, d, m, ukn);
}

// 32 lines per workgroup read and write 256-byte runs on the y and z passes
// (42-window complex leg: 5.36 -> 5.33 ms per MD step against 16) but take
// 50 KB of LDS and halve the workgroups: launches that would have fewer than
// kFftWideBlocks workgroups at 32 lines (a single window) and the u_kn
// transforms, which run alone, keep 16 (one-window legs 637 vs 594
// ns*windows/day, u_kn 26,800 vs 23,900 frames/s with 32)
constexpr long long kFftWideBlocks = 4096;

template <int AXIS, int MODE>
void fft_pass(hipStream_t s, const LegDev* d, const LegHost* h, int nl, int ukn, bool allow_wide) {
  long long wide = 0;
  for (int i = 0; i < nl; ++i) {
    const int inner = (AXIS == 0) ? h[i].K[1] : h[i].K[0];
    const int outer = (AXIS == 2) ? h[i].K[1] : h[i].K[2];
    wide += (long long)h[i].npair * outer * ((inner + 31) / 32);
  }
  if (allow_wide && wide >= kFftWideBlocks) fft_launch<AXIS, MODE, 32>(s, d, h, nl, ukn);
  else fft_launch<AXIS, MODE, 16>(s, d, h, nl, ukn);
}

}  // namespace

// Largest dynamic LDS a whole-plane workgroup may take on this device (gfx950:
// 160 KB per workgroup), with the kernels opted in above 64 KB; 0 when the
// device or the runtime refuses.
size_t plane_lds_limit() {
  static size_t limit = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
      return (size_t)0;
    const size_t lim = (size_t)v;
    if (lim > 65536 &&
        (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_xy<false>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim) != hipSuccess ||
         hipFuncSetAttribute(reinterpret_cast<const void*>(&k_fft_xy<true>),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim) != hipSuccess)) {
      (void)hipGetLastError();
      return (size_t)65536;
    }
    return lim;
  }();
  return limit;
}

void launch_pme_fft(hipStream_t s, const LegDev* d, const LegHost* h, int nl, int ukn_mode) {
  const bool wide = ukn_mode == 0;              // MD and force passes; u_kn keeps 16 lines
  const bool from_int64 = ukn_mode != 0;
  int plane = 0, kxy = 0;
  for (int i = 0; i < nl; ++i) {
    plane = std::max(plane, h[i].K[0] * h[i].K[1] + std::max(h[i].K[0], h[i].K[1]));   // one padded buffer
    kxy = std::max(kxy, h[i].K[0] + h[i].K[1]);
  }
  const size_t lds = (2 * (size_t)plane + kxy) * sizeof(float2);
  if (!from_int64 && lds <= std::min(plane_lds_limit(), kXYLdsCap)) {   // whole x-y planes in LDS
    BlockMap m;
    const int nb = make_map(m, nl, [&](int i) { return h[i].npair * h[i].K[2]; });
    if (nb) hipLaunchKernelGGL(k_fft_xy<false>, dim3(nb), dim3(kXYThreads), lds, s, d, m);
    fft_pass<2, 3>(s, d, h, nl, ukn_mode, wide);
    if (nb) hipLaunchKernelGGL(k_fft_xy<true>, dim3(nb), dim3(kXYThreads), lds, s, d, m);
    return;
  }
  if (from_int64) fft_pass<0, 2>(s, d, h, nl, 0, wide);
  else fft_pass<0, 0>(s, d, h, nl, 0, wide);
  fft_pass<1, 0>(s, d, h, nl, 0, wide);
  fft_pass<2, 3>(s, d, h, nl, ukn_mode, wide);
  fft_pass<1, 1>(s, d, h, nl, 0, wide);
  fft_pass<0, 1>(s, d, h, nl, 0, wide);
}

void launch_pme(hipStream_t s, const LegDev* d, const LegHost* h, int nl, bool energy, bool step_forces) {
  BlockMap m;
  int nb = make_map(m, nl, [&](int i) {
    const int nbr = ((h[i].K[0] + kBX - 1) / kBX) * ((h[i].K[1] + kBY - 1) / kBY) * ((h[i].K[2] + kBZ - 1) / kBZ);
    return h[i].W * nbr;
  });
  if (!nb) return;
  hipLaunchKernelGGL(k_spread, dim3(nb), dim3(256), 0, s, d, m);
  launch_pme_fft(s, d, h, nl, 0);
  nb = make_map(m, nl, [&](int i) { return h[i].W * blocks_for((long long)h[i].npad, 64); });
  if (energy && step_forces) hipLaunchKernelGGL((k_gather<true, true>), dim3(nb), dim3(256), 0, s, d, m);
  else if (energy) hipLaunchKernelGGL((k_gather<true, false>), dim3(nb), dim3(256), 0, s, d, m);
  else if (step_forces) hipLaunchKernelGGL((k_gather<false, true>), dim3(nb), dim3(256), 0, s, d, m);
  else hipLaunchKernelGGL((k_gather<false, false>), dim3(nb), dim3(256), 0, s, d, m);
}

}  // namespace felis
