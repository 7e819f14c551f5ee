// Cross-lambda reduced potentials u_k(x_n) for MBAR (section "Simulation
// protocol").  With ligand charges scaled by lambda_e (section "Double
// annihilation protocol") a window's potential is
//   U_k = U_env + lam_e E_LE + lam_e^2 E_LL + E_sc(lam_v) + lam_r U_B,
// U_env is lambda-independent and dropped (MBAR is invariant to it).
//   E_LE: ligand-environment real-space erfc Coulomb + reciprocal cross term
//         sum_{i in L} q_i phi_E(r_i) + background cross term;
//   E_LL: ligand-ligand real-space Coulomb over non-excluded pairs, minus
//         erf terms of excluded pairs, 1/2 sum_{i in L} q_i phi_L(r_i),
//         ligand self term, ligand background term;
//   E_sc: softcore LJ of every ligand pair (ligand-environment and
//         non-excluded ligand-ligand) at lambda_ij = lam_v;
//   U_B:  Boresch energy.
// phi_E and phi_L come from one complex PME per frame: the environment's
// charges spread into the real part, the ligand's into the imaginary part.
// Sums run in FP64 per lane and combine in int64 fixed point.
#include "felis_internal.h"
#include "erfc_coeffs.h"
#include "restraint.h"

#include <algorithm>

namespace felis {
namespace {

struct UknArgs {
  const float *fx, *fy, *fz;
  long long stride, f0;
  int nf, KV;
  float lamv[kMaxLamV];
  float asc[kMaxLamV];
};

constexpr int kNU = 3 + kMaxLamV;    // accumulators per frame: LE, LL, UB, E_sc[KV]

__device__ __forceinline__ float erfc_fit(float x, float* ex) {
  const float t = __builtin_amdgcn_rcpf(fmaf(FELIS_ERFC_P, x, 1.0f));
  float p = felis_erfc_c[0];
#pragma unroll
  for (int k = 1; k < FELIS_ERFC_NC; ++k) p = fmaf(p, t, felis_erfc_c[k]);
  const float e = __expf(-x * x);
  *ex = e;
  return p * t * e;
}

__device__ __forceinline__ void bspline4(float f, float* w) {
  const float f2 = f * f, f3 = f2 * f, g1 = 1.0f - f;
  w[0] = f3 * (1.0f / 6.0f);
  w[1] = (-3.0f * f3 + 3.0f * f2 + 3.0f * f + 1.0f) * (1.0f / 6.0f);
  w[2] = (3.0f * f3 - 6.0f * f2 + 4.0f) * (1.0f / 6.0f);
  w[3] = g1 * g1 * g1 * (1.0f / 6.0f);
}


__device__ __forceinline__ float3 min_img(const LegDev& g, float dx, float dy, float dz) {
  dx = fmaf(-g.Lf[0], rintf(dx * g.invLf[0]), dx);
  dy = fmaf(-g.Lf[1], rintf(dy * g.invLf[1]), dy);
  dz = fmaf(-g.Lf[2], rintf(dz * g.invLf[2]), dz);
  return make_float3(dx, dy, dz);
}

__device__ __forceinline__ void acc_add(const LegDev& g, int f, int slot, double e) {
  atomicAdd((unsigned long long*)&g.uacc[(size_t)f * kNU + slot],
            (unsigned long long)to_fixed(e, kEnergyScale, g.err, kSiteUkn, f));
}

// items: frame x atom, 16 lanes per atom; environment charges into grid 2f,
// ligand charges into grid 2f+1 (unscaled charges)
__global__ __launch_bounds__(256) void k_ukn_spread(const LegDev* legs, UknArgs A) {
  const LegDev& g = legs[0];
  const long long local = (long long)blockIdx.x * 16 + (threadIdx.x >> 4);
  if (local >= (long long)A.nf * g.n) return;
  const int f = (int)(local / g.n);
  const int a = (int)(local - (long long)f * g.n);
  const int sub = threadIdx.x & 15, iy = sub & 3, iz = sub >> 2;
  const size_t o = (size_t)(A.f0 + f) * A.stride + a;
  float fxr, fyr, fzr, wx[4], wy[4], wz[4];
  const int bx = grid_base(A.fx[o], g.invL[0], g.K[0], &fxr);
  const int by = grid_base(A.fy[o], g.invL[1], g.K[1], &fyr);
  const int bz = grid_base(A.fz[o], g.invL[2], g.K[2], &fzr);
  bspline4(fxr, wx); bspline4(fyr, wy); bspline4(fzr, wz);
  int gy = by - iy; if (gy < 0) gy += g.K[1];
  int gz = bz - iz; if (gz < 0) gz += g.K[2];
  const int which = 2 * f + (g.lig[a] ? 1 : 0);
  long long* grid = g.grid64 + (size_t)which * g.Ktot + ((size_t)gz * g.K[1] + gy) * g.K[0];
  const double qyz = (double)(g.q[a] * wy[iy] * wz[iz]);
#pragma unroll
  for (int ix = 0; ix < 4; ++ix) {
    int gx = bx - ix; if (gx < 0) gx += g.K[0];
    const long long v = __double2ll_rn(qyz * (double)wx[ix] * kGridScale);
    if (v) atomicAdd((unsigned long long*)&grid[gx], (unsigned long long)v);
  }
}

// items: frame x ligand atom, 16 lanes per atom: E_LE += q phi_E, E_LL += q phi_L / 2
__global__ __launch_bounds__(256) void k_ukn_gather(const LegDev* legs, UknArgs A) {
  const LegDev& g = legs[0];
  const long long local = (long long)blockIdx.x * 16 + (threadIdx.x >> 4);
  if (local >= (long long)A.nf * g.nlig) return;
  const int f = (int)(local / g.nlig);
  const int a = g.lig_idx[local - (long long)f * g.nlig];
  const int sub = threadIdx.x & 15, iy = sub & 3, iz = sub >> 2;
  const size_t o = (size_t)(A.f0 + f) * A.stride + a;
  float fxr, fyr, fzr, wx[4], wy[4], wz[4];
  const int bx = grid_base(A.fx[o], g.invL[0], g.K[0], &fxr);
  const int by = grid_base(A.fy[o], g.invL[1], g.K[1], &fyr);
  const int bz = grid_base(A.fz[o], g.invL[2], g.K[2], &fzr);
  bspline4(fxr, wx); bspline4(fyr, wy); bspline4(fzr, wz);
  int gy = by - iy; if (gy < 0) gy += g.K[1];
  int gz = bz - iz; if (gz < 0) gz += g.K[2];
  const float2* cg = g.cgrid + (size_t)f * g.Ktot + ((size_t)gz * g.K[1] + gy) * g.K[0];
  float pe = 0.f, pl = 0.f;
#pragma unroll
  for (int ix = 0; ix < 4; ++ix) {
    int gx = bx - ix; if (gx < 0) gx += g.K[0];
    const float2 c = cg[gx];
    pe = fmaf(wx[ix], c.x, pe);
    pl = fmaf(wx[ix], c.y, pl);
  }
  const float wyz = wy[iy] * wz[iz];
  pe *= wyz; pl *= wyz;
  for (int off = 1; off < 16; off <<= 1) {
    pe += __shfl_xor(pe, off, 64);
    pl += __shfl_xor(pl, off, 64);
  }
  if (sub == 0) {
    const double q = (double)g.q[a];
    acc_add(g, f, 0, q * (double)pe);
    acc_add(g, f, 1, 0.5 * q * (double)pl);
  }
}

// items: frame x block of 256 atoms: ligand-environment pairs within r_c
__global__ __launch_bounds__(256) void k_ukn_pairs(const LegDev* legs, UknArgs A) {
  const LegDev& g = legs[0];
  const int nb = (g.n + 255) / 256;
  const int f = blockIdx.x / nb;
  const int j = (blockIdx.x - f * nb) * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63;
  __shared__ float4 s_lx[kMaxLigand];     // x, y, z, q
  __shared__ float2 s_lp[kMaxLigand];     // sigma/2, 2 sqrt(eps)
  const size_t fo = (size_t)(A.f0 + f) * A.stride;
  for (int t = threadIdx.x; t < g.nlig; t += blockDim.x) {
    const int a = g.lig_idx[t];
    s_lx[t] = make_float4(A.fx[fo + a], A.fy[fo + a], A.fz[fo + a], g.q[a]);
    s_lp[t] = make_float2(0.5f * g.sig[a], 2.0f * sqrtf(g.eps[a]));
  }
  __syncthreads();
  const bool env = j < g.n && !g.lig[j];
  float xj = 0.f, yj = 0.f, zj = 0.f, qj = 0.f, hs = 0.f, se = 0.f;
  if (env) {
    xj = A.fx[fo + j]; yj = A.fy[fo + j]; zj = A.fz[fo + j];
    qj = g.q[j]; hs = 0.5f * g.sig[j]; se = 2.0f * sqrtf(g.eps[j]);
  }
  const float c_ke = (float)kKE;
  double ec = 0.0, esc = 0.0;
  for (int li = 0; li < g.nlig; ++li) {
    const float4 L = s_lx[li];
    const float3 d = min_img(g, xj - L.x, yj - L.y, zj - L.z);
    const float r2 = d.x * d.x + d.y * d.y + d.z * d.z;
    const bool in = env && r2 < g.rc2;
    if (__ballot(in) == 0ull) continue;
    const float r2s = in ? r2 : 1.0f;
    const float rinv = __builtin_amdgcn_rsqf(r2s);
    float ex;
    const float erfcv = erfc_fit(g.alpha * r2s * rinv, &ex);
    if (in) ec += (double)(c_ke * L.w * qj * erfcv * rinv);
    const float sg = s_lp[li].x + hs;
    const float s2 = sg * sg;
    const float s6 = s2 * s2 * s2;
    const float r6 = r2s * r2s * r2s;
    const float e4 = s_lp[li].y * se;
    for (int kv = 0; kv < A.KV; ++kv) {
      const float inv = __builtin_amdgcn_rcpf(fmaf(A.asc[kv], s6, r6));
      const float u = s6 * inv;
      const float e = in ? A.lamv[kv] * e4 * fmaf(u, u, -u) : 0.0f;
      const double tot = wave_sum((double)e);
      if (lane == kv) esc += tot;
    }
  }
  // per-wave FP64 partials (unbounded: a frame evaluated at a state it was
  // not sampled in may carry enormous overlap energies); summed in a fixed
  // order by k_ukn_combine
  ec = wave_sum(ec);
  double* part = g.upart + ((size_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * (1 + kMaxLamV);
  if (lane == 0) part[0] = ec;
  if (lane < A.KV) part[1 + lane] = esc;
}

// one block per frame: ligand-ligand pairs, excluded-pair corrections and the
// Boresch energy
__global__ __launch_bounds__(256) void k_ukn_ligand(const LegDev* legs, UknArgs A) {
  const LegDev& g = legs[0];
  const int f = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const size_t fo = (size_t)(A.f0 + f) * A.stride;
  const int nl = g.nlig;
  const int np = nl * (nl - 1) / 2;
  const float c_ke = (float)kKE;
  double ell = 0.0, esc = 0.0;
  for (int base = 0; base < np; base += blockDim.x) {
    const int p = base + threadIdx.x;
    bool in = false, exc = false;
    float r2s = 1.0f, qq = 0.f, s6 = 0.f, e4 = 0.f;
    if (p < np) {
      // decode p -> (i, j), i < j, row-major over the upper triangle
      int i = 0, rem = p;
      while (rem >= nl - 1 - i) { rem -= nl - 1 - i; ++i; }
      const int jl = i + 1 + rem;
      const int a = g.lig_idx[i], b = g.lig_idx[jl];
      for (int k = g.excl_ptr[a]; k < g.excl_ptr[a + 1]; ++k) exc |= (g.excl_idx[k] == b);
      const float3 d = min_img(g, A.fx[fo + b] - A.fx[fo + a], A.fy[fo + b] - A.fy[fo + a],
                               A.fz[fo + b] - A.fz[fo + a]);
      const float r2 = d.x * d.x + d.y * d.y + d.z * d.z;
      qq = c_ke * g.q[a] * g.q[b];
      if (exc) {
        const float r = sqrtf(r2);
        ell -= (r > 1e-4f) ? (double)(qq * erff(g.alpha * r) / r)
                           : (double)(qq * 2.0f * g.alpha * 0.56418958354775628f);
      } else if (r2 < g.rc2) {
        in = true;
        r2s = r2;
        const float rinv = __builtin_amdgcn_rsqf(r2);
        float ex;
        ell += (double)(qq * erfc_fit(g.alpha * r2 * rinv, &ex) * rinv);
        const float sg = 0.5f * (g.sig[a] + g.sig[b]);
        const float s2 = sg * sg;
        s6 = s2 * s2 * s2;
        e4 = 4.0f * sqrtf(g.eps[a] * g.eps[b]);
      }
    }
    if (__ballot(in) == 0ull) continue;
    const float r6 = r2s * r2s * r2s;
    for (int kv = 0; kv < A.KV; ++kv) {
      const float inv = __builtin_amdgcn_rcpf(fmaf(A.asc[kv], s6, r6));
      const float u = s6 * inv;
      const float e = in ? A.lamv[kv] * e4 * fmaf(u, u, -u) : 0.0f;
      const double tot = wave_sum((double)e);
      if (lane == kv) esc += tot;
    }
  }
  ell = wave_sum(ell);
  double* part = g.lpart + ((size_t)f * 4 + (threadIdx.x >> 6)) * (1 + kMaxLamV);
  if (lane == 0) part[0] = ell;
  if (lane < A.KV) part[1 + lane] = esc;
  if (threadIdx.x == 0 && g.has_rest) {
    v3 p[6];
    const size_t o1 = fo + g.ranch[0];
    for (int t = 0; t < 6; ++t) {
      const size_t ot = fo + g.ranch[t];
      const float3 d = min_img(g, A.fx[ot] - A.fx[o1], A.fy[ot] - A.fy[o1], A.fz[ot] - A.fz[o1]);
      p[t] = mk(d.x, d.y, d.z);
    }
    acc_add(g, f, 2, boresch_eval(p, g.rg0, g.rk, nullptr));
  }
}

// one block: lambda-independent constants of E_LE / E_LL that depend only on
// charges: ligand self term and the two background terms
__global__ __launch_bounds__(256) void k_ukn_const(const LegDev* legs, double* out) {
  const LegDev& g = legs[0];
  double qe = 0.0, ql = 0.0, ql2 = 0.0;
  for (int a = threadIdx.x; a < g.n; a += blockDim.x) {
    const double q = (double)g.q[a];
    if (g.lig[a]) { ql += q; ql2 += q * q; } else qe += q;
  }
  __shared__ double r[3][256];
  r[0][threadIdx.x] = qe; r[1][threadIdx.x] = ql; r[2][threadIdx.x] = ql2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int k = 0; k < 3; ++k) r[k][threadIdx.x] += r[k][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = -g.bg_pref * 2.0 * r[0][0] * r[1][0];                          // E_LE background
    out[1] = -(double)g.self_pref * r[2][0] - g.bg_pref * r[1][0] * r[1][0];  // E_LL self + background
  }
}

struct CombineArgs {
  double le[kMaxStates], lr[kMaxStates];
  unsigned char kv[kMaxStates];
};

// items: frame x state
__global__ __launch_bounds__(256) void k_ukn_combine(const LegDev* legs, UknArgs A, CombineArgs C,
                                                     const double* cst, int K, double beta, double* u,
                                                     long long u_stride) {
  const LegDev& g = legs[0];
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)A.nf * K) return;
  const int f = (int)(i / K), k = (int)(i - (long long)(i / K) * K);
  const long long* acc = g.uacc + (size_t)f * kNU;
  const double s = 1.0 / kEnergyScale;
  const int kv = C.kv[k];
  double ele = (double)acc[0] * s + cst[0];
  double ell = (double)acc[1] * s + cst[1];
  const double ub = (double)acc[2] * s;
  double esc = 0.0;
  const int nb = g.nlig > 0 ? (g.n + 255) / 256 : 0;     // no ligand: no pair partials
  const double* pp = g.upart + (size_t)f * nb * 4 * (1 + kMaxLamV);
  for (int t = 0; t < 4 * nb; ++t) {
    ele += pp[(size_t)t * (1 + kMaxLamV)];
    esc += pp[(size_t)t * (1 + kMaxLamV) + 1 + kv];
  }
  const double* lp = g.lpart + (size_t)f * 4 * (1 + kMaxLamV);
  for (int t = 0; t < (g.nlig > 0 ? 4 : 0); ++t) {
    ell += lp[t * (1 + kMaxLamV)];
    esc += lp[t * (1 + kMaxLamV) + 1 + kv];
  }
  const double le = C.le[k], lr = C.lr[k];
  u[(long long)k * u_stride + A.f0 + f] = beta * (le * ele + le * le * ell + esc + lr * ub);
}

}  // namespace

int launch_ukn(hipStream_t s, const LegDev* d, const LegHost& h, double sc_alpha, const double* lambdas,
               int K, const float* fx, const float* fy, const float* fz, long long frame_stride,
               long long n_frames, double beta, double* u, long long u_stride, long long* uacc,
               double* cst) {
  if (K < 1 || K > kMaxStates) return FELIS_E_UNSUPPORTED;
  if (h.nlig > kMaxLigand) return FELIS_E_UNSUPPORTED;
  UknArgs A;
  CombineArgs C;
  A.fx = fx; A.fy = fy; A.fz = fz;
  A.stride = frame_stride;
  A.KV = 0;
  for (int k = 0; k < K; ++k) {
    const float lv = (float)lambdas[3 * k + 1];
    int found = -1;
    for (int t = 0; t < A.KV; ++t)
      if (A.lamv[t] == lv) found = t;
    if (found < 0) {
      if (A.KV == kMaxLamV) return FELIS_E_UNSUPPORTED;
      found = A.KV;
      A.lamv[A.KV] = lv;
      A.asc[A.KV] = (float)(sc_alpha * (1.0 - lambdas[3 * k + 1]));
      ++A.KV;
    }
    C.kv[k] = (unsigned char)found;
    C.le[k] = lambdas[3 * k];
    C.lr[k] = lambdas[3 * k + 2];
  }
  hipLaunchKernelGGL(k_ukn_const, dim3(1), dim3(256), 0, s, d, cst);
  const int F = h.npair;
  for (long long f0 = 0; f0 < n_frames; f0 += F) {
    const int nf = (int)std::min<long long>(F, n_frames - f0);
    A.f0 = f0;
    A.nf = nf;
    launch_fill_i64(s, uacc, (size_t)nf * kNU);
    hipLaunchKernelGGL(k_ukn_spread, dim3((unsigned)(((long long)nf * h.n + 15) / 16)), dim3(256), 0, s, d, A);
    launch_pme_fft(s, d, &h, 1, true);
    if (h.nlig) {
      hipLaunchKernelGGL(k_ukn_gather, dim3((unsigned)(((long long)nf * h.nlig + 15) / 16)), dim3(256), 0, s, d, A);
      hipLaunchKernelGGL(k_ukn_pairs, dim3((unsigned)(nf * ((h.n + 255) / 256))), dim3(256), 0, s, d, A);
      hipLaunchKernelGGL(k_ukn_ligand, dim3(nf), dim3(256), 0, s, d, A);
    }
    hipLaunchKernelGGL(k_ukn_combine, dim3((unsigned)(((long long)nf * K + 255) / 256)), dim3(256), 0, s, d,
                       A, C, (const double*)cst, K, beta, u, u_stride);
  }
  return FELIS_OK;
}

}  // namespace felis
