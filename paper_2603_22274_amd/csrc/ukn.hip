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
// The reciprocal parts need only the ligand's potential phi_L: the PME
// reciprocal energy is a symmetric bilinear form of two spread charge grids,
// so sum_{i in L} q_i phi_E(r_i) = sum_{j in E} q_j phi_L(r_j).  Each frame
// spreads its few ligand charges, two frames share one complex FFT (real and
// imaginary part), and phi_L is gathered at every atom: a read-only pass over
// the environment instead of scattering all of its charges.  Pair distances
// and the softcore LJ are FP64 (a frame evaluated at a state it was not
// sampled in can hold r^-12 overlaps of 1e6 kT), the erfc Coulomb FP32; pair
// sums run in FP64 per lane; block partials combine in a fixed order (pair
// terms) or in int64 fixed point (reciprocal terms).  Frames may each have
// their own box (NPT); with a pressure, u gains beta P V of the frame.
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
  int upk;                             // 1: one frame per complex grid (frames in their own boxes)
  float lamv[kMaxLamV];
  float asc[kMaxLamV];
};

constexpr int kNU = 3 + kMaxLamV;    // accumulators per frame: LE, LL, UB, UT (slot 3; rest unused)

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


__device__ __forceinline__ float3 min_img(const BoxW& B, float dx, float dy, float dz) {
  dx = fmaf(-B.Lf[0], rintf(dx * B.invLf[0]), dx);
  dy = fmaf(-B.Lf[1], rintf(dy * B.invLf[1]), dy);
  dz = fmaf(-B.Lf[2], rintf(dz * B.invLf[2]), dz);
  return make_float3(dx, dy, dz);
}

// The alchemical charge set B: the ligand atoms, then the alchemical-water
// atoms.  A window's charges are a + lambda_elec b: b is the ligand charge
// (minus the offset on an alchemical water, zero elsewhere) and a the
// environment charge plus the offset (zero on ligand atoms), so the
// electrostatic energy is E[a,a] + lambda_elec 2 E[a,b] + lambda_elec^2
// E[b,b]; E_LE = 2 E[a,b] and E_LL = E[b,b].
__device__ __forceinline__ int bset_atom(const LegDev& g, int t) {
  return t < g.nlig ? g.lig_idx[t] : g.aw_idx[t - g.nlig];
}
__device__ __forceinline__ float charge_b(const LegDev& g, int a) {
  return g.lig[a] ? g.q[a] : (g.aoff ? -g.aoff[a] : 0.0f);
}
__device__ __forceinline__ float charge_a(const LegDev& g, int a) {
  return g.lig[a] ? 0.0f : (g.aoff ? g.q[a] + g.aoff[a] : g.q[a]);
}

__device__ __forceinline__ void acc_add(const LegDev& g, int f, int slot, double e) {
  atomicAdd((unsigned long long*)&g.uacc[(size_t)f * kNU + slot],
            (unsigned long long)to_fixed(e, kEnergyScale, g.err, kSiteUkn, f));
}

// items: frame x atom of the alchemical charge set, 16 lanes per atom: the
// b charges of frame f into int64 grid f
__global__ __launch_bounds__(256) void k_ukn_spread(const LegDev* legs, UknArgs A) {
  const LegDev& g = legs[0];
  const int nB = g.nlig + g.naw;
  const long long local = (long long)blockIdx.x * 16 + (threadIdx.x >> 4);
  if (local >= (long long)A.nf * nB) return;
  const int f = (int)(local / nB);
  const int a = bset_atom(g, (int)(local - (long long)f * nB));
  const int sub = threadIdx.x & 15, iy = sub & 3, iz = sub >> 2;
  const size_t o = (size_t)(A.f0 + f) * A.stride + a;
  float fxr, fyr, fzr, wx[4], wy[4], wz[4];
  const BoxW& B = g.ubox[f];
  const int bx = grid_base(A.fx[o], B.invL[0], g.K[0], &fxr);
  const int by = grid_base(A.fy[o], B.invL[1], g.K[1], &fyr);
  const int bz = grid_base(A.fz[o], B.invL[2], g.K[2], &fzr);
  bspline4(fxr, wx); bspline4(fyr, wy); bspline4(fzr, wz);
  int gy = by - iy; if (gy < 0) gy += g.K[1];
  int gz = bz - iz; if (gz < 0) gz += g.K[2];
  // int64 grids 2p, 2p+1 become the real and imaginary parts of complex grid
  // p: frame f takes grid f, or grid 2f (imaginary part left zero) when
  // every frame has a grid of its own
  long long* grid = g.grid64 + (size_t)(A.upk ? 2 * f : f) * g.Ktot + ((size_t)gz * g.K[1] + gy) * g.K[0];
  const double qyz = (double)(charge_b(g, a) * wy[iy] * wz[iz]);
#pragma unroll
  for (int ix = 0; ix < 4; ++ix) {
    int gx = bx - ix; if (gx < 0) gx += g.K[0];
    const long long v = __double2ll_rn(qyz * (double)wx[ix] * kGridScale);
    if (v) atomicAdd((unsigned long long*)&grid[gx], (unsigned long long)v);
  }
}

// items: frame x block of 256 atoms, 16 lanes per atom, 16 atoms per pass:
// phi_b of frame f (part f & 1 of complex grid f / 2) at every atom;
// E_LE += a phi_b, E_LL += b phi_b / 2 over all atoms
__global__ __launch_bounds__(256) void k_ukn_gather(const LegDev* legs, UknArgs A) {
  const LegDev& g = legs[0];
  const int nb = (g.n + 255) / 256;
  const int f = blockIdx.x / nb;
  const int a0 = (blockIdx.x - f * nb) * 256 + (threadIdx.x >> 4);
  const int sub = threadIdx.x & 15, iy = sub & 3, iz = sub >> 2;
  const float* cg = A.upk ? (const float*)(g.cgrid + (size_t)f * g.Ktot)
                          : (const float*)(g.cgrid + (size_t)(f >> 1) * g.Ktot) + (f & 1);
  const BoxW& B = g.ubox[f];
  const size_t fo = (size_t)(A.f0 + f) * A.stride;
  double le = 0.0, ll = 0.0;
  for (int t = 0; t < 16; ++t) {
    const int a = a0 + 16 * t;
    const bool valid = a < g.n;                      // uniform over the 16 lanes of an atom
    const int ac = valid ? a : g.n - 1;
    float fxr, fyr, fzr, wx[4], wy[4], wz[4];
    const int bx = grid_base(A.fx[fo + ac], B.invL[0], g.K[0], &fxr);
    const int by = grid_base(A.fy[fo + ac], B.invL[1], g.K[1], &fyr);
    const int bz = grid_base(A.fz[fo + ac], B.invL[2], g.K[2], &fzr);
    bspline4(fxr, wx); bspline4(fyr, wy); bspline4(fzr, wz);
    int gy = by - iy; if (gy < 0) gy += g.K[1];
    int gz = bz - iz; if (gz < 0) gz += g.K[2];
    const float* row = cg + 2 * ((size_t)gz * g.K[1] + gy) * g.K[0];
    float ph = 0.f;
#pragma unroll
    for (int ix = 0; ix < 4; ++ix) {
      int gx = bx - ix; if (gx < 0) gx += g.K[0];
      ph = fmaf(wx[ix], row[2 * gx], ph);
    }
    ph *= wy[iy] * wz[iz];
    for (int off = 1; off < 16; off <<= 1) ph += __shfl_xor(ph, off, 64);
    if (sub == 0 && valid) {
      le += (double)charge_a(g, ac) * (double)ph;
      ll += 0.5 * (double)charge_b(g, ac) * (double)ph;
    }
  }
  le = wave_sum(le);
  ll = wave_sum(ll);
  __shared__ double s_r[2][4];
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) { s_r[0][wv] = le; s_r[1][wv] = ll; }
  __syncthreads();
  if (threadIdx.x == 0) {
    acc_add(g, f, 0, ((s_r[0][0] + s_r[0][1]) + s_r[0][2]) + s_r[0][3]);
    acc_add(g, f, 1, ((s_r[1][0] + s_r[1][1]) + s_r[1][2]) + s_r[1][3]);
  }
}

constexpr int kGV = 16;              // lambda_vdw values accumulated per lane at once

// block partials of one frame: the 4 waves' sums in LDS, added in wave order
__device__ __forceinline__ void block_partial(double* s_red, int slot, double v) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) s_red[(threadIdx.x >> 6) * (1 + kMaxLamV) + slot] = v;
}

__device__ __forceinline__ void block_flush(const double* s_red, double* out, int nslot) {
  __syncthreads();
  for (int t = threadIdx.x; t < nslot; t += blockDim.x)
    out[t] = ((s_red[t] + s_red[(1 + kMaxLamV) + t]) + s_red[2 * (1 + kMaxLamV) + t]) +
             s_red[3 * (1 + kMaxLamV) + t];
}

// items: frame x block of 256 atoms: pairs of the alchemical charge set with
// environment atoms within r_c (an alchemical water's own atoms: excluded-pair
// erf correction), softcore LJ for the ligand entries.
// Each lane keeps its own FP64 sums over the ligand atoms for kGV lambda_vdw
// values at a time; one block partial per frame, block and slot (slot 0
// Coulomb, 1 + kv softcore LJ at lamv[kv]), unbounded (a frame evaluated at a
// state it was not sampled in may carry enormous overlap energies) and summed
// in a fixed order by k_ukn_combine
__global__ __launch_bounds__(256) void k_ukn_pairs(const LegDev* legs, UknArgs A) {
  const LegDev& g = legs[0];
  const int nb = (g.n + 255) / 256;
  const int f = blockIdx.x / nb;
  const int j = (blockIdx.x - f * nb) * 256 + threadIdx.x;
  __shared__ float4 s_lx[kMaxLigand];     // x, y, z, b charge
  __shared__ float2 s_lp[kMaxLigand];     // sigma/2, eps (ligand entries)
  __shared__ int3 s_aw[kMaxLigand];       // alchemical-water entries: the atom and its two exclusion partners
  __shared__ double s_red[4 * (1 + kMaxLamV)];
  const size_t fo = (size_t)(A.f0 + f) * A.stride;
  const BoxW& B = g.ubox[f];
  const int nB = g.nlig + g.naw;
  for (int t = threadIdx.x; t < nB; t += blockDim.x) {
    const int a = bset_atom(g, t);
    s_lx[t] = make_float4(A.fx[fo + a], A.fy[fo + a], A.fz[fo + a], charge_b(g, a));
    s_lp[t] = make_float2(0.5f * g.sig[a], g.eps[a]);
    if (t >= g.nlig) {
      const int k = t - g.nlig;
      s_aw[t] = make_int3(a, g.aw_idx[g.naw + 2 * k], g.aw_idx[g.naw + 2 * k + 1]);
    }
  }
  __syncthreads();
  const bool env = j < g.n && !g.lig[j];
  float xj = 0.f, yj = 0.f, zj = 0.f, qj = 0.f;
  double hs = 0.0, epsj = 0.0;
  if (env) {
    xj = A.fx[fo + j]; yj = A.fy[fo + j]; zj = A.fz[fo + j];
    qj = charge_a(g, j); hs = 0.5 * (double)g.sig[j]; epsj = (double)g.eps[j];
  }
  const double Lx = B.L[0], Ly = B.L[1], Lz = B.L[2], iLx = B.invL[0], iLy = B.invL[1], iLz = B.invL[2];
  const float c_ke = (float)kKE;
  double ec = 0.0;
  for (int v0 = 0; v0 < A.KV; v0 += kGV) {
    double esc[kGV];
#pragma unroll
    for (int t = 0; t < kGV; ++t) esc[t] = 0.0;
    for (int li = 0; li < nB; ++li) {
      const float4 L = s_lx[li];
      const bool awe = li >= g.nlig;             // uniform: an alchemical-water entry (no softcore)
      // the distance in FP64 (minimum image included): a frame evaluated at a
      // state it was not sampled in can hold r^-12 overlaps of 1e6 kT, where
      // FP32 distances would lose six digits
      double dx = (double)xj - (double)L.x, dy = (double)yj - (double)L.y, dz = (double)zj - (double)L.z;
      dx = fma(-Lx, rint(dx * iLx), dx);
      dy = fma(-Ly, rint(dy * iLy), dy);
      dz = fma(-Lz, rint(dz * iLz), dz);
      const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
      bool in = env && r2 < g.rc2d;
      bool exc = false;
      if (awe) {
        const int3 e3 = s_aw[li];
        in = in && j != e3.x;                    // never the water's own atom
        exc = in && (j == e3.y || j == e3.z);    // its own water: excluded pair
      }
      if (__ballot(in) == 0ull) continue;
      const double r2s = in ? r2 : 1.0;
      if (v0 == 0) {
        const float r2f = (float)r2s;
        const float rinv = __builtin_amdgcn_rsqf(r2f);
        if (exc) {
          ec -= (double)(c_ke * L.w * qj * erff(g.alpha * r2f * rinv) * rinv);
        } else {
          float ex;
          const float erfcv = erfc_fit(g.alpha * r2f * rinv, &ex);
          if (in) ec += (double)(c_ke * L.w * qj * erfcv * rinv);
        }
      }
      if (awe) continue;                         // an alchemical water keeps its LJ (no lambda dependence)
      const double sg = (double)s_lp[li].x + hs;
      const double s2 = sg * sg;
      const double s6 = s2 * s2 * s2;
      const double r6 = r2s * r2s * r2s;
      const double e4 = in ? 4.0 * sqrt((double)s_lp[li].y * epsj) : 0.0;
#pragma unroll
      for (int t = 0; t < kGV; ++t) {
        if (v0 + t < A.KV) {
          const double u = s6 / fma((double)A.asc[v0 + t], s6, r6);
          esc[t] += (double)A.lamv[v0 + t] * e4 * fma(u, u, -u);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < kGV; ++t)
      if (v0 + t < A.KV) block_partial(s_red, 1 + v0 + t, esc[t]);
  }
  block_partial(s_red, 0, ec);
  block_flush(s_red, g.upart + (size_t)blockIdx.x * (1 + kMaxLamV), 1 + A.KV);
}

// one block per frame: pairs within the alchemical charge set (Coulomb of the
// b charges; softcore LJ between ligand atoms), excluded-pair corrections and
// the Boresch energy; one partial row per frame (slot 0 E_LL real space, 1 + kv
// softcore LJ), the same per-lane accumulation as k_ukn_pairs
__global__ __launch_bounds__(256) void k_ukn_ligand(const LegDev* legs, UknArgs A) {
  const LegDev& g = legs[0];
  const int f = blockIdx.x;
  const size_t fo = (size_t)(A.f0 + f) * A.stride;
  const int nl = g.nlig + g.naw;                 // the alchemical charge set
  const int np = nl * (nl - 1) / 2;
  const float c_ke = (float)kKE;
  __shared__ double s_red[4 * (1 + kMaxLamV)];
  double ell = 0.0;
  for (int v0 = 0; v0 < A.KV; v0 += kGV) {
    double esc[kGV];
#pragma unroll
    for (int t = 0; t < kGV; ++t) esc[t] = 0.0;
    for (int base = 0; base < np; base += blockDim.x) {
      const int p = base + threadIdx.x;
      bool in = false;
      double r2s = 1.0, s6 = 0.0, e4 = 0.0;
      if (p < np) {
        // decode p -> (i, j), i < j, row-major over the upper triangle
        int i = 0, rem = p;
        while (rem >= nl - 1 - i) { rem -= nl - 1 - i; ++i; }
        const int jl = i + 1 + rem;
        const int a = bset_atom(g, i), b = bset_atom(g, jl);
        const bool both_lig = i < g.nlig && jl < g.nlig;   // softcore only between ligand atoms
        bool exc = false;
        for (int k = g.excl_ptr[a]; k < g.excl_ptr[a + 1]; ++k) exc |= (g.excl_idx[k] == b);
        const BoxW& B = g.ubox[f];
        double dxd = (double)A.fx[fo + b] - (double)A.fx[fo + a];
        double dyd = (double)A.fy[fo + b] - (double)A.fy[fo + a];
        double dzd = (double)A.fz[fo + b] - (double)A.fz[fo + a];
        dxd = fma(-B.L[0], rint(dxd * B.invL[0]), dxd);
        dyd = fma(-B.L[1], rint(dyd * B.invL[1]), dyd);
        dzd = fma(-B.L[2], rint(dzd * B.invL[2]), dzd);
        const double r2d = fma(dxd, dxd, fma(dyd, dyd, dzd * dzd));
        const float r2 = (float)r2d;
        const float qq = c_ke * charge_b(g, a) * charge_b(g, b);
        if (exc) {
          if (v0 == 0) {
            const float r = sqrtf(r2);
            ell -= (r > 1e-4f) ? (double)(qq * erff(g.alpha * r) / r)
                               : (double)(qq * 2.0f * g.alpha * 0.56418958354775628f);
          }
        } else if (r2d < g.rc2d) {
          in = both_lig;
          r2s = r2d;
          if (v0 == 0) {
            const float rinv = __builtin_amdgcn_rsqf(r2);
            float ex;
            ell += (double)(qq * erfc_fit(g.alpha * r2 * rinv, &ex) * rinv);
          }
          const double sg = 0.5 * ((double)g.sig[a] + (double)g.sig[b]);
          const double s2 = sg * sg;
          s6 = s2 * s2 * s2;
          e4 = 4.0 * sqrt((double)g.eps[a] * (double)g.eps[b]);
        }
      }
      if (__ballot(in) == 0ull) continue;
      const double r6 = r2s * r2s * r2s;
#pragma unroll
      for (int t = 0; t < kGV; ++t) {
        if (v0 + t < A.KV) {
          const double u = s6 / fma((double)A.asc[v0 + t], s6, r6);
          esc[t] += in ? (double)A.lamv[v0 + t] * e4 * fma(u, u, -u) : 0.0;
        }
      }
    }
#pragma unroll
    for (int t = 0; t < kGV; ++t)
      if (v0 + t < A.KV) block_partial(s_red, 1 + v0 + t, esc[t]);
  }
  block_partial(s_red, 0, ell);
  block_flush(s_red, g.lpart + (size_t)f * (1 + kMaxLamV), 1 + A.KV);
  if (threadIdx.x == 0 && g.has_rest) {
    v3 p[6];
    const size_t o1 = fo + g.ranch[0];
    for (int t = 0; t < 6; ++t) {
      const size_t ot = fo + g.ranch[t];
      const float3 d = min_img(g.ubox[f], A.fx[ot] - A.fx[o1], A.fy[ot] - A.fy[o1], A.fz[ot] - A.fz[o1]);
      p[t] = mk(d.x, d.y, d.z);
    }
    acc_add(g, f, 2, boresch_eval(p, g.rg0, g.rk, nullptr));
  }
  if (threadIdx.x == 64 && g.ntors > 0) {
    // rotatable torsions, unscaled, in FP64 (slot 3)
    double ut = 0.0;
    for (int t = 0; t < g.ntors; ++t) {
      const size_t o0 = fo + g.tors[4 * t];
      const BoxW& B = g.ubox[f];
      double p[4][3];
      for (int s = 0; s < 4; ++s) {
        const size_t os = fo + g.tors[4 * t + s];
        double d[3] = {(double)A.fx[os] - (double)A.fx[o0], (double)A.fy[os] - (double)A.fy[o0],
                       (double)A.fz[os] - (double)A.fz[o0]};
        for (int c = 0; c < 3; ++c) p[s][c] = d[c] - B.L[c] * rint(d[c] * B.invL[c]);
      }
      ut += torsion_energy_fp64(p, (double)g.tors_k[t], g.tors_n[t], (double)g.tors_phase[t]);
    }
    acc_add(g, f, 3, ut);
  }
}

// one block: the constants of E_LE / E_LL that depend only on charges: the
// self terms and the two background terms
__global__ __launch_bounds__(256) void k_ukn_const(const LegDev* legs, double* out) {
  const LegDev& g = legs[0];
  double qa = 0.0, qb = 0.0, qb2 = 0.0, qab = 0.0;
  for (int a = threadIdx.x; a < g.n; a += blockDim.x) {
    const double ca = (double)charge_a(g, a), cb = (double)charge_b(g, a);
    qa += ca; qb += cb; qb2 += cb * cb; qab += ca * cb;
  }
  __shared__ double r[4][256];
  r[0][threadIdx.x] = qa; r[1][threadIdx.x] = qb; r[2][threadIdx.x] = qb2; r[3][threadIdx.x] = qab;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s)
      for (int k = 0; k < 4; ++k) r[k][threadIdx.x] += r[k][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = 2.0 * r[0][0] * r[1][0];             // E_LE background / (-bg_pref)
    out[1] = r[1][0] * r[1][0];                   // E_LL background / (-bg_pref)
    out[2] = -g.self_pref * r[2][0];              // E_LL self term
    out[3] = -2.0 * g.self_pref * r[3][0];        // E_LE self term (atoms with both a and b charges)
  }
}

struct CombineArgs {
  double le[kMaxStates], lr[kMaxStates];
  unsigned char kv[kMaxStates];
  double pressure;                     // kcal/(mol A^3): u gains beta P V of the frame's box (NPT)
};

// one block: the box of every frame of the pass (given edges, or the leg's box)
__global__ __launch_bounds__(256) void k_ukn_boxes(const LegDev* legs, UknArgs A, const double* fbox) {
  const LegDev& g = legs[0];
  for (int f = threadIdx.x; f < 2 * g.npair; f += blockDim.x)      // unused entries: the leg's box
    g.ubox[f] = (fbox && f < A.nf) ? make_box(fbox + 3 * (A.f0 + f), (double)g.alpha) : g.box0;
}

// one block per frame: the pair partials of every block of k_ukn_pairs summed
// per slot (one wave per slot, lanes over blocks, fixed tree), then u at every
// state
__global__ __launch_bounds__(256) void k_ukn_combine(const LegDev* legs, UknArgs A, CombineArgs C,
                                                     const double* cst, int K, double beta, double* u,
                                                     long long u_stride) {
  const LegDev& g = legs[0];
  const int f = blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nb = g.nlig + g.naw > 0 ? (g.n + 255) / 256 : 0;     // no alchemical charges: no pair partials
  __shared__ double s_p[1 + kMaxLamV];
  const double* pp = g.upart + (size_t)f * nb * (1 + kMaxLamV);
  const double* lp = g.lpart + (size_t)f * (1 + kMaxLamV);
  for (int slot = wv; slot < 1 + A.KV; slot += 4) {
    double v = 0.0;
    for (int t = lane; t < nb; t += 64) v += pp[(size_t)t * (1 + kMaxLamV) + slot];
    v = wave_sum(v);
    if (lane == 0) s_p[slot] = v;
  }
  __syncthreads();
  const long long* acc = g.uacc + (size_t)f * kNU;
  const double s = 1.0 / kEnergyScale;
  const bool has_l = g.nlig + g.naw > 0;
  const double bg = g.ubox[f].bg_pref;
  const double pv = C.pressure * g.ubox[f].vol;
  for (int k = threadIdx.x; k < K; k += blockDim.x) {
    const int kv = C.kv[k];
    const double ele = (double)acc[0] * s - bg * cst[0] + s_p[0] + cst[3];
    const double ell = (double)acc[1] * s + cst[2] - bg * cst[1] + (has_l ? lp[0] : 0.0);
    const double ub = (double)acc[2] * s;
    const double ut = (double)acc[3] * s;
    const double esc = s_p[1 + kv] + (has_l ? lp[1 + kv] : 0.0);
    const double le = C.le[k], lr = C.lr[k], lv = (double)A.lamv[kv];
    u[(long long)k * u_stride + A.f0 + f] = beta * (le * ele + le * le * ell + esc + lr * ub + lv * ut + pv);
  }
}

}  // namespace

int launch_ukn(hipStream_t s, const LegDev* d, const LegHost& h, double sc_alpha, const double* lambdas,
               int K, const float* fx, const float* fy, const float* fz, long long frame_stride,
               long long n_frames, const double* frame_box, double pressure, double beta, double* u,
               long long u_stride, long long* uacc, double* cst) {
  if (K < 1 || K > kMaxStates) return FELIS_E_UNSUPPORTED;
  const int nB = h.nlig + h.naw;
  if (nB > kMaxLigand) return FELIS_E_UNSUPPORTED;
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
  C.pressure = pressure;
  hipLaunchKernelGGL(k_ukn_const, dim3(1), dim3(256), 0, s, d, cst);
  // two frames per complex grid (2 npair frames per pass) when they share the
  // leg's box; frames with boxes of their own take a grid each
  A.upk = frame_box ? 1 : 0;
  const int F = frame_box ? h.npair : 2 * h.npair;
  for (long long f0 = 0; f0 < n_frames; f0 += F) {
    const int nf = (int)std::min<long long>(F, n_frames - f0);
    const int nb = (h.n + 255) / 256;
    A.f0 = f0;
    A.nf = nf;
    launch_fill_i64(s, uacc, (size_t)nf * kNU);
    hipLaunchKernelGGL(k_ukn_boxes, dim3(1), dim3(256), 0, s, d, A, frame_box);
    if (nB) {
      hipLaunchKernelGGL(k_ukn_spread, dim3((unsigned)(((long long)nf * nB + 15) / 16)), dim3(256), 0, s, d, A);
      launch_pme_fft(s, d, &h, 1, frame_box ? 2 : 1);
      hipLaunchKernelGGL(k_ukn_gather, dim3((unsigned)(nf * nb)), dim3(256), 0, s, d, A);
      hipLaunchKernelGGL(k_ukn_pairs, dim3((unsigned)(nf * nb)), dim3(256), 0, s, d, A);
      hipLaunchKernelGGL(k_ukn_ligand, dim3(nf), dim3(256), 0, s, d, A);
    }
    hipLaunchKernelGGL(k_ukn_combine, dim3((unsigned)nf), dim3(256), 0, s, d, A, C, (const double*)cst, K, beta,
                       u, u_stride);
  }
  return FELIS_OK;
}

}  // namespace felis
