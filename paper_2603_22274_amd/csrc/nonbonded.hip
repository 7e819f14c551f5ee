// Real-space alchemical pair kernel, Ewald corrections, bonds and the Boresch
// restraint.
//
// Pair terms follow section "Double annihilation protocol": ligand charges
// scaled by lambda_elec; Beutler softcore U = lam 4 eps (s6^2/s^2 - s6/s),
// s = alpha (1 - lam) s6 + r^6 (p = 1), lam = lambda_vdw for any pair touching
// the ligand and 1 otherwise; Lorentz-Berthelot mixing; everything cut at r_c
// (appendix B).  Real-space Coulomb is the Ewald direct term erfc(a r)/r.
//
// Pair kernel layout (gfx950, wave64): one wave per 8-atom i-cluster; the
// cluster's i-atoms are wave-uniform (scalar registers).  The cluster's two
// half-lists (partners of atoms 0-3, then of atoms 4-7) are swept in turn:
// each lane takes one listed j-atom per step and interacts it with the half's
// 4 i-atoms, so a j entry is loaded, decoded and imaged once for 4 pairs, and
// the next steps' entries and partner data are already in flight.  Each
// cluster lists all its partners (both directions), so every atom's pair force
// is summed by one wave in a fixed order and written once: no atomics and no
// cross-wave ordering.  FP32 arithmetic; energies summed in FP64 per lane and
// combined in int64 fixed point.
#include "felis_internal.h"

#include "erfc_coeffs.h"
#include "restraint.h"

namespace felis {
namespace {

// items: window x slot -- current coordinates (wrapped into the box) and
// scaled charges in sorted order, and each slot's PME stencil (grid base and
// B-spline offsets).  REBUILD (inside a list build): for windows being
// rebuilt also the sorted per-slot LJ parameters and each 8-slot cluster's
// bounding box of wrapped positions (8 consecutive lanes hold one cluster:
// N_pad is a multiple of 8).
template <bool REBUILD>
__global__ __launch_bounds__(256) void k_pack(const LegDev* legs, BlockMap map) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const long long i = (long long)(blockIdx.x - map.start[leg]) * blockDim.x + threadIdx.x;
  const bool valid = i < (long long)g.W * g.npad;
  const long long ic = valid ? i : (long long)g.W * g.npad - 1;
  const int w = (int)(ic / g.npad);
  const int a = valid ? g.perm[ic] : -1;
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (a >= 0) {
    // coordinates wrapped into the window's box [0, L): the pair kernel
    // needs no periodic shift for a cluster lying r_c inside every face
    const size_t o = (size_t)w * g.n + a;
    const float q = window_charge(g, a, g.lam[4 * w]);
    const BoxW& Bp = g.box[w];
    v = make_float4(wrapf(g.x[o], Bp.Lf[0], Bp.invLf[0]), wrapf(g.y[o], Bp.Lf[1], Bp.invLf[1]),
                    wrapf(g.z[o], Bp.Lf[2], Bp.invLf[2]), q * (float)sqrt(kKE));
  }
  if (valid) {
    g.xyzq[i] = v;
    // PME stencil of the slot (read by spreading and the gather)
    float f[3];
    const BoxW& B = g.box[w];
    const int bx = grid_base(v.x, B.invL[0], g.K[0], &f[0]);
    const int by = grid_base(v.y, B.invL[1], g.K[1], &f[1]);
    const int bz = grid_base(v.z, B.invL[2], g.K[2], &f[2]);
    g.gsten[i] = make_float4(f[0], f[1], f[2], pack_bases(bx, by, bz));
  }
  if (REBUILD) {
    const bool fl = valid && g.flag[w] != 0;
    if (fl) {
      // the ligand flag rides in the sign bit of 2 sqrt(eps) (-0 for a
      // ligand atom without LJ), so a partner's parameters are 8 bytes
      float2 p = make_float2(0.f, 0.f);
      if (a >= 0) {
        const float e2 = 2.0f * sqrtf(g.eps[a]);
        p = make_float2(0.5f * g.sig[a], g.lig[a] ? -e2 : e2);
      }
      g.prm[i] = p;
    }
    float lo[3] = {3.0e38f, 3.0e38f, 3.0e38f}, hi[3] = {-3.0e38f, -3.0e38f, -3.0e38f};
    if (a >= 0) {
      const BoxW& B = g.box[w];
      const float r[3] = {wrapf(v.x, B.Lf[0], B.invLf[0]), wrapf(v.y, B.Lf[1], B.invLf[1]),
                          wrapf(v.z, B.Lf[2], B.invLf[2])};
      for (int d = 0; d < 3; ++d) { lo[d] = r[d]; hi[d] = r[d]; }
    }
    for (int k = 1; k < kClus; k <<= 1)
      for (int d = 0; d < 3; ++d) {
        lo[d] = fminf(lo[d], __shfl_xor(lo[d], k, 64));
        hi[d] = fmaxf(hi[d], __shfl_xor(hi[d], k, 64));
      }
    if (fl && (i & (kClus - 1)) == 0) {
      g.bblo[i / kClus] = make_float4(lo[0], lo[1], lo[2], 0.f);
      g.bbhi[i / kClus] = make_float4(hi[0], hi[1], hi[2], 0.f);
    }
  }
}

__device__ __forceinline__ float3 min_img(const BoxW& B, float dx, float dy, float dz) {
  dx = fmaf(-B.Lf[0], rintf(dx * B.invLf[0]), dx);
  dy = fmaf(-B.Lf[1], rintf(dy * B.invLf[1]), dy);
  dz = fmaf(-B.Lf[2], rintf(dz * B.invLf[2]), dz);
  return make_float3(dx, dy, dz);
}

// The 8 i-atoms of a cluster, wave-uniform (held in scalar registers).
struct ICluster {
  float x[kClus], y[kClus], z[kClus], q[kClus], sig[kClus], eps[kClus], lig[kClus];
  int ai[kClus];                            // atom indices (FP64 energies)
};

// One pair's real-space Coulomb and LJ energies with every term in FP64 (the
// energy level 2 of the pair kernel): the minimum-image distance from the
// raw (unwrapped) FP32 coordinates of atoms ai, aj as d - L rint(d (1/L)) and d^2 = (dx^2 + dy^2) + dz^2
// without contraction, the cutoff r < r_c on r = sqrt(d^2), the window's
// charges of atoms ai, aj in FP64, Lorentz-Berthelot parameters from the packed (sigma/2,
// 2 sqrt(eps)) and the softcore form at lambda_vdw for pairs touching the
// ligand.  Out of line: its registers stay out of the force path.
__device__ __attribute__((noinline)) void pair_energy_fp64(const LegDev& g, const BoxW& B, size_t base, int ai,
                                                           int aj, float ligi, float ligj, float hsi, float hsj,
                                                           float e2i, float e2j, float lam_e, float lam_v,
                                                           double& ec, double& el) {
#pragma clang fp contract(off)
  const size_t oi = base + ai, oj = base + aj;
  double dx = (double)g.x[oi] - (double)g.x[oj], dy = (double)g.y[oi] - (double)g.y[oj];
  double dz = (double)g.z[oi] - (double)g.z[oj];
  dx = dx - B.L[0] * rint(dx * B.invL[0]);
  dy = dy - B.L[1] * rint(dy * B.invL[1]);
  dz = dz - B.L[2] * rint(dz * B.invL[2]);
  const double r2 = (dx * dx + dy * dy) + dz * dz;
  const double r = sqrt(r2);
  if (!(r < g.rcd)) return;
  const bool li = ligi > 0.0f, lj = ligj > 0.0f;
  const double qa = window_charge_fp64(g, ai, (double)lam_e), qb = window_charge_fp64(g, aj, (double)lam_e);
  ec += kKE * qa * qb * erfc(g.alphad * r) / r;
  const double sig = (double)hsi + (double)hsj;
  const double eps = 0.25 * (double)e2i * (double)e2j;
  if (eps == 0.0) return;
  const double lam = (li || lj) ? (double)lam_v : 1.0;
  const double s2 = sig * sig, s6 = s2 * s2 * s2;
  const double s = g.sc_alphad * (1.0 - lam) * s6 + r2 * r2 * r2;
  el += lam * 4.0 * eps * (s6 * s6 / (s * s) - s6 / s);
}

__device__ __forceinline__ float uniform(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// a window's box edges held in scalar registers for a whole kernel
struct BoxF {
  float L[3], iL[3];
};

__device__ __forceinline__ BoxF box_f(const BoxW& B) {
  BoxF b;
  for (int d = 0; d < 3; ++d) { b.L[d] = uniform(B.Lf[d]); b.iL[d] = uniform(B.invLf[d]); }
  return b;
}

// Sweep a cluster's j-list: lane = listed j, unrolled loop over the cluster's
// i-atoms.  IMG 1: the periodic image of j is chosen once against the
// cluster's first atom (exact when r_c + cluster extent < L/2 on every axis);
// IMG 2: none (the cluster lies r_c inside every face of the box, so every
// partner within r_c has its wrapped coordinates as its nearest image, and
// any other image only lengthens the separation); IMG 0: every (i, j) takes
// its own minimum image.
template <int ENERGY, int IMG, int HALF>
__device__ __forceinline__ void sweep(const LegDev& g, const BoxF B, const ICluster& I, gptr<unsigned> ent, int cnt,
                                      gptr<f32x4> xq, gptr<f32x2> pr, int lane,
                                      float lam_v, float a_sc, bool soft_window, float (&fx)[4],
                                      float (&fy)[4], float (&fz)[4], double& ec, double& el, const BoxW* Bw,
                                      float lam_e, const int* permw, size_t base) {
  const float Lx = B.L[0], Ly = B.L[1], Lz = B.L[2];
  const float iLx = B.iL[0], iLy = B.iL[1], iLz = B.iL[2];
  const float rc2 = g.rc2, alpha = g.alpha;
  const float c2a = 2.0f * alpha * 0.56418958354775628f;   // 2 alpha / sqrt(pi)
  const float pa = FELIS_ERFC_P * alpha;                    // fit variable t = 1 / (1 + P alpha r)
  const float kx2 = -alpha * alpha * 1.4426950408889634f;   // exp(-alpha^2 r^2) = 2^(kx2 r^2)
  // software pipeline: the entries two steps ahead and the partner data one
  // step ahead are in flight while a step computes
  unsigned e_next = lane < cnt ? ent[lane] : 0u;          // slot 0 with an empty mask
  unsigned e_next2 = 64 + lane < cnt ? ent[64 + lane] : 0u;
  f32x4 xj_next = xq[(int)(e_next >> 8)];
  f32x2 pj_next = pr[(int)(e_next >> 8)];
  for (int it = 0; it < cnt; it += 64) {
    const unsigned e = e_next;
    const f32x4 xj = xj_next;
    const f32x2 pj = pj_next;
    const int s = (int)(e >> 8);
    e_next = e_next2;
    const int nidx = it + 128 + lane;
    e_next2 = nidx < cnt ? ent[nidx] : 0u;
    xj_next = xq[(int)(e_next >> 8)];
    pj_next = pr[(int)(e_next >> 8)];
    const float ligj = (__float_as_uint(pj.y) >> 31) ? 1.0f : 0.0f;
    float jx = xj.x, jy = xj.y, jz = xj.z;
    if (IMG == 1) {
      jx = fmaf(-Lx, rintf((jx - I.x[0]) * iLx), jx);
      jy = fmaf(-Ly, rintf((jy - I.y[0]) * iLy), jy);
      jz = fmaf(-Lz, rintf((jz - I.z[0]) * iLz), jz);
    }
    // wave-uniform: does any listed j of this step belong to the ligand?
    const bool jlig = soft_window && __ballot(ligj > 0.0f) != 0ull;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int ii = 4 * HALF + k;
      float dx = jx - I.x[ii], dy = jy - I.y[ii], dz = jz - I.z[ii];
      if (IMG == 0) {
        dx = fmaf(-Lx, rintf(dx * iLx), dx);
        dy = fmaf(-Ly, rintf(dy * iLy), dy);
        dz = fmaf(-Lz, rintf(dz * iLz), dz);
      }
      const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
      // r^2 of a listed pair, 3e38 for an unlisted one (excluded, the atom
      // itself or beyond r_list): one compare gives the in-range mask
      const float r2m = ((e >> k) & 1u) ? r2 : 3.0e38f;
      const bool in = r2m < rc2;
      // wave-uniform: no lane's partner lies within r_c of this i-atom (the
      // list's entries are consecutive in the Hilbert order, so a wave's
      // partners are near one another and often all beyond r_c of one side
      // of the half-cluster); a skipped lane adds nothing, exactly as the
      // select below would.  The FP64 energy form decides its own cutoff.
      if (ENERGY < 2 && __ballot(in) == 0ull) continue;
      // lanes outside (in == false) may compute inf or NaN below: every
      // result they feed is dropped by the selects on `in`
      const float r2s = r2;
      const float rinv = __builtin_amdgcn_rsqf(r2s);
      const float rinv2 = rinv * rinv;
      const float r = r2s * rinv;
      // erfc(alpha r) = t P(t) exp(-alpha^2 r^2), t = 1 / (1 + P alpha r): the
      // degree-6 fit of erfc_coeffs.h with alpha folded into its constants
      const float t = __builtin_amdgcn_rcpf(fmaf(pa, r, 1.0f));
      float pt = felis_erfc_c[0];
#pragma unroll
      for (int c = 1; c < FELIS_ERFC_NC; ++c) pt = fmaf(pt, t, felis_erfc_c[c]);
      pt *= t;
      const float ex = __builtin_amdgcn_exp2f(kx2 * r2s);
      const float qq = I.q[ii] * xj.w;
      const float fc = qq * (ex * fmaf(pt, rinv, c2a)) * rinv2;
      float flj = 0.0f, elj = 0.0f;
      if (I.eps[ii] == 0.0f) {
        // wave-uniform: an i-atom without LJ (a water hydrogen) contributes
        // exactly zero LJ force and energy with every partner
      } else if (const float sig = I.sig[ii] + pj.x, eps4 = I.eps[ii] * fabsf(pj.y);
                 (jlig || (soft_window && I.lig[ii] > 0.0f)) &&
                 __ballot(in && (I.lig[ii] + ligj) > 0.0f) != 0ull) {
        const bool ligp = (I.lig[ii] + ligj) > 0.0f;
        const float lam = ligp ? lam_v : 1.0f;
        const float a = ligp ? a_sc : 0.0f;
        const float s2 = sig * sig;
        const float s6 = s2 * s2 * s2;
        const float r4 = r2s * r2s;
        const float den = fmaf(a, s6, r4 * r2s);
        const float inv = __builtin_amdgcn_rcpf(den);
        const float u = s6 * inv;
        const float le = lam * eps4;
        flj = 6.0f * le * fmaf(2.0f, u, -1.0f) * u * inv * r4;
        if (ENERGY) elj = le * fmaf(u, u, -u);
      } else {
        const float s2 = sig * sig * rinv2;
        const float s6 = s2 * s2 * s2;
        flj = eps4 * fmaf(12.0f, s6, -6.0f) * s6 * rinv2;
        if (ENERGY) elj = eps4 * fmaf(s6, s6, -s6);
      }
      const float fs = in ? (fc + flj) : 0.0f;
      fx[k] = fmaf(-fs, dx, fx[k]);
      fy[k] = fmaf(-fs, dy, fy[k]);
      fz[k] = fmaf(-fs, dz, fz[k]);
      if (ENERGY == 1 && in) {
        ec += (double)(qq * (pt * ex) * rinv);
        el += (double)elj;
      }
      if (ENERGY == 2 && ((e >> k) & 1u))
        pair_energy_fp64(g, *Bw, base, I.ai[ii], permw[s], I.lig[ii], ligj, I.sig[ii], pj.x, I.eps[ii],
                         fabsf(pj.y), lam_e, lam_v, ec, el);
    }
  }
}

// An excluded pair's reciprocal-space removal -KE q_a q_b erf(alpha r)/r in
// FP64 (its r -> 0 limit -KE q_a q_b 2 alpha / sqrt(pi) below 1e-6 A)
__device__ __attribute__((noinline)) double excl_energy_fp64(const LegDev& g, const BoxW& B, size_t oa, size_t ob,
                                                             double qa, double qb) {
#pragma clang fp contract(off)
  double dx = (double)g.x[ob] - (double)g.x[oa], dy = (double)g.y[ob] - (double)g.y[oa];
  double dz = (double)g.z[ob] - (double)g.z[oa];
  dx = dx - B.L[0] * rint(dx * B.invL[0]);
  dy = dy - B.L[1] * rint(dy * B.invL[1]);
  dz = dz - B.L[2] * rint(dz * B.invL[2]);
  const double r = sqrt((dx * dx + dy * dy) + dz * dz);
  const double qq = kKE * qa * qb;
  if (r < 1e-6) return -qq * 2.0 * g.alphad * 0.56418958354775628;
  return -qq * erf(g.alphad * r) / r;
}

template <int ENERGY>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(5))) void k_pairs(const LegDev* legs,
                                                                                      BlockMap map, int step) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const long long item = (long long)(blockIdx.x - map.start[leg]) * 4 + wave;
  if (item >= (long long)g.W * g.nclus) return;
  const int w = (int)(item / g.nclus);
  const int c = (int)(item - (long long)w * g.nclus);
  const gptr<f32x4> xq = as_global4(g.xyzq + (size_t)w * g.npad);
  const gptr<f32x2> pr = as_global2(g.prm + (size_t)w * g.npad);
  const BoxF B = box_f(g.box[w]);
  const float lam_v = g.lam[4 * w + 1];
  const float a_sc = g.lam[4 * w + 3];
  const float lam_e = g.lam[4 * w];
  const bool soft_window = lam_v < 1.0f;
  const BoxW* Bw = &g.box[w];
  const int* permw = g.perm + (size_t)w * g.npad;

  // i-atoms: images nearest the cluster's first atom (always a real atom:
  // padding only follows the last atom), and the cluster's extent
  ICluster I;
  float ext[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int ii = 0; ii < kClus; ++ii) {
    const f32x4 a = xq[c * kClus + ii];
    const f32x2 p = pr[c * kClus + ii];
    float v[3] = {uniform(a.x), uniform(a.y), uniform(a.z)};
    if (ii > 0) {
      const float r0[3] = {I.x[0], I.y[0], I.z[0]};
      for (int d = 0; d < 3; ++d) {
        v[d] = fmaf(-B.L[d], rintf((v[d] - r0[d]) * B.iL[d]), v[d]);
        if (c * kClus + ii < g.n) ext[d] = fmaxf(ext[d], fabsf(v[d] - r0[d]));
      }
    }
    if (ENERGY == 2) I.ai[ii] = __builtin_amdgcn_readfirstlane(g.perm[(size_t)w * g.npad + c * kClus + ii]);
    I.x[ii] = v[0]; I.y[ii] = v[1]; I.z[ii] = v[2];
    I.q[ii] = uniform(a.w);
    I.sig[ii] = uniform(p.x);
    I.eps[ii] = uniform(fabsf(p.y));
    I.lig[ii] = uniform((__float_as_uint(p.y) >> 31) ? 1.0f : 0.0f);
  }
  const float rc = sqrtf(g.rc2) + 0.01f;
  const bool shift = rc + ext[0] < 0.5f * B.L[0] && rc + ext[1] < 0.5f * B.L[1] && rc + ext[2] < 0.5f * B.L[2];
  bool inside = shift;
  for (int d = 0; d < 3; ++d) {
    const float x0 = d == 0 ? I.x[0] : (d == 1 ? I.y[0] : I.z[0]);
    inside = inside && x0 - ext[d] - rc >= 0.0f && x0 + ext[d] + rc < B.L[d];
  }
  const int img = inside ? 2 : (shift ? 1 : 0);
  const size_t base = (size_t)w * g.n;
  // the two half-cluster lists (partners of atoms 0-3, then of atoms 4-7);
  // each half's forces are reduced over the wave before the next half
  const gptr<unsigned> ent = as_global(g.lent + (size_t)item * 2 * g.cap);
  double ec = 0.0, el = 0.0;
  __shared__ float s_f[4][kClus][3];                  // per wave: the 8 atoms' pair forces
#pragma unroll
  for (int half = 0; half < 2; ++half) {
    float fx[4] = {0.f, 0.f, 0.f, 0.f}, fy[4] = {0.f, 0.f, 0.f, 0.f}, fz[4] = {0.f, 0.f, 0.f, 0.f};
    const gptr<unsigned> eh = ent + half * g.cap;
    const int cnt = g.lcount[2 * item + half];
#define FELIS_SWEEP(M, H) sweep<ENERGY, M, H>(g, B, I, eh, cnt, xq, pr, lane, lam_v, a_sc, soft_window, fx, fy, fz, ec, el, Bw, lam_e, permw, base)
    if (half == 0) {
      if (img == 2) FELIS_SWEEP(2, 0);
      else if (img == 1) FELIS_SWEEP(1, 0);
      else FELIS_SWEEP(0, 0);
    } else {
      if (img == 2) FELIS_SWEEP(2, 1);
      else if (img == 1) FELIS_SWEEP(1, 1);
      else FELIS_SWEEP(0, 1);
    }
#undef FELIS_SWEEP
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float sx = wave_sum(fx[k]), sy = wave_sum(fy[k]), sz = wave_sum(fz[k]);
      if (lane == 0) {
        s_f[wave][4 * half + k][0] = sx;
        s_f[wave][4 * half + k][1] = sy;
        s_f[wave][4 * half + k][2] = sz;
      }
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();

  // Excluded pairs: remove their reciprocal-space (erf) interaction, each
  // pair from both of its sides; lane = ii + 8 k takes the k-th exclusion of
  // i-atom ii (at most kMaxExcl = 8 per atom).
  const int ai = g.perm[(size_t)w * g.npad + c * kClus + (lane & 7)];
  float cx = 0.f, cy = 0.f, cz = 0.f;
  double ex = 0.0;
  if (ai >= 0) {
    const int e0 = g.excl_ptr[ai], ne = min(g.excl_ptr[ai + 1] - e0, kMaxExcl);
    const int k = lane >> 3;
    if (k < ne) {
      const int b = g.excl_idx[e0 + k];
      const float le = g.lam[4 * w];
      const float qa = window_charge(g, ai, le), qb = window_charge(g, b, le);
      const size_t oa = (size_t)w * g.n + ai, ob = (size_t)w * g.n + b;
      float3 d = make_float3(g.x[ob] - g.x[oa], g.y[ob] - g.y[oa], g.z[ob] - g.z[oa]);
      d.x = fmaf(-B.L[0], rintf(d.x * B.iL[0]), d.x);
      d.y = fmaf(-B.L[1], rintf(d.y * B.iL[1]), d.y);
      d.z = fmaf(-B.L[2], rintf(d.z * B.iL[2]), d.z);
      const float r2 = d.x * d.x + d.y * d.y + d.z * d.z;
      const float qq = (float)kKE * qa * qb;
      const float c2a = 2.0f * g.alpha * 0.56418958354775628f;
      float fs, en;
      if (r2 > 1e-8f) {
        const float r = sqrtf(r2), rinv = 1.0f / r;
        const float erfv = erff(g.alpha * r);
        en = -qq * erfv * rinv;
        fs = qq * (c2a * __expf(-g.alpha * g.alpha * r2) - erfv * rinv) * rinv * rinv;
      } else {
        en = -qq * c2a;
        fs = 0.f;
      }
      cx = -fs * d.x; cy = -fs * d.y; cz = -fs * d.z;      // F_i = fs (r_i - r_j)
      ex = 0.5 * (double)en;
      if (ENERGY == 2)
        ex = 0.5 * excl_energy_fp64(g, g.box[w], oa, ob, window_charge_fp64(g, ai, (double)le),
                                    window_charge_fp64(g, b, (double)le));
    }
  }
  for (int o = 8; o < 64; o <<= 1) {
    cx += __shfl_xor(cx, o, 64);
    cy += __shfl_xor(cy, o, 64);
    cz += __shfl_xor(cz, o, 64);
  }
  float ox = cx, oy = cy, oz = cz;
  if (lane < kClus) { ox += s_f[wave][lane][0]; oy += s_f[wave][lane][1]; oz += s_f[wave][lane][2]; }
  if (lane < kClus) {
    const int a = ai;
    if (a >= 0) {
      const size_t o = (size_t)w * g.n + a;
      if (step && g.plain) {
        // the plain form: FP64 atomics into the leg's FP64 sums
        const size_t wn = (size_t)g.W * g.n;
        unsafeAtomicAdd(&g.fd[o], (double)ox);
        unsafeAtomicAdd(&g.fd[wn + o], (double)oy);
        unsafeAtomicAdd(&g.fd[2 * wn + o], (double)oz);
      } else {
        const int where = (w << 20) | a;
        g.fx[o] = to_fixed((double)ox, kForceScale, g.err, kSitePairs, where, g.leg_index);
        g.fy[o] = to_fixed((double)oy, kForceScale, g.err, kSitePairs, where, g.leg_index);
        g.fz[o] = to_fixed((double)oz, kForceScale, g.err, kSitePairs, where, g.leg_index);
      }
    }
  }
  if (ENERGY) {
    ec = wave_sum(ec);
    el = wave_sum(el);
    ex = wave_sum(ex);
    if (lane == 0) {
      long long* acc = g.eacc + (size_t)w * FELIS_NE;
      atomicAdd((unsigned long long*)&acc[FELIS_E_COUL_REAL],
                (unsigned long long)to_fixed(0.5 * ec, kEnergyScale, g.err, kSitePairsE, w));
      atomicAdd((unsigned long long*)&acc[FELIS_E_LJ],
                (unsigned long long)to_fixed(0.5 * el, kEnergyScale, g.err, kSitePairsE, w));
      atomicAdd((unsigned long long*)&acc[FELIS_E_EXCL],
                (unsigned long long)to_fixed(ex, kEnergyScale, g.err, kSitePairsE, w));
    }
  }
}

__device__ __forceinline__ void add_force(const LegDev& g, size_t o, float fx, float fy, float fz, int site) {
  const int where = (int)(((o / g.n) << 20) | (o % g.n));     // window << 20 | atom
  atomicAdd((unsigned long long*)&g.fx[o], (unsigned long long)to_fixed((double)fx, kForceScale, g.err, site, where, g.leg_index));
  atomicAdd((unsigned long long*)&g.fy[o], (unsigned long long)to_fixed((double)fy, kForceScale, g.err, site, where, g.leg_index));
  atomicAdd((unsigned long long*)&g.fz[o], (unsigned long long)to_fixed((double)fz, kForceScale, g.err, site, where, g.leg_index));
}

__device__ __forceinline__ void add_energy(const LegDev& g, int w, int comp, double e, int lane) {
  e = wave_sum(e);
  if (lane == 0)
    atomicAdd((unsigned long long*)&g.eacc[(size_t)w * FELIS_NE + comp],
              (unsigned long long)to_fixed(e, kEnergyScale, g.err, kSiteEnergy, comp));
}


// one block per window: Ewald self term and neutralising background
__global__ __launch_bounds__(256) void k_self(const LegDev* legs, BlockMap map) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const int w = blockIdx.x - map.start[leg];
  const double le = (double)g.lam[4 * w];
  double s1 = 0.0, s2 = 0.0;
  for (int a = threadIdx.x; a < g.n; a += blockDim.x) {
    const double q = window_charge_fp64(g, a, le);
    s1 += q; s2 += q * q;
  }
  __shared__ double r1[256], r2[256];
  r1[threadIdx.x] = s1; r2[threadIdx.x] = s2;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) { r1[threadIdx.x] += r1[threadIdx.x + s]; r2[threadIdx.x] += r2[threadIdx.x + s]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double e = -(double)g.self_pref * r2[0] - g.box[w].bg_pref * r1[0] * r1[0];
    atomicAdd((unsigned long long*)&g.eacc[(size_t)w * FELIS_NE + FELIS_E_SELF],
              (unsigned long long)to_fixed(e, kEnergyScale, g.err));
  }
}

__device__ __forceinline__ float3 vec(const LegDev& g, const BoxW& B, size_t ofrom, size_t oto) {
  return min_img(B, g.x[oto] - g.x[ofrom], g.y[oto] - g.y[ofrom], g.z[oto] - g.z[ofrom]);
}

// Torsion t's energy in FP64 from the raw coordinates (consistent images
// relative to its first atom)
__device__ __attribute__((noinline)) double torsion_energy_at(const LegDev& g, int w, int t) {
  const BoxW& B = g.box[w];
  const size_t base = (size_t)w * g.n, o0 = base + g.tors[4 * t];
  double p[4][3];
  for (int s = 0; s < 4; ++s) {
    const size_t os = base + g.tors[4 * t + s];
    double d[3] = {(double)g.x[os] - (double)g.x[o0], (double)g.y[os] - (double)g.y[o0],
                   (double)g.z[os] - (double)g.z[o0]};
    for (int c = 0; c < 3; ++c) p[s][c] = d[c] - B.L[c] * rint(d[c] * B.invL[c]);
  }
  return torsion_energy_fp64(p, (double)g.tors_k[t], g.tors_n[t], (double)g.tors_phase[t]);
}

// items: window x (bonds + torsions + 1): harmonic bonds, lambda_vdw-scaled
// rotatable torsions (section "Double annihilation protocol"); the last item
// of a window is the lambda_restraint-scaled Boresch restraint (section
// "Restraints").
// A bond's energy (k/2)(r - r0)^2 with r in FP64 from the raw coordinates
__device__ __attribute__((noinline)) double bond_energy_fp64(const LegDev& g, const BoxW& B, size_t oa, size_t ob,
                                                             int k) {
  double d[3] = {(double)g.x[oa] - (double)g.x[ob], (double)g.y[oa] - (double)g.y[ob],
                 (double)g.z[oa] - (double)g.z[ob]};
  for (int t = 0; t < 3; ++t) d[t] -= B.L[t] * rint(d[t] * B.invL[t]);
  const double dr = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) - (double)g.bond_r0[k];
  return 0.5 * (double)g.bond_k[k] * dr * dr;
}

// The unscaled Boresch energy in FP64 (anchor positions relative to P1, minimum image)
__device__ __attribute__((noinline)) double restraint_energy_fp64(const LegDev& g, int w) {
  const BoxW& B = g.box[w];
  const size_t base = (size_t)w * g.n, o1 = base + g.ranch[0];
  double p[6][3];
  for (int t = 0; t < 6; ++t) {
    const size_t ot = base + g.ranch[t];
    double d[3] = {(double)g.x[ot] - (double)g.x[o1], (double)g.y[ot] - (double)g.y[o1],
                   (double)g.z[ot] - (double)g.z[o1]};
    for (int c = 0; c < 3; ++c) p[t][c] = d[c] - B.L[c] * rint(d[c] * B.invL[c]);
  }
  return boresch_energy_fp64(p, g.rg0d, g.rkd);
}

template <int ENERGY>
__global__ __launch_bounds__(256) void k_bonded(const LegDev* legs, BlockMap map) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const long long i = (long long)(blockIdx.x - map.start[leg]) * blockDim.x + threadIdx.x;
  const int per = g.nbonds + g.ntors + 1;
  const long long tot = (long long)g.W * per;
  const int lane = threadIdx.x & 63;
  double eb = 0.0, er = 0.0;
  const int w = (int)(min(i, tot - 1) / per);
  if (i < tot) {
    const int k = (int)(i - (long long)w * per);
    const size_t base = (size_t)w * g.n;
    if (k < g.nbonds) {
      const int a = g.bond_ij[2 * k], b = g.bond_ij[2 * k + 1];
      const float3 d = vec(g, g.box[w], base + b, base + a);          // r_a - r_b
      const float r = sqrtf(d.x * d.x + d.y * d.y + d.z * d.z);
      const float dr = r - g.bond_r0[k];
      const float fs = -g.bond_k[k] * dr / r;                // F_a = fs (r_a - r_b)
      add_force(g, base + a, fs * d.x, fs * d.y, fs * d.z, kSiteBonded);
      add_force(g, base + b, -fs * d.x, -fs * d.y, -fs * d.z, kSiteBonded);
      eb = ENERGY == 2 ? bond_energy_fp64(g, g.box[w], base + a, base + b, k)
                       : 0.5 * (double)g.bond_k[k] * (double)dr * (double)dr;
    } else if (k < g.nbonds + g.ntors) {
      const int t = k - g.nbonds;
      const float lv = g.lam[4 * w + 1];
      if (lv != 0.0f) {
        v3 p[4], F[4];
        const size_t o0 = base + g.tors[4 * t];
        for (int s = 0; s < 4; ++s) {
          const size_t os = base + g.tors[4 * t + s];
          const float3 d = min_img(g.box[w], g.x[os] - g.x[o0], g.y[os] - g.y[o0], g.z[os] - g.z[o0]);
          p[s] = mk(d.x, d.y, d.z);
        }
        const float e = torsion_eval(p, g.tors_k[t], g.tors_n[t], g.tors_phase[t], F);
        for (int s = 0; s < 4; ++s)
          add_force(g, base + g.tors[4 * t + s], lv * F[s].x, lv * F[s].y, lv * F[s].z, kSiteBonded);
        eb = (double)lv * (ENERGY == 2 ? torsion_energy_at(g, w, t) : (double)e);
      }
    } else if (g.has_rest && g.lam[4 * w + 2] != 0.0f) {
      const float lr = g.lam[4 * w + 2];
      v3 p[6], F[6];
      const size_t o1 = base + g.ranch[0];
      for (int t = 0; t < 6; ++t) {
        const size_t ot = base + g.ranch[t];
        const float3 d = min_img(g.box[w], g.x[ot] - g.x[o1], g.y[ot] - g.y[o1], g.z[ot] - g.z[o1]);
        p[t] = mk(d.x, d.y, d.z);
      }
      er = (double)lr * boresch_eval(p, g.rg0, g.rk, F);
      if (ENERGY == 2) er = (double)lr * restraint_energy_fp64(g, w);
      for (int t = 0; t < 6; ++t)
        add_force(g, base + g.ranch[t], lr * F[t].x, lr * F[t].y, lr * F[t].z, kSiteBonded);
    }
  }
  if (ENERGY) {
    const int w0 = __shfl(w, 0, 64);
    const bool same = __ballot(i < tot && w != w0) == 0ull;
    if (same) {
      add_energy(g, w0, FELIS_E_BOND, eb, lane);
      add_energy(g, w0, FELIS_E_RESTRAINT, er, lane);
    } else if (i < tot) {
      long long* acc = g.eacc + (size_t)w * FELIS_NE;
      atomicAdd((unsigned long long*)&acc[FELIS_E_BOND], (unsigned long long)to_fixed(eb, kEnergyScale, g.err));
      atomicAdd((unsigned long long*)&acc[FELIS_E_RESTRAINT], (unsigned long long)to_fixed(er, kEnergyScale, g.err));
    }
  }
}

// items: window -- zero energy accumulators [c0, c1)
__global__ void k_ezero(const LegDev* legs, BlockMap map, int c0, int c1) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const int w = (blockIdx.x - map.start[leg]) * blockDim.x + threadIdx.x;
  if (w >= g.W) return;
  for (int c = c0; c < c1; ++c) g.eacc[(size_t)w * FELIS_NE + c] = 0;
}

// items: window -- publish components [c0, c1) and the total
__global__ void k_efinish(const LegDev* legs, BlockMap map, int c0, int c1) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const int w = (blockIdx.x - map.start[leg]) * blockDim.x + threadIdx.x;
  if (w >= g.W) return;
  double* e = g.energy + (size_t)w * FELIS_NE;
  for (int c = c0; c < c1; ++c) e[c] = (double)g.eacc[(size_t)w * FELIS_NE + c] * (1.0 / kEnergyScale);
  double t = 0.0;
  for (int c = 0; c < FELIS_E_TOTAL; ++c) t += e[c];
  e[FELIS_E_TOTAL] = t;
}

__global__ void k_fill_i64(long long* p, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

inline int blocks_for(long long items, int per) { return (int)((items + per - 1) / per); }

}  // namespace

void launch_pack(hipStream_t s, const LegDev* d, const LegHost* h, int nl, bool rebuild) {
  BlockMap m;
  const int nb = make_map(m, nl, [&](int i) { return (int)(((long long)h[i].W * h[i].npad + 255) / 256); });
  if (!nb) return;
  if (rebuild) hipLaunchKernelGGL(k_pack<true>, dim3(nb), dim3(256), 0, s, d, m);
  else hipLaunchKernelGGL(k_pack<false>, dim3(nb), dim3(256), 0, s, d, m);
}

void launch_pairs(hipStream_t s, const LegDev* d, const LegHost* h, int nl, int energy, bool step) {
  BlockMap m;
  const int nb = make_map(m, nl, [&](int i) { return blocks_for((long long)h[i].W * h[i].nclus, 4); });
  if (!nb) return;
  const int st = step ? 1 : 0;
  if (energy == 2) hipLaunchKernelGGL(k_pairs<2>, dim3(nb), dim3(256), 0, s, d, m, 0);
  else if (energy == 1) hipLaunchKernelGGL(k_pairs<1>, dim3(nb), dim3(256), 0, s, d, m, 0);
  else hipLaunchKernelGGL(k_pairs<0>, dim3(nb), dim3(256), 0, s, d, m, st);
}

void launch_corrections(hipStream_t s, const LegDev* d, const LegHost* h, int nl, bool energy) {
  BlockMap m;
  if (energy) {             // excluded-pair corrections are part of the pair kernel
    const int nb = make_map(m, nl, [&](int i) { return h[i].W; });
    if (nb) hipLaunchKernelGGL(k_self, dim3(nb), dim3(256), 0, s, d, m);
  }
}

void launch_bonded(hipStream_t s, const LegDev* d, const LegHost* h, int nl, int energy) {
  BlockMap m;
  const int nb = make_map(m, nl, [&](int i) { return blocks_for((long long)h[i].W * (h[i].nbonds + h[i].ntors + 1), 256); });
  if (!nb) return;
  if (energy == 2) hipLaunchKernelGGL(k_bonded<2>, dim3(nb), dim3(256), 0, s, d, m);
  else if (energy == 1) hipLaunchKernelGGL(k_bonded<1>, dim3(nb), dim3(256), 0, s, d, m);
  else hipLaunchKernelGGL(k_bonded<0>, dim3(nb), dim3(256), 0, s, d, m);
}

void launch_zero_energy(hipStream_t s, const LegDev* d, const LegHost* h, int nl, int c0, int c1) {
  BlockMap m;
  const int nb = make_map(m, nl, [&](int i) { return blocks_for(h[i].W, 64); });
  if (nb) hipLaunchKernelGGL(k_ezero, dim3(nb), dim3(64), 0, s, d, m, c0, c1);
}

void launch_finish_energy(hipStream_t s, const LegDev* d, const LegHost* h, int nl, int c0, int c1) {
  BlockMap m;
  const int nb = make_map(m, nl, [&](int i) { return blocks_for(h[i].W, 64); });
  if (nb) hipLaunchKernelGGL(k_efinish, dim3(nb), dim3(64), 0, s, d, m, c0, c1);
}

void launch_fill_i64(hipStream_t s, long long* p, size_t n) {
  if (n) hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
}

}  // namespace felis
