// Langevin-middle step with SETTLE rigid water (section "Simulation protocol":
// LangevinMiddleIntegrator, rigid TIP3P).  Per window and atom, FP32:
//   v += dt F/m;  waters: v projected on the molecule's rigid-body motions;
//   dx = dt/2 v;  v = a v + sqrt((1 - a^2) kT/m) xi;  dx += dt/2 v;
//   waters: SETTLE on (old, old + dx);  v += (dx_constrained - dx)/dt;  x += dx.
// Displacements are kept relative to the old positions, so the constraint
// solve runs on O(1 A) numbers at full FP32 precision.
// xi: Philox4x32-10 (Salmon et al. 2011) on counter (atom, window, step_lo,
// step_hi) and key (seed_lo, seed_hi); words -> u = ((w >> 8) + 1/2) 2^-24 ->
// Box-Muller: (sqrt(-2 ln u0) cos 2pi u1, sqrt(-2 ln u0) sin 2pi u1,
// sqrt(-2 ln u2) cos 2pi u3).
#include "felis_internal.h"
#include "restraint.h"
#include "settle.h"

namespace felis {
namespace {

__device__ __forceinline__ v3 noise3(unsigned long long seed, int window, long long step, int atom) {
  unsigned c[4] = {(unsigned)atom, (unsigned)window, (unsigned)(step & 0xffffffffll),
                   (unsigned)((unsigned long long)step >> 32)};
  philox(c, (unsigned)(seed & 0xffffffffull), (unsigned)(seed >> 32));
  float u[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) u[k] = ((float)(c[k] >> 8) + 0.5f) * 5.9604644775390625e-8f;
  const float r1 = sqrtf(-2.0f * logf(u[0]));
  const float r2 = sqrtf(-2.0f * logf(u[2]));
  float s1, c1, s2, c2;
  sincospif(2.0f * u[1], &s1, &c1);
  sincospif(2.0f * u[3], &s2, &c2);
  return mk(r1 * c1, r1 * s1, r2 * c2);
}

struct StepArgs {
  long long step[kMaxLegs];
  unsigned long long seed[kMaxLegs];
  float dt, kT, gamma;
};

// Anchor `anchor`'s share of the lambda_r-scaled Boresch restraint force in
// window w (out of line: six atoms per window take this path, and its arrays
// stay out of the integrator's registers)
__device__ __attribute__((noinline)) v3 restraint_share(const LegDev& g, int w, int anchor) {
  const BoxW& B = g.box[w];
  const size_t base = (size_t)w * g.n;
  const size_t o1 = base + g.ranch[0];
  v3 p[6], Fr[6];
  for (int t = 0; t < 6; ++t) {
    const size_t ot = base + g.ranch[t];
    float dx = g.x[ot] - g.x[o1], dy = g.y[ot] - g.y[o1], dz = g.z[ot] - g.z[o1];
    dx = fmaf(-B.Lf[0], rintf(dx * B.invLf[0]), dx);
    dy = fmaf(-B.Lf[1], rintf(dy * B.invLf[1]), dy);
    dz = fmaf(-B.Lf[2], rintf(dz * B.invLf[2]), dz);
    p[t] = mk(dx, dy, dz);
  }
  boresch_eval(p, g.rg0, g.rk, Fr);
  const float lr = g.lam[4 * w + 2];
  v3 F = mk(0.f, 0.f, 0.f);
  for (int t = 0; t < 6; ++t)
    if (g.ranch[t] == g.ranch[anchor]) F = vadd(F, vmul(Fr[t], lr));
  return F;
}

// Atom `slot` of torsion t's share of its lambda_vdw-scaled force in window w
// (out of line, like the restraint share)
__device__ __attribute__((noinline)) v3 torsion_share(const LegDev& g, int w, int t, int slot) {
  const BoxW& B = g.box[w];
  const size_t base = (size_t)w * g.n;
  const size_t o0 = base + g.tors[4 * t];
  v3 p[4], F[4];
  for (int s = 0; s < 4; ++s) {
    const size_t os = base + g.tors[4 * t + s];
    float dx = g.x[os] - g.x[o0], dy = g.y[os] - g.y[o0], dz = g.z[os] - g.z[o0];
    dx = fmaf(-B.Lf[0], rintf(dx * B.invLf[0]), dx);
    dy = fmaf(-B.Lf[1], rintf(dy * B.invLf[1]), dy);
    dz = fmaf(-B.Lf[2], rintf(dz * B.invLf[2]), dz);
    p[s] = mk(dx, dy, dz);
  }
  torsion_eval(p, g.tors_k[t], g.tors_n[t], g.tors_phase[t], F);
  return vmul(F[slot], g.lam[4 * w + 1]);
}

// The bonded terms of atom a in window w: its harmonic bonds (each atom sums
// its own, from the per-atom bond table, in bond order), its lambda_vdw-scaled
// rotatable torsions (per-atom torsion table) and, for a Boresch
// anchor, its share of the lambda_r-scaled restraint -- the forces of
// k_bonded, computed where they are used instead of added by atomics.
__device__ __forceinline__ v3 bonded_force(const LegDev& g, int w, int a) {
  v3 F = mk(0.f, 0.f, 0.f);
  const int k0 = g.bptr[a], k1 = g.bptr[a + 1];
  const int t0 = g.tptr[a], t1 = g.lam[4 * w + 1] != 0.0f ? g.tptr[a + 1] : t0;
  int anchor = -1;
  if (g.has_rest && g.lam[4 * w + 2] != 0.0f)
    for (int t = 0; t < 6; ++t) anchor = (g.ranch[t] == a) ? t : anchor;
  if (k0 == k1 && anchor < 0 && t0 == t1) return F;
  const BoxW& B = g.box[w];
  const size_t base = (size_t)w * g.n;
  auto img = [&](size_t from, size_t to) {        // r_to - r_from, nearest image
    float dx = g.x[to] - g.x[from], dy = g.y[to] - g.y[from], dz = g.z[to] - g.z[from];
    dx = fmaf(-B.Lf[0], rintf(dx * B.invLf[0]), dx);
    dy = fmaf(-B.Lf[1], rintf(dy * B.invLf[1]), dy);
    dz = fmaf(-B.Lf[2], rintf(dz * B.invLf[2]), dz);
    return mk(dx, dy, dz);
  };
  for (int k = k0; k < k1; ++k) {
    const int b = g.bnb[k], id = g.bid[k];
    const v3 d = img(base + b, base + a);           // r_a - r_b
    const float r = sqrtf(d.x * d.x + d.y * d.y + d.z * d.z);
    const float fs = -g.bond_k[id] * (r - g.bond_r0[id]) / r;
    F = vadd(F, vmul(d, fs));
  }
  for (int e = t0; e < t1; ++e) {
    const int te = g.tid[e];
    F = vadd(F, torsion_share(g, w, te >> 2, te & 3));
  }
  if (anchor >= 0) F = vadd(F, restraint_share(g, w, anchor));
  return F;
}

// kick for one atom: returns v + dt F/m.  The total force (real-space terms
// in fx/fy/fz, this step's reciprocal-space term and the bonded terms) is
// stored back, so that fx/fy/fz hold the whole force of the step after the
// call.
__device__ __forceinline__ v3 kick(const LegDev& g, const StepArgs& S, int w, int a) {
  const size_t o = (size_t)w * g.n + a;
  const float acc = (float)kAccel / g.mass[a];
  const v3 fb = bonded_force(g, w, a);
  if (g.plain) {
    // the plain form: the step's pair and reciprocal forces were summed by
    // FP64 atomics; read them, clear the sums for the next step
    const size_t wn = (size_t)g.W * g.n;
    const double sx = g.fd[o] + (double)fb.x, sy = g.fd[wn + o] + (double)fb.y, sz = g.fd[2 * wn + o] + (double)fb.z;
    g.fd[o] = 0.0; g.fd[wn + o] = 0.0; g.fd[2 * wn + o] = 0.0;
    const int where = (w << 20) | a;
    g.fx[o] = to_fixed(sx, kForceScale, g.err, kSiteBonded, where, g.leg_index);
    g.fy[o] = to_fixed(sy, kForceScale, g.err, kSiteBonded, where, g.leg_index);
    g.fz[o] = to_fixed(sz, kForceScale, g.err, kSiteBonded, where, g.leg_index);
    const float dt = S.dt;
    return mk(g.vx[o] + dt * (float)sx * acc, g.vy[o] + dt * (float)sy * acc, g.vz[o] + dt * (float)sz * acc);
  }
  long long tx = g.fx[o] + g.frx[o], ty = g.fy[o] + g.fry[o], tz = g.fz[o] + g.frz[o];
  if (fb.x != 0.f || fb.y != 0.f || fb.z != 0.f) {
    const int where = (w << 20) | a;
    tx += to_fixed((double)fb.x, kForceScale, g.err, kSiteBonded, where, g.leg_index);
    ty += to_fixed((double)fb.y, kForceScale, g.err, kSiteBonded, where, g.leg_index);
    tz += to_fixed((double)fb.z, kForceScale, g.err, kSiteBonded, where, g.leg_index);
  }
  g.fx[o] = tx; g.fy[o] = ty; g.fz[o] = tz;
  const float F[3] = {(float)((double)tx * (1.0 / kForceScale)), (float)((double)ty * (1.0 / kForceScale)),
                      (float)((double)tz * (1.0 / kForceScale))};
  const float dt = S.dt;
  return mk(g.vx[o] + dt * F[0] * acc, g.vy[o] + dt * F[1] * acc, g.vz[o] + dt * F[2] * acc);
}

// half drift, O step, half drift from the post-kick velocity v: returns the
// total displacement and the post-O velocity
__device__ __forceinline__ void drift_o(const LegDev& g, const StepArgs& S, int leg, int w, int a, v3 v, v3& dx,
                                        v3& vel) {
  const float acc = (float)kAccel / g.mass[a];
  const float dt = S.dt;
  const float hd = 0.5f * dt;
  dx = vmul(v, hd);
  const float ea = expf(-S.gamma * dt);
  const float sd = sqrtf((1.0f - ea * ea) * S.kT * acc);
  const v3 xi = noise3(S.seed[leg], w, S.step[leg], a);
  v = vadd(vmul(v, ea), vmul(xi, sd));
  dx = vadd(dx, vmul(v, hd));
  vel = v;
}

__device__ __forceinline__ void advance(const LegDev& g, const StepArgs& S, int leg, int w, int a, v3& dx,
                                        v3& vel) {
  drift_o(g, S, leg, w, a, kick(g, S, w, a), dx, vel);
}

// writes the new position and velocity; returns the squared displacement
// from the position of the window's last list build, in the list check's own
// arithmetic (separately rounded products and sums)
__device__ __forceinline__ float store(const LegDev& g, int w, int a, v3 dx, v3 v) {
  const size_t o = (size_t)w * g.n + a;
  const float x = g.x[o] + dx.x, y = g.y[o] + dx.y, z = g.z[o] + dx.z;
  g.x[o] = x; g.y[o] = y; g.z[o] = z;
  g.vx[o] = v.x; g.vy[o] = v.y; g.vz[o] = v.z;
  const float ex = __fsub_rn(x, g.xr[o]), ey = __fsub_rn(y, g.yr[o]), ez = __fsub_rn(z, g.zr[o]);
  return __fadd_rn(__fadd_rn(__fmul_rn(ex, ex), __fmul_rn(ey, ey)), __fmul_rn(ez, ez));
}

// one unit (a rigid water, or any other atom): Langevin-middle update, SETTLE
// for waters; returns the largest squared displacement since the list build
__device__ __forceinline__ float unit_step(const LegDev& g, const StepArgs& S, int leg, int w, int u) {
  if (u >= g.nwat) {
    const int a = g.free_atoms[u - g.nwat];
    v3 dx, v;
    advance(g, S, leg, w, a, dx, v);
    return store(g, w, a, dx, v);
  }
  const int ao = g.water[3 * u], ah1 = g.water[3 * u + 1], ah2 = g.water[3 * u + 2];
  const size_t base = (size_t)w * g.n;
  const v3 xo = mk(g.x[base + ao], g.y[base + ao], g.z[base + ao]);
  const v3 b0 = vsub(mk(g.x[base + ah1], g.y[base + ah1], g.z[base + ah1]), xo);
  const v3 c0 = vsub(mk(g.x[base + ah2], g.y[base + ah2], g.z[base + ah2]), xo);
  v3 kO = kick(g, S, w, ao), kH1 = kick(g, S, w, ah1), kH2 = kick(g, S, w, ah2);
  rigid_velocity(b0, c0, g.mass[ao], g.mass[ah1], kO, kH1, kH2);
  v3 dO, dH1, dH2, vO, vH1, vH2;
  drift_o(g, S, leg, w, ao, kO, dO, vO);
  drift_o(g, S, leg, w, ah1, kH1, dH1, vH1);
  drift_o(g, S, leg, w, ah2, kH2, dH2, vH2);
  v3 a1 = dO, b1 = vadd(b0, dH1), c1 = vadd(c0, dH2);
  const v3 a1u = a1, b1u = b1, c1u = c1;
  settle(b0, c0, a1, b1, c1, g.mass[ao], g.mass[ah1], g.d_oh, g.d_hh);
  const float idt = 1.0f / S.dt;
  vO = vadd(vO, vmul(vsub(a1, a1u), idt));
  vH1 = vadd(vH1, vmul(vsub(b1, b1u), idt));
  vH2 = vadd(vH2, vmul(vsub(c1, c1u), idt));
  const float m0 = store(g, w, ao, a1, vO);
  const float m1 = store(g, w, ah1, vsub(b1, b0), vH1);
  const float m2 = store(g, w, ah2, vsub(c1, c0), vH2);
  return fmaxf(m0, fmaxf(m1, m2));
}

// items: window x unit (rigid waters first, then every other atom).  Each
// wave also records, for the next step's list check, the largest squared
// displacement in its first window and in its second (a wave of 64 units
// spans at most two windows when a window has at least 64 units; smaller
// windows use one atomic per lane instead).
__global__ __launch_bounds__(256) void k_integrate(const LegDev* legs, BlockMap map, StepArgs S) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const long long i = (long long)(blockIdx.x - map.start[leg]) * blockDim.x + threadIdx.x;
  const int units = g.units;
  const bool valid = i < (long long)g.W * units;
  const int w = valid ? (int)(i / units) : g.W - 1;
  float d2 = 0.f;
  if (valid) d2 = unit_step(g, S, leg, w, (int)(i - (long long)w * units));
  if (units < 64) {
    if (valid) atomicMax(&g.maxdisp[w], __float_as_uint(d2));
    return;
  }
  const int w0 = __shfl(w, 0, 64);
  float a = (w == w0) ? d2 : 0.f, b = (w == w0) ? 0.f : d2;
  for (int k = 32; k > 0; k >>= 1) {
    a = fmaxf(a, __shfl_xor(a, k, 64));
    b = fmaxf(b, __shfl_xor(b, k, 64));
  }
  const long long wave = i >> 6;
  if ((threadIdx.x & 63) == 0 && wave * 64 < (long long)g.W * units) {
    g.wmax[2 * wave] = __float_as_uint(a);
    g.wmax[2 * wave + 1] = __float_as_uint(b);
  }
}

}  // namespace

void launch_integrate(hipStream_t s, const LegDev* d, const LegHost* h, int nl, const long long* step,
                      const unsigned long long* seed, float dt, float temperature, float gamma) {
  BlockMap m;
  const int nb = make_map(m, nl, [&](int i) {
    return (int)(((long long)h[i].W * (h[i].nwat + h[i].nfree) + 255) / 256);
  });
  if (!nb) return;
  StepArgs S;
  for (int i = 0; i < nl; ++i) { S.step[i] = step[i]; S.seed[i] = seed[i]; }
  S.dt = dt;
  S.kT = (float)(kKB * temperature);
  S.gamma = gamma;
  hipLaunchKernelGGL(k_integrate, dim3(nb), dim3(256), 0, s, d, m, S);
}

}  // namespace felis
