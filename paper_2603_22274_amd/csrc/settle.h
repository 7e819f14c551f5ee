// Analytic rigid-water constraint (SETTLE, Miyamoto & Kollman 1992), FP32.
//
// Inputs are positions relative to the old oxygen: old O at the origin,
// old H1/H2 at b0/c0, and the unconstrained new positions a1/b1/c1.  The
// result places the three atoms at the rigid geometry (d_oh, d_hh) with the
// same centre of mass as a1/b1/c1, displaced from them along the old bond
// directions only (zero torque of the constraint forces about the old
// positions), i.e. the converged solution of the SHAKE equations.
//
// Derivation used here: in a frame whose z axis is normal to the old plane
// and whose x axis is perpendicular to the new O position (relative to the
// centre of mass), the constrained molecule is the canonical triangle rotated
// by phi about x, psi about y (fixed by the z coordinates of the new
// positions) and theta about z, where theta solves
//   alpha sin(theta) + beta cos(theta) = gamma,
// the z component of sum_i m_i r0_i x (r3_i - r1_i) = 0.
#pragma once

#ifdef __HIPCC__
#define FELIS_HD __host__ __device__
#else
#define FELIS_HD
#endif

#include <math.h>

namespace felis {

struct v3 {
  float x, y, z;
};

FELIS_HD inline v3 mk(float x, float y, float z) { v3 r; r.x = x; r.y = y; r.z = z; return r; }
FELIS_HD inline v3 vadd(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
FELIS_HD inline v3 vsub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
FELIS_HD inline v3 vmul(v3 a, float s) { return mk(a.x * s, a.y * s, a.z * s); }
FELIS_HD inline float vdot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
FELIS_HD inline v3 vcross(v3 a, v3 b) {
  return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
FELIS_HD inline v3 vnorm(v3 a) { return vmul(a, 1.0f / sqrtf(vdot(a, a))); }

// b0, c0: old H1, H2 relative to the old O (old O = origin).
// a1, b1, c1: new unconstrained O, H1, H2 in the same frame (overwritten).
FELIS_HD inline void settle(v3 b0, v3 c0, v3& a1, v3& b1, v3& c1, float mO, float mH, float d_oh,
                            float d_hh) {
  const float M = mO + 2.0f * mH;
  const float rc = 0.5f * d_hh;
  const float hgt = sqrtf(d_oh * d_oh - rc * rc);          // O to H-H midpoint
  const float ra = 2.0f * mH * hgt / M;                    // COM to O
  const float rb = hgt - ra;                               // COM to H-H midpoint
  const v3 com = vmul(vadd(vmul(a1, mO), vmul(vadd(b1, c1), mH)), 1.0f / M);
  const v3 A1 = vsub(a1, com), B1 = vsub(b1, com), C1 = vsub(c1, com);
  const v3 ez = vnorm(vcross(b0, c0));
  const v3 ex = vnorm(vcross(A1, ez));
  const v3 ey = vcross(ez, ex);
  // old positions (relative to old O) and new positions in the frame
  const float xb0 = vdot(b0, ex), yb0 = vdot(b0, ey);
  const float xc0 = vdot(c0, ex), yc0 = vdot(c0, ey);
  const float za1 = vdot(A1, ez);
  const float xb1 = vdot(B1, ex), yb1 = vdot(B1, ey), zb1 = vdot(B1, ez);
  const float xc1 = vdot(C1, ex), yc1 = vdot(C1, ey), zc1 = vdot(C1, ez);
  // tilt of the canonical triangle out of the xy plane
  const float sphi = za1 / ra;
  const float cphi = sqrtf(fmaxf(0.0f, 1.0f - sphi * sphi));
  const float spsi = (zb1 - zc1) / (2.0f * rc * cphi);
  const float cpsi = sqrtf(fmaxf(0.0f, 1.0f - spsi * spsi));
  const float ya2 = ra * cphi;
  const float xb2 = -rc * cpsi;
  const float yb2 = -rb * cphi - rc * spsi * sphi;
  const float yc2 = -rb * cphi + rc * spsi * sphi;
  // in-plane rotation theta from the zero-torque condition
  const float al = xb2 * (xb0 - xc0) + yb0 * yb2 + yc0 * yc2;
  const float be = xb2 * (yc0 - yb0) + xb0 * yb2 + xc0 * yc2;
  const float ga = xb0 * yb1 - xb1 * yb0 + xc0 * yc1 - xc1 * yc0;
  const float ab2 = al * al + be * be;
  const float sth = (al * ga - be * sqrtf(fmaxf(0.0f, ab2 - ga * ga))) / ab2;
  const float cth = sqrtf(fmaxf(0.0f, 1.0f - sth * sth));
  const float xa3 = -ya2 * sth, ya3 = ya2 * cth;
  const float xb3 = xb2 * cth - yb2 * sth, yb3 = xb2 * sth + yb2 * cth;
  const float xc3 = -xb2 * cth - yc2 * sth, yc3 = -xb2 * sth + yc2 * cth;
  a1 = vadd(com, vadd(vadd(vmul(ex, xa3), vmul(ey, ya3)), vmul(ez, za1)));
  b1 = vadd(com, vadd(vadd(vmul(ex, xb3), vmul(ey, yb3)), vmul(ez, zb1)));
  c1 = vadd(com, vadd(vadd(vmul(ex, xc3), vmul(ey, yc3)), vmul(ez, zc1)));
}

// Velocity constraint of a rigid water after the kick: the mass-weighted
// projection of (vO, vH1, vH2) on the molecule's rigid-body motions,
// v_i = V + omega x r_i with V the centre-of-mass velocity, r_i taken from
// the centre of mass and I omega = L (inertia tensor and angular momentum
// about the centre of mass), which is the velocity that keeps all three
// distances fixed to first order.  b0, c0: H1, H2 relative to O.
FELIS_HD inline void rigid_velocity(v3 b0, v3 c0, float mO, float mH, v3& vO, v3& vH1, v3& vH2) {
  const float M = mO + 2.0f * mH;
  const v3 com = vmul(vadd(b0, c0), mH / M);
  const v3 rO = vmul(com, -1.0f), r1 = vsub(b0, com), r2 = vsub(c0, com);
  const v3 V = vmul(vadd(vmul(vO, mO), vmul(vadd(vH1, vH2), mH)), 1.0f / M);
  const v3 L = vadd(vmul(vcross(rO, vO), mO), vmul(vadd(vcross(r1, vH1), vcross(r2, vH2)), mH));
  // inertia tensor about the centre of mass
  float xx = 0.f, yy = 0.f, zz = 0.f, xy = 0.f, xz = 0.f, yz = 0.f;
  const v3 rr[3] = {rO, r1, r2};
  const float mm[3] = {mO, mH, mH};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const v3 r = rr[k];
    xx += mm[k] * (r.y * r.y + r.z * r.z);
    yy += mm[k] * (r.x * r.x + r.z * r.z);
    zz += mm[k] * (r.x * r.x + r.y * r.y);
    xy -= mm[k] * r.x * r.y;
    xz -= mm[k] * r.x * r.z;
    yz -= mm[k] * r.y * r.z;
  }
  // omega = I^-1 L by the adjugate of the symmetric tensor
  const float c00 = yy * zz - yz * yz, c01 = xz * yz - xy * zz, c02 = xy * yz - xz * yy;
  const float c11 = xx * zz - xz * xz, c12 = xy * xz - xx * yz, c22 = xx * yy - xy * xy;
  const float idet = 1.0f / (xx * c00 + xy * c01 + xz * c02);
  const v3 om = mk((c00 * L.x + c01 * L.y + c02 * L.z) * idet, (c01 * L.x + c11 * L.y + c12 * L.z) * idet,
                   (c02 * L.x + c12 * L.y + c22 * L.z) * idet);
  vO = vadd(V, vcross(om, rO));
  vH1 = vadd(V, vcross(om, r1));
  vH2 = vadd(V, vcross(om, r2));
}

}  // namespace felis
