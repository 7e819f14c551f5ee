// Boresch restraint geometry (section "Restraints"), FP32 arithmetic with the
// energy accumulated in FP64.  Anchor slots: 0 P1, 1 P2, 2 P3, 3 L1, 4 L2, 5 L3.
// Terms: distance P1-L1 and angles P1-L1-L2, L1-P1-P2 with (k/2)(g - g0)^2;
// dihedrals P2-P1-L1-L2, P1-L1-L2-L3, L1-P1-P2-P3 with k[1 - cos(g - g0)].
// Angles use atan2(|u x v|, u.v); dihedral(a,b,c,d) = atan2(|b2| b1.(b2 x b3),
// (b1 x b2).(b2 x b3)), b1 = b - a, b2 = c - b, b3 = d - c.
#pragma once

#include "settle.h"   // v3 helpers

namespace felis {

// p[6]: anchor positions already made consistent (minimum image relative to
// P1).  Returns the unscaled energy; if F != nullptr, writes -dE/dp.
__device__ inline double boresch_eval(const v3* p, const float* g0, const float* k, v3* F) {
  double e = 0.0;
  if (F)
    for (int t = 0; t < 6; ++t) F[t] = mk(0.f, 0.f, 0.f);
  {
    const v3 d = vsub(p[0], p[3]);
    const float r = sqrtf(vdot(d, d));
    const float dr = r - g0[0];
    e += 0.5 * (double)k[0] * (double)dr * (double)dr;
    if (F) {
      const v3 gd = vmul(d, k[0] * dr / r);
      F[0] = vsub(F[0], gd);
      F[3] = vadd(F[3], gd);
    }
  }
  const int angs[2][3] = {{0, 3, 4}, {3, 0, 1}};
  for (int t = 0; t < 2; ++t) {
    const int sa = angs[t][0], sb = angs[t][1], sc = angs[t][2];
    const v3 u = vsub(p[sa], p[sb]);
    const v3 v = vsub(p[sc], p[sb]);
    const v3 cr = vcross(u, v);
    const float th = atan2f(sqrtf(vdot(cr, cr)), vdot(u, v));
    const float dth = th - g0[1 + t];
    e += 0.5 * (double)k[1 + t] * (double)dth * (double)dth;
    if (F) {
      const float nu = sqrtf(vdot(u, u)), nv = sqrtf(vdot(v, v));
      const float cs = cosf(th), sn = sinf(th);
      const v3 uh = vmul(u, 1.f / nu), vh = vmul(v, 1.f / nv);
      const v3 ga = vmul(vsub(vmul(uh, cs), vh), 1.f / (nu * sn));
      const v3 gc = vmul(vsub(vmul(vh, cs), uh), 1.f / (nv * sn));
      const float dE = k[1 + t] * dth;
      F[sa] = vsub(F[sa], vmul(ga, dE));
      F[sc] = vsub(F[sc], vmul(gc, dE));
      F[sb] = vadd(F[sb], vmul(vadd(ga, gc), dE));
    }
  }
  const int dih[3][4] = {{1, 0, 3, 4}, {0, 3, 4, 5}, {3, 0, 1, 2}};
  for (int t = 0; t < 3; ++t) {
    const int s0 = dih[t][0], s1 = dih[t][1], s2 = dih[t][2], s3 = dih[t][3];
    const v3 b1 = vsub(p[s1], p[s0]), b2 = vsub(p[s2], p[s1]), b3 = vsub(p[s3], p[s2]);
    const v3 n1 = vcross(b1, b2), n2 = vcross(b2, b3);
    const float nb2 = sqrtf(vdot(b2, b2));
    const float phi = atan2f(nb2 * vdot(b1, n2), vdot(n1, n2));
    const float dphi = phi - g0[3 + t];
    e += (double)k[3 + t] * (1.0 - cos((double)dphi));
    if (F) {
      const v3 ga = vmul(n1, -nb2 / vdot(n1, n1));
      const v3 gd = vmul(n2, nb2 / vdot(n2, n2));
      const float pp = -vdot(b1, b2) / (nb2 * nb2);
      const float qq = -vdot(b3, b2) / (nb2 * nb2);
      const v3 gb = vsub(vmul(ga, pp - 1.f), vmul(gd, qq));
      const v3 gc = vsub(vmul(gd, qq - 1.f), vmul(ga, pp));
      const float dE = k[3 + t] * sinf(dphi);
      F[s0] = vsub(F[s0], vmul(ga, dE));
      F[s1] = vsub(F[s1], vmul(gb, dE));
      F[s2] = vsub(F[s2], vmul(gc, dE));
      F[s3] = vsub(F[s3], vmul(gd, dE));
    }
  }
  return e;
}

// The same energy with every operation in FP64: p[6][3] anchor positions
// relative to P1 (minimum image), g0 and k in the leg's FP64 values.
__device__ inline double boresch_energy_fp64(const double (*p)[3], const double* g0, const double* k) {
  auto sub = [](const double* a, const double* b, double* o) { for (int c = 0; c < 3; ++c) o[c] = a[c] - b[c]; };
  auto dot = [](const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; };
  auto cross = [](const double* a, const double* b, double* o) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
  };
  double e = 0.0, d[3];
  sub(p[0], p[3], d);
  const double dr = sqrt(dot(d, d)) - g0[0];
  e += 0.5 * k[0] * dr * dr;
  const int angs[2][3] = {{0, 3, 4}, {3, 0, 1}};
  for (int t = 0; t < 2; ++t) {
    double u[3], v[3], cr[3];
    sub(p[angs[t][0]], p[angs[t][1]], u);
    sub(p[angs[t][2]], p[angs[t][1]], v);
    cross(u, v, cr);
    const double th = atan2(sqrt(dot(cr, cr)), dot(u, v)) - g0[1 + t];
    e += 0.5 * k[1 + t] * th * th;
  }
  const int dih[3][4] = {{1, 0, 3, 4}, {0, 3, 4, 5}, {3, 0, 1, 2}};
  for (int t = 0; t < 3; ++t) {
    double b1[3], b2[3], b3[3], n1[3], n2[3];
    sub(p[dih[t][1]], p[dih[t][0]], b1);
    sub(p[dih[t][2]], p[dih[t][1]], b2);
    sub(p[dih[t][3]], p[dih[t][2]], b3);
    cross(b1, b2, n1);
    cross(b2, b3, n2);
    const double phi = atan2(sqrt(dot(b2, b2)) * dot(b1, n2), dot(n1, n2));
    e += k[3 + t] * (1.0 - cos(phi - g0[3 + t]));
  }
  return e;
}

// A rotatable torsion k [1 + cos(n phi - delta)] (section "Double
// annihilation protocol": scaled by the caller with lambda_vdw) on four
// atoms with consistent images p[4], phi in the Boresch dihedral's
// convention.  Returns the unscaled energy; if F != nullptr, writes -dE/dp.
__device__ inline float torsion_eval(const v3* p, float k, int n, float delta, v3* F) {
  const v3 b1 = vsub(p[1], p[0]), b2 = vsub(p[2], p[1]), b3 = vsub(p[3], p[2]);
  const v3 n1 = vcross(b1, b2), n2 = vcross(b2, b3);
  const float nb2 = sqrtf(vdot(b2, b2));
  const float phi = atan2f(nb2 * vdot(b1, n2), vdot(n1, n2));
  const float a = (float)n * phi - delta;
  if (F) {
    const v3 ga = vmul(n1, -nb2 / vdot(n1, n1));
    const v3 gd = vmul(n2, nb2 / vdot(n2, n2));
    const float pp = -vdot(b1, b2) / (nb2 * nb2);
    const float qq = -vdot(b3, b2) / (nb2 * nb2);
    const v3 gb = vsub(vmul(ga, pp - 1.f), vmul(gd, qq));
    const v3 gc = vsub(vmul(gd, qq - 1.f), vmul(ga, pp));
    const float mdE = k * (float)n * sinf(a);          // -dE/dphi
    F[0] = vmul(ga, mdE); F[1] = vmul(gb, mdE); F[2] = vmul(gc, mdE); F[3] = vmul(gd, mdE);
  }
  return k * (1.0f + cosf(a));
}

// The same energy with every operation in FP64 (p[4][3] consistent images)
__device__ inline double torsion_energy_fp64(const double (*p)[3], double k, int n, double delta) {
  double b1[3], b2[3], b3[3], n1[3], n2[3];
  for (int c = 0; c < 3; ++c) { b1[c] = p[1][c] - p[0][c]; b2[c] = p[2][c] - p[1][c]; b3[c] = p[3][c] - p[2][c]; }
  n1[0] = b1[1] * b2[2] - b1[2] * b2[1]; n1[1] = b1[2] * b2[0] - b1[0] * b2[2]; n1[2] = b1[0] * b2[1] - b1[1] * b2[0];
  n2[0] = b2[1] * b3[2] - b2[2] * b3[1]; n2[1] = b2[2] * b3[0] - b2[0] * b3[2]; n2[2] = b2[0] * b3[1] - b2[1] * b3[0];
  const double nb2 = sqrt(b2[0] * b2[0] + b2[1] * b2[1] + b2[2] * b2[2]);
  const double phi = atan2(nb2 * (b1[0] * n2[0] + b1[1] * n2[1] + b1[2] * n2[2]),
                           n1[0] * n2[0] + n1[1] * n2[1] + n1[2] * n2[2]);
  return k * (1.0 + cos((double)n * phi - delta));
}

}  // namespace felis
