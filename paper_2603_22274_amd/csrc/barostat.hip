// Monte Carlo barostat (section "Simulation protocol": NPT at 1.01325 bar,
// a volume move every 25 MD steps).  Every window (replica) of a leg with a
// pressure has its own box and makes its own isotropic move:
//   V' = V + dV_max (2 u1 - 1),  s = (V'/V)^(1/3),  L' = s L;
//   each molecule moves rigidly so that its centre (mean atom position) goes
//   from c to s c;
//   w = U(x', L') - U(x, L) + P (V' - V) - N_mol kT ln(V'/V), accepted when
//   w <= 0 or u2 < exp(-w / kT); a rejected move restores x and L;
//   dV_max is divided by 1.1 after a block of 10 attempts with fewer than a
//   quarter accepted and multiplied by 1.1 (at most 0.3 V) with more than
//   three quarters.
// u1, u2 come from Philox4x32-10 with counter (window, 0x4241524F, attempt)
// and the leg's seed as key.  The energies are the library's own window
// totals, evaluated before and after the trial move.
#include "felis_internal.h"

#include <cmath>

namespace felis {
namespace {

constexpr unsigned kBaroTag = 0x4241524Fu;

__device__ __forceinline__ void baro_uniforms(int w, long long attempt, unsigned long long seed, double* u1,
                                              double* u2) {
  unsigned r[4] = {(unsigned)w, kBaroTag, (unsigned)(attempt & 0xffffffffll),
                    (unsigned)((unsigned long long)attempt >> 32)};
  philox(r, (unsigned)(seed & 0xffffffffull), (unsigned)(seed >> 32));
  *u1 = ((double)(r[0] >> 5) * 67108864.0 + (double)(r[1] >> 6)) * (1.0 / 9007199254740992.0);
  *u2 = ((double)(r[2] >> 5) * 67108864.0 + (double)(r[3] >> 6)) * (1.0 / 9007199254740992.0);
}

// items: leg x window (one thread each)
__global__ __launch_bounds__(64) void k_baro_propose(const LegDev* legs, BlockMap map, BaroArgs A) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const int w = (blockIdx.x - map.start[leg]) * blockDim.x + threadIdx.x;
  if (w >= g.W) return;
  BaroW& b = g.baro[w];
  b.due = A.due[leg];
  if (!b.due) return;
  double u1, u2;
  baro_uniforms(w, A.attempt[leg], A.seed[leg], &u1, &u2);
  const BoxW old = g.box[w];
  const double v_new = old.vol + b.dv_max * (2.0 * u1 - 1.0);
  b.vol_old = old.vol;
  b.vol_new = v_new;
  b.scale = v_new > 0.0 ? cbrt(v_new / old.vol) : 1.0;
  g.boxb[w] = old;
  if (v_new > 0.0) {
    const double L[3] = {b.scale * old.L[0], b.scale * old.L[1], b.scale * old.L[2]};
    g.box[w] = make_box(L, (double)g.alpha);
  }
  b.used_old = g.skin_used[w];
}

// items: leg x window x molecule, one wave each: the molecule's centre in FP64
// (lanes over its atoms, fixed reduction tree), then every atom saved and
// moved by (s - 1) c, its list reference position with it (the displacement
// since the last build is unchanged), and the molecule's radius recorded
__global__ __launch_bounds__(256) void k_baro_scale(const LegDev* legs, BlockMap map) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const long long item = (long long)(blockIdx.x - map.start[leg]) * 4 + (threadIdx.x >> 6);
  if (item >= (long long)g.W * g.nmol) return;
  const int w = (int)(item / g.nmol);
  const int mo = (int)(item - (long long)w * g.nmol);
  const BaroW& b = g.baro[w];
  if (!b.due) return;
  const int lane = threadIdx.x & 63;
  const int a0 = g.mol_ptr[mo], a1 = g.mol_ptr[mo + 1];
  const size_t o = (size_t)w * g.n;
  double cx = 0.0, cy = 0.0, cz = 0.0;
  for (int k = a0 + lane; k < a1; k += 64) {
    const int a = g.mol_atoms[k];
    cx += (double)g.x[o + a]; cy += (double)g.y[o + a]; cz += (double)g.z[o + a];
  }
  cx = wave_sum(cx); cy = wave_sum(cy); cz = wave_sum(cz);
  const double inv_n = 1.0 / (double)(a1 - a0);
  const double f = (b.scale - 1.0) * inv_n;
  const double dx = f * cx, dy = f * cy, dz = f * cz;
  const double mx = cx * inv_n, my = cy * inv_n, mz = cz * inv_n;
  float rm = 0.f;
  for (int k = a0 + lane; k < a1; k += 64) {
    const int a = g.mol_atoms[k];
    const float x = g.x[o + a], y = g.y[o + a], z = g.z[o + a];
    const double ex = (double)x - mx, ey = (double)y - my, ez = (double)z - mz;
    rm = fmaxf(rm, (float)sqrt(ex * ex + ey * ey + ez * ez));
    g.xb[o + a] = x; g.yb[o + a] = y; g.zb[o + a] = z;
    g.x[o + a] = (float)((double)x + dx);
    g.y[o + a] = (float)((double)y + dy);
    g.z[o + a] = (float)((double)z + dz);
    g.xr[o + a] = (float)((double)g.xr[o + a] + dx);
    g.yr[o + a] = (float)((double)g.yr[o + a] + dy);
    g.zr[o + a] = (float)((double)g.zr[o + a] + dz);
  }
  for (int off = 32; off > 0; off >>= 1) rm = fmaxf(rm, __shfl_xor(rm, off, 64));
  if (lane == 0) g.molr[item] = rm;
}

// one block per (leg, window): skin used by the trial move, |s - 1| (r_list +
// 2 r_mol + skin), r_mol the largest molecule radius (the bound that keeps
// the lists and cells of the last build valid)
__global__ __launch_bounds__(256) void k_baro_budget(const LegDev* legs, BlockMap map) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const int w = blockIdx.x - map.start[leg];
  const BaroW& b = g.baro[w];
  if (!b.due) return;                            // uniform over the block
  float rm = 0.f;
  for (int m = threadIdx.x; m < g.nmol; m += blockDim.x) rm = fmaxf(rm, g.molr[(size_t)w * g.nmol + m]);
  for (int off = 32; off > 0; off >>= 1) rm = fmaxf(rm, __shfl_xor(rm, off, 64));
  __shared__ float s_m[4];
  if ((threadIdx.x & 63) == 0) s_m[threadIdx.x >> 6] = rm;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double rmol = (double)fmaxf(fmaxf(s_m[0], s_m[1]), fmaxf(s_m[2], s_m[3])) * 1.0001 + 1e-4;
    g.skin_used[w] += (float)(fabs(b.scale - 1.0) * (g.rlist + 2.0 * rmol + (double)g.skin) * 1.001);
  }
}

// items: leg x window: the energy before the move
__global__ __launch_bounds__(64) void k_baro_keep_u0(const LegDev* legs, BlockMap map) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const int w = (blockIdx.x - map.start[leg]) * blockDim.x + threadIdx.x;
  if (w >= g.W) return;
  g.baro[w].u0 = g.energy[(size_t)w * FELIS_NE + FELIS_E_TOTAL];
}

// items: leg x window: Metropolis test; a rejected window gets its box back
// (positions by k_baro_restore) and a list rebuild at the next check
__global__ __launch_bounds__(64) void k_baro_accept(const LegDev* legs, BlockMap map, BaroArgs A) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const int w = (blockIdx.x - map.start[leg]) * blockDim.x + threadIdx.x;
  if (w >= g.W) return;
  BaroW& b = g.baro[w];
  if (!b.due) return;
  double u1, u2;
  baro_uniforms(w, A.attempt[leg], A.seed[leg], &u1, &u2);
  b.u1 = g.energy[(size_t)w * FELIS_NE + FELIS_E_TOTAL];
  const double kT = A.kT;
  bool ok = false;
  double work = INFINITY;
  if (b.vol_new > 0.0) {
    work = (b.u1 - b.u0) + A.pressure[leg] * (b.vol_new - b.vol_old) - (double)g.nmol * kT * log(b.vol_new / b.vol_old);
    ok = work <= 0.0 || u2 < exp(-work / kT);
    if (!(work == work)) ok = false;             // a non-finite energy is never accepted
  }
  b.work = work;
  b.accepted = ok ? 1 : 0;
  b.total_att += 1;
  b.total_acc += ok ? 1 : 0;
  b.n_att += 1;
  b.n_acc += ok ? 1 : 0;
  // lists rebuilt for the trial state (the check of the second energy
  // evaluation found the skin used up) are rebuilt again after a rejection;
  // otherwise the restored state is the one before the move, skin included
  b.rebuilt = g.flag[w];
  if (!ok) {
    g.box[w] = g.boxb[w];
    if (b.rebuilt) g.rbforce[w] = 1;
    else g.skin_used[w] = b.used_old;
  }
  if (b.n_att >= 10) {
    const double vol = g.box[w].vol;
    if (4 * b.n_acc < b.n_att) b.dv_max /= 1.1;
    else if (4 * b.n_acc > 3 * b.n_att) b.dv_max = fmin(b.dv_max * 1.1, 0.3 * vol);
    b.n_att = 0;
    b.n_acc = 0;
  }
}

// items: leg x window x atom: positions of rejected moves back
__global__ __launch_bounds__(256) void k_baro_restore(const LegDev* legs, BlockMap map) {
  const int leg = find_leg(map, blockIdx.x);
  const LegDev& g = legs[leg];
  const long long i = (long long)(blockIdx.x - map.start[leg]) * blockDim.x + threadIdx.x;
  if (i >= (long long)g.W * g.n) return;
  const int w = (int)(i / g.n);
  const BaroW& b = g.baro[w];
  if (!b.due || b.accepted) return;
  if (!b.rebuilt) {                              // the reference moved with the atom: move it back
    g.xr[i] -= g.x[i] - g.xb[i]; g.yr[i] -= g.y[i] - g.yb[i]; g.zr[i] -= g.z[i] - g.zb[i];
  }
  g.x[i] = g.xb[i]; g.y[i] = g.yb[i]; g.z[i] = g.zb[i];
}

inline int blocks_for(long long items, int per) { return (int)((items + per - 1) / per); }

}  // namespace

void launch_baro_propose(hipStream_t s, const LegDev* d, const LegHost* h, int nl, const BaroArgs& A) {
  BlockMap m;
  const int nb = make_map(m, nl, [&](int i) { return h[i].nmol ? blocks_for(h[i].W, 64) : 0; });
  if (nb) hipLaunchKernelGGL(k_baro_propose, dim3(nb), dim3(64), 0, s, d, m, A);
  const int nb2 = make_map(m, nl, [&](int i) { return h[i].nmol ? blocks_for((long long)h[i].W * h[i].nmol, 4) : 0; });
  if (nb2) hipLaunchKernelGGL(k_baro_scale, dim3(nb2), dim3(256), 0, s, d, m);
  const int nb3 = make_map(m, nl, [&](int i) { return h[i].nmol ? h[i].W : 0; });
  if (nb3) hipLaunchKernelGGL(k_baro_budget, dim3(nb3), dim3(256), 0, s, d, m);
}

void launch_baro_keep_u0(hipStream_t s, const LegDev* d, const LegHost* h, int nl) {
  BlockMap m;
  const int nb = make_map(m, nl, [&](int i) { return h[i].nmol ? blocks_for(h[i].W, 64) : 0; });
  if (nb) hipLaunchKernelGGL(k_baro_keep_u0, dim3(nb), dim3(64), 0, s, d, m);
}

void launch_baro_accept(hipStream_t s, const LegDev* d, const LegHost* h, int nl, const BaroArgs& A) {
  BlockMap m;
  const int nb = make_map(m, nl, [&](int i) { return h[i].nmol ? blocks_for(h[i].W, 64) : 0; });
  if (nb) hipLaunchKernelGGL(k_baro_accept, dim3(nb), dim3(64), 0, s, d, m, A);
  const int nb2 = make_map(m, nl, [&](int i) { return h[i].nmol ? blocks_for((long long)h[i].W * h[i].n, 256) : 0; });
  if (nb2) hipLaunchKernelGGL(k_baro_restore, dim3(nb2), dim3(256), 0, s, d, m);
}

}  // namespace felis
