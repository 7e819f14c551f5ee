// C ABI of the alchemical-window hot path (declarations and documentation in
// include/felis.h).  Host side: argument validation, the per-leg scratch
// layout, device descriptor upload and the launch sequences.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "felis_internal.h"

using namespace felis;

namespace {

struct Layout {
  size_t lam, lamS, rstate, free_atoms, lig_idx, aw_idx, fd, xr, yr, zr, flag, nbuild, maxdisp, wmax, hcell, box, ubox, rbforce, skin_used, bptr, bnb, bid, tptr, tid, mol_ptr, mol_atoms, baro, boxb, xb, yb, zb, molr, perm, cellcode, cellstart, cursor, xyzq, prm, bblo,
      bbhi, gsten, lcount, lent, frx, fry, frz, grid64, cgrid, tw[3], bmod[3], eacc, uacc, upart, lpart, ucst, total;
};

struct Plan {
  LegHost h;
  Layout lay;
  int nbits;
  int nrad[3], rad[3][kMaxRadix];
};

struct Meta {          // facts read from the topology at felis_leg_init
  int nfree, nlig;
  int naw;             // alchemical-water atoms
  int nmol;            // molecules (legs with a barostat; 0 otherwise)
  size_t work_bytes;
};

// HIP events bracketing one kind of launch on the context's stream
struct Timer {
  std::vector<hipEvent_t> ev;     // start, stop, start, stop ...
  size_t used = 0;
  long long seen = 0;             // stage occurrences since profiling was switched on
  bool skip = false;              // the current occurrence is not bracketed
};

}  // namespace

struct felis_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  // felis_step runs reciprocal space on a second stream (default priority)
  // beside the list build and pair kernel; two events fork and join it
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  LegDev* d_legs = nullptr;          // device table of kMaxLegs descriptors
  LegDev* h_stage = nullptr;         // pinned staging
  std::vector<LegDev> cache;         // last uploaded table
  int* d_err = nullptr;              // [0] error bits, [1] largest list length
  unsigned long long* d_count = nullptr;
  std::unordered_map<const void*, Meta> meta;
  std::string last_error;
  int prof = 0;                     // bit t: record events around stage t
  int prof_every = 1;               // bracket every prof_every-th occurrence of a stage
  Timer timers[FELIS_PROF_N];
};

namespace {

int fail(felis_ctx* c, int code, const char* msg) {
  if (c) c->last_error = msg;
  return code;
}

size_t al(size_t v) { return (v + 255) & ~size_t(255); }

bool factor_plan(int K, int* rad, int* nrad) {
  int m = K, n = 0;
  while (m % 8 == 0 && n < kMaxRadix) { rad[n++] = 8; m /= 8; }
  while (m % 12 == 0 && n < kMaxRadix) { rad[n++] = 12; m /= 12; }
  while (m % 4 == 0 && n < kMaxRadix) { rad[n++] = 4; m /= 4; }
  while (m % 2 == 0 && n < kMaxRadix) { rad[n++] = 2; m /= 2; }
  while (m % 3 == 0 && n < kMaxRadix) { rad[n++] = 3; m /= 3; }
  while (m % 5 == 0 && n < kMaxRadix) { rad[n++] = 5; m /= 5; }
  *nrad = n;
  return m == 1;
}

int make_plan(felis_ctx* c, const felis_leg* L, Plan& P) {
  if (!L) return fail(c, FELIS_E_INVAL, "null leg");
  if (L->n_atoms <= 0 || L->n_windows <= 0) return fail(c, FELIS_E_INVAL, "n_atoms and n_windows must be positive");
  if (L->n_atoms >= (1 << 24)) return fail(c, FELIS_E_UNSUPPORTED, "more than 2^24 atoms");
  for (int d = 0; d < 3; ++d)
    if (!(L->box[d] > 0)) return fail(c, FELIS_E_INVAL, "box edges must be positive");
  if (!(L->r_cut > 0) || !(L->skin >= 0) || !(L->ewald_alpha > 0))
    return fail(c, FELIS_E_INVAL, "r_cut, skin, ewald_alpha");
  const double lmin = std::min(L->box[0], std::min(L->box[1], L->box[2]));
  if (!(L->r_cut + L->skin < 0.5 * lmin)) return fail(c, FELIS_E_BOX, "r_cut + skin must be below half the box");
  if (L->sc_p != 1) return fail(c, FELIS_E_UNSUPPORTED, "softcore p must be 1");
  if (!(L->pressure_bar >= 0) || !(L->pressure_bar < 1e6) || (L->pressure_bar > 0 && L->barostat_every < 1))
    return fail(c, FELIS_E_INVAL, "pressure_bar >= 0 and, with a barostat, barostat_every >= 1");
  if (L->spline_order != 4) return fail(c, FELIS_E_UNSUPPORTED, "PME spline order must be 4");
  if (L->plain_fp64 && L->pressure_bar > 0)
    return fail(c, FELIS_E_UNSUPPORTED, "the plain (FP64-atomic) form runs at fixed box only");
  if (!(L->sc_alpha >= 0)) return fail(c, FELIS_E_INVAL, "sc_alpha");
  // the real-space erfc is a fit on [0, 3.5] (Ewald tolerances down to ~4e-7)
  if (!(L->ewald_alpha * L->r_cut <= 3.5))
    return fail(c, FELIS_E_UNSUPPORTED, "ewald_alpha * r_cut must not exceed 3.5");
  if (!L->charge || !L->sigma || !L->epsilon || !L->mass || !L->is_ligand)
    return fail(c, FELIS_E_INVAL, "null parameter array");
  if (!L->x || !L->y || !L->z || !L->vx || !L->vy || !L->vz || !L->fx || !L->fy || !L->fz || !L->energy)
    return fail(c, FELIS_E_INVAL, "null state array");
  if (!L->lambdas) return fail(c, FELIS_E_INVAL, "null lambdas");
  if (L->n_excl < 0 || (L->n_excl > 0 && (!L->excl_ij || !L->excl_ptr || !L->excl_idx)))
    return fail(c, FELIS_E_INVAL, "exclusions");
  if (!L->excl_ptr) return fail(c, FELIS_E_INVAL, "excl_ptr is required");
  if (L->n_bonds < 0 || (L->n_bonds > 0 && (!L->bond_ij || !L->bond_k || !L->bond_r0)))
    return fail(c, FELIS_E_INVAL, "bonds");
  if (L->n_waters < 0 || 3LL * L->n_waters > L->n_atoms || (L->n_waters > 0 && !L->water_ohh))
    return fail(c, FELIS_E_INVAL, "waters");
  if (L->n_torsions < 0 || (L->n_torsions > 0 && (!L->torsion_ijkl || !L->torsion_k || !L->torsion_n ||
                                                   !L->torsion_phase)))
    return fail(c, FELIS_E_INVAL, "torsions");
  if (L->has_restraint)
    for (int t = 0; t < 6; ++t)
      if (L->restraint_atoms[t] < 0 || L->restraint_atoms[t] >= L->n_atoms)
        return fail(c, FELIS_E_INVAL, "restraint atom out of range");
  Plan& p = P;
  LegHost& h = p.h;
  std::memset(&p, 0, sizeof(p));
  h.n = L->n_atoms;
  h.W = L->n_windows;
  h.npad = (h.n + 7) & ~7;
  h.nclus = h.npad / 8;
  const double V = L->box[0] * L->box[1] * L->box[2];
  const double rl = L->r_cut + L->skin;
  h.nexcl = L->n_excl;
  h.nbonds = L->n_bonds;
  h.nwat = L->n_waters;
  h.nfree = h.n - 3 * h.nwat;
  h.has_rest = L->has_restraint ? 1 : 0;
  h.ntors = L->n_torsions;
  for (int d = 0; d < 3; ++d) {
    const int K = L->grid[d];
    if (K < 4 || K > kMaxFFT || !factor_plan(K, p.rad[d], &p.nrad[d]))
      return fail(c, FELIS_E_UNSUPPORTED, "PME grid dimensions must be 2^a 3^b 5^c in [4, 128]");
    h.K[d] = K;
  }
  h.Ktot = h.K[0] * h.K[1] * h.K[2];
  // a barostat gives every window its own box: one window per complex grid
  h.npair = L->pressure_bar > 0 ? h.W : (h.W + 1) / 2;
  int nbits = (int)std::floor(std::log2(lmin / 2.4));
  nbits = std::max(1, std::min(7, nbits));
  p.nbits = nbits;
  h.ncell = 1 << (3 * nbits);
  int cap = L->list_cap;
  if (cap <= 0) {
    const double rho = h.n / V;
    // union of r_list spheres around a half-cluster: four atoms consecutive
    // along the Hilbert curve lie within about one cell edge of their centre
    // (cells are 2.4-4.8 A: a power-of-two split of the box), with 2x room
    // for density fluctuations
    const double cs = std::max(L->box[0], std::max(L->box[1], L->box[2])) / (double)(1 << nbits);
    cap = (int)std::ceil(2.0 * rho * 4.0 / 3.0 * M_PI * std::pow(rl + cs, 3) + 64.0);
  }
  cap = std::min((cap + 7) & ~7, h.npad);
  h.cap = std::max(cap, 8);
  Layout& y = p.lay;
  size_t o = 0;
  auto put = [&](size_t bytes) { size_t r = o; o += al(bytes); return r; };
  const size_t W = h.W, n = h.n, npad = h.npad, nc = h.nclus;
  y.lam = put(W * 4 * sizeof(float));
  y.lamS = put(W * 4 * sizeof(float));
  y.rstate = put(W * 4);
  y.free_atoms = put(n * 4);
  y.lig_idx = put(n * 4);
  y.aw_idx = put(3 * n * 4);
  y.fd = put(L->plain_fp64 ? 3 * W * n * 8 : 0);
  y.hcell = put((size_t)h.ncell * 4);            // filled once at set-up (outside every cleared range)
  y.box = put(W * sizeof(BoxW));                  // set at set-up, changed only by the barostat
  y.ubox = put(2 * (size_t)h.npair * sizeof(BoxW));
  y.rbforce = put(W * 4);
  y.skin_used = put(W * 4);
  y.bptr = put((n + 1) * 4);                      // per-atom bond table (filled at set-up)
  y.bnb = put(2 * (size_t)std::max(h.nbonds, 1) * 4);
  y.bid = put(2 * (size_t)std::max(h.nbonds, 1) * 4);
  y.tptr = put((n + 1) * 4);                      // per-atom torsion table (filled at set-up)
  y.tid = put(4 * (size_t)std::max(h.ntors, 1) * 4);
  {
    // barostat: molecule table, per-window state, positions before a move
    const bool npt = L->pressure_bar > 0;
    y.mol_ptr = put(npt ? (n + 1) * 4 : 0);
    y.mol_atoms = put(npt ? n * 4 : 0);
    y.baro = put(npt ? W * sizeof(BaroW) : 0);
    y.boxb = put(npt ? W * sizeof(BoxW) : 0);
    y.xb = put(npt ? W * n * 4 : 0); y.yb = put(npt ? W * n * 4 : 0); y.zb = put(npt ? W * n * 4 : 0);
    y.molr = put(npt ? W * n * 4 : 0);
  }
  y.xr = put(W * n * 4); y.yr = put(W * n * 4); y.zr = put(W * n * 4);
  y.flag = put(W * 4);
  y.nbuild = put(W * 8);
  y.maxdisp = put(W * 4);
  y.wmax = put(((W * (size_t)(h.nwat + h.nfree) + 63) / 64) * 8);
  y.perm = put(W * npad * 4);
  y.cellcode = put(W * n * 4);
  y.cellstart = put(W * (h.ncell + 1) * 4);
  y.cursor = put(W * h.ncell * 4);
  y.xyzq = put(W * npad * 16);
  y.prm = put(W * npad * 8);
  y.bblo = put(W * nc * 16);
  y.bbhi = put(W * nc * 16);
  y.gsten = put(W * npad * 16);
  y.lcount = put(W * nc * 2 * 4);
  y.lent = put(W * nc * 2 * (size_t)h.cap * 4);
  y.frx = put(W * n * 8); y.fry = put(W * n * 8); y.frz = put(W * n * 8);
  y.grid64 = put(2 * (size_t)h.npair * h.Ktot * 8);
  y.cgrid = put((size_t)h.npair * h.Ktot * 8);
  for (int d = 0; d < 3; ++d) { y.tw[d] = put(h.K[d] * 8); y.bmod[d] = put(h.K[d] * 4); }
  y.eacc = put(W * FELIS_NE * 8);
  y.uacc = put(2 * (size_t)h.npair * (3 + kMaxLamV) * 8);
  y.upart = put(2 * (size_t)h.npair * ((h.n + 255) / 256) * (1 + kMaxLamV) * 8);
  y.lpart = put(2 * (size_t)h.npair * (1 + kMaxLamV) * 8);
  y.ucst = put(8 * sizeof(double));
  y.total = o;
  return FELIS_OK;
}

LegDev make_dev(const felis_ctx* c, const felis_leg* L, const Plan& p, const Meta& m, int index) {
  LegDev g;
  std::memset(&g, 0, sizeof(g));
  const LegHost& h = p.h;
  g.n = h.n; g.W = h.W; g.npad = h.npad; g.nclus = h.nclus; g.cap = h.cap;
  g.nexcl = h.nexcl; g.nbonds = h.nbonds; g.nwat = h.nwat; g.nfree = m.nfree; g.nlig = m.nlig;
  for (int d = 0; d < 3; ++d) g.K[d] = h.K[d];
  g.Ktot = h.Ktot; g.npair = h.npair;
  g.nbits = p.nbits; g.ncoarse = 1 << (p.nbits - 1); g.ncell = h.ncell;
  for (int d = 0; d < 3; ++d) {
    g.nrad[d] = p.nrad[d];
    for (int k = 0; k < kMaxRadix; ++k) g.rad[d][k] = p.rad[d][k];
  }
  g.has_rest = h.has_rest;
  for (int t = 0; t < 6; ++t) {
    g.ranch[t] = L->restraint_atoms[t];
    g.rg0[t] = (float)L->restraint_g0[t];
    g.rk[t] = (float)L->restraint_k[t];
  }
  g.box0 = make_box(L->box, L->ewald_alpha);
  g.pack = L->pressure_bar > 0 ? 0 : 1;
  g.rc2 = (float)(L->r_cut * L->r_cut);
  g.rc2d = L->r_cut * L->r_cut;
  g.rcd = L->r_cut;
  g.alphad = L->ewald_alpha;
  g.sc_alphad = L->sc_alpha;
  for (int t = 0; t < 6; ++t) { g.rg0d[t] = L->restraint_g0[t]; g.rkd[t] = L->restraint_k[t]; }
  g.alpha = (float)L->ewald_alpha;
  g.sc_alpha = (float)L->sc_alpha;
  g.skin_half2 = (float)(0.25 * L->skin * L->skin);
  g.skin = (float)L->skin;
  g.rlist = L->r_cut + L->skin;
  g.rlist2 = g.rlist * g.rlist;
  g.d_oh = (float)L->d_oh;
  g.d_hh = (float)L->d_hh;
  g.self_pref = kKE * L->ewald_alpha / std::sqrt(M_PI);
  g.q = L->charge; g.sig = L->sigma; g.eps = L->epsilon; g.mass = L->mass; g.lig = L->is_ligand;
  g.excl_ij = L->excl_ij; g.excl_ptr = L->excl_ptr; g.excl_idx = L->excl_idx;
  g.bond_ij = L->bond_ij; g.bond_k = L->bond_k; g.bond_r0 = L->bond_r0;
  g.water = L->water_ohh;
  g.x = L->x; g.y = L->y; g.z = L->z; g.vx = L->vx; g.vy = L->vy; g.vz = L->vz;
  g.fx = (long long*)L->fx; g.fy = (long long*)L->fy; g.fz = (long long*)L->fz;
  g.energy = L->energy;
  char* w = (char*)L->work;
  const Layout& y = p.lay;
  g.lam = (float*)(w + y.lam);
  g.lamS = (const float*)(w + y.lamS);
  g.rstate = (int*)(w + y.rstate);
  g.free_atoms = (int*)(w + y.free_atoms);
  g.lig_idx = (int*)(w + y.lig_idx);
  g.aoff = L->alch_offset;
  g.naw = m.naw;
  g.aw_idx = (int*)(w + y.aw_idx);
  g.plain = L->plain_fp64 ? 1 : 0;
  g.fd = (double*)(w + y.fd);
  g.xr = (float*)(w + y.xr); g.yr = (float*)(w + y.yr); g.zr = (float*)(w + y.zr);
  g.flag = (int*)(w + y.flag);
  g.nbuild = (long long*)(w + y.nbuild);
  g.maxdisp = (unsigned*)(w + y.maxdisp);
  g.wmax = (unsigned*)(w + y.wmax);
  g.units = p.h.nwat + p.h.nfree;
  g.hcell = (const unsigned*)(w + y.hcell);
  g.box = (BoxW*)(w + y.box);
  g.ubox = (BoxW*)(w + y.ubox);
  g.rbforce = (int*)(w + y.rbforce);
  g.skin_used = (float*)(w + y.skin_used);
  g.bptr = (const int*)(w + y.bptr);
  g.bnb = (const int*)(w + y.bnb);
  g.bid = (const int*)(w + y.bid);
  g.ntors = h.ntors;
  g.tors = L->torsion_ijkl; g.tors_k = L->torsion_k; g.tors_n = L->torsion_n; g.tors_phase = L->torsion_phase;
  g.tptr = (const int*)(w + y.tptr);
  g.tid = (const int*)(w + y.tid);
  g.nmol = m.nmol;
  if (m.nmol) {
    g.mol_ptr = (const int*)(w + y.mol_ptr);
    g.mol_atoms = (const int*)(w + y.mol_atoms);
    g.baro = (BaroW*)(w + y.baro);
    g.boxb = (BoxW*)(w + y.boxb);
    g.xb = (float*)(w + y.xb); g.yb = (float*)(w + y.yb); g.zb = (float*)(w + y.zb);
    g.molr = (float*)(w + y.molr);
  }
  g.perm = (int*)(w + y.perm);
  g.cellcode = (int*)(w + y.cellcode);
  g.cellstart = (int*)(w + y.cellstart);
  g.cursor = (int*)(w + y.cursor);
  g.xyzq = (float4*)(w + y.xyzq);
  g.prm = (float2*)(w + y.prm);
  g.bblo = (float4*)(w + y.bblo);
  g.bbhi = (float4*)(w + y.bbhi);
  g.gsten = (float4*)(w + y.gsten);
  g.lcount = (int*)(w + y.lcount);
  g.lent = (unsigned*)(w + y.lent);
  g.frx = (long long*)(w + y.frx); g.fry = (long long*)(w + y.fry); g.frz = (long long*)(w + y.frz);
  g.grid64 = (long long*)(w + y.grid64);
  g.cgrid = (float2*)(w + y.cgrid);
  for (int d = 0; d < 3; ++d) { g.tw[d] = (float2*)(w + y.tw[d]); g.bmod[d] = (float*)(w + y.bmod[d]); }
  g.eacc = (long long*)(w + y.eacc);
  g.uacc = (long long*)(w + y.uacc);
  g.upart = (double*)(w + y.upart);
  g.lpart = (double*)(w + y.lpart);
  g.err = c->d_err;
  g.need = c->d_err + 1;
  g.leg_index = index;
  return g;
}

// Build descriptors for a batch; uploads the table when it changed.
int prepare(felis_ctx* c, const felis_leg* legs, int n_legs, std::vector<LegHost>& hs) {
  if (!c) return FELIS_E_INVAL;
  if (n_legs < 1 || n_legs > kMaxLegs || !legs) return fail(c, FELIS_E_INVAL, "n_legs must be in [1, 64]");
  std::vector<LegDev> devs(n_legs);
  hs.resize(n_legs);
  for (int i = 0; i < n_legs; ++i) {
    Plan p;
    int rc = make_plan(c, &legs[i], p);
    if (rc) return rc;
    auto it = c->meta.find(legs[i].work);
    if (it == c->meta.end()) return fail(c, FELIS_E_INVAL, "leg not initialised (felis_leg_init)");
    if (!legs[i].work || legs[i].work_bytes < p.lay.total) return fail(c, FELIS_E_INVAL, "leg work buffer too small");
    p.h.nfree = it->second.nfree;
    p.h.nlig = it->second.nlig;
    p.h.naw = it->second.naw;
    p.h.nmol = it->second.nmol;
    hs[i] = p.h;
    devs[i] = make_dev(c, &legs[i], p, it->second, i);
  }
  if ((int)c->cache.size() == n_legs && std::memcmp(c->cache.data(), devs.data(), sizeof(LegDev) * n_legs) == 0)
    return FELIS_OK;
  std::memcpy(c->h_stage, devs.data(), sizeof(LegDev) * n_legs);
  if (hipMemcpyAsync(c->d_legs, c->h_stage, sizeof(LegDev) * n_legs, hipMemcpyHostToDevice, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return fail(c, FELIS_E_DEVICE, "descriptor upload failed");
  c->cache = devs;
  return FELIS_OK;
}

// Records an event for timer t when profiling is on (start when stop == false).
void mark(felis_ctx* c, int t, bool stop, hipStream_t s) {
  if (!((c->prof >> t) & 1)) return;
  Timer& T = c->timers[t];
  if (!stop) T.skip = (T.seen++ % c->prof_every) != 0;
  if (T.skip) return;
  if (!stop && T.used + 2 > T.ev.size()) {
    for (int k = 0; k < 2; ++k) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      T.ev.push_back(e);
    }
  }
  if (!stop && T.used + 2 > T.ev.size()) return;
  (void)hipEventRecord(T.ev[T.used], s);
  ++T.used;
}
void mark(felis_ctx* c, int t, bool stop) { mark(c, t, stop, c->stream); }

int launched(felis_ctx* c) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(c, FELIS_E_DEVICE, hipGetErrorString(e));
  return FELIS_OK;
}

}  // namespace

extern "C" {

int felis_create(felis_ctx** out, int device, void* hip_stream) {
  if (!out) return FELIS_E_INVAL;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return FELIS_E_DEVICE;
  felis_ctx* c = new felis_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  if (hipMalloc((void**)&c->d_legs, sizeof(LegDev) * kMaxLegs) != hipSuccess ||
      hipHostMalloc((void**)&c->h_stage, sizeof(LegDev) * kMaxLegs, hipHostMallocDefault) != hipSuccess ||
      hipMalloc((void**)&c->d_err, 8 * sizeof(int)) != hipSuccess ||
      hipMalloc((void**)&c->d_count, sizeof(unsigned long long)) != hipSuccess ||
      hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->ev_join, hipEventDisableTiming) != hipSuccess ||
      hipMemset(c->d_err, 0, 8 * sizeof(int)) != hipSuccess ||
      mbar_scratch_setup(device) != FELIS_OK) {
    felis_destroy(c);
    return FELIS_E_DEVICE;
  }
  *out = c;
  return FELIS_OK;
}

void felis_destroy(felis_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream); else (void)hipDeviceSynchronize();
  if (c->d_legs) (void)hipFree(c->d_legs);
  if (c->h_stage) (void)hipHostFree(c->h_stage);
  if (c->d_err) (void)hipFree(c->d_err);
  if (c->d_count) (void)hipFree(c->d_count);
  if (c->side) { (void)hipStreamSynchronize(c->side); (void)hipStreamDestroy(c->side); }
  if (c->ev_fork) (void)hipEventDestroy(c->ev_fork);
  if (c->ev_join) (void)hipEventDestroy(c->ev_join);
  for (auto& T : c->timers)
    for (hipEvent_t e : T.ev) (void)hipEventDestroy(e);
  delete c;
}

const char* felis_last_error(const felis_ctx* c) { return c ? c->last_error.c_str() : "null context"; }

int felis_check(felis_ctx* c, int32_t* needed_cap) {
  return felis_check_detail(c, needed_cap, nullptr, nullptr, nullptr);
}

int felis_check_detail(felis_ctx* c, int32_t* needed_cap, int32_t* leg, int32_t* window, int32_t* atom) {
  if (!c) return FELIS_E_INVAL;
  int e[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (hipStreamSynchronize(c->stream) != hipSuccess ||
      hipMemcpy(e, c->d_err, sizeof(e), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemset(c->d_err, 0, 8 * sizeof(int)) != hipSuccess)
    return fail(c, FELIS_E_DEVICE, "device error word unreadable");
  if (needed_cap) *needed_cap = e[1];
  if (leg) *leg = e[0] ? e[4] : -1;
  if (window) *window = (e[0] && e[3] >= 0) ? (e[3] >> 20) : -1;
  if (atom) *atom = (e[0] && e[3] >= 0) ? (e[3] & 0xfffff) : -1;
  if (e[0] & kErrListCap) {
    char msg[160];
    std::snprintf(msg, sizeof msg, "neighbour list capacity exceeded (raise list_cap; leg %d, window %d)", e[4],
                  e[3] >> 20);
    return fail(c, FELIS_E_CAPACITY, msg);
  }
  if (e[0] & kErrOverflow) {
    static const char* sites[] = {"?", "pair forces", "pair energies", "excluded pairs", "bonded/restraint",
                                  "PME gather", "PME energy", "u_kn", "self", "energy sum", "list", "exclusions"};
    char msg[200];
    const int st = (e[2] >= 0 && e[2] <= 11) ? e[2] : 0;
    std::snprintf(msg, sizeof msg,
                  "fixed-point overflow or non-finite value (first at %s, leg %d, window %d, atom %d)", sites[st],
                  e[4], e[3] >> 20, e[3] & 0xfffff);
    return fail(c, FELIS_E_OVERFLOW, msg);
  }
  if (e[0] & kErrExcl) return fail(c, FELIS_E_UNSUPPORTED, "an atom has more than 8 exclusions");
  if (e[0]) return fail(c, FELIS_E_INVAL, "device reported an invalid configuration");
  return FELIS_OK;
}

int felis_leg_work_size(const felis_leg* leg, size_t* bytes) {
  if (!bytes) return FELIS_E_INVAL;
  Plan p;
  int rc = make_plan(nullptr, leg, p);
  if (rc) return rc;
  *bytes = p.lay.total;
  return FELIS_OK;
}

int felis_leg_rebuilds(felis_ctx* c, const felis_leg* L, int64_t* counts) {
  if (!c || !counts) return FELIS_E_INVAL;
  Plan p;
  int rc = make_plan(c, L, p);
  if (rc) return rc;
  if (!L->work || L->work_bytes < p.lay.total) return fail(c, FELIS_E_INVAL, "leg work buffer too small");
  if (hipStreamSynchronize(c->stream) != hipSuccess ||
      hipMemcpy(counts, (char*)L->work + p.lay.nbuild, sizeof(int64_t) * p.h.W, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(c, FELIS_E_DEVICE, "rebuild counters unreadable");
  return FELIS_OK;
}

int felis_leg_states(felis_ctx* c, const felis_leg* L, int32_t* state_of_replica) {
  if (!c || !state_of_replica) return FELIS_E_INVAL;
  Plan p;
  int rc = make_plan(c, L, p);
  if (rc) return rc;
  if (!L->work || L->work_bytes < p.lay.total) return fail(c, FELIS_E_INVAL, "leg work buffer too small");
  if (hipStreamSynchronize(c->stream) != hipSuccess ||
      hipMemcpy(state_of_replica, (char*)L->work + p.lay.rstate, sizeof(int32_t) * p.h.W, hipMemcpyDeviceToHost) !=
          hipSuccess)
    return fail(c, FELIS_E_DEVICE, "replica states unreadable");
  return FELIS_OK;
}

int felis_leg_init(felis_ctx* c, felis_leg* L) {
  if (!c) return FELIS_E_INVAL;
  Plan p;
  int rc = make_plan(c, L, p);
  if (rc) return rc;
  if (!L->work || L->work_bytes < p.lay.total) return fail(c, FELIS_E_INVAL, "leg work buffer too small");
  const LegHost& h = p.h;
  char* w = (char*)L->work;
  const Layout& y = p.lay;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, FELIS_E_DEVICE, "stream sync failed");
  // topology facts
  std::vector<uint8_t> lig(h.n);
  std::vector<int> wat(3 * (size_t)h.nwat);
  if (hipMemcpy(lig.data(), L->is_ligand, h.n, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(c, FELIS_E_DEVICE, "is_ligand copy failed");
  if (h.nwat && hipMemcpy(wat.data(), L->water_ohh, wat.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(c, FELIS_E_DEVICE, "water copy failed");
  std::vector<char> inwat(h.n, 0);
  for (int v : wat) {
    if (v < 0 || v >= h.n || inwat[v]) return fail(c, FELIS_E_INVAL, "water atom out of range or repeated");
    inwat[v] = 1;
  }
  std::vector<int> freeat, ligi;
  for (int a = 0; a < h.n; ++a) {
    if (!inwat[a]) freeat.push_back(a);
    if (lig[a]) ligi.push_back(a);
  }
  // lambda table: elec, vdw, restraint, sc_alpha (1 - vdw)
  std::vector<float> lam(4 * (size_t)h.W);
  for (int k = 0; k < h.W; ++k) {
    const double le = L->lambdas[3 * k], lv = L->lambdas[3 * k + 1], lr = L->lambdas[3 * k + 2];
    if (!(le >= 0 && le <= 1 && lv >= 0 && lv <= 1 && lr >= 0 && lr <= 1))
      return fail(c, FELIS_E_INVAL, "lambdas must lie in [0, 1]");
    lam[4 * k] = (float)le; lam[4 * k + 1] = (float)lv; lam[4 * k + 2] = (float)lr;
    lam[4 * k + 3] = (float)(L->sc_alpha * (1.0 - lv));
  }
  bool ok = hipMemcpy(w + y.lam, lam.data(), lam.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
  ok &= hipMemcpy(w + y.lamS, lam.data(), lam.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
  {
    std::vector<int> ident(h.W);
    for (int k = 0; k < h.W; ++k) ident[k] = k;
    ok &= hipMemcpy(w + y.rstate, ident.data(), ident.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
  }
  if (!freeat.empty()) ok &= hipMemcpy(w + y.free_atoms, freeat.data(), freeat.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
  if (!ligi.empty()) ok &= hipMemcpy(w + y.lig_idx, ligi.data(), ligi.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
  {
    // Hilbert indices of the fine cells
    const int nb = p.nbits, nf = 1 << nb;
    std::vector<unsigned> hc((size_t)h.ncell);
    for (int x = 0; x < nf; ++x)
      for (int yy = 0; yy < nf; ++yy)
        for (int z = 0; z < nf; ++z) hc[((size_t)x * nf + yy) * nf + z] = hilbert3(x, yy, z, nb);
    ok &= hipMemcpy(w + y.hcell, hc.data(), hc.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
  }
  {
    const std::vector<BoxW> bw((size_t)h.W, make_box(L->box, L->ewald_alpha));
    ok &= hipMemcpy(w + y.box, bw.data(), bw.size() * sizeof(BoxW), hipMemcpyHostToDevice) == hipSuccess;
  }
  for (int d = 0; d < 3; ++d) {
    const int K = h.K[d];
    std::vector<float> tw(2 * (size_t)K), bm(K);
    for (int k = 0; k < K; ++k) {
      const double a = 2.0 * M_PI * k / K;
      tw[2 * k] = (float)std::cos(a);
      tw[2 * k + 1] = (float)-std::sin(a);
      const double den = (2.0 + std::cos(a)) / 3.0;     // order-4 Euler spline denominator
      bm[k] = (float)(1.0 / (den * den));
    }
    ok &= hipMemcpy(w + y.tw[d], tw.data(), tw.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
    ok &= hipMemcpy(w + y.bmod[d], bm.data(), bm.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
  }
  // zeroed accumulators and grids, forced list build
  const float far = 1.0e18f;
  unsigned farbits;
  std::memcpy(&farbits, &far, 4);
  ok &= hipMemsetD32Async((hipDeviceptr_t)(w + y.xr), farbits, 3 * ((y.yr - y.xr) / 4), c->stream) == hipSuccess;
  ok &= hipMemsetD32Async((hipDeviceptr_t)(w + y.flag), 1, h.W, c->stream) == hipSuccess;
  ok &= hipMemsetAsync(w + y.nbuild, 0, h.W * 8, c->stream) == hipSuccess;
  ok &= hipMemsetAsync(w + y.maxdisp, 0, h.W * 4, c->stream) == hipSuccess;
  ok &= hipMemsetAsync(w + y.wmax, 0, y.perm - y.wmax, c->stream) == hipSuccess;
  ok &= hipMemsetAsync(w + y.rbforce, 0, h.W * 4, c->stream) == hipSuccess;
  if (L->plain_fp64) ok &= hipMemsetAsync(w + y.fd, 0, 3 * (size_t)h.W * h.n * 8, c->stream) == hipSuccess;
  ok &= hipMemsetAsync(w + y.skin_used, 0, h.W * 4, c->stream) == hipSuccess;
  ok &= hipMemsetAsync(w + y.lcount, 0, (size_t)h.W * h.nclus * 2 * 4, c->stream) == hipSuccess;
  ok &= hipMemsetAsync(w + y.grid64, 0, y.cgrid - y.grid64, c->stream) == hipSuccess;
  ok &= hipMemsetAsync(w + y.eacc, 0, y.ucst - y.eacc, c->stream) == hipSuccess;
  ok &= hipStreamSynchronize(c->stream) == hipSuccess;
  if (!ok) return fail(c, FELIS_E_DEVICE, "leg initialisation copies failed");
  Meta m;
  m.nfree = (int)freeat.size();
  m.nlig = (int)ligi.size();
  m.naw = 0;
  if (L->alch_offset) {
    // alchemical-water atoms (nonzero offset, never ligand atoms) and their
    // two exclusion partners each (the other atoms of the rigid water)
    std::vector<float> off(h.n);
    std::vector<int> ep(h.n + 1), ei;
    if (hipMemcpy(off.data(), L->alch_offset, h.n * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(ep.data(), L->excl_ptr, (h.n + 1) * 4, hipMemcpyDeviceToHost) != hipSuccess)
      return fail(c, FELIS_E_DEVICE, "alchemical offset copy failed");
    ei.resize(std::max(ep[h.n], 1));
    if (ep[h.n] && hipMemcpy(ei.data(), L->excl_idx, ep[h.n] * 4, hipMemcpyDeviceToHost) != hipSuccess)
      return fail(c, FELIS_E_DEVICE, "exclusion copy failed");
    std::vector<int> aw, part;
    for (int a = 0; a < h.n; ++a) {
      if (off[a] == 0.0f) continue;
      if (lig[a]) return fail(c, FELIS_E_INVAL, "an alchemical offset on a ligand atom");
      if (ep[a + 1] - ep[a] != 2) return fail(c, FELIS_E_INVAL, "an alchemical-water atom needs two exclusions");
      aw.push_back(a);
      part.push_back(ei[ep[a]]);
      part.push_back(ei[ep[a] + 1]);
    }
    m.naw = (int)aw.size();
    if (m.nlig + m.naw > kMaxLigand)
      return fail(c, FELIS_E_UNSUPPORTED, "more than 256 ligand and alchemical-water atoms");
    aw.insert(aw.end(), part.begin(), part.end());
    if (!aw.empty() && hipMemcpy(w + y.aw_idx, aw.data(), aw.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
      return fail(c, FELIS_E_DEVICE, "alchemical water table");
  }
  m.nmol = 0;
  std::vector<int> bij(2 * (size_t)h.nbonds);
  if (h.nbonds && hipMemcpy(bij.data(), L->bond_ij, bij.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(c, FELIS_E_DEVICE, "bond copy failed");
  {
    // per-atom bond table for the integrator: for atom a, its partners and
    // bond indices in bond order
    std::vector<int> ptr(h.n + 1, 0), nb(std::max(2 * h.nbonds, 2)), id(std::max(2 * h.nbonds, 2));
    for (int k = 0; k < h.nbonds; ++k) {
      const int a = bij[2 * k], b = bij[2 * k + 1];
      if (a < 0 || b < 0 || a >= h.n || b >= h.n) return fail(c, FELIS_E_INVAL, "bond atom out of range");
      ++ptr[a + 1]; ++ptr[b + 1];
    }
    for (int a = 0; a < h.n; ++a) ptr[a + 1] += ptr[a];
    std::vector<int> fill(ptr.begin(), ptr.end() - 1);
    for (int k = 0; k < h.nbonds; ++k) {
      const int a = bij[2 * k], b = bij[2 * k + 1];
      nb[fill[a]] = b; id[fill[a]++] = k;
      nb[fill[b]] = a; id[fill[b]++] = k;
    }
    ok &= hipMemcpy(w + y.bptr, ptr.data(), ptr.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
    ok &= hipMemcpy(w + y.bnb, nb.data(), nb.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
    ok &= hipMemcpy(w + y.bid, id.data(), id.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) return fail(c, FELIS_E_DEVICE, "bond table");
  }
  {
    // per-atom torsion table for the integrator: for atom a, entries 4 t + s
    // (torsion t, a is its s-th atom) in torsion order
    std::vector<int> tq(4 * (size_t)h.ntors);
    if (h.ntors && hipMemcpy(tq.data(), L->torsion_ijkl, tq.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)
      return fail(c, FELIS_E_DEVICE, "torsion copy failed");
    std::vector<int> ptr(h.n + 1, 0), id(std::max(4 * h.ntors, 1));
    for (size_t e = 0; e < tq.size(); ++e) {
      if (tq[e] < 0 || tq[e] >= h.n) return fail(c, FELIS_E_INVAL, "torsion atom out of range");
      ++ptr[tq[e] + 1];
    }
    for (int a = 0; a < h.n; ++a) ptr[a + 1] += ptr[a];
    std::vector<int> fill(ptr.begin(), ptr.end() - 1);
    for (size_t e = 0; e < tq.size(); ++e) id[fill[tq[e]]++] = (int)e;
    ok &= hipMemcpy(w + y.tptr, ptr.data(), ptr.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
    ok &= hipMemcpy(w + y.tid, id.data(), id.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) return fail(c, FELIS_E_DEVICE, "torsion table");
  }
  if (L->pressure_bar > 0) {
    // molecules: connected components of the bonds with each rigid water's
    // atoms joined (union-find), numbered by their lowest atom
    std::vector<int> parent(h.n);
    for (int a = 0; a < h.n; ++a) parent[a] = a;
    auto find = [&](int a) {
      while (parent[a] != a) { parent[a] = parent[parent[a]]; a = parent[a]; }
      return a;
    };
    auto join = [&](int a, int b) {
      if (a < 0 || b < 0 || a >= h.n || b >= h.n) return false;
      const int ra = find(a), rb = find(b);
      if (ra != rb) parent[std::max(ra, rb)] = std::min(ra, rb);
      return true;
    };
    for (int k = 0; k < h.nbonds; ++k)
      if (!join(bij[2 * k], bij[2 * k + 1])) return fail(c, FELIS_E_INVAL, "bond atom out of range");
    for (int k = 0; k < h.nwat; ++k) { join(wat[3 * k], wat[3 * k + 1]); join(wat[3 * k], wat[3 * k + 2]); }
    std::vector<int> id(h.n, -1), cnt;
    for (int a = 0; a < h.n; ++a) {
      const int r = find(a);
      if (id[r] < 0) { id[r] = (int)cnt.size(); cnt.push_back(0); }
      ++cnt[id[r]];
    }
    m.nmol = (int)cnt.size();
    std::vector<int> ptr(m.nmol + 1, 0), atoms(h.n), fill;
    for (int t = 0; t < m.nmol; ++t) ptr[t + 1] = ptr[t] + cnt[t];
    fill.assign(ptr.begin(), ptr.end() - 1);
    for (int a = 0; a < h.n; ++a) atoms[fill[id[find(a)]]++] = a;
    std::vector<BaroW> bw((size_t)h.W);
    std::memset(bw.data(), 0, bw.size() * sizeof(BaroW));
    for (auto& b : bw) b.dv_max = 0.01 * L->box[0] * L->box[1] * L->box[2];
    ok &= hipMemcpy(w + y.mol_ptr, ptr.data(), ptr.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
    ok &= hipMemcpy(w + y.mol_atoms, atoms.data(), atoms.size() * 4, hipMemcpyHostToDevice) == hipSuccess;
    ok &= hipMemcpy(w + y.baro, bw.data(), bw.size() * sizeof(BaroW), hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) return fail(c, FELIS_E_DEVICE, "barostat tables");
  }
  m.work_bytes = L->work_bytes;
  c->meta[L->work] = m;
  c->cache.clear();
  return FELIS_OK;
}

int felis_build_nlist(felis_ctx* c, felis_leg* legs, int n_legs, int force) {
  std::vector<LegHost> hs;
  int rc = prepare(c, legs, n_legs, hs);
  if (rc) return rc;
  launch_check(c->stream, c->d_legs, hs.data(), n_legs, force ? 1 : 0, false);
  launch_build(c->stream, c->d_legs, hs.data(), n_legs);
  return launched(c);
}

int felis_nlist_export_pairs(felis_ctx* c, const felis_leg* leg, int window, double r, int32_t* pairs,
                             int64_t cap, int64_t* n_pairs) {
  std::vector<LegHost> hs;
  int rc = prepare(c, leg, 1, hs);
  if (rc) return rc;
  if (window < 0 || window >= leg->n_windows || !n_pairs || (cap > 0 && !pairs))
    return fail(c, FELIS_E_INVAL, "export arguments");
  unsigned long long cnt = 0;
  if (hipMemsetAsync(c->d_count, 0, sizeof(cnt), c->stream) != hipSuccess) return fail(c, FELIS_E_DEVICE, "memset");
  launch_export(c->stream, c->d_legs, hs[0], window, r, pairs, cap, c->d_count);
  if ((rc = launched(c))) return rc;
  if (hipMemcpyAsync(&cnt, c->d_count, sizeof(cnt), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return fail(c, FELIS_E_DEVICE, "export count copy failed");
  *n_pairs = (int64_t)cnt;
  return (int64_t)cnt > cap ? fail(c, FELIS_E_CAPACITY, "export buffer too small") : FELIS_OK;
}

int felis_nonbonded(felis_ctx* c, felis_leg* legs, int n_legs, int flags) {
  std::vector<LegHost> hs;
  int rc = prepare(c, legs, n_legs, hs);
  if (rc) return rc;
  const bool en = flags & FELIS_ENERGY;
  if (en) launch_zero_energy(c->stream, c->d_legs, hs.data(), n_legs, FELIS_E_COUL_REAL, FELIS_E_SELF + 1);
  launch_pack(c->stream, c->d_legs, hs.data(), n_legs, false);
  mark(c, FELIS_PROF_PAIRS, false);
  launch_pairs(c->stream, c->d_legs, hs.data(), n_legs, en ? 2 : 0);
  mark(c, FELIS_PROF_PAIRS, true);
  launch_corrections(c->stream, c->d_legs, hs.data(), n_legs, en);
  if (en) launch_finish_energy(c->stream, c->d_legs, hs.data(), n_legs, FELIS_E_COUL_REAL, FELIS_E_SELF + 1);
  return launched(c);
}

int felis_pme(felis_ctx* c, felis_leg* legs, int n_legs, int flags) {
  std::vector<LegHost> hs;
  int rc = prepare(c, legs, n_legs, hs);
  if (rc) return rc;
  const bool en = flags & FELIS_ENERGY;
  if (en) launch_zero_energy(c->stream, c->d_legs, hs.data(), n_legs, FELIS_E_RECIP, FELIS_E_RECIP + 1);
  // spreading finds atoms through the cell sort of the last list build: bring
  // it up to date (rebuilds only windows that moved more than skin/2)
  launch_check(c->stream, c->d_legs, hs.data(), n_legs, 0, false);
  launch_build(c->stream, c->d_legs, hs.data(), n_legs);
  launch_pme(c->stream, c->d_legs, hs.data(), n_legs, en);
  if (en) launch_finish_energy(c->stream, c->d_legs, hs.data(), n_legs, FELIS_E_RECIP, FELIS_E_RECIP + 1);
  return launched(c);
}

int felis_bonded(felis_ctx* c, felis_leg* legs, int n_legs, int flags) {
  std::vector<LegHost> hs;
  int rc = prepare(c, legs, n_legs, hs);
  if (rc) return rc;
  const bool en = flags & FELIS_ENERGY;
  if (en) launch_zero_energy(c->stream, c->d_legs, hs.data(), n_legs, FELIS_E_BOND, FELIS_E_RESTRAINT + 1);
  launch_bonded(c->stream, c->d_legs, hs.data(), n_legs, en ? 2 : 0);
  if (en) launch_finish_energy(c->stream, c->d_legs, hs.data(), n_legs, FELIS_E_BOND, FELIS_E_RESTRAINT + 1);
  return launched(c);
}

// Every energy component of every window of the batch (lists brought up to
// date first); the window totals land in each leg's energy array.
void energy_pass(felis_ctx* c, const std::vector<LegHost>& hs, int n_legs, bool from_word) {
  const LegHost* h = hs.data();
  launch_zero_energy(c->stream, c->d_legs, h, n_legs, 0, FELIS_E_TOTAL);
  launch_check(c->stream, c->d_legs, h, n_legs, 0, from_word);
  launch_sort_pack(c->stream, c->d_legs, h, n_legs);
  // reciprocal space beside the list build and the pair kernel, as in a step;
  // its forces go to frx.. (the pair kernel stores fx.. meanwhile), and the
  // next step overwrites both: only the energy is wanted here
  (void)hipEventRecord(c->ev_fork, c->stream);
  (void)hipStreamWaitEvent(c->side, c->ev_fork, 0);
  launch_pme(c->side, c->d_legs, h, n_legs, true, true);
  (void)hipEventRecord(c->ev_join, c->side);
  launch_lists(c->stream, c->d_legs, h, n_legs);
  // the Metropolis test needs energy differences: FP32 pair terms summed in FP64
  launch_pairs(c->stream, c->d_legs, h, n_legs, 1);
  launch_corrections(c->stream, c->d_legs, h, n_legs, true);
  launch_bonded(c->stream, c->d_legs, h, n_legs, 1);
  (void)hipStreamWaitEvent(c->stream, c->ev_join, 0);
  launch_finish_energy(c->stream, c->d_legs, h, n_legs, 0, FELIS_E_TOTAL);
}

// One volume move of every window of the due legs: energies, trial move
// (box, molecule centres), energies in the trial boxes, Metropolis test and
// restore of rejected windows.
void baro_attempt(felis_ctx* c, const std::vector<LegHost>& hs, int n_legs, const BaroArgs& A, bool from_word) {
  // every launcher sizes its grid from the window (and grid) counts: legs
  // that make no move get no workgroups and are left exactly as they are
  std::vector<LegHost> hd(hs);
  for (int i = 0; i < n_legs; ++i)
    if (!A.due[i]) { hd[i].W = 0; hd[i].npair = 0; hd[i].nmol = 0; }
  mark(c, FELIS_PROF_BARO, false);
  energy_pass(c, hd, n_legs, from_word);
  launch_baro_keep_u0(c->stream, c->d_legs, hd.data(), n_legs);
  launch_baro_propose(c->stream, c->d_legs, hd.data(), n_legs, A);
  energy_pass(c, hd, n_legs, false);
  launch_baro_accept(c->stream, c->d_legs, hd.data(), n_legs, A);
  mark(c, FELIS_PROF_BARO, true);
}

int felis_step(felis_ctx* c, felis_leg* legs, int n_legs, int n_steps, double dt, double temperature,
               double gamma) {
  std::vector<LegHost> hs;
  int rc = prepare(c, legs, n_legs, hs);
  if (rc) return rc;
  if (n_steps < 0 || !(dt > 0) || !(temperature >= 0) || !(gamma >= 0))
    return fail(c, FELIS_E_INVAL, "n_steps, dt, temperature, gamma");
  std::vector<long long> step(n_legs);
  std::vector<unsigned long long> seed(n_legs);
  BaroArgs A;
  std::memset(&A, 0, sizeof(A));
  A.kT = kKB * temperature;
  for (int s = 0; s < n_steps; ++s) {
    bool baro = false;
    for (int i = 0; i < n_legs; ++i) {
      step[i] = legs[i].step + s;
      seed[i] = legs[i].seed;
      // volume moves before the steps whose index is a positive multiple of
      // barostat_every
      const bool due = legs[i].pressure_bar > 0 && step[i] > 0 && step[i] % legs[i].barostat_every == 0;
      A.due[i] = due ? 1 : 0;
      A.attempt[i] = due ? step[i] / legs[i].barostat_every : 0;
      A.seed[i] = legs[i].seed;
      A.pressure[i] = legs[i].pressure_bar * kBar;
      baro |= due;
    }
    if (baro) baro_attempt(c, hs, n_legs, A, s > 0);
    mark(c, FELIS_PROF_NLIST, false);
    // the first step scans positions; later steps read the largest
    // displacement the previous step's integrator recorded (after a volume
    // move: scan again)
    launch_check(c->stream, c->d_legs, hs.data(), n_legs, 0, s > 0 && !baro);
    launch_sort_pack(c->stream, c->d_legs, hs.data(), n_legs);
    // reciprocal space needs only the cell sort and the packed coordinates
    // and parameters: it runs on the side stream beside the list build, the
    // pair kernel and the bonded terms, and stores its forces apart (frx..)
    (void)hipEventRecord(c->ev_fork, c->stream);
    (void)hipStreamWaitEvent(c->side, c->ev_fork, 0);
    mark(c, FELIS_PROF_PME, false, c->side);
    launch_pme(c->side, c->d_legs, hs.data(), n_legs, false, true);
    mark(c, FELIS_PROF_PME, true, c->side);
    (void)hipEventRecord(c->ev_join, c->side);
    launch_lists(c->stream, c->d_legs, hs.data(), n_legs);
    mark(c, FELIS_PROF_NLIST, true);       // the build stage also packs the sorted coordinates
    mark(c, FELIS_PROF_PAIRS, false);
    launch_pairs(c->stream, c->d_legs, hs.data(), n_legs, 0, true);
    mark(c, FELIS_PROF_PAIRS, true);
    // bonded and restraint forces are summed by the integrator itself
    (void)hipStreamWaitEvent(c->stream, c->ev_join, 0);
    mark(c, FELIS_PROF_INTEGRATE, false);
    launch_integrate(c->stream, c->d_legs, hs.data(), n_legs, step.data(), seed.data(), (float)dt,
                     (float)temperature, (float)gamma);
    mark(c, FELIS_PROF_INTEGRATE, true);
  }
  for (int i = 0; i < n_legs; ++i) legs[i].step += n_steps;
  return launched(c);
}

int felis_barostat(felis_ctx* c, felis_leg* legs, int n_legs, double temperature, int64_t attempt) {
  std::vector<LegHost> hs;
  int rc = prepare(c, legs, n_legs, hs);
  if (rc) return rc;
  if (!(temperature > 0) || attempt < 0) return fail(c, FELIS_E_INVAL, "temperature > 0, attempt >= 0");
  BaroArgs A;
  std::memset(&A, 0, sizeof(A));
  A.kT = kKB * temperature;
  bool any = false;
  for (int i = 0; i < n_legs; ++i) {
    A.due[i] = legs[i].pressure_bar > 0 ? 1 : 0;
    A.attempt[i] = attempt;
    A.seed[i] = legs[i].seed;
    A.pressure[i] = legs[i].pressure_bar * kBar;
    any |= A.due[i] != 0;
  }
  if (!any) return fail(c, FELIS_E_INVAL, "no leg of the batch has a pressure");
  baro_attempt(c, hs, n_legs, A, false);
  // lists of rejected windows were built for the trial move: rebuild them now
  launch_check(c->stream, c->d_legs, hs.data(), n_legs, 0, false);
  launch_build(c->stream, c->d_legs, hs.data(), n_legs);
  return launched(c);
}

int felis_leg_boxes(felis_ctx* c, const felis_leg* L, double* edges) {
  std::vector<LegHost> hs;
  int rc = prepare(c, L, 1, hs);
  if (rc) return rc;
  if (!edges) return fail(c, FELIS_E_INVAL, "null output");
  Plan p;
  make_plan(c, L, p);
  std::vector<BoxW> b((size_t)L->n_windows);
  if (hipMemcpyAsync(b.data(), (char*)L->work + p.lay.box, b.size() * sizeof(BoxW), hipMemcpyDeviceToHost,
                     c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return fail(c, FELIS_E_DEVICE, "box copy failed");
  for (int w = 0; w < L->n_windows; ++w)
    for (int d = 0; d < 3; ++d) edges[3 * w + d] = b[w].L[d];
  return FELIS_OK;
}

int felis_leg_boxes_async(felis_ctx* c, const felis_leg* L, double* edges) {
  std::vector<LegHost> hs;
  int rc = prepare(c, L, 1, hs);
  if (rc) return rc;
  if (!edges) return fail(c, FELIS_E_INVAL, "null output");
  Plan p;
  make_plan(c, L, p);
  const char* src = (const char*)L->work + p.lay.box + offsetof(BoxW, L);
  if (hipMemcpy2DAsync(edges, 3 * sizeof(double), src, sizeof(BoxW), 3 * sizeof(double), L->n_windows,
                       hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return fail(c, FELIS_E_DEVICE, "box copy failed");
  return FELIS_OK;
}

int felis_barostat_stats(felis_ctx* c, const felis_leg* L, double* out) {
  std::vector<LegHost> hs;
  int rc = prepare(c, L, 1, hs);
  if (rc) return rc;
  if (!out) return fail(c, FELIS_E_INVAL, "null output");
  if (!(L->pressure_bar > 0)) return fail(c, FELIS_E_INVAL, "the leg has no barostat");
  Plan p;
  make_plan(c, L, p);
  std::vector<BaroW> b((size_t)L->n_windows);
  if (hipMemcpyAsync(b.data(), (char*)L->work + p.lay.baro, b.size() * sizeof(BaroW), hipMemcpyDeviceToHost,
                     c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return fail(c, FELIS_E_DEVICE, "barostat state copy failed");
  for (int w = 0; w < L->n_windows; ++w) {
    double* o = out + (size_t)FELIS_BARO_NS * w;
    o[0] = b[w].u0; o[1] = b[w].u1; o[2] = b[w].work; o[3] = b[w].vol_old; o[4] = b[w].vol_new;
    o[5] = b[w].scale; o[6] = b[w].accepted; o[7] = b[w].dv_max; o[8] = (double)b[w].total_att;
    o[9] = (double)b[w].total_acc;
  }
  return FELIS_OK;
}

int felis_ukn(felis_ctx* c, felis_leg* leg, const double* lambdas, int K, const float* fx, const float* fy,
              const float* fz, int64_t frame_stride, int64_t n_frames, const double* frame_box, double beta,
              double* u, int64_t u_stride) {
  std::vector<LegHost> hs;
  int rc = prepare(c, leg, 1, hs);
  if (rc) return rc;
  if (!lambdas || K < 1 || n_frames < 0) return fail(c, FELIS_E_INVAL, "u_kn arguments");
  for (int k = 0; k < K; ++k)
    for (int t = 0; t < 3; ++t)
      if (!(lambdas[3 * k + t] >= 0 && lambdas[3 * k + t] <= 1)) return fail(c, FELIS_E_INVAL, "lambdas in [0, 1]");
  if (n_frames == 0) return FELIS_OK;                 // nothing to read or write
  if (!fx || !fy || !fz || !u || frame_stride < leg->n_atoms || u_stride < n_frames)
    return fail(c, FELIS_E_INVAL, "u_kn arguments");
  Plan p;
  make_plan(c, leg, p);
  char* w = (char*)leg->work;
  mark(c, FELIS_PROF_UKN, false);
  rc = launch_ukn(c->stream, c->d_legs, hs[0], leg->sc_alpha, lambdas, K, fx, fy, fz, frame_stride, n_frames,
                  frame_box, leg->pressure_bar * kBar, beta, u, u_stride, (long long*)(w + p.lay.uacc),
                  (double*)(w + p.lay.ucst));
  mark(c, FELIS_PROF_UKN, true);
  if (rc) return fail(c, rc, "u_kn: more than 128 states, 64 distinct lambda_vdw or 256 ligand atoms");
  return launched(c);
}

int felis_hrex(felis_ctx* c, felis_leg* leg, const double* u, int64_t u_stride, int64_t attempt, uint64_t seed,
               int32_t* n_accepted) {
  std::vector<LegHost> hs;
  int rc = prepare(c, leg, 1, hs);
  if (rc) return rc;
  if (!u || u_stride < leg->n_windows || attempt < 0) return fail(c, FELIS_E_INVAL, "replica exchange arguments");
  if (leg->n_windows > kMaxHrex) return fail(c, FELIS_E_UNSUPPORTED, "replica exchange among at most 256 windows");
  int* acc = reinterpret_cast<int*>(c->d_count);
  launch_hrex(c->stream, c->d_legs, hs[0], u, u_stride, attempt, seed, acc);
  if ((rc = launched(c))) return rc;
  if (n_accepted) {
    if (hipMemcpyAsync(n_accepted, acc, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
      return fail(c, FELIS_E_DEVICE, "replica exchange count copy failed");
  }
  return FELIS_OK;
}

int felis_restraint_dg(const double* g0, const double* k, double temperature, double* dg) {
  if (!g0 || !k || !dg || !(temperature > 0) || !std::isfinite(temperature)) return FELIS_E_INVAL;
  double prodk = 1.0;
  for (int t = 0; t < 6; ++t) {
    if (!(k[t] > 0) || !std::isfinite(k[t]) || !std::isfinite(g0[t])) return FELIS_E_INVAL;
    prodk *= k[t];
  }
  if (!(g0[0] > 0) || !(g0[1] > 0 && g0[1] < M_PI) || !(g0[2] > 0 && g0[2] < M_PI)) return FELIS_E_INVAL;
  const double kT = kKB * temperature;
  const double v0 = 1660.5390;                       // A^3 per molecule at 1 mol/L
  const double num = 8.0 * M_PI * M_PI * v0 * std::sqrt(prodk);
  const double den = g0[0] * g0[0] * std::sin(g0[1]) * std::sin(g0[2]) * std::pow(2.0 * M_PI * kT, 3);
  *dg = kT * std::log(num / den);
  return FELIS_OK;
}

int felis_delta_g(const double* f, int K, double temperature, double* dg) {
  if (!f || !dg || K < 2 || !(temperature > 0) || !std::isfinite(temperature)) return FELIS_E_INVAL;
  if (!std::isfinite(f[0]) || !std::isfinite(f[K - 1])) return FELIS_E_INVAL;
  *dg = kKB * temperature * (f[K - 1] - f[0]);
  return FELIS_OK;
}

int felis_segment_bounds(int n_windows, int n_segments, int32_t* first) {
  if (!first || n_segments < 1 || n_windows < n_segments + 1) return FELIS_E_INVAL;
  for (int s = 0; s <= n_segments; ++s) first[s] = (int32_t)(((long long)s * (n_windows - 1)) / n_segments);
  return FELIS_OK;
}

int felis_binding_dg(const double* dg_solvent_segments, int n_solvent, const double* dg_complex_segments,
                     int n_complex, const double* g0, const double* k, double temperature, double* dg_bind) {
  if (!dg_solvent_segments || !dg_complex_segments || !dg_bind || n_solvent < 1 || n_complex < 1)
    return FELIS_E_INVAL;
  double solv = 0.0, cplx = 0.0, rest = 0.0;
  for (int i = 0; i < n_solvent; ++i) solv += dg_solvent_segments[i];
  for (int i = 0; i < n_complex; ++i) cplx += dg_complex_segments[i];
  if (!std::isfinite(solv) || !std::isfinite(cplx)) return FELIS_E_INVAL;
  const int rc = felis_restraint_dg(g0, k, temperature, &rest);
  if (rc) return rc;
  *dg_bind = solv - cplx + rest;
  return FELIS_OK;
}

int felis_profile(felis_ctx* c, int enable) {
  if (!c) return FELIS_E_INVAL;
  c->prof = enable == 1 ? (1 << FELIS_PROF_N) - 1 : (enable & ((1 << FELIS_PROF_N) - 1));
  for (auto& T : c->timers) { T.seen = 0; T.skip = false; }
  return FELIS_OK;
}

int felis_profile_every(felis_ctx* c, int every) {
  if (!c || every < 1) return FELIS_E_INVAL;
  c->prof_every = every;
  return FELIS_OK;
}

int felis_profile_read(felis_ctx* c, int which, double* total_ms, int64_t* launches) {
  if (!c || which < 0 || which >= FELIS_PROF_N || !total_ms || !launches) return FELIS_E_INVAL;
  if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, FELIS_E_DEVICE, "stream sync failed");
  Timer& T = c->timers[which];
  double tot = 0.0;
  int64_t n = 0;
  for (size_t k = 0; k + 1 < T.used; k += 2) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, T.ev[k], T.ev[k + 1]) != hipSuccess) return fail(c, FELIS_E_DEVICE, "event timing");
    tot += ms;
    ++n;
  }
  T.used = 0;
  *total_ms = tot;
  *launches = n;
  return FELIS_OK;
}

int felis_mbar_work_size(int K, int64_t n_total, size_t* bytes) {
  if (!bytes || K < 2 || n_total < 1) return FELIS_E_INVAL;
  *bytes = mbar_work_bytes(K, n_total);
  return FELIS_OK;
}

int felis_mbar(felis_ctx* c, const double* u, const int32_t* N_k, int K, int64_t n_total, double rel_tol,
               int max_iter, double* f_out, int* iters, void* work, size_t work_bytes) {
  if (!c) return FELIS_E_INVAL;
  int rc = launch_mbar(c->stream, u, N_k, K, n_total, rel_tol, max_iter, f_out, iters, work, work_bytes);
  if (rc == FELIS_E_INVAL) return fail(c, rc, "MBAR arguments (K in [2, 512], sum N_k = n_total, work size)");
  if (rc == FELIS_E_NOCONV) return fail(c, rc, "MBAR did not converge within max_iter");
  if (rc) return fail(c, rc, "MBAR device error");
  return launched(c);
}

int felis_mbar_noalloc(felis_ctx* c, const double* u, const int32_t* N_k, int K, int64_t n_total, double rel_tol,
                       int max_iter, double* f_out, int* iters) {
  if (!c) return FELIS_E_INVAL;
  if (!u || !N_k || !f_out || !(rel_tol > 0) || max_iter < 1)
    return fail(c, FELIS_E_INVAL, "MBAR arguments (K in [2, 512], sum N_k = n_total)");
  if (K >= 2 && K <= 512 && n_total >= 1 && mbar_work_bytes(K, n_total) > kMbarStaticBytes) {
    char msg[200];
    std::snprintf(msg, sizeof msg,
                  "K = %d states x %lld samples need %zu bytes of MBAR scratch; the allocation-free entry point "
                  "holds %zu (use felis_mbar with a workspace)",
                  K, (long long)n_total, mbar_work_bytes(K, n_total), kMbarStaticBytes);
    return fail(c, FELIS_E_CAPACITY, msg);
  }
  int rc = launch_mbar_noalloc(c->device, c->stream, u, N_k, K, n_total, rel_tol, max_iter, f_out, iters);
  if (rc == FELIS_E_INVAL) return fail(c, rc, "MBAR arguments (K in [2, 512], sum N_k = n_total)");
  if (rc == FELIS_E_NOCONV) return fail(c, rc, "MBAR did not converge within max_iter");
  if (rc) return fail(c, rc, "MBAR device error");
  return launched(c);
}

}  // extern "C"
