// Internal definitions shared by the HIP kernels and the C-ABI host code.
// Not part of the public interface (see include/felis.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/felis.h"

namespace felis {

constexpr int kMaxLegs = 64;        // legs per batched launch
constexpr int kMaxExcl = 8;         // exclusions per atom handled by the list build
constexpr int kMaxLigand = 256;     // ligand atoms handled by the u_kn kernels
constexpr int kMaxLamV = 64;        // distinct lambda_vdw values per u_kn call
constexpr int kMaxStates = 128;     // lambda states per u_kn call
constexpr int kMaxRadix = 8;        // FFT stages per axis
constexpr int kMaxHrex = 256;       // most windows a leg may exchange among
constexpr int kMaxFFT = 128;        // largest PME grid dimension (bases pack in 7 bits)
constexpr int kClus = 8;            // atoms per i-cluster (pair kernel)

constexpr double kKE = 332.06371;                 // kcal A / (mol e^2)
constexpr double kBar = 1.0e-25 * 6.02214076e23 / 4184.0;   // 1 bar in kcal / (mol A^3)
constexpr double kKB = 0.0019872043;              // kcal / (mol K)
constexpr double kAccel = 418.4;                  // (kcal/mol/A/amu) -> A/ps^2
constexpr double kForceScale = 4294967296.0;      // 2^32 int64 units per kcal/mol/A
constexpr double kGridScale = 1099511627776.0;    // 2^40 int64 units per e
constexpr double kEnergyScale = 1073741824.0;     // 2^30 int64 units per kcal/mol

// error bits in the context's device error word
enum : int {
  kErrListCap = 1,       // a cluster's neighbour list exceeded its capacity
  kErrOverflow = 2,      // fixed-point range exceeded or non-finite force/energy
  kErrExcl = 4,          // an atom has more than kMaxExcl exclusions
  kErrBox = 8,           // cutoff or list radius inconsistent with the box
};

// One window's periodic box.  Every window starts in the leg's box; with a
// barostat each window's box changes on its own.
struct BoxW {
  float Lf[3], invLf[3];
  float pme_pref;                       // KE / (pi V)
  float pad_;
  double L[3], invL[3];
  double bg_pref;                       // KE pi / (2 V alpha^2)
  double vol;
};

__host__ __device__ inline BoxW make_box(const double* L, double alpha) {
  BoxW b;
  for (int d = 0; d < 3; ++d) {
    b.L[d] = L[d];
    b.invL[d] = 1.0 / L[d];
    b.Lf[d] = (float)L[d];
    b.invLf[d] = (float)(1.0 / L[d]);
  }
  b.vol = L[0] * L[1] * L[2];
  b.pme_pref = (float)(kKE / (3.14159265358979323846 * b.vol));
  b.bg_pref = kKE * 3.14159265358979323846 / (2.0 * b.vol * alpha * alpha);
  b.pad_ = 0.f;
  return b;
}

// Barostat state of one window
struct BaroW {
  double dv_max;                        // half-width of the volume proposal, A^3
  double u0, u1;                        // window energy before / after the trial move
  double vol_old, vol_new, scale, work;
  int due, accepted, n_att, n_acc;      // this attempt; attempts and acceptances in the block of 10
  float used_old;                       // skin_used before the trial move
  int pad2_;
  int rebuilt, pad_;                    // lists rebuilt for the trial move
  long long total_att, total_acc;
};

// Per-leg device descriptor: sizes, parameters, and pointers into the
// caller's state and the leg's private workspace.
struct LegDev {
  int n, W, npad, nclus, cap;           // atoms, windows, padded atoms, clusters, list cap
  int nexcl, nbonds, nwat, nfree, nlig;
  int K[3], Ktot, npair;
  int nbits, ncoarse, ncell;            // fine cells = 2^nbits per axis (Hilbert order)
  int nrad[3], rad[3][kMaxRadix];       // FFT radix plan per axis
  int has_rest, ranch[6];
  float rg0[6], rk[6];
  BoxW box0;                            // the leg's box at set-up (u_kn frames given without boxes)
  int pack;                             // 1: windows 2p, 2p+1 share complex grid p (equal boxes);
                                        // 0: one window per grid (each window its own box)
  float rc2, alpha, sc_alpha, skin_half2, skin;
  double rc2d;                          // r_cut^2 in FP64 (u_kn distance test)
  double rcd, alphad, sc_alphad;        // r_cut, Ewald alpha and softcore alpha in FP64 (energy terms)
  double rg0d[6], rkd[6];               // restraint reference geometry and force constants in FP64
  double rlist, rlist2;
  float d_oh, d_hh;
  double self_pref;                     // KE alpha / sqrt(pi)
  // topology (caller-owned)
  const float *q, *sig, *eps, *mass;
  const uint8_t* lig;
  const int *excl_ij, *excl_ptr, *excl_idx;
  const int* bond_ij;
  const float *bond_k, *bond_r0;
  const int* water;
  const int *bptr, *bnb, *bid;          // per-atom bonds: CSR [n + 1] over (partner atom, bond index)
  int ntors;                            // rotatable torsions (scaled by lambda_vdw)
  const int* tors;                      // [ntors][4] atoms
  const float *tors_k, *tors_phase;     // [ntors]
  const int* tors_n;                    // [ntors]
  const int *tptr, *tid;                // per-atom torsions: CSR [n + 1] over 4 t + (the atom's place in t)
  const float* aoff;                    // [n] alchemical-water charge offsets (NULL: none)
  int naw;                              // alchemical-water atoms (nonzero offset)
  int* aw_idx;                          // [naw] those atoms, then their two exclusion partners each [2 naw]
  int plain;                            // 1: felis_step accumulates pair and reciprocal forces in fd
  double* fd;                           // [3][W][n] FP64 force sums of the plain form (cleared by the integrator)
  // state (caller-owned) [W][n]
  float *x, *y, *z, *vx, *vy, *vz;
  long long *fx, *fy, *fz;
  double* energy;                       // [W][FELIS_NE]
  // workspace (library-owned layout)
  BoxW* box;                            // [W] each window's box
  BoxW* ubox;                           // [2 npair] boxes of the u_kn frames of one pass
  int* rbforce;                         // [W] 1: rebuild the window's lists at the next check
  float* skin_used;                     // [W] list skin consumed by volume moves since the last build (A)
  // barostat (legs with a pressure; nmol = 0 otherwise)
  int nmol;                             // molecules: bonded components, rigid waters joined
  const int* mol_ptr;                   // [nmol + 1] CSR over mol_atoms
  const int* mol_atoms;                 // [n]
  BaroW* baro;                          // [W]
  BoxW* boxb;                           // [W] box before the trial move
  float *xb, *yb, *zb;                  // [W][n] positions before the trial move
  float* molr;                          // [W][nmol] largest atom distance from its molecule's centre
  float* lam;                           // [W][4] per replica: elec, vdw, restraint, sc_alpha*(1-vdw) of
                                        // the state it holds
  const float* lamS;                    // [W][4] the same rows in state order (the leg's lambda table)
  int* rstate;                          // [W] state held by each replica (identity until an exchange)
  int* free_atoms;                      // [nfree] atoms not in a rigid water
  int* lig_idx;                         // [nlig] ligand atoms
  float *xr, *yr, *zr;                  // [W][n] positions at the last list build
  int* flag;                            // [W] rebuild flags
  long long* nbuild;                    // [W] list builds since init
  unsigned* maxdisp;                    // [W] largest squared displacement since the last check (float bits),
                                        // used when a window has fewer than 64 integration units
  unsigned* wmax;                       // [waves][2] per integrator wave: largest squared displacement in
                                        // its first and in its second window (float bits)
  int units;                            // integration units per window (rigid waters + other atoms)
  const unsigned* hcell;                // [ncell] Hilbert index of fine cell (x * 2^nbits + y) * 2^nbits + z
  int* perm;                            // [W][npad] sorted slot -> atom (-1 = padding)
  int* cellcode;                        // [W][n]
  int* cellstart;                       // [W][ncell + 1]
  int* cursor;                          // [W][ncell]
  float4* xyzq;                         // [W][npad] x, y, z, q_scaled * sqrt(KE)
  float2* prm;                          // [W][npad] sigma/2 and 2 sqrt(eps), negated (sign bit set) for a ligand atom
  float4* gsten;                        // [W][npad] PME stencil: offsets fx, fy, fz and the packed bases
  float4* bblo;                         // [W][nclus] cluster bounding boxes (wrapped)
  float4* bbhi;
  int* lcount;                          // [W][nclus][2] entries per half-cluster list
  unsigned* lent;                       // [W][nclus][2][cap]: list of the cluster's atoms 0-3 and of
                                        // atoms 4-7 (slot << 8 | 4-bit mask over the half's atoms)
  long long *frx, *fry, *frz;           // [W][n] reciprocal-space forces of the current MD step
  long long* grid64;                    // [2 npair][Ktot] u_kn ligand charge grids, fixed point
  float2* cgrid;                        // [npair][Ktot] complex grids
  float2* tw[3];                        // [K] exp(-2 pi i k / K) per axis
  float* bmod[3];                       // [K] B-spline moduli factor per axis
  long long* eacc;                      // [W][FELIS_NE] fixed-point energies
  long long* uacc;                      // [2 npair][3 + kMaxLamV] u_kn fixed-point sums (PME, restraint)
  double* upart;                        // [2 npair][ceil(n/256)][1 + kMaxLamV] u_kn pair partials
  double* lpart;                        // [2 npair][1 + kMaxLamV] ligand-ligand partials
  int* err;                             // context error word
  int* need;                            // context: largest list length seen
  int leg_index;                        // position of this leg in the launched batch
};

// Maps a flat block index to (leg, block within leg) for batched launches.
struct BlockMap {
  int n_legs;
  int start[kMaxLegs + 1];
};

// Charge of atom a in a window with lambda_elec le (section "Double
// annihilation protocol"): ligand charges scaled by le; alchemical-water
// atoms take up (1 - le) of their offset.
__device__ __forceinline__ float window_charge(const LegDev& g, int a, float le) {
  const float q = g.q[a] * (g.lig[a] ? le : 1.0f);
  return g.aoff ? fmaf(1.0f - le, g.aoff[a], q) : q;
}
__device__ __forceinline__ double window_charge_fp64(const LegDev& g, int a, double le) {
  const double q = (double)g.q[a] * (g.lig[a] ? le : 1.0);
  return g.aoff ? q + (1.0 - le) * (double)g.aoff[a] : q;
}

__device__ __forceinline__ int find_leg(const BlockMap& m, int b) {
  int lo = 0, hi = m.n_legs - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (m.start[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Sites that convert to fixed point; the first overflow records its site and
// the window/atom (or item) it happened at in err[2], err[3].
enum : int {
  kSitePairs = 1, kSitePairsE = 2, kSiteExcl = 3, kSiteBonded = 4, kSiteGather = 5, kSiteGatherE = 6,
  kSiteUkn = 7, kSiteSelf = 8, kSiteEnergy = 9, kSiteList = 10, kSiteExclCount = 11
};

// err[2] = site, err[3] = where (window << 20 | atom for per-atom sites),
// err[4] = leg index in the batch, all recorded by the first overflow only.
// Latch an error bit; the first error to arrive also records where it
// happened (site code, window << 20 | atom, leg index in the batch).
__device__ __forceinline__ void latch(int* err, int bit, int site, int where, int leg) {
  atomicOr(err, bit);
  if (atomicCAS(&err[2], 0, site ? site : -1) == 0) { err[3] = where; err[4] = leg; }
}

__device__ __forceinline__ long long to_fixed(double v, double scale, int* err, int site = 0, int where = -1,
                                              int leg = -1) {
  double s = v * scale;
  if (!(fabs(s) < 9.0e18)) {
    latch(err, kErrOverflow, site, where, leg);
    return 0;
  }
  return __double2ll_rn(s);
}

// A device pointer seen in the global address space: loads through it are
// global (not flat) instructions, which count only against the vector-memory
// counter, so a load issued early stays in flight across later work.
template <typename T>
using gptr = const T __attribute__((address_space(1)))*;
template <typename T>
__device__ __forceinline__ gptr<T> as_global(const T* p) { return (gptr<T>)p; }
// float4 records read through a global pointer as a native 4-vector
typedef float f32x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ gptr<f32x4> as_global4(const float4* p) { return (gptr<f32x4>)p; }
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ gptr<f32x2> as_global2(const float2* p) { return (gptr<f32x2>)p; }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Index of cell (x, y, z) along a 3D Hilbert curve of 2^bits cells per axis
// (Skilling's transpose construction: undo excess work, Gray-code, then
// interleave).  Consecutive indices are face-adjacent cells, and the 8
// children of every aligned 2x2x2 block hold 8 consecutive indices, so a
// coarse block's atoms form one contiguous range of the sorted order.  The
// kernels read it from per-leg tables filled on the host at leg set-up.
// PME grid coordinate of a position along one axis, in FP64: the base grid
// index b (the stencil covers b, b-1, b-2, b-3, periodic) and the offset
// f in [0, 1) of the order-4 B-spline weights
__device__ __forceinline__ int grid_base(float x, double invL, int K, float* f) {
  double u = (double)x * invL * (double)K;
  if (!(fabs(u) < 1.0e15)) u = 0.0;              // non-finite input -> 0 (keeps indices in range)
  const double b = floor(u);
  *f = (float)(u - b);
  // b mod K without 64-bit integer division: |b| < 2^53, so the FP64 floor
  // of b / K is off by at most one, which the integer fix-ups absorb
  int k = (int)(b - (double)K * floor(b * (1.0 / (double)K)));
  if (k < 0) k += K;
  if (k >= K) k -= K;
  return k;
}

// a slot's three base indices (7 bits each: K <= 128) packed in one word
__device__ __forceinline__ float pack_bases(int bx, int by, int bz) {
  return __int_as_float(bx | (by << 7) | (bz << 14));
}
__device__ __forceinline__ void unpack_bases(float v, int* b) {
  const int u = __float_as_int(v);
  b[0] = u & 127; b[1] = (u >> 7) & 127; b[2] = (u >> 14) & 127;
}

// Philox4x32-10 (Salmon et al. 2011): ten rounds on the counter c with key
// (k0, k1); the output words replace c.
__device__ __forceinline__ void philox(unsigned c[4], unsigned k0, unsigned k1) {
  const unsigned M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const unsigned hi0 = __umulhi(M0, c[0]), lo0 = M0 * c[0];
    const unsigned hi1 = __umulhi(M1, c[2]), lo1 = M1 * c[2];
    const unsigned n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
    k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
  }
}

__host__ __device__ inline unsigned hilbert3(unsigned x, unsigned y, unsigned z, int bits) {
  unsigned X[3] = {x, y, z};
  for (unsigned Q = 1u << (bits - 1); Q > 1u; Q >>= 1) {
    const unsigned P = Q - 1u;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      if (X[i] & Q) {
        X[0] ^= P;
      } else {
        const unsigned t = (X[0] ^ X[i]) & P;
        X[0] ^= t;
        X[i] ^= t;
      }
    }
  }
  X[1] ^= X[0];
  X[2] ^= X[1];
  unsigned t = 0;
  for (unsigned Q = 1u << (bits - 1); Q > 1u; Q >>= 1)
    if (X[2] & Q) t ^= Q - 1u;
  X[0] ^= t; X[1] ^= t; X[2] ^= t;
  unsigned h = 0;
  for (int b = bits - 1; b >= 0; --b)
    h = (h << 3) | (((X[0] >> b) & 1u) << 2) | (((X[1] >> b) & 1u) << 1) | ((X[2] >> b) & 1u);
  return h;
}

__device__ __forceinline__ float wrapf(float x, float L, float invL) {
  const float r = x - L * floorf(x * invL);
  return (r >= 0.f && r < L) ? r : 0.f;          // non-finite input -> 0 (keeps indices in range)
}

// Block-map construction on the host: blocks_of(leg) blocks for each leg.
template <typename F>
inline int make_map(BlockMap& m, int n_legs, F blocks_of) {
  m.n_legs = n_legs;
  int s = 0;
  for (int i = 0; i < n_legs; ++i) { m.start[i] = s; s += blocks_of(i); }
  m.start[n_legs] = s;
  for (int i = n_legs + 1; i <= kMaxLegs; ++i) m.start[i] = s;
  return s;
}

// Host-side mirror of the sizes each launcher needs.
struct LegHost {
  int n, W, npad, nclus, cap, nexcl, nbonds, nwat, nfree, nlig, K[3], Ktot, npair, ncell, ntors, naw;
  int has_rest;
  int nmol;                             // > 0 only for legs with a barostat
};

// One barostat attempt for a batch: which legs move, their attempt index,
// noise key and pressure (kcal / (mol A^3))
struct BaroArgs {
  int due[kMaxLegs];
  long long attempt[kMaxLegs];
  unsigned long long seed[kMaxLegs];
  double pressure[kMaxLegs];
  double kT;
};

// ---- launchers (one per translation unit) ----
void launch_check(hipStream_t s, const LegDev* d, const LegHost* h, int nl, int force, bool from_word);
void launch_build(hipStream_t s, const LegDev* d, const LegHost* h, int nl);
// launch_build in two parts: the cell sort of large legs and the pack (all
// that PME needs), then the cluster lists
void launch_sort_pack(hipStream_t s, const LegDev* d, const LegHost* h, int nl);
void launch_lists(hipStream_t s, const LegDev* d, const LegHost* h, int nl);
void launch_export(hipStream_t s, const LegDev* d, const LegHost& h, int window, double r,
                   int* pairs, long long cap, unsigned long long* count);
void launch_pack(hipStream_t s, const LegDev* d, const LegHost* h, int nl, bool rebuild);
// energy: 0 forces only; 1 also energies from the FP32 pair terms (summed in
// FP64); 2 also energies with every term evaluated in FP64
// step: inside felis_step (legs in the plain form accumulate in fd)
void launch_pairs(hipStream_t s, const LegDev* d, const LegHost* h, int nl, int energy, bool step = false);
void launch_corrections(hipStream_t s, const LegDev* d, const LegHost* h, int nl, bool energy);
void launch_bonded(hipStream_t s, const LegDev* d, const LegHost* h, int nl, int energy);
// step_forces: the gather stores each atom's force in frx/fry/frz (read by the
// integrator) instead of adding it to fx/fy/fz
void launch_pme(hipStream_t s, const LegDev* d, const LegHost* h, int nl, bool energy, bool step_forces = false);
void launch_integrate(hipStream_t s, const LegDev* d, const LegHost* h, int nl,
                      const long long* step, const unsigned long long* seed, float dt,
                      float temperature, float gamma);
void launch_zero_energy(hipStream_t s, const LegDev* d, const LegHost* h, int nl, int c0, int c1);
void launch_finish_energy(hipStream_t s, const LegDev* d, const LegHost* h, int nl, int c0, int c1);
void launch_fill_i64(hipStream_t s, long long* p, size_t n);
// ukn_mode: 0 the MD grids; u_kn int64 grids of 1 two frames per complex grid
// or 2 one frame per grid (boxes from ubox)
void launch_pme_fft(hipStream_t s, const LegDev* d, const LegHost* h, int nl, int ukn_mode);
void launch_hrex(hipStream_t s, const LegDev* d, const LegHost& h, const double* u, long long u_stride,
                 long long attempt, unsigned long long seed, int* accepted);
int launch_ukn(hipStream_t s, const LegDev* d, const LegHost& h, double sc_alpha, const double* lambdas,
               int K, const float* fx, const float* fy, const float* fz, long long frame_stride,
               long long n_frames, const double* frame_box, double pressure, double beta, double* u,
               long long u_stride, long long* uacc, double* cst);
// barostat: proposal, box change and molecule move of the due windows; the
// energy before the move; Metropolis test, restore of rejected moves
void launch_baro_propose(hipStream_t s, const LegDev* d, const LegHost* h, int nl, const BaroArgs& A);
void launch_baro_keep_u0(hipStream_t s, const LegDev* d, const LegHost* h, int nl);
void launch_baro_accept(hipStream_t s, const LegDev* d, const LegHost* h, int nl, const BaroArgs& A);
int launch_mbar(hipStream_t s, const double* u, const int* N_k, int K, long long Ntot, double tol,
                int max_iter, double* f_out, int* iters, void* work, size_t work_bytes);
size_t mbar_work_bytes(int K, long long Ntot);
// allocation-free MBAR: workspace in a static device array of kMbarStaticBytes
constexpr size_t kMbarStaticBytes = size_t(64) << 20;
int mbar_scratch_setup(int device);
int launch_mbar_noalloc(int device, hipStream_t s, const double* u, const int* N_k, int K, long long Ntot,
                        double tol, int max_iter, double* f_out, int* iters);

}  // namespace felis
