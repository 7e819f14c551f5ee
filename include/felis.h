/* felis.h -- C ABI of the MI355X (gfx950) alchemical-window hot path.
 *
 * For every lambda window of an absolute-binding decoupling leg the library
 * evaluates alchemically scaled nonbonded forces and energies, PME reciprocal
 * space, Langevin-middle dynamics with rigid water, the cross-lambda reduced
 * potential matrix u_kn and its MBAR solve.  The method is the one of the
 * paper's sections "Double annihilation protocol" (ligand charges scaled
 * linearly to zero, Beutler softcore 12-6 LJ with lambda_ij = min(lambda_i,
 * lambda_j), alpha = 0.5, p = 1, Lorentz-Berthelot mixing), "Restraints"
 * (Boresch distance/angle/dihedral set), "Simulation protocol" (Langevin
 * middle integrator, 2 fs, rigid TIP3P, MBAR) and appendix B (1 nm PME and
 * vdW cutoffs, universal lambda schedules).
 *
 * Units: angstrom, ps, amu, e, kcal/mol, K.
 * Precision: pair, PME and integrator arithmetic in FP32; forces accumulate in
 * int64 fixed point (FELIS_FORCE_SCALE units per kcal/mol/A), so results are
 * bitwise reproducible; energies, u_kn and MBAR in FP64 (energy partial sums
 * are combined in int64 fixed point at 2^-30 kcal/mol).
 * Memory: every device buffer is allocated and owned by the caller (e.g. a
 * PyTorch tensor's data pointer).  The library never frees caller memory and
 * allocates device memory only in felis_create (a few KB of tables and an
 * error word); felis_mbar_noalloc uses a static 64 MiB device array instead
 * of a workspace.  Per-leg scratch lives in caller memory sized by
 * felis_leg_work_size.
 * Streams: every call is enqueued on the HIP stream given to felis_create and
 * returns without waiting, except felis_leg_init, felis_check,
 * felis_check_detail, felis_leg_rebuilds, felis_nlist_export_pairs,
 * felis_mbar and felis_mbar_noalloc (they synchronise that stream).
 * Errors: every function returns FELIS_OK (0) or a negative FELIS_E_* code; no
 * exception crosses the ABI and nothing aborts.  Device-side faults (list
 * capacity, fixed-point overflow, non-finite forces) are latched in a device
 * error word and reported by the next felis_check.  felis_last_error gives a
 * message for the last failing call on the context.
 * Threads: one context per host thread and stream; no global state.
 */
#ifndef FELIS_H
#define FELIS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FELIS_OK 0
#define FELIS_E_INVAL (-1)       /* bad argument, size or pointer */
#define FELIS_E_DEVICE (-2)      /* HIP runtime error */
#define FELIS_E_BOX (-3)         /* r_cut + skin >= half the shortest box edge */
#define FELIS_E_CAPACITY (-4)    /* neighbour list capacity exceeded (see felis_check) */
#define FELIS_E_OVERFLOW (-5)    /* fixed-point range exceeded or non-finite value */
#define FELIS_E_NOCONV (-6)      /* MBAR reached max_iter */
#define FELIS_E_UNSUPPORTED (-7) /* spline order != 4, softcore p != 1, grid > 128 ... */

#define FELIS_FORCE_SCALE 4294967296.0   /* int64 force units per kcal/mol/A (2^32) */

/* energy vector of one window, kcal/mol */
#define FELIS_NE 8
enum {
  FELIS_E_COUL_REAL = 0, /* real-space erfc Coulomb over non-excluded pairs < r_cut */
  FELIS_E_LJ = 1,        /* softcore / plain 12-6 LJ over non-excluded pairs < r_cut */
  FELIS_E_EXCL = 2,      /* -KE q_i q_j erf(alpha r)/r over excluded pairs */
  FELIS_E_SELF = 3,      /* Ewald self term + neutralising-background term */
  FELIS_E_RECIP = 4,     /* PME reciprocal energy */
  FELIS_E_BOND = 5,      /* bonded: harmonic bonds (k/2)(r - r0)^2 + lambda_vdw x rotatable torsions */
  FELIS_E_RESTRAINT = 6, /* lambda_restraint x Boresch energy */
  FELIS_E_TOTAL = 7
};

/* flags for felis_nonbonded / felis_pme / felis_bonded */
#define FELIS_ENERGY 1   /* also compute the call's energy components */

typedef struct felis_ctx felis_ctx;

/* One decoupling leg: a periodic orthorhombic system and its windows.
 * Pointers marked (dev) are device pointers owned by the caller and must stay
 * valid while the leg is used; (host) pointers are read during the call only. */
typedef struct felis_leg {
  int32_t n_atoms;
  double box[3];                 /* edges, A */
  double r_cut;                  /* real-space Coulomb and LJ cutoff, A */
  double skin;                   /* neighbour-list buffer: list radius = r_cut + skin */
  double ewald_alpha;            /* Ewald splitting parameter, 1/A */
  double sc_alpha;               /* softcore alpha (paper: 0.5) */
  int32_t sc_p;                  /* softcore power (paper: 1; only 1 is supported) */
  int32_t grid[3];               /* PME grid, each 2^a 3^b 5^c and <= 128 */
  int32_t spline_order;          /* PME B-spline order (only 4 is supported) */
  const float* charge;           /* (dev) [n_atoms] e, unscaled */
  const float* sigma;            /* (dev) [n_atoms] LJ sigma, A */
  const float* epsilon;          /* (dev) [n_atoms] LJ epsilon, kcal/mol */
  const float* mass;             /* (dev) [n_atoms] amu */
  const uint8_t* is_ligand;      /* (dev) [n_atoms] 1 = alchemical ligand atom */
  int32_t n_excl;                /* excluded pairs (rigid-water and bonded 1-2 / 1-3) */
  const int32_t* excl_ij;        /* (dev) [n_excl][2], i < j */
  const int32_t* excl_ptr;       /* (dev) [n_atoms + 1] CSR of the same set, symmetric */
  const int32_t* excl_idx;       /* (dev) [2 n_excl] */
  int32_t n_bonds;
  const int32_t* bond_ij;        /* (dev) [n_bonds][2] */
  const float* bond_k;           /* (dev) [n_bonds] kcal/mol/A^2, energy (k/2)(r - r0)^2 */
  const float* bond_r0;          /* (dev) [n_bonds] A */
  int32_t n_waters;
  const int32_t* water_ohh;      /* (dev) [n_waters][3] O, H1, H2 (rigid, SETTLE) */
  double d_oh, d_hh;             /* rigid water geometry, A */
  int32_t has_restraint;         /* 1: Boresch restraint on the anchors below */
  int32_t restraint_atoms[6];    /* P1 P2 P3 L1 L2 L3 */
  double restraint_g0[6];        /* r0 (A), thetaA0, thetaB0, phiA0, phiB0, phiC0 (rad) */
  double restraint_k[6];         /* k_r (kcal/mol/A^2), k_theta x2 (kcal/mol/rad^2), k_phi x3 (kcal/mol) */
  int32_t n_windows;
  const double* lambdas;         /* (host) [n_windows][3] lambda_elec, lambda_vdw, lambda_restraint */
  float *x, *y, *z;              /* (dev) [n_windows][n_atoms] positions, A (never wrapped) */
  float *vx, *vy, *vz;           /* (dev) [n_windows][n_atoms] velocities, A/ps */
  int64_t *fx, *fy, *fz;         /* (dev) [n_windows][n_atoms] forces, FELIS_FORCE_SCALE units */
  double* energy;                /* (dev) [n_windows][FELIS_NE] */
  uint64_t seed;                 /* noise key of this leg */
  int64_t step;                  /* index of the next MD step (advanced by felis_step) */
  int32_t list_cap;              /* list entries per 8-atom cluster; 0 = sized from density */
  double pressure_bar;           /* > 0: NPT; a Monte Carlo barostat at this pressure gives each
                                    window its own box (section "Simulation protocol"); 0: every
                                    window keeps `box` */
  int32_t barostat_every;        /* MD steps between volume moves (with pressure_bar > 0) */
  int32_t n_torsions;            /* rotatable ligand torsions, scaled linearly with lambda_vdw
                                    (section "Double annihilation protocol"); 0 = none */
  const int32_t* torsion_ijkl;   /* (dev) [n_torsions][4] atoms a, b, c, d (rotatable bond b-c) */
  const float* torsion_k;        /* (dev) [n_torsions] kcal/mol: energy lambda_vdw k [1 + cos(n phi - delta)] */
  const int32_t* torsion_n;      /* (dev) [n_torsions] periodicity n >= 1 */
  const float* torsion_phase;    /* (dev) [n_torsions] delta, rad */
  const float* alch_offset;      /* (dev) [n_atoms] or NULL: alchemical waters (section "Double
                                    annihilation protocol": charged ligands): atom i's charge in a
                                    window is q_i (x lambda_elec for ligand atoms) + (1 - lambda_elec)
                                    alch_offset[i], nonzero on the designated waters only, so the net
                                    charge is the same in every window */
  int32_t plain_fp64;            /* 1: the plain form, for comparison only: inside felis_step the pair
                                    and reciprocal-space forces are accumulated with FP64 atomics
                                    (order-dependent, not bitwise reproducible) instead of int64 fixed
                                    point; 0: the default fixed-point accumulation */
  void* work;                    /* (dev) library scratch of work_bytes */
  size_t work_bytes;
} felis_leg;

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t, NULL = default stream).  FELIS_E_DEVICE if the device or
 * its allocation of the context's tables fails. */
int felis_create(felis_ctx** out, int device, void* hip_stream);
void felis_destroy(felis_ctx* ctx);
const char* felis_last_error(const felis_ctx* ctx);

/* Synchronise the stream and report the device error word:
 * FELIS_E_CAPACITY (list overflow; *needed_cap, if non-NULL, receives the
 * longest cluster list seen), FELIS_E_OVERFLOW, FELIS_E_INVAL, or FELIS_OK.
 * Clears the word. */
int felis_check(felis_ctx* ctx, int32_t* needed_cap);

/* As felis_check, and also reports where the first fixed-point overflow was
 * latched: the leg's position in the batch of the failing call, the window
 * and the atom (-1 where unknown or when no error is latched).  Lets a caller
 * running many legs in one batch evict only the failing leg. */
int felis_check_detail(felis_ctx* ctx, int32_t* needed_cap, int32_t* leg, int32_t* window, int32_t* atom);

/* Bytes of device scratch a leg needs (lists, sorted copies, PME grids,
 * accumulators).  Validates the leg's sizes: FELIS_E_BOX, FELIS_E_UNSUPPORTED,
 * FELIS_E_INVAL.  The descriptor's array pointers are checked for null but
 * never dereferenced, so a size query needs no allocation. */
int felis_leg_work_size(const felis_leg* leg, size_t* bytes);

/* Fill the leg's scratch (lambda table, FFT tables, water/ligand index
 * tables) and mark every window for a list build.  Call once after the
 * topology and initial positions are in place, and again after positions are
 * replaced from outside.  Synchronises the stream. */
int felis_leg_init(felis_ctx* ctx, felis_leg* leg);

/* Neighbour lists (appendix B cutoffs; list radius r_cut + skin).  Per window,
 * atoms are sorted along a Hilbert curve of fine cells and grouped into
 * 8-atom clusters; each cluster lists every atom j with, for each of its atoms
 * i, a bit that is set when j != i, (i, j) is not excluded and the FP32
 * minimum-image distance is below r_cut + skin + 0.01 A.  The 0.01 A margin
 * is far above the FP32 error of the distance, so the listed pairs are a
 * superset of the exact set {|d_ij| < r_cut + skin in FP64}; the pair kernel
 * applies the cutoff r_cut itself, and felis_nlist_export_pairs applies the
 * FP64 test to give the exact set.  With force = 0 only windows whose atoms
 * moved more than skin/2 since their last build are rebuilt; force = 1
 * rebuilds all. */
int felis_build_nlist(felis_ctx* ctx, felis_leg* legs, int n_legs, int force);

/* Neighbour-list builds of each window since felis_leg_init (forced builds
 * included): counts (host) [n_windows].  Synchronises the stream. */
int felis_leg_rebuilds(felis_ctx* ctx, const felis_leg* leg, int64_t* counts);

/* Test/diagnostic export of window `window`'s list: every pair (i < j) whose
 * list bit is set and whose FP64 minimum-image distance (dx = x_j - x_i,
 * dx -= L rint(dx / L) as a separate multiply and subtract, d^2 = (dx^2 +
 * dy^2) + dz^2, no contraction) is < r is written to pairs[2 k],
 * pairs[2 k + 1] (dev, capacity `cap` pairs, unordered).  With r = r_cut +
 * skin the result is the exact FP64 list.  *n_pairs receives the count (also
 * when it exceeds cap, then FELIS_E_CAPACITY; cap = 0 with pairs = NULL only
 * counts).  Synchronises. */
int felis_nlist_export_pairs(felis_ctx* ctx, const felis_leg* leg, int window, double r,
                             int32_t* pairs, int64_t cap, int64_t* n_pairs);

/* Real-space part for every window of every leg ("Double annihilation
 * protocol"): erfc Coulomb with ligand charges x lambda_elec, softcore LJ
 * (lambda_ij = lambda_vdw when i or j is ligand, else plain LJ), both cut at
 * r_cut, plus the excluded-pair, self and background Ewald terms.  Forces are
 * OVERWRITTEN (this call starts a force evaluation); with FELIS_ENERGY the
 * components COUL_REAL, LJ, EXCL, SELF and TOTAL are written. */
int felis_nonbonded(felis_ctx* ctx, felis_leg* legs, int n_legs, int flags);

/* PME reciprocal space, the long-range part of the electrostatics that
 * appendix B cuts at 1 nm in real space (the paper names PME and prints no
 * formula; this is smooth PME of Essmann et al. 1995): charges (ligand ones
 * scaled by lambda_elec, section "Double annihilation protocol") spread with
 * order-4 cardinal B-splines, 3D FFT, the influence function
 * exp(-pi^2 m^2 / alpha^2) / (pi V m^2) times the B-spline moduli, inverse FFT
 * and gather; E_rec = (KE / 2) sum_m G(m) |F(Q)(m)|^2.  Forces are ADDED;
 * with FELIS_ENERGY writes RECIP and TOTAL.
 * Spreading locates atoms through the neighbour-list cell sort, so this call
 * first rebuilds the lists of windows that moved more than skin/2 (as
 * felis_build_nlist with force = 0 does). */
int felis_pme(felis_ctx* ctx, felis_leg* legs, int n_legs, int flags);

/* Harmonic bonds, lambda_vdw-scaled rotatable torsions (section "Double
 * annihilation protocol") and the lambda_restraint-scaled Boresch restraint
 * (section "Restraints"); forces are ADDED; with FELIS_ENERGY writes BOND
 * (bonds and torsions), RESTRAINT and TOTAL. */
int felis_bonded(felis_ctx* ctx, felis_leg* legs, int n_legs, int flags);

/* n_steps Langevin-middle steps ("Simulation protocol") for every window:
 * list check/rebuild, forces (nonbonded + PME + bonded), then
 * v += dt F/m; x += dt/2 v; v = a v + sqrt((1-a^2) kT/m) xi; x += dt/2 v;
 * SETTLE on rigid waters; v += (x_constrained - x_unconstrained)/dt, with
 * a = exp(-gamma dt) and xi from Philox4x32-10 keyed by (leg seed) and
 * counted by (atom, window, step), so a window's trajectory does not depend
 * on the batch it runs in.  Each leg's `step` advances by n_steps.  Reciprocal
 * space runs on a second stream owned by the context, forked after the cell
 * sort and joined before the integrator, so all of the call's work is ordered
 * on the context's stream; after the call fx/fy/fz hold the total force of
 * the last step. */
int felis_step(felis_ctx* ctx, felis_leg* legs, int n_legs, int n_steps, double dt,
               double temperature, double gamma);

/* Reduced potentials of n_frames frames of one leg at K lambda states, the
 * input MBAR needs for each segment's free energy (section "Simulation
 * protocol"); the lambda dependence follows section "Double annihilation
 * protocol" (charges scaled by lambda_elec, so ligand-environment terms scale
 * as lambda_elec and ligand-ligand terms as lambda_elec^2; softcore LJ at
 * lambda_vdw) and section "Restraints" (Boresch energy x lambda_restraint):
 * u[k * u_stride + f] = beta [lam_e E_LE + lam_e^2 E_LL + E_sc(lam_v) + lam_v U_T + lam_r U_B + P V_f]
 * (U_T: the rotatable torsions, unscaled)
 * (lambda-independent terms dropped; MBAR is invariant to them; the P V term
 * only for legs with pressure_bar > 0).  Frame f's coordinates are
 * fx/fy/fz + f * frame_stride (dev, float, n_atoms each); frame_box (dev,
 * [n_frames][3] edges in A, or NULL: every frame in the leg's `box`) gives
 * each frame's periodic box (NPT frames).  lambdas (host) [K][3].  Uses the
 * leg's scratch (call felis_leg_init first); at most 64 distinct lambda_vdw
 * values and 256 ligand atoms.  n_frames = 0 is a no-op (the frame and u
 * pointers are then not read); FELIS_E_INVAL for K < 1, lambdas outside
 * [0, 1], frame_stride < n_atoms or u_stride < n_frames. */
int felis_ukn(felis_ctx* ctx, felis_leg* leg, const double* lambdas, int K, const float* fx,
              const float* fy, const float* fz, int64_t frame_stride, int64_t n_frames,
              const double* frame_box, double beta, double* u, int64_t u_stride);

/* Monte Carlo barostat ("Simulation protocol": NPT at 1.01325 bar, a volume
 * move every 25 steps) for legs with pressure_bar > 0.  Each window (replica)
 * has its own box and moves on its own: V' = V + dV_max (2 u1 - 1), box edges
 * scaled by s = (V'/V)^(1/3), every molecule (bonded component, rigid waters
 * joined) translated rigidly so that the mean of its atom positions scales
 * by s; accepted when w = U' - U + P (V' - V) - N_mol kT ln(V'/V) <= 0 or
 * u2 < exp(-w/kT), otherwise positions and box are restored (velocities are
 * never scaled).  U is the window's total energy (all FELIS_NE components,
 * computed by the library before and after the move).  dV_max starts at
 * 0.01 V and is divided by 1.1 after a block of 10 attempts with fewer than
 * a quarter accepted, multiplied by 1.1 (at most 0.3 V) with more than three
 * quarters.  u1, u2 from Philox4x32-10 on counter (window, 0x4241524F,
 * attempt) with the leg's seed as key: u1 = ((w0 >> 5) 2^26 + (w1 >> 6))
 * 2^-53, u2 the same from (w2, w3).
 * felis_step makes the move before every step whose index is a positive
 * multiple of barostat_every (attempt = step / barostat_every);
 * felis_barostat makes one now for every leg of the batch with a pressure
 * (others are left untouched), at the given attempt index, and
 * leaves every window's lists valid for its positions and box.
 * FELIS_E_INVAL if no leg of the batch has a pressure. */
int felis_barostat(felis_ctx* ctx, felis_leg* legs, int n_legs, double temperature, int64_t attempt);

/* Each window's current box edges, edges (host) [n_windows][3].  Synchronises. */
int felis_leg_boxes(felis_ctx* ctx, const felis_leg* leg, double* edges);
/* The same into device memory edges (dev) [n_windows][3], enqueued on the
 * context's stream (e.g. the frame boxes of a felis_ukn sample of the leg's
 * current coordinates). */
int felis_leg_boxes_async(felis_ctx* ctx, const felis_leg* leg, double* edges);

/* Barostat state of each window after the last move, out (host)
 * [n_windows][FELIS_BARO_NS]: U before, U after the trial move (kcal/mol),
 * w (kcal/mol), V, V' (A^3), s, accepted (0/1), dV_max (A^3), attempts and
 * acceptances so far.  Synchronises.  FELIS_E_INVAL for a leg without a
 * pressure. */
#define FELIS_BARO_NS 10
int felis_barostat_stats(felis_ctx* ctx, const felis_leg* leg, double* out);

/* Hamiltonian replica exchange among the windows of one leg (simulation
 * details: exchanges among one GPU's windows every 5 ps).  The leg's windows
 * are replicas; window r holds state state_of_replica[r] (identity after
 * felis_leg_init), and every kernel uses the lambda row of the state a replica
 * holds.  One attempt swaps neighbouring states: pairs (0,1), (2,3), ... when
 * `attempt` is even, (1,2), (3,4), ... when odd; the swap of states s, s+1
 * held by replicas i, j is taken when D = u[s][j] + u[s+1][i] - u[s][i] -
 * u[s+1][j] <= 0 or U < exp(-D), U from Philox4x32-10 on counter
 * (s, 0x48524558, attempt) with key `seed`.  u (dev, FP64): u[k * u_stride + r]
 * is the reduced potential of replica r's current coordinates in state k
 * (felis_ukn of the leg's own lambda table over its n_windows current frames);
 * u_stride >= n_windows.  Coordinates, velocities and lists stay with their
 * replica.  n_accepted (host, may be NULL) receives the number of swaps taken
 * (synchronises when given).  FELIS_E_UNSUPPORTED above 256 windows. */
int felis_hrex(felis_ctx* ctx, felis_leg* leg, const double* u, int64_t u_stride, int64_t attempt, uint64_t seed,
               int32_t* n_accepted);

/* State held by each replica: state_of_replica (host) [n_windows].
 * Synchronises the stream. */
int felis_leg_states(felis_ctx* ctx, const felis_leg* leg, int32_t* state_of_replica);

/* Free energy (kcal/mol, written to *dg) of imposing the Boresch restraints
 * on the decoupled ligand from the 1 mol/L standard state (V0 = 1660.539 A^3),
 * the analytic term of dG_bind = dG_solvent - dG_complex + dG_restrain (figure 1,
 * section "Restraints").  The paper's closed form is not printed; this is the
 * harmonic-limit expression of Boresch et al. 2003:
 *   kT ln[8 pi^2 V0 sqrt(k_r k_thA k_thB k_phA k_phB k_phC) / (r0^2 sin thA0 sin thB0 (2 pi kT)^3)]
 * with the cosine dihedrals k[1 - cos] at their second-order limit.  g0, k
 * (host) [6] in the leg's restraint order (distance, the angles at L1 and P1,
 * the three dihedrals; A, rad, kcal/mol/A^2, kcal/mol/rad^2).  Host arithmetic
 * only (no context, no device).  FELIS_E_INVAL unless every k > 0, r0 > 0,
 * 0 < thA0, thB0 < pi and temperature > 0. */
int felis_restraint_dg(const double* g0, const double* k, double temperature, double* dg);

/* A leg's (or segment's) free-energy difference from MBAR's dimensionless
 * free energies (section "Simulation protocol"): *dg = kT (f[K-1] - f[0])
 * kcal/mol, the decoupling direction when the leg's windows run from the
 * coupled to the decoupled state.  f (host) [K].  Host arithmetic only.
 * FELIS_E_INVAL unless K >= 2, temperature > 0 and f is finite. */
int felis_delta_g(const double* f, int K, double temperature, double* dg);

/* Boundary windows of n_segments overlapping segments of a leg of n_windows
 * windows (section "Simulation protocol": each GPU runs a segment of the
 * path, neighbouring segments duplicate their boundary window): segment s
 * spans windows first[s] .. first[s + 1], first[s] = floor(s (n_windows - 1)
 * / n_segments); first (host) [n_segments + 1].  FELIS_E_INVAL unless every
 * segment gets at least two windows. */
int felis_segment_bounds(int n_windows, int n_segments, int32_t* first);

/* Binding free energy (figure 1, section "Restraints"): the leg free
 * energies are the sums of their segments' differences (host arrays of
 * n_solvent and n_complex values, each from felis_delta_g), and
 *   dG_bind = dG_solvent - dG_complex + dG_restrain,
 * with dG_restrain from felis_restraint_dg(g0, k, temperature).  Host
 * arithmetic only; errors as felis_restraint_dg, FELIS_E_INVAL for empty
 * segment lists or non-finite values. */
int felis_binding_dg(const double* dg_solvent_segments, int n_solvent, const double* dg_complex_segments,
                     int n_complex, const double* g0, const double* k, double temperature, double* dg_bind);

/* Kernel timing with HIP events recorded on the context's stream around the
 * launches of one stage inside felis_step / felis_ukn, and around the pair
 * kernel of felis_nonbonded (the events bracket exactly the stage's kernels,
 * so their elapsed time is the stage's device time).  felis_profile(ctx, 1)
 * starts recording every stage, felis_profile(ctx, FELIS_PROF_MASK | m) only
 * the stages whose bit (1 << FELIS_PROF_x) is set in
 * m (each recorded event adds a queue packet between two kernels), 0 stops;
 * felis_profile_read synchronises, returns the summed milliseconds and the
 * number of bracketed launches for stage `which` since the last read, and
 * resets it. */
#define FELIS_PROF_MASK 0x40000000
enum {
  FELIS_PROF_PAIRS = 0,     /* the real-space pair kernel */
  FELIS_PROF_PME = 1,       /* spreading, FFT passes, gather (in felis_step on the context's
                               second stream, sharing compute units with the list build and the
                               pair kernel) */
  FELIS_PROF_NLIST = 2,     /* displacement check and list rebuild */
  FELIS_PROF_INTEGRATE = 3, /* Langevin-middle update with SETTLE */
  FELIS_PROF_UKN = 4,       /* one felis_ukn call */
  FELIS_PROF_BARO = 5,      /* one volume move (two energy evaluations, move, test) */
  FELIS_PROF_N = 6
};
int felis_profile(felis_ctx* ctx, int enable);
/* Bracket only every `every`-th occurrence of each recorded stage (1: all;
 * counted from the last felis_profile call).  FELIS_E_INVAL if every < 1. */
int felis_profile_every(felis_ctx* ctx, int every);
int felis_profile_read(felis_ctx* ctx, int which, double* total_ms, int64_t* launches);

/* Scratch bytes for felis_mbar: about (K + 1) n_total + K^2 (n_total/4096 + 1)
 * doubles. */
int felis_mbar_work_size(int K, int64_t n_total, size_t* bytes);

/* MBAR (Shirts & Chodera 2008; "Simulation protocol") on u (dev, FP64,
 * [K][n_total] row-major, reduced potentials of every sample at every state)
 * and N_k (host, samples drawn from each state; only the counts matter, not
 * the column order).  Solves the MBAR equations by Newton's method on their
 * convex objective (self-consistent steps where the Newton system is
 * singular, a backtracking line search while steps are large) until the full
 * (undamped) step of an iteration satisfies max|df| <= rel_tol * max(1, max|f|);
 * states with N_k = 0 follow from the converged denominators.  f_out (host)
 * [K] dimensionless free energies, gauge f_0 = 0; *iters the Newton
 * iterations used.  FELIS_E_NOCONV at max_iter or on a non-finite result.
 * K in [2, 512].  Synchronises. */
int felis_mbar(felis_ctx* ctx, const double* u, const int32_t* N_k, int K, int64_t n_total,
               double rel_tol, int max_iter, double* f_out, int* iters, void* work,
               size_t work_bytes);

/* felis_mbar without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same solver and result as felis_mbar, with its
 * scratch in a static device array of 64 MiB that each device holds from the
 * first felis_create on it until the process ends.  Allocates nothing (no
 * hipMalloc, hipFree or allocating library call).  FELIS_E_CAPACITY (with a
 * message giving the bytes needed) when the input needs more than 64 MiB of
 * scratch (about (K + 1) n_total + K^2 (n_total / 4096 + 1) doubles; e.g.
 * 42 states x 84,000 samples fit); other errors as felis_mbar.  The array is
 * shared by every call on a device and keeps the last call's contents: calls
 * that overlap on one device (several contexts or threads) race.
 * Synchronises the context's stream. */
int felis_mbar_noalloc(felis_ctx* ctx, const double* u, const int32_t* N_k, int K, int64_t n_total,
                       double rel_tol, int max_iter, double* f_out, int* iters);

#ifdef __cplusplus
}
#endif
#endif /* FELIS_H */
