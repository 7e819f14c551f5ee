"""Seeded synthetic systems for alchemical decoupling legs.

This module only places atoms and draws parameters.  It holds no part of the
method's arithmetic (no pair potential, no Ewald sum, no integrator, no
estimator), so both the FP64 oracle and the HIP path can consume its output.

Systems follow the shapes the paper works with (section "Double annihilation
protocol" for the ligand scaling, section "Restraints" for the Boresch anchor
set, appendix B for cutoffs and the universal schedules):

* ``solvent_leg`` -- rigid 3-site waters on a cubic lattice with random
  orientations plus one bonded ligand chain (a ligand-solvent leg).
* ``complex_leg`` -- a bonded synthetic "protein" chain packed into a sphere,
  a ligand at its surface with a 6-DOF Boresch anchor set, counter-ions and
  lattice water (a protein-ligand leg).

Every array is a numpy array; coordinates are float32 (the canonical inputs),
box and schedule values float64.  Atom order: solute chains first (ligand
first in solvent legs, protein then ligand in complex legs), then ions, then
water.
"""
from __future__ import annotations

import dataclasses
import hashlib
import math

import numpy as np
from scipy.spatial import cKDTree

# TIP3P-geometry water, ion and heavy-atom parameters used by the synthetic
# systems (units: angstrom, e, kcal/mol, amu).
Q_OW, Q_HW = -0.834, 0.417
SIG_OW, EPS_OW = 3.1507, 0.1521
D_OH, ANGLE_HOH = 0.9572, 104.52
M_O, M_H, M_HEAVY = 15.9994, 1.008, 12.011
ION_NA = dict(q=1.0, sigma=2.439, eps=0.0874, mass=22.99)
ION_CL = dict(q=-1.0, sigma=4.478, eps=0.0356, mass=35.45)
BOND_K, BOND_R0 = 300.0, 1.5
BASE_SEED = 22274


@dataclasses.dataclass
class System:
    """One leg: topology, canonical coordinates and the lambda schedule."""

    name: str
    box: np.ndarray            # (3,) float64, orthorhombic box edges
    pos: np.ndarray            # (N, 3) float32
    charge: np.ndarray         # (N,) float32
    sigma: np.ndarray          # (N,) float32
    epsilon: np.ndarray        # (N,) float32
    mass: np.ndarray           # (N,) float32
    is_ligand: np.ndarray      # (N,) uint8
    bonds: np.ndarray          # (nb, 2) int32
    bond_k: np.ndarray         # (nb,) float32
    bond_r0: np.ndarray        # (nb,) float32
    waters: np.ndarray         # (nw, 3) int32  O, H1, H2
    excl: np.ndarray           # (ne, 2) int32  excluded pairs, i < j, sorted
    lambdas: np.ndarray        # (W, 3) float64 columns: elec, vdw, restraint
    r_cut: float
    skin: float
    ewald_alpha: float
    grid: tuple
    sc_alpha: float = 0.5
    sc_p: int = 1
    temperature: float = 300.0
    dt: float = 0.002          # ps
    gamma: float = 0.5         # 1/ps
    d_oh: float = D_OH
    d_hh: float = 2.0 * D_OH * math.sin(math.radians(ANGLE_HOH / 2.0))
    restraint_atoms: np.ndarray | None = None   # (6,) P1 P2 P3 L1 L2 L3
    restraint_g0: np.ndarray | None = None      # (6,) r, thetaA, thetaB, phiA, phiB, phiC
    restraint_k: np.ndarray | None = None       # (6,)
    spline_order: int = 4
    # rotatable ligand torsions, scaled by lambda_vdw: energy k [1 + cos(n phi - delta)]
    torsions: np.ndarray | None = None          # (nt, 4) int32 atoms a-b-c-d (rotatable bond b-c)
    torsion_k: np.ndarray | None = None         # (nt,) float32 kcal/mol
    torsion_n: np.ndarray | None = None         # (nt,) int32 periodicity
    torsion_phase: np.ndarray | None = None     # (nt,) float32 rad
    # alchemical waters (charged ligands): the oxygen of each designated water
    # carries (1 - lambda_elec) * alch_offset[i] on top of its charge, so that
    # the system's net charge stays that of the coupled state in every window
    alch_offset: np.ndarray | None = None       # (N,) float32 e, nonzero only on alchemical-water oxygens

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])

    @property
    def n_windows(self) -> int:
        return int(self.lambdas.shape[0])

    @property
    def r_list(self) -> float:
        return self.r_cut + self.skin

    def excl_csr(self):
        """Symmetric exclusion lists as CSR (ptr[N+1], idx), idx sorted per atom."""
        n = self.n_atoms
        a = np.concatenate([self.excl[:, 0], self.excl[:, 1]])
        b = np.concatenate([self.excl[:, 1], self.excl[:, 0]])
        order = np.lexsort((b, a))
        a, b = a[order], b[order]
        ptr = np.zeros(n + 1, np.int32)
        np.add.at(ptr, a + 1, 1)
        return np.cumsum(ptr).astype(np.int32), b.astype(np.int32)

    def digest(self) -> str:
        h = hashlib.sha256()
        for arr in (self.box, self.pos, self.charge, self.sigma, self.epsilon, self.mass,
                    self.is_ligand, self.bonds, self.waters, self.excl, self.lambdas):
            h.update(np.ascontiguousarray(arr).tobytes())
        return h.hexdigest()


# ---------------------------------------------------------------------------
# geometry helpers (placement only)

def _rng(config: int, purpose: int, seed: int = BASE_SEED) -> np.random.Generator:
    return np.random.default_rng([seed, config, purpose])


def _random_rotations(rng, n):
    """Uniform random rotation matrices from uniform unit quaternions."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a = np.sqrt(1 - u1) * np.sin(2 * np.pi * u2)
    b = np.sqrt(1 - u1) * np.cos(2 * np.pi * u2)
    c = np.sqrt(u1) * np.sin(2 * np.pi * u3)
    d = np.sqrt(u1) * np.cos(2 * np.pi * u3)
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (c * c + d * d); R[:, 0, 1] = 2 * (b * c - a * d); R[:, 0, 2] = 2 * (b * d + a * c)
    R[:, 1, 0] = 2 * (b * c + a * d); R[:, 1, 1] = 1 - 2 * (b * b + d * d); R[:, 1, 2] = 2 * (c * d - a * b)
    R[:, 2, 0] = 2 * (b * d - a * c); R[:, 2, 1] = 2 * (c * d + a * b); R[:, 2, 2] = 1 - 2 * (b * b + c * c)
    return R


def _water_template():
    h = math.radians(ANGLE_HOH / 2.0)
    return np.array([[0.0, 0.0, 0.0],
                     [D_OH * math.sin(h), D_OH * math.cos(h), 0.0],
                     [-D_OH * math.sin(h), D_OH * math.cos(h), 0.0]])


def _orient_waters(rng, centers, box, fixed_pts=None, tries=60):
    """Random orientations for waters with O at ``centers``; orientations whose
    H atoms come too close to another molecule are re-drawn."""
    tmpl = _water_template()
    n = len(centers)
    R = _random_rotations(rng, n)
    for _ in range(tries):
        xyz = centers[:, None, :] + np.einsum('nij,aj->nai', R, tmpl)
        flat = np.mod(xyz.reshape(-1, 3), box)
        mol = np.repeat(np.arange(n), 3)
        is_h = np.tile([False, True, True], n)
        tree = cKDTree(flat, boxsize=box)
        pairs = tree.query_pairs(1.75, output_type='ndarray')
        bad = set()
        if len(pairs):
            p = pairs[mol[pairs[:, 0]] != mol[pairs[:, 1]]]
            p = p[is_h[p[:, 0]] | is_h[p[:, 1]]]
            for a, b in p:
                bad.add(int(mol[b]) if is_h[b] else int(mol[a]))
        if fixed_pts is not None and len(fixed_pts):
            ft = cKDTree(np.mod(fixed_pts, box), boxsize=box)
            hits = ft.query_ball_point(flat[is_h], 1.9)
            hmol = mol[is_h]
            for k, h in enumerate(hits):
                if h:
                    bad.add(int(hmol[k]))
        if not bad:
            break
        idx = np.array(sorted(bad))
        R[idx] = _random_rotations(rng, len(idx))
    return centers[:, None, :] + np.einsum('nij,aj->nai', R, tmpl)


def _self_avoiding_walk(rng, n, start, box, obstacles=None, d_obs=2.2, d_nb=2.5,
                        d_13=2.2, step=BOND_R0, center_pull=None, max_tries=400):
    """Chain of ``n`` atoms with ``step``-long bonds; non-bonded atoms at least
    ``d_nb`` apart, 1-3 atoms at least ``d_13`` apart, every atom at least
    ``d_obs`` from the obstacle points (periodic)."""
    otree = cKDTree(np.mod(obstacles, box), boxsize=box) if obstacles is not None and len(obstacles) else None
    pts = [np.asarray(start, float)]
    backtracks = 0
    while len(pts) < n:
        placed = False
        for _ in range(max_tries):
            v = rng.normal(size=3)
            v /= np.linalg.norm(v)
            if center_pull is not None:
                v = v + center_pull(pts[-1])
                v /= np.linalg.norm(v)
            p = pts[-1] + step * v
            P = np.array(pts)
            d = P - p
            d -= box * np.rint(d / box)
            r = np.sqrt((d * d).sum(1))
            k = len(pts)
            if k >= 2 and r[k - 2] < d_13:
                continue
            if k >= 3 and np.any(r[: k - 2] < d_nb):
                continue
            if otree is not None and otree.query_ball_point(np.mod(p, box), d_obs):
                continue
            pts.append(p)
            placed = True
            break
        if not placed:
            backtracks += 1
            if backtracks > 200 or len(pts) < 3:
                raise RuntimeError("self-avoiding walk got stuck")
            del pts[-2:]
    return np.array(pts)


def _chain_topology(first, n):
    """Bonds (i, i+1) and 1-2 / 1-3 exclusions of a linear chain starting at ``first``."""
    idx = np.arange(first, first + n)
    bonds = np.stack([idx[:-1], idx[1:]], 1)
    excl = [bonds, np.stack([idx[:-2], idx[2:]], 1)]
    return bonds, np.concatenate(excl)


def ewald_alpha(r_cut, tol):
    """Ewald splitting parameter from the direct-space tolerance
    erfc(alpha r_c) ~ 2 tol (OpenMM's documented convention)."""
    return math.sqrt(-math.log(2.0 * tol)) / r_cut


def pme_grid_for(box, spacing=0.92):
    """Smallest 2^a 3^b 5^c grid dimension with spacing <= ``spacing`` A."""
    out = []
    for L in box:
        k = int(math.ceil(L / spacing))
        while True:
            m = k
            for p in (2, 3, 5):
                while m % p == 0:
                    m //= p
            if m == 1:
                break
            k += 1
        out.append(k)
    return tuple(out)


# ---------------------------------------------------------------------------
# lambda schedules (stages joined with the shared boundary state counted once)

def schedule(kind: str) -> np.ndarray:
    """Rows (lambda_elec, lambda_vdw, lambda_restraint), coupled -> decoupled.

    ``cfg0``: 4 electrostatic windows then 8 vdW windows; ``cfg1``: 8 + 12;
    ``cfg2``: 12 restraint, 10 electrostatic, 20 vdW.  Solvent legs carry no
    restraint (its column is 0).  ``paper_solvent`` / ``paper_complex`` use the
    universal factor lists of appendix B (73 and 80 windows).
    """
    rows = []
    if kind == 'cfg0':
        rows += [(1 - i / 4, 1.0, 0.0) for i in range(4)]
        rows += [(0.0, 1 - j / 7, 0.0) for j in range(8)]
    elif kind == 'cfg1':
        rows += [(1 - i / 8, 1.0, 0.0) for i in range(8)]
        rows += [(0.0, 1 - j / 11, 0.0) for j in range(12)]
    elif kind == 'cfg2':
        rows += [(1.0, 1.0, i / 12) for i in range(12)]
        rows += [(1 - i / 10, 1.0, 1.0) for i in range(10)]
        rows += [(0.0, 1 - j / 19, 1.0) for j in range(20)]
    elif kind in ('paper_solvent', 'paper_complex'):
        elec = [0.00, 0.05, 0.10, 0.15, 0.20, 0.25, 0.30, 0.35, 0.40, 0.44, 0.48, 0.52, 0.56, 0.60,
                0.64, 0.68, 0.72, 0.76, 0.80, 0.82, 0.84, 0.86, 0.88, 0.90, 0.92, 0.94, 0.96, 0.98, 1.00]
        vdw = [0.000, 0.040, 0.080, 0.115, 0.150, 0.180, 0.210, 0.240, 0.270, 0.300, 0.330, 0.360,
               0.390, 0.420, 0.450, 0.480, 0.510, 0.540, 0.568, 0.596, 0.624, 0.650, 0.676, 0.702,
               0.728, 0.752, 0.776, 0.798, 0.820, 0.840, 0.860, 0.878, 0.894, 0.908, 0.921, 0.933,
               0.945, 0.956, 0.966, 0.975, 0.983, 0.990, 0.996, 0.999, 1.000]
        rest = [0.00, 0.01, 0.03, 0.10, 0.30, 0.50, 0.75, 1.00]
        r = 1.0 if kind == 'paper_complex' else 0.0
        if kind == 'paper_complex':
            rows += [(1.0, 1.0, x) for x in rest[:-1]]
        rows += [(x, 1.0, r) for x in reversed(elec)]
        rows += [(0.0, x, r) for x in reversed(vdw[:-1])]
    else:
        raise ValueError(kind)
    return np.array(rows, np.float64)


# ---------------------------------------------------------------------------
# assembly

class _Builder:
    def __init__(self):
        self.pos, self.q, self.sig, self.eps, self.m, self.lig = [], [], [], [], [], []
        self.bonds, self.excl, self.waters = [], [], []
        self.extra = []            # (i, j, r0): bonds with their own rest length
        self.n = 0

    def add(self, xyz, q, sig, eps, m, lig):
        k = len(xyz)
        self.pos.append(np.asarray(xyz, float)); self.q.append(np.broadcast_to(q, k))
        self.sig.append(np.broadcast_to(sig, k)); self.eps.append(np.broadcast_to(eps, k))
        self.m.append(np.broadcast_to(m, k)); self.lig.append(np.broadcast_to(lig, k))
        first = self.n
        self.n += k
        return first

    def add_chain(self, xyz, q, sig, eps, lig):
        first = self.add(xyz, q, sig, eps, M_HEAVY, lig)
        b, e = _chain_topology(first, len(xyz))
        self.bonds.append(b); self.excl.append(e)
        return first

    def add_bond(self, i, j, r0):
        self.extra.append((int(i), int(j), float(r0)))

    def add_waters(self, wxyz):
        for w in wxyz:
            o = self.add(w, [Q_OW, Q_HW, Q_HW], [SIG_OW, 1.0, 1.0], [EPS_OW, 0.0, 0.0],
                         [M_O, M_H, M_H], 0)
            self.waters.append([o, o + 1, o + 2])
            self.excl.append(np.array([[o, o + 1], [o, o + 2], [o + 1, o + 2]]))

    def finish(self, name, box, lambdas, r_cut, skin, tol, grid, restraint=None):
        pos = np.concatenate(self.pos)
        q = np.concatenate(self.q).astype(np.float32)
        sig = np.concatenate(self.sig).astype(np.float32)
        eps = np.concatenate(self.eps).astype(np.float32)
        m = np.concatenate(self.m).astype(np.float32)
        lig = np.concatenate(self.lig).astype(np.uint8)
        bonds = (np.concatenate(self.bonds) if self.bonds else np.zeros((0, 2))).astype(np.int32)
        r0 = np.full(len(bonds), BOND_R0, np.float32)
        if self.extra:
            bonds = np.concatenate([bonds, np.array([[i, j] for i, j, _ in self.extra], np.int32)])
            r0 = np.concatenate([r0, np.array([v for _, _, v in self.extra], np.float32)])
        excl = np.concatenate(self.excl).astype(np.int32)
        excl = np.sort(excl, axis=1)
        excl = np.unique(excl, axis=0)
        waters = np.array(self.waters, np.int32).reshape(-1, 3)
        nb = len(bonds)
        sysd = System(name=name, box=np.asarray(box, np.float64), pos=pos.astype(np.float32),
                      charge=q, sigma=sig, epsilon=eps, mass=m, is_ligand=lig, bonds=bonds,
                      bond_k=np.full(nb, BOND_K, np.float32), bond_r0=r0,
                      waters=waters, excl=excl, lambdas=lambdas, r_cut=r_cut, skin=skin,
                      ewald_alpha=ewald_alpha(r_cut, tol), grid=tuple(int(g) for g in grid))
        if restraint is not None:
            sysd.restraint_atoms = np.asarray(restraint[0], np.int32)
            sysd.restraint_g0 = np.asarray(restraint[1], np.float64)
            sysd.restraint_k = np.asarray(restraint[2], np.float64)
        return sysd


def _ligand_params(rng, n, q_sd=0.3):
    q = rng.normal(0.0, q_sd, n)
    q -= q.mean()
    return q, rng.uniform(3.0, 4.0, n), rng.uniform(0.05, 0.2, n)


def _lattice(nside, spacing):
    g = (np.arange(nside) + 0.5) * spacing
    return np.stack(np.meshgrid(g, g, g, indexing='ij'), -1).reshape(-1, 3)


def solvent_leg(config=1, seed=BASE_SEED, n_waters=2500, lattice_n=14, box_edge=42.0,
                n_lig=40, r_cut=10.0, grid=(48, 48, 48), skin=1.0, sched='cfg1',
                keep_all_sites=False):
    """Ligand-solvent leg: ``n_lig``-atom ligand chain plus lattice water."""
    box = np.array([box_edge] * 3)
    spacing = box_edge / lattice_n
    sites = _lattice(lattice_n, spacing)
    rng_l = _rng(config, 1, seed)
    center = box / 2 + rng_l.uniform(-0.3, 0.3, 3)
    obstacles = sites if keep_all_sites else None
    lig_xyz = _self_avoiding_walk(rng_l, n_lig, center, box, obstacles=obstacles, d_obs=2.1)
    if keep_all_sites:
        keep = np.arange(len(sites))
    else:
        t = cKDTree(np.mod(lig_xyz, box), boxsize=box)
        clash = np.array([bool(t.query_ball_point(s, 3.0)) for s in sites])
        free = np.where(~clash)[0]
        rng_s = _rng(config, 2, seed)
        if len(free) < n_waters:
            raise RuntimeError("not enough lattice sites")
        keep = np.sort(rng_s.choice(free, n_waters, replace=False))
    wxyz = _orient_waters(_rng(config, 3, seed), sites[keep], box, fixed_pts=lig_xyz)
    q, s, e = _ligand_params(_rng(config, 4, seed), n_lig)
    b = _Builder()
    b.add_chain(lig_xyz, q, s, e, 1)
    b.add_waters(wxyz)
    sysd = b.finish(f'solvent{config}', box, schedule(sched), r_cut, skin, 5e-4, grid)
    return sysd


def config0(seed=BASE_SEED):
    """216 waters on a 6x6x6 lattice (18.6 A box) plus a 20-atom ligand;
    cutoff 9 A, PME grid 20^3, 12 windows."""
    return solvent_leg(config=0, seed=seed, n_waters=216, lattice_n=6, box_edge=18.6, n_lig=20,
                       r_cut=9.0, grid=(20, 20, 20), skin=0.25, sched='cfg0', keep_all_sites=True)


def ligand_torsions(sysd, seed=BASE_SEED, config=50):
    """Give the ligand chain of ``sysd`` rotatable torsions: every consecutive
    quadruple a-b-c-d of the chain (rotatable bond b-c), with seeded
    k ~ U[0.5, 3] kcal/mol, periodicity n ~ {1, 2, 3} and phase {0, pi}
    (synthetic stand-ins for a force field's terms on rotatable bonds)."""
    lig = np.where(sysd.is_ligand.astype(bool))[0]
    quads = np.array([lig[i:i + 4] for i in range(len(lig) - 3)], np.int32).reshape(-1, 4)
    rng = _rng(config, 7, seed)
    t = len(quads)
    return dataclasses.replace(sysd, torsions=quads, torsion_k=rng.uniform(0.5, 3.0, t).astype(np.float32),
                               torsion_n=rng.integers(1, 4, t).astype(np.int32),
                               torsion_phase=(np.pi * rng.integers(0, 2, t)).astype(np.float32))


def torsion_leg(seed=BASE_SEED):
    """The 12-window small solvent leg (216 waters, 20-atom ligand) whose
    ligand carries 17 rotatable torsions scaled with lambda_vdw."""
    return ligand_torsions(config0(seed), seed)


AW_MAX_POS, AW_MAX_NEG = 0.6, 0.4      # largest charge one alchemical water takes up (e)


def alchemical_water_count(q_ligand):
    """Fewest alchemical waters that take up a ligand net charge q_ligand with
    every water's offset within [-0.4, +0.6] e (the count is the same in every
    window: the decoupled window needs the whole charge)."""
    if abs(q_ligand) < 1e-12:
        return 0
    cap = AW_MAX_POS if q_ligand > 0 else AW_MAX_NEG
    return int(math.ceil(abs(q_ligand) / cap - 1e-9))


def charged_leg(seed=BASE_SEED, q_ligand=1.0, config=51):
    """The small solvent leg (18.6 A box, 20-atom ligand, cutoff 9 A, PME 20^3,
    12 windows) with a charged ligand: ligand charges N(0, 0.3) shifted to a
    net q_ligand, the lattice waters farthest from the ligand replaced by
    counter-ions (one per unit charge: the coupled state is neutral for an
    integer q_ligand), rotatable ligand torsions, and
    the alchemical waters that keep every window neutral -- the waters whose
    oxygens lie farthest from the ligand's centre."""
    box = np.array([18.6] * 3)
    sites = _lattice(6, 3.1)
    rng_l = _rng(config, 1, seed)
    center = box / 2 + rng_l.uniform(-0.3, 0.3, 3)
    lig_xyz = _self_avoiding_walk(rng_l, 20, center, box, obstacles=sites, d_obs=2.1)
    q, sg, ep = _ligand_params(_rng(config, 4, seed), 20)
    q = q + q_ligand / 20.0
    c = lig_xyz.mean(0)
    dist = np.linalg.norm((sites - c) - box * np.round((sites - c) / box), axis=1)
    order = np.argsort(-dist, kind='stable')            # farthest first
    n_ion = int(round(abs(q_ligand)))                    # one counter-ion per unit of ligand charge
    ion_sites = set(int(k) for k in order[:n_ion])
    n_aw = alchemical_water_count(q_ligand)
    wsites = np.array([k for k in range(len(sites)) if k not in ion_sites])
    wxyz = _orient_waters(_rng(config, 3, seed), sites[wsites], box, fixed_pts=lig_xyz)
    b = _Builder()
    b.add_chain(lig_xyz, q, sg, ep, 1)
    ion = ION_CL if q_ligand > 0 else ION_NA
    for k in order[:n_ion]:
        b.add(sites[k][None], ion['q'], ion['sigma'], ion['eps'], ion['mass'], 0)
    b.add_waters(wxyz)
    sysd = b.finish(f'charged{config}', box, schedule('cfg0'), 9.0, 0.25, 5e-4, (20, 20, 20))
    # alchemical waters: the next-farthest sites, as waters
    aw_sites = [int(k) for k in order[n_ion:]][:n_aw]
    off = np.zeros(sysd.n_atoms, np.float32)
    for k in aw_sites:
        w = int(np.where(wsites == k)[0][0])
        off[sysd.waters[w, 0]] = q_ligand / n_aw
    return ligand_torsions(dataclasses.replace(sysd, alch_offset=off), seed, config)


def config1(seed=BASE_SEED):
    """2,500 waters (14^3 lattice, 42 A box) plus a 40-atom ligand; cutoff 10 A,
    PME grid 48^3, 20 windows."""
    return solvent_leg(config=1, seed=seed)


def _raster_protein(rng, n_atoms, row_dy=2.9, amp=0.4, step=BOND_R0):
    """Bonded chain of ``n_atoms`` packed in the smallest sphere that holds it:
    zig-zag rows along x (bond angle ~116 deg) on a square row lattice, rows
    joined boustrophedon-style.  Each row starts in the column where the
    previous one ended, and the bridge between them is a zig-zag of exact bond
    length bulging outward along x, so no bridge folds back into a row."""
    dx = math.sqrt(step * step - (2 * amp) ** 2)
    R = (n_atoms * dx * row_dy * row_dy * 3 / (4 * math.pi)) ** (1 / 3)
    while True:
        pts = []
        nrow = 0
        last_j = None
        zs = np.arange(-R, R + 1e-9, row_dy)
        zs = zs - zs.mean()
        for iz, z in enumerate(zs):
            ys = np.arange(-R, R + 1e-9, row_dy); ys = ys - ys.mean()
            if iz % 2:
                ys = ys[::-1]
            for y in ys:
                rr = R * R - y * y - z * z
                if rr <= 0:
                    continue
                X = math.sqrt(rr)
                jlo, jhi = math.ceil(-X / dx), math.floor(X / dx)
                if jlo > jhi:
                    continue
                forward = nrow % 2 == 0
                if last_j is not None:
                    if forward:
                        jlo, jhi = last_j, max(jhi, last_j)
                    else:
                        jlo, jhi = min(jlo, last_j), last_j
                js = list(range(jlo, jhi + 1)) if forward else list(range(jhi, jlo - 1, -1))
                row = [(j * dx, y + (amp if j % 2 == 0 else -amp), z) for j in js]
                if pts:
                    a = np.array(pts[-1]); bpt = np.array(row[0])
                    D = np.linalg.norm(bpt - a)
                    nseg = max(2, int(math.ceil(D / step)))
                    if nseg % 2:
                        nseg += 1
                    u = (bpt - a) / D
                    out = np.array([-1.0 if forward else 1.0, 0.0, 0.0])
                    out = out - u * (out @ u)
                    if np.linalg.norm(out) < 1e-6:
                        out = np.cross(u, [0.0, 0.0, 1.0])
                    out /= np.linalg.norm(out)
                    h = math.sqrt(max(step * step - (D / nseg) ** 2, 0.0))
                    for k in range(1, nseg):
                        pts.append(tuple(a + u * (D * k / nseg) + (out * h if k % 2 else 0)))
                pts += row
                last_j = js[-1]
                nrow += 1
                if len(pts) >= n_atoms:
                    break
            if len(pts) >= n_atoms:
                break
        if len(pts) >= n_atoms:
            break
        R *= 1.03
    P = np.array(pts[:n_atoms]) + rng.normal(0, 0.05, (n_atoms, 3))
    return _untangle_chain(P, step), R


def _untangle_chain(P, step, d_min=2.5, iters=400):
    """Push apart non-bonded chain atoms (|i-j| >= 3) closer than ``d_min``
    and re-project bond lengths to ``step`` (a purely geometric clean-up)."""
    P = P.copy()
    n = len(P)
    for _ in range(iters):
        pairs = cKDTree(P).query_pairs(d_min, output_type='ndarray')
        if len(pairs):
            pairs = pairs[np.abs(pairs[:, 0] - pairs[:, 1]) >= 3]
        if len(pairs) == 0:
            break
        d = P[pairs[:, 1]] - P[pairs[:, 0]]
        r = np.linalg.norm(d, axis=1, keepdims=True)
        push = 0.5 * (d_min - r) * d / np.maximum(r, 1e-9)
        disp = np.zeros_like(P)
        np.add.at(disp, pairs[:, 0], -push)
        np.add.at(disp, pairs[:, 1], push)
        P += 0.5 * disp
        for _ in range(4):
            for par in (0, 1):
                i = np.arange(par, n - 1, 2)
                b = P[i + 1] - P[i]
                rb = np.linalg.norm(b, axis=1, keepdims=True)
                corr = 0.5 * (rb - step) * b / rb
                P[i] += corr
                P[i + 1] -= corr
    return P


def _angle(a, b, c):
    u, v = a - b, c - b
    return math.acos(np.clip(u @ v / (np.linalg.norm(u) * np.linalg.norm(v)), -1, 1))


def _dihedral(a, b, c, d):
    b1, b2, b3 = b - a, c - b, d - c
    n1, n2 = np.cross(b1, b2), np.cross(b2, b3)
    return math.atan2(np.linalg.norm(b2) * (b1 @ n2), n1 @ n2)


def _choose_anchors(P, L):
    """Synthetic Boresch anchor rule: L1 = ligand atom nearest the protein,
    L2/L3 its chain neighbours, P1 among the 20 protein atoms nearest L1,
    P2/P3 its chain neighbours; angles P1-L1-L2 and L1-P1-P2 within
    45-135 deg, triples' own angles within 30-150 deg, preferring both
    angles near 90 deg, ties broken by atom index.  When no set around the
    nearest ligand atom satisfies the angles, the next-nearest ligand atoms
    (up to the fifth) are tried as L1 in turn."""
    dPL = np.linalg.norm(P[:, None] - L[None], axis=2)
    nl = len(L)
    for l1 in np.argsort(dPL.min(0), kind='stable')[:5]:
        l1 = int(l1)
        ldirs = [(l1 + 1, l1 + 2), (l1 - 1, l1 - 2)]
        best = None
        near = np.argsort(dPL[:, l1], kind='stable')[:20]
        for p1 in near:
            for l2, l3 in ldirs:
                if not (0 <= l3 < nl and 0 <= l2 < nl):
                    continue
                for p2, p3 in ((p1 + 1, p1 + 2), (p1 - 1, p1 - 2)):
                    if not (0 <= p3 < len(P) and 0 <= p2 < len(P)):
                        continue
                    ta = math.degrees(_angle(P[p1], L[l1], L[l2]))
                    tb = math.degrees(_angle(L[l1], P[p1], P[p2]))
                    if not (45 <= ta <= 135 and 45 <= tb <= 135):
                        continue
                    if not (30 <= math.degrees(_angle(L[l1], L[l2], L[l3])) <= 150):
                        continue
                    if not (30 <= math.degrees(_angle(P[p1], P[p2], P[p3])) <= 150):
                        continue
                    score = (abs(ta - 90) + abs(tb - 90), int(p1), int(p2), int(l2))
                    if best is None or score < best[0]:
                        best = (score, (int(p1), int(p2), int(p3), l1, l2, l3))
        if best is not None:
            return best[1]
    raise RuntimeError("no anchor set satisfies the angle rule")


def complex_leg(config=2, seed=BASE_SEED, n_prot=5000, n_lig=50, box_edge=88.0, lattice_n=29,
                n_ion_pairs=4, r_cut=10.0, grid=(96, 96, 96), skin=1.0, sched='cfg2',
                k_r=10.0, k_theta=100.0, k_phi=100.0):
    """Protein-ligand leg: chain 'protein' in a sphere, ligand at its surface
    with Boresch anchors, counter-ions and lattice water."""
    box = np.array([box_edge] * 3)
    rng_p = _rng(config, 10, seed)
    Pc, R = _raster_protein(rng_p, n_prot)
    Rm = _random_rotations(rng_p, 1)[0]
    P = Pc @ Rm.T + box / 2
    qp = rng_p.normal(0, 0.4, n_prot)
    qp += (-4.0 - qp.sum()) / n_prot
    sp = rng_p.uniform(2.5, 3.9, n_prot)
    ep = rng_p.uniform(0.05, 0.2, n_prot)
    rng_l = _rng(config, 11, seed)
    d = rng_l.normal(size=3); d /= np.linalg.norm(d)
    start = box / 2 + d * (R + 3.2)
    while cKDTree(P).query(start)[0] < 3.0:
        start = start + d * 0.5
    L = _self_avoiding_walk(rng_l, n_lig, start, box, obstacles=P, d_obs=2.9, center_pull=None)
    ql, sl, el = _ligand_params(_rng(config, 12, seed), n_lig)
    sites = _lattice(lattice_n, box_edge / lattice_n)
    solute = np.concatenate([P, L])
    st = cKDTree(np.mod(solute, box), boxsize=box)
    free = np.array([not st.query_ball_point(s, 3.1) for s in sites])
    sites = sites[free]
    rng_i = _rng(config, 13, seed)
    far = np.array([st.query(s)[0] > 8.0 for s in sites])
    ion_sites = rng_i.choice(np.where(far)[0], 2 * n_ion_pairs, replace=False)
    wmask = np.ones(len(sites), bool); wmask[ion_sites] = False
    wxyz = _orient_waters(_rng(config, 14, seed), sites[wmask], box, fixed_pts=solute)
    p1, p2, p3, l1, l2, l3 = _choose_anchors(P, L)
    g0 = [np.linalg.norm(P[p1] - L[l1]), _angle(P[p1], L[l1], L[l2]), _angle(L[l1], P[p1], P[p2]),
          _dihedral(P[p2], P[p1], L[l1], L[l2]), _dihedral(P[p1], L[l1], L[l2], L[l3]),
          _dihedral(L[l1], P[p1], P[p2], P[p3])]
    b = _Builder()
    pf = b.add_chain(P, qp, sp, ep, 0)
    lf = b.add_chain(L, ql, sl, el, 1)
    for k, s in enumerate(ion_sites):
        ion = ION_NA if k < n_ion_pairs else ION_CL
        b.add(sites[s][None], ion['q'], ion['sigma'], ion['eps'], ion['mass'], 0)
    b.add_waters(wxyz)
    anchors = [pf + p1, pf + p2, pf + p3, lf + l1, lf + l2, lf + l3]
    # The chains carry no angle terms, so the anchor triples' own angles
    # (which enter the Boresch dihedrals and make them singular at 180 deg)
    # are held near their initial values by a 1-3 bond each, as a force
    # field's angle terms would.  Both pairs are already 1-3 exclusions.
    b.add_bond(pf + p1, pf + p3, np.linalg.norm(P[p1] - P[p3]))
    b.add_bond(lf + l1, lf + l3, np.linalg.norm(L[l1] - L[l3]))
    ks = [k_r, k_theta, k_theta, k_phi, k_phi, k_phi]
    sysd = b.finish(f'complex{config}', box, schedule(sched), r_cut, skin, 5e-4, grid,
                    restraint=(anchors, g0, ks))
    return sysd


def config2(seed=BASE_SEED):
    """~68k-atom complex leg: 5,000-atom chain protein, 50-atom ligand with a
    Boresch restraint, 4 Na+/Cl- pairs, lattice water in an 88 A box; 42 windows."""
    return complex_leg(config=2, seed=seed)


def small_complex(seed=BASE_SEED):
    """A reduced complex leg (same recipe as ``config2`` at ~1/10 scale) for
    parity tests that the brute-force oracle finishes in seconds."""
    return complex_leg(config=5, seed=seed, n_prot=400, n_lig=16, box_edge=36.0, lattice_n=12,
                       n_ion_pairs=1, grid=(40, 40, 40))


def sized_leg(n_atoms, n_windows, seed):
    """A leg of about ``n_atoms`` atoms for served-batch workloads: ``n_windows``
    of 12 or 20 gives a solvent leg with the cfg0 / cfg1 schedule type, 42 a
    complex leg with the cfg2 schedule type."""
    rho = 0.0334
    if n_windows in (12, 20):
        n_lig = 40
        nw = max(64, (n_atoms - n_lig) // 3)
        L = (nw / rho) ** (1 / 3)
        nside = int(math.ceil((nw * 1.08) ** (1 / 3)))
        return solvent_leg(config=100 + seed % 1000, seed=seed, n_waters=nw, lattice_n=nside,
                           box_edge=L, n_lig=n_lig, r_cut=10.0, grid=pme_grid_for([L] * 3),
                           sched='cfg0' if n_windows == 12 else 'cfg1')
    n_prot = int(round(0.074 * n_atoms))
    L = ((n_atoms - n_prot) / 3 / rho + n_prot * 10.7) ** (1 / 3)
    nside = int(round(L / 3.03))
    return complex_leg(config=100 + seed % 1000, seed=seed, n_prot=n_prot, n_lig=50, box_edge=L,
                       lattice_n=nside, n_ion_pairs=4, grid=pme_grid_for([L] * 3))
