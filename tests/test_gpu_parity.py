"""GPU parity: every C-ABI call against the FP64 oracle on the same seeded inputs.

Tolerances (spec bar): neighbour lists bit-exact; force relative RMS
<= 1e-5 (real-space, reciprocal and total separately); energy relative error
<= 1e-6 of |E| for every component and for the total (energies requested with
FELIS_ENERGY are evaluated term by term in FP64); the integrator is compared
over a short horizon with identical noise, also with the restraint on; u_kn
and MBAR to |ddG| <= 0.01 kcal/mol.
"""
import numpy as np
import pytest
import torch

from oracle import bonded as obonded, energy as oenergy, integrate as ointeg, mbar as ombar, pairs as opairs, ukn as oukn
from oracle.ewald import PME
from paper_2603_22274_amd import gen

pytestmark = pytest.mark.gpu

KB = 0.0019872043


@pytest.fixture(scope='module')
def F():
    if not torch.cuda.is_available():
        pytest.skip('no HIP device')
    from paper_2603_22274_amd import felis
    ctx = felis.Context(0)
    yield felis, ctx
    torch.cuda.synchronize()
    ctx.close()


def rel_rms(a, b):
    return float(np.sqrt(((a - b) ** 2).sum() / (b ** 2).sum()))


def _leg(felis, ctx, s, windows=None, positions=None, seed=7):
    leg = felis.Leg(ctx, s, windows=windows, positions=positions, seed=seed)
    felis.build_nlist(ctx, [leg], force=True)
    ctx.device_check()
    return leg


def _jitter(s, W, amp=0.05, seed=3):
    rng = np.random.default_rng(seed)
    return (s.pos[None].astype(np.float64) + rng.normal(0, amp, (W, s.n_atoms, 3))).astype(np.float32)


@pytest.mark.parametrize('name', ['config0', 'small_complex', 'config1', 'config2'])
def test_nlist_bit_exact(F, name):
    felis, ctx = F
    s = getattr(gen, name)()
    W = 3
    pos = _jitter(s, W)
    leg = _leg(felis, ctx, s, windows=[0, 21, 41] if name == 'config2' else [0, 1, 2], positions=pos)
    for w in range(W):
        got = felis.nlist_export_pairs(ctx, leg, w)
        if s.n_atoms > 20000:               # the canonical list by k-d tree candidates (pinned to brute force)
            ref = opairs.neighbor_pairs_tree(pos[w], s.box, s, s.r_list)
        else:
            ref = opairs.neighbor_pairs(pos[w], s.box, s, s.r_list)
        assert got.shape == ref.shape and np.array_equal(got, ref), (name, w, got.shape, ref.shape)


def _sum_abs_pairs(s, pos, lam):
    """sum over pairs of |E_coul| and |E_lj| (normaliser for cancelling sums)."""
    x = np.asarray(pos, np.float64)
    p = opairs.neighbor_pairs(pos, s.box, s, s.r_cut)
    i, j, ec, elj, _ = opairs._pair_block(x, s.box, s, lam, p[:, 0], p[:, 1])
    return np.abs(ec).sum(), np.abs(elj).sum()


@pytest.mark.parametrize('name,windows', [('config0', list(range(12))), ('small_complex', [0, 12, 16, 25, 35, 41]),
                                          ('config1', [0, 9, 19]), ('small_complex', [20])])
def test_nonbonded_and_pme(F, name, windows):
    felis, ctx = F
    s = getattr(gen, name)()
    leg = _leg(felis, ctx, s, windows=windows)
    felis.nonbonded(ctx, [leg])
    f_real = leg.forces().cpu().numpy()
    felis.pme(ctx, [leg])
    f_all = leg.forces().cpu().numpy()
    f_rec = f_all - f_real
    E = leg.energy.cpu().numpy()
    ctx.device_check()
    pme = PME(s.box, s.grid, s.ewald_alpha)
    x = s.pos.astype(np.float64)
    for k, w in enumerate(windows):
        lam = s.lambdas[w]
        ec, elj, fr = opairs.real_space(x, s, lam)
        ex, fx = opairs.exclusion_correction(x, s, lam)
        es = opairs.self_and_background(s, lam)
        q = opairs.scaled_charges(s, lam[0])
        er, frec = pme.energy_forces(x, q)
        assert abs(E[k, 0] - ec) <= 1e-6 * abs(ec), (w, 'coul', E[k, 0], ec)
        assert abs(E[k, 1] - elj) <= 1e-6 * abs(elj), (w, 'lj', E[k, 1], elj)
        assert abs(E[k, 2] - ex) <= 1e-6 * abs(ex), (w, 'excl', E[k, 2], ex)
        assert abs(E[k, 3] - es) <= 1e-6 * abs(es), (w, 'self', E[k, 3], es)
        assert abs(E[k, 4] - er) <= 1e-6 * abs(er), (w, 'recip', E[k, 4], er)
        assert rel_rms(f_real[k], fr + fx) <= 1e-5, (w, 'real forces', rel_rms(f_real[k], fr + fx))
        assert rel_rms(f_rec[k], frec) <= 1e-5, (w, 'recip forces', rel_rms(f_rec[k], frec))
        assert rel_rms(f_all[k], fr + fx + frec) <= 1e-5, (w, 'forces', rel_rms(f_all[k], fr + fx + frec))


def _sample_atoms(s, k=40, seed=11):
    rng = np.random.default_rng(seed)
    pick = list(np.where(s.is_ligand)[0][:8])
    if s.restraint_atoms is not None:
        pick += [int(a) for a in s.restraint_atoms]
    pick += [int(a) for a in rng.choice(s.n_atoms, k, replace=False)]
    return np.unique(np.array(pick, np.int64))


@pytest.mark.parametrize('name', ['config1', 'config2'])
def test_full_size_launch_sampled_atoms(F, name):
    """Every window of a full-size leg in one launch, as the bench and the
    served batches run them (20-window solvent leg; 42-window, ~70k-atom
    complex leg with a 96^3 grid), each window on its own perturbed
    coordinates: real-space + excluded-pair forces of sampled atoms against
    the oracle's per-atom brute force, reciprocal forces of the same atoms and
    the whole-system reciprocal, excluded-pair and self energies against the
    FP64 PME and closed forms."""
    felis, ctx = F
    s = getattr(gen, name)()
    W = s.n_windows
    pos = _jitter(s, W, amp=0.03, seed=5)
    leg = _leg(felis, ctx, s, positions=pos)
    felis.nonbonded(ctx, [leg])
    f_real = leg.forces().cpu().numpy()
    felis.pme(ctx, [leg])
    f_all = leg.forces().cpu().numpy()
    f_rec = f_all - f_real
    E = leg.energy.cpu().numpy()
    ctx.device_check()
    atoms = _sample_atoms(s)
    pme = PME(s.box, s.grid, s.ewald_alpha)
    windows = range(W) if W <= 20 else [0, 11, 12, 21, 22, 41]
    for w in windows:
        lam = s.lambdas[w]
        x = pos[w].astype(np.float64)
        fo, _ = opairs.real_space_atoms(x, s, lam, atoms)
        ex, fx = opairs.exclusion_correction(x, s, lam)
        es = opairs.self_and_background(s, lam)
        er, frec = pme.energy_forces(x, opairs.scaled_charges(s, lam[0]))
        ref_real = fo + fx[atoms]
        assert rel_rms(f_real[w][atoms], ref_real) <= 1e-5, (w, 'real', rel_rms(f_real[w][atoms], ref_real))
        assert rel_rms(f_rec[w][atoms], frec[atoms]) <= 1e-5, (w, 'recip', rel_rms(f_rec[w][atoms], frec[atoms]))
        assert rel_rms(f_all[w][atoms], ref_real + frec[atoms]) <= 1e-5, (w, 'total')
        assert abs(E[w, 2] - ex) <= 1e-6 * abs(ex), (w, 'excl', E[w, 2], ex)
        assert abs(E[w, 3] - es) <= 1e-6 * abs(es), (w, 'self', E[w, 3], es)
        assert abs(E[w, 4] - er) <= 1e-6 * abs(er), (w, 'recip', E[w, 4], er)


def test_bonded_and_restraint(F):
    felis, ctx = F
    s = gen.small_complex()
    windows = [0, 3, 11, 12, 41]
    pos = _jitter(s, len(windows), amp=0.1)
    leg = _leg(felis, ctx, s, windows=windows, positions=pos)
    leg.fx.zero_(); leg.fy.zero_(); leg.fz.zero_()
    felis.bonded(ctx, [leg])
    f = leg.forces().cpu().numpy()
    E = leg.energy.cpu().numpy()
    for k, w in enumerate(windows):
        x = pos[k].astype(np.float64)
        eb, fb = obonded.bonds(x, s)
        er, fre = obonded.boresch(x, s, s.lambdas[w][2])
        assert abs(E[k, 5] - eb) <= 1e-6 * abs(eb), (w, E[k, 5], eb)
        assert abs(E[k, 6] - er) <= 1e-6 * max(abs(er), 1e-3), (w, E[k, 6], er)
        assert rel_rms(f[k], fb + fre) <= 1e-5, (w, rel_rms(f[k], fb + fre))


def test_total_force_energy_complex(F):
    felis, ctx = F
    s = gen.small_complex()
    windows = [0, 12, 25, 41]
    leg = _leg(felis, ctx, s, windows=windows)
    felis.forces_and_energy(ctx, [leg])
    f = leg.forces().cpu().numpy()
    E = leg.energy.cpu().numpy()
    pme = PME(s.box, s.grid, s.ewald_alpha)
    for k, w in enumerate(windows):
        e, fo = oenergy.window_energy(s, s.pos.astype(np.float64), s.lambdas[w], pme=pme)
        assert rel_rms(f[k], fo) <= 1e-5, (w, rel_rms(f[k], fo))
        comp = {c: E[k, i] - e[c] for i, c in enumerate(oenergy.COMPONENTS)}
        assert abs(E[k, 7] - e['total']) <= 1e-6 * abs(e['total']), (w, comp, e['total'])


def test_deterministic_and_batch_independent(F):
    felis, ctx = F
    s0, s1 = gen.config0(), gen.small_complex()
    a = _leg(felis, ctx, s0, windows=[0, 5, 9])
    b = _leg(felis, ctx, s1, windows=[1, 20])
    felis.forces_and_energy(ctx, [a])
    fa1 = (a.fx.clone(), a.fy.clone(), a.fz.clone(), a.energy.clone())
    felis.forces_and_energy(ctx, [a, b])
    fa2 = (a.fx.clone(), a.fy.clone(), a.fz.clone(), a.energy.clone())
    felis.forces_and_energy(ctx, [b, a])
    fa3 = (a.fx.clone(), a.fy.clone(), a.fz.clone(), a.energy.clone())
    for u, v, t in zip(fa1, fa2, fa3):
        assert torch.equal(u, v) and torch.equal(u, t)


def test_step_matches_oracle_short_horizon(F):
    felis, ctx = F
    s = gen.config0()
    windows = [0, 7]
    leg = _leg(felis, ctx, s, windows=windows, seed=11)
    rng = np.random.default_rng(5)
    v0 = rng.normal(0, 3.0, (len(windows), s.n_atoms, 3)).astype(np.float32)
    # project initial velocities onto the rigid-water constraint by one SHAKE-consistent step:
    leg.vx.copy_(torch.as_tensor(v0[..., 0])); leg.vy.copy_(torch.as_tensor(v0[..., 1])); leg.vz.copy_(torch.as_tensor(v0[..., 2]))
    nsteps = 10
    felis.step(ctx, [leg], nsteps, dt=0.002, temperature=300.0, gamma=0.5)
    ctx.device_check()
    got = leg.positions().cpu().numpy()
    pme = PME(s.box, s.grid, s.ewald_alpha)
    for k, w in enumerate(windows):
        x = s.pos.astype(np.float64)
        v = v0[k].astype(np.float64)
        force = lambda y: oenergy.window_energy(s, y, s.lambdas[w], pme=pme)[1]
        for st in range(nsteps):
            x, v = ointeg.langevin_middle_step(s, x, v, force, 0.002, 300.0, 0.5, 11, k, st)
        err = np.max(np.abs(got[k] - x))
        print('window', w, 'max |dx|', err, 'rms', np.sqrt(np.mean((got[k] - x) ** 2)))
        assert err < 1e-4, (w, err)
        assert np.sqrt(np.mean((got[k] - x) ** 2)) < 2e-5, (w, np.sqrt(np.mean((got[k] - x) ** 2)))


def test_step_matches_oracle_restrained_complex(F):
    """felis_step on the small complex leg at lambda_restraint 0.5 (restraint
    stage) and 1 (vdW stage, lambda_elec 0): bonded and restraint forces are
    summed inside the integrator; 8 steps against the oracle with identical
    noise, from protein/ligand/ion coordinates jittered so the restraint acts
    from the first step."""
    felis, ctx = F
    s = gen.small_complex()
    windows = [6, 30]
    assert s.lambdas[6][2] == 0.5 and s.lambdas[30][2] == 1.0
    rng = np.random.default_rng(8)
    free = np.setdiff1d(np.arange(s.n_atoms), s.waters.ravel())
    pos = np.repeat(s.pos[None].astype(np.float64), len(windows), 0)
    pos[:, free] += rng.normal(0, 0.05, (len(windows), len(free), 3))
    pos = pos.astype(np.float32)
    leg = _leg(felis, ctx, s, windows=windows, positions=pos, seed=19)
    v0 = rng.normal(0, 2.0, (len(windows), s.n_atoms, 3)).astype(np.float32)
    leg.vx.copy_(torch.as_tensor(v0[..., 0])); leg.vy.copy_(torch.as_tensor(v0[..., 1])); leg.vz.copy_(torch.as_tensor(v0[..., 2]))
    nsteps = 8
    felis.step(ctx, [leg], nsteps, dt=0.002, temperature=300.0, gamma=0.5)
    ctx.device_check()
    got = leg.positions().cpu().numpy()
    pme = PME(s.box, s.grid, s.ewald_alpha)
    for k, w in enumerate(windows):
        x = pos[k].astype(np.float64)
        v = v0[k].astype(np.float64)
        force = lambda y: oenergy.window_energy(s, y, s.lambdas[w], pme=pme)[1]
        e0, _ = oenergy.window_energy(s, x, s.lambdas[w], pme=pme)
        assert e0['restraint'] > 1e-3, e0['restraint']
        for st in range(nsteps):
            x, v = ointeg.langevin_middle_step(s, x, v, force, 0.002, 300.0, 0.5, 19, k, st)
        err = np.max(np.abs(got[k] - x))
        anchors = np.asarray(s.restraint_atoms)
        print('window', w, 'max |dx|', err, 'anchors', np.max(np.abs(got[k][anchors] - x[anchors])))
        assert err < 1e-4, (w, err)
        assert np.sqrt(np.mean((got[k] - x) ** 2)) < 2e-5, (w, np.sqrt(np.mean((got[k] - x) ** 2)))


def test_ukn_matches_oracle(F):
    felis, ctx = F
    s = gen.small_complex()
    nf = 6
    frames = _jitter(s, nf, amp=0.08, seed=9)
    leg = _leg(felis, ctx, s, windows=list(range(8)))
    xt = torch.as_tensor(frames[..., 0]).cuda()
    yt = torch.as_tensor(frames[..., 1]).cuda()
    zt = torch.as_tensor(frames[..., 2]).cuda()
    beta = 1.0 / (KB * 300.0)
    u = felis.ukn(ctx, leg, s.lambdas, xt, yt, zt, beta).cpu().numpy()
    ctx.device_check()
    ref = oukn.ukn(s, frames.astype(np.float64), s.lambdas, beta)
    # per-frame differences between states (what MBAR sees) within 1e-6 relative + 2e-4 kT
    du = (u - u[0]) - (ref - ref[0])
    scale = np.abs(ref - ref[0]).max()
    assert np.max(np.abs(du)) <= 1e-6 * scale + 2e-4, (np.max(np.abs(du)), scale)
    assert np.max(np.abs(u - ref)) <= 1e-6 * np.abs(ref).max() + 2e-4


def test_ukn_full_size_complex(F):
    """u_kn of the ~70k-atom complex leg (96^3 grid) at all 42 states for
    perturbed frames, through the leg's 42-window scratch, against the oracle
    frame by frame."""
    felis, ctx = F
    s = gen.config2()
    nf = 4
    frames = _jitter(s, nf, amp=0.05, seed=13)
    leg = _leg(felis, ctx, s)
    xt = torch.as_tensor(frames[..., 0]).cuda()
    yt = torch.as_tensor(frames[..., 1]).cuda()
    zt = torch.as_tensor(frames[..., 2]).cuda()
    beta = 1.0 / (KB * 300.0)
    u = felis.ukn(ctx, leg, s.lambdas, xt, yt, zt, beta).cpu().numpy()
    ctx.device_check()
    ref = oukn.ukn(s, frames.astype(np.float64), s.lambdas, beta)
    du = (u - u[0]) - (ref - ref[0])
    scale = np.abs(ref - ref[0]).max()
    assert np.max(np.abs(du)) <= 1e-6 * scale + 2e-4, (np.max(np.abs(du)), scale)
    assert np.max(np.abs(u - ref)) <= 1e-6 * np.abs(ref).max() + 2e-4


def test_mbar_full_size(F):
    """MBAR at 42 states x 84,000 samples (2,000 per state): harmonic states
    whose exact free energies are known; GPU against the oracle's fixed point."""
    felis, ctx = F
    rng = np.random.default_rng(17)
    K, n = 42, 2000
    ks = np.exp(np.linspace(0.0, np.log(3.0), K))
    x2 = np.concatenate([(rng.normal(0, 1 / np.sqrt(k), (n, 3)) ** 2).sum(1) for k in ks])
    u = 0.5 * ks[:, None] * x2[None, :]
    N = np.full(K, n)
    f_ref, _ = ombar.mbar(u, N, tol=1e-13)
    f, it = felis.mbar(ctx, torch.as_tensor(u).cuda(), N, tol=1e-12)
    assert np.max(np.abs(f - f_ref)) < 1e-8, np.max(np.abs(f - f_ref))
    assert abs((f[-1] - f[0]) - 1.5 * np.log(ks[-1] / ks[0])) < 0.02        # sampling error only


def test_mbar_matches_oracle(F):
    felis, ctx = F
    rng = np.random.default_rng(2)
    ks = np.array([1.0, 1.3, 1.7, 2.2, 2.9, 3.8])
    n = 2000
    x2 = np.concatenate([(rng.normal(0, 1 / np.sqrt(k), (n, 3)) ** 2).sum(1) for k in ks])
    u = 0.5 * ks[:, None] * x2[None, :]
    N = np.full(len(ks), n)
    f_ref, _ = ombar.mbar(u, N, tol=1e-12)
    f, it = felis.mbar(ctx, torch.as_tensor(u).cuda(), N, tol=1e-12)
    assert np.max(np.abs(f - f_ref)) < 1e-9, (f, f_ref)


def test_mbar_unsampled_states_and_column_order(F):
    """States with no samples get their f from the converged denominators;
    the result does not depend on the order of the sample columns; widely
    spaced states (slow for plain fixed-point iteration) converge in a few
    Newton steps."""
    felis, ctx = F
    rng = np.random.default_rng(5)
    ks = np.array([1.0, 1.6, 2.6, 4.2, 6.8, 11.0])
    n = 800
    N = np.array([n, 0, n, 0, n, n])
    x2 = np.concatenate([(rng.normal(0, 1 / np.sqrt(k), (c, 3)) ** 2).sum(1) for k, c in zip(ks, N) if c])
    u = 0.5 * ks[:, None] * x2[None, :]
    f_ref, it_ref = ombar.mbar(u, N, tol=1e-14)
    f, it = felis.mbar(ctx, torch.as_tensor(u).cuda(), N, tol=1e-12)
    assert np.max(np.abs(f - f_ref)) < 1e-9, (f, f_ref)
    assert it <= 30 < it_ref
    perm = rng.permutation(u.shape[1])
    f2, _ = felis.mbar(ctx, torch.as_tensor(np.ascontiguousarray(u[:, perm])).cuda(), N, tol=1e-12)
    assert np.max(np.abs(f2 - f)) < 1e-9


def test_ddg_from_gpu_frames(F):
    """Short sampled leg: GPU dynamics -> frames; Delta G from GPU u_kn + GPU
    MBAR equals the oracle's u_kn + MBAR on the same frames."""
    felis, ctx = F
    s = gen.config0()
    # a closely spaced segment of the path (the paper runs windows in short
    # overlapping segments), so every neighbouring pair of states overlaps
    s.lambdas = np.array([(1.0 - 0.03 * k, 1.0, 0.0) for k in range(6)] +
                         [(0.85, 1.0 - 0.02 * k, 0.0) for k in range(1, 7)])
    leg = _leg(felis, ctx, s, seed=21)
    beta = 1.0 / (KB * 300.0)
    frames = []
    felis.step(ctx, [leg], 300, temperature=300.0, gamma=5.0)
    for it in range(16):
        felis.step(ctx, [leg], 10, temperature=300.0, gamma=5.0)
        frames.append(leg.positions().clone())
    ctx.device_check()
    fr = torch.stack(frames, 1)             # (W, n_per, N, 3)
    W, npw = fr.shape[0], fr.shape[1]
    flat = fr.reshape(W * npw, s.n_atoms, 3)
    u = felis.ukn(ctx, leg, s.lambdas, flat[..., 0].contiguous(), flat[..., 1].contiguous(),
                  flat[..., 2].contiguous(), beta)
    N = np.full(W, npw)
    f_gpu, it_gpu = felis.mbar(ctx, u, N, tol=1e-8, max_iter=400000)
    ref_u = oukn.ukn(s, flat.cpu().numpy().astype(np.float64), s.lambdas, beta)
    f_ref, it_ref = ombar.mbar(ref_u, N, tol=1e-8, max_iter=400000)
    print('mbar iterations gpu/oracle', it_gpu, it_ref, 'max |du|', float(np.abs(u.cpu().numpy() - ref_u).max()))
    dg_gpu = (f_gpu[-1] - f_gpu[0]) / beta
    dg_ref = (f_ref[-1] - f_ref[0]) / beta
    assert abs(dg_gpu - dg_ref) <= 0.01, (dg_gpu, dg_ref)
