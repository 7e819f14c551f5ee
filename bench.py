"""Throughput of the alchemical-window hot path on one MI355X.

Headline workload: the 42-window complex leg (a 5,000-atom chain protein, a
50-atom ligand held by a Boresch restraint, 4 Na+/4 Cl- and 21,823 waters in
an 88 A box: 70,527 atoms; cutoff 10 A, skin 1 A, PME 96^3 order 4; 12
restraint, 10 electrostatic and 20 vdW windows), every window batched in
every launch.  The smaller 20-window solvent leg is available with
``--workload solvent20``.

One bench step = one pass of the whole hot path over the batch: ``--md``
Langevin-middle steps of 2 fs for every window (list check/rebuild, real-space
pair kernel, PME, bonded and restraint terms, integrator with SETTLE), then
the reduced potentials u_kn of every window's current frame at all states.
After the timed steps MBAR solves the collected u_kn (inside the timed
region).

The throughput counts only if the run's free energy is right: after the timed
region, the frames that a segment of neighbouring windows produced are handed
to the FP64 oracle (its own u_kn and MBAR, on the host cores), and |ddG|
between the GPU's segment Delta G (GPU u_kn + GPU MBAR on the same frames) and
the oracle's must be <= 0.01 kcal/mol, else ``value`` is reported as 0.

Prints one JSON line: aggregate ns.windows/day, the pair kernel's roofline
(FP32 ALU bound; algorithmic flops = unique in-cutoff pairs x 60; duration
from HIP events recorded around the kernel inside the timed region), the FP64
oracle timed on the host as the CPU baseline, the plain per-window form of
the same leg, and a served stream of uneven legs with its p50/p99 latency.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "aggregate ns·windows/day at |ΔΔG|≤0.01 kcal/mol; p50/p99 leg latency"
KB = 0.0019872043
DT = 0.002                      # ps
PEAK_FP32 = 157.3               # TFLOP/s, MI355X FP32 vector (published; counts packed FP32)
ISSUE_FP32 = 78.6               # TFLOP/s, non-packed FP32 issue: 256 CU x 4 SIMD x 16 lanes x 2 x 2.4 GHz
FLOP_PER_PAIR = 60              # FP32 flops per unique in-cutoff pair (FMA = 2)
PAIR_BYTES_PER_ATOM = 48        # algorithmic HBM bytes per atom-window of one pair launch: coordinates +
                                # charge (16) and LJ parameters with the ligand flag (8) read, 3 int64 forces written
PAIR_SAMPLE = 5                 # the timed region brackets every 5th pair-kernel launch with HIP events
DDG_TOL = 0.01                  # kcal/mol
TRAFFIC_FILES = {'complex42': os.path.join(ROOT, 'profiles', 'pairs_traffic_complex42.json'),
                 'solvent20': os.path.join(ROOT, 'profiles', 'pairs_traffic_solvent20.json')}


def _workers():
    """Host worker processes for the oracle: the machine's CPU share (at most 15
    besides this process)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, 'sched_getaffinity') else (os.cpu_count() or 1)
    return max(1, min(15, n - 1))


def _traffic(workload):
    try:
        t = json.load(open(TRAFFIC_FILES[workload]))
    except (OSError, ValueError, KeyError):
        return None
    from paper_2603_22274_amd.profiling import src_digest
    if t.get('kernel_digest') != src_digest():
        return None
    return t.get('bytes_per_launch')


# ---- host workers (spawned processes; they import numpy, scipy and the oracle only)

_W = {}


def _init_worker(sysd):
    os.environ['OMP_NUM_THREADS'] = '1'
    from threadpoolctl import threadpool_limits
    from oracle.ewald import PME
    _W['limit'] = threadpool_limits(limits=1)
    _W['sys'] = sysd
    _W['pme'] = PME(sysd.box, sysd.grid, sysd.ewald_alpha)


def _ukn_task(args):
    pos, lambdas, beta = args
    from oracle import ukn as oukn
    return oukn.ukn_frame(_W['sys'], pos.astype(np.float64), lambdas, beta, _W['pme'])


def _rsa_task(args):
    pos, lam, atoms = args
    from oracle import pairs as opairs
    t0 = time.perf_counter()
    opairs.real_space_atoms(pos.astype(np.float64), _W['sys'], lam, atoms)
    return time.perf_counter() - t0


def _gen_task(spec):
    from paper_2603_22274_amd import gen
    n, w, seed = spec
    return gen.sized_leg(n, w, seed)


def _pool(sysd, n):
    return mp.get_context('spawn').Pool(n, initializer=_init_worker, initargs=(sysd,))


def ddg_check(sysd, frames, states, seg, u_gpu, beta, ctx, felis, nproc):
    """|ddG| of the segment ``seg`` (consecutive window indices) between
    GPU u_kn + GPU MBAR and oracle u_kn + oracle MBAR on the same frames.
    frames: (n, N, 3) float32 host array; states: the state each frame was
    sampled in; u_gpu: (K_all, n) device tensor of the frames' GPU u_kn."""
    import torch
    from oracle import mbar as ombar
    lam = sysd.lambdas[seg]
    t0 = time.perf_counter()
    with _pool(sysd, nproc) as p:
        ref = np.stack(p.map(_ukn_task, [(f, lam, beta) for f in frames], chunksize=1), 1)
    t_or = time.perf_counter() - t0
    N_k = np.array([(states == s).sum() for s in seg])
    ug = u_gpu[seg].contiguous()
    f_gpu, it_gpu = felis.mbar(ctx, ug, N_k, tol=1e-12, max_iter=20000)
    f_ref, it_ref = ombar.mbar(ref, N_k, tol=1e-12, max_iter=2000000)
    dg_gpu = felis.delta_g(f_gpu, 300.0)
    dg_ref = float((f_ref[-1] - f_ref[0]) / beta)
    du = (ug.cpu().numpy() - ug.cpu().numpy()[0]) - (ref - ref[0])
    return {"segment_windows": [int(s) for s in seg], "frames": int(len(frames)),
            "lambdas": [[float(v) for v in r] for r in lam],
            "dG_gpu_kcal_per_mol": dg_gpu, "dG_oracle_kcal_per_mol": dg_ref, "abs_ddG": abs(dg_gpu - dg_ref),
            "tolerance": DDG_TOL, "passed": bool(abs(dg_gpu - dg_ref) <= DDG_TOL),
            "max_abs_du_kT": float(np.abs(du).max()), "mbar_iterations_gpu_oracle": [int(it_gpu), int(it_ref)],
            "oracle_s": round(t_or, 1), "oracle_processes": nproc}


def cpu_baseline(sysd, lam_index, nproc, n_atoms_sample):
    """One window-step of the FP64 oracle on the host cores, as a bounded
    sample: real-space forces of ``n_atoms_sample`` atoms by the oracle's
    per-atom brute force spread over worker processes, scaled to every atom,
    plus (in this process) one FP64 PME, the exclusion, bonded and restraint
    terms and one Langevin-middle step with SHAKE; scaled to ns.windows/day."""
    from threadpoolctl import threadpool_limits
    from oracle import bonded as obonded, integrate as ointeg, pairs as opairs
    from oracle.ewald import PME
    lam = sysd.lambdas[lam_index]
    x = sysd.pos.astype(np.float64)
    rng = np.random.default_rng(22274)
    atoms = np.sort(rng.choice(sysd.n_atoms, n_atoms_sample, replace=False))
    chunks = np.array_split(atoms, nproc)
    t0 = time.perf_counter()
    with _pool(sysd, nproc) as p:
        cpu_s = p.map(_rsa_task, [(sysd.pos, lam, c) for c in chunks], chunksize=1)
    wall_rs = time.perf_counter() - t0
    rs_cpu = float(np.sum(cpu_s))                   # CPU seconds for the sampled atoms
    with threadpool_limits(limits=1):
        t1 = time.perf_counter()
        pme = PME(sysd.box, sysd.grid, sysd.ewald_alpha)
        er, fr = pme.energy_forces(x, opairs.scaled_charges(sysd, lam[0]))
        ex, fx = opairs.exclusion_correction(x, sysd, lam)
        eb, fb = obonded.bonds(x, sysd)
        erst, frst = obonded.boresch(x, sysd, lam[2])
        f_rest = fr + fx + fb + frst
        v = np.zeros_like(x)
        ointeg.langevin_middle_step(sysd, x, v, lambda y: f_rest, DT, 300.0, 0.5, 1, lam_index, 0)
        t_rest = time.perf_counter() - t1
    # CPU seconds of one whole window-step, and its wall time on nproc + 1 cores
    cpu_step = rs_cpu * sysd.n_atoms / n_atoms_sample + t_rest
    wall_step = cpu_step / (nproc + 1)
    return {"value": DT * 1e-3 / wall_step * 86400.0, "unit": "ns·windows/day", "cores": nproc + 1,
            "kind": "oracle",
            "sample": f"window {lam_index} of the {sysd.n_atoms}-atom leg: FP64 real-space forces of "
                      f"{n_atoms_sample} sampled atoms by the oracle's per-atom brute force ({rs_cpu:.1f} CPU-s "
                      f"over {nproc} processes, {wall_rs:.1f} s wall), scaled to all atoms, plus one FP64 PME "
                      f"{'x'.join(map(str, sysd.grid))}, exclusion/bond/restraint terms and one Langevin-middle "
                      f"step with SHAKE ({t_rest:.1f} s); one window-step = {cpu_step:.0f} CPU-s, "
                      f"{wall_step:.1f} s on {nproc + 1} cores"}


def ukn_at_scale(ctx, felis, leg, sysd, beta, n_per_window, chunk_per_window, n_oracle, seg, nproc):
    """u_kn of every state over n_per_window frames per window (seeded
    Gaussian perturbations, 0.02 A, of each window's current frame, made on
    the device chunk by chunk: the coordinates are input, the u_kn calls are
    timed), MBAR on the whole K x (K n_per_window) matrix, and the oracle on a
    seeded subset: n_oracle frames from the windows of ``seg``, every state
    element by element and Delta G over the segment."""
    import torch
    from oracle import mbar as ombar
    W, N = leg.n_windows, leg.n_atoms
    nf = W * n_per_window
    u = torch.empty((W, nf), dtype=torch.float64, device='cuda')
    base = leg.positions()                               # (W, N, 3)
    gen_t = torch.Generator(device='cuda')
    gen_t.manual_seed(22274)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t_ukn = 0.0
    nch = chunk_per_window * W
    for c0 in range(0, n_per_window, chunk_per_window):
        m = min(chunk_per_window, n_per_window - c0)
        fr = base.repeat(m, 1, 1)                         # frame k of the chunk: window k % W
        fr += torch.randn(fr.shape, generator=gen_t, device='cuda') * 0.02
        xs, ys, zs = fr[..., 0].contiguous(), fr[..., 1].contiguous(), fr[..., 2].contiguous()
        del fr
        ev0.record()
        felis.ukn(ctx, leg, sysd.lambdas, xs, ys, zs, beta, out=u[:, c0 * W:(c0 + m) * W])
        ev1.record()
        torch.cuda.synchronize()
        t_ukn += ev0.elapsed_time(ev1) / 1000.0
        if c0 == 0:
            first = (xs[:nch].clone(), ys[:nch].clone(), zs[:nch].clone())
        del xs, ys, zs
    ctx.device_check()
    N_k = np.full(W, n_per_window)
    ev0.record()
    f, iters = felis.mbar(ctx, u, N_k, tol=1e-10, max_iter=20000)
    ev1.record()
    torch.cuda.synchronize()
    mbar_ms = ev0.elapsed_time(ev1)
    dg_full = felis.delta_g(f, 300.0)
    # oracle subset: frames of the first chunk from the segment's windows
    rng = np.random.default_rng(22274)
    cand = np.array([k for k in range(nch) if (k % W) in seg])
    pick = np.sort(rng.choice(cand, size=min(n_oracle, len(cand)), replace=False))
    fx, fy, fz = (t[torch.as_tensor(pick, device='cuda')].cpu().numpy() for t in first)
    frames = np.stack([fx, fy, fz], -1)
    t0 = time.perf_counter()
    with _pool(sysd, nproc) as p:
        ref = np.stack(p.map(_ukn_task, [(fr, sysd.lambdas, beta) for fr in frames], chunksize=1), 1)
    t_or = time.perf_counter() - t0
    cols = torch.as_tensor(pick, device='cuda')             # first chunk: frame k is column k
    ug = u[:, cols].cpu().numpy()
    du = (ug - ug[0]) - (ref - ref[0])
    states = pick % W
    ss = np.array(seg)
    Nk_s = np.array([(states == s).sum() for s in ss])
    f_g, _ = felis.mbar(ctx, torch.as_tensor(np.ascontiguousarray(ug[ss])).cuda(), Nk_s, tol=1e-12, max_iter=20000)
    f_o, it_o = ombar.mbar(ref[ss], Nk_s, tol=1e-12, max_iter=2000000)
    dg_g, dg_o = felis.delta_g(f_g, 300.0), felis.delta_g(f_o, 300.0)
    bytes_per_frame = N * 12
    return {"frames": int(nf), "states": int(W), "frames_per_window": int(n_per_window),
            "ukn_s": round(t_ukn, 3), "frames_per_s": nf / t_ukn,
            "coordinate_stream_gb_per_s": nf * bytes_per_frame / t_ukn / 1e9,
            "coordinate_stream_frac_of_hbm": nf * bytes_per_frame / t_ukn / 8e12,
            "mbar_ms": mbar_ms, "mbar_iterations": int(iters), "dG_kcal_per_mol": dg_full,
            "oracle_subset": {"frames": int(len(pick)), "windows": [int(s) for s in seg],
                              "max_abs_du_kT_all_states": float(np.abs(du).max()),
                              "dG_gpu": dg_g, "dG_oracle": dg_o, "abs_ddG": abs(dg_g - dg_o),
                              "passed": bool(abs(dg_g - dg_o) <= DDG_TOL), "oracle_s": round(t_or, 1),
                              "oracle_mbar_iterations": int(it_o)},
            "frames_from": "seeded Gaussian perturbations (0.02 A) of each window's frame after the timed run, "
                           "generated on the device in chunks (untimed)"}


def served_stream(ctx, systems, specs, n_steps, sample_every, rate, compare=True):
    """The served form: a seeded Poisson stream of uneven legs, admitted by
    device memory and stepped together with continuous batching; latency is
    arrival -> Delta G of each leg."""
    from paper_2603_22274_amd import serve
    reqs = serve.poisson_requests(len(systems), rate, 22274, lambda i: systems[i], n_steps, sample_every)
    eng = serve.FelisEngine(ctx, mbar_max_iter=5000)
    srv = serve.Server(eng, hbm_budget=200 << 30, epoch_steps=50)
    out, stats = srv.serve(reqs)
    stats = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in stats.items()}
    stats["workload"] = (f"{len(systems)} legs, atoms {[s.n_atoms for s in systems]}, windows "
                         f"{[s.n_windows for s in systems]}, {n_steps} steps per window, u_kn every "
                         f"{sample_every}, Poisson arrivals at {rate} legs/s, HBM budget 200 GiB, starts relaxed by "
                         f"400 high-friction steps of the coupled state")
    stats["mbar_converged"] = sum(1 for r in out if r.status == 'ok')
    if compare:
        # the same legs and arrivals, one leg and one window at a time in the
        # plain form (FP32 forces summed with FP64 atomics)
        reqs = serve.poisson_requests(len(systems), rate, 22274, lambda i: systems[i], n_steps, sample_every)
        seq = serve.run_sequential_per_window(ctx, reqs, plain=True)
        stats["plain_sequential"] = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in seq.items()}
    stats["not_ok"] = [{"leg": r.rid, "status": str(r.status)[:200]} for r in out if r.status != 'ok']
    stats["latencies_s"] = [round(r.latency, 3) for r in out]
    return stats


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=20)
    ap.add_argument('--warmup', type=int, default=3)
    ap.add_argument('--md', type=int, default=50, help='MD steps per bench step (u_kn sample interval)')
    ap.add_argument('--workload', choices=('complex42', 'solvent20'), default='complex42')
    ap.add_argument('--equil', type=int, default=200, help='untimed equilibration MD steps of every window')
    ap.add_argument('--ddg-segment', type=str, default='16:23',
                    help="neighbouring windows a:b whose frames the oracle re-evaluates (ddG gate); '' to skip")
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--cpu-atoms', type=int, default=6000, help='atoms of the CPU-baseline sample')
    ap.add_argument('--no-per-window', action='store_true')
    ap.add_argument('--hrex-every', type=int, default=2500,
                    help='MD steps between replica-exchange attempts among the windows (0: none); 5 ps as in the paper')
    ap.add_argument('--serve-legs', type=int, default=16, help='legs in the served stream (0: skip)')
    ap.add_argument('--serve-steps', type=int, default=400, help='MD steps per window of a served leg')
    ap.add_argument('--no-serve-compare', action='store_true',
                    help='skip the same stream run one leg and one window at a time in the plain form')
    ap.add_argument('--schedule', choices=('bench', 'paper'), default='bench',
                    help="'paper': the production schedule of appendix B on the same system (80 complex or "
                         "73 solvent windows)")
    ap.add_argument('--npt', action='store_true',
                    help='also measure the leg in NPT (Monte Carlo barostat, a volume move every 25 steps)')
    ap.add_argument('--ukn-frames', type=int, default=2000,
                    help='frames per window of the u_kn + MBAR measurement at scale (0: skip)')
    ap.add_argument('--ukn-oracle-frames', type=int, default=210, help='frames of its oracle subset')
    ap.add_argument('--copy-calibration', action='store_true',
                    help='run a plain 256 MiB device copy first (reference for traffic counters)')
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get('WORLD_SIZE', '1')) > 1:
        print("bench.py measures one GPU: the path needs no collective and nothing here runs on a second GPU; "
              "legs and window segments shard across GPUs without exchange.", file=sys.stderr)
        sys.exit(2)

    from paper_2603_22274_amd import gen
    nproc = _workers()
    # inputs first, before anything touches the GPU: the headline leg and the
    # served stream's legs (atoms ~ U[5k, 80k], windows ~ {12, 20, 42})
    t_gen = time.perf_counter()
    sysd = gen.config2() if args.workload == 'complex42' else gen.config1()
    if args.schedule == 'paper':
        import dataclasses
        sysd = dataclasses.replace(sysd, lambdas=gen.schedule('paper_complex' if args.workload == 'complex42'
                                                              else 'paper_solvent'))
    specs = []
    if args.serve_legs > 0:
        rng = np.random.default_rng([22274, 4])
        specs = [(int(rng.integers(5000, 80001)), int(rng.choice([12, 20, 42])), 22274 + i)
                 for i in range(args.serve_legs)]
        with mp.get_context('spawn').Pool(nproc) as p:
            served_systems = p.map(_gen_task, specs, chunksize=1)
    t_gen = time.perf_counter() - t_gen
    print(f"# inputs generated in {t_gen:.1f} s ({nproc} processes)", file=sys.stderr, flush=True)

    import torch
    from paper_2603_22274_amd import felis, serve

    if args.copy_calibration:
        src = torch.empty(256 << 20, dtype=torch.uint8, device='cuda')
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ctx = felis.Context(0)
    # relaxed start of the coupled state (input preparation, untimed)
    serve.relax_start(ctx, sysd)
    leg = felis.Leg(ctx, sysd, seed=22274)
    W, N = leg.n_windows, leg.n_atoms
    beta = 1.0 / (KB * 300.0)
    felis.build_nlist(ctx, [leg], force=True)
    felis.step(ctx, [leg], args.equil, DT, 300.0, 5.0)
    ctx.device_check()
    print(f"# {args.workload}: {N} atoms, {W} windows equilibrated", file=sys.stderr, flush=True)
    # algorithmic work: unique pairs within r_c per window (FP64 distances)
    felis.build_nlist(ctx, [leg])
    npairs_cut = sum(felis.nlist_count_pairs(ctx, leg, w, sysd.r_cut) for w in range(W))

    seg = []
    if args.ddg_segment:
        a, b = (int(v) for v in args.ddg_segment.split(':'))
        seg = list(range(max(0, a), min(W, b)))
    n_samples = args.steps
    u = torch.empty((W, W * n_samples), dtype=torch.float64, device='cuda')
    frames = torch.empty((n_samples, len(seg), N, 3), dtype=torch.float32, device='cuda') if seg else None
    seg_idx = torch.as_tensor(seg, dtype=torch.long, device='cuda') if seg else None
    state_of = np.arange(W)                  # replica -> state held (changes only at an exchange)
    sample_states = []
    md_done = [0]
    attempts = [0]

    def bench_step(k, timed):
        felis.step(ctx, [leg], args.md, DT, 300.0, 0.5)
        col = u[:, k * W:(k + 1) * W] if timed else None
        col = felis.ukn(ctx, leg, sysd.lambdas, leg.x, leg.y, leg.z, beta, out=col)
        if timed and seg:
            frames[k, :, :, 0].copy_(leg.x.index_select(0, seg_idx))
            frames[k, :, :, 1].copy_(leg.y.index_select(0, seg_idx))
            frames[k, :, :, 2].copy_(leg.z.index_select(0, seg_idx))
            sample_states.append(state_of.copy())
        md_done[0] += args.md
        if args.hrex_every and md_done[0] % args.hrex_every == 0:
            felis.hrex(ctx, leg, col, attempts[0], 22274, count=False)   # from this sample's u_kn
            attempts[0] += 1
            state_of[:] = felis.leg_states(ctx, leg)

    for k in range(args.warmup):
        bench_step(0, False)
    torch.cuda.synchronize()
    ctx.device_check()
    # live timing of the pair kernel (every PAIR_SAMPLE-th launch) and of u_kn:
    # every recorded event is a queue packet between two kernels, ~6 us of
    # idle queue each (the stage breakdown is taken after the timed region)
    felis.profile(ctx, True, stages=(felis.PROF_PAIRS, felis.PROF_UKN), every=PAIR_SAMPLE)
    for which in range(felis.PROF_BARO + 1):
        felis.profile_read(ctx, which)
    sample_states.clear()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        bench_step(k, True)
    timed_attempts = attempts[0]
    N_k = np.full(W, n_samples)
    mbar_ok = True
    try:
        f, iters = felis.mbar(ctx, u, N_k, tol=1e-10, max_iter=20000)
    except felis.FelisError as e:
        if e.code != felis.E_NOCONV:
            raise
        mbar_ok, f, iters = False, None, 20000
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    felis.profile(ctx, False)
    prof = {name: felis.profile_read(ctx, i) for i, name in enumerate(('pairs', 'pme', 'nlist', 'integrate', 'ukn'))}
    ctx.device_check()
    print(f"# timed region {t1 - t0:.2f} s", file=sys.stderr, flush=True)
    # stage breakdown (untimed): two more bench steps with every stage bracketed
    felis.profile(ctx, True, every=1)
    for k in range(2):
        bench_step(0, False)
    torch.cuda.synchronize()
    felis.profile(ctx, False)
    stages = {name: felis.profile_read(ctx, i) for i, name in enumerate(('pairs', 'pme', 'nlist', 'integrate'))}
    # the same pair kernel alone (felis_nonbonded: no reciprocal space beside
    # it), every launch bracketed
    felis.profile(ctx, True, stages=(felis.PROF_PAIRS,), every=1)
    for which in range(felis.PROF_BARO + 1):
        felis.profile_read(ctx, which)
    for k in range(6):
        felis.nonbonded(ctx, [leg], False)
    torch.cuda.synchronize()
    felis.profile(ctx, False)
    iso_ms, iso_n = felis.profile_read(ctx, felis.PROF_PAIRS)
    iso_s = iso_ms / max(iso_n, 1) / 1000.0
    wall = t1 - t0
    md_steps = args.steps * args.md
    ns_windows = md_steps * DT * W / 1000.0
    rate = ns_windows / (wall / 86400.0)
    pairs_ms, pairs_n = prof['pairs']
    avg_pairs_s = pairs_ms / max(pairs_n, 1) / 1000.0
    achieved = npairs_cut * FLOP_PER_PAIR / avg_pairs_s / 1e12
    alg_bytes = PAIR_BYTES_PER_ATOM * N * W
    traffic = _traffic(args.workload)
    dg = felis.delta_g(f, 300.0) if f is not None else None
    # device time of one replica-exchange attempt (its u_kn is the sample's)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ucol = u[:, :W]
    felis.hrex(ctx, leg, ucol, attempts[0], 22274, count=False)
    ev0.record()
    for k in range(10):
        felis.hrex(ctx, leg, ucol, attempts[0] + 1 + k, 22274, count=False)
    ev1.record()
    torch.cuda.synchronize()
    hrex_us = ev0.elapsed_time(ev1) / 10 * 1000.0

    ddg = None
    if seg:
        # frames of the segment's windows, grouped by the state each was sampled in
        fr = frames.reshape(n_samples * len(seg), N, 3).cpu().numpy()
        st = np.concatenate([np.asarray(s)[seg] for s in sample_states])
        cols = np.concatenate([k * W + np.asarray(seg) for k in range(n_samples)])
        keep = np.isin(st, seg)                  # a replica may hold a state outside the segment after an exchange
        fr, st, cols = fr[keep], st[keep], cols[keep]
        ucols = u[:, torch.as_tensor(cols, device='cuda')]
        ddg = ddg_check(sysd, fr, st, seg, ucols, beta, ctx, felis, nproc)
        print(f"# ddG check {ddg['abs_ddG']:.2e} kcal/mol ({ddg['oracle_s']} s)", file=sys.stderr, flush=True)
        del fr
    del frames
    value = rate if (ddg is None or ddg['passed']) else 0.0

    ukn_scale = None
    if args.ukn_frames > 0 and seg:
        ukn_scale = ukn_at_scale(ctx, felis, leg, sysd, beta, args.ukn_frames, 50, args.ukn_oracle_frames, seg,
                                 nproc)
        print(f"# u_kn at scale: {ukn_scale['frames']} frames in {ukn_scale['ukn_s']} s; oracle subset "
              f"|ddG| {ukn_scale['oracle_subset']['abs_ddG']:.2e}", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()

    per_window = None
    if not args.no_per_window:
        # the same leg as one-window legs, each launched on its own: the plain
        # form (FP32 pairs, FP64 atomic force sums) and the default kernels
        wins = list(range(W))
        pos0 = leg.positions().cpu().numpy()
        nrep = 10
        forms = {}
        for name, plain in (("plain", True), ("unbatched_same_kernels", False)):
            legs1 = [felis.Leg(ctx, sysd, windows=[w], seed=22274, positions=pos0[w], plain_fp64=plain)
                     for w in wins]
            for l in legs1:
                felis.build_nlist(ctx, [l], force=True)
            for l in legs1:
                felis.step(ctx, [l], 5, DT, 300.0, 0.5)
            torch.cuda.synchronize()
            ta = time.perf_counter()
            for l in legs1:
                felis.step(ctx, [l], nrep, DT, 300.0, 0.5)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            ctx.device_check()
            forms[name] = nrep * DT * len(wins) / 1000.0 / ((tb - ta) / 86400.0)
            del legs1
            torch.cuda.empty_cache()
        per_window = {"value": forms["plain"], "unit": "ns·windows/day",
                      "form": "plain: one window per leg and launch chain, FP32 pair and reciprocal forces summed "
                              "with FP64 atomics, MD only",
                      "unbatched_same_kernels": forms["unbatched_same_kernels"],
                      "md_steps_per_window": nrep, "windows": len(wins)}

    npt = None
    if args.npt:
        # the same leg in the paper's ensemble: NPT at 1.01325 bar, a volume
        # move of every window every 25 steps (two energy evaluations each)
        every = 25
        nl = felis.Leg(ctx, sysd, seed=22274, positions=leg.positions().cpu().numpy(), pressure_bar=1.01325,
                       barostat_every=every)
        felis.build_nlist(ctx, [nl], force=True)
        felis.step(ctx, [nl], 2 * every, DT, 300.0, 0.5)
        torch.cuda.synchronize()
        n_npt = 4 * every
        felis.profile(ctx, True, stages=(felis.PROF_BARO,))
        for which in range(felis.PROF_BARO + 1):
            felis.profile_read(ctx, which)
        tc = time.perf_counter()
        felis.step(ctx, [nl], n_npt, DT, 300.0, 0.5)
        torch.cuda.synchronize()
        td = time.perf_counter()
        baro_ms, baro_n = felis.profile_read(ctx, felis.PROF_BARO)
        felis.profile(ctx, False)
        st = felis.barostat_stats(ctx, nl)
        vols = np.prod(felis.leg_boxes(ctx, nl), axis=1)
        ctx.device_check()
        npt = {"value": n_npt * DT * W / 1000.0 / ((td - tc) / 86400.0), "unit": "ns·windows/day",
               "pressure_bar": 1.01325, "move_every_md_steps": every, "md_steps": n_npt,
               "move_ms": baro_ms / max(baro_n, 1), "moves": int(baro_n),
               "acceptance": float(st[:, 9].sum() / max(st[:, 8].sum(), 1)),
               "volume_over_start": [float(v / np.prod(sysd.box)) for v in (vols.min(), vols.mean(), vols.max())],
               "note": "every window its own box and complex PME grid; MD + volume moves, no u_kn"}
        del nl
        torch.cuda.empty_cache()

    served = None
    if args.serve_legs > 0:
        del leg
        torch.cuda.empty_cache()
        for s in served_systems:                # relaxed starting coordinates (input preparation, untimed)
            serve.relax_start(ctx, s)
        served = served_stream(ctx, served_systems, specs, args.serve_steps, 50, 2.0,
                               compare=not args.no_serve_compare)
        print(f"# served {served['completed']}/{served['legs']} legs in {served['wall_s']} s", file=sys.stderr,
              flush=True)

    cpu = None if args.no_cpu_baseline else cpu_baseline(sysd, min(W - 1, 30), nproc, args.cpu_atoms)
    work = ("complex leg, 42 windows (12 restraint, 10 electrostatic, 20 vdW), 70527 atoms (5,000-atom chain "
            "protein, 50-atom Boresch-restrained ligand, 4 Na+/4 Cl-, 21,823 TIP3P-geometry waters), 88 A box, "
            "r_c 10 A, skin 1 A, PME 96^3 order 4, 2 fs, 300 K" if args.workload == 'complex42' else
            "solvent leg, 20 windows, 7540 atoms (2500 TIP3P-geometry waters + 40-atom ligand), 42 A box, "
            "r_c 10 A, skin 1 A, PME 48^3 order 4, 2 fs, 300 K")
    if args.schedule == 'paper':
        work += f"; the production schedule of appendix B ({W} windows)"
    out = {
        "metric": METRIC, "value": value, "unit": "ns·windows/day", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1000.0, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
        "config": {"workload": work, "md_steps_per_step": args.md, "windows": W, "atoms": N, "ukn_states": W,
                   "mbar_samples": int(W * n_samples)},
        "throughput_before_gate": rate,
        "ddg_check": ddg,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32, "traffic": traffic,
                     "nonpacked_issue_peak": ISSUE_FP32, "frac_of_nonpacked_peak": achieved / ISSUE_FP32,
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "traffic_over_algorithmic": (traffic / alg_bytes) if traffic else None,
                     "kernel": f"k_pairs (real-space pair kernel, all {W} windows per launch)",
                     "pairs_in_cutoff_per_launch": int(npairs_cut), "flop_per_pair": FLOP_PER_PAIR,
                     "avg_launch_ms": avg_pairs_s * 1000.0, "launches": pairs_n,
                     "alone": {"avg_launch_ms": iso_s * 1000.0, "launches": iso_n,
                               "achieved": npairs_cut * FLOP_PER_PAIR / iso_s / 1e12,
                               "frac": npairs_cut * FLOP_PER_PAIR / iso_s / 1e12 / PEAK_FP32,
                               "frac_of_nonpacked_peak": npairs_cut * FLOP_PER_PAIR / iso_s / 1e12 / ISSUE_FP32,
                               "note": "the same kernel launched by felis_nonbonded after the timed region, "
                                       "with nothing beside it; the timed figures above include the "
                                       "reciprocal-space kernels sharing the compute units"},
                     "launches_timed_of": args.steps * args.md},
        "cpu_baseline": cpu,
        "per_window_form": per_window,
        "ukn_cfg3": ukn_scale,
        "npt": npt,
        "stage_ms_per_md_step": {k: v[0] / max(v[1], 1) for k, v in stages.items()},
        "ukn_ms_per_call": prof['ukn'][0] / max(prof['ukn'][1], 1),
        "replica_exchange": {"every_md_steps": args.hrex_every, "attempts_in_timed_region": timed_attempts,
                             "attempt_us": hrex_us,
                             "note": "neighbour swaps from the sample-time u_kn; one single-workgroup kernel"},
        "mbar": {"converged": mbar_ok, "iterations": iters, "dG_kcal_per_mol": dg},
        "leg_latency_s": ({"p50": served["latency_p50_s"], "p99": served["latency_p99_s"],
                           "legs": served["completed"], "from": "served stream, arrival to Delta G"}
                          if served else None),
        "served": served,
    }
    print(json.dumps(out))


if __name__ == '__main__':
    main()
