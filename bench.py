"""Throughput of the alchemical-window hot path on one MI355X.

Workload: the 20-window solvent leg (2,500 seeded-orientation 3-site waters in
a 42 A box plus a 40-atom ligand; cutoff 10 A, skin 1 A, PME 48^3 order 4;
8 electrostatic then 12 vdW windows), all windows batched in every launch.

One bench step = one pass of the whole hot path over the batch: `--md` Langevin
-middle steps of 2 fs for every window (list check/rebuild, real-space pair
kernel, PME, bonded terms, integrator with SETTLE), then the reduced
potentials u_kn of every window's current frame at all 20 states.  After the
timed steps, MBAR solves the collected u_kn (inside the timed region).

Prints one JSON line: aggregate ns.windows/day, the pair kernel's roofline
(FP32 ALU bound; algorithmic flops from in-cutoff pairs; duration from HIP
events recorded around the kernel inside the timed region), the FP64 oracle
timed on the host as the CPU baseline, and the unbatched per-window form of
the same leg for comparison.
"""
from __future__ import annotations

import argparse
import json
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
FLOP_PER_PAIR = 75              # FP32 flops per in-cutoff pair (FMA = 2)
PAIR_SAMPLE = 5                 # the timed region brackets every 5th pair-kernel launch with HIP events
TRAFFIC_FILE = os.path.join(ROOT, 'profiles', 'pairs_traffic_solvent20.json')


def _traffic():
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    from paper_2603_22274_amd.profiling import src_digest
    if t.get('kernel_digest') != src_digest():
        return None
    return t.get('bytes_per_launch')


def cpu_baseline(sysd, windows=(0, 5, 9, 14, 19)):
    """Window-steps of the FP64 oracle (forces by brute force + PME, one
    Langevin-middle step) on one host thread (library thread pools limited to
    one), a bounded sample of ~10 s; scaled to ns.windows/day."""
    from threadpoolctl import threadpool_limits
    from oracle import energy as oenergy, integrate as ointeg
    from oracle.ewald import PME
    pme = PME(sysd.box, sysd.grid, sysd.ewald_alpha)
    x = sysd.pos.astype(np.float64)
    v = np.zeros_like(x)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        for w in windows:
            lam = sysd.lambdas[w]
            force = lambda y, lam=lam: oenergy.window_energy(sysd, y, lam, pme=pme)[1]
            ointeg.langevin_middle_step(sysd, x, v, force, DT, 300.0, 0.5, 1, w, 0)
        t = (time.perf_counter() - t0) / len(windows)
    return {"value": DT * 1e-3 / t * 86400.0, "unit": "ns·windows/day", "cores": 1, "kind": "oracle",
            "sample": f"{len(windows)} window-steps (windows {list(windows)}) of the {sysd.n_atoms}-atom leg: "
                      f"brute-force FP64 pair sums, FP64 PME 48^3, one Langevin-middle step with SHAKE each; "
                      f"{t * len(windows):.1f} s on one thread (thread pools limited to 1) of "
                      f"{os.cpu_count()} host cores"}


def serve_mix(ctx, n_legs, per_window):
    """A seeded stream of uneven legs (4,000-12,000 atoms; 12, 20 or 42
    windows; 400 steps, u_kn every 50; Poisson arrivals at 8 legs/s, so the
    stream arrives faster than the GPU finishes it) served with continuous
    batching, then the same stream one leg and one window at a time.
    Latency = arrival to Delta G."""
    from paper_2603_22274_amd import serve
    reqs = serve.served_workload(n_legs=n_legs, rate=8.0, seed=22274, atoms=(4000, 12000), n_steps=400,
                                 sample_every=50)
    for r in reqs:                      # relaxed starting coordinates (input preparation, untimed)
        serve.relax_start(ctx, r.sysd)
    eng = serve.FelisEngine(ctx, mbar_max_iter=5000)
    srv = serve.Server(eng, hbm_budget=64 << 30, epoch_steps=50)
    out, stats = srv.serve(reqs)
    stats = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in stats.items()}
    stats["workload"] = (f"{n_legs} legs, atoms {sorted(r.sysd.n_atoms for r in reqs)}, windows "
                         f"{[r.sysd.n_windows for r in reqs]}, 400 steps each, u_kn every 50, Poisson 8 legs/s, "
                         f"starts relaxed by 400 high-friction steps of the coupled state")
    stats["mbar_converged"] = sum(1 for r in out if r.status == 'ok')
    if per_window:
        seq = serve.run_sequential_per_window(ctx, reqs)
        stats["per_window_sequential"] = {k: round(v, 4) for k, v in seq.items()}
    return stats


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument('--gpus', type=int, default=1)
    ap.add_argument('--steps', type=int, default=20)
    ap.add_argument('--warmup', type=int, default=3)
    ap.add_argument('--md', type=int, default=50, help='MD steps per bench step (u_kn sample interval)')
    ap.add_argument('--no-cpu-baseline', action='store_true')
    ap.add_argument('--no-per-window', action='store_true')
    ap.add_argument('--equil', type=int, default=200, help='untimed equilibration MD steps')
    ap.add_argument('--schedule', choices=('bench', 'paper'), default='bench',
                    help="'paper': the 73-window production solvent schedule of appendix B on the same system")
    ap.add_argument('--hrex-every', type=int, default=2500,
                    help='MD steps between replica-exchange attempts among the windows (0: none); 5 ps as in the paper')
    ap.add_argument('--serve-legs', type=int, default=8, help='legs in the served mixed workload (0: skip)')
    ap.add_argument('--no-npt', action='store_true', help='skip the NPT (Monte Carlo barostat) line')
    ap.add_argument('--copy-calibration', action='store_true',
                    help='run a plain 256 MiB device copy first (reference for traffic counters)')
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get('WORLD_SIZE', '1')) > 1:
        print("bench.py measures one GPU: the path needs no collective and nothing here runs on a second GPU; "
              "legs and window segments shard across GPUs without exchange (see DESIGN.md).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_22274_amd import felis, gen

    if args.copy_calibration:
        src = torch.empty(256 << 20, dtype=torch.uint8, device='cuda')
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    sysd = gen.config1()
    if args.schedule == 'paper':
        import dataclasses
        sysd = dataclasses.replace(sysd, lambdas=gen.schedule('paper_solvent'))
    ctx = felis.Context(0)
    leg = felis.Leg(ctx, sysd, seed=22274)
    W = leg.n_windows
    beta = 1.0 / (KB * 300.0)
    felis.build_nlist(ctx, [leg], force=True)
    # settle the lattice start before anything is measured
    felis.step(ctx, [leg], args.equil, DT, 300.0, 5.0)
    ctx.device_check()
    # algorithmic work: unique pairs within r_c per window (FP64 distances)
    felis.build_nlist(ctx, [leg])
    npairs_cut = sum(len(felis.nlist_export_pairs(ctx, leg, w, sysd.r_cut)) for w in range(W))

    n_samples = args.steps
    u = torch.empty((W, W * n_samples), dtype=torch.float64, device='cuda')

    md_done = [0]
    attempts = [0]

    def bench_step(k, timed):
        felis.step(ctx, [leg], args.md, DT, 300.0, 0.5)
        col = u[:, k * W:(k + 1) * W] if timed else None
        col = felis.ukn(ctx, leg, sysd.lambdas, leg.x, leg.y, leg.z, beta, out=col)
        md_done[0] += args.md
        if args.hrex_every and md_done[0] % args.hrex_every == 0:
            felis.hrex(ctx, leg, col, attempts[0], 22274, count=False)   # from this sample's u_kn
            attempts[0] += 1

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
    # stage breakdown (untimed): two more bench steps with every stage bracketed
    felis.profile(ctx, True, every=1)
    for k in range(2):
        bench_step(0, False)
    torch.cuda.synchronize()
    felis.profile(ctx, False)
    stages = {name: felis.profile_read(ctx, i) for i, name in enumerate(('pairs', 'pme', 'nlist', 'integrate'))}
    wall = t1 - t0
    md_steps = args.steps * args.md
    ns_windows = md_steps * DT * W / 1000.0
    value = ns_windows / (wall / 86400.0)
    pairs_ms, pairs_n = prof['pairs']
    avg_pairs_s = pairs_ms / max(pairs_n, 1) / 1000.0
    flops = npairs_cut * FLOP_PER_PAIR
    achieved = flops / avg_pairs_s / 1e12
    traffic = _traffic()
    dg = float((f[-1] - f[0]) / beta) if f is not None else None
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

    per_window = None
    if not args.no_per_window:
        # the same leg as 20 one-window legs, each launched on its own
        legs1 = [felis.Leg(ctx, sysd, windows=[w], seed=22274, positions=leg.positions()[w].cpu().numpy())
                 for w in range(W)]
        for l in legs1:
            felis.build_nlist(ctx, [l], force=True)
        nrep = max(1, args.md // 2)
        for l in legs1:
            felis.step(ctx, [l], 5, DT, 300.0, 0.5)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for l in legs1:
            felis.step(ctx, [l], nrep, DT, 300.0, 0.5)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        per_window = {"value": nrep * DT * W / 1000.0 / ((tb - ta) / 86400.0), "unit": "ns·windows/day",
                      "form": "one window per leg and launch chain (same kernels), MD only",
                      "md_steps_per_window": nrep}

    npt = None
    if not args.no_npt:
        # the same leg in the paper's ensemble: NPT at 1.01325 bar, a volume
        # move of every window every 25 steps (two energy evaluations each)
        every = 25
        nl = felis.Leg(ctx, sysd, seed=22274, positions=leg.positions().cpu().numpy(), pressure_bar=1.01325,
                       barostat_every=every)
        felis.build_nlist(ctx, [nl], force=True)
        felis.step(ctx, [nl], 4 * every, DT, 300.0, 0.5)
        torch.cuda.synchronize()
        n_npt = 8 * every
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

    served = None
    if args.serve_legs > 0:
        served = serve_mix(ctx, args.serve_legs, not args.no_per_window)

    cpu = None if args.no_cpu_baseline else cpu_baseline(sysd)
    out = {
        "metric": METRIC, "value": value, "unit": "ns·windows/day", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": wall / args.steps * 1000.0, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp32", "data": "synthetic",
        "config": {"workload": f"solvent leg, {W} windows" + (" (the paper's 73-window production schedule)"
                                                             if args.schedule == 'paper' else "") +
                               ", 7540 atoms (2500 TIP3P-geometry waters + 40-atom "
                               "ligand), 42 A box, r_c 10 A, skin 1 A, PME 48^3 order 4, 2 fs, 300 K",
                   "md_steps_per_step": args.md, "windows": W, "atoms": sysd.n_atoms,
                   "ukn_states": W, "mbar_samples": int(W * n_samples)},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32, "traffic": traffic,
                     "nonpacked_issue_peak": ISSUE_FP32, "frac_of_nonpacked_peak": achieved / ISSUE_FP32,
                     "traffic_gb_per_s": (traffic / avg_pairs_s / 1e9) if traffic else None,
                     "kernel": f"k_pairs (real-space pair kernel, all {W} windows per launch)",
                     "pairs_in_cutoff_per_launch": int(npairs_cut), "flop_per_pair": FLOP_PER_PAIR,
                     "avg_launch_ms": avg_pairs_s * 1000.0, "launches": pairs_n,
                     "launches_timed_of": args.steps * args.md},
        "cpu_baseline": cpu,
        "per_window_form": per_window,
        "npt": npt,
        "stage_ms_per_md_step": {k: v[0] / max(v[1], 1) for k, v in stages.items()},
        "ukn_ms_per_call": prof['ukn'][0] / max(prof['ukn'][1], 1),
        "replica_exchange": {"every_md_steps": args.hrex_every, "attempts_in_timed_region": timed_attempts,
                             "attempt_us": hrex_us,
                             "note": "neighbour swaps from the sample-time u_kn; one single-workgroup kernel"},
        "mbar": {"converged": mbar_ok, "iterations": iters, "dG_kcal_per_mol": dg},
        "leg_latency_s": {"p50": wall, "p99": wall, "legs": 1,
                          "note": "one leg in this workload; the served mixed batch reports its own"},
        "served": served,
    }
    print(json.dumps(out))


if __name__ == '__main__':
    main()
