"""Served, continuously batched decoupling legs.

Requests (legs) arrive over time.  The server keeps every admitted leg's
coordinates, velocities, neighbour lists and u_kn samples resident in device
memory and advances all of them together: one epoch = one batched
``felis_step`` over every window of every active leg, so windows of different
legs share each kernel launch.  Between epochs it

* admits waiting legs first-come first-served while their device footprint
  fits the memory budget (and the batch has room),
* samples u_kn for legs at a sample boundary (every window's current frame at
  all of the leg's states),
* finishes legs that completed their steps (MBAR -> Delta G) and frees them,
* evicts a leg whose kernels latched an error (the rest of the batch goes on).

A window's trajectory depends only on its own leg (noise keyed by the leg's
seed, window and step; lists rebuilt on its own displacement; PME grids paired
inside the leg), so each result is bitwise the same alone and in any mix.

The scheduling logic talks to an engine object; ``FelisEngine`` drives the
C ABI on the GPU, tests substitute a CPU fake to check the logic alone.
"""
from __future__ import annotations

import dataclasses
import math
import sys
import time
import types
from typing import List

import numpy as np

KB = 0.0019872043


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float            # seconds after serving starts
    sysd: object              # gen.System (topology, coordinates, schedule)
    n_steps: int              # MD steps per window
    sample_every: int         # steps between u_kn samples
    seed: int = 1
    list_cap: int = 0         # neighbour-list capacity per cluster (0: library default)
    exchange_every: int = 0   # MD steps between replica-exchange attempts among the leg's windows
                              # (a multiple of sample_every; 0: none; the paper uses 5 ps)
    pressure_bar: float = 0.0  # > 0: NPT, a Monte Carlo volume move of every window every
    barostat_every: int = 25   # barostat_every MD steps (the paper: 1.01325 bar, 25 steps)


@dataclasses.dataclass
class Result:
    rid: int
    arrival: float
    admitted: float = math.nan
    finished: float = math.nan
    windows: int = 0
    atoms: int = 0
    steps: int = 0
    dG: float | None = None
    mbar_iters: int = 0
    retries: int = 0
    status: str = 'pending'

    @property
    def latency(self):
        return self.finished - self.arrival


def percentile(v, q):
    v = sorted(v)
    if not v:
        return math.nan
    k = (len(v) - 1) * q / 100.0
    lo, hi = int(math.floor(k)), int(math.ceil(k))
    return v[lo] + (v[hi] - v[lo]) * (k - lo)


class LegFailed(Exception):
    """A leg's kernels latched an error; ``needed_cap`` > 0 when the cause was
    neighbour-list capacity (the longest list that was asked for)."""

    def __init__(self, reason, needed_cap=0):
        super().__init__(reason)
        self.needed_cap = needed_cap


class Server:
    """First-come first-served admission by memory, epoch-wise batched stepping.

    A leg that fails is released at once; the rest of the batch carries on.  A
    list-capacity failure is retried (up to ``max_retries`` times) by queueing
    the leg again at the head of the line with the capacity it asked for plus
    a margin: the rerun starts from the same state and seed, so its result is
    the one a large enough capacity would have given from the start.
    """

    def __init__(self, engine, hbm_budget, epoch_steps=50, max_legs=64, dt=0.002, max_retries=1,
                 clock=time.perf_counter, sleep=time.sleep, on_event=None):
        self.engine = engine
        self.budget = hbm_budget
        self.epoch = epoch_steps
        self.max_legs = max_legs
        self.dt = dt
        self.max_retries = max_retries
        self.clock = clock
        self.sleep = sleep
        self.on_event = on_event          # called with each log entry as it happens
        self.log: List[dict] = []

    def _note(self, entry):
        self.log.append(entry)
        if self.on_event is not None:
            self.on_event(entry)

    def serve(self, requests):
        for r in requests:
            if r.n_steps % self.epoch or r.sample_every % self.epoch:
                raise ValueError("n_steps and sample_every must be multiples of the epoch")
        t0 = self.clock()
        now = lambda: self.clock() - t0
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        results = {r.rid: Result(r.rid, r.arrival, windows=r.sysd.n_windows, atoms=r.sysd.n_atoms)
                   for r in requests}
        waiting, active = [], []
        state = {'used': 0}

        def drop(a, exc):
            r, h, done, need = a
            self.engine.release(h)
            state['used'] -= need
            res = results[r.rid]
            if exc.needed_cap > 0 and res.retries < self.max_retries:
                res.retries += 1
                # the failed epoch ran on truncated lists (wrong forces), so the
                # longest list it saw understates the lists of the correct run:
                # retry with twice that length
                cap = (2 * int(exc.needed_cap) + 7) // 8 * 8
                waiting.insert(0, dataclasses.replace(r, list_cap=cap))
                self._note({'t': now(), 'event': 'retry', 'rid': r.rid, 'list_cap': cap})
            else:
                res.status = f'evicted: {exc}'
                res.finished = now()
                self._note({'t': now(), 'event': 'evict', 'rid': r.rid})

        while pending or waiting or active:
            t = now()
            while pending and pending[0].arrival <= t:
                waiting.append(pending.pop(0))
            while waiting and len(active) < self.max_legs:
                r = waiting[0]
                need = self.engine.footprint(r)
                if need > self.budget:                      # can never fit
                    waiting.pop(0)
                    results[r.rid].status = 'rejected: footprint above budget'
                    results[r.rid].finished = now()
                    continue
                if state['used'] + need > self.budget:
                    break
                waiting.pop(0)
                h = self.engine.admit(r)
                active.append([r, h, 0, need])
                state['used'] += need
                if math.isnan(results[r.rid].admitted):
                    results[r.rid].admitted = now()
                self._note({'t': now(), 'event': 'admit', 'rid': r.rid, 'used': state['used']})
            if not active:
                if pending:
                    self.sleep(max(0.0, pending[0].arrival - now()))
                continue
            failed = self.engine.run_epoch([a[1] for a in active], self.epoch)
            if self.on_event is not None:
                self.on_event({'t': now(), 'event': 'epoch', 'rid': None, 'active': len(active)})
            keep = []
            for a in active:
                r, h, done, need = a
                if id(h) in failed:
                    drop(a, failed[id(h)])
                    continue
                done += self.epoch
                a[2] = done
                try:
                    if done % r.sample_every == 0:
                        self.engine.sample(h)
                    if done >= r.n_steps:
                        dG, iters, ok = self.engine.finish(h)
                except LegFailed as e:
                    drop(a, e)
                    continue
                if done >= r.n_steps:
                    self.engine.release(h)
                    state['used'] -= need
                    res = results[r.rid]
                    res.dG, res.mbar_iters, res.steps = dG, iters, done
                    res.status = 'ok' if ok else 'ok (MBAR not converged)'
                    res.finished = now()
                    self._note({'t': now(), 'event': 'finish', 'rid': r.rid})
                    continue
                keep.append(a)
            active = keep
        wall = now()
        out = [results[r.rid] for r in requests]
        done = [x for x in out if x.status.startswith('ok')]
        lat = [x.latency for x in done]
        nsw = sum(x.windows * x.steps * self.dt * 1e-3 for x in done)
        stats = {'legs': len(out), 'completed': len(done), 'wall_s': wall,
                 'ns_windows_per_day': nsw / (wall / 86400.0) if wall > 0 else math.nan,
                 'latency_p50_s': percentile(lat, 50), 'latency_p99_s': percentile(lat, 99)}
        return out, stats


class FelisEngine:
    """Engine over the C ABI: one context, device-resident legs."""

    def __init__(self, ctx, dt=0.002, temperature=300.0, gamma=0.5, list_cap=0, mbar_tol=1e-10,
                 mbar_max_iter=20000, keep_frames=False):
        from . import felis
        self.felis = felis
        self.ctx = ctx
        self.dt, self.T, self.gamma = dt, temperature, gamma
        self.beta = 1.0 / (KB * temperature)
        self.list_cap = list_cap
        self.tol, self.max_iter = mbar_tol, mbar_max_iter
        # keep_frames: every sample's coordinates and replica -> state map stay
        # on the device after the leg finishes (frames[rid]: list of (W, N, 3)
        # tensors; states[rid]: list of numpy arrays), for checking a served
        # result against another implementation on the same frames
        self.keep_frames = keep_frames
        self.frames, self.states = {}, {}

    def footprint(self, r):
        """Device bytes a leg holds while active: scratch, state, topology and
        its u_kn sample matrix."""
        W = r.sysd.n_windows
        samples = r.n_steps // r.sample_every
        return (self.felis.leg_footprint(r.sysd, list_cap=r.list_cap or self.list_cap, pressure_bar=r.pressure_bar)
                + W * W * samples * 8)

    def admit(self, r):
        import torch
        leg = self.felis.Leg(self.ctx, r.sysd, seed=r.seed, list_cap=r.list_cap or self.list_cap,
                             pressure_bar=r.pressure_bar, barostat_every=r.barostat_every)
        h = types.SimpleNamespace(leg=leg, req=r, k=0, attempts=0)   # first step builds every window's list
        W = leg.n_windows
        # NPT: each sample's frames in their windows' current boxes
        h.boxes = (torch.empty((W, 3), dtype=torch.float64, device=leg.x.device) if r.pressure_bar > 0
                   else None)
        h.u = torch.empty((W, W * (r.n_steps // r.sample_every)), dtype=torch.float64, device=leg.x.device)
        return h

    def _failure(self, e):
        return LegFailed(str(e), e.needed_cap if e.code == self.felis.E_CAPACITY else 0)

    def run_epoch(self, handles, n):
        f = self.felis
        f.step(self.ctx, [h.leg for h in handles], n, self.dt, self.T, self.gamma)
        try:
            self.ctx.device_check()
        except f.FelisError as e:
            bad = getattr(e, 'leg', -1)
            if 0 <= bad < len(handles):
                return {id(handles[bad]): self._failure(e)}
            return {id(h): self._failure(e) for h in handles}    # unattributable: the whole batch
        return {}

    def sample(self, h):
        f = self.felis
        W = h.leg.n_windows
        col = h.u[:, h.k * W:(h.k + 1) * W]
        boxes = f.leg_boxes_device(self.ctx, h.leg, h.boxes) if h.boxes is not None else None
        f.ukn(self.ctx, h.leg, h.leg.lambdas, h.leg.x, h.leg.y, h.leg.z, self.beta, out=col, boxes=boxes)
        r = h.req
        if self.keep_frames:
            self.frames.setdefault(r.rid, []).append(h.leg.positions().clone())
            self.states.setdefault(r.rid, []).append(f.leg_states(self.ctx, h.leg))
        if r.exchange_every and ((h.k + 1) * r.sample_every) % r.exchange_every == 0:
            # replica exchange from this sample's u[state][replica] (no host sync)
            f.hrex(self.ctx, h.leg, col, h.attempts, r.seed, count=False)
            h.attempts += 1
        try:
            self.ctx.device_check()
        except f.FelisError as e:
            raise self._failure(e)
        h.k += 1

    def finish(self, h):
        f = self.felis
        W = h.leg.n_windows
        u = h.u[:, :h.k * W]
        try:
            fe, it = f.mbar(self.ctx, u, np.full(W, h.k), tol=self.tol, max_iter=self.max_iter)
            return f.delta_g(fe, self.T), it, True
        except f.FelisError as e:
            if e.code != f.E_NOCONV:
                raise LegFailed(str(e))
            return None, self.max_iter, False

    def release(self, h):
        h.leg = None
        h.u = None
        h.boxes = None


def relax_start(ctx, sysd, steps=400, seed=7, dt=0.002, temperature=300.0):
    """Replace ``sysd.pos`` with coordinates relaxed by high-friction Langevin
    dynamics of the fully coupled state with the Boresch restraint (if any)
    at full strength -- the fully coupled window with the largest
    lambda_restraint: a synthetic lattice start releases enough potential
    energy to heat a leg far above the target temperature under the
    production friction, and relaxing without the restraint lets the anchors
    drift from the restraint's reference geometry, which then strains every
    restrained window from the first step.  Input preparation, done before a
    leg is submitted."""
    from . import felis
    lam = np.asarray(sysd.lambdas, np.float64)
    coupled = np.where((lam[:, 0] == 1.0) & (lam[:, 1] == 1.0))[0]
    w = int(coupled[np.argmax(lam[coupled, 2])]) if len(coupled) else 0
    leg = felis.Leg(ctx, sysd, windows=[w], seed=seed)
    felis.step(ctx, [leg], steps // 2, dt, temperature, 20.0)
    felis.step(ctx, [leg], steps - steps // 2, dt, temperature, 5.0)
    ctx.device_check()
    sysd.pos = leg.positions()[0].cpu().numpy().astype(np.float32)
    return sysd


def poisson_requests(n, rate, seed, make_system, n_steps, sample_every):
    """n requests with exponential inter-arrival times (mean 1/rate s)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    return [Request(i, float(t[i]), make_system(i), n_steps, sample_every, seed=1000 + i) for i in range(n)]


def served_workload(n_legs=12, rate=2.0, seed=22274, atoms=(5000, 16000), n_steps=300, sample_every=50):
    """Seeded mix of uneven legs: atoms ~ U[atoms], windows ~ {12, 20, 42}."""
    from . import gen
    rng = np.random.default_rng([seed, 4])
    specs = [(int(rng.integers(atoms[0], atoms[1] + 1)), int(rng.choice([12, 20, 42]))) for _ in range(n_legs)]
    systems = [gen.sized_leg(n, w, seed + i) for i, (n, w) in enumerate(specs)]
    return poisson_requests(n_legs, rate, seed, lambda i: systems[i], n_steps, sample_every)


def run_sequential_per_window(ctx, requests, dt=0.002, temperature=300.0, gamma=0.5, mbar_max_iter=5000,
                              clock=time.perf_counter, plain=True):
    """The same legs one at a time, each window on its own launch chain: FIFO,
    a leg starts when it has arrived and the previous one is done.  plain:
    the plain form (FP32 forces summed with FP64 atomics), else the default
    kernels unbatched."""
    import torch
    from . import felis
    beta = 1.0 / (KB * temperature)
    t0 = clock()
    lat, nsw = [], 0.0
    for r in sorted(requests, key=lambda r: r.arrival):
        while clock() - t0 < r.arrival:
            time.sleep(min(0.01, r.arrival - (clock() - t0)))
        s = r.sysd
        W = s.n_windows
        legs = [felis.Leg(ctx, s, windows=[w], seed=r.seed, plain_fp64=plain) for w in range(W)]
        for l in legs:
            felis.build_nlist(ctx, [l], force=True)
        nsamp = r.n_steps // r.sample_every
        u = torch.empty((W, W * nsamp), dtype=torch.float64, device='cuda')
        for k in range(nsamp):
            for w, l in enumerate(legs):
                felis.step(ctx, [l], r.sample_every, dt, temperature, gamma)
                felis.ukn(ctx, l, s.lambdas, l.x, l.y, l.z, beta, out=u[:, k * W + w:k * W + w + 1])
        try:
            felis.mbar(ctx, u, np.full(W, nsamp), max_iter=mbar_max_iter)
        except felis.FelisError as e:
            if e.code != felis.E_NOCONV:
                raise
        ctx.device_check()
        lat.append(clock() - t0 - r.arrival)
        nsw += W * r.n_steps * dt * 1e-3
        del legs, u
        torch.cuda.empty_cache()
    wall = clock() - t0
    return {'form': 'plain, one leg and one window at a time' if plain else 'default kernels, one leg and one '
                    'window at a time', 'wall_s': wall, 'ns_windows_per_day': nsw / (wall / 86400.0),
            'latency_p50_s': percentile(lat, 50), 'latency_p99_s': percentile(lat, 99)}


def main(argv=None):
    """Serve a seeded stream of uneven legs on device 0 and print its
    statistics as one JSON line (atoms ~ U[lo, hi], windows ~ {12, 20, 42},
    Poisson arrivals)."""
    import argparse
    import json
    import multiprocessing as mp

    ap = argparse.ArgumentParser(prog='python -m paper_2603_22274_amd.serve')
    ap.add_argument('--legs', type=int, default=16)
    ap.add_argument('--atoms', type=str, default='5000:80000', help='lo:hi atoms per leg')
    ap.add_argument('--steps', type=int, default=400, help='MD steps per window')
    ap.add_argument('--sample-every', type=int, default=50)
    ap.add_argument('--rate', type=float, default=2.0, help='mean arrivals per second')
    ap.add_argument('--epoch', type=int, default=50, help='MD steps per batched felis_step call')
    ap.add_argument('--hbm-gib', type=float, default=200.0)
    ap.add_argument('--seed', type=int, default=22274)
    ap.add_argument('--pause-s', type=float, default=0.0,
                    help='host idle time between the relaxation and the stream (marks the boundary in a '
                         'kernel trace)')
    ap.add_argument('--procs', type=int, default=8,
                    help='processes generating the legs (1: in this process, e.g. under a profiler)')
    ap.add_argument('--progress', action='store_true',
                    help='print a line to stderr as the legs are built and as each leg finishes')
    a = ap.parse_args(argv)

    def say(msg):
        if a.progress:
            print(msg, file=sys.stderr, flush=True)

    lo, hi = (int(v) for v in a.atoms.split(':'))
    rng = np.random.default_rng([a.seed, 4])
    specs = [(int(rng.integers(lo, hi + 1)), int(rng.choice([12, 20, 42])), a.seed + i) for i in range(a.legs)]
    from . import gen
    if a.procs > 1:
        with mp.get_context('spawn').Pool(a.procs) as p:
            systems = p.starmap(gen.sized_leg, specs, chunksize=1)
    else:
        systems = [gen.sized_leg(*sp) for sp in specs]
    say(f'built {len(systems)} legs')
    from . import felis
    ctx = felis.Context(0)
    for i, s in enumerate(systems):
        relax_start(ctx, s)
        say(f'relaxed leg {i}: {s.n_atoms} atoms, {s.n_windows} windows')
    reqs = poisson_requests(a.legs, a.rate, a.seed, lambda i: systems[i], a.steps, a.sample_every)
    if a.pause_s > 0:
        import torch
        torch.cuda.synchronize()
        time.sleep(a.pause_s)
    last = [0.0]

    def event(e):
        if e['event'] == 'epoch':                   # at most one line every 30 s
            if e['t'] - last[0] >= 30.0:
                last[0] = e['t']
                say(f"{e['t']:.1f} s: {e['active']} legs stepping")
        elif e['event'] != 'admit':
            say(f"{e['t']:.1f} s: {e['event']} leg {e['rid']}")

    srv = Server(FelisEngine(ctx, mbar_max_iter=5000), hbm_budget=int(a.hbm_gib * (1 << 30)),
                 epoch_steps=a.epoch, on_event=event)
    out, stats = srv.serve(reqs)
    stats["legs_ok"] = sum(1 for r in out if r.status == 'ok')
    stats["not_ok"] = [{"leg": r.rid, "atoms": r.atoms, "windows": r.windows, "status": str(r.status)[:300]}
                       for r in out if r.status != 'ok']
    stats["events"] = [e for e in srv.log if e.get('event') in ('retry', 'evict')]
    stats["atoms"] = [s.n_atoms for s in systems]
    stats["windows"] = [s.n_windows for s in systems]
    print(json.dumps(stats), flush=True)
    ctx.close()


if __name__ == '__main__':
    main()
