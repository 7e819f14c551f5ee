"""Scheduling logic of the served, continuously batched form, driven by a CPU
engine that only keeps books (no kernels): admission by memory, first come
first served, continuous joining at epoch boundaries, eviction of a failing
leg without disturbing the others, latency and throughput accounting."""
import math
import types

import numpy as np
import pytest

from paper_2603_22274_amd.serve import LegFailed, Request, Server, percentile


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, d):
        self.t += max(d, 1e-9)


class BookEngine:
    """Costs one unit of time per window-step plus a fixed launch cost per epoch."""

    def __init__(self, clock, budget, launch=0.01, per_window_step=1e-4, fail=None):
        self.clock, self.budget = clock, budget
        self.launch, self.per = launch, per_window_step
        self.live = {}
        self.batches = []
        self.samples = {}
        self.finished = []
        self.fail = fail or {}          # rid -> (epoch index, 'cap' | 'overflow')
        self.epochs = 0

    def footprint(self, r):
        return r.sysd.n_atoms * r.sysd.n_windows

    def admit(self, r):
        h = types.SimpleNamespace(r=r)
        self.live[id(h)] = self.footprint(r)
        assert sum(self.live.values()) <= self.budget
        self.samples[r.rid] = 0
        return h

    def run_epoch(self, handles, n):
        self.batches.append(sorted(h.r.rid for h in handles))
        self.clock.t += self.launch + self.per * n * sum(h.r.sysd.n_windows for h in handles)
        bad = {}
        for h in handles:
            kind = self.fail.get(h.r.rid, (None, None))
            if kind[0] == self.epochs:
                bad[id(h)] = LegFailed('capacity', 100) if kind[1] == 'cap' else LegFailed('overflow')
            if h.r.list_cap and h.r.list_cap < 100:
                bad[id(h)] = LegFailed('capacity', 100)
        self.epochs += 1
        return bad

    def sample(self, h):
        self.samples[h.r.rid] += 1

    def finish(self, h):
        self.finished.append(h.r.rid)
        return 0.1 * h.r.rid, 7, True

    def release(self, h):
        del self.live[id(h)]


def req(rid, t, atoms, windows, steps=200, every=50):
    return Request(rid, t, types.SimpleNamespace(n_atoms=atoms, n_windows=windows), steps, every)


def run(reqs, budget, **kw):
    clk = Clock()
    eng = BookEngine(clk, budget, **kw)
    srv = Server(eng, budget, epoch_steps=50, clock=clk, sleep=clk.sleep)
    out, stats = srv.serve(reqs)
    return eng, srv, out, stats


def test_budget_and_first_come_first_served():
    reqs = [req(i, 0.01 * i, 1000, 10) for i in range(6)]
    eng, srv, out, stats = run(reqs, budget=2 * 10000)
    assert all(r.status == 'ok' for r in out)
    assert max(len(b) for b in eng.batches) == 2          # never more than the budget holds
    admits = [e['rid'] for e in srv.log if e['event'] == 'admit']
    assert admits == list(range(6))
    assert all(e['used'] <= 20000 for e in srv.log if e['event'] == 'admit')
    assert eng.live == {}
    assert all(eng.samples[i] == 4 for i in range(6))
    assert sorted(eng.finished) == list(range(6))
    for r in out:
        assert r.arrival <= r.admitted <= r.finished
        assert r.steps == 200 and r.dG == pytest.approx(0.1 * r.rid)


def test_continuous_joining():
    # a long leg is running when a short one arrives: the short one joins at
    # the next epoch boundary and leaves first
    reqs = [req(0, 0.0, 1000, 20, steps=1000), req(1, 0.05, 1000, 10, steps=100)]
    eng, srv, out, stats = run(reqs, budget=10 ** 9)
    assert eng.batches[0] == [0]
    assert [0, 1] in eng.batches
    assert out[1].finished < out[0].finished
    assert out[1].admitted < out[0].finished
    assert eng.batches[-1] == [0]


def test_head_of_line_waits_for_memory():
    # a big leg blocks later small ones (first come first served), then all run
    reqs = [req(0, 0.0, 1000, 10), req(1, 0.001, 3000, 10), req(2, 0.002, 100, 10)]
    eng, srv, out, stats = run(reqs, budget=35000)
    admits = [e['rid'] for e in srv.log if e['event'] == 'admit']
    assert admits == [0, 1, 2]
    assert all(r.status == 'ok' for r in out)


def test_oversize_rejected():
    reqs = [req(0, 0.0, 1000, 10), req(1, 0.0, 10 ** 6, 10), req(2, 0.1, 1000, 10)]
    eng, srv, out, stats = run(reqs, budget=50000)
    assert out[1].status.startswith('rejected')
    assert out[0].status == 'ok' and out[2].status == 'ok'
    assert stats['completed'] == 2


def test_eviction_isolates_failing_leg():
    reqs = [req(i, 0.0, 1000, 10) for i in range(3)]
    eng, srv, out, stats = run(reqs, budget=10 ** 9, fail={1: (1, 'overflow')})
    assert out[1].status.startswith('evicted')
    assert out[0].status == 'ok' and out[2].status == 'ok'
    assert eng.samples[1] == 1                 # sampled after epoch 0 only
    assert eng.live == {}
    assert 1 not in eng.finished
    assert all(1 not in b for b in eng.batches[2:])


def test_idle_gaps_and_accounting():
    reqs = [req(0, 0.0, 1000, 10, steps=100), req(1, 5.0, 1000, 10, steps=100)]
    eng, srv, out, stats = run(reqs, budget=10 ** 9)
    per_leg = 2 * (0.01 + 1e-4 * 50 * 10)
    assert out[0].latency == pytest.approx(per_leg)
    assert out[1].admitted == pytest.approx(5.0, abs=1e-6)
    assert out[1].latency == pytest.approx(per_leg, abs=1e-6)
    nsw = 2 * 10 * 100 * 0.002e-3
    assert stats['ns_windows_per_day'] == pytest.approx(nsw / (stats['wall_s'] / 86400.0))
    assert stats['latency_p50_s'] == pytest.approx(per_leg, abs=1e-6)


def test_epoch_multiple_required():
    with pytest.raises(ValueError):
        run([req(0, 0.0, 10, 2, steps=120)], budget=10 ** 9)


@pytest.mark.parametrize('n', [1, 2, 7, 100])
def test_percentile_matches_linear_interpolation(n):
    v = list(np.random.default_rng(n).exponential(1.0, n))
    for q in (0, 50, 99, 100):
        assert percentile(v, q) == pytest.approx(float(np.percentile(v, q)))
    assert math.isnan(percentile([], 50))


def test_capacity_failure_requeued_with_larger_list():
    reqs = [req(0, 0.0, 1000, 10), req(1, 0.0, 1000, 10), req(2, 0.5, 1000, 10)]
    reqs[1].list_cap = 16
    eng, srv, out, stats = run(reqs, budget=10 ** 9)
    assert [r.status for r in out] == ['ok'] * 3
    assert out[1].retries == 1
    retry = [e for e in srv.log if e['event'] == 'retry']
    assert retry == [{'t': retry[0]['t'], 'event': 'retry', 'rid': 1, 'list_cap': 200}]
    assert out[1].steps == 200 and eng.samples[1] == 4       # counted afresh after the retry
    assert eng.live == {}


def test_capacity_failure_evicted_when_retries_spent():
    reqs = [req(0, 0.0, 1000, 10), req(1, 0.0, 1000, 10)]
    clk = Clock()
    eng = BookEngine(clk, 10 ** 9, fail={1: (0, 'cap')})
    srv = Server(eng, 10 ** 9, epoch_steps=50, max_retries=0, clock=clk, sleep=clk.sleep)
    out, stats = srv.serve(reqs)
    assert out[0].status == 'ok' and out[1].status.startswith('evicted')


def test_events_reported_as_they_happen():
    # the on_event hook sees every log entry when it is made, plus one
    # 'epoch' entry per batched epoch (with the number of legs stepping)
    clk = Clock()
    eng = BookEngine(clk, 10 ** 9, fail={0: (1, 'overflow')})
    seen = []
    srv = Server(eng, 10 ** 9, epoch_steps=50, clock=clk, sleep=clk.sleep, on_event=seen.append)
    out, stats = srv.serve([req(0, 0.0, 1000, 10), req(1, 0.05, 1000, 10), req(2, 0.1, 1000, 10)])
    logged = [e for e in seen if e['event'] != 'epoch']
    assert logged == srv.log
    epochs = [e for e in seen if e['event'] == 'epoch']
    assert len(epochs) == len(eng.batches)
    assert [e['active'] for e in epochs] == [len(b) for b in eng.batches]
    assert [e['t'] for e in seen] == sorted(e['t'] for e in seen)
    assert {e['event'] for e in logged} == {'admit', 'finish', 'evict'}
