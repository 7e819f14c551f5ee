"""Host logic of the kernel-trace summaries on a hand-built trace database:
per-step device time, busy and idle time, and the whole-run queue and host
gaps, and the per-dispatch counter averages of a kernel's workload launches
(no GPU, no profiler)."""
import sqlite3

import pytest

from paper_2603_22274_amd import profiling


def _trace(tmp_path, rows):
    d = tmp_path / 'trace'
    d.mkdir()
    con = sqlite3.connect(str(d / 'run_results.db'))
    con.execute("create table kernels (name text, start integer, end integer)")
    con.executemany("insert into kernels values (?, ?, ?)", rows)
    con.commit()
    con.close()
    return str(d)


def test_union_of_intervals():
    assert profiling._union([]) == 0
    assert profiling._union([(0, 10), (5, 15), (20, 30)]) == 25
    assert profiling._union([(20, 30), (0, 10), (10, 12)]) == 22


def test_step_breakdown_busy_and_idle(tmp_path):
    us = 1000            # ns per microsecond
    rows = []
    # three steps of 100 us; in each: pairs 0-60, a side kernel 10-50 (overlapping), integrate 70-80
    for k in range(3):
        t = k * 100 * us
        rows += [("void felis::k_pairs<0>(...)", t, t + 60 * us),
                 ("felis::k_spread(...)", t + 10 * us, t + 50 * us),
                 ("felis::k_integrate(...)", t + 70 * us, t + 80 * us)]
    rows.append(("void felis::k_pairs<0>(...)", 300 * us, 360 * us))
    b = profiling.step_breakdown(_trace(tmp_path, rows))
    assert b['steps'] == 3
    assert b['wall_us_per_step'] == pytest.approx(100.0)
    assert b['busy_us_per_step'] == pytest.approx(70.0)        # union: 0-60 and 70-80
    assert b['idle_us_per_step'] == pytest.approx(30.0)
    assert b['kernel_sum_us_per_step'] == pytest.approx(110.0)
    assert b['kernels']['k_pairs<0>']['us_per_step'] == pytest.approx(60.0)
    assert b['kernels']['k_spread']['launches_per_step'] == pytest.approx(1.0)


def test_timeline_splits_queue_and_host_gaps(tmp_path):
    us = 1000
    rows = [("felis::k_prep(...)", 0, 10 * us)]                 # before a 5 ms pause: excluded below
    t = 5010 * us
    for k in range(4):                                           # 4 steps: 50 us pair + 5 us gap + 20 us kernel
        rows += [("void felis::k_pairs<0>(...)", t, t + 50 * us),
                 ("felis::k_integrate(...)", t + 55 * us, t + 75 * us)]
        t += 75 * us + (500 * us if k == 1 else 5 * us)          # one 500 us host gap after step 2
    d = _trace(tmp_path, rows)
    tl = profiling.timeline(d, host_gap_us=100.0, after_gap_ms=1.0)
    assert tl['md_steps'] == 4
    assert tl['host_gaps'] == 1
    assert tl['host_gaps_us_per_md_step'] == pytest.approx(500.0 / 4)
    # the span ends with the last pair launch: 3 gaps of 5 us inside steps, 2 of 5 us between them
    assert tl['queue_gaps_us_per_md_step'] == pytest.approx((3 * 5.0 + 2 * 5.0) / 4)
    whole = profiling.timeline(d)
    assert whole['md_steps'] == 4                                 # k_prep comes before the first pair launch


def test_counters_take_the_workload_launches(tmp_path):
    # per-dispatch counter averages over a kernel's largest-grid launches only,
    # and the FFT passes of the step told apart from the u_kn ones by their
    # line count (the third template argument)
    d = tmp_path / 'pmc'
    d.mkdir()
    con = sqlite3.connect(str(d / 'run_results.db'))
    con.execute("create table counters_collection (kernel_name text, grid_size integer, counter_name text, "
                "value real)")
    rows = [("void felis::k_fft<1, 0, 32>(...)", 6048, "SQ_INSTS_VALU", 100.0),
            ("void felis::k_fft<1, 0, 32>(...)", 6048, "SQ_INSTS_VALU", 120.0),
            ("void felis::k_fft<1, 0, 32>(...)", 288, "SQ_INSTS_VALU", 5.0),       # a one-window launch
            ("void felis::k_fft<1, 0, 16>(...)", 24192, "SQ_INSTS_VALU", 900.0),   # u_kn, more workgroups
            ("void felis::k_pairs<0>(...)", 92568, "SQ_INSTS_VALU", 7.0)]
    con.executemany("insert into counters_collection values (?, ?, ?, ?)", rows)
    con.commit()
    con.close()
    c = profiling.counters(str(d), ['k_fft<1, 0, 32>', 'k_pairs<0>'])
    assert c['k_fft<1, 0, 32>']['SQ_INSTS_VALU'] == pytest.approx(110.0)
    assert c['k_pairs<0>']['SQ_INSTS_VALU'] == pytest.approx(7.0)
    # a prefix without the line count would have picked the u_kn launches
    assert profiling.counters(str(d), ['k_fft<1, 0'])['k_fft<1, 0']['SQ_INSTS_VALU'] == pytest.approx(900.0)
