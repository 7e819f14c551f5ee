"""Summaries of rocprofv3 output databases (kernel traces and PMC counters).

    python -m paper_2603_22274_amd.profiling stats <trace_dir> [n]
    python -m paper_2603_22274_amd.profiling traffic <fetch_dir> <write_dir> <kernel-substring>
    python -m paper_2603_22274_amd.profiling counters <pmc_dir> <kernel-substring> ...

``stats`` prints per-kernel call counts, average and total durations.
``traffic`` scales the FETCH_SIZE / WRITE_SIZE counters (KiB per dispatch)
of one kernel by what the same counters read for the largest plain device
copy in the run (bytes actually moved / bytes counted), and prints the
per-launch HBM traffic as JSON.
"""
from __future__ import annotations

import glob
import json
import sqlite3
import sys


def _db(d):
    hits = glob.glob(d.rstrip('/') + '/*results.db')
    if not hits:
        raise FileNotFoundError(f"no rocprofv3 database under {d}")
    return sqlite3.connect(hits[0])


def short(name):
    n = name.replace('felis::(anonymous namespace)::', '')
    return n.split('(felis::')[0].split('(double const')[0].split('(long long')[0].strip()


def kernel_stats(trace_dir, top=25):
    con = _db(trace_dir)
    rows = con.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    out = [f"{'kernel':44s} {'calls':>7s} {'avg_us':>10s} {'total_ms':>10s} {'pct':>6s}"]
    for name, n, tot, avg, pct in rows[:top]:      # the view reports microseconds
        out.append(f"{short(name)[:44]:44s} {n:7d} {avg:10.2f} {tot / 1e3:10.3f} {pct:6.1f}")
    return "\n".join(out)


def _counter(con, kernel_sub):
    vals = [v for (n, v) in con.execute("select kernel_name, value from counters_collection")
            if kernel_sub in n]
    return sum(vals) / len(vals) if vals else None, len(vals)


def _copy_reference(con):
    r = con.execute("select grid_size, value from counters_collection where kernel_name like '%copyBuffer%' "
                    "order by value desc limit 1").fetchone()
    return r


def traffic(fetch_dir, write_dir, kernel_sub, copy_bytes=256 << 20):
    cf, cw = _db(fetch_dir), _db(write_dir)
    f_kib, nf = _counter(cf, kernel_sub)
    w_kib, nw = _counter(cw, kernel_sub)
    f_copy = _copy_reference(cf)[1]
    w_copy = _copy_reference(cw)[1]
    f_scale = copy_bytes / (f_copy * 1024.0)
    w_scale = copy_bytes / (w_copy * 1024.0)
    fetch = f_kib * 1024.0 * f_scale
    write = w_kib * 1024.0 * w_scale
    return {"kernel": kernel_sub, "dispatches": [nf, nw],
            "fetch_kib_per_dispatch": f_kib, "write_kib_per_dispatch": w_kib,
            "copy_reference": {"bytes": copy_bytes, "fetch_kib": f_copy, "write_kib": w_copy,
                               "fetch_scale": f_scale, "write_scale": w_scale},
            "fetch_bytes_per_launch": fetch, "write_bytes_per_launch": write,
            "bytes_per_launch": fetch + write}


def counters(pmc_dir, kernels):
    """Per-dispatch averages of every counter collected in ``pmc_dir`` for the
    kernels whose names contain one of ``kernels``."""
    con = _db(pmc_dir)
    rows = con.execute("select kernel_name, counter_name, value from counters_collection").fetchall()
    out = {}
    for name, cname, v in rows:
        for k in kernels:
            if k in name:
                out.setdefault(k, {}).setdefault(cname, []).append(v)
    return {k: {c: sum(v) / len(v) for c, v in d.items()} for k, d in out.items()}


if __name__ == '__main__':
    if sys.argv[1] == 'stats':
        print(kernel_stats(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 25))
    elif sys.argv[1] == 'counters':
        print(json.dumps(counters(sys.argv[2], sys.argv[3:]), indent=1))
    elif sys.argv[1] == 'traffic':
        print(json.dumps(traffic(sys.argv[2], sys.argv[3], sys.argv[4]), indent=1))
