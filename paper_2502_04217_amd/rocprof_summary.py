"""Summarises a rocprofv3 result database (rocpd SQLite): per-kernel dispatch
count, total and average duration, and the average over "working" dispatches
only (longer than --min-us; Krylov iterations are queued ahead in batches and
the ones past convergence return at once, in a few microseconds), plus the
per-dispatch mean of any collected counters (FETCH_SIZE, WRITE_SIZE in KiB).

    python -m paper_2502_04217_amd.rocprof_summary prof/x_results.db [--top 25] [--min-us 8]
"""
from __future__ import annotations

import argparse
import collections
import re
import sqlite3
import sys


def short(name: str) -> str:
    name = re.sub(r"\(anonymous namespace\)::", "", name)
    name = re.sub(r"(csipm|fftk)::", "", name)
    m = re.match(r"(void )?([A-Za-z_0-9]+(<[^()]*>)?)", name)
    return m.group(2) if m else name[:80]


def summarize(db: str, top: int = 25, min_us: float = 8.0):
    c = sqlite3.connect(db)
    rows = c.execute("select name, duration from kernels").fetchall()
    agg = collections.OrderedDict()
    for name, dur in rows:
        k = short(name)
        a = agg.setdefault(k, [0, 0.0, 0, 0.0])
        a[0] += 1
        a[1] += dur
        if dur >= min_us * 1e3:
            a[2] += 1
            a[3] += dur
    total = sum(a[1] for a in agg.values()) or 1.0
    out = []
    for k, (n, t, nw, tw) in sorted(agg.items(), key=lambda kv: -kv[1][1])[:top]:
        out.append({"kernel": k, "calls": n, "total_us": t / 1e3, "avg_us": t / n / 1e3, "pct": 100 * t / total,
                    "working_calls": nw, "working_avg_us": (tw / nw / 1e3) if nw else 0.0})
    ctr = collections.defaultdict(lambda: collections.defaultdict(list))
    try:
        for kname, cname, val in c.execute("select kernel_name, counter_name, value from counters_collection"):
            ctr[short(kname)][cname].append(val)
    except sqlite3.Error:
        pass
    counters = {k: {cn: {"dispatches": len(v), "mean": sum(v) / len(v)} for cn, v in d.items()}
                for k, d in ctr.items()}
    return out, counters, total / 1e3


def calibrated_traffic(fetch_db: str, write_db: str, calib_bytes: int, working_frac: float = 0.1):
    """Per-kernel HBM bytes per working dispatch from a FETCH_SIZE run and a
    WRITE_SIZE run (KiB per dispatch), each scaled by what the counter reads
    for a kernel of known traffic in the same run: the reduction (torch sum,
    reads calib_bytes) for FETCH_SIZE and the fill (writes calib_bytes) for
    WRITE_SIZE.  A dispatch counts as working when its counter reaches
    working_frac of that kernel's largest dispatch (the Krylov launches queued
    past convergence return at once and read only a flag).
    Returns ({kernel: (fetch_bytes, write_bytes)}, factors)."""
    def per_dispatch(db, counter):
        c = sqlite3.connect(db)
        rows = c.execute("select kernel_name, value from counters_collection where counter_name = ?",
                         (counter,)).fetchall()
        d = collections.defaultdict(list)
        for k, v in rows:
            d[k].append(v)
        return d
    f = per_dispatch(fetch_db, "FETCH_SIZE")
    w = per_dispatch(write_db, "WRITE_SIZE")
    red = [max(v) for k, v in f.items() if "reduce_kernel" in k]
    fill = [max(v) for k, v in w.items() if "FillFunctor" in k]
    ff = calib_bytes / 1024.0 / max(red) if red else 1.0
    fw = calib_bytes / 1024.0 / max(fill) if fill else 1.0
    def working_mean(v):
        if not v:
            return 0.0
        top = max(v)
        keep = [x for x in v if x >= working_frac * top]
        return sum(keep) / len(keep)
    out = {}
    for k in set(f) | set(w):
        out[short(k)] = (working_mean(f.get(k, [])) * 1024.0 * ff, working_mean(w.get(k, [])) * 1024.0 * fw)
    return out, (ff, fw)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("db")
    ap.add_argument("--top", type=int, default=25)
    ap.add_argument("--min-us", type=float, default=8.0)
    ap.add_argument("--fetch-db")
    ap.add_argument("--write-db")
    ap.add_argument("--calib-bytes", type=int, default=1 << 30)
    ap.add_argument("--record", nargs=3, metavar=("KERNEL", "NAME", "GRID"), action="append", default=[],
                    help="(repeatable) "
                         "print a traffic-record line for the rocprof kernel KERNEL (short name), timed as NAME "
                         "by csipm_timing, at GRID^3, stamped with the current kernel-source digest")
    ap.add_argument("--record-group", nargs="+", metavar="ARG", action="append", default=[],
                    help="(repeatable) "
                         "NAME GRID KERNEL [KERNEL ...]: a traffic-record line for the sum of one working "
                         "dispatch of each listed rocprof kernel (short names), e.g. the kernels of one K-apply")
    a = ap.parse_args(argv)
    if a.fetch_db and a.write_db:
        tr, (ff, fw) = calibrated_traffic(a.fetch_db, a.write_db, a.calib_bytes)
        print(f"# calibrated HBM traffic per working dispatch (FETCH_SIZE x {ff:.4f}, WRITE_SIZE x {fw:.4f})")
        for k in sorted(tr):
            fe, wr = tr[k]
            if fe + wr > 1e6:
                print(f"{k[:60]:60s} read {fe / 1e6:10.2f} MB  write {wr / 1e6:10.2f} MB")
        import json
        from .build import source_digest
        digest = source_digest()
        for kern, name, grid in a.record:
            fe, wr = tr[kern]
            print("traffic-record: " + json.dumps({"kernel": name, "rocprof_kernel": kern, "grid": int(grid),
                                                   "read_bytes": round(fe), "write_bytes": round(wr),
                                                   "fetch_factor": round(ff, 4), "write_factor": round(fw, 4),
                                                   "source_sha256": digest}))
        for group in a.record_group:
            name, grid, kerns = group[0], group[1], group[2:]
            fe = sum(tr[k][0] for k in kerns)
            wr = sum(tr[k][1] for k in kerns)
            print("traffic-record: " + json.dumps({"kernel": name, "rocprof_kernels": kerns, "grid": int(grid),
                                                   "read_bytes": round(fe), "write_bytes": round(wr),
                                                   "fetch_factor": round(ff, 4), "write_factor": round(fw, 4),
                                                   "source_sha256": digest}))
    out, counters, total_us = summarize(a.db, a.top, a.min_us)
    print(f"# kernel time total {total_us:.1f} us; working = dispatches >= {a.min_us} us")
    print(f"{'kernel':60s} {'calls':>6s} {'total_us':>11s} {'avg_us':>9s} {'pct':>6s} {'work':>5s} {'work_avg_us':>11s}")
    for r in out:
        print(f"{r['kernel'][:60]:60s} {r['calls']:6d} {r['total_us']:11.1f} {r['avg_us']:9.2f} {r['pct']:6.2f} "
              f"{r['working_calls']:5d} {r['working_avg_us']:11.2f}")
    if counters:
        print("# counters (mean per dispatch)")
        for k, d in counters.items():
            for cn, v in d.items():
                print(f"{k[:60]:60s} {cn:12s} n={v['dispatches']:5d} mean={v['mean']:.1f}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
