"""Throughput of many small independent solves: one after another against
csipm_solve_batch (each problem on its own stream, solves on a pool of host
threads) and against csipm_solve_small_batch (one kernel, one workgroup per
problem).  The paper's synthetic problem at a small grid, seeds
0..count-1.

    python -m paper_2502_04217_amd.batch_throughput [--grid 16] [--count 64] [--threads 1 2 4 8]

Prints one JSON line per configuration: solves per second and the speed-up
over the sequential loop.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

from . import csipm
from . import workload as wl


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--grid", type=int, default=16)
    ap.add_argument("--count", type=int, default=64)
    ap.add_argument("--threads", type=int, nargs="+", default=[1, 2, 4, 8])
    ap.add_argument("--tol", type=float, default=1e-8)
    a = ap.parse_args(argv)
    import torch
    probs = []
    for seed in range(a.count):
        w = wl.paper_synthetic(a.grid, seed)
        pr = csipm.Problem(w.signal, w.observed, stream=torch.cuda.Stream())
        pr.lambda_rule(0.05)
        probs.append(pr)
    for pr in probs[:4]:
        pr.solve(tol=a.tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for pr in probs:
        pr.solve(tol=a.tol)
    torch.cuda.synchronize()
    seq = time.perf_counter() - t0
    print(json.dumps({"grid": a.grid, "count": a.count, "mode": "sequential", "seconds": seq,
                      "solves_per_s": a.count / seq}), flush=True)
    for nt in a.threads:
        csipm.solve_batch(probs[:4], tol=a.tol, max_threads=nt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        infos = csipm.solve_batch(probs, tol=a.tol, max_threads=nt)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ok = all(i["status"] >= 0 for i in infos)
        print(json.dumps({"grid": a.grid, "count": a.count, "mode": "batch", "threads": nt, "seconds": dt,
                          "solves_per_s": a.count / dt, "speedup": seq / dt, "all_ok": ok}), flush=True)
    # one launch: the same problems in one kernel (signals and masks already
    # on the device, as for the contexts above)
    import numpy as np
    ws = [wl.paper_synthetic(a.grid, seed) for seed in range(a.count)]
    sig = torch.tensor(np.stack([w.signal for w in ws]), device="cuda")
    obs = torch.tensor(np.stack([w.observed for w in ws]).astype(np.uint8), device="cuda")
    csipm.solve_small_batch(sig, obs, lambda_frac=0.05, tol=a.tol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    beta, info = csipm.solve_small_batch(sig, obs, lambda_frac=0.05, tol=a.tol)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(json.dumps({"grid": a.grid, "count": a.count, "mode": "one_launch", "seconds": dt,
                      "solves_per_s": a.count / dt, "speedup": seq / dt, "all_ok": bool((info[:, 0] == 0).all()),
                      "ipm_iters_mean": float(info[:, 1].mean()), "pcg_iters_mean": float(info[:, 2].mean())}),
          flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
