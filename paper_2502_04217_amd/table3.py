"""Time-to-solve on the paper's artificial test problem (section "Synthetic
Dataset", table "tab:cpu_gpu_comparison_artificial") at the grid sizes of
that table, for a table beside it.

    python -m paper_2502_04217_amd.table3 [--sizes 8 16 32 64 96 128 192 256 384 512 560] [--tol 1e-8] [--reps 3]

Each size: the workload of workload.paper_synthetic, lambda = 0.05 ||M^T b||_inf,
solved to rel_kkt <= tol (the paper stops at a primal-dual residual of 1e-8)
in the paper's form (FP64, P) and in the FP32 form with the learned
correction when trained parameters exist; median of `reps` timed solves after
one warm-up, inputs resident on the device.  The paper's GH200 times are
printed beside as context (other hardware, Julia/MadNLP, unstated lambda and
missing pattern).
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

from . import csipm
from . import workload as wl

# GPU seconds of the paper's table for the same grid sizes (GH200)
PAPER_GPU_S = {8: 0.63, 16: 0.72, 32: 0.68, 64: 0.71, 96: 0.79, 128: 1.07, 192: 3.22, 256: 5.88, 384: 20.66,
               512: 104.55, 560: 159.66}
PARAMS_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pc_params.json")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", type=int, nargs="+", default=[8, 16, 32, 64, 96, 128, 192, 256, 384, 512, 560])
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args(argv)
    import torch
    params = None
    if os.path.exists(PARAMS_FILE):
        with open(PARAMS_FILE) as f:
            params = torch.tensor(json.load(f)["params"], dtype=torch.float32, device="cuda")
    forms = {"fp64_plain": dict(precision=csipm.FP64, pc=csipm.PC_PLAIN),
             "fp32_plain": dict(precision=csipm.FP32, pc=csipm.PC_PLAIN)}
    if params is not None:
        forms["fp32_learned"] = dict(precision=csipm.FP32, pc=csipm.PC_LEARNED)
    rows = []
    for N in a.sizes:
        w = wl.paper_synthetic(N)
        pr = csipm.Problem(w.signal, w.observed)
        pr.lambda_rule(0.05)
        if params is not None:
            pr.set_pc_params(params)
        row = {"N": N, "variables": 2 * w.n, "missing": round(w.missing_fraction, 4),
               "paper_gh200_s": PAPER_GPU_S.get(N)}
        for name, f in forms.items():
            pr.solve(tol=a.tol, **f)
            times, info = [], None
            for _ in range(a.reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = pr.solve(tol=a.tol, **f)
                torch.cuda.synchronize()
                times.append(time.perf_counter() - t0)
            row[name] = {"s": statistics.median(times), "ipm": info["ipm_iters"], "cg": info["cg_iters_total"],
                         "rel_kkt": info["rel_kkt"], "status": info["status_name"]}
        print(json.dumps(row), flush=True)
        rows.append(row)
        del pr
        torch.cuda.empty_cache()
    print("| N | variables | missing | paper GH200 (s) | FP64, P (s) | IPM / PCG | FP32 + learned (s) | IPM / PCG |")
    print("|---|---|---|---|---|---|---|---|")
    for r in rows:
        c = r.get("fp32_learned", r["fp32_plain"])
        print(f"| {r['N']}³ | {r['variables']:,} | {r['missing']:.3f} | {r['paper_gh200_s']} | "
              f"{r['fp64_plain']['s']:.4f} | {r['fp64_plain']['ipm']} / {r['fp64_plain']['cg']} | "
              f"{c['s']:.4f} | {c['ipm']} / {c['cg']} |")
    return 0


if __name__ == "__main__":
    sys.exit(main())
