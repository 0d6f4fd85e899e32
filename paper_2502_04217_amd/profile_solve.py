"""Runs interior-point solves of one seeded workload for profiler runs
(rocprofv3 kernel traces and FETCH_SIZE / WRITE_SIZE counter passes), then a
1 GiB fill and a 1 GiB sum that calibrate the two counters.

    python -m paper_2502_04217_amd.profile_solve --grid 256 --form chosen

`chosen` is the FP32 form with the learned correction when trained parameters
exist (the form bench.py times), `fp64` the plain FP64 form.  Prints one JSON
line with the solve summaries.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

from . import csipm
from . import workload as wl

PARAMS_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pc_params.json")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--grid", type=int, default=256, choices=[16, 64, 128, 256, 512])
    ap.add_argument("--form", choices=["chosen", "fp64", "both"], default="both")
    ap.add_argument("--solves", type=int, default=1)
    ap.add_argument("--calib-mib", type=int, default=1024)
    a = ap.parse_args(argv)
    import torch
    w = {16: lambda: wl.grid16(1), 64: lambda: wl.grid64(1), 128: lambda: wl.grid128_family(10000),
         256: lambda: wl.grid256(1), 512: lambda: wl.grid512(1)}[a.grid]()
    pr = csipm.Problem(w.signal, w.observed)
    pr.lambda_rule(0.05)
    learned = os.path.exists(PARAMS_FILE)
    if learned:
        with open(PARAMS_FILE) as f:
            pr.set_pc_params(torch.tensor(json.load(f)["params"], dtype=torch.float32, device="cuda"))
    forms = {"chosen": dict(tol=1e-6, precision=csipm.FP32, pc=csipm.PC_LEARNED if learned else csipm.PC_PLAIN),
             "fp64": dict(tol=1e-6, precision=csipm.FP64, pc=csipm.PC_PLAIN)}
    out = {"workload": w.name}
    for name in (["chosen", "fp64"] if a.form == "both" else [a.form]):
        infos = [pr.solve(**forms[name]) for _ in range(a.solves)]
        out[name] = {k: infos[-1][k] for k in ("ipm_iters", "cg_iters_total", "refine_steps_total", "rel_kkt")}
    nbytes = a.calib_mib * 1024 * 1024
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    out["calibration_bytes"] = nbytes
    out["calibration_sum"] = float(x.sum())
    torch.cuda.synchronize()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
