"""Runs K-applies of one grid for profiler runs (rocprofv3 kernel traces and
HBM counters), plus a device copy of known size that calibrates the
FETCH_SIZE / WRITE_SIZE counters.

    python -m paper_2502_04217_amd.profile_kapply --grid 256 --reps 10 --precision fp32

Prints one JSON line with the per-kernel event timings (ms), the
algorithmic bytes of each kernel, and the time of a whole K-apply among
applies back to back (replayed from a HIP graph, and launched directly).
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import csipm
from . import workload as wl

PASS_NAMES = ["axis1_inverse", "axis2_inverse", "axis3_c2r_mask_r2c", "axis2_forward", "axis1_forward_K_epilogue"]


def pass_bytes(shape, w):
    """Algorithmic HBM bytes of each K-apply kernel (w = word size): every
    volume pass reads and writes the n-real work array once; the axis-3 pass
    also reads the n-bit mask; the last pass also reads p_beta, p_z, Sigma_1,
    Sigma_2 and writes q_beta, q_z instead of the work array.  Sum:
    15 n w + n/8.  (The m = 0 plane's mirror rows, re-read by the axis-1
    inverse pass, are not algorithmic bytes.)"""
    n1, n2, n3 = shape
    n = n1 * n2 * n3
    return [2 * n * w, 2 * n * w, 2 * n * w + n // 8, 2 * n * w, 7 * n * w]


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--precision", choices=["fp32", "fp64", "both"], default="both")
    ap.add_argument("--copy-mib", type=int, default=1024)
    a = ap.parse_args(argv)
    import torch
    shape = (a.grid,) * 3
    rng = np.random.default_rng(0)
    obs = wl.lattice_cube_mask(shape, 3, 32) if a.grid % 32 == 0 else np.zeros(shape, bool)
    pr = csipm.Problem(rng.standard_normal(shape), (~obs).astype(np.uint8))
    s1, s2 = wl.random_barrier(shape, 1, spread=3.0)
    pr.set_barrier(torch.tensor(s1, device="cuda"), torch.tensor(s2, device="cuda"))
    out = {"grid": shape}
    precs = {"fp32": (csipm.FP32, 4), "fp64": (csipm.FP64, 8)}
    for name in (["fp32", "fp64"] if a.precision == "both" else [a.precision]):
        p, w = precs[name]
        pr.profile_kapply(p, 2)                       # warm-up
        ms, whole, launched = pr.profile_kapply_all(p, a.reps)
        by = pass_bytes(shape, w)
        out[name] = {k: {"ms": m, "bytes": b, "GBps": b / (m * 1e-3) / 1e9} for k, m, b in zip(PASS_NAMES, ms, by)}
        out[name]["kapply_back_to_back"] = {"ms": whole, "bytes": sum(by), "GBps": sum(by) / (whole * 1e-3) / 1e9}
        out[name]["kapply_launched_directly"] = {"ms": launched, "GBps": sum(by) / (launched * 1e-3) / 1e9}
    # counter calibration: a fill that writes copy_mib MiB and a sum that
    # reads them once (FETCH_SIZE / WRITE_SIZE of these two kernels against
    # the known byte counts give the scale factors)
    nbytes = a.copy_mib * 1024 * 1024
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    s = x.sum()
    torch.cuda.synchronize()
    out["calibration_bytes"] = nbytes
    out["calibration_sum"] = float(s)
    # achievable device-to-device copy bandwidth (read + write), for context
    y = torch.empty_like(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    y.copy_(x)
    e0.record()
    for _ in range(5):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    out["copy_GBps"] = 2 * nbytes * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    sys.exit(main())
