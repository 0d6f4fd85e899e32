#!/usr/bin/env python3
"""Time-to-solve benchmark of the sparse-3D-DFT interior-point solver on one
MI355X.

Workload: 256^3 crystal-like grid (0.1% of DFT bins nonzero with
N(0,1) exp(-|k|/32) amplitudes, SNR 10 dB, cubes of half-width 3 removed on a
period-32 lattice plus 2% uniform dropouts, lambda = 0.05 ||M_perp^T b||_inf),
seeded synthetic data.  A step is one complete interior-point solve to
relative KKT residual 1e-6 (csipm_solve: residuals, Newton systems, PCG with
every K-apply, step length and updates), with the signal and mask already
resident in HBM and the problem created (xi, diag H) outside the timed region.

The chosen form (FP32 Krylov with FP64 refinement, learned preconditioner
correction when trained parameters are present) gives `value`; the plain FP64
form is timed alongside.  Every form reports the LASSO certificate the
library computes with the solve (relative duality gap, natural residual).

`roofline` is the metric's matvec: one K-apply (the five kernels of
q = K p) in the chosen form's precision, FP32, timed with HIP events on the
library's stream around K-applies queued back to back (csipm_profile_kapply,
at the last solve's barrier diagonals), against its design bytes 15 n w + n/8 (five volume passes that
each read and write the work array, the K epilogue's inputs and outputs,
the mask bits); `frac_minimum` uses the least bytes any K-apply must move,
6 n w + n/8 (read p and the two diagonals, write q).  `traffic` is the
calibrated rocprofv3 FETCH_SIZE + WRITE_SIZE of the same kernels from a
committed profile record taken on the current kernel sources (null
otherwise).  `roofline.fp64` is the FP64 K-apply, `roofline.secondary` the
largest HBM-bound kernel of the chosen form's event-timed solve
(csipm_timing), and `kapply_in_solve` the FP32 K-apply kernels of that solve.

`cpu_baseline` times the CPU oracle on one K-apply of the same problem and
scales it by the number of operator applies of the FP64 solve; the same leg
certifies the chosen form's solution with the oracle (two naive transforms)
and times whole oracle solves of the 16^3 and 64^3 workloads beside the GPU's.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--grid 256]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "time-to-solve at rel KKT res 1e-6, plain vs FP32+learned-PC; matvec HBM GB/s"
PEAK_HBM_GBPS = 8000.0
from paper_2502_04217_amd.profile_kapply import PASS_NAMES, pass_bytes  # noqa: E402
PARAMS_FILE = os.path.join(ROOT, "paper_2502_04217_amd", "pc_params.json")


def kernel_bytes(name, shape, learned):
    """Algorithmic HBM bytes of one working launch of a timed kernel (names
    of csipm_timing_report), or None for the small finalize kernels and the
    correction inference, which is bound by arithmetic, not bytes.  FFT
    passes move the n-real work array once each way; the epilogues add the
    vectors they read and write; elementwise kernels count each FP64 array
    as 8n bytes and each FP32 array as 4n."""
    n1, n2, n3 = shape
    n = n1 * n2 * n3
    base, _, prec = name.partition(".")
    w = 8 if prec == "f64" else 4
    c = 4 if learned else 0   # FP32 correction read by P_c^{-1}
    table = {
        "axis1_inv": 2 * n * w, "axis2_inv": 2 * n * w, "axis2_fwd": 2 * n * w, "axis1_fwd": 2 * n * w,
        "axis3": 2 * n * w + n // 8,
        "axis1_fwd_K": 7 * n * w,
        # the K-apply of a CG direction with p <- z + beta p fused in: z read and
        # p written back by the passes that first read p
        "axis1_inv_P": 4 * n * w,
        "axis1_fwd_KP": 9 * n * w,
        # T, d (2), Sigma (2), h (2) in FP64, c; H d_beta out
        "axis1_fwd_R": (64 + c) * n,
        # h, d, Sigma (2 each), H d_beta in FP64, c; r32, z32, p32 (2 each, FP32) out
        "ref_restart+fin": (56 + c + 24) * n,
        # x, p, q, r, Sigma (2 each) in, x, r, z out (the first update of a solve skips reading x)
        "cg_update": 16 * n * w + c * n,
        # beta, z, nu1, nu2, G = H beta - xi in; Sigma, CG start r, p (and h, FP32 Sigma) out
        "newton_init": (96 + c) * n,
        "newton_init_noh": (64 + c) * n,   # FP32 system taken without refinement: no FP64 h, Sigma
        # beta, z, nu1, nu2 and the direction (FP64, or FP32 after an unrefined FP32 solve)
        "ipm_ratio+fin": 48 * n,
        "ipm_ratio_d32+fin": 40 * n,
        # beta, z, nu1, nu2, G, direction, H d_beta source (beta part) in; state and G out
        "ipm_advance+fin": 104 * n,
        "ipm_advance_d32+fin": 92 * n,
        # the same with the next Newton system built from the new iterate:
        # FP32 Sigma, r, p (ni32), also FP64 Sigma and h (ni32r), or FP64
        # Sigma, r, p (ni64)
        "ipm_advance_ni32+fin": 128 * n,
        "ipm_advance_ni32r+fin": 160 * n,
        "ipm_advance_ni64+fin": 152 * n,
        "ipm_advance_d32_ni32+fin": 116 * n,
        "ipm_advance_d32_ni32r+fin": 148 * n,
        "ipm_advance_d32_ni64+fin": 140 * n,
        # beta, z, nu1, nu2, H beta, xi in, G = H beta - xi out (after a full H-apply)
        "ipm_resid+fin": 56 * n,
        "set_f2d": 24 * n,
        "add_f2d": 40 * n,
        "log_l1+fin": 32 * n,
    }
    return table.get(base)


def working_min_us(shape):
    """Least duration of a launch that does its work: every volume kernel
    moves at least 2 n FP32 words, which takes 2 n 4 / 8 TB/s at the HBM peak
    (13.4 us at 256^3 with a 20 % margin).  Launches queued past a Krylov
    solve's convergence only read the device flag and return; with an event
    pair around each they still last several microseconds, so a fixed 8 us
    cut counts some of them as working."""
    n = shape[0] * shape[1] * shape[2]
    return max(8.0, 0.8 * 2 * n * 4 / (PEAK_HBM_GBPS * 1e9) * 1e6)


def kernel_breakdown(pr, opts, shape, learned):
    """One extra solve with per-kernel event timing; returns the per-kernel
    records (ms per solve) with algorithmic bytes attached, and the wall time
    of that same solve (event recording included).  A PCG iteration launches
    cg_update once, so its working launches are at most the solve's PCG
    iterations."""
    import torch
    pr.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    info_k = pr.solve(**opts)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rep = pr.timing_report(working_min_us(shape))
    pr.timing(False)
    # launches of cg_update that start a PCG solve read no x: 2nw fewer bytes
    starts = int(info_k["refine_steps_total"]) if opts["precision"] == 1 else int(info_k["ipm_iters"])
    out = []
    for r in rep:
        b = kernel_bytes(r["name"], shape, learned)
        if r["name"].startswith("cg_update"):
            r["working_calls"] = min(r["working_calls"], int(info_k["cg_iters_total"]))
        if b is not None and r["name"].startswith("cg_update"):
            n = shape[0] * shape[1] * shape[2]
            w = 8 if r["name"].endswith("f64") else 4
            tot = b * r["working_calls"] - 2 * n * w * min(starts, r["working_calls"])
            b = tot / max(1, r["working_calls"])
        r["bytes_per_launch"] = b
        out.append(r)
    out.sort(key=lambda r: -r["total_ms"])
    return out, wall


# the K-apply kernels of a PCG iteration as csipm_timing names them (with the
# fused direction update: *_P, *_KP)
KAPPLY_NAMES = ("axis1_inv", "axis1_inv_P", "axis2_inv", "axis3", "axis2_fwd", "axis1_fwd_K", "axis1_fwd_KP")


def kapply_in_solve(kern, prec, shape):
    """Algorithmic bytes over time of the precision-`prec` K-apply kernels
    of an event-timed solve (working launches: those queued past a Krylov
    solve's convergence return at once)."""
    n = shape[0] * shape[1] * shape[2]
    w = 4 if prec == "f32" else 8
    b = t = 0.0
    for r in kern:
        base, _, p = r["name"].partition(".")
        if p == prec and base in KAPPLY_NAMES and r["bytes_per_launch"] is not None:
            b += r["bytes_per_launch"] * r["working_calls"]
            t += r["working_ms"] * 1e-3
    napply = b / (15 * n * w + n // 8) if b else 0.0
    return {"GBps": b / t / 1e9 if t else None, "ms": t * 1e3, "applies_equiv": round(napply, 2)}


PROFILE_RECORDS = os.path.join(ROOT, "profiles")


def traffic_record(kernel, grid):
    """Calibrated rocprofv3 FETCH_SIZE + WRITE_SIZE bytes per launch of
    `kernel` at `grid`^3 from a committed profile summary, when it was taken
    on the current kernel sources; None otherwise."""
    if not os.path.isdir(PROFILE_RECORDS):
        return None
    from paper_2502_04217_amd.build import source_digest
    digest = source_digest()
    for f in sorted(os.listdir(PROFILE_RECORDS)):
        if not f.endswith((".md", ".txt")):
            continue
        with open(os.path.join(PROFILE_RECORDS, f)) as fh:
            for line in fh:
                if not line.startswith("traffic-record: "):
                    continue
                rec = json.loads(line[len("traffic-record: "):])
                if rec.get("kernel") == kernel and rec.get("grid") == grid and rec.get("source_sha256") == digest:
                    return rec
    return None


def load_params(torch):
    if not os.path.exists(PARAMS_FILE):
        return None
    with open(PARAMS_FILE) as f:
        d = json.load(f)
    return torch.tensor(d["params"], dtype=torch.float32, device="cuda")


def cpu_baseline(w, lam, info64, sig_for_k, beta_chosen, gpu_small):
    """Oracle (numpy float64, naive separable DFT) on a bounded sample: one
    K-apply of this problem, scaled by the operator-apply count of the GPU
    FP64 solve (PCG K-applies + one H-apply per interior-point iteration);
    the oracle's LASSO certificate of the chosen form's solution; whole
    oracle solves of the 16^3 and 64^3 workloads (gpu_small: the GPU's
    times on the same problems)."""
    import numpy as np
    from oracle import ipm
    from paper_2502_04217_amd import workload as wl
    host_cpus = os.cpu_count() or 1
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = host_cpus
    rng = np.random.default_rng(0)
    pb = rng.standard_normal(w.shape)
    pz = rng.standard_normal(w.shape)
    s1, s2 = sig_for_k
    obs = w.observed.astype(np.float64)
    t0 = time.perf_counter()
    ipm.K_apply(pb, pz, s1, s2, obs)
    t_apply = time.perf_counter() - t0
    applies = int(info64["cg_iters_total"]) + int(info64["ipm_iters"]) + 1
    t0 = time.perf_counter()
    cert = ipm.lasso_certificate(beta_chosen, w.signal, w.observed, lam)
    t_cert = time.perf_counter() - t0
    small = {}
    for name, make in (("grid16", lambda: wl.grid16(1)), ("grid64", lambda: wl.grid64(1))):
        ws = make()
        lam_s = ipm.lambda_rule(ws.signal, ws.observed)
        t0 = time.perf_counter()
        ref = ipm.ipm_solve(ws.signal, ws.observed, lam_s, ipm.IPMOptions(tol=1e-6))
        small[name] = {"oracle_s": time.perf_counter() - t0, "oracle_ipm_iters": ref.iters,
                       "gpu_fp64_s": gpu_small.get(name)}
    return {"value": t_apply * applies, "unit": "s", "cores": int(threads), "kind": "oracle",
            "host_cpus": int(host_cpus), "blas_threads": int(threads),
            "sample": f"one oracle K-apply at {w.shape[0]}^3 ({t_apply:.2f} s) x {applies} operator applies "
                      f"of the GPU FP64 solve (extrapolated time-to-solve)",
            "oracle_certificate_chosen": {"rel_dual_gap": cert.rel_gap, "natural_residual": cert.natural_residual,
                                          "max_offsupport_ratio": cert.max_offsupport_ratio,
                                          "max_onsupport_dev": cert.max_onsupport_dev, "seconds": t_cert},
            "oracle_full_solves_tol_1e-6": small}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--grid", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-reps", type=int, default=20)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the solver is single-device "
              f"and the library has no multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a HIP device")
    from paper_2502_04217_amd import csipm
    from paper_2502_04217_amd import workload as wl

    t0 = time.perf_counter()
    if args.grid == 256:
        w = wl.grid256(1)
    elif args.grid == 512:
        w = wl.grid512(1)
    elif args.grid == 64:
        w = wl.grid64(1)
    elif args.grid == 128:
        w = wl.grid128_family(10000)
    else:
        raise SystemExit("grid must be 64, 128, 256 or 512")
    gen_s = time.perf_counter() - t0
    print(f"[bench] workload {w.name}: missing {w.missing_fraction:.4f}, generated in {gen_s:.1f} s",
          file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    pr = csipm.Problem(w.signal, w.observed)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    lam = pr.lambda_rule(0.05)
    params = load_params(torch)
    learned = params is not None
    if learned:
        pr.set_pc_params(params)
    chosen = dict(tol=1e-6, precision=csipm.FP32, pc=csipm.PC_LEARNED if learned else csipm.PC_PLAIN)
    plain = dict(tol=1e-6, precision=csipm.FP64, pc=csipm.PC_PLAIN)

    for _ in range(args.warmup):
        pr.solve(**chosen)
        pr.solve(**plain)
    torch.cuda.synchronize()

    t0 = time.perf_counter()
    infos = []
    for _ in range(args.steps):
        infos.append(pr.solve(**chosen))
    torch.cuda.synchronize()
    chosen_s = (time.perf_counter() - t0) / args.steps
    chosen_log = pr.log()
    beta_chosen = pr.get(csipm.BETA)
    print(f"[bench] chosen form: {chosen_s * 1e3:.1f} ms/solve {infos[-1]}", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    infos64 = []
    for _ in range(args.steps):
        infos64.append(pr.solve(**plain))
    torch.cuda.synchronize()
    plain_s = (time.perf_counter() - t0) / args.steps
    beta64 = pr.get(csipm.BETA)
    print(f"[bench] plain FP64: {plain_s * 1e3:.1f} ms/solve {infos64[-1]}", file=sys.stderr, flush=True)

    # the FP32 form with the paper's preconditioner: what the learned correction adds or saves
    fp32_plain = dict(tol=1e-6, precision=csipm.FP32, pc=csipm.PC_PLAIN)
    pr.solve(**fp32_plain)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos32 = [pr.solve(**fp32_plain) for _ in range(args.steps)]
    torch.cuda.synchronize()
    fp32_plain_s = (time.perf_counter() - t0) / args.steps
    fp32_plain_log = pr.log()
    rel_diff = float((beta_chosen - beta64).norm() / beta64.norm())

    # the other Krylov methods and preconditioner of the paper's list, and
    # predictor-corrector steps, FP64
    alternatives = {}
    for name, f in (("cr_fp64", dict(krylov=csipm.KRYLOV_CR)), ("car_fp64", dict(krylov=csipm.KRYLOV_CAR)),
                    ("scaled_pc_fp64", dict(pc=csipm.PC_SCALED)), ("mehrotra_fp64", dict(mehrotra=1))):
        alt = dict(plain, **f)
        pr.solve(**alt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ia = [pr.solve(**alt) for _ in range(args.steps)]
        torch.cuda.synchronize()
        alternatives[name] = {"seconds": (time.perf_counter() - t0) / args.steps, "ipm_iters": ia[-1]["ipm_iters"],
                              "krylov_iters_total": ia[-1]["cg_iters_total"], "rel_kkt": ia[-1]["rel_kkt"],
                              "status": ia[-1]["status_name"], "rel_dual_gap": ia[-1]["rel_dual_gap"],
                              "natural_residual": ia[-1]["natural_residual"]}

    # per-kernel event timing of one more solve of each form; the largest
    # HBM-bound kernel of the chosen form is the secondary roofline entry
    n = int(np.prod(w.shape))
    kern, kern_wall = kernel_breakdown(pr, chosen, w.shape, learned)
    kern64, kern64_wall = kernel_breakdown(pr, plain, w.shape, False)
    top = next(r for r in kern if r["bytes_per_launch"] is not None)
    dominant_is_top = top is kern[0]

    # per-kernel timing of the K-apply at the last Newton system's barrier diagonals
    prof = {}
    for name, prec, wsz in (("fp32", csipm.FP32, 4), ("fp64", csipm.FP64, 8)):
        pr.profile_kapply(prec, 3)
        ms, whole, launched = pr.profile_kapply_all(prec, args.profile_reps)
        by = pass_bytes(w.shape, wsz)
        prof[name] = {"ms": ms, "whole_ms": whole, "launched_ms": launched, "bytes": by}
    k_bytes = top["bytes_per_launch"] * top["working_calls"]
    achieved = k_bytes / (top["total_ms"] * 1e-3) / 1e9
    rec = traffic_record(top["name"], w.shape[0])
    traffic = None
    if rec is not None:
        traffic = rec["read_bytes"] + rec["write_bytes"]
    kapply = {}
    for name, wsz in (("fp32", 4), ("fp64", 8)):
        # one K-apply among applies replayed back to back from a HIP graph, as
        # the PCG iterations of a solve are (one event pair around them all);
        # the per-kernel times below carry an event pair each
        t = prof[name]["whole_ms"] * 1e-3
        design = 15 * n * wsz + n // 8
        minimum = 6 * n * wsz + n // 8
        krec = traffic_record("kapply." + ("f32" if wsz == 4 else "f64"), w.shape[0])
        kapply[name] = {"ms": t * 1e3, "design_bytes": design, "minimum_bytes": minimum,
                        "design_GBps": design / t / 1e9,
                        "minimum_GBps": minimum / t / 1e9,
                        "traffic": (krec["read_bytes"] + krec["write_bytes"]) if krec else None,
                        "ms_launched_directly": prof[name]["launched_ms"],
                        "per_kernel_ms": dict(zip(PASS_NAMES, [round(v, 5) for v in prof[name]["ms"]])),
                        "per_kernel_sum_ms": round(sum(prof[name]["ms"]), 5)}
    roofline = {"bound": "hbm", "kernel": "K-apply q = K p (5 kernels), fp32",
                "achieved": kapply["fp32"]["design_GBps"], "peak": PEAK_HBM_GBPS, "unit": "GB/s",
                "frac": kapply["fp32"]["design_GBps"] / PEAK_HBM_GBPS, "traffic": kapply["fp32"]["traffic"],
                "bytes_per_launch": kapply["fp32"]["design_bytes"], "avg_ms": kapply["fp32"]["ms"],
                "frac_minimum": kapply["fp32"]["minimum_GBps"] / PEAK_HBM_GBPS,
                "fp64": {"achieved": kapply["fp64"]["design_GBps"],
                         "frac": kapply["fp64"]["design_GBps"] / PEAK_HBM_GBPS,
                         "frac_minimum": kapply["fp64"]["minimum_GBps"] / PEAK_HBM_GBPS,
                         "traffic": kapply["fp64"]["traffic"], "avg_ms": kapply["fp64"]["ms"],
                         "bytes_per_launch": kapply["fp64"]["design_bytes"]},
                "secondary": {"kernel": top["name"], "achieved": achieved, "frac": achieved / PEAK_HBM_GBPS,
                              "traffic": traffic, "dominant": dominant_is_top, "launches": top["calls"],
                              "working_launches": top["working_calls"],
                              "avg_ms": top["total_ms"] / max(1, top["calls"]),
                              "bytes_per_launch": top["bytes_per_launch"]}}

    # learned-correction inference on every coefficient (the network's two
    # dense layers on the matrix cores): 2 (4*32 + 32*32) MFMA flops per coefficient
    corr = None
    if learned:
        feat = torch.randn((n, 4), dtype=torch.float32, device="cuda")
        csipm.mlp_forward(params, feat)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        e0.record()
        for _ in range(reps):
            csipm.mlp_forward(params, feat)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        tf = 2 * (4 * 32 + 32 * 32) * n / (ms * 1e-3) / 1e12
        corr = {"kernel": "k_forward, all n coefficients", "ms": ms, "bound": "alu",
                "mfma_tflops": tf, "mfma_peak_fp32": 157.3, "mfma_frac": tf / 157.3,
                "note": "bound by the VALU tanh (exp2 + reciprocal per neuron), not by the matrix cores"}
        del feat

    cpu = None
    if not args.no_cpu_baseline:
        # the GPU's FP64 solve times of the small workloads the oracle solves whole
        gpu_small = {}
        for name, make in (("grid16", lambda: wl.grid16(1)), ("grid64", lambda: wl.grid64(1))):
            ws = make()
            ps = csipm.Problem(ws.signal, ws.observed)
            ps.lambda_rule(0.05)
            ps.solve(tol=1e-6)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                ps.solve(tol=1e-6)
            torch.cuda.synchronize()
            gpu_small[name] = (time.perf_counter() - t0) / 3
            ps.close()
        sig1, sig2 = wl.random_barrier(w.shape, 1, spread=3.0)
        cpu = cpu_baseline(w, lam, infos64[-1], (sig1, sig2), beta_chosen.cpu().numpy(), gpu_small)
        print(f"[bench] cpu baseline: {cpu}", file=sys.stderr, flush=True)

    def cert_of(i):
        return {"rel_dual_gap": i["rel_dual_gap"], "natural_residual": i["natural_residual"],
                "objective": i["objective"]}

    last = infos[-1]
    out = {
        "metric": METRIC,
        "value": chosen_s,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": chosen_s * 1e3,
        "higher_is_better": False,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32 Krylov + f64 refinement" if chosen["precision"] == csipm.FP32 else "f64",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.shape[0]}x{w.shape[1]}x{w.shape[2]} crystal-like grid, "
                               f"missing {w.missing_fraction:.4f}, lambda = 0.05 |M^T b|_inf",
                   "form": ("fp32+refine+learned-pc" if learned else "fp32+refine+plain-pc (no trained params)"),
                   "tol_rel_kkt": 1e-6, "n": n},
        "solve": {"ipm_iters": last["ipm_iters"], "cg_iters_total": last["cg_iters_total"],
                  "cg_per_iter": [r["cg_iters"] for r in chosen_log],
                  "learned_per_iter": [r["learned"] for r in chosen_log],
                  "refine_steps": last["refine_steps_total"], "fallbacks": last["fallbacks"],
                  "rel_kkt": last["rel_kkt"], "rel_diff_vs_fp64": rel_diff, "certificate": cert_of(last)},
        "plain_fp64": {"seconds": plain_s, "ipm_iters": infos64[-1]["ipm_iters"],
                       "cg_iters_total": infos64[-1]["cg_iters_total"], "rel_kkt": infos64[-1]["rel_kkt"],
                       "certificate": cert_of(infos64[-1])},
        "fp32_plain_pc": {"seconds": fp32_plain_s, "ipm_iters": infos32[-1]["ipm_iters"],
                          "cg_per_iter": [r["cg_iters"] for r in fp32_plain_log],
                          "cg_iters_total": infos32[-1]["cg_iters_total"], "rel_kkt": infos32[-1]["rel_kkt"],
                          "refine_steps": infos32[-1]["refine_steps_total"], "certificate": cert_of(infos32[-1])},
        "alternatives_fp64": alternatives,
        "correction_inference": corr,
        "setup_seconds": setup_s,
        "setup_seconds_library": last["setup_seconds"],
        "roofline": roofline,
        "kapply_in_solve": {"fp32": kapply_in_solve(kern, "f32", w.shape),
                            "fp64": kapply_in_solve(kern64, "f64", w.shape)},
        # summed kernel durations of the event-timed solve of each form, beside
        # the wall time of that same solve: the difference is time the device
        # sat idle (host synchronisation, launch latency and event recording)
        "kernel_busy_ms_per_solve": {"chosen": round(sum(r["total_ms"] for r in kern), 3),
                                     "chosen_same_solve_wall": round(kern_wall * 1e3, 3),
                                     "plain_fp64": round(sum(r["total_ms"] for r in kern64), 3),
                                     "plain_fp64_same_solve_wall": round(kern64_wall * 1e3, 3)},
        "kernels_ms_per_solve": {r["name"]: round(r["total_ms"], 3) for r in kern[:10]},
        "kernels_ms_per_solve_fp64": {r["name"]: round(r["total_ms"], 3) for r in kern64[:8]},
        "kapply": kapply,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
