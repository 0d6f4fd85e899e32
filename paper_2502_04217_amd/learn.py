"""Training and evaluation of the learned preconditioner correction.

Data: plain-preconditioner FP64 solves of seeded 128^3 problems (the 128^3
family: sparsity log-uniform in [0.05%, 0.5%], SNR uniform in [5, 20] dB,
lattice period in {8, 16, 32}) with record capture on.  By default the
capture follows the learned form's policy (csipm_capture mode 2): only at
the interior-point iterations where the correction would be applied, the
first Krylov direction of the Newton solve is reduced to `n_per_iter`
records (features + loss terms) at pseudo-random coefficients among those
where the correction can act, weighted by that system's PCG count.  With
--all-iterations every iteration is captured at uniformly drawn
coefficients.

Training: Adam on the records with the library's forward/backward kernels
(csipm_mlp_train_step: loss_grad, then adam); each step uses the records of one
captured iteration, iterations visited in a seeded random order.

Evaluation: held-out seeds solved with the paper's preconditioner and with
the learned correction, in FP64 and FP32+refinement, comparing PCG
iterations, wall time (the faster of each form's second and third solves
on the problem: the first records its HIP graphs) and the true final KKT
residual.

    python -m paper_2502_04217_amd.learn --train 200 --eval 50
    python -m paper_2502_04217_amd.learn --eval-only --eval 50 --md learned_eval.md

writes paper_2502_04217_amd/pc_params.json (or --params-out; not with
--eval-only), learn_eval.json (or --out) and, with --md, the per-seed
evaluation as a markdown table.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import random
import sys
import time

import numpy as np

from . import csipm
from . import workload as wl

HERE = os.path.dirname(os.path.abspath(__file__))
PARAMS_FILE = os.path.join(HERE, "pc_params.json")
TRAIN_SEEDS = range(0, 200)
EVAL_SEEDS = range(10000, 10050)


def init_params(seed: int = 0, out_scale: float = 0.01):
    """Glorot-uniform hidden layers, small output layer with the output bias
    at softplus^{-1}(1): the untrained correction is c ~ 1, the paper's P."""
    rng = np.random.default_rng(seed)
    H1, H2, NIN = 32, 32, 4

    def glorot(fo, fi):
        a = math.sqrt(6.0 / (fi + fo))
        return rng.uniform(-a, a, size=(fo, fi))

    p = np.concatenate([glorot(H1, NIN).ravel(), np.zeros(H1), glorot(H2, H1).ravel(), np.zeros(H2),
                        rng.uniform(-out_scale, out_scale, H2), [math.log(math.e - 1.0)]])
    assert p.size == csipm.MLP_PARAMS
    return p.astype(np.float32)


def collect(seeds, n_per_iter=4096, max_iters=80, policy=True, periods=(8, 16, 32), log=print):
    import torch
    feats, recs = [], []
    t0 = time.time()
    for s in seeds:
        w = wl.grid128_family(s, periods)
        pr = csipm.Problem(w.signal, w.observed)
        pr.lambda_rule(0.05)
        feat = torch.empty((max_iters * n_per_iter, 4), dtype=torch.float32, device="cuda")
        rec = torch.empty((max_iters * n_per_iter, 6), dtype=torch.float32, device="cuda")
        pr.capture(feat, rec, n_per_iter, max_iters, seed=1000003 * (s + 1), policy=policy)
        info = pr.solve(tol=1e-6, precision=csipm.FP64, pc=csipm.PC_PLAIN)
        k, cg = pr.captured()
        for i in range(k):
            if cg[i] > 0:
                feats.append(feat[i * n_per_iter:(i + 1) * n_per_iter])
                recs.append(rec[i * n_per_iter:(i + 1) * n_per_iter])
        pr.close()
        log(f"[collect] seed {s}: {w.name} missing {w.missing_fraction:.3f} ipm {info['ipm_iters']} "
            f"cg {info['cg_iters_total']} captured {k} ({time.time() - t0:.0f} s)")
    return feats, recs


def train(feats, recs, epochs=20, lr=2e-3, seed=0, log=print):
    import torch
    params = torch.tensor(init_params(seed), device="cuda")
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    n_per = feats[0].shape[0]
    scratch = csipm._scratch(n_per, params.device)
    order = list(range(len(feats)))
    rng = random.Random(seed)
    t = 0
    hist = []
    for ep in range(epochs):
        rng.shuffle(order)
        tot = 0.0
        losses = []
        for i in order:
            t += 1
            lr_t = lr * 0.5 * (1 + math.cos(math.pi * min(1.0, t / (epochs * len(order)))))
            loss, _ = csipm.mlp_train_step(params, m, v, t, max(lr_t, 1e-5), feats[i], recs[i], scratch)
            losses.append(loss)
        tot = float(torch.cat(losses).sum().item())
        hist.append(tot)
        log(f"[train] epoch {ep}: total loss {tot:.6e}")
    return params, hist


def baseline_loss(feats, recs):
    """Loss of the untrained correction (c = 1) on the same records."""
    import torch
    p0 = torch.tensor(init_params(0, out_scale=0.0), device="cuda")
    scratch = csipm._scratch(feats[0].shape[0], p0.device)
    return float(sum(csipm.mlp_loss_grad(p0, f, r, scratch)[0].item() for f, r in zip(feats, recs)))


# evaluation workloads by grid: the 128^3 family (held-out seeds) and the
# 256^3 and 512^3 recipes of the full-size runs (seeds 1, 2, ...; the network
# never sees these grids in training)
EVAL_FAMILIES = {
    128: (wl.grid128_family, "the 128^3 family (sparsity log-uniform in [0.05 %, 0.5 %], SNR uniform in "
                             "[5, 20] dB, lattice period in {8, 16, 32})"),
    256: (wl.grid256, "the 256^3 recipe (0.1 % of the bins, N(0,1) exp(-|k|/32) parts, SNR 10 dB, cubes of "
                      "half-width 3 on a period-32 lattice plus 2 % dropouts)"),
    512: (wl.grid512, "the 512^3 recipe (0.02 % of the bins, N(0,1) parts, SNR 10 dB, cubes of half-width 4 on "
                      "a period-64 lattice)"),
}


def eval_seeds(grid, count):
    return list(EVAL_SEEDS)[:count] if grid == 128 else list(range(1, 1 + count))


def evaluate(params, seeds, log=print, grid=128, **solve_kw):
    """Each problem solved in the four forms; solve_kw adds solve options
    (e.g. pc_min_missing) to every solve."""
    out = []
    family = EVAL_FAMILIES[grid][0]
    for s in seeds:
        w = family(s)
        pr = csipm.Problem(w.signal, w.observed)
        pr.lambda_rule(0.05)
        pr.set_pc_params(params)
        row = {"seed": s, "name": w.name, "missing": w.missing_fraction}
        for tag, prec, pc in (("fp64_plain", csipm.FP64, csipm.PC_PLAIN), ("fp64_learned", csipm.FP64, csipm.PC_LEARNED),
                              ("fp32_plain", csipm.FP32, csipm.PC_PLAIN), ("fp32_learned", csipm.FP32, csipm.PC_LEARNED)):
            # the first solve of a form on a context records its HIP graphs;
            # the time is the faster of the next two (the counts do not change)
            pr.solve(tol=1e-6, precision=prec, pc=pc, **solve_kw)
            info = pr.solve(tol=1e-6, precision=prec, pc=pc, **solve_kw)
            again = pr.solve(tol=1e-6, precision=prec, pc=pc, **solve_kw)
            info["solve_seconds"] = min(info["solve_seconds"], again["solve_seconds"])
            true = pr.residuals()
            row[tag] = {"cg": info["cg_iters_total"], "ipm": info["ipm_iters"], "s": info["solve_seconds"],
                        "fallbacks": info["fallbacks"], "rel_kkt": true["rel_kkt"], "status": info["status"]}
        pr.close()
        out.append(row)
        log(f"[eval] seed {s}: " + " ".join(f"{k}={row[k]['cg']}/{row[k]['s'] * 1e3:.0f}ms"
                                             for k in ("fp64_plain", "fp64_learned", "fp32_plain", "fp32_learned")))
    return out


def summarize(rows):
    def tot(k, f):
        return float(sum(r[k][f] for r in rows))
    s = {}
    for k in ("fp64_plain", "fp64_learned", "fp32_plain", "fp32_learned"):
        s[k] = {"cg_total": tot(k, "cg"), "seconds_total": tot(k, "s"), "fallbacks": tot(k, "fallbacks"),
                "max_true_rel_kkt": max(r[k]["rel_kkt"] for r in rows)}
    s["cg_ratio_fp64"] = s["fp64_learned"]["cg_total"] / max(1.0, s["fp64_plain"]["cg_total"])
    s["cg_ratio_fp32"] = s["fp32_learned"]["cg_total"] / max(1.0, s["fp32_plain"]["cg_total"])
    s["time_ratio_fp64"] = s["fp64_learned"]["seconds_total"] / s["fp64_plain"]["seconds_total"]
    s["time_ratio_fp32"] = s["fp32_learned"]["seconds_total"] / s["fp32_plain"]["seconds_total"]
    return s


def markdown(rows, summ, command, params_note, grid=128):
    """The per-seed evaluation as a markdown record."""
    held = (" (held out: training uses seeds 0-199 of the 128^3 family)" if grid == 128 else
            " (training sees only 128^3 problems)")
    head = [f"# Learned preconditioner correction on held-out {grid}^3 problems", "",
            "Workload: " + EVAL_FAMILIES[grid][1] + ", seeds " + f"{rows[0]['seed']}-{rows[-1]['seed']}" + held +
            ", lambda = 0.05 |M^T b|_inf, each solved to rel_kkt 1e-6 with the "
            "paper's P and with the learned correction, in FP64 and in FP32 with FP64 refinement.", "",
            "Parameters: " + params_note, "", "Command:", "", "    " + command, "",
            "PCG: total PCG iterations of the solve; ms: solve wall time (the faster `solve_seconds` of the second "
            "and third solves of the form on the problem; the first records its HIP graphs); true rel_kkt: the "
            "KKT residual recomputed with a fresh FP64 H-apply after the solve; fb: learned systems that "
            "restarted with the paper's P.", "",
            "## Totals", "",
            "| form | PCG total | time total (ms) | fallbacks | max true rel_kkt |", "|---|---|---|---|---|"]
    for k in ("fp64_plain", "fp64_learned", "fp32_plain", "fp32_learned"):
        t = summ[k]
        head.append(f"| {k} | {t['cg_total']:.0f} | {t['seconds_total'] * 1e3:.1f} | {t['fallbacks']:.0f} | "
                    f"{t['max_true_rel_kkt']:.2e} |")
    head += ["", f"PCG ratio learned/plain: FP64 {summ['cg_ratio_fp64']:.3f}, FP32 {summ['cg_ratio_fp32']:.3f}; "
             f"time ratio: FP64 {summ['time_ratio_fp64']:.3f}, FP32 {summ['time_ratio_fp32']:.3f}.", "",
             "## Per seed", "",
             "| seed | missing | FP64 P: PCG / ms / rel_kkt | FP64 learned: PCG / ms / rel_kkt / fb "
             "| FP32 P: PCG / ms / rel_kkt | FP32 learned: PCG / ms / rel_kkt / fb |", "|---|---|---|---|---|---|"]
    for r in rows:
        cells = []
        for k in ("fp64_plain", "fp64_learned", "fp32_plain", "fp32_learned"):
            e = r[k]
            c = f"{e['cg']} / {e['s'] * 1e3:.2f} / {e['rel_kkt']:.1e}"
            if k.endswith("learned"):
                c += f" / {e['fallbacks']}"
            cells.append(c)
        head.append(f"| {r['seed']} | {r['missing']:.4f} | " + " | ".join(cells) + " |")
    return "\n".join(head) + "\n"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=200)
    ap.add_argument("--eval", type=int, default=50)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", default="learn_eval.json")
    ap.add_argument("--eval-only", action="store_true", help="evaluate the stored parameters, no training")
    ap.add_argument("--all-iterations", action="store_true",
                    help="capture every interior-point iteration at uniform coefficients (default: the policy's)")
    ap.add_argument("--params-in", default=PARAMS_FILE, help="parameters evaluated by --eval-only")
    ap.add_argument("--params-out", default=PARAMS_FILE)
    ap.add_argument("--md", help="also write the per-seed evaluation as markdown to this path")
    ap.add_argument("--periods", type=int, nargs="+", default=[8, 16, 32],
                    help="lattice periods of the training problems (the evaluation family keeps 8, 16, 32)")
    ap.add_argument("--eval-grid", type=int, choices=sorted(EVAL_FAMILIES), default=128,
                    help="evaluation workloads: the 128^3 family, or seeds 1.. of the 256^3 or 512^3 recipe")
    ap.add_argument("--pc-min-missing", type=float, default=None,
                    help="the solve option pc_min_missing in the evaluation (default: the library's, 0.01)")
    args = ap.parse_args()
    command = "python -m paper_2502_04217_amd.learn " + " ".join(sys.argv[1:])
    solve_kw = {} if args.pc_min_missing is None else {"pc_min_missing": args.pc_min_missing}
    log = lambda *a: print(*a, flush=True)
    if args.eval_only:
        import torch
        with open(args.params_in) as f:
            stored = json.load(f)
        params = torch.tensor(stored["params"], dtype=torch.float32, device="cuda")
        rows = evaluate(params, eval_seeds(args.eval_grid, args.eval), log=log, grid=args.eval_grid, **solve_kw)
        summ = summarize(rows)
        log(json.dumps(summ))
        os.makedirs(os.path.dirname(args.out) or ".", exist_ok=True)
        with open(args.out, "w") as f:
            json.dump({"summary": summ, "rows": rows}, f)
        if args.md:
            note = (f"`{os.path.relpath(args.params_in, os.path.dirname(HERE))}`, written by "
                    f"`{stored.get('command', '?')}` (training loss {stored.get('loss_untrained', float('nan')):.4g} "
                    f"with c = 1, {stored.get('loss_trained', float('nan')):.4g} trained).")
            with open(args.md, "w") as f:
                f.write(markdown(rows, summ, command, note, grid=args.eval_grid))
        return 0
    t0 = time.time()
    feats, recs = collect(list(TRAIN_SEEDS)[:args.train], policy=not args.all_iterations,
                          periods=tuple(args.periods), log=log)
    log(f"[collect] {len(feats)} record groups in {time.time() - t0:.0f} s")
    l0 = baseline_loss(feats, recs)
    t1 = time.time()
    params, hist = train(feats, recs, epochs=args.epochs, lr=args.lr, log=log)
    log(f"[train] {time.time() - t1:.0f} s; loss c=1: {l0:.6e} trained: {hist[-1]:.6e}")
    os.makedirs(os.path.dirname(args.params_out) or ".", exist_ok=True)
    with open(args.params_out, "w") as f:
        json.dump({"params": params.cpu().tolist(), "train_seeds": [0, args.train], "epochs": args.epochs,
                   "lr": args.lr, "loss_untrained": l0, "loss_trained": hist[-1],
                   "capture": "all iterations" if args.all_iterations else "policy", "periods": args.periods,
                   "record_groups": len(feats), "command": command}, f)
    rows = evaluate(params, eval_seeds(args.eval_grid, args.eval), log=log, grid=args.eval_grid, **solve_kw)
    summ = summarize(rows)
    log(json.dumps(summ))
    os.makedirs(os.path.dirname(args.out) or ".", exist_ok=True)
    with open(args.out, "w") as f:
        json.dump({"summary": summ, "rows": rows, "loss_hist": hist, "loss_untrained": l0}, f)
    if args.md:
        note = (f"trained by this command on {len(feats)} captured iterations (training loss {l0:.4g} with c = 1, "
                f"{hist[-1]:.4g} trained).")
        with open(args.md, "w") as f:
            f.write(markdown(rows, summ, command, note, grid=args.eval_grid))


if __name__ == "__main__":
    sys.exit(main())
