"""GPU kernels of the learned preconditioner correction against the CPU
oracle (oracle/mlp.py): forward, backward, loss gradient and Adam within
float32 tolerance; features of an iterate; the learned solve reaching the
same LASSO solution; the fallback to the paper's preconditioner; and the
gain of the trained network on held-out problems."""
import json
import os

import numpy as np
import pytest

from oracle import dft3, ipm, mlp
from paper_2502_04217_amd import workload as wl
from tests._gpu_common import need_gpu, rel2, rel_inf, say

pytestmark = pytest.mark.gpu


def _records(n, seed):
    rng = np.random.default_rng(seed)
    feats = np.stack([rng.normal(0, 2, n), rng.uniform(-1, 1, n), rng.uniform(-27, 0, n),
                      rng.uniform(0.8, 1.0, n)], axis=1)
    s1, s2 = wl.random_barrier((n,), seed + 1, spread=2.0)
    rec = np.stack([rng.standard_normal(n), rng.standard_normal(n), s1 + s2, s1 - s2, 4 * s1 * s2,
                    rng.uniform(0.5, 1.5, n) / n], axis=1)
    return feats.astype(np.float32), rec.astype(np.float32)


def _params(seed, scale=0.5):
    p = mlp.init_params(seed, out_scale=scale) + 0.05 * np.random.default_rng(seed).standard_normal(mlp.N_PARAMS)
    return p.astype(np.float32)


@pytest.mark.parametrize("n", [1, 63, 64, 1000, 70001])
def test_forward_backward_loss_grad(n):
    torch = need_gpu()
    from paper_2502_04217_amd import csipm
    say("mlp kernels n =", n)
    feats, rec = _records(n, 3)
    p = _params(1)
    f64 = feats.astype(np.float64)
    r64 = rec.astype(np.float64)
    tp = torch.tensor(p, device="cuda")
    tf = torch.tensor(feats, device="cuda")
    tr = torch.tensor(rec, device="cuda")
    c = csipm.mlp_forward(tp, tf).cpu().numpy()
    cref, cache = mlp.forward(p.astype(np.float64), f64)
    assert rel_inf(c, cref) <= 1e-5
    dc = np.random.default_rng(4).standard_normal(n).astype(np.float32)
    g = csipm.mlp_backward(tp, tf, torch.tensor(dc, device="cuda")).cpu().numpy()
    gref = mlp.backward(p.astype(np.float64), cache, dc.astype(np.float64))
    assert rel_inf(g, gref) <= 1e-4
    loss, g2 = csipm.mlp_loss_grad(tp, tf, tr)
    lref, g2ref = mlp.loss_and_grad(p.astype(np.float64), f64, *[r64[:, i] for i in range(6)])
    assert abs(float(loss.item()) - lref) <= 1e-5 * abs(lref)
    assert rel_inf(g2.cpu().numpy(), g2ref) <= 1e-4
    # bitwise reproducible reduction
    loss_b, g2b = csipm.mlp_loss_grad(tp, tf, tr)
    assert torch.equal(g2, g2b) and torch.equal(loss, loss_b)


def test_adam_matches_oracle():
    torch = need_gpu()
    from paper_2502_04217_amd import csipm
    p = _params(2)
    rng = np.random.default_rng(5)
    tp = torch.tensor(p, device="cuda")
    m = torch.zeros_like(tp)
    v = torch.zeros_like(tp)
    pr, mr, vr = p.astype(np.float64), np.zeros(p.size), np.zeros(p.size)
    for t in range(1, 6):
        g = rng.standard_normal(p.size).astype(np.float32)
        csipm.mlp_adam(tp, torch.tensor(g, device="cuda"), m, v, t, 1e-3)
        pr, mr, vr = mlp.adam_step(pr, g.astype(np.float64), mr, vr, t, 1e-3)
    assert np.abs(tp.cpu().numpy() - pr).max() <= 1e-6


def test_train_step_equals_loss_grad_then_adam():
    """csipm_mlp_train_step queues the loss_grad and adam kernels in that
    order: parameters, moments, loss and gradient equal (bit for bit) those of
    the two separate calls, over three steps."""
    torch = need_gpu()
    from paper_2502_04217_amd import csipm
    f, r = _records(3000, 21)
    tf, tr = torch.tensor(f, device="cuda"), torch.tensor(r, device="cuda")
    p0 = torch.tensor(_params(5), device="cuda")
    pa, ma, va = p0.clone(), torch.zeros_like(p0), torch.zeros_like(p0)
    pb, mb, vb = p0.clone(), torch.zeros_like(p0), torch.zeros_like(p0)
    for t in (1, 2, 3):
        la, ga = csipm.mlp_train_step(pa, ma, va, t, 1e-3, tf, tr)
        lb, gb = csipm.mlp_loss_grad(pb, tf, tr)
        csipm.mlp_adam(pb, gb, mb, vb, t, 1e-3)
        assert torch.equal(la, lb) and torch.equal(ga, gb)
        assert torch.equal(pa, pb) and torch.equal(ma, mb) and torch.equal(va, vb)
    assert not torch.equal(pa, p0)


def test_features_of_iterate():
    torch = need_gpu()
    from paper_2502_04217_amd import csipm
    w = wl.grid16(2)
    pr = csipm.Problem(w.signal, w.observed)
    pr.lambda_rule(0.05)
    pr.solve(tol=1e-3)
    s1, s2 = wl.random_barrier(w.shape, 7, spread=4.0)
    pr.set_barrier(torch.tensor(s1, device="cuda"), torch.tensor(s2, device="cuda"))
    f = pr.features().cpu().numpy()
    beta = pr.get(csipm.BETA).cpu().numpy()
    ref = mlp.features(s1, s2, beta, dft3.diag_H(w.observed.astype(np.float64)))
    assert np.abs(f - ref).max() <= 1e-5 * np.abs(ref).max()


def test_correction_of_iterate_matches_oracle():
    """c at an iterate: network where L1/(L1 + 4 S1 S2) >= 1e-3, 1 elsewhere."""
    torch = need_gpu()
    from paper_2502_04217_amd import csipm
    w = wl.grid16(3)
    pr = csipm.Problem(w.signal, w.observed)
    pr.lambda_rule(0.05)
    p = _params(5)
    pr.set_pc_params(torch.tensor(p, device="cuda"))
    for tol in (1e-1, 1e-4):
        pr.solve(tol=tol)
        st = [pr.get(v).cpu().numpy() for v in (csipm.BETA, csipm.Z, csipm.NU1, csipm.NU2)]
        c = pr.pc_correction().cpu().numpy()
        ref, act = mlp.correction(p.astype(np.float64), *st, dft3.diag_H(w.observed.astype(np.float64)))
        say("correction active fraction", act.mean())
        assert np.abs(c - ref).max() <= 1e-5 * np.abs(ref).max()
        assert np.all(c[~act] == 1.0)


def test_learned_solve_same_solution_and_fallback():
    torch = need_gpu()
    from paper_2502_04217_amd import csipm
    w = wl.grid16(4)
    lam = ipm.lambda_rule(w.signal, w.observed)
    ref = ipm.ipm_solve(w.signal, w.observed, lam, ipm.IPMOptions(tol=1e-11))
    pr = csipm.Problem(w.signal, w.observed)
    pr.set_lambda(lam)
    pr.set_pc_params(torch.tensor(_params(3), device="cuda"))
    for prec in (0, 1):
        for min_cg, max_rel in ((0, 1.0), (2, 1.0), (2, 0.5)):
            info = pr.solve(tol=1e-11, pc=1, precision=prec, pc_min_cg=min_cg, pc_max_relevant=max_rel)
            beta = pr.get(csipm.BETA).cpu().numpy()
            log = pr.log()
            say("learned solve precision", prec, "pc_min_cg", min_cg, "pc_max_relevant", max_rel, info)
            say("  relevant", [round(r["relevant"], 4) for r in log])
            assert info["status"] in (0, 3)
            assert rel2(beta, ref.state.beta) <= 1e-7
            # the correction is applied exactly where the previous system needed
            # >= pc_min_cg iterations and at most max_rel of the coefficients are relevant
            prev = [0] + [r["cg_iters"] for r in log[:-1]]
            assert all(0.0 <= r["relevant"] <= 1.0 for r in log)
            assert [r["learned"] for r in log] == [int(p >= min_cg and r["relevant"] <= max_rel)
                                                   for p, r in zip(prev, log)]
    # the logged relevant fraction of iterate m equals L1 / (L1 + 4 S1 S2) >= 1e-3
    # counted on the host from that iterate (a solve stopped after m iterations)
    for m in (2, 6):
        pr.solve(tol=1e-11, pc=1, precision=0, pc_min_cg=0, pc_max_relevant=1.0, max_iter=m)
        b, z, n1, n2 = (pr.get(v).cpu().numpy() for v in (csipm.BETA, csipm.Z, csipm.NU1, csipm.NU2))
        s1, s2 = z + b, z - b
        num = n1 * s2 + n2 * s1
        frac = float(np.mean(num >= 1e-3 * (num + 4 * n1 * n2)))
        pr.solve(tol=1e-11, pc=1, precision=0, pc_min_cg=0, pc_max_relevant=1.0, max_iter=m + 1)
        logged = pr.log()[m]["relevant"]
        say("  iterate", m, "relevant fraction host", frac, "logged", logged)
        assert abs(logged - frac) <= 2.0 / b.size
    # a correction of 1e6 makes P_c a poor preconditioner: the learned
    # systems exceed the budget and restart with the paper's P
    bad = mlp.init_params(0, out_scale=0.0)
    bad[-1] = 1e6
    pr.set_pc_params(torch.tensor(bad.astype(np.float32), device="cuda"))
    info = pr.solve(tol=1e-11, pc=1, cg_max=30, pc_min_cg=0, pc_max_relevant=1.0)
    say("forced fallback", info)
    assert info["fallbacks"] > 0 and info["status"] == 3
    assert rel2(pr.get(csipm.BETA).cpu().numpy(), ref.state.beta) <= 1e-7
    c = pr.get(csipm.PC_C).cpu().numpy()
    assert np.all(c > 0)


@pytest.mark.parametrize("precision", [0, 1])
def test_corrected_system_patched_in_place_matches_separate_build(precision):
    """With the correction on every system, the systems the iterate update
    builds with the paper's P are turned into corrected ones in place
    (correction_patch: c, p = P_c^{-1} r where c acts, the start sums) instead
    of the correction pass plus a newton_init rebuild; against build_next = 0
    the solve reaches the same solution up to rounding.  FP64: the same
    interior-point and Krylov counts.  FP32 (stopped at 1e-11, near its
    floor, with the correction on every system): the two roundings agree on
    the first Krylov counts and then drift, and the last system can exceed
    its budget and fall back, so the interior-point counts may differ by one."""
    torch = need_gpu()
    from paper_2502_04217_amd import csipm
    w = wl.grid64(1)
    lam = ipm.lambda_rule(w.signal, w.observed)
    pr = csipm.Problem(w.signal, w.observed)
    pr.set_lambda(lam)
    pr.set_pc_params(torch.tensor(_params(3), device="cuda"))
    out = {}
    for bn in (1, 0):
        pr.timing(True)
        info = pr.solve(tol=1e-11, precision=precision, pc=csipm.PC_LEARNED, pc_min_cg=0, pc_max_relevant=1.0,
                        build_next=bn)
        rep = {r["name"]: r["calls"] for r in pr.timing_report(0.0)}
        pr.timing(False)
        patched = sum(c for nm, c in rep.items() if nm.startswith("correction_patch"))
        separate = rep.get("correction", 0)
        ninit = sum(c for nm, c in rep.items() if nm.startswith("newton_init"))
        log = pr.log()
        out[bn] = (info, [r["cg_iters"] for r in log], pr.get(csipm.BETA).cpu().numpy(), patched, separate, ninit)
        say("  build_next", bn, info["status_name"], info["ipm_iters"], out[bn][1], "fallbacks", info["fallbacks"],
            "patched", patched, "separate", separate, "newton_init", ninit)
        assert all(r["learned"] == 1 for r in log)
    (i1, cg1, b1, p1, s1, n1), (i0, cg0, b0, p0, s0, n0) = out[1], out[0]
    assert i1["status"] in (0, 3) and i0["status"] in (0, 3)
    if precision == 0:
        assert i1["ipm_iters"] == i0["ipm_iters"]
        assert cg1 == cg0
    else:
        assert abs(i1["ipm_iters"] - i0["ipm_iters"]) <= 1
        assert cg1[:8] == cg0[:8]
    assert p0 == 0 and s0 == i0["ipm_iters"]
    assert p1 > 0 and p1 + s1 == i1["ipm_iters"] and n1 < n0
    err = rel2(b1, b0)
    say("  rel diff", err)
    assert err <= (1e-12 if precision == 0 else 1e-7)
    ref = ipm.ipm_solve(w.signal, w.observed, lam, ipm.IPMOptions(tol=1e-11))
    assert rel2(b1, ref.state.beta) <= 1e-7


def test_capture_records_consistent():
    torch = need_gpu()
    from paper_2502_04217_amd import csipm
    w = wl.grid16(1)
    pr = csipm.Problem(w.signal, w.observed)
    pr.lambda_rule(0.05)
    per, mx = 256, 40
    feat = torch.zeros((per * mx, 4), dtype=torch.float32, device="cuda")
    rec = torch.zeros((per * mx, 6), dtype=torch.float32, device="cuda")
    pr.capture(feat, rec, per, mx, seed=11)
    info = pr.solve(tol=1e-8)
    k, cg = pr.captured()
    assert k == info["ipm_iters"] and len(cg) == k
    r = rec[:k * per].cpu().numpy()
    f = feat[:k * per].cpu().numpy()
    assert np.all(r[:, 2] > 0) and np.all(np.abs(r[:, 3]) <= r[:, 2] * (1 + 1e-6)) and np.all(r[:, 4] > 0)
    assert np.allclose(f[:, 1], r[:, 3] / r[:, 2], rtol=1e-4, atol=1e-6)
    for i in range(k):
        wsum = r[i * per:(i + 1) * per, 5]
        assert np.allclose(wsum, wsum[0]) and wsum[0] > 0
    pr.capture_off()


def test_policy_capture_records():
    """Capture mode 2 (csipm_capture): only at the iterations where the
    learned form would apply the correction (previous system >= pc_min_cg
    PCG iterations, 1 <= relevant coefficients <= pc_max_relevant of them),
    and only at coefficients where the correction can act."""
    torch = need_gpu()
    from paper_2502_04217_amd import csipm
    w = wl.grid64(1)
    pr = csipm.Problem(w.signal, w.observed)
    pr.lambda_rule(0.05)
    n = w.signal.size
    per, mx = 512, 40
    feat = torch.zeros((per * mx, 4), dtype=torch.float32, device="cuda")
    rec = torch.zeros((per * mx, 6), dtype=torch.float32, device="cuda")
    pr.capture(feat, rec, per, mx, seed=7, policy=True)
    info = pr.solve(tol=1e-8, precision=csipm.FP64, pc=csipm.PC_PLAIN, pc_min_cg=2, pc_max_relevant=0.5)
    k, cg = pr.captured()
    log = pr.log()
    prev = [0] + [r["cg_iters"] for r in log[:-1]]
    want = [i for i, (p, r) in enumerate(zip(prev, log))
            if p >= 2 and r["relevant"] * n >= 0.5 and r["relevant"] <= 0.5]
    say("policy capture", info["ipm_iters"], "iterations, captured", k, "expected at", want,
        "relevant", [round(r["relevant"], 5) for r in log])
    assert k == len(want) and k >= 1
    assert cg == [log[i]["cg_iters"] for i in want]
    r = rec[:k * per].cpu().numpy().astype(np.float64)
    L1, q4 = r[:, 2], r[:, 4]
    assert np.all(L1 >= 1e-3 * (L1 + q4) * (1 - 1e-5))
    assert np.all(r[:, 5] > 0)
    f = feat[:k * per].cpu().numpy()
    assert np.allclose(f[:, 1], r[:, 3] / r[:, 2], rtol=1e-4, atol=1e-6)
    # the same solve without the policy captures every iteration
    pr.capture(feat, rec, per, mx, seed=7)
    info2 = pr.solve(tol=1e-8, precision=csipm.FP64, pc=csipm.PC_PLAIN)
    assert pr.captured()[0] == info2["ipm_iters"]
    pr.capture_off()


PARAMS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2502_04217_amd",
                      "pc_params.json")


@pytest.mark.skipif(not os.path.exists(PARAMS), reason="no trained parameters committed")
def test_trained_network_on_held_out_problems():
    """Held-out 128^3 problems (the first 8 of the 50 in
    profiles/learned_eval_128cubed.md): the trained correction reaches the
    same true KKT residual as the paper's preconditioner with no more PCG
    iterations in either form (the 50-seed record: 0.984x in FP64, 0.970x in
    FP32), and no slowdown beyond 10 % (the record: 1.025x and 1.020x the time;
    at 128^3 the inference on the last systems costs about what the saved
    iterations gain; at 256^3 it pays, test_trained_network_gains_at_256)."""
    torch = need_gpu()
    from paper_2502_04217_amd import csipm, learn
    with open(PARAMS) as fh:
        params = torch.tensor(json.load(fh)["params"], dtype=torch.float32, device="cuda")
    rows = learn.evaluate(params, list(range(10000, 10008)), log=say)
    s = learn.summarize(rows)
    say("held-out summary", json.dumps(s))
    assert s["fp64_learned"]["max_true_rel_kkt"] <= 1e-6
    assert s["fp32_learned"]["max_true_rel_kkt"] <= 1e-6
    assert s["fp64_learned"]["fallbacks"] == 0 and s["fp32_learned"]["fallbacks"] == 0
    assert s["cg_ratio_fp64"] <= 1.0
    assert s["cg_ratio_fp32"] <= 1.0
    assert s["time_ratio_fp64"] <= 1.10
    assert s["time_ratio_fp32"] <= 1.10


@pytest.mark.skipif(not os.path.exists(PARAMS), reason="no trained parameters committed")
def test_trained_network_gains_at_256():
    """Problems of the 256^3 recipe the network never saw (it trains on 128^3
    problems only; seeds 1-3 of the 8 in profiles/learned_eval_256cubed.md,
    whose totals are 0.938x (FP64) and 0.881x (FP32) the PCG iterations and
    0.964x and 0.948x the time of the paper's preconditioner): on every seed
    and in both forms the trained correction takes fewer PCG iterations than
    the paper's P, reaches the same true KKT residual with no fallback, and the
    FP32 form, the chosen one, takes less time in total."""
    torch = need_gpu()
    from paper_2502_04217_amd import learn
    with open(PARAMS) as fh:
        params = torch.tensor(json.load(fh)["params"], dtype=torch.float32, device="cuda")
    rows = learn.evaluate(params, [1, 2, 3], log=say, grid=256)
    for r in rows:
        assert r["fp64_learned"]["cg"] < r["fp64_plain"]["cg"], r["seed"]
        assert r["fp32_learned"]["cg"] < r["fp32_plain"]["cg"], r["seed"]
        for k in ("fp64_learned", "fp32_learned"):
            assert r[k]["rel_kkt"] <= 1e-6 and r[k]["fallbacks"] == 0 and r[k]["status"] == 0
    s = learn.summarize(rows)
    say("256^3 summary", json.dumps(s))
    assert s["time_ratio_fp32"] < 1.0


def test_learned_form_outside_its_training_range_is_the_papers_P():
    """A problem with 0.08 % of its samples missing (period-32 lattice cubes
    of half-width 1 at 64^3), below the training range the default
    pc_min_missing = 0.01 guards: the learned form solves exactly as the
    paper's P (bit for bit, no corrected system); with the guard off
    (pc_min_missing = 0) the correction is applied."""
    torch = need_gpu()
    from paper_2502_04217_amd import csipm
    w = wl.make_workload((64, 64, 64), n_freq=200, amplitude="normal", snr_db=15.0, half_width=1, period=32, seed=3)
    assert w.missing_fraction < 0.01
    pr = csipm.Problem(w.signal, w.observed)
    pr.lambda_rule(0.05)
    pr.set_pc_params(torch.tensor(_params(3), device="cuda"))
    for prec in (0, 1):
        ip = pr.solve(tol=1e-8, precision=prec, pc=csipm.PC_PLAIN)
        bp = pr.get(csipm.BETA).cpu().numpy()
        il = pr.solve(tol=1e-8, precision=prec, pc=csipm.PC_LEARNED, pc_min_cg=0, pc_max_relevant=1.0)
        bl = pr.get(csipm.BETA).cpu().numpy()
        say("  guarded", prec, ip["cg_iters_total"], il["cg_iters_total"], [r["learned"] for r in pr.log()])
        assert all(r["learned"] == 0 for r in pr.log())
        assert il["cg_iters_total"] == ip["cg_iters_total"] and il["ipm_iters"] == ip["ipm_iters"]
        assert np.array_equal(bl, bp)
        pr.solve(tol=1e-8, precision=prec, pc=csipm.PC_LEARNED, pc_min_cg=0, pc_max_relevant=1.0, pc_min_missing=0.0)
        assert all(r["learned"] == 1 for r in pr.log())
