"""csipm_solve_small_batch (one kernel, one workgroup per problem) against
the oracle's interior-point solve, against the library's csipm_solve, and
batched against one problem at a time (bit for bit)."""
import numpy as np
import pytest

from oracle import ipm
from paper_2502_04217_amd import workload as wl
from tests._gpu_common import need_gpu, rel2, say

pytestmark = pytest.mark.gpu

TOL = 1e-11


def _batch(ws, lams=None, **kw):
    torch = need_gpu()
    from paper_2502_04217_amd import csipm
    sig = torch.tensor(np.stack([w.signal for w in ws]), device="cuda")
    obs = torch.tensor(np.stack([w.observed for w in ws]).astype(np.uint8), device="cuda")
    return csipm.solve_small_batch(sig, obs, lambdas=lams, **kw)


@pytest.mark.parametrize("shape", [(16, 16, 16), (9, 15, 7), (1, 16, 24), (8, 6, 5), (16, 16, 32), (32, 8, 9),
                                   (32, 32, 32), (24, 40, 12)],
                         ids=lambda s: "x".join(map(str, s)))
def test_small_batch_matches_oracle(shape):
    """Each problem of a batch reaches the oracle's LASSO solution (both
    stopped at rel_kkt 1e-11) with the oracle's interior-point iteration
    count up to one.  The shapes cover the register pencils (2 to 32), the
    direct DFTs of other lengths (with their scratch buffer), spectra in
    LDS (up to 128 KB) and in the workspace (32^3, 24 x 40 x 12)."""
    if shape == (16, 16, 16):
        ws = [wl.grid16(s) for s in (1, 2, 3)]
    else:
        ws = [wl.make_workload(shape, n_freq=12, amplitude="normal", snr_db=20.0, half_width=-1, period=1,
                               dropout=0.15, seed=s) for s in (1, 2)]
    lams = [ipm.lambda_rule(w.signal, w.observed) for w in ws]
    beta, info = _batch(ws, lams, tol=TOL)
    beta = beta.cpu().numpy()
    for k, w in enumerate(ws):
        ref = ipm.ipm_solve(w.signal, w.observed, lams[k], ipm.IPMOptions(tol=TOL))
        err = rel2(beta[k], ref.state.beta)
        say("small batch", shape, k, "status", info[k, 0], "ipm", info[k, 1], "oracle", ref.iters, "pcg",
            info[k, 2], "oracle", sum(ref.cg_iters), "rel_kkt", info[k, 3], "err", err)
        assert info[k, 0] == 0 and info[k, 3] <= TOL
        assert abs(info[k, 1] - ref.iters) <= 1
        assert info[k, 5] == lams[k]
        assert err <= 1e-7


def test_small_batch_bit_identical_to_one_at_a_time():
    """64 problems at 16^3 in one launch give the same bits as each problem
    launched alone, and the lambda rule on the device gives the host's
    lambda."""
    torch = need_gpu()
    ws = [wl.paper_synthetic(16, s) for s in range(64)]
    beta, info = _batch(ws, lambda_frac=0.05, tol=1e-8)
    beta = beta.cpu().numpy()
    assert (info[:, 0] == 0).all()
    for k in (0, 17, 63):
        b1, i1 = _batch([ws[k]], lambda_frac=0.05, tol=1e-8)
        assert np.array_equal(b1.cpu().numpy()[0], beta[k])
        assert np.array_equal(i1[0], info[k])
        lam = ipm.lambda_rule(ws[k].signal, ws[k].observed)
        assert abs(info[k, 5] - lam) <= 1e-12 * lam
    say("64 problems: ipm", info[:, 1].min(), "-", info[:, 1].max(), "pcg mean", info[:, 2].mean())


def test_small_batch_agrees_with_library_solve():
    """The same problems through csipm_solve (FP64, the paper's P): the same
    solution at rel_kkt 1e-11."""
    torch = need_gpu()
    from paper_2502_04217_amd import csipm
    ws = [wl.grid16(s) for s in (4, 5)]
    lams = [ipm.lambda_rule(w.signal, w.observed) for w in ws]
    beta, info = _batch(ws, lams, tol=TOL)
    for k, w in enumerate(ws):
        pr = csipm.Problem(w.signal, w.observed)
        pr.set_lambda(lams[k])
        i = pr.solve(tol=TOL)
        b = pr.get(csipm.BETA).cpu().numpy()
        say("library", i["ipm_iters"], "small", info[k, 1], "diff", rel2(beta[k].cpu().numpy(), b))
        assert rel2(beta[k].cpu().numpy(), b) <= 1e-7


def test_small_batch_errors():
    torch = need_gpu()
    from paper_2502_04217_amd import csipm
    with pytest.raises(csipm.CsipmError) as e:
        csipm.solve_small_batch(np.zeros((1, 4, 4, 65)), np.ones((1, 4, 4, 65)))
    assert e.value.status == -5
    assert csipm.small_workspace_bytes((4, 4, 65), 1) == 0
    assert csipm.small_workspace_bytes((16, 16, 16), 2) > 0
    with pytest.raises(csipm.CsipmError) as e:   # no lambdas and no positive rule
        csipm.solve_small_batch(np.random.default_rng(0).standard_normal((1, 4, 4, 4)), np.ones((1, 4, 4, 4)),
                                lambda_frac=0.0)
    assert e.value.status == -1
