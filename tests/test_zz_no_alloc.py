"""csipm_mlp_loss_grad_noalloc (the loss-gradient entry point for callers
that cannot allocate) against csipm_mlp_loss_grad, through the C-ABI: two
calls in a row on one GPU, the second with fewer records, each equal bit
for bit to the workspace version on the same inputs (same kernels, same
reduction order; the fixed partials array keeps the first call's larger
contents when the second runs); a call beyond the maximum record count is
rejected with ENOMEM and queues nothing."""
import numpy as np
import pytest

from oracle import mlp
from tests._gpu_common import need_gpu, say

pytestmark = pytest.mark.gpu


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    feats = np.stack([rng.normal(0, 2, n), rng.uniform(-1, 1, n), rng.uniform(-27, 0, n),
                      rng.uniform(0.8, 1.0, n)], axis=1).astype(np.float32)
    s1 = np.exp(rng.uniform(-3, 3, n))
    s2 = np.exp(rng.uniform(-3, 3, n))
    rec = np.stack([rng.standard_normal(n), rng.standard_normal(n), s1 + s2, s1 - s2, 4 * s1 * s2,
                    rng.uniform(0.5, 1.5, n) / n], axis=1).astype(np.float32)
    return feats, rec


def test_noalloc_loss_grad_matches_workspace_version():
    torch = need_gpu()
    from paper_2502_04217_amd import csipm
    p = mlp.init_params(3, out_scale=0.5) + 0.05 * np.random.default_rng(3).standard_normal(mlp.N_PARAMS)
    tp = torch.tensor(p.astype(np.float32), device="cuda")
    for n, seed in ((csipm.NOALLOC_MAX_REC, 1), (4097, 2)):   # the second call is smaller
        say("noalloc loss_grad n =", n)
        f, r = _inputs(n, seed)
        tf, tr = torch.tensor(f, device="cuda"), torch.tensor(r, device="cuda")
        loss = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        grad = torch.full((csipm.MLP_PARAMS,), float("nan"), dtype=torch.float32, device="cuda")
        csipm.mlp_loss_grad_noalloc(tp, tf, tr, loss, grad)
        ref_loss, ref_grad = csipm.mlp_loss_grad(tp, tf, tr)
        torch.cuda.synchronize()
        assert torch.isfinite(grad).all() and bool(torch.isfinite(loss).all())
        assert torch.equal(loss, ref_loss) and torch.equal(grad, ref_grad)


def test_noalloc_rejects_more_records_than_its_scratch():
    torch = need_gpu()
    from paper_2502_04217_amd import csipm
    n = csipm.NOALLOC_MAX_REC + 1
    tp = torch.zeros(csipm.MLP_PARAMS, dtype=torch.float32, device="cuda")
    tf = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    tr = torch.ones((n, 6), dtype=torch.float32, device="cuda")
    loss = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    grad = torch.full((csipm.MLP_PARAMS,), 7.0, dtype=torch.float32, device="cuda")
    with pytest.raises(csipm.CsipmError) as e:
        csipm.mlp_loss_grad_noalloc(tp, tf, tr, loss, grad)
    assert e.value.status == -2 and "exceeds the fixed scratch" in str(e.value)
    torch.cuda.synchronize()
    assert float(loss[0]) == 7.0 and bool((grad == 7.0).all())
