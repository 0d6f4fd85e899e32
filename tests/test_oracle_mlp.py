"""Pins of the learned-correction oracle: gradients against central finite
differences, positivity of the correction, positive definiteness of the
corrected preconditioner, the closed-form inverse, the loss as the norm of
P_c^{-1}(K - P_c)p, and the first Adam step."""
import numpy as np
import pytest

from oracle import dft3, ipm, mlp
from paper_2502_04217_amd import workload as wl


def _records(n, seed):
    rng = np.random.default_rng(seed)
    feats = np.stack([rng.normal(0, 2, n), rng.uniform(-1, 1, n),
                      rng.uniform(-27, 0, n), rng.uniform(0.8, 1.0, n)], axis=1)
    s1, s2 = wl.random_barrier((n,), seed + 1, spread=3.0)
    u = rng.standard_normal(n)
    p = rng.standard_normal(n)
    w = rng.uniform(0.5, 1.5, n)
    return feats, u, p, s1 + s2, s1 - s2, 4 * s1 * s2, w


def test_param_count():
    assert mlp.N_PARAMS == 1249
    assert mlp.init_params(0).size == 1249


def test_gradient_central_differences():
    params = mlp.init_params(3, out_scale=0.5)
    params = params + 0.1 * np.random.default_rng(4).standard_normal(params.size)
    feats, u, p, L1, L2, S12, w = _records(64, 5)
    L, g = mlp.loss_and_grad(params, feats, u, p, L1, L2, S12, w)
    h = 1e-6
    idx = np.random.default_rng(6).choice(params.size, 80, replace=False)
    for i in idx:
        e = np.zeros_like(params); e[i] = h
        Lp, _ = mlp.loss_and_grad(params + e, feats, u, p, L1, L2, S12, w)
        Lm, _ = mlp.loss_and_grad(params - e, feats, u, p, L1, L2, S12, w)
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


def test_correction_positive_and_pc_spd():
    params = mlp.init_params(1, out_scale=5.0)
    feats, *_ = _records(500, 2)
    feats[:, 0] *= 50.0                     # drive the output far negative/positive
    c, _ = mlp.forward(params, feats)
    assert np.all(c > 0)
    s1, s2 = wl.random_barrier((500,), 9, spread=8.0)
    L1, L2 = s1 + s2, s1 - s2
    for i in range(500):
        blk = np.array([[c[i] + L1[i], L2[i]], [L2[i], L1[i]]])
        assert np.all(np.linalg.eigvalsh(blk / np.abs(blk).max()) > 0)
    # closed-form inverse of P_c (moderate spread keeps the round trip exact)
    s1, s2 = wl.random_barrier((500,), 10, spread=3.0)
    rng = np.random.default_rng(3)
    xb, xz = rng.standard_normal(500), rng.standard_normal(500)
    pb, pz = ipm.P_apply(xb, xz, s1, s2, c)
    yb, yz = ipm.Pinv_apply(pb, pz, s1, s2, c)
    assert np.abs(yb - xb).max() < 1e-9 and np.abs(yz - xz).max() < 1e-9


def test_loss_minimiser_is_jacobi_for_white_directions():
    """Over many iid directions the least-squares optimum of a common c_i
    is diag(M_perp^T M_perp)_i."""
    shape = (4, 4, 8)
    rng = np.random.default_rng(12)
    obs = (rng.random(shape) > 0.3).astype(np.float64)
    num = np.zeros(shape)
    den = np.zeros(shape)
    for _ in range(4000):
        p = rng.standard_normal(shape)
        u = dft3.apply_H(p, obs)
        num += u * p
        den += p * p
    assert np.abs(num / den - dft3.diag_H(obs)).max() < 0.05


def test_untrained_network_is_the_paper_preconditioner():
    c, _ = mlp.forward(mlp.init_params(0, out_scale=0.0), _records(10, 1)[0])
    assert np.allclose(c, 1.0 + mlp.C_FLOOR, atol=1e-12)


def test_loss_is_norm_of_preconditioned_deviation():
    """sum_i e_i(c) = ||P^{-1}(K - P_c) p||^2 with u = H p_beta and P the
    paper's preconditioner (c = 1)."""
    shape = (4, 4, 8)
    rng = np.random.default_rng(7)
    obs = (rng.random(shape) > 0.2).astype(np.float64)
    s1, s2 = wl.random_barrier(shape, 8, spread=2.0)
    c = rng.uniform(0.5, 1.5, shape)
    pb, pz = rng.standard_normal(shape), rng.standard_normal(shape)
    qb, qz = ipm.K_apply(pb, pz, s1, s2, obs)
    Pb, Pz = ipm.P_apply(pb, pz, s1, s2, c)
    yb, yz = ipm.Pinv_apply(qb - Pb, qz - Pz, s1, s2)
    direct = float(np.sum(yb ** 2) + np.sum(yz ** 2))
    u = dft3.apply_H(pb, obs)
    e, _ = mlp.record_loss(c.ravel(), u.ravel(), pb.ravel(), (s1 + s2).ravel(),
                           (s1 - s2).ravel(), (4 * s1 * s2).ravel(), 1.0)
    assert abs(e.sum() - direct) < 1e-10 * direct


def test_adam_first_step_is_lr_times_sign():
    p = np.zeros(5)
    g = np.array([3.0, -0.5, 1e-3, -20.0, 7.0])
    p1, m, v = mlp.adam_step(p, g, np.zeros(5), np.zeros(5), 1, 0.01, eps=0.0)
    assert np.allclose(p1, -0.01 * np.sign(g), rtol=1e-12)


def test_features_shape_and_ranges():
    shape = (4, 4, 4)
    s1, s2 = wl.random_barrier(shape, 1)
    beta = np.random.default_rng(2).standard_normal(shape)
    obs = np.ones(shape)
    f = mlp.features(s1, s2, beta, mlp.diag_H_closed_form(obs))
    assert f.shape == (64, 4)
    assert abs(f[:, 0].mean()) < 1e-12
    assert np.all(np.abs(f[:, 1]) < 1)
    assert f[:, 2].max() < 1e-11
    assert np.allclose(f[:, 3], 1.0)
