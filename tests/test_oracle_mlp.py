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


# --- features and gate pinned by values worked out by hand -------------------
# Three coefficients with barrier diagonals chosen so that L1 = S1 + S2 and
# L2 = S1 - S2 are small integers:
#   S1 = (1, 2, 0.5), S2 = (1, 6, 1.5)  ->  L1 = (2, 8, 2), L2 = (0, -4, -1).
# log L1 = (ln 2, 3 ln 2, ln 2) has mean (5/3) ln 2, so
#   f1 = (-2/3 ln 2, 4/3 ln 2, -2/3 ln 2),   f2 = L2/L1 = (0, -1/2, -1/2).
# beta = (0, -3, 1.5), max|beta| = 3:
#   f3 = (ln 1e-12, ln(1 + 1e-12), ln(1/2 + 1e-12)).
# A feature formed from log S1 (mean 0: f1 = (0, ln 2, -ln 2)) or from
# S1/L1 = (1/2, 1/4, 1/4) differs from these in every coefficient.
_HAND_S1 = np.array([1.0, 2.0, 0.5])
_HAND_S2 = np.array([1.0, 6.0, 1.5])
_HAND_BETA = np.array([0.0, -3.0, 1.5])
_HAND_DIAG = np.array([0.25, 0.5, 0.96875])
_LN2 = 0.6931471805599453
_HAND_F = np.array([[-2.0 / 3.0 * _LN2, 0.0, -27.631021115928547, 0.25],
                    [4.0 / 3.0 * _LN2, -0.5, 9.999778782798785e-13, 0.5],
                    [-2.0 / 3.0 * _LN2, -0.5, -0.6931471805579453, 0.96875]])


def test_features_hand_values():
    f = mlp.features(_HAND_S1, _HAND_S2, _HAND_BETA, _HAND_DIAG)
    assert f.shape == (3, 4)
    assert np.abs(f - _HAND_F).max() <= 1e-15 * 30


def _one_path(feature):
    """Parameters of a network whose output is o = tanh(tanh(x_feature)):
    W1[0][feature] = 1, W2[0][0] = 1, w3[0] = 1, every other weight and
    bias 0; the correction is then c = ln(1 + e^o) + 1e-6."""
    W1 = np.zeros((mlp.H1, mlp.NIN))
    W1[0, feature] = 1.0
    W2 = np.zeros((mlp.H2, mlp.H1))
    W2[0, 0] = 1.0
    w3 = np.zeros(mlp.H2)
    w3[0] = 1.0
    return mlp.pack(W1, np.zeros(mlp.H1), W2, np.zeros(mlp.H2), w3, 0.0)


@pytest.mark.parametrize("feature", [0, 1, 2, 3])
def test_forward_one_path_network_hand_values(feature):
    """Each feature routed alone through one hidden unit per layer: the
    output is ln(1 + exp(tanh(tanh(f)))) + 1e-6, written out here for the
    hand-evaluated features above.  A network that reads its inputs in
    another order, drops a layer or uses another output map fails."""
    import math
    c, _ = mlp.forward(_one_path(feature), _HAND_F)
    want = [math.log1p(math.exp(math.tanh(math.tanh(f)))) + 1e-6 for f in _HAND_F[:, feature]]
    assert np.abs(c - np.array(want)).max() <= 1e-15


def _gate_state(s1, s2):
    """An iterate with beta = 0 and z = 1 (so both slacks are 1) whose
    barrier diagonals are S1 = nu1, S2 = nu2."""
    k = len(s1)
    return np.zeros(k), np.ones(k), np.asarray(s1, float), np.asarray(s2, float)


def test_relevance_gate_either_side_of_threshold():
    """The correction acts where L1 >= 1e-3 (L1 + 4 S1 S2).  With S1 = S2 = s
    that is 2s >= 1e-3 (2s + 4s^2), i.e. s <= 499.5; with S1 = 1e4, S2 = 1 it
    is 10001 >= 1e-3 * 50001 (relevant), with S1 = S2 = 1e4 it is
    2e4 >= 1e-3 * 4.00002e8 (not).  s = 600 separates the reading 4 S1 S2
    from 2 S1 S2 (threshold s <= 999), and s = 499.4 / 499.6 sit either side
    of the true one."""
    s1 = [499.4, 499.6, 600.0, 1e4, 1e4, 1e-3]
    s2 = [499.4, 499.6, 600.0, 1.0, 1e4, 1e-3]
    want = np.array([True, False, False, True, False, True])
    beta, z, nu1, nu2 = _gate_state(s1, s2)
    diag = np.full(len(s1), 0.5)
    params = mlp.init_params(0, out_scale=0.0)
    params[-1] = 0.0      # c = ln 2 + 1e-6 wherever the network runs
    c, act = mlp.correction(params, beta, z, nu1, nu2, diag)
    assert np.array_equal(act, want)
    assert np.allclose(c[want], np.log(2.0) + 1e-6, rtol=0, atol=1e-15)
    assert np.all(c[~want] == 1.0)


def test_correction_features_come_from_the_iterate():
    """correction() forms S_j = nu_j / s_j with s1 = z + beta, s2 = z - beta:
    for beta = (0, -3, 1.5), z = 4 the slacks are s1 = (4, 1, 5.5),
    s2 = (4, 7, 2.5); nu1 = S1 s1 and nu2 = S2 s2 give back the hand
    diagonals above, so the one-path network on f2 returns the values of
    the hand features (all three coefficients relevant)."""
    import math
    z = np.full(3, 4.0)
    s1, s2 = z + _HAND_BETA, z - _HAND_BETA
    nu1, nu2 = _HAND_S1 * s1, _HAND_S2 * s2
    c, act = mlp.correction(_one_path(1), _HAND_BETA, z, nu1, nu2, _HAND_DIAG)
    assert np.all(act)
    want = [math.log1p(math.exp(math.tanh(math.tanh(f)))) + 1e-6 for f in _HAND_F[:, 1]]
    assert np.abs(c - np.array(want)).max() <= 1e-15
