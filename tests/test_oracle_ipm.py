"""Pins of the oracle's interior-point method, condensed KKT system,
preconditioner and PCG (paper sections "KKT stationary conditions",
"Primal-dual interior-point method", "KKT linear systems", "Krylov methods and
preconditioners") against closed forms, dense linear algebra, an independent
bound-constrained optimiser (scipy L-BFGS-B) and invariants."""
import math

import numpy as np
import pytest
import scipy.optimize

from oracle import dft3, ipm
from paper_2502_04217_amd import workload as wl


def _barrier(shape, seed, spread=3.0):
    return wl.random_barrier(shape, seed, spread)


def test_pinv_closed_form_and_D():
    """P^{-1} P = I blockwise (equation "invprecond1"); D = S1 + S2 + 4 S1 S2
    (proposition "exprbd"); L1 D^{-1} lies in (0, 1) (equation "11block")."""
    shape = (4, 4, 4)
    s1, s2 = _barrier(shape, 1, spread=6.0)
    rng = np.random.default_rng(2)
    xb, xz = rng.standard_normal(shape), rng.standard_normal(shape)
    pb, pz = ipm.P_apply(xb, xz, s1, s2)
    yb, yz = ipm.Pinv_apply(pb, pz, s1, s2)
    assert np.abs(yb - xb).max() < 1e-9 * np.abs(xb).max()
    assert np.abs(yz - xz).max() < 1e-9 * np.abs(xz).max()
    t1, t2 = _barrier(shape, 3, spread=1.0)     # moderate spread: no cancellation
    L1, L2 = t1 + t2, t1 - t2
    D = L1 * (1 + L1) - L2 ** 2
    assert np.allclose(D, t1 + t2 + 4 * t1 * t2, rtol=1e-12)
    L1 = s1 + s2
    D = s1 + s2 + 4 * s1 * s2
    r = L1 / D
    assert np.all((r > 0) & (r < 1))
    # stable form of the (1,1) block
    assert np.allclose(r, (1 / s1 + 1 / s2) / (1 / s1 + 1 / s2 + 4), rtol=1e-12)


def test_preconditioned_operator_structure():
    """P^{-1} K = [[I + L1 D^{-1}(H - I), 0], [-D^{-1} L2 (H - I), I]]
    (equation "precond1"), checked on the dense 2n x 2n matrices."""
    shape = (2, 4, 4)
    n = 32
    rng = np.random.default_rng(4)
    obs = (rng.random(shape) > 0.3).astype(np.float64)
    s1, s2 = _barrier(shape, 5, spread=2.0)
    cols = []
    for i in range(2 * n):
        e = np.zeros(2 * n); e[i] = 1.0
        qb, qz = ipm.K_apply(e[:n].reshape(shape), e[n:].reshape(shape), s1, s2, obs)
        yb, yz = ipm.Pinv_apply(qb, qz, s1, s2)
        cols.append(np.concatenate([yb.ravel(), yz.ravel()]))
    PK = np.stack(cols, axis=1)
    A = dft3.dense_A(shape)
    Hd = A.T @ np.diag(obs.ravel()) @ A
    L1, L2 = (s1 + s2).ravel(), (s1 - s2).ravel()
    D = L1 + 4 * s1.ravel() * s2.ravel()
    I = np.eye(n)
    assert np.abs(PK[:n, :n] - (I + np.diag(L1 / D) @ (Hd - I))).max() < 1e-12
    assert np.abs(PK[:n, n:]).max() < 1e-12
    assert np.abs(PK[n:, n:] - I).max() < 1e-12
    assert np.abs(PK[n:, :n] - (-np.diag(L2 / D) @ (Hd - I))).max() < 1e-12


def test_condensed_step_equals_dense_newton_on_kktmu():
    """The condensed system with the oracle's right-hand side gives the same
    (d beta, d z) as a dense Newton step on the full perturbed KKT system
    (equation "kktmu", all eight blocks).  The Jacobian is formed by central
    differences, exact for this quadratic residual."""
    shape = (2, 4, 4)
    n = 32
    w = wl.make_workload(shape, n_freq=4, amplitude="normal", snr_db=10.0,
                         half_width=0, period=2, seed=3)
    obs = w.observed.astype(np.float64)
    xi = dft3.xi(w.signal, obs)
    lam = 0.1 * float(np.abs(xi).max())
    rng = np.random.default_rng(8)
    beta = 0.3 * rng.standard_normal(shape)
    z = np.abs(beta) + rng.uniform(0.1, 1.0, shape)
    nu1 = rng.uniform(0.1, 1.0, shape) * lam
    nu2 = rng.uniform(0.1, 1.0, shape) * lam
    st = ipm.IPMState(beta, z, nu1, nu2)
    s1, s2 = z + beta, z - beta
    sigma = 0.1
    mu = float((s1 * nu1).sum() + (s2 * nu2).sum()) / (2 * n)
    wvec = np.concatenate([a.ravel() for a in (beta, z, s1, s2, nu1, nu2, nu1, nu2)])
    F = ipm.kktmu_residual(wvec, xi, lam, obs, sigma * mu)
    J = np.zeros((8 * n, 8 * n))
    for i in range(8 * n):
        e = np.zeros(8 * n); e[i] = 1.0
        J[:, i] = (ipm.kktmu_residual(wvec + e, xi, lam, obs, sigma * mu)
                   - ipm.kktmu_residual(wvec - e, xi, lam, obs, sigma * mu)) / 2.0
    dw = np.linalg.solve(J, -F)
    Hb = dft3.apply_H(beta, obs)
    rb, rz = ipm.newton_rhs(st, Hb, xi, lam, sigma, mu)
    sig1, sig2 = nu1 / s1, nu2 / s2
    # dense condensed solve
    A = dft3.dense_A(shape)
    Hd = A.T @ np.diag(obs.ravel()) @ A
    L1, L2 = np.diag((sig1 + sig2).ravel()), np.diag((sig1 - sig2).ravel())
    Kd = np.block([[Hd + L1, L2], [L2, L1]])
    d = np.linalg.solve(Kd, np.concatenate([rb.ravel(), rz.ravel()]))
    assert np.abs(d[:n] - dw[:n]).max() < 1e-10
    assert np.abs(d[n:] - dw[n:2 * n]).max() < 1e-10
    # dual recovery matches the Newton step's nu blocks
    _, _, dnu1, dnu2 = ipm.recover_dnu(st, d[:n].reshape(shape), d[n:].reshape(shape),
                                       sig1, sig2, sigma, mu)
    assert np.abs(dnu1.ravel() - dw[6 * n:7 * n]).max() < 1e-9
    assert np.abs(dnu2.ravel() - dw[7 * n:]).max() < 1e-9
    # and PCG on the matrix-free K reaches the same direction
    res = ipm.pcg(lambda pb, pz: ipm.K_apply(pb, pz, sig1, sig2, obs),
                  lambda qb, qz: ipm.Pinv_apply(qb, qz, sig1, sig2), rb, rz, rtol=1e-14, maxit=400)
    assert np.abs(res.xb.ravel() - d[:n]).max() < 1e-9
    assert np.abs(res.xz.ravel() - d[n:]).max() < 1e-9


def test_predictor_corrector_steps_equal_dense_newton():
    """Mehrotra's two directions against dense Newton solves of "kktmu": the
    affine one with target 0, the corrector with target sigma mu and the
    complementarity rows shifted by d s_a * d nu_a of the affine step."""
    shape = (2, 4, 4)
    n = 32
    w = wl.make_workload(shape, n_freq=4, amplitude="normal", snr_db=10.0,
                         half_width=0, period=2, seed=5)
    obs = w.observed.astype(np.float64)
    xi = dft3.xi(w.signal, obs)
    lam = 0.1 * float(np.abs(xi).max())
    rng = np.random.default_rng(3)
    beta = 0.3 * rng.standard_normal(shape)
    z = np.abs(beta) + rng.uniform(0.1, 1.0, shape)
    nu1 = rng.uniform(0.1, 1.0, shape) * lam
    nu2 = rng.uniform(0.1, 1.0, shape) * lam
    st = ipm.IPMState(beta, z, nu1, nu2)
    s1, s2 = z + beta, z - beta
    mu = float((s1 * nu1).sum() + (s2 * nu2).sum()) / (2 * n)
    wvec = np.concatenate([a.ravel() for a in (beta, z, s1, s2, nu1, nu2, nu1, nu2)])

    def jac(target):
        J = np.zeros((8 * n, 8 * n))
        for i in range(8 * n):
            e = np.zeros(8 * n); e[i] = 1.0
            J[:, i] = (ipm.kktmu_residual(wvec + e, xi, lam, obs, target)
                       - ipm.kktmu_residual(wvec - e, xi, lam, obs, target)) / 2.0
        return J
    A = dft3.dense_A(shape)
    Hd = A.T @ np.diag(obs.ravel()) @ A
    sig1, sig2 = nu1 / s1, nu2 / s2
    L1, L2 = np.diag((sig1 + sig2).ravel()), np.diag((sig1 - sig2).ravel())
    Kd = np.block([[Hd + L1, L2], [L2, L1]])
    Hb = dft3.apply_H(beta, obs)
    # affine direction
    Fa = ipm.kktmu_residual(wvec, xi, lam, obs, 0.0)
    dwa = np.linalg.solve(jac(0.0), -Fa)
    da = np.linalg.solve(Kd, np.concatenate([a.ravel() for a in ipm.newton_rhs(st, Hb, xi, lam, 0.0, mu)]))
    assert np.abs(da - dwa[:2 * n]).max() < 1e-10
    ds1a, ds2a, dn1a, dn2a = ipm.recover_dnu(st, da[:n].reshape(shape), da[n:].reshape(shape), sig1, sig2, 0.0, mu)
    # corrector with sigma = 0.2
    sigma = 0.2
    corr = (ds1a * dn1a, ds2a * dn2a)
    F = ipm.kktmu_residual(wvec, xi, lam, obs, sigma * mu)
    F[6 * n:7 * n] += corr[0].ravel()
    F[7 * n:] += corr[1].ravel()
    dw = np.linalg.solve(jac(sigma * mu), -F)
    d = np.linalg.solve(Kd, np.concatenate([a.ravel() for a in ipm.newton_rhs(st, Hb, xi, lam, sigma, mu, corr)]))
    assert np.abs(d[:n] - dw[:n]).max() < 1e-10
    assert np.abs(d[n:] - dw[n:2 * n]).max() < 1e-10
    _, _, dnu1, dnu2 = ipm.recover_dnu(st, d[:n].reshape(shape), d[n:].reshape(shape), sig1, sig2, sigma, mu, corr)
    assert np.abs(dnu1.ravel() - dw[6 * n:7 * n]).max() < 1e-9
    assert np.abs(dnu2.ravel() - dw[7 * n:]).max() < 1e-9


def test_predictor_corrector_reaches_the_lasso_solution_in_fewer_iterations():
    for seed in (1, 4):
        w = wl.grid16(seed)
        lam = ipm.lambda_rule(w.signal, w.observed)
        ref = ipm.ipm_solve(w.signal, w.observed, lam, ipm.IPMOptions(tol=1e-11))
        mpc = ipm.ipm_solve(w.signal, w.observed, lam, ipm.IPMOptions(tol=1e-11, mehrotra=True))
        assert mpc.converged and mpc.iters < ref.iters
        err = np.linalg.norm(mpc.state.beta - ref.state.beta) / np.linalg.norm(ref.state.beta)
        assert err < 1e-8, err


def test_no_missing_closed_form_and_one_cg_step():
    """Nothing missing: H = I, K = P, so PCG converges in one iteration and
    the LASSO solution is soft(A^T b, lambda)."""
    shape = (8, 8, 8)
    w = wl.make_workload(shape, n_freq=20, amplitude="normal", snr_db=15.0,
                         half_width=-1, period=2, seed=4)
    assert w.observed.min() == 1
    lam = ipm.lambda_rule(w.signal, w.observed, 0.1)
    res = ipm.ipm_solve(w.signal, w.observed, lam, ipm.IPMOptions(tol=1e-11))
    assert res.converged
    # exact arithmetic gives one step; at tight tolerances round-off in the
    # large barrier diagonals can force one more
    assert max(res.cg_iters) <= 2
    exact = ipm.soft(dft3.xi(w.signal, w.observed), lam)
    assert np.abs(res.state.beta - exact).max() < 1e-8 * np.abs(exact).max()
    s1, s2 = wl.random_barrier(shape, 3, spread=3.0)
    obs = np.ones(shape)
    rng = np.random.default_rng(1)
    out = ipm.pcg(lambda pb, pz: ipm.K_apply(pb, pz, s1, s2, obs),
                  lambda qb, qz: ipm.Pinv_apply(qb, qz, s1, s2),
                  rng.standard_normal(shape), rng.standard_normal(shape), rtol=1e-9)
    assert out.iters == 1 and out.res_hist[1] < 1e-9 * out.res_hist[0]


def test_large_lambda_gives_zero():
    w = wl.grid16(2)
    lam = 1.01 * float(np.abs(dft3.xi(w.signal, w.observed)).max())
    res = ipm.ipm_solve(w.signal, w.observed, lam, ipm.IPMOptions(tol=1e-10))
    assert res.converged
    assert np.abs(res.state.beta).max() < 1e-8


def test_noiseless_planted_closed_form():
    """Noiseless planted spectrum with the right support S and signs:
    beta*_S = beta_S - lam (N_S^T N_S)^{-1} sign(beta_S), zero elsewhere,
    certified by |g_i| <= lam off S (N_S = columns S of M_perp)."""
    shape = (8, 8, 8)
    w = wl.make_workload(shape, n_freq=12, amplitude="lognormal", snr_db=np.inf,
                         half_width=1, period=4, seed=6)
    btrue = dft3.waves_to_beta(shape, w.wave_k, w.wave_c)
    A = dft3.dense_A(shape)
    obs = w.observed.ravel() == 1
    Mp = A[obs]
    S = np.nonzero(btrue.ravel())[0]
    lam = 0.02
    NS = Mp[:, S]
    bS = btrue.ravel()[S] - lam * np.linalg.solve(NS.T @ NS, np.sign(btrue.ravel()[S]))
    assert np.all(np.sign(bS) == np.sign(btrue.ravel()[S]))
    closed = np.zeros(A.shape[0]); closed[S] = bS
    g = Mp.T @ (w.signal.ravel()[obs] - Mp @ closed)
    off = np.setdiff1d(np.arange(A.shape[0]), S)
    assert np.abs(g[off]).max() < lam           # certificate holds: closed is optimal
    res = ipm.ipm_solve(w.signal, w.observed, lam, ipm.IPMOptions(tol=1e-11))
    assert res.converged
    assert np.linalg.norm(res.state.beta.ravel() - closed) < 1e-7 * np.linalg.norm(closed)


def test_matches_independent_bound_constrained_solver():
    """Same LASSO solved by scipy's L-BFGS-B on the split beta = u - w,
    u, w >= 0 (a smooth bound-constrained problem)."""
    shape = (4, 8, 8)
    w = wl.make_workload(shape, n_freq=10, amplitude="normal", snr_db=12.0,
                         half_width=1, period=4, seed=9)
    A = dft3.dense_A(shape)
    obs = w.observed.ravel() == 1
    Mp = A[obs]
    b = w.signal.ravel()[obs]
    lam = ipm.lambda_rule(w.signal, w.observed, 0.05)
    n = A.shape[0]

    def f(v):
        beta = v[:n] - v[n:]
        r = Mp @ beta - b
        g = Mp.T @ r
        return 0.5 * r @ r + lam * v.sum(), np.concatenate([g + lam, -g + lam])

    out = scipy.optimize.minimize(f, np.zeros(2 * n), jac=True, method="L-BFGS-B",
                                  bounds=[(0, None)] * (2 * n),
                                  options=dict(maxiter=20000, ftol=1e-16, gtol=1e-13, maxcor=50))
    ref = out.x[:n] - out.x[n:]
    res = ipm.ipm_solve(w.signal, w.observed, lam, ipm.IPMOptions(tol=1e-11))
    assert res.converged
    assert np.linalg.norm(res.state.beta.ravel() - ref) < 1e-6 * np.linalg.norm(ref)
    obj = lambda beta: 0.5 * np.sum((Mp @ beta - b) ** 2) + lam * np.abs(beta).sum()
    assert obj(res.state.beta.ravel()) <= obj(ref) + 1e-9 * abs(obj(ref))


def test_grid16_invariants_and_certificate():
    """On the 16^3 workload: positivity of s and nu at every iterate, mu
    decreasing, final LASSO optimality conditions and a vanishing duality gap,
    and the Sigma pattern of the corollary "convergencespeed" (Lambda_1 large
    everywhere, Sigma_1 small on I+, Sigma_2 small on I-)."""
    w = wl.grid16(1)
    lam = ipm.lambda_rule(w.signal, w.observed)
    seen = []

    def cb(it, st, res):
        s1, s2 = st.z + st.beta, st.z - st.beta
        assert s1.min() > 0 and s2.min() > 0 and st.nu1.min() > 0 and st.nu2.min() > 0
        seen.append(float(((s1 * st.nu1).sum() + (s2 * st.nu2).sum()) / (2 * s1.size)))

    res = ipm.ipm_solve(w.signal, w.observed, lam, ipm.IPMOptions(tol=1e-10), callback=cb)
    assert res.converged
    assert all(b < a for a, b in zip(seen, seen[1:]))
    cert = ipm.lasso_certificate(res.state.beta, w.signal, w.observed, lam)
    assert cert.natural_residual < 1e-7
    assert cert.rel_gap < 1e-6
    assert cert.max_offsupport_ratio <= 1.0 + 1e-6
    st = res.state
    s1, s2 = st.z + st.beta, st.z - st.beta
    sig1, sig2 = st.nu1 / s1, st.nu2 / s2
    supp = ipm.support(st.beta, 1e-3)
    pos = supp & (st.beta > 0)
    neg = supp & (st.beta < 0)
    assert pos.any() and neg.any()
    assert (sig1[pos].max() < 1e-3 * (sig1 + sig2)[pos].min())
    assert (sig2[neg].max() < 1e-3 * (sig1 + sig2)[neg].min())
    assert (sig1 + sig2).min() > 1e3


def test_limit_condition_number_tiny():
    """Near the end of the IPM, the spectrum of P^{-1}K approaches
    {1} U spec(Q*) (proposition "boundskappa"), Q* = (M^T M) on the active set."""
    shape = (4, 4, 4)
    w = wl.make_workload(shape, n_freq=4, amplitude="normal", snr_db=30.0,
                         half_width=0, period=2, seed=12)
    obs = w.observed.astype(np.float64)
    lam = ipm.lambda_rule(w.signal, w.observed, 0.05)
    res = ipm.ipm_solve(w.signal, w.observed, lam, ipm.IPMOptions(tol=1e-12))
    st = res.state
    s1, s2 = st.z + st.beta, st.z - st.beta
    sig1, sig2 = st.nu1 / s1, st.nu2 / s2
    n = obs.size
    cols = []
    for i in range(2 * n):
        e = np.zeros(2 * n); e[i] = 1.0
        qb, qz = ipm.K_apply(e[:n].reshape(shape), e[n:].reshape(shape), sig1, sig2, obs)
        yb, yz = ipm.Pinv_apply(qb, qz, sig1, sig2)
        cols.append(np.concatenate([yb.ravel(), yz.ravel()]))
    ev = np.sort(np.linalg.eigvals(np.stack(cols, axis=1)).real)
    A = dft3.dense_A(shape)
    Hd = A.T @ np.diag(obs.ravel()) @ A
    act = np.nonzero(ipm.support(st.beta, 1e-6).ravel())[0]
    q = np.linalg.eigvalsh(Hd[np.ix_(act, act)])
    expected = np.sort(np.concatenate([np.ones(2 * n - len(act)), q]))
    assert np.abs(ev - expected).max() < 1e-4


# ------------------------------------------------- CR and the scaled P --

def _dense_system(m, seed):
    """A random SPD 2m x 2m K with the block structure [[G + L1, L2], [L2, L1]]
    (G a random PSD matrix standing in for H) and random barrier diagonals."""
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((m, m // 2))
    G = B @ B.T / m
    s1 = np.exp(rng.uniform(-2, 2, m))
    s2 = np.exp(rng.uniform(-2, 2, m))
    L1, L2 = s1 + s2, s1 - s2
    K = np.block([[G + np.diag(L1), np.diag(L2)], [np.diag(L2), np.diag(L1)]])
    applyK = lambda pb, pz: (G @ pb + L1 * pb + L2 * pz, L2 * pb + L1 * pz)
    return K, applyK, s1, s2, rng


def test_pcr_solves_dense_system_and_is_exact_for_K_equal_P():
    m = 24
    K, applyK, s1, s2, rng = _dense_system(m, 5)
    b = rng.standard_normal(2 * m)
    pinv = lambda rb, rz: ipm.Pinv_apply(rb, rz, s1, s2)
    out = ipm.pcr(applyK, pinv, b[:m], b[m:], rtol=1e-13, maxit=200)
    x = np.linalg.solve(K, b)
    assert out.converged
    assert np.abs(np.concatenate([out.xb, out.xz]) - x).max() < 1e-10 * np.abs(x).max()
    # K = P (G = I): one step
    applyP = lambda pb, pz: ipm.P_apply(pb, pz, s1, s2)
    one = ipm.pcr(applyP, pinv, b[:m], b[m:], rtol=1e-10)
    assert one.iters == 1


def test_pcr_iterates_minimise_preconditioned_residual_over_krylov_space():
    """x_k = argmin over K_k(P^{-1}K, P^{-1}b) of (b - Kx)^T P^{-1} (b - Kx),
    computed by a dense weighted least-squares solve on the Krylov basis."""
    m = 20
    K, applyK, s1, s2, rng = _dense_system(m, 9)
    b = rng.standard_normal(2 * m)
    Pinv = np.zeros((2 * m, 2 * m))
    for j in range(2 * m):
        e = np.zeros(2 * m)
        e[j] = 1.0
        zb, zz = ipm.Pinv_apply(e[:m], e[m:], s1, s2)
        Pinv[:, j] = np.concatenate([zb, zz])
    pinv = lambda rb, rz: ipm.Pinv_apply(rb, rz, s1, s2)
    res_prev = math.inf
    for k in (1, 2, 3, 5):
        out = ipm.pcr(applyK, pinv, b[:m], b[m:], rtol=0.0, maxit=k)
        xk = np.concatenate([out.xb, out.xz])
        V = [Pinv @ b]
        for _ in range(k - 1):
            V.append(Pinv @ (K @ V[-1]))
        V = np.array(V).T
        KV = K @ V
        y = np.linalg.solve(KV.T @ Pinv @ KV, KV.T @ Pinv @ b)
        assert np.abs(xk - V @ y).max() < 1e-8 * np.abs(V @ y).max()
        r = b - K @ xk
        res = float(r @ Pinv @ r)
        assert res <= res_prev * (1 + 1e-12)
        res_prev = res


def test_pcar_solves_dense_system_and_is_exact_for_K_equal_P():
    m = 24
    K, applyK, s1, s2, rng = _dense_system(m, 6)
    b = rng.standard_normal(2 * m)
    pinv = lambda rb, rz: ipm.Pinv_apply(rb, rz, s1, s2)
    out = ipm.pcar(applyK, pinv, b[:m], b[m:], rtol=1e-12, maxit=300)
    x = np.linalg.solve(K, b)
    assert out.converged
    assert np.abs(np.concatenate([out.xb, out.xz]) - x).max() < 1e-9 * np.abs(x).max()
    applyP = lambda pb, pz: ipm.P_apply(pb, pz, s1, s2)
    one = ipm.pcar(applyP, pinv, b[:m], b[m:], rtol=1e-10)
    assert one.iters == 1


def test_pcar_iterates_minimise_preconditioned_A_residual_over_krylov_space():
    """x_k = argmin over K_k(P^{-1}K, P^{-1}b) of ||K P^{-1}(b - Kx)||_{P^{-1}}
    (dense weighted least squares on the Krylov basis); that norm decreases
    monotonically, and so does the preconditioned residual."""
    m = 20
    K, applyK, s1, s2, rng = _dense_system(m, 10)
    b = rng.standard_normal(2 * m)
    Pinv = np.zeros((2 * m, 2 * m))
    for j in range(2 * m):
        e = np.zeros(2 * m)
        e[j] = 1.0
        zb, zz = ipm.Pinv_apply(e[:m], e[m:], s1, s2)
        Pinv[:, j] = np.concatenate([zb, zz])
    pinv = lambda rb, rz: ipm.Pinv_apply(rb, rz, s1, s2)
    W = K @ Pinv                     # r -> K P^{-1} r, the A-residual
    prev_a = prev_r = math.inf
    for k in (1, 2, 3, 5, 8):
        out = ipm.pcar(applyK, pinv, b[:m], b[m:], rtol=0.0, maxit=k)
        xk = np.concatenate([out.xb, out.xz])
        V = [Pinv @ b]
        for _ in range(k - 1):
            V.append(Pinv @ (K @ V[-1]))
        V = np.linalg.qr(np.array(V).T)[0]       # orthonormal basis of the same space
        G = W @ K @ V
        y = np.linalg.solve(G.T @ Pinv @ G, G.T @ Pinv @ (W @ b))
        assert np.abs(xk - V @ y).max() < 1e-7 * np.abs(V @ y).max()
        r = b - K @ xk
        a = float((W @ r) @ Pinv @ (W @ r))
        res = float(r @ Pinv @ r)
        assert a <= prev_a * (1 + 1e-12) and res <= prev_r * (1 + 1e-12)
        prev_a, prev_r = a, res


def test_cr_and_scaled_preconditioner_reach_the_lasso_solution():
    """The Krylov method and the preconditioner change only how each Newton
    system is solved: CR, CAr, and the scaled-identity P with rho = m/n,
    reach the solution of the plain PCG solve."""
    w = wl.grid16(4)
    lam = ipm.lambda_rule(w.signal, w.observed)
    ref = ipm.ipm_solve(w.signal, w.observed, lam, ipm.IPMOptions(tol=1e-11))
    rho = float(w.observed.mean())
    for opts in (ipm.IPMOptions(tol=1e-11, krylov="cr"), ipm.IPMOptions(tol=1e-11, pc_rho=rho),
                 ipm.IPMOptions(tol=1e-11, krylov="cr", pc_rho=rho)):
        res = ipm.ipm_solve(w.signal, w.observed, lam, opts)
        assert res.converged
        err = np.linalg.norm(res.state.beta - ref.state.beta) / np.linalg.norm(ref.state.beta)
        assert err < 1e-8, (opts, err)
    # CAr minimises ||K z||_{P^{-1}}, which reaches its floating-point floor
    # near a 1e-9 relative residual on these systems: compared at 1e-9, where
    # it takes the same interior-point and Krylov steps as CG
    cg9 = ipm.ipm_solve(w.signal, w.observed, lam, ipm.IPMOptions(tol=1e-9))
    car9 = ipm.ipm_solve(w.signal, w.observed, lam, ipm.IPMOptions(tol=1e-9, krylov="car"))
    assert car9.converged and car9.iters == cg9.iters
    err = np.linalg.norm(car9.state.beta - cg9.state.beta) / np.linalg.norm(cg9.state.beta)
    assert err < 1e-8, err


def test_duality_measure_after_step_from_step_sums():
    """The duality measure after a step of length alpha along a Newton
    direction is (s.nu + alpha (s.dnu + nu.ds) + alpha^2 ds.dnu) / 2n, with
    s_j dnu_j + nu_j ds_j = sigma mu - s_j nu_j elementwise (the
    linearised complementarity rows of equation "kktmu").  The iterate
    update that also builds the next Newton system takes its target from
    these sums; here they are checked against the product of the stepped
    iterate."""
    shape = (4, 4, 6)
    n = 96
    w = wl.make_workload(shape, n_freq=5, amplitude="normal", snr_db=10.0,
                         half_width=0, period=2, seed=5)
    obs = w.observed.astype(np.float64)
    xi = dft3.xi(w.signal, obs)
    lam = 0.1 * float(np.abs(xi).max())
    rng = np.random.default_rng(11)
    beta = 0.3 * rng.standard_normal(shape)
    z = np.abs(beta) + rng.uniform(0.1, 1.0, shape)
    nu1 = rng.uniform(0.1, 1.0, shape) * lam
    nu2 = rng.uniform(0.1, 1.0, shape) * lam
    st = ipm.IPMState(beta, z, nu1, nu2)
    s1, s2 = z + beta, z - beta
    sig1, sig2 = nu1 / s1, nu2 / s2
    sigma = 0.1
    mu = float((s1 * nu1).sum() + (s2 * nu2).sum()) / (2 * n)
    rb, rz = ipm.newton_rhs(st, dft3.apply_H(beta, obs), xi, lam, sigma, mu)
    res = ipm.pcg(lambda pb, pz: ipm.K_apply(pb, pz, sig1, sig2, obs),
                  lambda qb, qz: ipm.Pinv_apply(qb, qz, sig1, sig2), rb, rz, rtol=1e-13, maxit=400)
    ds1, ds2, dnu1, dnu2 = ipm.recover_dnu(st, res.xb, res.xz, sig1, sig2, sigma, mu)
    assert np.allclose(s1 * dnu1 + nu1 * ds1, sigma * mu - s1 * nu1, rtol=0, atol=1e-12 * lam)
    assert np.allclose(s2 * dnu2 + nu2 * ds2, sigma * mu - s2 * nu2, rtol=0, atol=1e-12 * lam)
    amax = min(ipm.max_step(s1, ds1), ipm.max_step(s2, ds2), ipm.max_step(nu1, dnu1), ipm.max_step(nu2, dnu2))
    S0 = float((s1 * nu1).sum() + (s2 * nu2).sum())
    S1 = float((s1 * dnu1 + nu1 * ds1).sum() + (s2 * dnu2 + nu2 * ds2).sum())
    S2 = float((ds1 * dnu1).sum() + (ds2 * dnu2).sum())
    for alpha in (0.0, 0.3, min(1.0, 0.99 * amax)):
        direct = float(((s1 + alpha * ds1) * (nu1 + alpha * dnu1)).sum()
                       + ((s2 + alpha * ds2) * (nu2 + alpha * dnu2)).sum()) / (2 * n)
        from_sums = (S0 + alpha * S1 + alpha * alpha * S2) / (2 * n)
        assert abs(from_sums - direct) <= 1e-13 * S0 / (2 * n)
