"""Primal-dual interior-point method for the l1-penalised least squares
problem, with PCG on the condensed KKT system (oracle; test infrastructure).

Problem (paper, equation "realopt"):
    beta* = argmin_beta  1/2 ||b - M_perp beta||^2 + lambda ||beta||_1,
rewritten with z and slacks s1 = z + beta >= 0, s2 = z - beta >= 0
(equations "problem", "slackproblem"); multipliers y = nu (equation "kkt").

Readings where the paper is silent (the barrier strategy "depends on the IPM
implementation"):
  * the slacks are eliminated, s1 = z + beta and s2 = z - beta, so the two
    equality constraints hold exactly at every iterate;
  * start: beta = 0, z = ||xi||_inf * e (1 if xi = 0), nu1 = nu2 = lambda/2;
  * each iteration takes one Newton step on the perturbed KKT system
    (equation "kktmu") with centring target sigma*mu, sigma = 0.1 fixed,
    mu = (s1.nu1 + s2.nu2)/(2n) (the duality measure of the paper);
  * the step is solved in condensed form K [dbeta; dz] = [r_beta; r_z]
    (equation "condensedkkt": K = [[H + L1, L2], [L2, L1]], L1 = S1 + S2,
    L2 = S1 - S2, S_j = nu_j / s_j) with the Newton right-hand side derived
    from "kktmu" directly:
        r_beta = -(H beta - xi) + sigma mu (1/s1 - 1/s2)
        r_z    = -lambda e      + sigma mu (1/s1 + 1/s2)
    (the printed r_6 and the sign of the Delta s entries in "augkkt" contain
    typos; the test suite checks this RHS against a dense Newton solve of
    "kktmu" itself);
  * d nu_j = sigma mu / s_j - nu_j - S_j d s_j, with d s1 = dbeta + dz,
    d s2 = dz - dbeta;
  * one common step length alpha = min(1, tau * max step keeping s, nu > 0),
    tau = 0.99;
  * as an option (mehrotra), Mehrotra's predictor-corrector: an affine
    direction (sigma = 0), its step to the boundary alpha_a (at most 1) and
    mu_a = (s + alpha_a ds).(nu + alpha_a dnu)/(2n); sigma = (mu_a/mu)^3,
    at least 0.1 tol (1 + ||xi||_inf) / mu; then the corrector, a second
    solve with the same K whose complementarity rows carry - ds_a dnu_a;
  * stop when rel_kkt = max(||F_beta||_inf, ||F_z||_inf, max_i s_i nu_i)
    / (1 + ||xi||_inf) <= tol, where F_beta = H beta - xi - nu1 + nu2 and
    F_z = lambda e - nu1 - nu2 are the first two rows of "kkt";
  * K is solved by textbook PCG (or, as an option, preconditioned CR) with
    the paper's preconditioner
    P = [[I + L1, L2], [L2, L1]] (section "Krylov methods and
    preconditioners"; as an option its scaled-identity relative
    [[rho I + L1, L2], [L2, L1]], the variant the paper attributes to earlier
    work, with rho tied to the observed fraction), x0 = 0, stopping on the
    preconditioned residual norm
    sqrt(r^T P^{-1} r) <= max(cg_atol, eta sqrt(r0^T P^{-1} r0)),
    eta = min(cg_rtol, 0.1 rel_kkt).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import dft3


# ---------------------------------------------------------------- operators --

def K_apply(pb, pz, sig1, sig2, observed):
    """q = K p for K = [[H + L1, L2], [L2, L1]] (equation "condensedkkt")."""
    L1 = sig1 + sig2
    L2 = sig1 - sig2
    qb = dft3.apply_H(pb, observed) + L1 * pb + L2 * pz
    qz = L2 * pb + L1 * pz
    return qb, qz


def P_apply(pb, pz, sig1, sig2, c=None):
    """P p for P = [[C + L1, L2], [L2, L1]]; C = I for the paper's
    preconditioner, C = diag(c) for the learned correction."""
    L1 = sig1 + sig2
    L2 = sig1 - sig2
    cc = 1.0 if c is None else c
    return (cc + L1) * pb + L2 * pz, L2 * pb + L1 * pz


def Pinv_apply(rb, rz, sig1, sig2, c=None):
    """P^{-1} r from the closed form (equation "invprecond1"):
    P^{-1} = [[L1 D^{-1}, -L2 D^{-1}], [-D^{-1} L2, (C + L1) D^{-1}]] with
    D = C L1 + 4 S1 S2 (= S1 + S2 + 4 S1 S2 for C = I, proposition
    "exprbd")."""
    L1 = sig1 + sig2
    L2 = sig1 - sig2
    cc = 1.0 if c is None else c
    D = cc * L1 + 4.0 * sig1 * sig2
    return (L1 * rb - L2 * rz) / D, (-L2 * rb + (cc + L1) * rz) / D


def soft(x, lam):
    """Soft threshold sign(x) max(|x| - lam, 0)."""
    return np.sign(x) * np.maximum(np.abs(x) - lam, 0.0)


# ---------------------------------------------------------------------- PCG --

@dataclasses.dataclass
class PCGResult:
    xb: np.ndarray
    xz: np.ndarray
    iters: int
    res_hist: list          # sqrt(r^T P^{-1} r) before each iteration and at exit
    converged: bool


def pcg(apply_K, apply_Pinv, rb, rz, *, atol=0.0, rtol=1e-10, maxit=500):
    """Textbook preconditioned conjugate gradients (Hestenes-Stiefel) on the
    2n-vector (b, z) blocks, x0 = 0."""
    xb = np.zeros_like(rb)
    xz = np.zeros_like(rz)
    rb = rb.copy()
    rz = rz.copy()
    zb, zz = apply_Pinv(rb, rz)
    pb, pz = zb.copy(), zz.copy()
    rho = float(np.sum(rb * zb) + np.sum(rz * zz))
    hist = [math.sqrt(max(rho, 0.0))]
    tol = max(atol, rtol * hist[0])
    it = 0
    while hist[-1] > tol and it < maxit:
        qb, qz = apply_K(pb, pz)
        pq = float(np.sum(pb * qb) + np.sum(pz * qz))
        alpha = rho / pq
        xb += alpha * pb
        xz += alpha * pz
        rb -= alpha * qb
        rz -= alpha * qz
        zb, zz = apply_Pinv(rb, rz)
        rho_new = float(np.sum(rb * zb) + np.sum(rz * zz))
        beta = rho_new / rho
        rho = rho_new
        pb = zb + beta * pb
        pz = zz + beta * pz
        it += 1
        hist.append(math.sqrt(max(rho, 0.0)))
    return PCGResult(xb, xz, it, hist, hist[-1] <= tol)


def pcr(apply_K, apply_Pinv, rb, rz, *, atol=0.0, rtol=1e-10, maxit=500):
    """Preconditioned conjugate residuals (the CR method of Hestenes and
    Stiefel, which section "Krylov methods and preconditioners" lists beside
    CG) on the 2n-vector blocks, x0 = 0.  With z = P^{-1} r and w = K z,
    each step takes alpha = (z.w) / (q.P^{-1}q) along p, where q = K p, and
    the next direction p = z + beta p with beta = (z.w)_new / (z.w)_old
    (q = w + beta q follows without a second product).  The iterates
    minimise ||b - K x|| in the P^{-1} norm over the Krylov space.  Stops on
    the same preconditioned residual norm as pcg."""
    xb = np.zeros_like(rb)
    xz = np.zeros_like(rz)
    rb = rb.copy()
    rz = rz.copy()
    zb, zz = apply_Pinv(rb, rz)
    rho = float(np.sum(rb * zb) + np.sum(rz * zz))
    hist = [math.sqrt(max(rho, 0.0))]
    tol = max(atol, rtol * hist[0])
    it = 0
    zw_old = None
    pb = pz = qb = qz = None
    while hist[-1] > tol and it < maxit:
        wb, wz = apply_K(zb, zz)
        zw = float(np.sum(zb * wb) + np.sum(zz * wz))
        if zw_old is None:
            pb, pz, qb, qz = zb.copy(), zz.copy(), wb, wz
        else:
            beta = zw / zw_old
            pb, pz = zb + beta * pb, zz + beta * pz
            qb, qz = wb + beta * qb, wz + beta * qz
        ub, uz = apply_Pinv(qb, qz)
        alpha = zw / float(np.sum(qb * ub) + np.sum(qz * uz))
        xb += alpha * pb
        xz += alpha * pz
        rb -= alpha * qb
        rz -= alpha * qz
        zb, zz = apply_Pinv(rb, rz)
        zw_old = zw
        rho = float(np.sum(rb * zb) + np.sum(rz * zz))
        it += 1
        hist.append(math.sqrt(max(rho, 0.0)))
    return PCGResult(xb, xz, it, hist, hist[-1] <= tol)


def pcar(apply_K, apply_Pinv, rb, rz, *, atol=0.0, rtol=1e-10, maxit=500):
    """Preconditioned conjugate A-residuals (CAr, the third Krylov method that
    section "Krylov methods and preconditioners" lists for SPD systems, from
    the MinAres work it cites), x0 = 0.  With the split P = L L^T and the
    symmetric operator A = L^{-1} K L^{-T}, CAr is CG in the inner product
    <a, b> = a^T A^3 b: it minimises ||A r~|| = ||K z||_{P^{-1}} (z = P^{-1} r,
    the preconditioned A-residual) over the Krylov space.  Vectors, with
    w = K z and u = P^{-1} w:
      alpha = (u.s) / (t.P^{-1}t), where s = K u, and t = K v, v = P^{-1} q,
      q = K p along the direction p;
      x += alpha p,  r -= alpha q,  w -= alpha t,  then z, u, s anew;
      beta = (u.s)_new / (u.s)_old;  p = z + beta p, q = w + beta q,
      t = s + beta t  (v = P^{-1} q follows).
    One K product per step (s = K u).  Stops on the same preconditioned
    residual norm sqrt(r.P^{-1}r) as pcg, or when the A-residual has vanished
    in floating point (u.s or t.P^{-1}t no longer positive)."""
    xb = np.zeros_like(rb)
    xz = np.zeros_like(rz)
    rb = rb.copy()
    rz = rz.copy()
    zb, zz = apply_Pinv(rb, rz)
    rho = float(np.sum(rb * zb) + np.sum(rz * zz))
    hist = [math.sqrt(max(rho, 0.0))]
    tol = max(atol, rtol * hist[0])
    it = 0
    wb, wz = apply_K(zb, zz)
    ub, uz = apply_Pinv(wb, wz)
    sb, sz = apply_K(ub, uz)
    pb, pz, qb, qz, tb, tz = zb.copy(), zz.copy(), wb.copy(), wz.copy(), sb.copy(), sz.copy()
    us = float(np.sum(ub * sb) + np.sum(uz * sz))
    while hist[-1] > tol and it < maxit:
        yb, yz = apply_Pinv(tb, tz)
        den = float(np.sum(tb * yb) + np.sum(tz * yz))
        if not (den > 0.0 and us > 0.0):
            break           # the A-residual vanished in floating point: nothing left to minimise
        alpha = us / den
        xb += alpha * pb
        xz += alpha * pz
        rb -= alpha * qb
        rz -= alpha * qz
        wb -= alpha * tb
        wz -= alpha * tz
        zb, zz = apply_Pinv(rb, rz)
        ub, uz = apply_Pinv(wb, wz)
        sb, sz = apply_K(ub, uz)
        us_new = float(np.sum(ub * sb) + np.sum(uz * sz))
        beta = us_new / us
        us = us_new
        pb, pz = zb + beta * pb, zz + beta * pz
        qb, qz = wb + beta * qb, wz + beta * qz
        tb, tz = sb + beta * tb, sz + beta * tz
        rho = float(np.sum(rb * zb) + np.sum(rz * zz))
        it += 1
        hist.append(math.sqrt(max(rho, 0.0)))
    return PCGResult(xb, xz, it, hist, hist[-1] <= tol)


# ---------------------------------------------------------------------- IPM --

@dataclasses.dataclass
class IPMOptions:
    tol: float = 1e-6
    max_iter: int = 200
    sigma: float = 0.1
    tau: float = 0.99
    cg_max: int = 500
    cg_rtol: float = 1e-2
    cg_atol: float = 0.0
    krylov: str = "cg"              # "cg" (pcg), "cr" (pcr) or "car" (pcar)
    mehrotra: bool = False          # predictor-corrector steps (see ipm_solve)
    pc_rho: float | None = None     # C = rho I: the scaled-identity variant of P


@dataclasses.dataclass
class IPMState:
    beta: np.ndarray
    z: np.ndarray
    nu1: np.ndarray
    nu2: np.ndarray


@dataclasses.dataclass
class IPMResult:
    state: IPMState
    iters: int
    cg_iters: list
    rel_kkt: float
    mu: float
    converged: bool
    log: list


def kkt_parts(st: IPMState, xi, lam, observed):
    """(F_beta, F_z, s1, s2, comp_max, mu) of an iterate."""
    s1 = st.z + st.beta
    s2 = st.z - st.beta
    Hb = dft3.apply_H(st.beta, observed)
    Fb = Hb - xi - st.nu1 + st.nu2
    Fz = lam - st.nu1 - st.nu2
    c1 = s1 * st.nu1
    c2 = s2 * st.nu2
    n = st.beta.size
    mu = float(c1.sum() + c2.sum()) / (2 * n)
    comp = float(max(c1.max(), c2.max()))
    return Fb, Fz, s1, s2, Hb, comp, mu


def rel_kkt_of(Fb, Fz, comp, xinorm):
    return max(float(np.abs(Fb).max()), float(np.abs(Fz).max()), comp) / (1.0 + xinorm)


def initial_state(xi, lam):
    xinorm = float(np.abs(xi).max())
    z0 = xinorm if xinorm > 0 else 1.0
    return IPMState(np.zeros_like(xi), np.full_like(xi, z0),
                    np.full_like(xi, lam / 2.0), np.full_like(xi, lam / 2.0))


def newton_rhs(st: IPMState, Hb, xi, lam, sigma, mu, corr=None):
    """Condensed right-hand side.  `corr` = (c1, c2): the complementarity rows
    of "kktmu" read s_j d nu_j + nu_j d s_j = sigma mu - s_j nu_j - c_j (the
    corrector of a predictor-corrector step, c_j = d s_j d nu_j of the
    predictor), i.e. sigma mu / s_j becomes (sigma mu - c_j) / s_j."""
    s1 = st.z + st.beta
    s2 = st.z - st.beta
    t = sigma * mu
    if corr is None:
        rb = -(Hb - xi) + t * (1.0 / s1 - 1.0 / s2)
        rz = -lam + t * (1.0 / s1 + 1.0 / s2)
    else:
        u1 = (t - corr[0]) / s1
        u2 = (t - corr[1]) / s2
        rb = -(Hb - xi) + u1 - u2
        rz = -lam + u1 + u2
    return rb, rz


def recover_dnu(st: IPMState, db, dz, sig1, sig2, sigma, mu, corr=None):
    s1 = st.z + st.beta
    s2 = st.z - st.beta
    t = sigma * mu
    ds1 = db + dz
    ds2 = dz - db
    if corr is None:
        dnu1 = t / s1 - st.nu1 - sig1 * ds1
        dnu2 = t / s2 - st.nu2 - sig2 * ds2
    else:
        dnu1 = (t - corr[0]) / s1 - st.nu1 - sig1 * ds1
        dnu2 = (t - corr[1]) / s2 - st.nu2 - sig2 * ds2
    return ds1, ds2, dnu1, dnu2


def max_step(v, dv):
    """Largest a in (0, inf] with v + a dv >= 0 (v > 0)."""
    neg = dv < 0
    if not np.any(neg):
        return math.inf
    return float(np.min(-v[neg] / dv[neg]))


def ipm_solve(signal, observed, lam, opts: IPMOptions | None = None,
              state: IPMState | None = None, callback=None) -> IPMResult:
    """The primal-dual interior-point method described in the module doc."""
    opts = opts or IPMOptions()
    observed = observed.astype(np.float64)
    xi = dft3.xi(signal, observed)
    xinorm = float(np.abs(xi).max())
    st = state or initial_state(xi, lam)
    log = []
    cg_counts = []
    rel = math.inf
    mu = math.nan
    for it in range(opts.max_iter + 1):
        Fb, Fz, s1, s2, Hb, comp, mu = kkt_parts(st, xi, lam, observed)
        rel = rel_kkt_of(Fb, Fz, comp, xinorm)
        if rel <= opts.tol or it == opts.max_iter:
            break
        sig1 = st.nu1 / s1
        sig2 = st.nu2 / s2
        eta = min(opts.cg_rtol, 0.1 * rel)
        solver = {"cg": pcg, "cr": pcr, "car": pcar}[opts.krylov]

        def newton(rb, rz):
            return solver(lambda pb, pz: K_apply(pb, pz, sig1, sig2, observed),
                          lambda qb, qz: Pinv_apply(qb, qz, sig1, sig2, opts.pc_rho),
                          rb, rz, atol=opts.cg_atol, rtol=eta, maxit=opts.cg_max)
        sigma, corr, iters = opts.sigma, None, 0
        if opts.mehrotra:
            # predictor: the affine-scaling direction (sigma = 0), its full
            # step to the boundary (capped at 1) and the duality measure there
            ra = newton(*newton_rhs(st, Hb, xi, lam, 0.0, mu))
            iters += ra.iters
            da1, da2, dna1, dna2 = recover_dnu(st, ra.xb, ra.xz, sig1, sig2, 0.0, mu)
            aa = min(1.0, max_step(s1, da1), max_step(s2, da2), max_step(st.nu1, dna1), max_step(st.nu2, dna2))
            mu_aff = float(np.sum((s1 + aa * da1) * (st.nu1 + aa * dna1)) +
                           np.sum((s2 + aa * da2) * (st.nu2 + aa * dna2))) / (2 * xi.size)
            # centring sigma = (mu_aff / mu)^3, never aiming below the
            # complementarity the tolerance needs (0.1 tol (1 + |xi|_inf))
            sigma = min(1.0, max((mu_aff / mu) ** 3, 0.1 * opts.tol * (1.0 + xinorm) / mu))
            corr = (da1 * dna1, da2 * dna2)
        res = newton(*newton_rhs(st, Hb, xi, lam, sigma, mu, corr))
        iters += res.iters
        db, dz = res.xb, res.xz
        ds1, ds2, dnu1, dnu2 = recover_dnu(st, db, dz, sig1, sig2, sigma, mu, corr)
        amax = min(max_step(s1, ds1), max_step(s2, ds2),
                   max_step(st.nu1, dnu1), max_step(st.nu2, dnu2))
        alpha = min(1.0, opts.tau * amax)
        st = IPMState(st.beta + alpha * db, st.z + alpha * dz,
                      st.nu1 + alpha * dnu1, st.nu2 + alpha * dnu2)
        cg_counts.append(iters)
        log.append(dict(it=it, mu=mu, rel_kkt=rel, alpha=alpha, cg=iters, sigma=sigma))
        if callback is not None:
            callback(it, st, res)
    return IPMResult(st, len(cg_counts), cg_counts, rel, mu, rel <= opts.tol, log)


# ------------------------------------------------------------- certificates --

def kktmu_residual(w, xi, lam, observed, mu_target):
    """Residual of the perturbed KKT system (equation "kktmu") at
    w = (beta, z, s1, s2, y1, y2, nu1, nu2), each block of size n, with
    M_perp^T (M_perp beta - b) written as H beta - xi."""
    n = xi.size
    shape = xi.shape
    beta, z, s1, s2, y1, y2, nu1, nu2 = (w[i * n:(i + 1) * n].reshape(shape) for i in range(8))
    Hb = dft3.apply_H(beta, observed)
    r = [Hb - xi - y1 + y2,
         lam - y1 - y2,
         y1 - nu1,
         y2 - nu2,
         z + beta - s1,
         z - beta - s2,
         s1 * nu1 - mu_target,
         s2 * nu2 - mu_target]
    return np.concatenate([a.ravel() for a in r])


@dataclasses.dataclass
class Certificate:
    g: np.ndarray              # M_perp^T (b - M_perp beta)
    natural_residual: float    # ||beta - soft(beta + g, lam)||_inf / max(1, ||beta||_inf)
    primal: float
    dual: float
    rel_gap: float
    max_offsupport_ratio: float  # max |g_i| / lam over i off the support
    max_onsupport_dev: float     # max |g_i - lam sign(beta_i)| / lam on the support


def lasso_certificate(beta, signal, observed, lam, support_rel=1e-6) -> Certificate:
    """LASSO optimality and duality gap (the dual of 1/2||b - M beta||^2 +
    lam||beta||_1 is max b^T theta - 1/2 ||theta||^2 s.t. ||M^T theta||_inf <= lam)."""
    observed = observed.astype(np.float64)
    b_hat = np.where(observed != 0, signal, 0.0)
    Ab = dft3.apply_A(beta)
    r = observed * (b_hat - Ab)
    g = dft3.apply_At(r)
    nat = float(np.abs(beta - soft(beta + g, lam)).max()) / max(1.0, float(np.abs(beta).max()))
    primal = 0.5 * float(np.sum(r * r)) + lam * float(np.abs(beta).sum())
    gnorm = float(np.abs(g).max())
    theta = r * min(1.0, lam / gnorm) if gnorm > 0 else r
    dual = 0.5 * float(np.sum(b_hat * b_hat)) - 0.5 * float(np.sum((b_hat - theta) ** 2 * observed))
    gap = (primal - dual) / max(abs(primal), 1e-300)
    bmax = float(np.abs(beta).max())
    supp = np.abs(beta) > support_rel * bmax if bmax > 0 else np.zeros(beta.shape, bool)
    off = float((np.abs(g[~supp]).max() / lam)) if np.any(~supp) else 0.0
    on = float((np.abs(g[supp] - lam * np.sign(beta[supp])).max() / lam)) if np.any(supp) else 0.0
    return Certificate(g, nat, primal, dual, gap, off, on)


def support(beta, rel=1e-6):
    bmax = float(np.abs(beta).max())
    return np.abs(beta) > rel * bmax if bmax > 0 else np.zeros(beta.shape, bool)


def lambda_rule(signal, observed, frac=0.05):
    """lambda = frac * ||M_perp^T b||_inf."""
    return frac * float(np.abs(dft3.xi(signal, observed.astype(np.float64))).max())
