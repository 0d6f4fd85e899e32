"""Learned diagonal correction of the preconditioner (oracle; test
infrastructure only).

Not in the paper.  The paper's preconditioner P = [[I + L1, L2], [L2, L1]]
(section "Krylov methods and preconditioners") replaces M_perp^T M_perp by I;
the cited alternative scales I by a constant, and the conclusions name the
periodic missing structure as a route to better preconditioning.  Here I is
replaced by C = diag(c) with c_i = softplus(o_i) + 1e-6 > 0, o = MLP(phi_i),
so every 2x2 block [[c + L1, L2], [L2, L1]] has determinant c L1 + 4 S1 S2 > 0
and positive trace: P_c stays symmetric positive definite.

Network: 4 -> 32 -> 32 -> 1, tanh hidden units, float32 on the GPU, float64
here.  Flat parameter layout (1249 values):
    W1[32][4], b1[32], W2[32][32], b2[32], w3[32], b3
Features per coefficient i:
    f1 = log L1_i - mean_j log L1_j
    f2 = L2_i / L1_i                       (in (-1, 1))
    f3 = log(|beta_i| / max|beta| + 1e-12)  (max|beta| = 0 gives log 1e-12)
    f4 = diag(M_perp^T M_perp)_i            (the share of basis function i's
                                             energy that falls on observed
                                             samples)
Loss (one training record per sampled coefficient i of a captured Krylov
direction p with u = H p_beta):
    e_i(c) = (L1_i^2 + L2_i^2) (u_i - c_i p_i)^2 / (L1_i + 4 S1_i S2_i)^2
which is the squared i-th block of P^{-1}(K - P_c)p, the deviation of the
corrected preconditioner from K along p measured through the paper's P
(c = 1); the total loss is sum_i w_i e_i with per-record weights w_i supplied
by the caller.  It is a weighted least-squares problem in c whose optimum
for white directions is the Jacobi choice c_i = (M_perp^T M_perp)_ii.
"""
from __future__ import annotations

import math

import numpy as np

H1 = 32
H2 = 32
NIN = 4
N_PARAMS = H1 * NIN + H1 + H2 * H1 + H2 + H2 + 1   # 1249
C_FLOOR = 1e-6
SOFTPLUS_ONE = math.log(math.e - 1.0)   # softplus(x) = 1 at this x


def unpack(params):
    p = np.asarray(params, dtype=np.float64)
    assert p.size == N_PARAMS
    o = 0
    W1 = p[o:o + H1 * NIN].reshape(H1, NIN); o += H1 * NIN
    b1 = p[o:o + H1]; o += H1
    W2 = p[o:o + H2 * H1].reshape(H2, H1); o += H2 * H1
    b2 = p[o:o + H2]; o += H2
    w3 = p[o:o + H2]; o += H2
    b3 = p[o]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, [b3]])


def init_params(seed=0, out_scale=0.01):
    """Glorot-uniform hidden layers; output layer small with bias at
    softplus^{-1}(1), so an untrained network gives c ~ 1 (the paper's P)."""
    rng = np.random.default_rng(seed)
    def glorot(fo, fi):
        a = math.sqrt(6.0 / (fi + fo))
        return rng.uniform(-a, a, size=(fo, fi))
    W1 = glorot(H1, NIN)
    W2 = glorot(H2, H1)
    w3 = rng.uniform(-out_scale, out_scale, size=H2)
    return pack(W1, np.zeros(H1), W2, np.zeros(H2), w3, SOFTPLUS_ONE)


def softplus(x):
    return np.maximum(x, 0.0) + np.log1p(np.exp(-np.abs(x)))


def sigmoid(x):
    return 0.5 * (1.0 + np.tanh(0.5 * x))


def forward(params, feats):
    """c = softplus(MLP(feats)) + 1e-6 for feats [N, 4]; returns (c, cache)."""
    W1, b1, W2, b2, w3, b3 = unpack(params)
    x = np.asarray(feats, dtype=np.float64)
    a1 = x @ W1.T + b1
    h1 = np.tanh(a1)
    a2 = h1 @ W2.T + b2
    h2 = np.tanh(a2)
    o = h2 @ w3 + b3
    c = softplus(o) + C_FLOOR
    return c, (x, h1, h2, o)


def backward(params, cache, dc):
    """Gradient of sum_i dc_i * c_i with respect to the flat parameters."""
    W1, b1, W2, b2, w3, b3 = unpack(params)
    x, h1, h2, o = cache
    do = dc * sigmoid(o)
    gw3 = h2.T @ do
    gb3 = do.sum()
    dh2 = np.outer(do, w3)
    da2 = dh2 * (1.0 - h2 * h2)
    gW2 = da2.T @ h1
    gb2 = da2.sum(axis=0)
    dh1 = da2 @ W2
    da1 = dh1 * (1.0 - h1 * h1)
    gW1 = da1.T @ x
    gb1 = da1.sum(axis=0)
    return pack(gW1, gb1, gW2, gb2, gw3, gb3)


def record_loss(c, u, p, L1, L2, S12, w):
    """Per-record loss w (L1^2 + L2^2)(u - c p)^2 / (L1 + S12)^2 and its
    derivative with respect to c (S12 = 4 S1 S2)."""
    D = L1 + S12
    res = u - c * p
    a = (L1 * L1 + L2 * L2) / (D * D)
    e = w * a * res * res
    de = -2.0 * w * a * p * res
    return e, de


def loss_and_grad(params, feats, u, p, L1, L2, S12, w):
    c, cache = forward(params, feats)
    e, de = record_loss(c, u, p, L1, L2, S12, w)
    return float(e.sum()), backward(params, cache, de)


def adam_step(params, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba), t counted from 1; returns new (params, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def features(sig1, sig2, beta, diagH):
    """The four features of every coefficient, shape [n, 4]."""
    L1 = (sig1 + sig2).ravel()
    L2 = (sig1 - sig2).ravel()
    lg = np.log(L1)
    f1 = lg - lg.mean()
    f2 = L2 / L1
    bmax = float(np.abs(beta).max())
    f3 = np.log(np.abs(beta).ravel() / (bmax if bmax > 0 else 1.0) + 1e-12)
    f4 = np.asarray(diagH, dtype=np.float64).ravel()
    return np.stack([f1, f2, f3, f4], axis=1)


PC_RELEVANCE = 1e-3


def correction(params, beta, z, nu1, nu2, diagH, rmin=PC_RELEVANCE):
    """The correction the solver applies at an interior-point iterate:
    c = softplus(MLP(features)) + 1e-6 where the correction can act on
    P_c^{-1}, i.e. where L1 / (L1 + 4 S1 S2) >= rmin; c = 1 elsewhere (there
    every entry of P_c^{-1} moves by less than rmin relative with c)."""
    s1, s2 = z + beta, z - beta
    sig1, sig2 = nu1 / s1, nu2 / s2
    c, _ = forward(params, features(sig1, sig2, beta, diagH))
    L1 = (sig1 + sig2).ravel()
    act = L1 >= rmin * (L1 + 4.0 * (sig1 * sig2).ravel())
    return np.where(act, c, 1.0).reshape(beta.shape), act.reshape(beta.shape)


def diag_H_closed_form(observed):
    """diag(M_perp^T M_perp) from one DFT of the mask: the square of column i
    of A is (1/n)(1 +- cos(2 theta)) for the sqrt2 Re / sqrt2 Im coordinates
    of bin k and 1/n for a self-conjugate bin, so
        H_ii = m/n + s_i Re(Mhat[2k]) / sqrt(n),
    s_i = +1 / -1 / 0, Mhat the unitary DFT of the 0/1 mask."""
    from . import dft3
    shape = observed.shape
    n = observed.size
    sc, can, mir = dft3.classes(shape)
    Mhat = dft3.dft3(observed.astype(np.float64))
    Nv = np.asarray(shape)
    k = np.stack(np.unravel_index(np.arange(n), shape), axis=1)
    k2 = (2 * k) % Nv
    re2 = Mhat[k2[:, 0], k2[:, 1], k2[:, 2]].real
    s = np.zeros(n)
    s[can] = 1.0
    s[mir[can]] = -1.0
    m = float(observed.sum())
    return (m / n + s * re2 / math.sqrt(n)).reshape(shape)
