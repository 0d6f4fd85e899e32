"""Naive separable 3D DFT and the real parametrisation of conjugate-symmetric
spectra (oracle; test infrastructure only).

Paper, section "Problem formulation":
  * unitary DFT  v_k = n^{-1/2} sum_j w^{jk} x_j,  w = exp(-2 pi i / n), and
    its inverse with conj(w);
  * a real signal has a conjugate-symmetric spectrum (subspace F);
  * the map beta = B v keeps the self-conjugate bins as they are and replaces
    each conjugate pair (v_k, v_{-k}) by (sqrt2 Re v_k, sqrt2 Im v_k)
    (equation "beta"), B is unitary, and A = C^H B^H is real orthogonal
    (derivation "map").
The paper writes the 1D case and says 2D/3D mappings are analogous; it
notes that for odd n the subspace F has no Nyquist bin.  Reading used here
(3D, every N_d even, odd or 1; for odd N_d the sets {0, N_d/2} below are
just {0}):
  * k = (k1,k2,k3), -k = ((N_d - k_d) mod N_d)_d;
  * k is self-conjugate iff k == -k; then beta[k] = v_k (real);
  * otherwise k is canonical iff  k3 in [1, N3/2)
        or k3 in {0, N3/2} and k2 in [1, N2/2)
        or k3 in {0, N3/2}, k2 in {0, N2/2} and k1 in [1, N1/2);
    exactly one of k, -k is canonical;
  * for canonical k:  beta[k] = sqrt2 Re v_k,  beta[-k] = sqrt2 Im v_k.
beta is stored as a real array [N1][N2][N3] (row-major), index k.

Transforms are dense N x N matrix products per axis (O(n N) work, no FFT
factorisation).  DFT matrix entries use exact integer angle reduction
(j*k mod N) before the trigonometric call.
"""
from __future__ import annotations

import functools
import math

import numpy as np

SQRT2 = math.sqrt(2.0)


@functools.lru_cache(maxsize=32)
def dft_matrix(N: int) -> np.ndarray:
    """Unitary DFT matrix C[k, j] = N^{-1/2} exp(-2 pi i (jk mod N)/N)."""
    j = np.arange(N)
    ang = 2.0 * np.pi * ((np.outer(j, j)) % N) / N
    C = (np.cos(ang) - 1j * np.sin(ang)) / math.sqrt(N)
    C.setflags(write=False)
    return C


def _apply_axis(M: np.ndarray, a: np.ndarray, axis: int) -> np.ndarray:
    """out[..., k, ...] = sum_j M[k, j] a[..., j, ...] along `axis`."""
    out = np.tensordot(M, a, axes=([1], [axis]))
    return np.moveaxis(out, 0, axis)


def dft3(x: np.ndarray) -> np.ndarray:
    """Unitary 3D DFT (C applied along every axis)."""
    y = x.astype(np.complex128)
    for ax in range(3):
        y = _apply_axis(dft_matrix(y.shape[ax]), y, ax)
    return y


def idft3(v: np.ndarray) -> np.ndarray:
    """Unitary 3D inverse DFT (C^H applied along every axis)."""
    y = v.astype(np.complex128)
    for ax in range(3):
        y = _apply_axis(dft_matrix(y.shape[ax]).conj().T, y, ax)
    return y


@functools.lru_cache(maxsize=32)
def classes(shape) -> tuple:
    """(self_conj, canonical, mirror_flat) over the flat index of `shape`.

    mirror_flat[f] is the flat index of -k for k = unravel(f)."""
    N1, N2, N3 = shape
    k1, k2, k3 = np.meshgrid(np.arange(N1), np.arange(N2), np.arange(N3), indexing="ij")
    m1, m2, m3 = (-k1) % N1, (-k2) % N2, (-k3) % N3
    self_conj = (k1 == m1) & (k2 == m2) & (k3 == m3)
    half3 = (k3 >= 1) & (2 * k3 < N3)
    edge3 = k3 == m3
    half2 = (k2 >= 1) & (2 * k2 < N2)
    edge2 = k2 == m2
    half1 = (k1 >= 1) & (2 * k1 < N1)
    canonical = half3 | (edge3 & half2) | (edge3 & edge2 & half1)
    mirror = np.ravel_multi_index((m1.ravel(), m2.ravel(), m3.ravel()), shape)
    out = (self_conj.ravel(), canonical.ravel(), mirror)
    for a in out:
        a.setflags(write=False)
    return out


def beta_to_spectrum(beta: np.ndarray) -> np.ndarray:
    """B^H: real beta [N1,N2,N3] -> conjugate-symmetric complex spectrum v."""
    shape = beta.shape
    sc, can, mir = classes(shape)
    b = beta.ravel()
    v = np.zeros(b.size, dtype=np.complex128)
    v[sc] = b[sc]
    idx = np.nonzero(can)[0]
    vk = (b[idx] + 1j * b[mir[idx]]) / SQRT2
    v[idx] = vk
    v[mir[idx]] = np.conj(vk)
    return v.reshape(shape)


def spectrum_to_beta(v: np.ndarray) -> np.ndarray:
    """B: complex spectrum v -> real beta (for conjugate-symmetric v this is
    the inverse of beta_to_spectrum; in general it is the real-linear map
    beta[k] = (v_k + v_-k)/sqrt2, beta[-k] = -i (v_k - v_-k)/sqrt2 for
    canonical k, real part taken)."""
    shape = v.shape
    sc, can, mir = classes(shape)
    f = v.ravel()
    b = np.zeros(f.size, dtype=np.float64)
    b[sc] = f[sc].real
    idx = np.nonzero(can)[0]
    b[idx] = ((f[idx] + f[mir[idx]]) / SQRT2).real
    b[mir[idx]] = ((-1j) * (f[idx] - f[mir[idx]]) / SQRT2).real
    return b.reshape(shape)


def apply_A(beta: np.ndarray) -> np.ndarray:
    """A beta = IDFT(B^H beta) (real; the imaginary part is round-off)."""
    return idft3(beta_to_spectrum(beta)).real


def apply_At(x: np.ndarray) -> np.ndarray:
    """A^T x = (C^H B^H)^T x = B C x: unitary DFT, then the real map B.

    Note: the paper's closing formula for xi reads as a DFT of the vector
    mapped from the zero-filled signal through equation "v"; taken literally
    that gives the index-reversed R A x.  The adjoint of A is B C, which is
    what this function computes (A^T A = I is tested)."""
    return spectrum_to_beta(dft3(x))


def apply_H(beta: np.ndarray, observed: np.ndarray) -> np.ndarray:
    """H beta = M_perp^T M_perp beta = A^T D A beta, D = diag(observed)."""
    return apply_At(observed * apply_A(beta))


def xi(signal: np.ndarray, observed: np.ndarray) -> np.ndarray:
    """xi = M_perp^T b = A^T b_hat with b_hat the zero-filled signal
    (equation "xi")."""
    return apply_At(np.where(observed != 0, signal, 0.0))


def dense_A(shape) -> np.ndarray:
    """A as an explicit n x n matrix (columns A e_i), tiny grids only."""
    n = int(np.prod(shape))
    cols = [apply_A(np.eye(n)[i].reshape(shape)).ravel() for i in range(n)]
    return np.stack(cols, axis=1)


def diag_H(observed: np.ndarray) -> np.ndarray:
    """diag(M_perp^T M_perp)_i = sum over observed j of A_ji^2, computed from
    the columns of A one at a time (brute force; small grids)."""
    shape = observed.shape
    n = observed.size
    d = np.empty(n)
    e = np.zeros(n)
    for i in range(n):
        e[i] = 1.0
        col = apply_A(e.reshape(shape)).ravel()
        d[i] = np.sum(observed.ravel() * col * col)
        e[i] = 0.0
    return d.reshape(shape)


def waves_to_beta(shape, wave_k, wave_c) -> np.ndarray:
    """beta of the signal sum_w sqrt(2/n) Re(c_w exp(2 pi i <k_w, j/N>)).

    That wave equals n^{-1/2}(c/sqrt2 e^{i theta} + conj(c)/sqrt2 e^{-i theta}),
    so v_k = c/sqrt2 and v_{-k} = conj(c)/sqrt2; through B:
    beta[k] = Re c, beta[-k] = Im c for canonical k (and for canonical -k,
    beta[-k] = Re c, beta[k] = -Im c)."""
    sc, can, mir = classes(tuple(shape))
    b = np.zeros(int(np.prod(shape)))
    for kv, c in zip(wave_k, wave_c):
        f = int(np.ravel_multi_index(tuple(int(a) for a in kv), shape))
        if can[f]:
            b[f] += c.real
            b[mir[f]] += c.imag
        else:
            b[mir[f]] += c.real
            b[f] += -c.imag
    return b.reshape(shape)
