"""Pins of the oracle's operators (section "Problem formulation" and
"Matrix-free operators" of the paper) against facts that do not come from the
oracle itself: orthogonality, the paper's own 1D formula (derivation "map"),
numpy's FFT, Parseval, adjointness and projection identities."""
import math

import numpy as np
import pytest

from oracle import dft3, mlp
from paper_2502_04217_amd import workload as wl


@pytest.mark.parametrize("shape", [(4, 6, 8), (2, 4, 4), (1, 1, 8), (8, 2, 2), (6, 10, 14), (3, 5, 8), (5, 7, 4),
                                   (3, 3, 3)])
def test_A_real_orthogonal(shape):
    A = dft3.dense_A(shape)
    n = A.shape[0]
    assert np.abs(A.T @ A - np.eye(n)).max() < 1e-13
    # the imaginary part of IDFT(B^H beta) vanishes for every beta
    beta = np.random.default_rng(0).standard_normal(shape)
    assert np.abs(dft3.idft3(dft3.beta_to_spectrum(beta)).imag).max() < 1e-14


@pytest.mark.parametrize("shape", [(4, 6, 8), (6, 4, 2), (1, 1, 10), (3, 5, 8), (7, 1, 9)])
def test_exactly_one_of_pair_canonical(shape):
    sc, can, mir = dft3.classes(shape)
    n = int(np.prod(shape))
    assert np.all(mir[mir] == np.arange(n))
    assert np.all(sc == (mir == np.arange(n)))
    # for every non-self-conjugate k exactly one of k, -k is canonical
    nsc = ~sc
    assert np.all((can[nsc].astype(int) + can[mir[nsc]].astype(int)) == 1)
    assert not np.any(can & sc)
    assert sc.sum() == np.prod([2 if N % 2 == 0 else 1 for N in shape])


@pytest.mark.parametrize("N", [4, 8, 12])
def test_1d_matches_paper_formula(N):
    """With N1 = N2 = 1 the 3D map reduces to the paper's 1D map: row k of A
    is n^{-1/2}(beta_0 + (-1)^k beta_1 + sum_j sqrt2 Re(conj(w)^{jk}) beta_{j+1}
    - sum_j sqrt2 Im(conj(w)^{jk}) beta_{j+n/2}) (derivation "map") with the
    ordering of equation "beta"; ours is a permutation of it."""
    n = N
    h = n // 2
    Ap = np.zeros((n, n))
    for k in range(n):
        Ap[k, 0] = 1.0
        Ap[k, 1] = (-1.0) ** k
        for j in range(1, h):
            wbar = complex(math.cos(2 * math.pi * j * k / n), math.sin(2 * math.pi * j * k / n))
            Ap[k, j + 1] = math.sqrt(2) * wbar.real
            Ap[k, j + h] = -math.sqrt(2) * wbar.imag
    Ap /= math.sqrt(n)
    ours = dft3.dense_A((1, 1, n))
    perm = np.empty(n, dtype=int)          # perm[paper index] = our index
    perm[0] = 0
    perm[1] = h
    for j in range(1, h):
        perm[j + 1] = j
        perm[j + h] = n - j
    assert np.abs(ours[:, perm] - Ap).max() < 1e-14


GOLDEN = __import__("pathlib").Path(__file__).parent / "golden"


def _read_paper_1d_A():
    """The hand-worked matrices of tests/golden/paper_1d_map_A.txt, as
    {n: A} with A in the paper's ordering of beta (equation "beta")."""
    value = {"0": 0.0, "1": 1.0, "r2": math.sqrt(2), "r2/2": math.sqrt(2) / 2, "r6/2": math.sqrt(6) / 2}
    out, rows, n = {}, [], None
    for line in (GOLDEN / "paper_1d_map_A.txt").read_text().splitlines():
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("n "):
            if n is not None:
                out[n] = np.array(rows) / math.sqrt(n)
            n, rows = int(line.split()[1]), []
            continue
        rows.append([-value[t[1:]] if t.startswith("-") else value[t] for t in line.split()])
    out[n] = np.array(rows) / math.sqrt(n)
    return out


def test_1d_map_matches_hand_worked_golden():
    """The oracle's A for a 1D grid (N1 = N2 = 1) equals the hand-evaluated
    matrices of the paper's 1D map at n = 4 and n = 6 (derivation "map"),
    after the permutation from the paper's ordering of beta to ours."""
    golden = _read_paper_1d_A()
    assert sorted(golden) == [4, 6]
    for n, Ap in golden.items():
        assert Ap.shape == (n, n)
        h = n // 2
        perm = np.empty(n, dtype=int)          # perm[paper index] = our index
        perm[0], perm[1] = 0, h
        for j in range(1, h):
            perm[j + 1] = j
            perm[j + h] = n - j
        ours = dft3.dense_A((1, 1, n))
        assert np.abs(ours[:, perm] - Ap).max() < 1e-15
        # the fixture itself is orthogonal, so a mistyped entry shows here too
        assert np.abs(Ap.T @ Ap - np.eye(n)).max() < 1e-15


@pytest.mark.parametrize("shape", [(8, 6, 10), (5, 6, 7), (4, 9, 15), (3, 5, 3)])
def test_synthesised_waves_match_A(shape):
    """numpy's irfftn synthesis of plane waves equals A applied to the beta
    the oracle derives from the wave list (two independent routes), with an
    even N3 and with odd ones (no Nyquist plane: k3 = floor(N3/2) is an
    interior bin)."""
    w = wl.make_workload(shape, n_freq=14, amplitude="normal", snr_db=np.inf,
                         half_width=-1, period=2, seed=7)
    beta = dft3.waves_to_beta(w.shape, w.wave_k, w.wave_c)
    assert np.count_nonzero(beta) == 14
    assert np.abs(dft3.apply_A(beta) - w.clean).max() < 1e-14
    # and the naive DFT agrees with numpy's FFT
    x = np.random.default_rng(3).standard_normal(shape)
    assert np.abs(dft3.dft3(x) - np.fft.fftn(x, norm="ortho")).max() < 1e-13


@pytest.mark.parametrize("shape", [(8, 8, 8), (4, 16, 8), (12, 10, 14), (15, 7, 6)])
def test_parseval_adjoint_projection(shape):
    rng = np.random.default_rng(11)
    beta = rng.standard_normal(shape)
    x = rng.standard_normal(shape)
    Ab = dft3.apply_A(beta)
    assert abs(np.linalg.norm(Ab) - np.linalg.norm(beta)) < 1e-12 * np.linalg.norm(beta)
    lhs = float(np.sum(Ab * x))
    rhs = float(np.sum(beta * dft3.apply_At(x)))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs) + 1e-12
    assert np.abs(dft3.apply_At(dft3.apply_A(beta)) - beta).max() < 1e-13
    obs = (rng.random(shape) > 0.3).astype(np.float64)
    Hb = dft3.apply_H(beta, obs)
    HHb = dft3.apply_H(Hb, obs)
    assert np.abs(HHb - Hb).max() < 1e-13          # H is a projection
    y = rng.standard_normal(shape)
    assert abs(float(np.sum(dft3.apply_H(y, obs) * beta)) - float(np.sum(y * Hb))) < 1e-11


def test_xi_is_adjoint_not_literal_formula():
    """The paper's closing formula for xi (DFT of the vector mapped from the
    zero-filled signal through equation "v") yields the index-reversed R A x.
    The adjoint A^T x = B C x is what the method needs (M_perp^T b)."""
    shape = (4, 6, 8)
    x = np.random.default_rng(5).standard_normal(shape)
    literal = dft3.dft3(dft3.beta_to_spectrum(x))
    assert np.abs(literal.imag).max() < 1e-13
    Ax = dft3.apply_A(x)
    sc, can, mir = dft3.classes(shape)
    RAx = Ax.ravel()[mir].reshape(shape)
    assert np.abs(literal.real - RAx).max() < 1e-13
    assert np.abs(literal.real - dft3.apply_At(x)).max() > 1e-3


def test_xi_equals_dense_Mperp_transpose_b():
    shape = (4, 4, 6)
    w = wl.make_workload(shape, n_freq=6, amplitude="normal", snr_db=10.0,
                         half_width=0, period=2, seed=2)
    A = dft3.dense_A(shape)
    obs = w.observed.ravel() == 1
    Mp = A[obs]
    b = w.signal.ravel()[obs]
    assert np.abs(dft3.xi(w.signal, w.observed).ravel() - Mp.T @ b).max() < 1e-13


@pytest.mark.parametrize("shape", [(4, 6, 8), (8, 8, 4), (6, 10, 14), (3, 5, 8), (9, 7, 6)])
def test_diag_H_closed_form(shape):
    rng = np.random.default_rng(9)
    obs = (rng.random(shape) > 0.25).astype(np.float64)
    brute = dft3.diag_H(obs)
    A = dft3.dense_A(shape)
    dense = np.sum(A * A * obs.ravel()[:, None], axis=0).reshape(shape)
    assert np.abs(brute - dense).max() < 1e-13
    assert np.abs(mlp.diag_H_closed_form(obs) - dense).max() < 1e-13
