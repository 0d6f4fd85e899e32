"""The paper's artificial test problem (workload.paper_synthetic): the
product formula of section "Synthetic Dataset", U[0, 1] noise, and the
lattice-cube missing pattern with the stated fractions."""
import numpy as np
import pytest

from paper_2502_04217_amd import workload as wl


@pytest.mark.parametrize("N,frac", [(8, 125 / 512), (16, 729 / 4096), (32, 4913 / 32768)])
def test_paper_synthetic(N, frac):
    w = wl.paper_synthetic(N, seed=3)
    assert w.shape == (N, N, N)
    assert abs(w.missing_fraction - frac) < 1e-12
    i, j, k = 1, 2, 3 % N
    t = 2 * np.pi / N
    f = (np.cos(t * i) + 2 * np.sin(t * i)) * (np.cos(2 * t * j) + 2 * np.sin(2 * t * j)) * \
        (np.cos(3 * t * k) + 2 * np.sin(3 * t * k))
    assert abs(w.clean[i, j, k] - f) < 1e-12
    obs = w.observed == 1
    noise = w.signal[obs] - w.clean[obs]
    assert noise.min() >= 0.0 and noise.max() < 1.0 and abs(noise.mean() - 0.5) < 0.05
    assert np.all(w.signal[~obs] == 0.0)
    # the clean signal is a product of three real waves: 8 nonzero DFT bins
    spec = np.fft.fftn(w.clean)
    assert int((np.abs(spec) > 1e-8 * np.abs(spec).max()).sum()) == 8


@pytest.mark.parametrize("N,period,half", [(96, 32, 8), (192, 32, 8), (384, 32, 8), (560, 70, 18), (40, 40, 10)])
def test_paper_mask_params(N, period, half):
    """The 15 % lattice at the non-power-of-two extents of the paper's table:
    a period that divides N, and a missing fraction within 1 % of 15 %."""
    assert wl.paper_mask_params(N) == (period, half)
    assert N % period == 0
    assert abs(((2 * half + 1) / period) ** 3 - 0.15) < 1e-2


def test_paper_synthetic_mixed_extent():
    w = wl.paper_synthetic(40, seed=1)
    assert abs(w.missing_fraction - (21 / 40) ** 3) < 1e-12
