"""Seeded synthetic inputs: crystal-like signals with a sparse spectrum, noise and
a periodic missing-sample pattern.

This module only draws random numbers and synthesises a physical test signal.
It holds none of the solver's arithmetic: no real parametrisation of the
spectrum, no operator, no lambda rule.  Both the HIP path and the CPU oracle
receive exactly the arrays produced here (signal + observed mask).

Signal model (the problem statement of the paper, "Problem formulation":
noisy real signal = true signal + additive noise, with a set of missing
samples).  The true signal is a sum of real standing plane waves

    x[j] = sum_w sqrt(2/n) * Re( c_w * exp(2*pi*i * <k_w, j/N>) ),

one per wave vector k_w (none of them self-conjugate, all distinct up to sign),
with complex amplitude c_w.  Each wave occupies the two DFT bins k_w and -k_w,
so "F nonzero frequencies" means F/2 waves.  With this normalisation one wave
has Euclidean norm |c_w|.  The signal is synthesised with numpy's inverse real
FFT, a library routine independent of both implementations under test.

Missing samples: the union of cubes of half-width h (periodic wrap) centred on
the lattice points p = 0 (mod P) on every axis, the way Bragg peaks of the
average crystal structure are punched out, optionally united with independent
Bernoulli dropouts.

Noise: iid Gaussian with standard deviation rms(x) * 10^(-SNR/20), rms over
the whole grid, added to every sample before masking.  Missing samples of the
returned signal hold 0.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class Workload:
    shape: tuple
    signal: np.ndarray        # float64 [N1,N2,N3], noisy, 0 at missing samples
    observed: np.ndarray      # uint8 [N1,N2,N3], 1 = observed, 0 = missing
    clean: np.ndarray         # float64 [N1,N2,N3], noiseless true signal
    wave_k: np.ndarray        # int64 [W,3], wave vectors, k_d in [0, N_d)
    wave_c: np.ndarray        # complex128 [W], amplitudes (see module doc)
    noise_sigma: float
    name: str = ""

    @property
    def n(self) -> int:
        return int(np.prod(self.shape))

    @property
    def missing_fraction(self) -> float:
        return 1.0 - float(self.observed.mean())


def lattice_cube_mask(shape, half_width: int, period: int) -> np.ndarray:
    """Boolean [N1,N2,N3]: True where a sample lies inside a cube of
    half-width `half_width` around a lattice point (all coordinates = 0 mod
    `period`), with periodic wrap.  Every N_d must be a multiple of period."""
    axes = []
    for N in shape:
        if N % period != 0:
            raise ValueError(f"grid size {N} is not a multiple of period {period}")
        j = np.arange(N) % period
        dist = np.minimum(j, period - j)
        axes.append(dist <= half_width)
    a0, a1, a2 = axes
    return a0[:, None, None] & a1[None, :, None] & a2[None, None, :]


def draw_wave_vectors(rng, shape, count_waves: int) -> np.ndarray:
    """`count_waves` distinct wave vectors, none self-conjugate, no two equal up
    to sign.  Uniform over the admissible set (rejection sampling)."""
    N = np.asarray(shape, dtype=np.int64)
    n = int(np.prod(N))
    max_waves = (n - int(np.prod([2 if d % 2 == 0 else 1 for d in shape]))) // 2
    if count_waves > max_waves:
        raise ValueError("too many waves for this grid")
    chosen = {}
    order = []
    while len(order) < count_waves:
        need = count_waves - len(order)
        flat = rng.integers(0, n, size=max(2 * need, 16))
        k = np.stack(np.unravel_index(flat, shape), axis=1)
        mk = (-k) % N
        mflat = np.ravel_multi_index(mk.T, shape)
        for f, mf, kv in zip(flat.tolist(), mflat.tolist(), k):
            if f == mf:
                continue  # self-conjugate bin: a real cosine of a single bin
            key = min(f, mf)
            if key in chosen:
                continue
            chosen[key] = True
            order.append(kv.copy())
            if len(order) == count_waves:
                break
    return np.asarray(order, dtype=np.int64).reshape(-1, 3)


def synthesize(shape, wave_k: np.ndarray, wave_c: np.ndarray) -> np.ndarray:
    """x[j] = sum_w sqrt(2/n) Re(c_w exp(2 pi i <k_w, j/N>)), via numpy.fft.irfftn.

    numpy's irfftn computes (1/n) sum over the full Hermitian spectrum, using
    only bins with k3 <= N3/2.  A wave placed as c at k and conj(c) at -k
    contributes (2/n) Re(c e^{i theta}); bins with k3 > N3/2 are written at -k
    (conjugated), and in the self-paired planes (k3 = 0, and k3 = N3/2 for an
    even N3) both k and -k are written because irfftn keeps only the real
    part of those planes' 2D inverse."""
    N1, N2, N3 = shape
    n = N1 * N2 * N3
    half = N3 // 2
    S = np.zeros((N1, N2, half + 1), dtype=np.complex128)
    scale = math.sqrt(n / 2.0)
    Nv = np.asarray(shape, dtype=np.int64)
    for kv, c in zip(wave_k, wave_c):
        cs = c * scale
        mk = (-kv) % Nv
        k3 = int(kv[2])
        paired = k3 == 0 or (N3 % 2 == 0 and k3 == half)
        if paired:                                 # a self-paired plane: both bins
            S[kv[0], kv[1], k3] += cs
            S[mk[0], mk[1], mk[2]] += np.conj(cs)
        elif k3 <= half:                           # inside the stored half
            S[kv[0], kv[1], k3] += cs
        else:                                      # mirror lies inside the half
            S[mk[0], mk[1], mk[2]] += np.conj(cs)
    return np.fft.irfftn(S, s=shape, axes=(0, 1, 2))


def make_workload(shape, *, n_freq: int, amplitude: str, snr_db: float,
                  half_width: int, period: int, dropout: float = 0.0,
                  seed: int = 0, name: str = "") -> Workload:
    """Generic seeded workload.  `n_freq` counts nonzero DFT bins (both k and
    -k), so n_freq/2 waves are drawn.  `amplitude` selects how the real and
    imaginary parts of each wave's amplitude are drawn:
      'normal'      iid N(0,1)
      'lognormal'   random sign times exp(N(0,1))
      'decay32'     N(0,1) * exp(-|k|/32), |k| the Euclidean norm of the
                    signed frequency (k_d taken in [-N_d/2, N_d/2))."""
    rng = np.random.default_rng(seed)
    shape = tuple(int(s) for s in shape)
    n_waves = max(1, n_freq // 2)
    k = draw_wave_vectors(rng, shape, n_waves)
    if amplitude == "normal":
        re, im = rng.standard_normal(n_waves), rng.standard_normal(n_waves)
    elif amplitude == "lognormal":
        re = rng.choice([-1.0, 1.0], n_waves) * np.exp(rng.standard_normal(n_waves))
        im = rng.choice([-1.0, 1.0], n_waves) * np.exp(rng.standard_normal(n_waves))
    elif amplitude == "decay32":
        Nv = np.asarray(shape)
        ks = np.where(k >= (Nv + 1) // 2, k - Nv, k).astype(np.float64)
        damp = np.exp(-np.sqrt((ks ** 2).sum(axis=1)) / 32.0)
        re = rng.standard_normal(n_waves) * damp
        im = rng.standard_normal(n_waves) * damp
    else:
        raise ValueError(amplitude)
    c = re + 1j * im
    clean = synthesize(shape, k, c)
    rms = float(np.sqrt(np.mean(clean ** 2)))
    sigma = rms * 10.0 ** (-snr_db / 20.0) if np.isfinite(snr_db) else 0.0
    noisy = clean + (rng.standard_normal(shape) * sigma if sigma > 0 else 0.0)
    missing = lattice_cube_mask(shape, half_width, period) if half_width >= 0 else np.zeros(shape, bool)
    if dropout > 0:
        missing |= rng.random(shape) < dropout
    observed = (~missing).astype(np.uint8)
    signal = np.where(observed == 1, noisy, 0.0)
    return Workload(shape, signal, observed, clean, k, c, sigma, name)


# ---- the five named workloads -------------------------------------------------

def grid16(seed: int = 1) -> Workload:
    """16^3, 24 nonzero frequencies with N(0,1) parts, SNR 20 dB, cubes of
    half-width 1 on a period-8 lattice."""
    return make_workload((16, 16, 16), n_freq=24, amplitude="normal", snr_db=20.0,
                         half_width=1, period=8, seed=seed, name=f"grid16-s{seed}")


def grid64(seed: int = 1) -> Workload:
    """64^3, 400 nonzero frequencies with log-normal parts, SNR 15 dB, cubes of
    half-width 2 on a period-16 lattice."""
    return make_workload((64, 64, 64), n_freq=400, amplitude="lognormal", snr_db=15.0,
                         half_width=2, period=16, seed=seed, name=f"grid64-s{seed}")


def grid256(seed: int = 1) -> Workload:
    """256^3, 0.1% of the DFT bins nonzero with N(0,1) exp(-|k|/32) parts,
    SNR 10 dB, cubes of half-width 3 on a period-32 lattice plus 2% uniform
    dropouts."""
    shape = (256, 256, 256)
    return make_workload(shape, n_freq=int(round(0.001 * 256 ** 3)), amplitude="decay32",
                         snr_db=10.0, half_width=3, period=32, dropout=0.02, seed=seed,
                         name=f"grid256-s{seed}")


def grid128_family(seed: int, periods=(8, 16, 32)) -> Workload:
    """128^3 training/evaluation family: sparsity log-uniform in [0.05%, 0.5%]
    of the DFT bins, SNR uniform in [5, 20] dB, lattice period drawn from
    `periods` ({8, 16, 32} for the evaluation family) with cube half-width
    log2(P) - 2, N(0,1) parts."""
    rng = np.random.default_rng(10_000_019 + seed)
    frac = math.exp(rng.uniform(math.log(5e-4), math.log(5e-3)))
    snr = float(rng.uniform(5.0, 20.0))
    period = int(rng.choice(list(periods)))
    hw = int(math.log2(period)) - 2
    shape = (128, 128, 128)
    return make_workload(shape, n_freq=int(round(frac * 128 ** 3)), amplitude="normal",
                         snr_db=snr, half_width=hw, period=period, seed=seed,
                         name=f"grid128-s{seed}")


def grid512(seed: int = 1) -> Workload:
    """512^3, 0.02% of the DFT bins nonzero with N(0,1) parts, SNR 10 dB,
    cubes of half-width 4 on a period-64 lattice."""
    shape = (512, 512, 512)
    return make_workload(shape, n_freq=int(round(2e-4 * 512 ** 3)), amplitude="normal",
                         snr_db=10.0, half_width=4, period=64, seed=seed,
                         name=f"grid512-s{seed}")


def paper_mask_params(N: int):
    """(period, half-width) of the lattice-cube mask of paper_synthetic at
    extent N: period 32 with half-width 8 (15.0 % missing) where 32 divides N,
    period 16 with half-width 4 (17.8 %) at N = 16 and period 8 with
    half-width 2 (24.4 %) at N = 8; otherwise the divisor P of N in [32, 128]
    and half-width h whose missing fraction ((2h+1)/P)^3 is closest to 15 %
    (N = 560: P = 70, h = 18, 14.8 %)."""
    if N % 32 == 0:
        return 32, 8
    if N < 32:
        return (16, 4) if N >= 16 else (8, 2)
    best = None
    for P in range(32, 129):
        if N % P:
            continue
        for h in range(P // 2):
            d = abs(((2 * h + 1) / P) ** 3 - 0.15)
            if best is None or d < best[0]:
                best = (d, P, h)
    if best is None:
        raise ValueError(f"no lattice period in [32, 128] divides {N}")
    return best[1], best[2]


def paper_synthetic(n_side: int, seed: int = 1) -> Workload:
    """The paper's artificial test problem (section "Synthetic Dataset"):
    x_ijk = f1(i) f2(j) f3(k) with f_a(t) = cos(2 pi a t / N) + 2 sin(2 pi a t / N)
    for a = 1, 2, 3 along the three axes, plus iid U[0, 1] noise on every
    sample.  The paper's "~15 %" missing samples come in an unspecified
    pattern; here they are lattice cubes as in the other workloads, with the
    period and half-width of paper_mask_params.  The planted spectrum is the
    product formula itself, so wave_k and wave_c are empty."""
    N = int(n_side)
    if N < 8 or N % 8 != 0:
        raise ValueError("paper_synthetic needs N >= 8, a multiple of 8")
    shape = (N, N, N)
    t = np.arange(N) * (2.0 * np.pi / N)
    f = [np.cos(a * t) + 2.0 * np.sin(a * t) for a in (1, 2, 3)]
    clean = f[0][:, None, None] * f[1][None, :, None] * f[2][None, None, :]
    rng = np.random.default_rng(seed)
    noisy = clean + rng.uniform(0.0, 1.0, shape)
    period, half = paper_mask_params(N)
    observed = (~lattice_cube_mask(shape, half, period)).astype(np.uint8)
    signal = np.where(observed == 1, noisy, 0.0)
    return Workload(shape=shape, signal=signal, observed=observed, clean=clean,
                    wave_k=np.zeros((0, 3), dtype=np.int64), wave_c=np.zeros(0, dtype=np.complex128),
                    noise_sigma=1.0 / np.sqrt(12.0), name=f"paper-synthetic-{N}-s{seed}")


def random_vector(shape, seed: int, dtype=np.float64) -> np.ndarray:
    """iid N(0,1) array of the given shape (operator-parity inputs)."""
    return np.random.default_rng(seed).standard_normal(shape).astype(dtype)


def random_barrier(shape, seed: int, spread: float = 4.0):
    """Two positive arrays log-uniform over [10^-spread, 10^spread], standing
    in for the barrier diagonals of an interior-point iterate."""
    rng = np.random.default_rng(seed)
    s1 = 10.0 ** rng.uniform(-spread, spread, size=shape)
    s2 = 10.0 ** rng.uniform(-spread, spread, size=shape)
    return s1, s2
