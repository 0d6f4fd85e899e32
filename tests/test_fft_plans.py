"""The Stockham stage plans of the pencil FFT kernels, restated on the CPU
(no GPU): for every length the register-resident kernels are instantiated
at (csrc/fft_kernels.h: Radix<L, E> with the elements per thread of each
pass) and every length 2^a 3^b 5^c 7^d up to 1024 of the LDS-resident passes
(csrc/fft_any.hip: the plan computed at launch, TM pencils of NT threads,
in both precisions' workgroup shapes),
the stages, run in numpy with the kernels' butterfly indexing, give numpy's
FFT in both directions; each stage's butterflies are all taken by some
thread, and its outputs write every element exactly once.  The stage
twiddles, formed from one table entry per butterfly (one per thread where
its butterflies share it, or one per thread times a uniform entry) by
products, equal the table's powers, and every index read stays in the table; the axis-3 packing twiddle of element
t + k is the product of the entries t and k with k below L.  The axis-3
packing algebra and the scale the launch passes per mode reproduce numpy's
orthonormal rfft/irfft."""
import numpy as np
import pytest


def odd_part(x):
    while x > 0 and x % 2 == 0:
        x //= 2
    return x


def smallest_odd_factor(x):
    p = 3
    while p <= x:
        if x % p == 0:
            return p
        p += 2
    return x


def odd_factors(F):
    out = []
    while F > 1:
        p = smallest_odd_factor(F)
        out.append(p)
        F //= p
    return out


def radix_plan(L, E):
    """Radix<L, E>: power-of-two stages of radix P2 (the power-of-two part of
    E; 4 when E is odd), one remainder stage, then the odd prime factors."""
    if L == 1:
        return [1]
    LP = L // odd_part(L)
    P2 = E // odd_part(E) if E // odd_part(E) > 1 else min(LP, 4)
    st, r = [], LP
    while P2 > 1 and r >= P2:
        st.append(P2)
        r //= P2
    if r > 1:
        st.append(r)
    return st + odd_factors(odd_part(L))


def any_plan(L):
    """The LDS-resident passes' plan: radix 8, then one 4 or 2, then 3, 5, 7."""
    a, r = 0, L
    while r % 2 == 0:
        r //= 2
        a += 1
    st = [8] * (a // 3) + ([1 << (a % 3)] if a % 3 else [])
    for f in (3, 5, 7):
        while r % f == 0:
            st.append(f)
            r //= f
    return st if r == 1 else None


# threads per workgroup of the LDS-resident passes: FP32 512, FP64 256
ANY_THREADS = {"f32": 512, "f64": 256}


def any_tm(threads, L):
    tm = threads
    while tm > 1 and tm * L > 4096:
        tm //= 2
    return tm


def run_stages(x, plan, nthreads, nb_of, direction):
    """The Stockham stages with the kernels' indexing: stage radix R, Ns the
    product of the earlier radices; butterfly j (taken by thread j % nthreads
    in round j // nthreads) reads elements j + q L/R, multiplies input q by
    w^(jm q L/(Ns R)) (jm = j mod Ns, w = exp(-+2 pi i / L)), and writes its
    DFT output q to (j - jm) R + jm + q Ns."""
    L = len(x)
    a = x.astype(np.complex128)
    tw = np.exp(-2j * np.pi * np.arange(L) / L)
    if direction > 0:
        tw = tw.conj()
    ns = 1
    for R in plan:
        nbf = L // R
        assert nbf * R == L
        # every butterfly has a thread in one of the stage's rounds
        assert nb_of(R) * nthreads >= nbf, (L, R)
        j = np.arange(nbf)
        jm = j % ns
        q = np.arange(R)
        v = a[j[:, None] + q[None, :] * nbf]
        v = v * tw[(jm[:, None] * q[None, :] * (L // (ns * R))) % L]
        dft = np.exp(direction * 2j * np.pi * np.outer(q, q) / R)
        y = v @ dft
        dst = (j - jm)[:, None] * R + jm[:, None] + q[None, :] * ns
        assert dst.min() >= 0 and dst.max() < L
        assert np.array_equal(np.sort(dst.ravel()), np.arange(L)), "each element written once"
        out = np.empty_like(a)
        out[dst.ravel()] = y.ravel()
        a = out
        ns *= R
    assert ns == L
    return a


def check_fft(L, plan, nthreads, nb_of):
    rng = np.random.default_rng(L)
    x = rng.standard_normal(L) + 1j * rng.standard_normal(L)
    scale = np.abs(np.fft.fft(x)).max()
    assert np.abs(run_stages(x, plan, nthreads, nb_of, -1) - np.fft.fft(x)).max() <= 1e-12 * scale
    assert np.abs(run_stages(x, plan, nthreads, nb_of, +1) - np.fft.ifft(x) * L).max() <= 1e-12 * scale


MIXED = [12, 20, 24, 28, 40, 48, 56, 70, 96, 192, 384, 560]
ODD = [3, 5, 7, 9, 15, 21, 35, 45]


def mixed_e(L):
    F = odd_part(L)
    P = L // F
    f = F if F <= 7 else smallest_odd_factor(F)
    return f * min(P, 4)


def a3_e(L):
    if odd_part(L) == 1:
        return min(L, 8)
    if odd_part(L) > 7:
        P = L // odd_part(L)
        return smallest_odd_factor(odd_part(L)) * min(P, 2)
    return mixed_e(L)


def register_cases():
    """(L, E) of every instantiated pencil: strided passes (E 8 or 16 at
    powers of two, mixed_e otherwise) and axis-3 half lengths (a3_e)."""
    cases = set()
    for k in range(0, 11):
        L = 1 << k
        cases.add((L, min(L, 8)))
        cases.add((L, min(L, 16)))
    for L in MIXED + ODD:
        cases.add((L, mixed_e(L)))
    for L in [1 << k for k in range(1, 10)] + [N // 2 for N in MIXED]:
        cases.add((L, a3_e(L)))
    return sorted(cases)


@pytest.mark.parametrize("L,E", register_cases())
def test_register_plan(L, E):
    assert L % E == 0
    NT = L // E
    plan = radix_plan(L, E)
    if L == 1:
        return
    check_fft(L, plan, NT, lambda R: -(-(L // R) // NT))


SMOOTH = [L for L in range(1, 1025) if any_plan(L) is not None]


def test_any_lengths():
    assert len(SMOOTH) == 143
    assert all(any_plan(L) is None for L in (11, 13, 22, 1001))


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("L", [L for L in SMOOTH if L >= 3])
def test_any_plan(L, prec):
    plan = any_plan(L)
    assert len(plan) <= 12
    threads = ANY_THREADS[prec]
    emax = 4096 // threads
    tm = any_tm(threads, L)
    nt = threads // tm
    # the self-paired rows of the axis-1 passes take four lanes of one
    # workgroup; a thread holds at most emax values (8 in FP32, 16 in FP64)
    assert tm >= 4 and -(-L // nt) <= emax
    check_fft(L, plan, nt, lambda R: -(-emax // R))


def product_twiddles(w1, r):
    """w^q for q < r from w^1 by the kernels' product tree: w^q = (w^(q/2))^2
    for q a power of two, else w^(q - hb) w^hb (hb the highest power of two
    below q)."""
    wq = [1.0 + 0j, w1]
    for q in range(2, r):
        hb = 1 << (q.bit_length() - 1)
        wq.append(wq[hb // 2] * wq[hb // 2] if q == hb else wq[q - hb] * wq[hb])
    return wq


def kernel_stage_twiddles(L, stage_radices, s, t, i, NT, direction):
    """The twiddles w^(jm q TS) of butterfly j = t + i NT of stage s as the
    kernels form them: where NT is a multiple of Ns (several butterflies per
    thread) the entry of (t mod Ns) TS, shared by the thread's butterflies;
    else, where every butterfly of the thread has jm = j (L / r <= Ns), the
    entry of t TS times the uniform entry of i NT TS; else the entry of
    jm TS; then the product tree.  Returns (powers, table indices read)."""
    r = stage_radices[s]
    ns = int(np.prod(stage_radices[:s]))
    TS = L // (ns * r)
    NB = -(-(L // r) // NT)
    tab = np.exp(-2j * np.pi * np.arange(L) / L)
    if direction > 0:
        tab = tab.conj()
    j = t + i * NT
    if NB > 1 and NT % ns == 0:
        idx = [(t % ns) * TS]
        w1 = tab[idx[0]]
    elif NB > 1 and L // r <= ns:
        idx = [t * TS, i * NT * TS]
        w1 = tab[idx[0]] * (tab[idx[1]] if i else 1.0)
    else:
        idx = [(j % ns) * TS]
        w1 = tab[idx[0]]
    return product_twiddles(w1, r), idx


@pytest.mark.parametrize("L,E", [c for c in register_cases() if c[0] >= 3])
def test_product_twiddles_match_table(L, E):
    """Every pencil the register-resident kernels instantiate: in the stages
    whose thread shares one load (by jm = t mod Ns or by jm = j), the shared
    index is the butterfly's own up to the uniform factor, every index read
    stays inside the length-L table, and the product-formed twiddles equal
    w^(jm q TS) to rounding."""
    plan = radix_plan(L, E)
    NT = L // E
    for s, r in enumerate(plan):
        ns = int(np.prod(plan[:s]))
        if ns == 1:
            continue
        TS = L // (ns * r)
        NB = -(-(L // r) // NT)
        if NB > 1 and NT % ns != 0 and L // r <= ns:
            assert TS == 1
        for direction in (-1, 1):
            for t in range(NT):
                for i in range(NB):
                    j = t + i * NT
                    if j >= L // r:
                        continue
                    wq, idx = kernel_stage_twiddles(L, plan, s, t, i, NT, direction)
                    assert all(0 <= x < L for x in idx)
                    jm = j % ns
                    want = np.exp(direction * 2j * np.pi * jm * TS * np.arange(r) / L)
                    assert np.abs(np.array(wq) - want).max() < 1e-13


@pytest.mark.parametrize("L", [1 << k for k in range(1, 10)] + [N // 2 for N in MIXED])
def test_packing_twiddle_offsets(L):
    """The c2r/r2c packing twiddle exp(-2 pi i e / N3) of element e = t + k
    of the first-stage pattern is tw3[t] tw3[k]: k = e - t is fixed by the
    unrolled slot (the same for every thread) and stays below L, the table's
    first L entries."""
    E = a3_e(L)
    NT = L // E
    plan = radix_plan(L, E)
    r0 = plan[0]
    N3 = 2 * L
    offsets = None
    for t in range(NT):
        ks = []
        for i in range(-(-(L // r0) // NT)):
            j = t + i * NT
            if j >= L // r0:
                continue
            for q in range(r0):
                e = j + q * (L // r0)
                k = e - t
                assert 0 <= k < L
                assert abs(np.exp(-2j * np.pi * t / N3) * np.exp(-2j * np.pi * k / N3) - np.exp(-2j * np.pi * e / N3)) < 1e-14
                ks.append((i, q, k))
        if offsets is None:
            offsets = ks
        elif len(ks) == len(offsets):
            assert ks == offsets


def _axis3_model(X, L, mode, mask=None):
    """The axis-3 pass of one pencil as the kernels compute it, in numpy:
    the unscaled packing (sqrt2 times the inverse input; twice the half
    spectrum, DC and Nyquist once) and the one scale per output kind that the
    launch passes for each mode (n = N3 here: a single pencil)."""
    N3 = 2 * L
    rn, r2 = 1.0 / np.sqrt(N3), np.sqrt(2.0)
    w = np.exp(-2j * np.pi * np.arange(L) / N3)
    if mode == "r2c":
        z = X
    else:
        Z = np.empty(L, complex)
        Z[0] = r2 * complex(X[0].real + X[0].imag, X[0].real - X[0].imag)
        e = np.arange(1, L)
        a, b = X[e], np.conj(X[L - e])
        Z[e] = (a + b) + 1j * np.conj(w[e]) * (a - b)
        z = np.fft.ifft(Z) * L                       # unnormalised inverse
        if mode == "c2r":
            return z * (rn / r2)
        z = z.real * mask[0::2] + 1j * z.imag * mask[1::2]
    full = mode == "full"
    sc_dc = rn * rn / r2 if full else rn
    sc_ac = rn * rn / 2 if full else rn / r2
    Y = np.fft.fft(z)                                # unnormalised forward
    out = np.empty(L, complex)
    out[0] = sc_dc * complex(Y[0].real + Y[0].imag, Y[0].real - Y[0].imag)
    e = np.arange(1, L)
    a, b = Y[e], np.conj(Y[L - e])
    out[e] = sc_ac * ((a + b) - 1j * w[e] * (a - b))
    return out


@pytest.mark.parametrize("L", [2, 4, 8, 12, 64, 128, 280])
def test_axis3_packing_and_scales(L):
    """Against numpy's orthonormal rfft/irfft of a length-2L pencil, with the
    half spectrum in the kernels' layout (slot 0 = (DC, Nyquist), the other
    coefficients times sqrt2): the c2r and r2c modes with their scales are
    the orthonormal transforms, and the full pass (no scale between its two
    transforms) equals r2c(mask(c2r(.)))."""
    N3 = 2 * L
    rng = np.random.default_rng(L)
    x = rng.standard_normal(N3)
    F = np.fft.rfft(x, norm="ortho")                 # F_0 .. F_L
    X = np.sqrt(2.0) * F[:L].copy()
    X[0] = complex(F[0].real, F[L].real)
    z = _axis3_model(X, L, "c2r")
    assert np.abs(np.concatenate([[v.real, v.imag] for v in z]) - x).max() < 1e-12
    pairs = x[0::2] + 1j * x[1::2]
    assert np.abs(_axis3_model(pairs, L, "r2c") - X).max() < 1e-12
    mask = (rng.random(N3) < 0.7).astype(float)
    xm = np.fft.irfft(F, n=N3, norm="ortho") * mask
    Fm = np.fft.rfft(xm, norm="ortho")
    Xm = np.sqrt(2.0) * Fm[:L].copy()
    Xm[0] = complex(Fm[0].real, Fm[L].real)
    assert np.abs(_axis3_model(X, L, "full", mask) - Xm).max() < 1e-12
