"""Pins of the oracle's two-sided checksum (TurboFFT paper, Sections II-C and III).

What pins it, other than itself:
* the closed form of c = (e^T W)^T against the term-by-term sum, and its norm
  ||c||_2 = M (W^T W = M I up to conjugation);
* exact Gaussian-integer arithmetic at N in {2, 4}, where every DFT entry is
  in {1, -1, i, -i}, so Eq. (1), (2), (4), (5), the quotient location and the
  correction must hold with no rounding at all;
* exhaustive single-fault injection at every node and index of the radix-2
  recursion (N = 8..64): every fault is detected, located and corrected, and
  |d1| >= (sqrt 3 / 2) |eps| (the bound for e = w_3^k);
* the all-ones encoding vector, which the paper says misses errors, must
  leave some of the same faults undetected (so the pin above has teeth);
* the per-pass domains of a two-pass plan: clean passes are never flagged
  and pass-1 output faults are corrected through the twiddle.
"""
import math

import numpy as np
import pytest

import oracle

U64 = 2.0 ** -52


def rnd(seed, *shape):
    r = np.random.default_rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


def gauss_int(seed, *shape, lo=-5, hi=6):
    r = np.random.default_rng(seed)
    return r.integers(lo, hi, size=shape) + 1j * r.integers(lo, hi, size=shape)


# --------------------------------------------------------------- vectors

@pytest.mark.parametrize("m", [2, 4, 8, 64, 256, 1024])
@pytest.mark.parametrize("inverse", [False, True])
def test_checksum_vector_closed_form(m, inverse):
    s = 1.0 / m if inverse else 1.0
    c = oracle.checksum_vector(m, inverse, s)
    d = oracle.checksum_vector_direct(m, inverse, s, exact_sum=True)
    # each binary64 term of the direct sum is off by about an ulp, so the two
    # agree to a random walk of m such errors
    assert np.max(np.abs(c - d)) <= 32 * np.finfo(float).eps * math.sqrt(m) * s
    assert abs(np.linalg.norm(c) - m * s) <= 1e-12 * m * s
    assert np.min(np.abs(c)) > 0.8 * s   # never zero: every single fault is seen


@pytest.mark.parametrize("m", [8, 64, 256])
@pytest.mark.parametrize("inverse", [False, True])
def test_checksum_vector_vs_high_precision_direct_sum(m, inverse):
    """Every entry, small or large, within a few ulp of the defining sum
    sum_k w_3^k w_m^{+-kn} evaluated term by term in 40-digit arithmetic."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    c = oracle.checksum_vector(m, inverse)
    w3 = mpmath.exp(-2j * mpmath.pi / 3)
    sgn = 1 if inverse else -1
    worst = 0.0
    for n in range(m):
        z = w3 * mpmath.exp(sgn * 2j * mpmath.pi * n / m)
        acc, zk = mpmath.mpc(0), mpmath.mpc(1)
        for _ in range(m):
            acc += zk
            zk *= z
        worst = max(worst, float(abs(mpmath.mpc(c[n]) - acc) / abs(acc)))
    assert worst <= 4 * np.finfo(float).eps


def test_encoding_vector_is_w3_powers():
    e = oracle.encoding_vector(7)
    w3 = complex(-0.5, -math.sqrt(3) / 2)
    ref = np.array([w3 ** k for k in range(7)])
    assert np.max(np.abs(e - ref)) < 1e-15
    assert e[0] == 1 and e[3] == 1 and e[6] == 1


@pytest.mark.parametrize("m", [64, 4096])
@pytest.mark.parametrize("inverse", [False, True])
def test_left_right_identity_fp64(m, inverse):
    """Eq. (2): (e^T W) x = e^T (W x) for random x."""
    x = rnd(m, m)
    s = 1.0 / m if inverse else 1.0
    lhs = np.dot(oracle.checksum_vector(m, inverse, s), x)
    rhs = np.dot(oracle.encoding_vector(m), oracle.fft(x, inverse=inverse, scale=s))
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs) + 1e-12 * np.linalg.norm(x) * math.sqrt(m)


# ------------------------------------------------- exact small-N algebra

@pytest.mark.parametrize("m", [2, 4])
@pytest.mark.parametrize("e_kind", ["quarter", "random"])
def test_exact_gaussian_integer_algebra(m, e_kind):
    """At N in {2, 4} the DFT matrix has entries in {1, -i, -1, i}; with
    Gaussian-integer inputs, faults and encoding vectors every quantity of
    Eq. (4)-(5) is an exact small integer in binary64."""
    G = 5
    e = (np.array([1, 1j, -1, -1j])[:m] if e_kind == "quarter" else gauss_int(99, m, lo=-3, hi=4))
    X = gauss_int(m, G, m)
    Y = oracle.fft(X)
    W = oracle.omega(np.outer(np.arange(m), np.arange(m)) % m, m)
    assert np.array_equal(Y, X @ W.T)                       # exact DFT
    c = oracle.checksum_vector_direct(m, False, 1.0, e)
    assert np.array_equal(c, W.T @ e)
    for b in range(G):
        assert np.dot(c, X[b]) == np.dot(e, Y[b])           # Eq. (2), exactly
    w1 = np.ones(G)
    assert np.array_equal(oracle.fft(w1 @ X), w1 @ Y)       # W(Xw) = (WX)w
    for j in range(G):
        for k in range(m):
            delta = complex(3, -2)
            Yf = Y.copy()
            Yf[j, k] += delta
            if np.dot(e, np.eye(m)[k]) == 0:
                continue
            out, rec = oracle.two_sided_group(X, Yf, e=e, u=0.0, kappa=1.0)
            assert rec.flagged
            assert rec.d1 == e[k] * delta
            assert rec.d2 == (j + 1) * e[k] * delta
            assert rec.rho == j + 1
            assert rec.located == j and rec.method == "quotient"
            assert rec.action == oracle.CORRECTED
            assert np.array_equal(out, Y)                    # exact restoration
    out, rec = oracle.two_sided_group(X, Y, e=e, u=0.0, kappa=1.0)
    assert not rec.flagged and rec.d1 == 0 and rec.d2 == 0


# ------------------------------------------------- exhaustive injection

def all_faults(n):
    L = int(math.log2(n))
    for level in range(L + 1):
        for node in range(1 << level):
            for idx in range(n >> level):
                yield level, node, idx


@pytest.mark.parametrize("n", [8, 16, 32, 64])
@pytest.mark.parametrize("G", [1, 4, 16])
def test_exhaustive_single_fault(n, G):
    X = rnd(1000 + n + G, G, n)
    Y = oracle.fft(X)
    ph = np.random.default_rng(n * G)
    worst = np.inf
    count = 0
    for i, (level, node, idx) in enumerate(all_faults(n)):
        j = i % G
        eps = np.exp(2j * np.pi * ph.uniform())
        Yf = Y.copy()
        Yf[j] = oracle.fft_faulty(X[j], [(level, node, idx, eps)])
        out, rec = oracle.two_sided_group(X, Yf, u=U64, kappa=16.0)
        assert rec.flagged, (level, node, idx)
        assert rec.located == j and rec.method == "quotient", (level, node, idx, rec.rho)
        assert rec.action == oracle.CORRECTED
        assert oracle.rel_l2(out, Y) < 1e-13
        worst = min(worst, abs(rec.d1) / abs(eps))
        count += 1
    assert count == n * (int(math.log2(n)) + 1)
    assert worst >= math.sqrt(3) / 2 * (1 - 1e-9)


def test_all_ones_vector_misses_faults():
    """The paper: the 1's vector misses errors.  With e = ones the same
    single faults that e = w_3^k always catches can leave d1 = 0."""
    n, G = 64, 1
    X = rnd(5, G, n)
    Y = oracle.fft(X)
    missed = 0
    for level, node, idx in all_faults(n):
        if level == int(math.log2(n)):
            continue
        Yf = Y.copy()
        Yf[0] = oracle.fft_faulty(X[0], [(level, node, idx, 1.0)])
        _, rec = oracle.two_sided_group(X, Yf, e=np.ones(n), u=U64, kappa=16.0)
        missed += not rec.flagged
    assert missed > 100


# ------------------------------------------------- outside the single fault

def test_two_faults_in_one_group_are_uncorrectable():
    G, n = 8, 64
    X = rnd(21, G, n)
    Y = oracle.fft(X)
    Yf = Y.copy()
    Yf[1, 5] += 2.0 + 1.0j
    Yf[6, 40] += -1.5 + 3.0j
    out, rec = oracle.two_sided_group(X, Yf, u=U64, kappa=16.0)
    assert rec.flagged and rec.located == -1
    assert rec.action == oracle.UNCORRECTABLE


def test_fault_in_checksum_arithmetic_is_benign():
    G, n = 8, 64
    X = rnd(22, G, n)
    Y = oracle.fft(X)
    tau = oracle.threshold(n, float(np.sum(np.abs(X) ** 2)), 16.0, U64)
    out, rec = oracle.two_sided_group(X, Y, u=U64, kappa=16.0, r1_fault=1e3 * tau)
    assert rec.flagged and rec.located == -1 and rec.action == oracle.BENIGN
    assert np.array_equal(out, Y)


@pytest.mark.parametrize("bad", [np.inf, np.nan])
def test_non_finite_fault_is_located_per_signal_and_corrected(bad):
    G, n = 4, 32
    X = rnd(23, G, n)
    Y = oracle.fft(X)
    Yf = Y.copy()
    Yf[2, 7] = complex(bad, 0.0)
    out, rec = oracle.two_sided_group(X, Yf, u=U64, kappa=16.0)
    assert rec.flagged and rec.located == 2 and rec.method == "per-signal"
    assert oracle.rel_l2(out, Y) < 1e-13


def test_detect_mode_reports_without_correcting():
    G, n = 4, 64
    X = rnd(24, G, n)
    Y = oracle.fft(X)
    Yf = Y.copy()
    Yf[3, 0] += 1.0
    out, rec = oracle.two_sided_group(X, Yf, u=U64, kappa=16.0, mode="detect")
    assert rec.action == oracle.DETECTED and rec.located == 3
    assert np.array_equal(out, Yf)


@pytest.mark.parametrize("inverse", [False, True])
def test_inverse_direction_checksum(inverse):
    G, n = 4, 256
    X = rnd(25, G, n)
    s = 1.0 / n if inverse else 1.0
    Y = oracle.fft(X, inverse=inverse, scale=s)
    _, rec = oracle.two_sided_group(X, Y, inverse=inverse, scale=s, u=U64, kappa=16.0)
    assert not rec.flagged
    Yf = Y.copy()
    Yf[1, 100] += 0.01
    out, rec = oracle.two_sided_group(X, Yf, inverse=inverse, scale=s, u=U64, kappa=16.0)
    assert rec.located == 1 and oracle.rel_l2(out, Y) < 1e-13


# ---------------------------------------------- the FP32 noise floor

def test_fp32_noise_below_threshold():
    """Single-precision outputs (numpy's own float32 FFT) on uniform inputs
    never cross tau at kappa = 16, while a unit fault always does."""
    M, G, groups = 1024, 16, 64
    r = np.random.default_rng(7)
    X = (r.uniform(-1, 1, (groups * G, M)) + 1j * r.uniform(-1, 1, (groups * G, M))).astype(np.complex64)
    Y = np.fft.fft(X)
    assert Y.dtype == np.complex64
    _, recs = oracle.two_sided_batch(X, Y, G, u=2.0 ** -24, kappa=16.0)
    assert recs == []
    Yf = Y.astype(np.complex128)
    Yf[5 * G + 3, 17] += 1.0
    out, recs = oracle.two_sided_batch(X, Yf, G, u=2.0 ** -24, kappa=16.0)
    assert len(recs) == 1 and recs[0].group == 5 and recs[0].located == 3
    assert oracle.rel_l2(out[5 * G + 3], oracle.fft(X[5 * G + 3].astype(np.complex128))) < 1e-6


# ------------------------------------------------------ two-pass domains

@pytest.mark.parametrize("inverse", [False, True])
def test_two_pass_domains(inverse):
    n1, n2, G = 16, 32, 8
    x = rnd(31, 1, n1 * n2)
    r = oracle.fourstep(x, n1, n2, inverse=inverse)
    N = n1 * n2
    X1 = x[0].reshape(n1, n2).T           # signals = columns n2
    Y1 = r["mid"][0].T                    # twiddled column transforms
    tw1 = r["tw"].T
    kw = dict(inverse=inverse, u=U64, kappa=16.0)
    _, recs = oracle.two_sided_batch(X1, Y1, G, out_twiddle=tw1, **kw)
    assert recs == []
    # without absorbing the twiddle into e the clean pass would be flagged
    _, recs = oracle.two_sided_batch(X1, Y1, G, **kw)
    assert len(recs) > 0
    Y1f = Y1.copy()
    Y1f[11, 3] += 0.5j
    out, recs = oracle.two_sided_batch(X1, Y1f, G, out_twiddle=tw1, **kw)
    assert len(recs) == 1 and recs[0].located == 3
    assert oracle.rel_l2(out, Y1) < 1e-13
    # pass 2: rows of the pass-1 output, scale 1/N for the inverse
    s = 1.0 / N if inverse else 1.0
    X2, Y2 = r["mid"][0], r["out"][0]
    _, recs = oracle.two_sided_batch(X2, Y2, G, scale=s, **kw)
    assert recs == []
    Y2f = Y2.copy()
    Y2f[9, 30] -= 0.25 * s
    out, recs = oracle.two_sided_batch(X2, Y2f, G, scale=s, **kw)
    assert len(recs) == 1 and recs[0].located == 1
    assert oracle.rel_l2(out, Y2) < 1e-13
