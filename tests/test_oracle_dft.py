"""Pins of the oracle's DFT against what the mathematics fixes.

Each test pins the oracle to something other than itself: closed forms of the
DFT of special signals, Parseval, linearity, the shift theorem, conjugate
symmetry, a hand-worked fixture, numpy's independent FFT, and the exact
twiddle values at the octant points.  The DFT definition is the one of the
TurboFFT paper, Section II (forward w_N^{jn}, inverse (1/N) w_N^{-jn}).
"""
import math
import os

import numpy as np
import pytest

import oracle

POW2 = [2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 4096]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rnd(seed, *shape):
    r = np.random.default_rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


# ------------------------------------------------------------------ twiddles

@pytest.mark.parametrize("n", [8, 64, 1024, 1 << 24])
def test_twiddle_exact_octant_points(n):
    w = oracle.omega(np.array([0, n // 4, n // 2, 3 * n // 4]), n)
    assert w[0] == 1 + 0j
    assert w[1] == -1j
    assert w[2] == -1 + 0j
    assert w[3] == 1j
    h = oracle.omega(np.array([n // 8]), n)[0]
    r = math.sqrt(0.5)
    assert abs(h.real - r) <= 2.3e-16 and abs(h.imag + r) <= 2.3e-16


@pytest.mark.parametrize("n", [3, 5, 12, 64, 4096, 1 << 20])
def test_twiddle_vs_direct_libm(n):
    t = np.unique(np.linspace(0, n - 1, num=min(n, 4000)).astype(np.int64))
    w = oracle.omega(t, n)
    ang = 2.0 * np.pi * (t.astype(np.float64) / n)
    ref = np.cos(ang) - 1j * np.sin(ang)
    # the reference itself rounds 2*pi*t/n at full angle: allow a few ulp of pi
    assert np.max(np.abs(w - ref)) < 8 * np.finfo(float).eps
    assert np.max(np.abs(np.abs(w) - 1.0)) < 3 * np.finfo(float).eps


def test_twiddle_symmetries():
    n = 1 << 12
    t = np.arange(n)
    w = oracle.omega(t, n)
    # w^t and w^{n-t} are conjugates, w^{t + n/2} = -w^t: exact by construction
    assert np.array_equal(w[1:], np.conj(w[::-1][:-1]))
    assert np.array_equal(w[n // 2:], -w[: n // 2])


# ---------------------------------------------------------- closed forms

@pytest.mark.parametrize("n", POW2)
def test_delta_and_shifted_delta(n):
    x = np.zeros(n, complex)
    x[0] = 1
    assert np.allclose(oracle.fft(x), np.ones(n), atol=1e-15, rtol=0)
    m = 3 % n
    x = np.zeros(n, complex)
    x[m] = 1
    k = np.arange(n)
    ref = np.exp(-2j * np.pi * ((m * k) % n) / n)
    assert np.max(np.abs(oracle.fft(x) - ref)) < 1e-14


@pytest.mark.parametrize("n", POW2)
def test_constant_to_spike(n):
    y = oracle.fft(np.ones(n, complex))
    ref = np.zeros(n, complex)
    ref[0] = n
    assert np.max(np.abs(y - ref)) <= 1e-13 * n


@pytest.mark.parametrize("n", [8, 64, 256, 4096])
def test_cosine_to_two_spikes(n):
    f = 3
    k = np.arange(n)
    x = np.cos(2 * np.pi * f * k / n).astype(complex)
    ref = np.zeros(n, complex)
    ref[f] += n / 2
    ref[n - f] += n / 2
    assert np.max(np.abs(oracle.fft(x) - ref)) < 1e-11 * n
    assert np.max(np.abs(oracle.dft_naive(x) - ref)) < 1e-11 * n


@pytest.mark.parametrize("n", POW2)
def test_parseval(n):
    x = rnd(n, n)
    y = oracle.fft(x)
    assert abs(np.vdot(y, y).real - n * np.vdot(x, x).real) <= 1e-12 * n * np.vdot(x, x).real


@pytest.mark.parametrize("n", [16, 256, 2048])
def test_linearity(n):
    x1, x2 = rnd(1, n), rnd(2, n)
    a, b = 0.3 - 1.7j, -2.5 + 0.25j
    lhs = oracle.fft(a * x1 + b * x2)
    rhs = a * oracle.fft(x1) + b * oracle.fft(x2)
    assert oracle.rel_l2(lhs, rhs) < 1e-14


@pytest.mark.parametrize("n", [16, 512])
def test_shift_theorem(n):
    x = rnd(5, n)
    s = 7
    k = np.arange(n)
    lhs = oracle.fft(np.roll(x, s))
    rhs = oracle.fft(x) * oracle.omega(s * k, n)
    assert oracle.rel_l2(lhs, rhs) < 1e-14


@pytest.mark.parametrize("n", [8, 1024])
def test_conjugate_symmetry_for_real_input(n):
    x = np.random.default_rng(9).standard_normal(n).astype(complex)
    y = oracle.fft(x)
    k = np.arange(n)
    assert np.max(np.abs(y[(n - k) % n] - np.conj(y))) < 1e-12 * n


def test_hand_worked_length4():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "dft4_by_hand.txt")) if l.strip() and l[0] != "#"]
    x = np.array([float(a) + 1j * float(b) for t, a, b in rows if t == "x"])
    y = np.array([float(a) + 1j * float(b) for t, a, b in rows if t == "y"])
    # small Gaussian integers and w_4 in {1, -i, -1, i}: every step is exact
    assert np.array_equal(oracle.fft(x), y)
    assert np.array_equal(oracle.dft_naive(x), y)


# ------------------------------------------------------- cross-checks

@pytest.mark.parametrize("n", POW2)
def test_naive_radix2_numpy_agree(n):
    x = rnd(100 + n, 3, n)
    yf = oracle.fft(x)
    yn = np.fft.fft(x)
    assert oracle.rel_l2(yf, yn) < 1e-13
    if n <= 1024:
        assert oracle.rel_l2(oracle.dft_naive(x), yf) < 1e-13


@pytest.mark.parametrize("n", [1 << 16, 1 << 20])
def test_large_radix2_vs_numpy(n):
    x = rnd(n, n)
    assert oracle.rel_l2(oracle.fft(x), np.fft.fft(x)) < 1e-13


@pytest.mark.parametrize("n", [2, 64, 4096])
def test_inverse(n):
    x = rnd(7 + n, 2, n)
    y = oracle.fft(x)
    assert oracle.rel_l2(oracle.ifft(y), x) < 1e-14
    assert oracle.rel_l2(oracle.ifft(x), np.conj(oracle.fft(np.conj(x))) / n) < 1e-15
    assert oracle.rel_l2(oracle.ifft(x), np.fft.ifft(x)) < 1e-13
    if n <= 1024:
        assert oracle.rel_l2(oracle.dft_naive(x, inverse=True), oracle.ifft(x)) < 1e-13


def test_rejects_non_power_of_two():
    with pytest.raises(ValueError):
        oracle.fft(np.ones(12, complex))
    # the direct sum has no such restriction
    x = rnd(3, 12)
    assert oracle.rel_l2(oracle.dft_naive(x), np.fft.fft(x)) < 1e-13


# ------------------------------------------------------- fault injection

def bitrev(v, bits):
    return int(format(v, f"0{bits}b")[::-1], 2) if bits else 0


@pytest.mark.parametrize("n", [8, 64])
def test_leaf_fault_equals_input_perturbation(n):
    """A fault on leaf v of the recursion is a perturbation of input element
    bitrev(v): its effect on the output is delta * w^{k bitrev(v)} (the DFT of a
    shifted delta), which pins the node numbering of the injection hook."""
    x = rnd(11, n)
    L = int(math.log2(n))
    k = np.arange(n)
    d = 0.5 - 0.25j
    for v in range(n):
        y = oracle.fft_faulty(x, [(L, v, 0, d)])
        ref = oracle.fft(x) + d * oracle.omega(k * bitrev(v, L), n)
        assert oracle.rel_l2(y, ref) < 1e-14


def test_root_fault_touches_one_output():
    n = 32
    x = rnd(12, n)
    y = oracle.fft_faulty(x, [(0, 0, 5, 1.0 + 2.0j)])
    diff = y - oracle.fft(x)
    assert np.count_nonzero(np.abs(diff) > 1e-12) == 1
    assert abs(diff[5] - (1.0 + 2.0j)) < 1e-13


def test_no_fault_is_plain_fft():
    x = rnd(13, 64)
    assert np.array_equal(oracle.fft_faulty(x, []), oracle.fft(x))


# ------------------------------------------------------------ four-step

@pytest.mark.parametrize("n1,n2", [(2, 4), (8, 8), (16, 64), (64, 16), (256, 512)])
@pytest.mark.parametrize("inverse", [False, True])
def test_fourstep_matches_direct(n1, n2, inverse):
    x = rnd(n1 * 7 + n2, 2, n1 * n2)
    r = oracle.fourstep(x, n1, n2, inverse=inverse)
    ref = np.fft.ifft(x) if inverse else np.fft.fft(x)
    assert oracle.rel_l2(r["y"], ref) < 1e-13
