"""Pins of the oracle's one-sided and thread-level checksum schemes (TurboFFT
Section II-C applied per signal, Section IV-B.1 per butterfly, compared in
Section V).

What pins them, other than themselves:
* c1 of a butterfly is the closed-form checksum vector of a length-r group
  (already pinned against a 40-digit sum); c2 = W^T ((k+1) e) against the
  derivative of the geometric series, sum_k (k+1) z^k =
  (1 - (r+1) z^r + r z^(r+1)) / (1 - z)^2, with z from the standard library;
* every output of every butterfly of radix 2, 4, 8: one wrong value eps is
  flagged, located (d2/d1 = k+1) and |d1| = |eps| because |e_k| = 1;
* butterflies computed in binary32 (numpy's single-precision FFT) raise no
  false alarm at kappa = 16, for uniform and six-decade inputs;
* the one-sided scheme detects every single fault at every node of the
  radix-2 recursion (N = 8..64) with |d1| >= (sqrt 3 / 2) |eps|, and its
  recomputation returns the exact transform; two faults in two signals are
  both corrected, which the two-sided group check cannot do.
"""
import cmath
import math

import numpy as np
import pytest

import oracle
import tfft_inputs as inputs

U64 = 2.0 ** -52


def rnd(seed, *shape):
    r = np.random.default_rng(seed)
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


@pytest.mark.parametrize("r", [2, 4, 8])
def test_butterfly_c1_is_the_group_checksum_vector(r):
    _, _, c1, _ = oracle.butterfly_vectors(r)
    assert np.max(np.abs(c1 - oracle.checksum_vector(r))) < 1e-14


@pytest.mark.parametrize("r", [2, 4, 8])
def test_butterfly_c2_closed_form(r):
    _, f, _, c2 = oracle.butterfly_vectors(r)
    for q in range(r):
        z = cmath.exp(-2j * math.pi * (1 / 3 + q / r))
        closed = (1 - (r + 1) * z ** r + r * z ** (r + 1)) / (1 - z) ** 2
        assert abs(c2[q] - closed) < 1e-13 * r * r, (q, c2[q], closed)
    assert np.allclose(f, np.arange(1, r + 1) * oracle.encoding_vector(r), rtol=0, atol=0)


@pytest.mark.parametrize("r", [2, 4, 8])
def test_butterfly_locates_every_output(r):
    rng = np.random.default_rng(77 + r)
    for t in range(40):
        v = rnd(1000 * r + t, r)
        y = oracle.dft_naive(v[None, :])[0]
        d1, _, _, flagged, _ = oracle.butterfly_check(v, y, u=U64)
        assert not flagged and abs(d1) < 1e-13 * np.linalg.norm(v)
        for k in range(r):
            eps = complex(*rng.uniform(-1, 1, 2)) * 10.0 ** rng.uniform(-6, 2)
            yf = y.copy()
            yf[k] += eps
            d1, d2, tau, flagged, loc = oracle.butterfly_check(v, yf, u=U64)
            assert flagged and loc == k, (t, k, d2 / d1)
            assert abs(abs(d1) - abs(eps)) <= 1e-12 * (abs(eps) + np.linalg.norm(v))


def test_butterfly_nonfinite_output_is_flagged_not_located():
    v = rnd(5, 8)
    y = oracle.dft_naive(v[None, :])[0]
    y[3] = complex(np.inf, 0.0)
    _, _, _, flagged, loc = oracle.butterfly_check(v, y)
    assert flagged and loc == -1


@pytest.mark.parametrize("kind", ["uniform", "dynamic"])
def test_butterfly_binary32_has_no_false_alarm(kind):
    gen = inputs.uniform if kind == "uniform" else inputs.dynamic
    for r in (2, 4, 8):
        v = gen(4242 + r, 20000, r, np.complex64)
        y = np.fft.fft(v, axis=1)
        assert y.dtype == np.complex64  # numpy computes it in binary32
        worst = 0.0
        for i in range(v.shape[0]):
            d1, _, tau, flagged, _ = oracle.butterfly_check(v[i], y[i], kappa=16.0, u=2.0 ** -24)
            assert not flagged, (r, i)
            worst = max(worst, abs(d1) / tau)
        assert worst < 0.5  # margin: the largest residual stays well inside tau


@pytest.mark.parametrize("n", [8, 16, 32, 64])
def test_one_sided_detects_every_single_fault(n):
    L = int(math.log2(n))
    x = rnd(300 + n, n)
    y = oracle.fft(x)
    ph = np.random.default_rng(n)
    worst = np.inf
    for level in range(L + 1):
        for node in range(1 << level):
            for idx in range(n >> level):
                eps = np.exp(2j * np.pi * ph.uniform())
                yf = oracle.fft_faulty(x, [(level, node, idx, eps)])
                out, rec = oracle.one_sided_signal(x, yf, u=U64)
                assert rec.flagged and rec.action == oracle.CORRECTED
                assert oracle.rel_l2(out, y) < 1e-15
                worst = min(worst, abs(rec.d1) / abs(eps))
    assert worst >= math.sqrt(3) / 2 * (1 - 1e-9)


def test_one_sided_corrects_two_faulty_signals_of_one_group():
    G, n = 4, 64
    X = rnd(21, G, n)
    Y = oracle.fft(X)
    Yf = Y.copy()
    Yf[1, 5] += 1.0
    Yf[2, 40] -= 0.5j
    _, grec = oracle.two_sided_group(X, Yf, u=U64)
    assert grec.action == oracle.UNCORRECTABLE
    out = np.empty_like(Y)
    for b in range(G):
        out[b], rec = oracle.one_sided_signal(X[b], Yf[b], u=U64, signal=b)
        assert rec.flagged == (b in (1, 2))
    assert oracle.rel_l2(out, Y) < 1e-15


def test_one_sided_inverse_scale():
    x = rnd(9, 256)
    y = oracle.fft(x, inverse=True)
    out, rec = oracle.one_sided_signal(x, y, inverse=True, scale=1.0 / 256, u=U64)
    assert not rec.flagged
    yf = y.copy()
    yf[17] += 1e-3
    out, rec = oracle.one_sided_signal(x, yf, inverse=True, scale=1.0 / 256, u=U64)
    assert rec.flagged and oracle.rel_l2(out, y) < 1e-15
