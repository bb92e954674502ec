"""Pin of the threshold's form (CPU).

The paper tests the checksum residual against a threshold picked from its ROC
study and prints no value (Section II-C and the fault-coverage study of
Section V).  The reading used here is tau = kappa * u * sqrt(log2 M) *
sqrt(M * S): the expected rounding noise of a length-M FFT of a group of
signals of total energy S.  kappa itself is calibrated, not pinned; what is
pinned below is the *form*: with two binary32 FFTs that share nothing with
either implementation (numpy's pocketfft in single precision, and a textbook
radix-2 written here with complex64 arithmetic), the noise-scaled residual
|d1| / (tau / kappa) of fault-free groups stays in one fixed band for
M = 2^4..2^12, groups of G = 1, 4, 16, 64 signals, and uniform and six-decade
lognormal inputs, and it stays well below the default kappa.  Forms with the
wrong growth in M or in G leave the band (negative controls).
"""
import functools
import math

import numpy as np
import pytest

import oracle
import tfft_inputs as inputs

U32 = 2.0 ** -24
KAPPA32 = 16.0  # the library's default for complex64


def radix2_binary32(x):
    """Iterative radix-2 decimation in time in complex64 arithmetic (twiddles
    rounded once from binary64): a binary32 FFT whose rounding error grows
    like sqrt(log2 M)."""
    x = np.asarray(x, np.complex64)
    B, n = x.shape
    bits = n.bit_length() - 1
    rev = np.array([int(format(i, f"0{bits}b")[::-1], 2) for i in range(n)])
    a = x[:, rev].copy()
    tw = oracle.omega_table(n, n // 2).astype(np.complex64)
    h = 1
    while h < n:
        w = tw[np.arange(h) * (n // (2 * h))]
        a = a.reshape(B, n // (2 * h), 2, h)
        t = a[:, :, 1, :] * w
        lo = a[:, :, 0, :]
        a = np.stack([lo + t, lo - t], axis=2).reshape(B, n)
        h *= 2
    return a


def numpy_binary32(x):
    y = np.fft.fft(np.asarray(x, np.complex64), axis=-1)
    assert y.dtype == np.complex64  # numpy >= 2 transforms complex64 in single precision
    return y


@functools.lru_cache(maxsize=None)
def residuals(M, G, kind, fft32):
    """d1 and S of fault-free groups (binary64 checksums on binary32
    transforms)."""
    gen = inputs.uniform if kind == "uniform" else inputs.dynamic
    ng = max(64, min(512, (1 << 18) // (M * G)))
    x = gen(4242 + M + 7 * G + (1 if kind == "dynamic" else 0), ng * G, M, np.complex64)
    y = fft32(x).astype(np.complex128)
    xd = x.astype(np.complex128)
    e = oracle.encoding_vector(M)
    c = oracle.checksum_vector(M)
    d1 = (y @ e - xd @ c).reshape(ng, G).sum(axis=1)
    S = (np.abs(xd) ** 2).sum(axis=1).reshape(ng, G).sum(axis=1)
    return d1, S


def noise_ratios(M, G, kind, fft32, form="tau"):
    """|d1| / (tau / kappa) of fault-free groups."""
    d1, S = residuals(M, G, kind, fft32)
    if form == "tau":
        den = np.array([oracle.threshold(M, s, 1.0, U32) for s in S])
    elif form == "linear_in_M":      # sqrt(M S) replaced by M sqrt(S)
        den = U32 * math.sqrt(math.log2(M)) * M * np.sqrt(S)
    elif form == "per_signal_energy":  # the group's energy replaced by one signal's
        den = U32 * math.sqrt(math.log2(M)) * np.sqrt(M * S / G)
    else:
        raise ValueError(form)
    return np.abs(d1) / den


CASES = [(1 << lm, G, kind) for kind in ("uniform", "dynamic") for G in (1, 4, 16, 64) for lm in range(4, 13)]


def band(fft32, form="tau"):
    rms, mx = [], []
    for M, G, kind in CASES:
        r = noise_ratios(M, G, kind, fft32, form)
        rms.append(float(np.sqrt(np.mean(r ** 2))))
        mx.append(float(r.max()))
    return np.array(rms), np.array(mx)


@pytest.mark.parametrize("fft32", [numpy_binary32, radix2_binary32], ids=["pocketfft32", "radix2_32"])
def test_noise_scaled_residual_stays_in_one_band(fft32):
    rms, mx = band(fft32)
    # one band over M = 2^4..2^12, G = 1..64, both input distributions
    assert rms.min() >= 0.05 and rms.max() <= 1.5, (rms.min(), rms.max())
    assert rms.max() / rms.min() <= 3.0, rms.max() / rms.min()
    # and no fault-free group anywhere near the default threshold
    assert mx.max() <= KAPPA32 / 2, mx.max()


def test_radix2_binary32_is_a_binary32_fft():
    x = inputs.uniform(3, 4, 256, np.complex64)
    err = oracle.rel_l2(radix2_binary32(x), oracle.fft(x.astype(np.complex128)))
    assert 1e-8 < err < 1e-6


@pytest.mark.parametrize("form", ["linear_in_M", "per_signal_energy"])
def test_wrong_forms_leave_the_band(form):
    """The band test discriminates: a threshold growing linearly in M, or one
    that ignores how many signals the group sums, spreads by far more than
    the factor 3 allowed above."""
    rms, _ = band(radix2_binary32, form)
    assert rms.max() / rms.min() > 8.0
