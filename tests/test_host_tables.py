"""Host tier (CPU, no device): the product's own table generators and pass
decomposition, through the C ABI, against the oracle.

* tfft_host_root (the twiddles every plan uploads) against the oracle's
  exactly reduced w_n^t, at angles spread over all octants and at n up to
  2^26;
* tfft_host_checksum_vector (the precomputed checksum vector c = (e^T W)^T of
  Section II-C) against the oracle's closed form and, for small m, against
  the direct sum of its definition;
* tfft_plan_describe (the tiled decomposition of Section IV-A.1): the pass
  lengths multiply to N, every pass's stage radices multiply to its length,
  and the oracle's P-pass tiled FFT with those lengths equals the DFT.
"""
import math

import numpy as np
import pytest

import oracle
import tfft_inputs as inputs


@pytest.fixture(scope="module")
def tf():
    import os
    import runpy

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if not os.path.exists(os.path.join(root, "paper_2405_02520_amd", "libtfft.so")):
        runpy.run_path(os.path.join(root, "paper_2405_02520_amd", "build.py"), run_name="__main__")
    import paper_2405_02520_amd

    return paper_2405_02520_amd


@pytest.mark.parametrize("n", [1, 2, 3, 8, 12, 256, 4096, 3 * 4096, 1 << 20, 1 << 24, 1 << 26])
def test_host_root_matches_oracle(tf, n):
    rng = np.random.default_rng(n)
    ts = np.unique(np.concatenate([np.arange(min(n, 64)), rng.integers(-4 * n, 4 * n, size=256),
                                   [n // 8, n // 4, n // 2, 3 * n // 4, n - 1, -1, n]]))
    ref = oracle.omega(ts, n)
    got = np.array([tf.host_root(int(t), n) for t in ts])
    # both reduce the angle exactly and call libm on [0, pi/4]: within an ulp of 1
    assert np.max(np.abs(got - ref)) <= 2.5e-16
    assert np.all(np.abs(np.abs(got) - 1.0) <= 4.5e-16)


@pytest.mark.parametrize("m", [2, 4, 8, 64, 256, 1024, 4096, 1 << 16])
@pytest.mark.parametrize("inverse", [False, True])
def test_host_checksum_vector_matches_oracle(tf, m, inverse):
    scale = 1.0 / m if inverse else 1.0
    got = tf.host_checksum_vector(m, inverse, scale)
    ref = oracle.checksum_vector(m, inverse, scale)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))
    if m <= 256:
        direct = oracle.checksum_vector_direct(m, inverse, scale)
        assert np.max(np.abs(got - direct)) <= 1e-12 * np.max(np.abs(ref))


def test_host_generators_reject_bad_arguments(tf):
    import ctypes

    out = (ctypes.c_double * 8)()
    assert tf.tfft_host_root(1, 0, out) == tf.E_INVALID
    assert tf.tfft_host_root(1, 4, None) == tf.E_INVALID
    for m in (0, 1, 3, 12, 1 << 25):
        assert tf.tfft_host_checksum_vector(m, 0, 1.0, out) == tf.E_INVALID
    assert tf.tfft_host_checksum_vector(4, 0, float("inf"), out) == tf.E_INVALID


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_describe_decomposition(tf, dtype):
    for k in range(1, 25):
        n = 1 << k
        batch = max(1, (1 << 20) >> k)
        d = tf.describe(n, batch, dtype)
        P = d["passes"]
        assert math.prod(d["pass_len"]) == n
        assert P == 1 or min(d["pass_len"]) >= 2
        for p in range(P):
            assert math.prod(d["radices"][p]) == d["pass_len"][p]
            assert d["stages"][p] == len(d["radices"][p])
            assert d["group"][p] % d["tile_signals"][p] == 0
        assert d["workspace_bytes"] == (0 if P == 1 else n * batch * (8 if dtype == "c64" else 16))
        assert d["kappa"] == (16.0 if dtype == "c64" else 96.0)


@pytest.mark.parametrize("k", [2, 7, 12, 13, 14, 15, 16, 17])
def test_describe_lengths_give_the_dft(tf, k):
    """The oracle's tiled FFT with the product's pass lengths is the DFT (the
    decomposition is a valid tiling of Section IV-A.1), also with forced pass
    counts."""
    n = 1 << k
    x = inputs.uniform(60 + k, 2, n, np.complex128)
    ref = oracle.fft(x)
    for passes in (0, 2, 3):
        try:
            d = tf.describe(n, 2, "c64", passes=passes)
        except tf.TfftError as e:
            assert e.status == tf.E_UNSUPPORTED
            continue
        y = oracle.tiled(x, d["pass_len"])["y"]
        assert oracle.rel_l2(y, ref) <= 1e-14


def test_describe_validates_like_create(tf):
    for n, batch, dtype in [(0, 1, "c64"), (12, 1, "c64"), (1 << 25, 1, "c64"), (64, 0, "c64")]:
        with pytest.raises(tf.TfftError) as e:
            tf.describe(n, batch, dtype)
        assert e.value.status == tf.E_INVALID
    with pytest.raises(tf.TfftError) as e:
        tf.describe(1 << 7, 4, "c64", passes=2)
    assert e.value.status == tf.E_UNSUPPORTED
