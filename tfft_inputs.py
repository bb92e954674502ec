"""Seeded synthetic signal generators shared by the tests, the smoke check and
the benchmark.

This module holds no transform or checksum arithmetic: it only draws numbers.
Both the oracle side and the HIP side receive their inputs from here, so that
they see bit-identical data.

Recipe (the paper measures on random signals, "generated with normal
distribution" in its fault-coverage study, and batched sizes with N*batch held
at 2^28 elements in its throughput study):

* ``uniform``: re and im i.i.d. U[-1, 1), drawn as two separate arrays, real
  part first, from ``numpy.random.default_rng(seed)`` (PCG64).
* ``gaussian``: re and im i.i.d. N(0, 1), same order.
* ``dynamic``: |x| = exp(sigma * Z), Z ~ N(0, 1), sigma = ln(1e6) / 6 (so that
  +-3 sigma spans six decades), phase ~ U[0, 2 pi); magnitudes first.

Fault positions come from a separate stream, ``default_rng(seed ^ 0xFA17)``.
"""
from __future__ import annotations

import math

import numpy as np

SEED_CORRECTNESS = 20240501
SEED_SWEEP = 20240502
SEED_PRECISION = 20240503
SEED_RAGGED = 20240504
SEED_GRAD = 20240505
FAULT_SEED_XOR = 0xFA17


def sweep_seed(log2n: int, fp64: bool) -> int:
    return SEED_SWEEP + log2n + (100 if fp64 else 0)


def precision_seed(log2n: int, dynamic: bool) -> int:
    return SEED_PRECISION + log2n + (1000 if dynamic else 0)


def fault_rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed ^ FAULT_SEED_XOR)


def _as_complex(re: np.ndarray, im: np.ndarray, dtype) -> np.ndarray:
    dtype = np.dtype(dtype)
    real = np.float32 if dtype == np.complex64 else np.float64
    out = np.empty(re.shape, dtype=dtype)
    out.real = re.astype(real)
    out.imag = im.astype(real)
    return out


def uniform(seed: int, batch: int, n: int, dtype=np.complex64) -> np.ndarray:
    rng = np.random.default_rng(seed)
    re = rng.uniform(-1.0, 1.0, size=(batch, n))
    im = rng.uniform(-1.0, 1.0, size=(batch, n))
    return _as_complex(re, im, dtype)


def gaussian(seed: int, batch: int, n: int, dtype=np.complex64) -> np.ndarray:
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(size=(batch, n))
    im = rng.standard_normal(size=(batch, n))
    return _as_complex(re, im, dtype)


def dynamic(seed: int, batch: int, n: int, dtype=np.complex64) -> np.ndarray:
    rng = np.random.default_rng(seed)
    sigma = math.log(1e6) / 6.0
    mag = np.exp(sigma * rng.standard_normal(size=(batch, n)))
    phase = rng.uniform(0.0, 2.0 * math.pi, size=(batch, n))
    return _as_complex(mag * np.cos(phase), mag * np.sin(phase), dtype)


def real_gaussian(seed: int, shape) -> np.ndarray:
    """Real N(0, 1) weights (float64), e.g. the fixed weights of the
    differentiable-layer loss sum |W * FFT(x)|^2."""
    return np.random.default_rng(seed).standard_normal(size=shape)


def ragged_lengths(seed: int, count: int, kmin: int = 6, kmax: int = 20) -> np.ndarray:
    """Signal lengths 2^k with k i.i.d. uniform on {kmin..kmax} (int64),
    from ``default_rng(seed)``."""
    k = np.random.default_rng(seed).integers(kmin, kmax + 1, size=count)
    return (np.int64(1) << k.astype(np.int64)).astype(np.int64)


def uniform_flat(seed: int, total: int, dtype=np.complex64) -> np.ndarray:
    """A flat buffer of ``total`` values, re and im i.i.d. U[-1, 1) as in
    ``uniform``, from ``default_rng(seed + 1)`` (so that one seed gives both
    the lengths and the data)."""
    rng = np.random.default_rng(seed + 1)
    re = rng.uniform(-1.0, 1.0, size=total)
    im = rng.uniform(-1.0, 1.0, size=total)
    return _as_complex(re, im, dtype)


def ragged_fault_signals(rng: np.random.Generator, lengths, nfaults: int, block: int = 64) -> np.ndarray:
    """``nfaults`` distinct signal indices of a ragged batch, at most one in
    each aligned block of ``block`` consecutive signals of one length
    (counted in index order), so that no two land in one checksum group of
    at most ``block`` signals: the one-fault-per-group model."""
    lengths = np.asarray(lengths)
    blocks: dict = {}
    rank: dict = {}
    for i, n in enumerate(lengths.tolist()):
        r = rank.get(n, 0)
        rank[n] = r + 1
        blocks.setdefault((n, r // block), []).append(i)
    keys = sorted(blocks)
    if nfaults > len(keys):
        raise ValueError(f"{nfaults} faults do not fit in {len(keys)} blocks")
    pick = rng.choice(len(keys), size=nfaults, replace=False)
    return np.sort(np.array([blocks[keys[k]][int(rng.integers(len(blocks[keys[k]])))] for k in pick], np.int64))


def device_gaussian(seed: int, batch: int, n: int, dtype, device="cuda"):
    """Like ``gaussian`` but drawn on the device with torch's generator seeded
    by ``seed`` (for large fault-free calibration runs that no oracle checks):
    re and im i.i.d. N(0, 1)."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    real = torch.float32 if dtype in (np.complex64, "c64") else torch.float64
    re = torch.randn((batch, n), generator=g, device=device, dtype=real)
    im = torch.randn((batch, n), generator=g, device=device, dtype=real)
    return torch.complex(re, im)


def device_dynamic(seed: int, batch: int, n: int, dtype, device="cuda"):
    """Like ``dynamic`` (six-decade lognormal magnitudes, uniform phases), drawn
    on the device with torch's generator seeded by ``seed``."""
    import torch

    g = torch.Generator(device=device)
    g.manual_seed(seed)
    real = torch.float64
    sigma = math.log(1e6) / 6.0
    mag = torch.exp(sigma * torch.randn((batch, n), generator=g, device=device, dtype=real))
    phase = 2.0 * math.pi * torch.rand((batch, n), generator=g, device=device, dtype=real)
    z = torch.polar(mag, phase)
    return z.to(torch.complex64 if dtype in (np.complex64, "c64") else torch.complex128)
