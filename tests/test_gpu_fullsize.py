"""GPU parity at the full sweep configuration, in the launch configuration
the benchmark times: N = 2^k, k = 8..24, N * batch = 2^28 (complex64) /
2^27 (complex128), the benchmark's own seeded input viewed as [batch][N],
FT CORRECT.  The oracle checks sampled signals one by one (a bounded number
of elements per size); Parseval, sum |y|^2 = N sum |x|^2 per signal, checks
every signal.  A second run injects one fault per 256 signals (at least one)
on the final values of a random pass and checks that all are corrected and
that the faulty signals match the oracle."""
import math

import numpy as np
import pytest

import oracle
import tfft_inputs as inputs

pytestmark = pytest.mark.gpu

TOL = {"c64": 1e-5, "c128": 1e-12}
NPDT = {"c64": np.complex64, "c128": np.complex128}
LOG2E = {"c64": 28, "c128": 27}
SAMPLE_ELEMS = 1 << 21  # oracle elements per size


@pytest.fixture(scope="module")
def tf():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_02520_amd

    return paper_2405_02520_amd


_DATA = {}


def data(dt):
    """(host array, device tensor) of the benchmark's input for one precision."""
    import torch

    if dt not in _DATA:
        _DATA.clear()
        x = inputs.uniform(inputs.sweep_seed(0, dt == "c128"), 1, 1 << LOG2E[dt], NPDT[dt]).reshape(-1)
        _DATA[dt] = (x, torch.from_numpy(x).cuda())
    return _DATA[dt]


def parseval_worst(xd, yd):
    import torch

    ex = (xd.real.double() ** 2 + xd.imag.double() ** 2).sum(dim=1)
    ey = (yd.real.double() ** 2 + yd.imag.double() ** 2).sum(dim=1)
    n = xd.shape[1]
    return float(torch.max(torch.abs(ey / (n * ex) - 1.0)))


def sample(b, n, rng, extra=()):
    cnt = max(1, min(b, SAMPLE_ELEMS // n))
    idx = {0, b - 1} | set(int(v) for v in rng.integers(b, size=cnt)) | set(extra)
    return sorted(idx)[: max(2, cnt) + len(extra)]


@pytest.mark.parametrize("dt,k", [(d, k) for d in ("c64", "c128") for k in range(8, 25)])
def test_sweep_size_full(tf, dt, k):
    import torch

    x, xdev = data(dt)
    n = 1 << k
    b = (1 << LOG2E[dt]) // n
    xd = xdev.view(b, n)
    plan = tf.Plan(n, b, dt)
    yd = plan.forward(xd, ft_mode="correct")
    counts, _ = plan.report()
    assert counts["detected"] == 0, counts
    assert parseval_worst(xd, yd) < (2e-5 if dt == "c64" else 1e-12)
    rng = np.random.default_rng(1000 + k)
    idx = sample(b, n, rng)
    ys = yd[torch.tensor(idx, device=yd.device)].cpu().numpy()
    ref = oracle.fft(x.reshape(b, n)[idx].astype(np.complex128))
    for r, i in enumerate(idx):
        assert oracle.rel_l2(ys[r], ref[r]) <= TOL[dt], (i, oracle.rel_l2(ys[r], ref[r]))
    plan.close()


@pytest.mark.parametrize("dt,k", [(d, k) for d in ("c64", "c128") for k in (8, 12, 13, 18, 19, 24)])
def test_sweep_size_full_with_faults(tf, dt, k):
    import torch

    x, xdev = data(dt)
    n = 1 << k
    b = (1 << LOG2E[dt]) // n
    xd = xdev.view(b, n)
    plan = tf.Plan(n, b, dt)
    info = plan.info()
    rng = inputs.fault_rng(inputs.sweep_seed(k, dt == "c128"))
    nf = max(1, b // 256)
    faults, sigs = [], []
    for i in range(nf):
        sig = min(b - 1, i * 256 + int(rng.integers(min(256, b))))
        ps = int(rng.integers(info["passes"]))
        plen = info["pass_len"][0] if ps == 0 else n
        faults.append(dict(signal=sig, pass_=ps, stage=-1, index=int(rng.integers(n)),
                           value=math.sqrt(2.0 * plen / 3.0) * complex(0.6, -0.8)))
        sigs.append(sig)
    plan.set_faults(faults)
    yd = plan.forward(xd, ft_mode="correct")
    counts, recs = plan.report()
    assert counts["corrected"] == nf and counts["uncorrectable"] == 0, counts
    assert sorted({r.signal for r in recs}) == sorted(set(sigs))
    assert parseval_worst(xd, yd) < (2e-5 if dt == "c64" else 1e-12)
    pick = sorted(set(sigs))[: max(1, SAMPLE_ELEMS // n)]
    ys = yd[torch.tensor(pick, device=yd.device)].cpu().numpy()
    ref = oracle.fft(x.reshape(b, n)[pick].astype(np.complex128))
    for r, i in enumerate(pick):
        assert oracle.rel_l2(ys[r], ref[r]) <= TOL[dt], (i, oracle.rel_l2(ys[r], ref[r]))
    plan.close()
