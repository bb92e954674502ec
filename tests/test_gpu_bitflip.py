"""Bit-flip campaign (the paper's fault-coverage protocol): half of the
checksum groups get one flipped bit in one register (any butterfly stage or
final value, real or imaginary part, any bit).  Checked: no false alarm at the
default threshold; every flagged group is located and corrected; every signal
ends within tolerance of the FP64 oracle, or, for a flip the checksum cannot
see, within the error such a flip can leave (|eps| <= tau / (sqrt(3)/2),
spread over at most M/8 outputs)."""
import math

import numpy as np
import pytest

import oracle
import tfft_inputs as inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype,tol", [("c64", 1e-5), ("c128", 1e-12)])
def test_bitflip_campaign(dtype, tol):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_02520_amd import campaign

    n, G, groups = 1024, 16, 400
    x = inputs.gaussian(inputs.SEED_PRECISION, groups * G, n, np.complex64 if dtype == "c64" else np.complex128)
    res = campaign.run(torch.from_numpy(x).cuda(), G, seed=inputs.SEED_PRECISION ^ 0xFA17)
    c = res["counts"]
    assert res["false_alarms"] == 0
    assert c["uncorrectable"] == 0 and c["corrected"] == c["detected"] == res["detected_faulty"]
    # the ROC from the probe run: detection never decreases as kappa falls
    det = [d for _, d, _ in res["roc"]]
    assert all(a >= b for a, b in zip(det, det[1:]))
    ref = oracle.fft(x.astype(np.complex128))
    y = res["y"].cpu().numpy()
    err = np.linalg.norm(y - ref, axis=1)
    nrm = np.linalg.norm(ref, axis=1)
    flagged = {r.group for r in res["records"]}
    u = 2.0 ** -24 if dtype == "c64" else 2.0 ** -53
    from paper_2405_02520_amd import Plan

    with Plan(n, G, dtype) as p:
        kappa = p.info()["kappa"]  # the CORRECT run's (default) threshold factor
    for f in res["specs"]:
        b = f["signal"]
        g = b // G
        if g in flagged:
            continue
        S = float(np.sum(np.abs(x[g * G:(g + 1) * G].astype(np.complex128)) ** 2))
        tau = oracle.threshold(n, S, kappa, u)
        assert err[b] <= tau / (math.sqrt(3) / 2) * math.sqrt(n / 8) + tol * nrm[b]
    faulty_signals = {f["signal"] for f in res["specs"] if f["signal"] // G not in flagged}
    clean = np.array([b for b in range(groups * G) if b not in faulty_signals])
    assert np.max(err[clean] / nrm[clean]) <= 10 * tol
    assert oracle.rel_l2(y[clean], ref[clean]) <= tol
