"""Precision study on the GPU: complex64 butterflies with twiddles generated
in binary64 and rounded once, against binary64 end to end; N in {2^10,
2^14, 2^18} with batch 4096 / 256 / 16, inputs N(0, 1) and a six-decade
lognormal-magnitude variant.  For each result: the relative L2 error of the
whole batch and the worst signal against the FP64 oracle, and the checksum's
false-alarm count with fault tolerance CORRECT (none expected at the default
kappa),
with the largest noise-scaled residual |d1| / (tau / kappa) of any group as
the margin.  The table is printed (pytest -s)."""
import numpy as np
import pytest

import oracle
import tfft_inputs as inputs

pytestmark = pytest.mark.gpu

TOL = {"c64": 1e-5, "c128": 1e-12}
NPDT = {"c64": np.complex64, "c128": np.complex128}
CASES = [(10, 4096), (14, 256), (18, 16)]
ROWS = []


@pytest.fixture(scope="module")
def tf():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_02520_amd

    return paper_2405_02520_amd


@pytest.mark.parametrize("kind", ["gaussian", "dynamic"])
@pytest.mark.parametrize("dt", ["c64", "c128"])
@pytest.mark.parametrize("log2n,batch", CASES)
def test_precision(tf, log2n, batch, dt, kind):
    import torch

    n = 1 << log2n
    gen = inputs.gaussian if kind == "gaussian" else inputs.dynamic
    x = gen(inputs.precision_seed(log2n, kind == "dynamic"), batch, n, NPDT[dt])
    xd = torch.from_numpy(x).cuda()
    plan = tf.Plan(n, batch, dt)
    y = plan.forward(xd, ft_mode="correct").cpu().numpy()
    counts, _ = plan.report()
    ref = oracle.fft(x.astype(np.complex128))
    err = oracle.rel_l2(y, ref)
    worst = max(oracle.rel_l2(y[i], ref[i]) for i in range(batch))
    # residuals of every group: a plan with a vanishing threshold flags them all
    probe = tf.Plan(n, batch, dt, kappa=1e-12)
    probe.forward(xd, ft_mode="detect")
    pc, recs = probe.report()
    margin = max((r.residual / r.threshold * 1e-12 for r in recs if r.threshold > 0), default=0.0)
    ROWS.append((dt, kind, n, batch, err, worst, counts["groups_checked"], counts["detected"], margin))
    print(f"\n{dt} {kind:8s} N=2^{log2n} batch={batch}: rel L2 {err:.3e} (worst signal {worst:.3e}), "
          f"groups {counts['groups_checked']}, false alarms {counts['detected']}, max |d1|/(tau/kappa) {margin:.3f}")
    assert err <= TOL[dt] and worst <= TOL[dt]
    assert counts["detected"] == 0
    # (the margin covers every group: one the probe did not flag has |d1|
    # below 1e-12 of its threshold, e.g. an exactly cancelling residual)
    assert pc["n_records"] > 0
    assert margin < plan.info()["kappa"] / 1.5  # the default threshold keeps a margin
    plan.close()
    probe.close()
