"""GPU parity of the one-sided (per-signal) and thread-level (per-butterfly)
checksum schemes against the FP64 oracle, through the C ABI.

Same bars as the default scheme: relative L2 <= 1e-5 (complex64) / 1e-12
(complex128) with FT on and no faults (and no false alarm), every injected
single fault detected and corrected.  The one-sided scheme also corrects
faults in several signals of one tile; the thread-level scheme reports the
butterfly (stage, and the wrong output through d2/d1 = k + 1).
"""
import math

import numpy as np
import pytest

import oracle
import tfft_inputs as inputs

pytestmark = pytest.mark.gpu

TOL = {"c64": 1e-5, "c128": 1e-12}
NPDT = {"c64": np.complex64, "c128": np.complex128}


@pytest.fixture(scope="module")
def tf():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2405_02520_amd

    return paper_2405_02520_amd


def to_dev(x):
    import torch

    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def run(plan, x, inverse=False, mode="correct"):
    xd = to_dev(x)
    y = plan.inverse(xd, ft_mode=mode) if inverse else plan.forward(xd, ft_mode=mode)
    counts, recs = plan.report()
    return y.cpu().numpy(), counts, recs


@pytest.mark.parametrize("scheme", ["signal", "thread"])
@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("log2n", [1, 3, 5, 6, 8, 10, 11, 12])
@pytest.mark.parametrize("inverse", [False, True])
def test_scheme_parity_no_false_alarm(tf, scheme, dtype, log2n, inverse):
    n = 1 << log2n
    B = 45 if n <= 1024 else 21
    x = inputs.uniform(700 + log2n, B, n, NPDT[dtype])
    plan = tf.Plan(n, B, dtype, scheme=scheme)
    y, counts, recs = run(plan, x, inverse)
    assert oracle.rel_l2(y, oracle.fft(x.astype(np.complex128), inverse=inverse)) <= TOL[dtype]
    assert counts["detected"] == 0 and not recs, recs[:3]


@pytest.mark.parametrize("scheme", ["signal", "thread"])
def test_scheme_dynamic_range_no_false_alarm(tf, scheme):
    n, B = 1024, 512
    x = inputs.dynamic(inputs.precision_seed(10, True), B, n, np.complex64)
    plan = tf.Plan(n, B, "c64", scheme=scheme)
    y, counts, _ = run(plan, x)
    assert counts["detected"] == 0
    assert oracle.rel_l2(y, oracle.fft(x.astype(np.complex128))) <= TOL["c64"]


def butterfly_output(info, stage, pos):
    """Output index q of the butterfly that writes position pos at this stage
    (stage -1: the final values, written by the last stage)."""
    rad = info["radices"][0]
    s = len(rad) - 1 if stage < 0 else stage
    ns = math.prod(rad[:s])
    return s, (pos // ns) % rad[s]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("log2n", [3, 8, 11, 12])
@pytest.mark.parametrize("inverse", [False, True])
def test_thread_scheme_corrects_every_stage(tf, dtype, log2n, inverse):
    n = 1 << log2n
    B = 24
    x = inputs.uniform(720 + log2n, B, n, NPDT[dtype])
    ref = oracle.fft(x.astype(np.complex128), inverse=inverse)
    plan = tf.Plan(n, B, dtype, scheme="thread")
    info = plan.info()
    rng = inputs.fault_rng(720 + log2n)
    for stage in range(-1, info["stages"][0]):
        sig, pos = int(rng.integers(B)), int(rng.integers(n))
        plan.set_faults([dict(signal=sig, stage=stage, index=pos, value=0.75 - 1.25j)])
        y, counts, recs = run(plan, x, inverse)
        assert counts["detected"] == 1 and counts["corrected"] == 1, (stage, counts)
        r = recs[0]
        s, q = butterfly_output(info, stage, pos)
        assert r.signal == sig and r.method == tf.LOC_THREAD and r.sub == s and r.action == "corrected"
        assert abs(r.ratio - (q + 1)) < 1e-3, (stage, r.ratio, q)
        assert oracle.rel_l2(y, ref) <= TOL[dtype], stage
    # detect mode reports the same event and leaves the output as it is
    plan.set_faults([dict(signal=1, stage=0, index=3, value=2.0)])
    y, counts, recs = run(plan, x, inverse, mode="detect")
    assert counts["detected"] == 1 and counts["corrected"] == 0 and recs[0].action == "detected"
    assert oracle.rel_l2(y, ref) > TOL[dtype]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("log2n", [3, 8, 11, 12])
@pytest.mark.parametrize("inverse", [False, True])
def test_signal_scheme_corrects_every_stage(tf, dtype, log2n, inverse):
    n = 1 << log2n
    B = 24
    x = inputs.uniform(740 + log2n, B, n, NPDT[dtype])
    ref = oracle.fft(x.astype(np.complex128), inverse=inverse)
    plan = tf.Plan(n, B, dtype, scheme="signal")
    info = plan.info()
    assert info["group"] == [1]
    rng = inputs.fault_rng(740 + log2n)
    for stage in range(-1, info["stages"][0]):
        sig, pos = int(rng.integers(B)), int(rng.integers(n))
        mag = math.sqrt(2 * n / 3) / (n if inverse and stage == -1 else 1)
        plan.set_faults([dict(signal=sig, stage=stage, index=pos, value=mag * (0.6 + 0.8j))])
        y, counts, recs = run(plan, x, inverse)
        assert counts["detected"] == 1 and counts["corrected"] == 1, (stage, counts)
        assert recs[0].signal == sig and abs(recs[0].ratio - 1) < 1e-9
        assert oracle.rel_l2(y, ref) <= TOL[dtype], stage


def test_signal_scheme_corrects_several_signals_of_one_tile(tf):
    n, B = 256, 64
    x = inputs.uniform(760, B, n, np.complex64)
    plan = tf.Plan(n, B, "c64", scheme="signal")
    faults = [dict(signal=s, stage=-1, index=(37 * s) % n, value=3.0 + 1.0j) for s in (0, 1, 2, 9, 10, 63)]
    plan.set_faults(faults)
    y, counts, recs = run(plan, x)
    assert counts["corrected"] == len(faults) and counts["uncorrectable"] == 0
    assert sorted(r.signal for r in recs) == [0, 1, 2, 9, 10, 63]
    assert oracle.rel_l2(y, oracle.fft(x.astype(np.complex128))) <= TOL["c64"]


def test_signal_scheme_residual_matches_oracle(tf):
    """Detect mode: the GPU's per-signal residual equals the oracle's d1 on
    the same outputs."""
    n, B = 1024, 32
    x = inputs.uniform(770, B, n, np.complex64)
    plan = tf.Plan(n, B, "c64", scheme="signal")
    plan.set_faults([dict(signal=5, stage=-1, index=100, value=2.0 + 1.0j),
                     dict(signal=17, stage=1, index=900, value=-1.5)])
    y, counts, recs = run(plan, x, mode="detect")
    assert counts["detected"] == 2
    for r in recs:
        _, orec = oracle.one_sided_signal(x[r.signal], y[r.signal], mode="detect", u=2.0 ** -24)
        assert orec.flagged
        assert abs(r.residual - abs(orec.d1)) <= 1e-6 * abs(orec.d1)
        assert abs(r.threshold - orec.tau) <= 1e-6 * orec.tau


def test_thread_scheme_bit_flips(tf):
    """Exponent bit flips (huge or non-finite outputs) inside a butterfly are
    recomputed from the butterfly's inputs."""
    n, B = 1024, 16
    x = inputs.uniform(780, B, n, np.complex64)
    plan = tf.Plan(n, B, "c64", scheme="thread")
    for k, bit in enumerate((30, 29, 28, 27)):
        plan.set_faults([dict(signal=k, stage=k % 3, index=11 * k + 5, flip="re", bit=bit)])
        y, counts, recs = run(plan, x)
        assert counts["corrected"] == 1, (bit, counts)
        assert oracle.rel_l2(y, oracle.fft(x.astype(np.complex128))) <= TOL["c64"]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("log2n,B", [(13, 6), (16, 3), (20, 2)])
@pytest.mark.parametrize("inverse", [False, True])
def test_thread_scheme_multi_pass(tf, dtype, log2n, B, inverse):
    """Thread-level checks in every pass of a multi-pass plan: parity, no
    false alarm, and a fault after every stage of every pass corrected in
    the butterfly that produced it."""
    n = 1 << log2n
    x = inputs.uniform(790 + log2n, B, n, NPDT[dtype])
    ref = oracle.fft(x.astype(np.complex128), inverse=inverse)
    plan = tf.Plan(n, B, dtype, scheme="thread")
    info = plan.info()
    assert info["passes"] >= 2
    y, counts, recs = run(plan, x, inverse)
    assert oracle.rel_l2(y, ref) <= TOL[dtype] and counts["detected"] == 0
    rng = inputs.fault_rng(790 + log2n)
    for p in range(info["passes"]):
        M = info["pass_len"][p]
        rad = info["radices"][p]
        for stage in range(info["stages"][p]):
            sig, idx = int(rng.integers(B)), int(rng.integers(n))
            plan.set_faults([dict(signal=sig, pass_=p, stage=stage, index=idx, value=0.9 + 0.4j)])
            y, counts, recs = run(plan, x, inverse)
            assert counts["detected"] == 1 and counts["corrected"] == 1, (p, stage, counts)
            r = recs[0]
            q = ((idx % M) // math.prod(rad[:stage])) % rad[stage]
            assert r.signal == sig and r.pass_ == p and r.method == tf.LOC_THREAD
            assert abs(r.ratio - (q + 1)) < 1e-3, (p, stage, r.ratio, q)
            assert oracle.rel_l2(y, ref) <= TOL[dtype], (p, stage)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("log2n,B", [(13, 6), (16, 3), (20, 2)])
@pytest.mark.parametrize("inverse", [False, True])
def test_signal_scheme_multi_pass(tf, dtype, log2n, B, inverse):
    """One-sided checks of every sub-signal in every pass: parity, no false
    alarm, a fault after every stage of every pass (and on the final values)
    recomputed, and faults in several sub-signals of one tile all corrected."""
    n = 1 << log2n
    x = inputs.uniform(810 + log2n, B, n, NPDT[dtype])
    ref = oracle.fft(x.astype(np.complex128), inverse=inverse)
    plan = tf.Plan(n, B, dtype, scheme="signal")
    info = plan.info()
    assert info["passes"] >= 2
    y, counts, recs = run(plan, x, inverse)
    assert oracle.rel_l2(y, ref) <= TOL[dtype] and counts["detected"] == 0
    rng = inputs.fault_rng(810 + log2n)
    for p in range(info["passes"]):
        M = info["pass_len"][p]
        done = math.prod(info["pass_len"][: p + 1])
        for stage in range(-1, info["stages"][p]):
            sig, idx = int(rng.integers(B)), int(rng.integers(n))
            mag = math.sqrt(2 * done / 3) / (n if inverse and p == info["passes"] - 1 and stage == -1 else 1)
            plan.set_faults([dict(signal=sig, pass_=p, stage=stage, index=idx, value=mag * (0.6 - 0.8j))])
            y, counts, recs = run(plan, x, inverse)
            assert counts["detected"] == 1 and counts["corrected"] == 1, (p, stage, counts)
            r = recs[0]
            assert r.signal == sig and r.pass_ == p and r.method == tf.LOC_SUBSIGNAL
            assert r.sub == idx // M
            assert oracle.rel_l2(y, ref) <= TOL[dtype], (p, stage)
    # adjacent sub-signals of one tile (one group of the block scheme)
    M0 = info["pass_len"][0]
    faults = [dict(signal=0, pass_=0, stage=-1, index=i * M0 + 3, value=2.0 - 1.0j) for i in (0, 1, 2)]
    plan.set_faults(faults)
    y, counts, recs = run(plan, x, inverse)
    assert counts["corrected"] == 3 and counts["uncorrectable"] == 0
    assert oracle.rel_l2(y, ref) <= TOL[dtype]
