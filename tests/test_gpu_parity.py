"""GPU parity: the HIP path against the FP64 oracle, through the C ABI.

Tolerances (relative L2 over the whole batch): 1e-5 for complex64, 1e-12 for
complex128.  Every injected single fault must be detected and corrected to the
same tolerance.
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


def run(tf, x, dtype, *, inverse=False, mode="correct", group=0, faults=None, plan=None):
    B, n = x.shape
    plan = plan or tf.Plan(n, B, dtype, group=group)
    if faults is not None:
        plan.set_faults(faults)
    xd = to_dev(x)
    y = plan.inverse(xd, ft_mode=mode) if inverse else plan.forward(xd, ft_mode=mode)
    counts, recs = plan.report()
    return y.cpu().numpy(), counts, recs, plan


def reference(x, inverse=False):
    return oracle.fft(x.astype(np.complex128), inverse=inverse)


# ------------------------------------------------------------ plain parity

@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("log2n", list(range(1, 13)))
@pytest.mark.parametrize("mode", ["off", "correct"])
def test_single_pass_forward(tf, dtype, log2n, mode):
    n = 1 << log2n
    B = 37 if n <= 1024 else 19  # not a multiple of the group size: ragged last group
    x = inputs.uniform(1000 + log2n, B, n, NPDT[dtype])
    y, counts, recs, _ = run(tf, x, dtype, mode=mode)
    assert oracle.rel_l2(y, reference(x)) <= TOL[dtype]
    assert counts["detected"] == 0, recs


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("log2n", [1, 3, 8, 10, 12])
def test_single_pass_inverse(tf, dtype, log2n):
    n = 1 << log2n
    x = inputs.uniform(2000 + log2n, 21, n, NPDT[dtype])
    y, counts, recs, _ = run(tf, x, dtype, inverse=True)
    assert oracle.rel_l2(y, reference(x, inverse=True)) <= TOL[dtype]
    assert counts["detected"] == 0


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("log2n,B", [(13, 5), (14, 3), (16, 3), (17, 3), (18, 2), (19, 2), (20, 2), (21, 1), (24, 1)])
@pytest.mark.parametrize("inverse", [False, True])
def test_multi_pass(tf, dtype, log2n, B, inverse):
    n = 1 << log2n
    x = inputs.uniform(3000 + log2n, B, n, NPDT[dtype])
    y, counts, recs, plan = run(tf, x, dtype, inverse=inverse)
    assert plan.info()["passes"] == (2 if log2n <= (19 if dtype == "c64" else 20) else 3)
    assert oracle.rel_l2(y, reference(x, inverse)) <= TOL[dtype]
    assert counts["detected"] == 0, recs


def test_inverse_unscaled_and_round_trip(tf):
    import torch

    n, B = 1024, 8
    x = inputs.uniform(77, B, n, np.complex64)
    p = tf.Plan(n, B, "c64", inverse_unscaled=True)
    y = p.inverse(to_dev(x)).cpu().numpy()
    assert oracle.rel_l2(y, reference(x, True) * n) <= 1e-5
    q = tf.Plan(n, B, "c64")
    back = q.inverse(q.forward(to_dev(x))).cpu().numpy()
    assert oracle.rel_l2(back, x) <= 1e-6


def test_deterministic(tf):
    x = inputs.uniform(5, 64, 4096, np.complex64)
    p = tf.Plan(4096, 64, "c64")
    xd = to_dev(x)
    a = p.forward(xd).cpu().numpy()
    b = p.forward(xd).cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


# --------------------------------------------- correctness config (N=256)

def config1_fault():
    rng = inputs.fault_rng(inputs.SEED_CORRECTNESS)
    return int(rng.integers(64)), int(rng.integers(256))


@pytest.mark.parametrize("group", [64, 16])
def test_config1_output_fault(tf, group):
    """complex64, N=256, batch 64, +1.0 on one output element of one signal."""
    x = inputs.uniform(inputs.SEED_CORRECTNESS, 64, 256, np.complex64)
    js, ks = config1_fault()
    fault = [dict(signal=js, pass_=0, stage=-1, index=ks, value=1.0)]
    y, counts, recs, plan = run(tf, x, "c64", group=group, faults=fault)
    ref = reference(x)
    assert counts["detected"] == 1 and counts["corrected"] == 1, (counts, recs)
    assert [r.signal for r in recs] == [js] and recs[0].action == "corrected"
    assert oracle.rel_l2(y, ref) <= 1e-5
    assert oracle.rel_l2(y[js], ref[js]) <= 1e-5
    # the same fault with fault tolerance off corrupts exactly that element
    yoff, c_off, _, _ = run(tf, x, "c64", group=group, faults=fault, mode="off", plan=plan)
    bad = np.argwhere(np.abs(yoff - ref) > 0.5)
    assert bad.tolist() == [[js, ks]] and c_off["detected"] == 0


@pytest.mark.parametrize("group", [64, 16])
def test_config1_stage_faults(tf, group):
    x = inputs.uniform(inputs.SEED_CORRECTNESS, 64, 256, np.complex64)
    js, ks = config1_fault()
    plan = tf.Plan(256, 64, "c64", group=group)
    ref = reference(x)
    for stage in range(plan.info()["stages"][0]):
        fault = [dict(signal=js, pass_=0, stage=stage, index=ks, value=1.0)]
        y, counts, recs, _ = run(tf, x, "c64", faults=fault, plan=plan)
        assert counts["detected"] == 1 and counts["corrected"] == 1, (stage, counts, recs)
        assert recs[0].signal == js
        assert oracle.rel_l2(y, ref) <= 1e-5
        assert oracle.rel_l2(y[js], ref[js]) <= 1e-5


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("log2n", [10, 12])
def test_every_stage_every_member(tf, dtype, log2n):
    """One fault per group, spread over stages, members and elements."""
    n, G = 1 << log2n, 16
    B = 8 * G
    x = inputs.uniform(400 + log2n, B, n, NPDT[dtype])
    plan = tf.Plan(n, B, dtype, group=G)
    nst = plan.info()["stages"][0]
    rng = inputs.fault_rng(400 + log2n)
    faults = []
    scale = math.sqrt(2 * n / 3)
    for g in range(B // G):
        stage = g % (nst + 1) - 1
        faults.append(dict(signal=g * G + int(rng.integers(G)), pass_=0, stage=stage, index=int(rng.integers(n)),
                           value=complex(rng.standard_normal(), rng.standard_normal()) * scale))
    y, counts, recs, _ = run(tf, x, dtype, faults=faults, plan=plan)
    assert counts["detected"] == len(faults) and counts["corrected"] == len(faults), (counts, recs)
    assert sorted(r.signal for r in recs) == sorted(f["signal"] for f in faults)
    assert oracle.rel_l2(y, reference(x)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("inverse", [False, True])
@pytest.mark.parametrize("log2n,B", [(16, 4), (20, 2)])
def test_multi_pass_faults(tf, dtype, inverse, log2n, B):
    """A fault after every stage of every pass, and on the final values of
    every pass, in a random signal and element: detected in that pass and
    corrected.  Magnitude: the RMS of the values at the end of the pass."""
    n = 1 << log2n
    x = inputs.uniform(500 + log2n, B, n, NPDT[dtype])
    plan = tf.Plan(n, B, dtype)
    info = plan.info()
    ref = reference(x, inverse)
    rng = inputs.fault_rng(500 + log2n)
    for p in range(info["passes"]):
        done = math.prod(info["pass_len"][: p + 1])
        for stage in range(-1, info["stages"][p]):
            sig = int(rng.integers(B))
            idx = int(rng.integers(n))
            mag = math.sqrt(2 * done / 3)
            if inverse and p == info["passes"] - 1 and stage == -1:
                mag /= n  # final values of the inverse carry the 1/N
            fault = [dict(signal=sig, pass_=p, stage=stage, index=idx, value=mag * (0.6 - 0.8j))]
            y, counts, recs, _ = run(tf, x, dtype, inverse=inverse, faults=fault, plan=plan)
            assert counts["detected"] == 1 and counts["corrected"] == 1, (p, stage, counts, recs)
            assert recs[0].signal == sig and recs[0].pass_ == p
            assert recs[0].sub == idx // info["pass_len"][p]
            assert oracle.rel_l2(y, ref) <= TOL[dtype], (p, stage)


@pytest.mark.parametrize("dtype,log2n,B,group", [("c64", 10, 16384, 16), ("c128", 14, 512, 0)])
def test_faults_with_many_groups_per_workgroup(tf, dtype, log2n, B, group):
    """The smallest grid (grid_scale -3) makes every workgroup walk several
    groups, so a group's decision is taken while the workgroup is in its
    next group, and the last group's after the loop.  Faults in every
    group (one pass) or in every eighth signal (two passes, one fault per
    group): each detected, located and corrected; faulty and sampled
    signals match the oracle."""
    n = 1 << log2n
    x = inputs.uniform(700 + log2n, B, n, NPDT[dtype])
    plan = tf.Plan(n, B, dtype, group=group, grid_scale=-3)
    info = plan.info()
    rng = inputs.fault_rng(700 + log2n)
    scale = math.sqrt(2 * n / 3)
    if info["passes"] == 1:
        G = info["group"][0]
        sigs = [g * G + int(rng.integers(G)) for g in range(B // G)]
        faults = [dict(signal=s, pass_=0, stage=-1, index=int(rng.integers(n)),
                       value=complex(rng.standard_normal(), rng.standard_normal()) * scale) for s in sigs]
    else:
        sigs = list(range(0, B, 8))
        m0 = info["pass_len"][0]
        faults = [dict(signal=s, pass_=0, stage=-1, index=int(rng.integers(n)),
                       value=complex(rng.standard_normal(), rng.standard_normal()) * math.sqrt(2 * m0 / 3)) for s in sigs]
    y, counts, recs, _ = run(tf, x, dtype, faults=faults, plan=plan)
    assert counts["detected"] == len(faults) and counts["corrected"] == len(faults), counts
    assert counts["uncorrectable"] == 0
    assert sorted(r.signal for r in recs) == sorted(sigs)
    rows = sorted(set(sigs[::4]) | set(range(1, B, 97)))
    assert oracle.rel_l2(y[rows], reference(x[rows])) <= TOL[dtype]


def test_detect_mode_report_matches_oracle(tf):
    """The GPU's d-statistics equal the oracle's on the same outputs."""
    n, G, B = 1024, 16, 64
    x = inputs.uniform(600, B, n, np.complex64)
    faults = [dict(signal=3, pass_=0, stage=-1, index=100, value=2.0 + 1.0j),
              dict(signal=37, pass_=0, stage=1, index=999, value=-3.0j)]
    y, counts, recs, plan = run(tf, x, "c64", group=G, faults=faults, mode="detect")
    assert counts["detected"] == 2 and counts["corrected"] == 0
    out, orecs = oracle.two_sided_batch(x, y, G, kappa=16.0, u=2.0 ** -24, mode="detect")
    assert [r.group for r in orecs] == [r.group for r in recs] == [0, 2]
    for g, o in zip(recs, orecs):
        assert g.member == o.located
        assert abs(g.residual - abs(o.d1)) <= 1e-6 * abs(o.d1)
        # the energy S that scales tau is summed in binary64 on both sides
        assert abs(g.threshold - o.tau) <= 1e-12 * o.tau
        assert abs(g.ratio - o.rho) <= 1e-6 * abs(o.rho)
    # outputs of DETECT mode are the faulty ones; the oracle corrects them
    fixed, _ = oracle.two_sided_batch(x, y, G, kappa=16.0, u=2.0 ** -24)
    assert oracle.rel_l2(fixed, reference(x)) <= 1e-5


def test_two_faults_in_one_group_uncorrectable(tf):
    n, G, B = 512, 16, 32
    x = inputs.uniform(700, B, n, np.complex64)
    faults = [dict(signal=1, pass_=0, stage=-1, index=5, value=3.0),
              dict(signal=9, pass_=0, stage=-1, index=77, value=-2.0 + 2.0j)]
    with pytest.warns(RuntimeWarning):
        y, counts, recs, plan = run(tf, x, "c64", group=G, faults=faults)
    assert counts["detected"] == 1 and counts["uncorrectable"] == 1
    assert plan.last_status == tf.UNCORRECTABLE


@pytest.mark.parametrize("bad", [float("inf"), float("nan")])
def test_non_finite_fault_corrected(tf, bad):
    n, G, B = 256, 64, 64
    x = inputs.uniform(800, B, n, np.complex64)
    faults = [dict(signal=10, pass_=0, stage=-1, index=3, value=complex(bad, 0.0))]
    y, counts, recs, _ = run(tf, x, "c64", group=G, faults=faults)
    assert counts["corrected"] == 1 and recs[0].signal == 10 and recs[0].method == tf.LOC_PER_SIGNAL
    assert oracle.rel_l2(y, reference(x)) <= 1e-5


def test_set_faults_validation(tf):
    p = tf.Plan(256, 8, "c64")
    bad = [dict(signal=8, index=0), dict(signal=0, index=256), dict(signal=0, index=0, pass_=1),
           dict(signal=0, index=0, stage=5)]
    for f in bad:
        with pytest.raises(tf.TfftError):
            p.set_faults([f])
    p.set_faults([])


def test_exec_validation(tf):
    import torch

    p = tf.Plan(256, 8, "c64")
    x = torch.zeros(8, 256, dtype=torch.complex64, device="cuda")
    y = torch.zeros(8, 256, dtype=torch.complex64, device="cuda")
    with pytest.raises(ValueError):
        p.forward(x.to(torch.complex128))
    with pytest.raises(tf.TfftError):  # in place, one pass, CORRECT: the inputs would be gone
        p.forward(x, out=x)
    # rejected before any launch: misaligned pointer, unknown mode
    assert tf.tfft_exec_forward(p.handle, x.data_ptr() + 8, y.data_ptr(), 0, None) == tf.E_INVALID
    assert tf.tfft_exec_forward(p.handle, x.data_ptr(), y.data_ptr(), 7, None) == tf.E_INVALID
    assert tf.tfft_exec_forward(p.handle, None, y.data_ptr(), 0, None) == tf.E_INVALID
