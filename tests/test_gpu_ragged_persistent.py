"""GPU parity of the persistent ragged path (TFFT_PERSISTENT): every pass of
every length class runs in one kernel launch that drains a queue of work
items (a range of checksum groups of one pass of one class), against the
FP64 oracle, through the C ABI.

Same bars as the uniform batches: relative L2 per signal <= 1e-5 (complex64)
/ 1e-12 (complex128); every injected single fault (any pass, any butterfly
stage or final value, one per checksum group) detected and corrected; the
transform itself bitwise equal to the per-class launches (the persistent
tiles only regroup signals per workgroup).
"""
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


def layout(seed, count, kmin, kmax, gaps):
    lengths = inputs.ragged_lengths(seed, count, kmin, kmax)
    rng = np.random.default_rng(seed + 7)
    order = rng.permutation(count) if gaps else np.arange(count)
    offsets = np.zeros(count, np.int64)
    pos = 0
    for i in order:
        pos += int(rng.integers(0, 5)) * 2 if gaps else 0
        offsets[i] = pos
        pos += int(lengths[i])
    return lengths, offsets, pos


def to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def check_signals(x, y, lengths, offsets, dtype, idx=None, inverse=False):
    idx = range(len(lengths)) if idx is None else idx
    for i in idx:
        n, o = int(lengths[i]), int(offsets[i])
        ref = oracle.fft(x[o:o + n].astype(np.complex128)[None, :], inverse=inverse)[0]
        err = oracle.rel_l2(y[o:o + n], ref)
        assert err <= TOL[dtype], (i, n, err)


def fault_specs(rg, lengths, rng, frac):
    """Faults in round(frac * count) signals, no two in one checksum group:
    each in a random pass, after a random butterfly stage or on a final
    value, at a random element, well above the rounding noise."""
    classes = {n: d for n, _, d in rg.info()}
    sigs = inputs.ragged_fault_signals(rng, lengths, max(1, int(round(frac * len(lengths)))))
    specs = []
    for s in sigs:
        n = int(lengths[s])
        d = classes[n]
        p = int(rng.integers(d["passes"]))
        stage = int(rng.integers(-1, d["stages"][p]))
        # the values grow as sqrt(points transformed so far) from U[-1, 1)
        rms = np.sqrt(2.0 / 3.0 * np.prod(d["pass_len"][: p + 1]))
        specs.append(dict(signal=int(s), pass_=p, stage=stage, index=int(rng.integers(n)),
                          value=rms * complex(rng.uniform(0.5, 4.0), rng.uniform(-4.0, 4.0))))
    return specs, sigs


def test_persistent_rejects_short_lengths(tf):
    with pytest.raises(tf.TfftError):
        tf.Ragged(np.array([32, 256], np.int64), dtype="c64", persistent=True)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("gaps,interleave,one_queue", [(False, False, False), (True, False, False),
                                                       (False, True, False), (True, True, False),
                                                       (True, False, True), (False, True, True)])
def test_persistent_forward_matches_oracle(tf, dtype, gaps, interleave, one_queue):
    lengths, offsets, total = layout(inputs.SEED_RAGGED + 10, 300, 6, 16, gaps)
    x = inputs.uniform_flat(inputs.SEED_RAGGED + 10, total, NPDT[dtype])
    print(f"persistent forward {dtype} gaps={gaps} interleave={interleave} one_queue={one_queue} total={total}",
          flush=True)
    rg = tf.Ragged(lengths, offsets, dtype, persistent=True, interleave=interleave, one_queue=one_queue)
    xd = to_dev(x)
    out = to_dev(np.full(total, 7 + 7j, NPDT[dtype]))
    rg.forward(xd, out)
    counts, recs = rg.report()
    y = out.cpu().numpy()
    check_signals(x, y, lengths, offsets, dtype)
    covered = np.zeros(total, bool)
    for n, o in zip(lengths, offsets):
        covered[o:o + n] = True
    assert np.all(y[~covered] == 7 + 7j), "elements outside every signal must stay untouched"
    assert counts["detected"] == 0 and not recs
    assert counts["groups_checked"] == sum(sum(d["groups"]) for _, _, d in rg.info())


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_persistent_equals_class_launches(tf, dtype):
    """The same transform as the per-class launches (FT off and fault-free
    CORRECT) to a few units of rounding: the butterflies and twiddles are the
    same, only the signals per workgroup differ (and, between two separately
    compiled kernels, the compiler's choice of fused multiply-adds); and the
    inverse against the oracle."""
    lengths, offsets, total = layout(inputs.SEED_RAGGED + 11, 200, 6, 17, True)
    x = inputs.uniform_flat(inputs.SEED_RAGGED + 11, total, NPDT[dtype])
    xd = to_dev(x)
    per = tf.Ragged(lengths, offsets, dtype)
    pst = tf.Ragged(lengths, offsets, dtype, persistent=True)
    agree = {"c64": 1e-6, "c128": 1e-14}[dtype]
    for mode in ("off", "correct"):
        a = per.forward(xd, to_dev(np.zeros(total, NPDT[dtype])), ft_mode=mode).cpu().numpy()
        b = pst.forward(xd, to_dev(np.zeros(total, NPDT[dtype])), ft_mode=mode).cpu().numpy()
        for n, o in zip(lengths, offsets):
            assert oracle.rel_l2(b[o:o + n], a[o:o + n]) <= agree, (mode, n)
        assert np.all(b[a == 0] == 0)
    yi = pst.inverse(xd).cpu().numpy()
    check_signals(x, yi, lengths, offsets, dtype, idx=range(0, 200, 3), inverse=True)


@pytest.mark.parametrize("dtype,interleave,one_queue", [("c64", False, False), ("c128", False, False),
                                                        ("c64", True, False), ("c128", True, False),
                                                        ("c64", False, True), ("c128", True, True)])
def test_persistent_faults_are_corrected(tf, dtype, interleave, one_queue):
    lengths, offsets, total = layout(inputs.SEED_RAGGED + 12, 400, 6, 17, True)
    x = inputs.uniform_flat(inputs.SEED_RAGGED + 12, total, NPDT[dtype])
    rg = tf.Ragged(lengths, offsets, dtype, persistent=True, interleave=interleave, one_queue=one_queue)
    specs, sigs = fault_specs(rg, lengths, inputs.fault_rng(inputs.SEED_RAGGED + 12), 0.03)
    print(f"persistent faults {dtype} interleave={interleave} one_queue={one_queue}: {len(specs)}", flush=True)
    rg.set_faults(specs)
    y = rg.forward(to_dev(x)).cpu().numpy()
    counts, recs = rg.report()
    check_signals(x, y, lengths, offsets, dtype)
    assert counts["uncorrectable"] == 0 and counts["dropped"] == 0
    assert counts["corrected"] == len(sigs)
    assert sorted({r.signal for r in recs if r.action == "corrected"}) == sorted(int(s) for s in sigs)
    by_sig = {int(s["signal"]): s for s in specs}
    for r in recs:
        assert r.pass_ == by_sig[r.signal]["pass_"]


def test_persistent_detect_mode_locates(tf):
    dtype = "c64"
    lengths, offsets, total = layout(inputs.SEED_RAGGED + 13, 256, 6, 16, False)
    x = inputs.uniform_flat(inputs.SEED_RAGGED + 13, total, NPDT[dtype])
    rg = tf.Ragged(lengths, offsets, dtype, persistent=True)
    specs, sigs = fault_specs(rg, lengths, inputs.fault_rng(inputs.SEED_RAGGED + 13), 0.03)
    rg.set_faults(specs)
    y = rg.forward(to_dev(x), ft_mode="detect").cpu().numpy()
    counts, recs = rg.report()
    assert counts["detected"] == len(sigs) and counts["corrected"] == 0
    assert sorted(r.signal for r in recs) == sorted(int(s) for s in sigs)
    for r in recs:
        assert r.action == "detected" and r.member >= 0
        assert abs(r.ratio - (r.member + 1)) <= 0.25
    clean = [i for i in range(len(lengths)) if i not in set(int(s) for s in sigs)]
    check_signals(x, y, lengths, offsets, dtype, idx=clean[::4])


def test_persistent_graph_replays_match_eager(tf):
    import torch

    dtype = "c64"
    lengths, offsets, total = layout(inputs.SEED_RAGGED + 14, 256, 6, 18, False)
    x = inputs.uniform_flat(inputs.SEED_RAGGED + 14, total, NPDT[dtype])
    rg = tf.Ragged(lengths, offsets, dtype, persistent=True)
    specs, sigs = fault_specs(rg, lengths, inputs.fault_rng(inputs.SEED_RAGGED + 14), 0.03)
    rg.set_faults(specs)
    xd = to_dev(x)
    eager = rg.forward(xd).clone()
    c_e, r_e = rg.report()
    assert c_e["corrected"] == len(sigs)
    out = torch.empty_like(xd)
    for rep in range(3):
        out.fill_(0)
        rg.forward(xd, out, use_graph=True)
        c_g, r_g = rg.report()
        assert torch.equal(out, eager), rep
        assert c_g["corrected"] == len(sigs) and c_g["uncorrectable"] == 0
        assert sorted(r.signal for r in r_g) == sorted(r.signal for r in r_e)
        torch.cuda.synchronize()
        _ = (xd * 2).sum().item()  # unrelated eager work between replays
    rg.set_faults([])
    rg.forward(xd, out, use_graph=True)
    c0, r0 = rg.report()
    assert c0["detected"] == 0 and not r0
    check_signals(x, out.cpu().numpy(), lengths, offsets, dtype, idx=range(0, 256, 5))


def test_persistent_tune(tf):
    dtype = "c64"
    lengths, offsets, total = layout(inputs.SEED_RAGGED + 15, 96, 6, 20, False)
    x = inputs.uniform_flat(inputs.SEED_RAGGED + 15, total, NPDT[dtype])
    rg = tf.Ragged(lengths, offsets, dtype, persistent=True)
    specs, sigs = fault_specs(rg, lengths, inputs.fault_rng(inputs.SEED_RAGGED + 15), 0.05)
    rg.set_faults(specs)
    xd = to_dev(x)
    out = rg.forward(xd)
    rg.tune(xd, out, reps=1)
    for n, cnt, d in rg.info():
        assert int(np.prod(d["pass_len"])) == n and d["batch"] == cnt
        if n <= 4096:
            assert d["passes"] == 1, (n, d)  # short classes stay one pass
    y = rg.forward(xd, use_graph=True).cpu().numpy()
    counts, _ = rg.report()  # the faults survive the new plans
    assert counts["corrected"] == len(sigs) and counts["uncorrectable"] == 0
    check_signals(x, y, lengths, offsets, dtype)


def test_persistent_full_size_sampled(tf):
    """4096 complex64 signals, lengths 2^k with k ~ U{6..20}, packed; faults
    in 1% of the signals (any pass, any stage); one persistent graph launch
    after tuning; the oracle checks every faulty signal up to 2^16 points and
    a stride of the rest."""
    import torch

    dtype = "c64"
    lengths = inputs.ragged_lengths(inputs.SEED_RAGGED, 4096, 6, 20)
    offsets = np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.int64)
    total = int(lengths.sum())
    x = inputs.uniform_flat(inputs.SEED_RAGGED, total, NPDT[dtype])
    rg = tf.Ragged(lengths, offsets, dtype, persistent=True)
    xd = to_dev(x)
    out = torch.empty_like(xd)
    print("persistent full size: tune", flush=True)
    rg.tune(xd, out, reps=1)
    specs, sigs = fault_specs(rg, lengths, inputs.fault_rng(inputs.SEED_RAGGED), 0.01)
    rg.set_faults(specs)
    rg.forward(xd, out, use_graph=True)
    counts, recs = rg.report()
    assert counts["uncorrectable"] == 0 and counts["corrected"] == len(sigs)
    assert sorted({r.signal for r in recs}) == sorted(int(s) for s in sigs)
    y = out.cpu().numpy()
    sample = sorted(set([int(s) for s in sigs if lengths[s] <= 1 << 16]) | set(range(0, 4096, 97)))
    check_signals(x, y, lengths, offsets, dtype, idx=sample)
