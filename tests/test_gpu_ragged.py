"""GPU parity of ragged batches (signals of mixed power-of-two lengths in one
flat buffer, each length class one plan, optionally replayed as one captured
HIP graph) against the FP64 oracle, through the C ABI.

Same bars as the uniform batches: relative L2 per signal <= 1e-5 (complex64)
/ 1e-12 (complex128), every injected single fault detected and corrected.
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
    """Lengths and offsets; with gaps, signals are separated by a few
    unused elements and listed in shuffled order."""
    lengths = inputs.ragged_lengths(seed, count, kmin, kmax)
    rng = np.random.default_rng(seed + 7)
    order = rng.permutation(count) if gaps else np.arange(count)
    offsets = np.zeros(count, np.int64)
    pos = 0
    for i in order:
        pos += int(rng.integers(0, 5)) * 2 if gaps else 0  # keeps 16-byte alignment of the buffer only
        offsets[i] = pos
        pos += int(lengths[i])
    return lengths, offsets, pos


def check_signals(x, y, lengths, offsets, dtype, idx=None, inverse=False):
    idx = range(len(lengths)) if idx is None else idx
    for i in idx:
        n, o = int(lengths[i]), int(offsets[i])
        ref = oracle.fft(x[o:o + n].astype(np.complex128)[None, :], inverse=inverse)[0]
        err = oracle.rel_l2(y[o:o + n], ref)
        assert err <= TOL[dtype], (i, n, err)


def to_dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("gaps", [False, True])
def test_ragged_forward_matches_oracle(tf, dtype, gaps):
    lengths, offsets, total = layout(inputs.SEED_RAGGED, 300, 1, 15, gaps)
    x = inputs.uniform_flat(inputs.SEED_RAGGED, total, NPDT[dtype])
    rg = tf.Ragged(lengths, offsets, dtype)
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
    classes = rg.info()
    assert sorted(c[0] for c in classes) == sorted(set(int(v) for v in lengths))
    assert sum(c[1] for c in classes) == len(lengths)


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_ragged_inverse_round_trip(tf, dtype):
    lengths, offsets, total = layout(inputs.SEED_RAGGED + 1, 120, 2, 17, True)
    x = inputs.uniform_flat(inputs.SEED_RAGGED + 1, total, NPDT[dtype])
    rg = tf.Ragged(lengths, offsets, dtype)
    xd = to_dev(x)
    y = rg.inverse(xd)
    yh = y.cpu().numpy()
    check_signals(x, yh, lengths, offsets, dtype, idx=range(0, 120, 7), inverse=True)
    z = rg.forward(y).cpu().numpy()
    for n, o in zip(lengths, offsets):
        assert oracle.rel_l2(z[o:o + n], x[o:o + n]) <= 4 * TOL[dtype]


def faults_for(lengths, rng, frac):
    """One additive fault on the final values of pass 0 in round(frac * count)
    signals, no two in one checksum group."""
    sigs = inputs.ragged_fault_signals(rng, lengths, max(1, int(round(frac * len(lengths)))))
    specs = []
    for s in sigs:
        n = int(lengths[s])
        specs.append(dict(signal=int(s), pass_=0, stage=-1, index=int(rng.integers(n)),
                          value=complex(rng.uniform(0.5, 4.0), rng.uniform(-4.0, 4.0))))
    return specs, sigs


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_ragged_faults_are_corrected(tf, dtype):
    lengths, offsets, total = layout(inputs.SEED_RAGGED + 2, 400, 3, 16, True)
    x = inputs.uniform_flat(inputs.SEED_RAGGED + 2, total, NPDT[dtype])
    rg = tf.Ragged(lengths, offsets, dtype)
    specs, sigs = faults_for(lengths, inputs.fault_rng(inputs.SEED_RAGGED + 2), 0.025)
    rg.set_faults(specs)
    y = rg.forward(to_dev(x)).cpu().numpy()
    counts, recs = rg.report()
    check_signals(x, y, lengths, offsets, dtype)
    assert counts["uncorrectable"] == 0
    fixed = sorted({r.signal for r in recs if r.action == "corrected"})
    assert fixed == sorted(int(s) for s in sigs)
    assert counts["corrected"] == len(sigs)


def test_ragged_graph_replays_match_eager(tf):
    import torch

    dtype = "c64"
    lengths, offsets, total = layout(inputs.SEED_RAGGED + 3, 256, 4, 18, False)
    x = inputs.uniform_flat(inputs.SEED_RAGGED + 3, total, NPDT[dtype])
    rg = tf.Ragged(lengths, offsets, dtype)
    specs, sigs = faults_for(lengths, inputs.fault_rng(inputs.SEED_RAGGED + 3), 0.03)
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
    # new faults drop the captured graph; the next replay re-captures
    rg.set_faults([])
    rg.forward(xd, out, use_graph=True)
    c0, r0 = rg.report()
    assert c0["detected"] == 0 and not r0
    check_signals(x, out.cpu().numpy(), lengths, offsets, dtype, idx=range(0, 256, 5))


def test_ragged_tune_keeps_results(tf):
    dtype = "c64"
    lengths, offsets, total = layout(inputs.SEED_RAGGED + 4, 64, 6, 20, False)
    x = inputs.uniform_flat(inputs.SEED_RAGGED + 4, total, NPDT[dtype])
    rg = tf.Ragged(lengths, offsets, dtype)
    xd = to_dev(x)
    out = rg.forward(xd)
    before = out.clone()
    rg.tune(xd, out, reps=1)
    info = rg.info()
    for n, cnt, d in info:
        assert int(np.prod(d["pass_len"])) == n and d["batch"] == cnt
    y = rg.forward(xd, use_graph=True).cpu().numpy()
    check_signals(x, y, lengths, offsets, dtype, idx=range(0, 64, 3))
    # every candidate is a correct plan: results agree with the untuned ones to rounding
    b = before.cpu().numpy()
    for n, o in zip(lengths, offsets):
        assert oracle.rel_l2(y[o:o + n], b[o:o + n]) <= 2 * TOL[dtype]


def test_ragged_full_size_sampled(tf):
    """4096 complex64 signals, lengths 2^k with k ~ U{6..20}, packed; faults
    in 1% of the signals; one graph launch after tuning.  The oracle checks a
    sample of signals (all faulty ones up to 2^16 and a stride of the rest);
    Parseval checks every signal."""
    import torch

    dtype = "c64"
    lengths = inputs.ragged_lengths(inputs.SEED_RAGGED, 4096, 6, 20)
    offsets = np.concatenate([[0], np.cumsum(lengths)[:-1]]).astype(np.int64)
    total = int(lengths.sum())
    x = inputs.uniform_flat(inputs.SEED_RAGGED, total, NPDT[dtype])
    rg = tf.Ragged(lengths, offsets, dtype)
    specs, sigs = faults_for(lengths, inputs.fault_rng(inputs.SEED_RAGGED), 0.01)
    xd = to_dev(x)
    out = torch.empty_like(xd)
    rg.tune(xd, out, reps=1)
    rg.set_faults(specs)
    rg.forward(xd, out, use_graph=True)
    counts, recs = rg.report()
    assert counts["uncorrectable"] == 0 and counts["corrected"] == len(sigs)
    assert sorted({r.signal for r in recs}) == sorted(int(s) for s in sigs)
    y = out.cpu().numpy()
    sample = sorted(set([int(s) for s in sigs if lengths[s] <= 1 << 16]) | set(range(0, 4096, 97)))
    check_signals(x, y, lengths, offsets, dtype, idx=sample)
    # Parseval per signal: sum |y|^2 = n sum |x|^2.  Energies are summed per
    # length class over a gathered [count, n] view (no atomics: 5.8e8
    # elements scattered into 4096 float64 bins contend heavily)
    def energy(t):
        e = torch.empty(4096, dtype=torch.float64, device="cuda")
        for n in np.unique(lengths):
            sel = np.nonzero(lengths == n)[0]
            idx = torch.from_numpy(offsets[sel]).cuda()[:, None] + torch.arange(int(n), device="cuda")[None, :]
            e[torch.from_numpy(sel).cuda()] = (t[idx].abs().double() ** 2).sum(1)
        return e

    ratio = (energy(out) / (energy(xd) * torch.from_numpy(lengths).cuda().double())).cpu().numpy()
    assert np.all(np.abs(ratio - 1) < 1e-5)
