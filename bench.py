"""Benchmark of the fault-tolerant batched C2C FFT on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--dtypes c64,c128] [--kmin 8] [--kmax 24]
                    [--no-cpu-baseline] [--no-extras]

Workload (the throughput sweep): forward C2C transforms of length N = 2^k for
k = 8..24 with N * batch = 2^28 elements in complex64 and 2^27 in complex128
(2 GiB in + 2 GiB out each), inputs i.i.d. U[-1, 1) drawn once per precision
and viewed as [batch][N]; fault tolerance CORRECT (two-sided checksum, no
faults injected).  One step = one forward transform of every (precision, k)
of the sweep with inputs resident in HBM.

Printed: one JSON line with the metric (nominal GFLOP/s = sum of 5 N log2 N
batch over the step / step time), the roofline of the dominant kernel from
HIP events on the execution stream, and the oracle's CPU throughput on a
bounded sample.  The per-size breakdown, checksum overhead (FT CORRECT vs OFF,
same kernels) and the cost of running with one injected fault per 256 signals
are in the same line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0
METRIC = "GFLOP/s & HBM GB/s, batched C2C FFT with checksum; FT overhead % vs no-FT"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--dtypes", default="c64,c128")
    ap.add_argument("--kmin", type=int, default=8)
    ap.add_argument("--kmax", type=int, default=24)
    ap.add_argument("--log2-elems", type=int, default=28, help="log2 of N*batch for complex64 (complex128: one less)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the FT off / faulty overhead runs")
    ap.add_argument("--extra-reps", type=int, default=20, help="timed runs per mode in the overhead extras "
                    "(median; after 3 warm-up runs)")
    ap.add_argument("--no-fault-runs", action="store_true", help="in the extras, skip the runs with injected faults")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="LOG2_BYTES",
                    help="only run a plain device-to-device copy of 2^LOG2_BYTES bytes (the reference kernel "
                         "for scaling the FETCH_SIZE / WRITE_SIZE counters) and exit")
    ap.add_argument("--summarize-pmc", metavar="DIR",
                    help="turn rocprofv3 --pmc output directories DIR/<label>_<FETCH_SIZE|WRITE_SIZE> (label: copy "
                         "or <dtype>_k<k>) into profiles/pmc_traffic.json")
    ap.add_argument("--workload", default="sweep",
                    choices=["sweep", "grad", "bitflip", "ragged", "ragged-class", "schemes", "calibrate"],
                    help="sweep: the throughput sweep (default, the headline line); grad: the differentiable "
                         "layer, complex64 [2048, 4096] forward + backward; bitflip: the fault-coverage campaign; "
                         "ragged: 4096 complex64 signals of lengths 2^U{6..20} in one graph launch; schemes: checksum "
                         "overhead of the block, one-sided and thread-level schemes, N = 2^8..2^16; calibrate: noise-scaled "
                         "checksum residuals of >= 10^6 fault-free groups per precision (the threshold factor kappa); "
                         "ragged-class: one length class (--class-log2, --class-count) as per-class launches and as "
                         "one persistent launch, side by side")
    ap.add_argument("--class-log2", type=int, default=19, help="ragged-class: log2 of the signal length")
    ap.add_argument("--class-count", type=int, default=64, help="ragged-class: number of signals")
    ap.add_argument("--tune", action="store_true", help="ragged-class: autotune both forms first")
    ap.add_argument("--ft", default="correct", choices=["off", "detect", "correct"],
                    help="fault-tolerance mode of the timed workload (the headline uses correct)")
    return ap.parse_args()


def cpu_baseline(sizes):
    """The FP64 oracle (C recursive radix-2, OpenMP over signals) on bounded
    samples of the same sweep (the whole sweep would take hours on the host):
    all host threads, median of 3 runs over max(1, 2^24 / N) signals of every
    size; one thread, one run over max(1, 2^20 / N) signals of every size;
    and the naive O(N^2) DFT on the correctness configuration (N = 256,
    batch 64, all threads, median of 5)."""
    import numpy as np

    import oracle
    import tfft_inputs as inputs

    threads = oracle.max_threads()

    def run(log2e, nthr, reps, kmax=24):
        times, flops, nsig = [], 0.0, 0
        xs = []
        for (dt, k) in sizes:
            if k > kmax:
                continue
            n = 1 << k
            b = max(1, (1 << log2e) // n)
            xs.append((inputs.uniform(inputs.sweep_seed(k, dt == "c128"), b, n, np.complex128), n, k, b))
            flops += 5.0 * n * k * b
            nsig += b
        for _ in range(reps):
            t = 0.0
            for x, n, k, b in xs:
                t0 = time.perf_counter()
                oracle.fft(x, threads=nthr)
                t += time.perf_counter() - t0
            times.append(t)
        return flops, sorted(times)[len(times) // 2], nsig

    fl_all, t_all, ns_all = run(24, threads, 3)
    fl_one, t_one, ns_one = run(20, 1, 1, kmax=20)
    x1 = inputs.uniform(inputs.SEED_CORRECTNESS, 64, 256, np.complex128)
    tn = []
    for _ in range(5):
        t0 = time.perf_counter()
        oracle.dft_naive(x1, threads=threads)
        tn.append(time.perf_counter() - t0)
    tn = sorted(tn)[2]
    return {"value": round(fl_all / t_all / 1e9, 3), "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 recursive radix-2 oracle over the {len(sizes)} sizes of the sweep, max(1, 2^24/N) "
                      f"signals per size ({ns_all} signals), OpenMP over signals on all {threads} host threads, "
                      f"median of 3 runs of {t_all:.2f} s; N = 2^23 and 2^24 offer 2 and 1 signals of parallelism",
            "seconds": round(t_all, 3),
            "one_core": {"value": round(fl_one / t_one / 1e9, 3), "unit": "GFLOP/s", "cores": 1,
                         "sample": f"2^20 elements of every size N <= 2^20 ({ns_one} signals), one run of "
                                   f"{t_one:.2f} s"},
            "dft_naive_correctness_config": {"seconds": tn, "n": 256, "batch": 64, "cores": threads,
                                             "GFLOPs_nominal": round(5.0 * 256 * 8 * 64 / tn / 1e9, 4)}}


def stream_copy_gbps(tf, src, dst, stream, reps=10):
    """Bandwidth (read + write bytes / time) of tfft_stream_copy copying the
    bytes of ``src`` into ``dst``, timed with events on ``stream``: the median
    of ``reps`` copies after one warm-up."""
    import torch

    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() >= nbytes
    ts = []
    with torch.cuda.stream(stream):
        tf.tfft_stream_copy(dst.data_ptr(), src.data_ptr(), nbytes, stream.cuda_stream)
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            rc = tf.tfft_stream_copy(dst.data_ptr(), src.data_ptr(), nbytes, stream.cuda_stream)
            e1.record(stream)
            assert rc == 0, rc
            e1.synchronize()
            ts.append(e0.elapsed_time(e1))
    return 2.0 * nbytes / (sorted(ts)[len(ts) // 2] * 1e-3) / 1e9


def kernel_source_sha():
    """Hash of the device code and its compile-time configuration (the
    kernel templates, their dispatch and the configuration header)."""
    h = hashlib.sha256()
    for f in ("tfft_kernels.h", "tfft_kernels.hip", "tfft_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2405_02520_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def pmc_traffic(kernel_key):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    try:
        d = json.load(open(path))
        if d.get("kernel_source_sha256") != kernel_source_sha():
            return None
        return d["entries"].get(kernel_key)
    except (OSError, ValueError, KeyError):
        return None


def copy_calibration(log2_bytes):
    """Three streaming copies of 2^log2_bytes bytes (tfft_stream_copy), the
    reference kernel whose FETCH_SIZE / WRITE_SIZE scale the pass kernels'."""
    import torch

    import paper_2405_02520_amd as tf

    n = 1 << log2_bytes
    a = torch.ones(n // 4, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    st = torch.cuda.current_stream()
    for _ in range(3):
        assert tf.tfft_stream_copy(b.data_ptr(), a.data_ptr(), n, st.cuda_stream) == 0
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "launches": 3}), flush=True)


def summarize_pmc(root):
    """Per-launch HBM traffic of the pass kernels from rocprofv3 --pmc runs.

    ``root`` holds one output directory per run, named <label>_<counter>:
    label "copy" for a plain device-to-device copy of 2^30 bytes
    (``--copy-calibration 30``), and "<dtype>_k<k>" for the sweep at one
    size; counter FETCH_SIZE or WRITE_SIZE (KiB per dispatch).  Each
    kernel's counter is scaled by bytes / counter of the copy, the same
    counter, so that the figure is in bytes whatever the counter's unit
    conventions on this chip."""
    import csv
    import glob

    def read(d):
        rows = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                rows.setdefault(r["Kernel_Name"], {}).setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
        return {k: {c: sorted(v)[len(v) // 2] for c, v in cs.items()} for k, cs in rows.items()}

    runs = {}
    for d in sorted(glob.glob(os.path.join(root, "*_FETCH_SIZE")) + glob.glob(os.path.join(root, "*_WRITE_SIZE"))):
        base = os.path.basename(d)
        label, ctr = base.rsplit("_", 2)[0], "_".join(base.rsplit("_", 2)[1:])
        runs.setdefault(label, {})[ctr] = read(d)
    copy_bytes = 1 << 30
    scale = {}
    for ctr in ("FETCH_SIZE", "WRITE_SIZE"):
        vals = [c[ctr] * 1024 for k, c in runs.get("copy", {}).get(ctr, {}).items()
                if "stream_copy" in k.lower() and ctr in c and c[ctr] * 1024 > 0.25 * copy_bytes]
        scale[ctr] = copy_bytes / max(vals) if vals else None
    out = {"kernel_source_sha256": kernel_source_sha(),
           "copy_bytes": copy_bytes, "fetch_scale": scale["FETCH_SIZE"], "write_scale": scale["WRITE_SIZE"],
           "entries": {}}
    lines = [f"copy of {copy_bytes} B: FETCH_SIZE scale {scale['FETCH_SIZE']}, WRITE_SIZE scale {scale['WRITE_SIZE']}"]
    for label, ctrs in sorted(runs.items()):
        if label == "copy" or "FETCH_SIZE" not in ctrs or "WRITE_SIZE" not in ctrs:
            continue
        for name in sorted(set(ctrs["FETCH_SIZE"]) & set(ctrs["WRITE_SIZE"])):
            if "pass_kernel" not in name:
                continue
            f = ctrs["FETCH_SIZE"][name]["FETCH_SIZE"] * 1024 * (scale["FETCH_SIZE"] or 1.0)
            w = ctrs["WRITE_SIZE"][name]["WRITE_SIZE"] * 1024 * (scale["WRITE_SIZE"] or 1.0)
            out["entries"][f"{label} {name}"] = {"fetch_bytes": f, "write_bytes": w, "traffic_bytes": f + w}
            lines.append(f"{label} {name}: fetch {f / 2**30:.3f} GiB, write {w / 2**30:.3f} GiB per launch")
    with open(os.path.join(ROOT, "profiles", "pmc_traffic.json"), "w") as fh:
        json.dump(out, fh, indent=1)
    print("\n".join(lines))


def bench_grad(args):
    """Differentiable layer: x complex64 [2048, 4096], loss sum |W * FFT(x)|^2
    with W ~ N(0,1); one step = forward transform + backward (adjoint)
    transform, both with the two-sided checksum; the loss arithmetic between
    them is torch elementwise work inside the step."""
    import numpy as np
    import torch

    from paper_2405_02520_amd import layer
    import tfft_inputs as inputs

    B, n = 2048, 4096
    x = torch.from_numpy(inputs.uniform(inputs.SEED_GRAD, B, n, np.complex64)).cuda().requires_grad_(True)
    w2 = torch.from_numpy((inputs.real_gaussian(inputs.SEED_GRAD + 1, (B, n)) ** 2).astype(np.float32)).cuda()

    def step(mode):
        x.grad = None
        y = layer.fft(x, ft_mode=mode)
        (w2 * (y.real ** 2 + y.imag ** 2)).sum().backward()

    res = {}
    for mode in ("off", "correct"):
        for _ in range(max(1, args.warmup)):
            step(mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(mode)
        torch.cuda.synchronize()
        res[mode] = (time.perf_counter() - t0) * 1e3 / args.steps
    fl = 2 * 5.0 * n * math.log2(n) * B
    out = {"metric": "GFLOP/s of the differentiable FT-FFT layer (forward + backward transforms)",
           "value": round(fl / (res["correct"] * 1e-3) / 1e9, 1), "unit": "GFLOP/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(res["correct"], 4),
           "ms_per_step_ft_off": round(res["off"], 4), "ft_overhead_pct": round((res["correct"] / res["off"] - 1) * 100, 2),
           "higher_is_better": True, "dtype": "f32", "data": "synthetic: U[-1,1) complex, W ~ N(0,1)",
           "config": {"workload": "differentiable layer, complex64 [2048, 4096], loss sum |W*FFT(x)|^2, forward + backward"}}
    print(json.dumps(out), flush=True)


def bench_bitflip(args):
    """The paper's fault-coverage protocol: 2000 test sequences (checksum
    groups of 16 signals of length 1024), one random bit flipped in half of
    them; ROC of the threshold and the CORRECT-mode outcome."""
    import numpy as np
    import torch

    import paper_2405_02520_amd as tf
    from paper_2405_02520_amd import campaign
    import tfft_inputs as inputs

    n, G, groups = 1024, 16, 2000
    out = {"metric": "bit-flip fault coverage of the two-sided checksum", "config": {
        "workload": f"{groups} groups of {G} N(0,1) signals of length {n}, one random single-bit flip in half of "
                    "the groups (random stage or final value, element, re/im part, bit)"}, "results": {}}
    for dt in args.dtypes.split(","):
        x = inputs.gaussian(inputs.SEED_PRECISION + (100 if dt == "c128" else 0), groups * G, n,
                            np.complex64 if dt == "c64" else np.complex128)
        res = campaign.run(torch.from_numpy(x).cuda(), G, seed=(inputs.SEED_PRECISION + 7) ^ 0xFA17)
        bits = np.array([f["bit"] for f in res["specs"]])
        faulty = res["faulty"]
        r = res["ratio"][faulty]
        width = 32 if dt == "c64" else 64
        mant = 23 if dt == "c64" else 52
        classes = {"mantissa_low": bits < mant // 2, "mantissa_high": (bits >= mant // 2) & (bits < mant),
                   "exponent": (bits >= mant) & (bits < width - 1), "sign": bits == width - 1}
        with tf.Plan(n, G, dt) as pl:
            kap = pl.info()["kappa"]
        det16 = ~(r <= kap)
        out["results"][dt] = {
            "roc_kappa_detection_falsealarm": [[round(k, 3), d, f] for k, d, f in res["roc"][::5]],
            "at_default_kappa": {"kappa": kap, "detected_faulty": res["detected_faulty"], "faulty": int(len(faulty)),
                            "false_alarms": res["false_alarms"], "clean": int(groups - len(faulty)),
                            "corrected": res["counts"]["corrected"], "uncorrectable": res["counts"]["uncorrectable"]},
            "detection_rate_by_bit_class": {k: (round(float(det16[m].mean()), 4) if m.any() else None)
                                            for k, m in classes.items()},
            "max_clean_ratio": float(np.max(res["ratio"][np.setdiff1d(np.arange(groups), faulty)])),
        }
    print(json.dumps(out), flush=True)


def bench_ragged(args):
    """Ragged batch: 4096 complex64 signals of lengths 2^k, k ~ U{6..20},
    packed back to back, inputs U[-1, 1); per-length plans chosen by the
    autotuner; faults injected into 1% of the signals; one step = one
    persistent kernel launch draining the work queue of every class's passes
    (replayed as a captured graph) with fault tolerance CORRECT.  Also timed:
    the same with FT off, without the graph, and the per-class launches of the
    same batch captured in one graph."""
    import numpy as np
    import torch

    import paper_2405_02520_amd as tf
    import tfft_inputs as inputs

    count = 4096
    lengths = inputs.ragged_lengths(inputs.SEED_RAGGED, count, 6, 20)
    total = int(lengths.sum())
    xd = torch.from_numpy(inputs.uniform_flat(inputs.SEED_RAGGED, total, np.complex64)).cuda()
    out = torch.empty_like(xd)
    st = torch.cuda.Stream()
    rng = inputs.fault_rng(inputs.SEED_RAGGED)
    sigs = inputs.ragged_fault_signals(rng, lengths, count // 100)  # at most one per checksum group
    faults = [dict(signal=int(s), stage=-1, index=int(rng.integers(lengths[s])),
                   value=complex(rng.uniform(0.5, 4.0), rng.uniform(-4.0, 4.0))) for s in sigs]

    # the same batch as per-class launches captured in one graph, for comparison
    rg = tf.Ragged(lengths, dtype="c64")
    with torch.cuda.stream(st):
        rg.tune(xd, out, reps=2)
    st.synchronize()

    def timed_rg(mode, graph):
        with torch.cuda.stream(st):
            for _ in range(max(1, args.warmup)):
                rg.forward(xd, out, ft_mode=mode, use_graph=graph)
            st.synchronize()
            t = time.perf_counter()
            for _ in range(args.steps):
                rg.forward(xd, out, ft_mode=mode, use_graph=graph)
            st.synchronize()
        return (time.perf_counter() - t) * 1e3 / args.steps

    rg.set_faults(faults)
    ms_class_graph = timed_rg("correct", True)
    rg.close()

    # the persistent launch: one kernel drains the queue of every class's passes
    rg = tf.Ragged(lengths, dtype="c64", persistent=True)
    t0 = time.perf_counter()
    with torch.cuda.stream(st):
        rg.tune(xd, out, reps=3)
    st.synchronize()
    tune_s = time.perf_counter() - t0

    def timed(mode, graph):
        with torch.cuda.stream(st):
            for _ in range(max(1, args.warmup)):
                rg.forward(xd, out, ft_mode=mode, use_graph=graph)
            st.synchronize()
            t = time.perf_counter()
            for _ in range(args.steps):
                rg.forward(xd, out, ft_mode=mode, use_graph=graph)
            st.synchronize()
        return (time.perf_counter() - t) * 1e3 / args.steps

    ms_off = timed("off", True)
    ms_clean = timed("correct", True)
    rg.set_faults(faults)
    ms_eager = timed("correct", False)
    ms = timed("correct", True)
    counts, _ = rg.report()
    fl = float(np.sum(5.0 * lengths * np.log2(lengths)))
    gbs = 2 * 8 * total / (ms * 1e-3) / 1e9
    classes = [{"n": n, "signals": c, "passes": d["passes"], "pass_len": d["pass_len"], "group": d["group"]}
               for n, c, d in rg.info()]
    res = {"metric": "GFLOP/s & HBM GB/s, ragged batched C2C FFT with checksum (one graph launch)",
           "value": round(fl / (ms * 1e-3) / 1e9, 1), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "dtype": "f32",
           "data": "synthetic: U[-1,1) complex", "effective_GBps": round(gbs, 1),
           "hbm_frac": round(gbs / HBM_PEAK_GBS, 4), "ms_ft_off_graph": round(ms_off, 4),
           "ms_ft_correct_eager": round(ms_eager, 4), "ms_ft_correct_no_faults": round(ms_clean, 4),
           "ms_per_class_graph": round(ms_class_graph, 4),
           "ft_overhead_pct": round((ms_clean / ms_off - 1) * 100, 2),
           "fault_overhead_pct": round((ms / ms_clean - 1) * 100, 2),
           "faults_injected": int(len(sigs)), "corrected": counts["corrected"],
           "uncorrectable": counts["uncorrectable"], "tune_s": round(tune_s, 2), "classes": classes,
           "config": {"workload": f"ragged: {count} complex64 signals, lengths 2^k with k ~ U{{6..20}} "
                                  f"({total} elements), faults in 1% of signals, autotuned, one persistent "
                                  f"kernel launch (replayed as a graph)"}}
    print(json.dumps(res), flush=True)


def bench_schemes(args):
    """Checksum overhead by granularity (the comparison of one-sided,
    thread-level two-sided and threadblock-level two-sided schemes): N =
    2^8..2^16, 2^28 (complex64) / 2^27 (complex128) elements, FT CORRECT
    without faults against FT OFF on the same kernels."""
    import numpy as np
    import torch

    import paper_2405_02520_amd as tf
    import tfft_inputs as inputs

    st = torch.cuda.Stream()
    rows = []
    for dt in args.dtypes.split(","):
        npdt = np.complex64 if dt == "c64" else np.complex128
        total = 1 << (args.log2_elems - (0 if dt == "c64" else 1))
        for k in range(max(8, args.kmin), min(16, args.kmax) + 1):
            n = 1 << k
            B = total // n
            xd = torch.from_numpy(inputs.uniform(inputs.sweep_seed(k, dt == "c128"), B, n, npdt)).cuda()
            out = torch.empty_like(xd)
            ms = {}
            schemes = ("block", "signal", "thread")
            for scheme in schemes:
                plan = tf.Plan(n, B, dt, scheme=scheme)
                for mode in (["off"] if scheme == "block" else []) + ["correct"]:
                    with torch.cuda.stream(st):
                        for _ in range(max(1, args.warmup)):
                            plan.forward(xd, out, ft_mode=mode)
                        st.synchronize()
                        t = time.perf_counter()
                        for _ in range(args.steps):
                            plan.forward(xd, out, ft_mode=mode)
                        st.synchronize()
                    ms["off" if mode == "off" else scheme] = (time.perf_counter() - t) * 1e3 / args.steps
                counts, _ = plan.report()
                assert counts["detected"] == 0, (dt, k, scheme, counts)
                plan.close()
            rows.append({"dtype": dt, "n": n, "batch": B, "ms_off": round(ms["off"], 4),
                         **{f"overhead_pct_{s}": round((ms[s] / ms["off"] - 1) * 100, 2)
                            for s in schemes},
                         "GBps_block": round(2 * total * (8 if dt == "c64" else 16) / (ms["block"] * 1e-3) / 1e9, 1)})
            del xd, out
    mean = {s: round(float(np.mean([r[f"overhead_pct_{s}"] for r in rows if f"overhead_pct_{s}" in r])), 2)
            for s in ("block", "signal", "thread")}
    print(json.dumps({"metric": "checksum overhead % vs FT off, by scheme granularity", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "mean_overhead_pct": mean, "sizes": rows,
                      "config": {"workload": "forward C2C, N = 2^8..2^16, N*batch = 2^28 (c64) / 2^27 (c128), U[-1,1), "
                                             "FT correct without faults"}}), flush=True)


def bench_calibrate(args):
    """Threshold calibration: for both precisions, fault-free transforms of
    N(0,1) and six-decade lognormal inputs at sizes spanning the one-, two- and
    three-pass plans (2^28 / 2^27 elements each), probed in DETECT mode with a
    vanishing kappa so that every group reports |d1|; the noise-scaled ratio
    |d1| / (tau / kappa) of every group is collected until each precision has
    seen at least 10^6 groups.  kappa must exceed the largest ratio."""
    import numpy as np
    import torch

    import paper_2405_02520_amd as tf
    import tfft_inputs as inputs

    out = {"metric": "noise-scaled checksum residual |d1| / (tau / kappa) of fault-free groups", "results": {}}
    for dt in args.dtypes.split(","):
        npdt = np.complex64 if dt == "c64" else np.complex128
        log2e = args.log2_elems - (0 if dt == "c64" else 1)
        rows, total, worst, rep = [], 0, 0.0, 0
        while total < 1_000_000:
            for k in (8, 10, 12, 13, 14, 16, 18, 19, 20, 22, 24):
                n = 1 << k
                b = (1 << log2e) // n
                for kind in ("gaussian", "dynamic"):
                    seed = inputs.SEED_PRECISION + 7919 * rep + 31 * k + (1 if kind == "dynamic" else 0)
                    gen = inputs.device_gaussian if kind == "gaussian" else inputs.device_dynamic
                    x = gen(seed, b, n, npdt)
                    probe = tf.Plan(n, b, dt, kappa=1e-12)
                    probe.forward(x, ft_mode="detect")
                    c, recs = probe.report()
                    probe.close()
                    r = np.array([q.residual / q.threshold * 1e-12 for q in recs if q.threshold > 0])
                    m = float(r.max()) if r.size else 0.0
                    rows.append({"k": k, "input": kind, "rep": rep, "groups": c["groups_checked"],
                                 "max_ratio": round(m, 3), "p99_ratio": round(float(np.quantile(r, 0.99)), 3)})
                    total += c["groups_checked"]
                    worst = max(worst, m)
                    del x
            rep += 1
        out["results"][dt] = {"groups": total, "max_ratio": round(worst, 3), "runs": rows}
    print(json.dumps(out), flush=True)


def bench_ragged_class(args):
    """One length class of a ragged batch (complex64, FT CORRECT, no faults):
    the per-class launches and the persistent launch (interleaved items) of
    the same signals, each replayed as a graph --steps times after --warmup
    replays; prints both times per replay (a comparison of the two forms,
    and the command its counter profiles are taken with)."""
    import numpy as np
    import torch

    import paper_2405_02520_amd as tf
    import tfft_inputs as inputs

    n = 1 << args.class_log2
    lengths = np.full(args.class_count, n, np.int64)
    xd = torch.from_numpy(inputs.uniform_flat(inputs.SEED_RAGGED, int(lengths.sum()), np.complex64)).cuda()
    out = torch.empty_like(xd)
    st = torch.cuda.Stream()
    res = {}
    for name, pers in (("per_class", False), ("persistent", True)):
        rg = tf.Ragged(lengths, dtype="c64", persistent=pers, interleave=pers)
        with torch.cuda.stream(st):
            if args.tune:
                rg.tune(xd, out, reps=2)
            for _ in range(max(1, args.warmup)):
                rg.forward(xd, out, ft_mode=args.ft, use_graph=True)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(st)
            for _ in range(args.steps):
                rg.forward(xd, out, ft_mode=args.ft, use_graph=True)
            e1.record(st)
        e1.synchronize()
        res[f"ms_{name}"] = round(e0.elapsed_time(e1) / args.steps, 4)
        rg.close()
    print(json.dumps({"workload": "ragged-class", "n": n, "signals": args.class_count, "ft": args.ft, "tuned": args.tune,
                      "steps": args.steps, **res,
                      "ratio": round(res["ms_persistent"] / res["ms_per_class"], 3)}), flush=True)


def main():
    args = parse()
    if args.workload == "calibrate":
        return bench_calibrate(args)
    if args.workload == "schemes":
        return bench_schemes(args)
    if args.workload == "ragged":
        return bench_ragged(args)
    if args.workload == "ragged-class":
        return bench_ragged_class(args)
    if args.workload == "grad":
        return bench_grad(args)
    if args.workload == "bitflip":
        return bench_bitflip(args)
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc)
        return
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only; a batched FFT shards on the batch axis with no "
              "exchange.  Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2405_02520_amd as tf
    import tfft_inputs as inputs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    dtypes = [d for d in args.dtypes.split(",") if d]
    ks = list(range(args.kmin, args.kmax + 1))
    sizes = [(dt, k) for dt in dtypes for k in ks]
    esz = {"c64": 8, "c128": 16}
    log2e = {"c64": args.log2_elems, "c128": args.log2_elems - 1}
    tdt = {"c64": torch.complex64, "c128": torch.complex128}

    # inputs: one draw per precision, resident in HBM
    xin = {}
    for dt in dtypes:
        e = 1 << log2e[dt]
        x = inputs.uniform(inputs.sweep_seed(0, dt == "c128"), 1, e, np.complex64 if dt == "c64" else np.complex128)
        xin[dt] = torch.from_numpy(x.reshape(-1)).to(dev)
        del x
    out_bytes = max(esz[dt] << log2e[dt] for dt in dtypes)
    ybuf = torch.empty(out_bytes, dtype=torch.uint8, device=dev)

    plans, xs, ys = {}, {}, {}
    for dt, k in sizes:
        n = 1 << k
        b = (1 << log2e[dt]) // n
        p = tf.Plan(n, b, dt)
        p.set_timing(True)
        plans[(dt, k)] = p
        xs[(dt, k)] = xin[dt].view(b, n)
        ys[(dt, k)] = ybuf[: n * b * esz[dt]].view(tdt[dt]).view(b, n)

    def step():
        for key in sizes:
            plans[key].forward(xs[key], out=ys[key], ft_mode=args.ft, stream=stream)

    # warm-up; the first warm-up step also checks Parseval on every size
    sanity = {}
    for w in range(max(1, args.warmup)):
        for key in sizes:
            plans[key].forward(xs[key], out=ys[key], ft_mode=args.ft, stream=stream)
            if w == 0:
                dt, k = key
                x, y = xs[key], ys[key]
                ex = torch.sum(x.real.double() ** 2 + x.imag.double() ** 2) * (1 << k)
                ey = torch.sum(y.real.double() ** 2 + y.imag.double() ** 2)
                sanity[f"{dt}_k{k}"] = abs(float(ey / ex) - 1.0)
                c, _ = plans[key].report()
                if c["detected"]:
                    raise SystemExit(f"clean run flagged {c['detected']} groups at {key}")
    torch.cuda.synchronize()
    worst_parseval = max(sanity.values())
    if worst_parseval > 1e-4:
        raise SystemExit(f"Parseval check failed: {sanity}")

    # timed region: exactly K steps
    kern = {key: [] for key in sizes}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        for key in sizes:
            pm, cm = plans[key].timings()
            kern[key].append((pm, cm))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps

    flops_step = sum(5.0 * (1 << k) * k * ((1 << log2e[dt]) >> k) for dt, k in sizes)
    value = flops_step / (ms_per_step * 1e-3) / 1e9

    # per-size breakdown and the dominant kernel
    breakdown = {}
    dom = None
    for dt, k in sizes:
        n = 1 << k
        b = (1 << log2e[dt]) // n
        rows = kern[(dt, k)]
        passes = len(rows[0][0])
        pass_ms = [sum(r[0][i] for r in rows) / len(rows) for i in range(passes)]
        corr_ms = [sum(r[1][i] for r in rows) / len(rows) for i in range(passes)]
        tot = sum(pass_ms) + sum(corr_ms)
        algo = 2.0 * n * b * esz[dt]
        breakdown[f"{dt}_k{k}"] = {
            "ms": round(tot, 4), "pass_ms": [round(v, 4) for v in pass_ms],
            "correct_ms": [round(v, 4) for v in corr_ms],
            "gflops": round(5.0 * n * k * b / (tot * 1e-3) / 1e9, 1),
            "eff_GBps": round(algo / (tot * 1e-3) / 1e9, 1),
            "pass_GBps": [round(algo / (v * 1e-3) / 1e9, 1) for v in pass_ms],
        }
        info = plans[(dt, k)].info()
        for i, v in enumerate(pass_ms):
            kind = "rows" if passes == 1 else ("last" if i == passes - 1 else "strided")
            cand = (v * len(rows), dt, k, i, kind, info["pass_len"][i], algo, v)
            if dom is None or cand[0] > dom[0]:
                dom = cand
    _, ddt, dk, dpass, dkind, dM, dalgo, dms = dom
    achieved = dalgo / (dms * 1e-3) / 1e9
    kind_code = {"rows": 0, "strided": 1, "last": 2}[dkind]
    kernel_key = (f"{ddt}_k{dk} void tfft::pass_kernel<{'float' if ddt == 'c64' else 'double'}, {dM}, {kind_code}, "
                  f"{0 if args.ft == 'off' else 1}>(tfft::PassArgs)")
    tr = pmc_traffic(kernel_key)
    if tr is not None:
        tr = tr["traffic_bytes"]
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr,
                "kernel": kernel_key, "pass": dpass, "algorithmic_bytes_per_launch": int(dalgo),
                "avg_launch_ms": round(dms, 4)}

    # checksum overhead (same kernels, FT off) and cost of injected faults
    extras = {}
    if not args.no_extras:
        for dt, k in sizes:
            key = (dt, k)
            p, x, y = plans[key], xs[key], ys[key]
            n = 1 << k
            b = (1 << log2e[dt]) // n

            def timed(mode):
                for _ in range(3):
                    p.forward(x, out=y, ft_mode=mode, stream=stream)
                ts = []
                for _ in range(args.extra_reps):
                    p.forward(x, out=y, ft_mode=mode, stream=stream)
                    pm, cm = p.timings()
                    ts.append(sum(pm) + sum(cm))
                return sorted(ts)[len(ts) // 2]

            t_off = timed("off")
            t_on = timed("correct")
            # one fault per aligned block of 256 signals (at least one), on a
            # final value of a pass, magnitude = RMS of the values there
            rng = inputs.fault_rng(inputs.sweep_seed(k, dt == "c128"))
            info = p.info()
            nf = max(1, b // 256)
            faults = []
            for i in range(nf):
                sig = min(b - 1, i * 256 + int(rng.integers(min(256, b))))
                ps = int(rng.integers(info["passes"]))
                plen = info["pass_len"][0] if ps == 0 else n
                faults.append(dict(signal=sig, pass_=ps, stage=-1, index=int(rng.integers(n)),
                                   value=math.sqrt(2.0 * plen / 3.0) * complex(0.6, -0.8)))
            if args.no_fault_runs:
                t_fault, c = float("nan"), {"corrected": 0, "detected": 0}
                nf = 0
            else:
                p.set_faults(faults)
                t_fault = timed("correct")
                c, recs = p.report()
                p.set_faults([])
            extras[f"{dt}_k{k}"] = {
                "ms_ft_off": round(t_off, 4), "ms_ft_on": round(t_on, 4), "ms_ft_on_faulty": round(t_fault, 4),
                "ft_overhead_pct": round((t_on / t_off - 1) * 100, 2),
                "fault_overhead_pct": round((t_fault / t_on - 1) * 100, 2),
                "faults": nf, "corrected": c["corrected"], "detected": c["detected"],
            }
        torch.cuda.synchronize()

    # what the library's streaming copy kernel reaches on the same bytes
    # (16-byte non-temporal loads and stores, the access the pass kernels
    # make): the attainable HBM ceiling next to the 8 TB/s peak
    copy_gbps = stream_copy_gbps(tf, xin[dtypes[0]], ybuf, stream)
    roofline["copy_GBps"] = round(copy_gbps, 1)
    roofline["frac_of_copy"] = round(achieved / copy_gbps, 4)

    res = {
        "metric": METRIC, "value": round(value, 1), "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "+".join("f32" if d == "c64" else "f64" for d in dtypes),
        "data": "synthetic: i.i.d. U[-1,1) complex, seeded",
        "config": {"workload": f"forward C2C sweep N=2^{args.kmin}..2^{args.kmax}, N*batch=2^{args.log2_elems} "
                               f"(c64) / 2^{args.log2_elems - 1} (c128), two-sided checksum CORRECT, no faults",
                   "sizes": len(sizes), "bytes_per_step": int(sum(2 * esz[dt] << log2e[dt] for dt, k in sizes))},
        "roofline": roofline,
    }
    res["effective_GBps"] = round(res["config"]["bytes_per_step"] / (ms_per_step * 1e-3) / 1e9, 1)
    res["breakdown"] = breakdown
    if extras:
        offs = [v["ms_ft_off"] for v in extras.values()]
        ons = [v["ms_ft_on"] for v in extras.values()]
        flt = [v["ms_ft_on_faulty"] for v in extras.values()]
        res["ft_overhead_pct"] = round((sum(ons) / sum(offs) - 1) * 100, 2)
        res["fault_overhead_pct"] = round((sum(flt) / sum(ons) - 1) * 100, 2)
        res["extras"] = extras
    res["parseval_worst_rel"] = worst_parseval
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(sizes)
    for p in plans.values():
        p.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
