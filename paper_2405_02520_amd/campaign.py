"""Bit-flip fault campaign and ROC of the two-sided checksum (TurboFFT
Section II-A and Section V-C: random test sequences, faults in half of them,
each fault flipping exactly one bit of the 32- or 64-bit representation of
one value; a checksum test with threshold delta; detection rate against
false-alarm rate as delta varies).

Here a test sequence is one checksum group of G signals.  Half of the groups
receive one flipped bit in one register of one member (a random butterfly
stage or the final value, a random element, the real or imaginary part, a
random bit).  One DETECT run with a vanishing threshold records the residual
|d1| of every group relative to the rounding-noise scale tau / kappa; the ROC
for every kappa follows from those ratios.  A CORRECT run at the plan's own
kappa then shows what is detected, located and corrected.
"""
from __future__ import annotations

import numpy as np
import torch

from . import Plan

BITS = {"c64": 32, "c128": 64}


def flip_specs(rng: np.random.Generator, n: int, G: int, groups: int, stages: int, dtype: str):
    """One random single-bit flip in each of the first half of the groups
    (shuffled), as tfft_fault dicts; returns (specs, faulty group indices)."""
    order = rng.permutation(groups)
    faulty = np.sort(order[: groups // 2])
    specs = []
    for g in faulty:
        specs.append(dict(signal=int(g) * G + int(rng.integers(G)), pass_=0, stage=int(rng.integers(-1, stages)),
                          index=int(rng.integers(n)), flip="re" if rng.integers(2) == 0 else "im",
                          bit=int(rng.integers(BITS[dtype]))))
    return specs, faulty


def run(x: torch.Tensor, G: int, seed: int, kappa: float = 0.0):
    """x: [groups * G, n] complex CUDA tensor (one plan pass, n <= 4096).
    ``kappa`` of the CORRECT run: 0 takes the plan's default.  Returns a dict
    with the per-group noise-scaled residuals, the ROC, the CORRECT-mode
    counts and the specs."""
    B, n = x.shape
    dtype = "c64" if x.dtype == torch.complex64 else "c128"
    groups = B // G
    probe = Plan(n, B, dtype, group=G, kappa=1e-12)  # flags every group: residuals of all of them
    info = probe.info()
    if info["passes"] != 1:
        raise ValueError("the campaign runs on one-pass sizes")
    rng = np.random.default_rng(seed)
    specs, faulty = flip_specs(rng, n, G, groups, info["stages"][0], dtype)
    probe.set_faults(specs)
    probe.forward(x, ft_mode="detect")
    counts, recs = probe.report()
    probe.close()
    ratio = np.zeros(groups)  # a group the probe did not flag has d1 = 0 exactly
    for r in recs:
        # residual / (tau / kappa) at the probe's kappa: the noise-scale ratio
        ratio[r.group] = r.residual / r.threshold * 1e-12 if r.threshold > 0 else np.inf
    is_faulty = np.zeros(groups, bool)
    is_faulty[faulty] = True
    clean_r, faulty_r = ratio[~is_faulty], ratio[is_faulty]
    kappas = np.logspace(-1, 4, 51)
    roc = [(float(k), float(np.mean(~(faulty_r <= k))), float(np.mean(~(clean_r <= k)))) for k in kappas]
    plan = Plan(n, B, dtype, group=G, kappa=kappa)
    plan.set_faults(specs)
    y = plan.forward(x, ft_mode="correct")
    c_counts, c_recs = plan.report()
    plan.close()
    detected_groups = {r.group for r in c_recs}
    return dict(ratio=ratio, faulty=faulty, specs=specs, roc=roc, y=y, counts=c_counts, records=c_recs,
                detected_faulty=int(np.sum(is_faulty[list(detected_groups)])) if detected_groups else 0,
                false_alarms=int(len(detected_groups - set(faulty.tolist()))))
