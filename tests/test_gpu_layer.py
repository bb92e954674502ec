"""Differentiable layer: the backward pass is the adjoint transform F^H run
through the same fault-tolerant kernels.  Checked against central finite
differences (FP64, N=64, batch 8) and against the FP64 oracle's gradient
2 F^H(|W|^2 * F x) of the loss sum |W * FFT(x)|^2 at the layer's full size."""
import numpy as np
import pytest

import oracle
import tfft_inputs as inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def layer():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_02520_amd import layer as L

    yield L
    L.clear_plan_cache()


def loss_fn(layer, x, w):
    y = layer.fft(x)
    return (w * (y.real ** 2 + y.imag ** 2)).sum()


def test_finite_differences_fp64(layer):
    import torch

    B, n = 8, 64
    x0 = inputs.uniform(inputs.SEED_GRAD, B, n, np.complex128)
    w = torch.from_numpy(inputs.real_gaussian(inputs.SEED_GRAD + 1, (B, n)) ** 2).cuda()
    x = torch.from_numpy(x0).cuda().requires_grad_(True)
    loss_fn(layer, x, w).backward()
    g = x.grad.cpu().numpy()
    h = 1e-6
    fd = np.zeros_like(x0)
    with torch.no_grad():
        for idx in np.ndindex(B, n):
            for part, unit in ((0, 1.0), (1, 1j)):
                xp = x0.copy()
                xm = x0.copy()
                xp[idx] += h * unit
                xm[idx] -= h * unit
                lp = float(loss_fn(layer, torch.from_numpy(xp).cuda(), w))
                lm = float(loss_fn(layer, torch.from_numpy(xm).cuda(), w))
                fd[idx] += unit * (lp - lm) / (2 * h)
    assert oracle.rel_l2(g, fd) <= 1e-6


def test_reference_gradient_full_size(layer):
    """complex64 [2048, 4096], loss sum |W * FFT(x)|^2 with W ~ N(0,1)."""
    import torch

    B, n = 2048, 4096
    x0 = inputs.uniform(inputs.SEED_GRAD, B, n, np.complex64)
    W = inputs.real_gaussian(inputs.SEED_GRAD + 1, (B, n))
    x = torch.from_numpy(x0).cuda().requires_grad_(True)
    w2 = torch.from_numpy((W ** 2).astype(np.float32)).cuda()
    loss_fn(layer, x, w2).backward()
    g = x.grad.cpu().numpy()
    xf = oracle.fft(x0.astype(np.complex128))
    ref = 2.0 * oracle.fft((W ** 2) * xf, inverse=True, scale=1.0)
    assert oracle.rel_l2(g, ref) <= 1e-5
    reps = layer.last_reports()
    for r in reps.values():
        assert r["forward"][0]["detected"] == 0 and r["backward"][0]["detected"] == 0


def test_fault_in_backward_is_corrected(layer):
    import torch

    B, n = 64, 1024
    x0 = inputs.uniform(inputs.SEED_GRAD + 2, B, n, np.complex64)
    W = inputs.real_gaussian(inputs.SEED_GRAD + 3, (B, n))
    w2 = torch.from_numpy((W ** 2).astype(np.float32)).cuda()
    x = torch.from_numpy(x0).cuda().requires_grad_(True)
    loss_fn(layer, x, w2)  # creates the plans
    fwd, adj = layer._plans(n, B, torch.complex64, x.device)
    adj.set_faults([dict(signal=17, pass_=0, stage=1, index=333, value=50.0 - 20.0j)])
    x.grad = None
    loss_fn(layer, x, w2).backward()
    counts, recs = adj.report()
    adj.set_faults([])
    assert counts["corrected"] == 1 and recs[0].signal == 17
    xf = oracle.fft(x0.astype(np.complex128))
    ref = 2.0 * oracle.fft((W ** 2) * xf, inverse=True, scale=1.0)
    assert oracle.rel_l2(x.grad.cpu().numpy(), ref) <= 1e-5
