"""The allocation-free entry point (tfft_exec_noalloc) against the ordinary
one (tfft_exec_forward / tfft_exec_inverse) on the same plans and inputs,
through the C ABI: two calls in a row, the second on a smaller input, one-
and multi-pass plans (the workspace in the static scratch), with an injected
fault (counters and records in the static scratch), and the size limit."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TOL = {"c64": 1e-5, "c128": 1e-12}


@pytest.fixture(scope="module")
def env():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2405_02520_amd as tf
    import tfft_inputs as inputs

    return torch, tf, inputs


def _rel(a, b):
    a = a.detach().cpu().numpy().astype(np.complex128)
    b = b.detach().cpu().numpy().astype(np.complex128)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _pair(env, n, batch, dt, inverse, fault_sig, seed):
    """Run one plan through both entry points; return outputs and reports."""
    torch, tf, inputs = env
    npdt = np.complex64 if dt == "c64" else np.complex128
    x = torch.from_numpy(inputs.uniform(seed, batch, n, npdt)).cuda()
    st = torch.cuda.current_stream()
    print(f"noalloc case: n={n} batch={batch} {dt} inverse={inverse} fault_signal={fault_sig}", flush=True)
    with tf.Plan(n, batch, dt) as p:
        info = p.info()
        if fault_sig is not None:
            p.set_faults([dict(signal=fault_sig, pass_=info["passes"] - 1, stage=-1, index=n // 3, value=0.75 - 0.5j)])
        y_ref = torch.empty_like(x)
        fn = tf.tfft_exec_inverse if inverse else tf.tfft_exec_forward
        assert fn(p.handle, x.data_ptr(), y_ref.data_ptr(), tf.FT_CORRECT, st.cuda_stream) == tf.OK
        c_ref, r_ref = p.report()
        y_na = torch.empty_like(x)
        assert tf.tfft_exec_noalloc(p.handle, x.data_ptr(), y_na.data_ptr(), tf.FT_CORRECT, 1 if inverse else 0,
                                    st.cuda_stream) == tf.OK
        c_na, r_na = p.report()
    return x, y_ref, y_na, c_ref, r_ref, c_na, r_na


@pytest.mark.parametrize("first,second", [
    ((1024, 256, "c64", False, 37), (256, 64, "c64", False, 5)),
    ((1 << 16, 32, "c128", False, 11), (1 << 13, 16, "c128", True, 3)),
    ((1 << 14, 256, "c64", True, 200), (4096, 16, "c64", False, None)),
])
def test_noalloc_matches_exec_two_calls(env, first, second):
    for k, (n, batch, dt, inv, fs) in enumerate((first, second)):
        x, y_ref, y_na, c_ref, r_ref, c_na, r_na = _pair(env, n, batch, dt, inv, fs, 20240600 + 17 * k + n)
        assert _rel(y_na, y_ref) <= TOL[dt], (n, batch, dt)
        # same kernels, same inputs: the same bits
        assert bool((y_na == y_ref).all())
        for key in ("groups_checked", "detected", "corrected", "uncorrectable", "benign"):
            assert c_na[key] == c_ref[key], (key, c_na, c_ref)
        assert [(r.signal, r.pass_, r.action) for r in r_na] == [(r.signal, r.pass_, r.action) for r in r_ref]
        if fs is not None:
            assert c_na["corrected"] == 1 and r_na[0].signal == fs


def test_noalloc_in_place_one_pass(env):
    torch, tf, inputs = env
    n, batch = 512, 128
    x = torch.from_numpy(inputs.uniform(20240611, batch, n, np.complex64)).cuda()
    st = torch.cuda.current_stream()
    with tf.Plan(n, batch, "c64") as p:
        y_ref = p.forward(x, ft_mode="detect")
        z = x.clone()
        assert tf.tfft_exec_noalloc(p.handle, z.data_ptr(), z.data_ptr(), tf.FT_DETECT, 0, st.cuda_stream) == tf.OK
        c, _ = p.report()
    assert c["detected"] == 0
    assert bool((z == y_ref).all())


def test_noalloc_rejects_beyond_the_scratch(env):
    torch, tf, inputs = env
    # a two-pass workspace of 2^20 x 16 complex64 = 128 MiB > 64 MiB
    n, batch = 1 << 20, 16
    x = torch.zeros(batch, n, dtype=torch.complex64, device="cuda")
    y = torch.empty_like(x)
    with tf.Plan(n, batch, "c64") as p:
        assert p.info()["workspace_bytes"] > tf.SCRATCH_BYTES
        st = tf.tfft_exec_noalloc(p.handle, x.data_ptr(), y.data_ptr(), tf.FT_CORRECT, 0,
                                  torch.cuda.current_stream().cuda_stream)
        assert st == tf.E_SCRATCH
        assert b"scratch" in tf.tfft_status_string(st)
        # the plan still runs through the ordinary entry point
        p.forward(x, y, ft_mode="off")
    torch.cuda.synchronize()
