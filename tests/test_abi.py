"""The C-ABI library loads and exports every entry point declared in
include/tfft.h; argument validation that needs no device work (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tfft.h")


@pytest.fixture(scope="module")
def tf():
    lib = os.path.join(ROOT, "paper_2405_02520_amd", "libtfft.so")
    if not os.path.exists(lib):
        import runpy
        runpy.run_path(os.path.join(ROOT, "paper_2405_02520_amd", "build.py"), run_name="__main__")
    import paper_2405_02520_amd

    return paper_2405_02520_amd


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(tfft_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["tfft_plan_create", "tfft_plan_create_with", "tfft_plan_destroy", "tfft_exec_forward",
              "tfft_exec_inverse", "tfft_get_report", "tfft_set_faults", "tfft_plan_info",
              "tfft_status_string", "tfft_version", "tfft_set_timing", "tfft_get_timings"]:
        assert n in names


def test_library_exports_every_declared_symbol(tf):
    lib = ctypes.CDLL(tf.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(tf.EXPORTED) == set(declared_functions())


def test_version_and_status_strings(tf):
    assert tf.tfft_version() == 1
    assert tf.tfft_status_string(tf.OK) == b"ok"
    assert b"invalid" in tf.tfft_status_string(tf.E_INVALID)
    assert b"scratch" in tf.tfft_status_string(tf.E_SCRATCH)
    assert tf.tfft_status_string(12345) == b"unknown status"


def test_noalloc_rejects_a_null_plan(tf):
    """Argument check before any device work."""
    assert tf.tfft_exec_noalloc(None, None, None, tf.FT_CORRECT, 0, None) == tf.E_INVALID


@pytest.mark.parametrize("n,batch,dtype", [(0, 1, 0), (3, 1, 0), (12, 4, 0), (1 << 25, 1, 0), (1024, 0, 0),
                                           (1024, -5, 0), (1024, 1, 2), (1024, 1, -1)])
def test_plan_create_rejects_bad_arguments(tf, n, batch, dtype):
    h = ctypes.c_void_p(1234)
    st = tf.tfft_plan_create(ctypes.byref(h), n, batch, dtype, 0)
    assert st == tf.E_INVALID
    assert not h.value


def test_plan_create_rejects_bad_options(tf):
    h = ctypes.c_void_p()
    for group, kappa, flags in [(3, 0.0, 0), (128, 0.0, 0), (-1, 0.0, 0), (0, -1.0, 0), (0, float("nan"), 0),
                                (0, 0.0, 1 << 7), (0, 0.0, tf.PERSISTENT), (0, 0.0, tf.PERSIST_INTERLEAVE),
                                (0, 0.0, tf.PERSIST_ONE_QUEUE)]:
        opt = tf.tfft_options(flags=flags, group=group, kappa=kappa)
        assert tf.tfft_plan_create_with(ctypes.byref(h), 1024, 4, 0, ctypes.byref(opt)) == tf.E_INVALID
    assert tf.tfft_plan_create(None, 1024, 4, 0, 0) == tf.E_INVALID


def test_null_plan_is_rejected(tf):
    assert tf.tfft_plan_destroy(None) == tf.OK
    assert tf.tfft_exec_forward(None, 16, 16, 0, None) == tf.E_INVALID
    assert tf.tfft_exec_inverse(None, 16, 16, 0, None) == tf.E_INVALID
    assert tf.tfft_get_report(None, None, None, 0) == tf.E_INVALID
    assert tf.tfft_set_faults(None, None, 0) == tf.E_INVALID
    assert tf.tfft_plan_info(None, None) == tf.E_INVALID
    assert tf.tfft_set_timing(None, 1) == tf.E_INVALID
    assert tf.tfft_get_timings(None, None, None) == tf.E_INVALID


def test_record_layouts_match_header(tf):
    assert ctypes.sizeof(tf.tfft_record) == 8 * 3 + 4 * 4 + 8 * 4
    assert ctypes.sizeof(tf.tfft_fault) == 8 + 4 + 4 + 8 + 16 + 8
    assert ctypes.sizeof(tf.tfft_counts) == 7 * 8


def test_options_layout_and_pass_forcing(tf):
    assert ctypes.sizeof(tf.tfft_options) == 4 + 4 + 8 + 4 + 4 + 4 + 5 * 4
    h = ctypes.c_void_p()
    for passes, grid_scale in [(4, 0), (-1, 0), (0, 4), (0, -4)]:
        opt = tf.tfft_options(passes=passes, grid_scale=grid_scale)
        assert tf.tfft_plan_create_with(ctypes.byref(h), 1024, 4, 0, ctypes.byref(opt)) == tf.E_INVALID
    # pass counts outside what the decomposition supports for that length
    for n, passes in [(1 << 13, 1), (1 << 7, 2), (1 << 21, 2), (1 << 11, 3)]:
        opt = tf.tfft_options(passes=passes)
        assert tf.tfft_plan_create_with(ctypes.byref(h), n, 4, 0, ctypes.byref(opt)) == tf.E_UNSUPPORTED
    assert not h.value


def _ragged_create(tf, lengths, offsets, dtype=0):
    h = ctypes.c_void_p(1234)
    L = (ctypes.c_int64 * max(1, len(lengths)))(*lengths)
    O = (ctypes.c_int64 * max(1, len(offsets)))(*offsets)
    st = tf.tfft_ragged_create(ctypes.byref(h), len(lengths), L, O, dtype, None)
    return st, h


@pytest.mark.parametrize("lengths,offsets,dtype", [
    ([], [], 0),                      # no signals
    ([64, 48], [0, 64], 0),           # not a power of two
    ([64, 1], [0, 64], 0),            # shorter than 2
    ([64, 1 << 25], [0, 64], 0),      # longer than 2^24
    ([64, 64], [0, -64], 0),          # negative offset
    ([64, 64], [0, 32], 0),           # overlapping signals
    ([64, 128], [100, 0], 0),         # overlapping, given out of order
    ([64], [0], 2),                   # unknown dtype
])
def test_ragged_create_rejects_bad_arguments(tf, lengths, offsets, dtype):
    st, h = _ragged_create(tf, lengths, offsets, dtype)
    assert st == tf.E_INVALID
    assert not h.value


def test_null_ragged_is_rejected(tf):
    assert tf.tfft_ragged_destroy(None) == tf.OK
    assert tf.tfft_ragged_exec(None, 16, 16, 0, 0, 0, None) == tf.E_INVALID
    assert tf.tfft_ragged_get_report(None, None, None, 0) == tf.E_INVALID
    assert tf.tfft_ragged_set_faults(None, None, 0) == tf.E_INVALID
    assert tf.tfft_ragged_tune(None, 16, 16, None, 1) == tf.E_INVALID
    assert tf.tfft_ragged_info(None, None, None, None, None, 0) == tf.E_INVALID
    assert tf.tfft_ragged_create(None, 1, None, None, 0, None) == tf.E_INVALID


def test_scheme_option_validation(tf):
    h = ctypes.c_void_p()
    for scheme in (-1, 3):
        opt = tf.tfft_options(scheme=scheme)
        assert tf.tfft_plan_create_with(ctypes.byref(h), 1024, 4, 0, ctypes.byref(opt)) == tf.E_INVALID
    assert not h.value
