"""Python binding of the fault-tolerant batched FFT library (``libtfft.so``).

Argument marshalling only: every step of the transform and of the two-sided
checksum runs in the HIP kernels behind the C ABI declared in
``include/tfft.h``.  PyTorch supplies device memory and the HIP stream.
There is no CPU fallback: if the library is not built, importing this package
raises.

The functions ``tfft_*`` mirror the C entry points one to one; ``Plan`` wraps
them for torch tensors.
"""
from __future__ import annotations

import ctypes
import os
import warnings
from dataclasses import dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
# TFFT_LIB selects another build of the library (a compile-time variant);
# the default is the in-tree build next to this file.
LIB_PATH = os.environ.get("TFFT_LIB") or os.path.join(_HERE, "libtfft.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is not built; run `python paper_2405_02520_amd/build.py` (hipcc, gfx950) first")

_lib = ctypes.CDLL(LIB_PATH)

# ----------------------------------------------------------- ABI constants
C64, C128 = 0, 1
FT_OFF, FT_DETECT, FT_CORRECT = 0, 1, 2
OK, UNCORRECTABLE = 0, 1
E_INVALID, E_UNSUPPORTED, E_NOMEM, E_HIP, E_STATE, E_SCRATCH = -1, -2, -3, -4, -5, -6
SCRATCH_BYTES = 64 << 20  # the library's static device scratch (tfft_exec_noalloc)
INVERSE_UNSCALED = 1
PERSISTENT = 2
PERSIST_INTERLEAVE = 4
PERSIST_ONE_QUEUE = 8
ACT_DETECTED, ACT_CORRECTED, ACT_BENIGN, ACT_UNCORRECTABLE = 1, 2, 3, 4
LOC_NONE, LOC_QUOTIENT, LOC_PER_SIGNAL, LOC_THREAD, LOC_SUBSIGNAL = 0, 1, 2, 3, 4
SCHEME_BLOCK, SCHEME_SIGNAL, SCHEME_THREAD = 0, 1, 2
_SCHEMES = {"block": SCHEME_BLOCK, "signal": SCHEME_SIGNAL, "thread": SCHEME_THREAD}
ACTION_NAMES = {ACT_DETECTED: "detected", ACT_CORRECTED: "corrected", ACT_BENIGN: "benign",
                ACT_UNCORRECTABLE: "uncorrectable"}
_MODES = {"off": FT_OFF, "detect": FT_DETECT, "correct": FT_CORRECT}


class tfft_options(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("group", ctypes.c_int32), ("kappa", ctypes.c_double),
                ("passes", ctypes.c_int32), ("grid_scale", ctypes.c_int32), ("scheme", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("split", ctypes.c_int32), ("reserved", ctypes.c_int32 * 3)]


MAX_PASSES = 3


class tfft_plan_desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("batch", ctypes.c_int64), ("dtype", ctypes.c_int32),
                ("passes", ctypes.c_int32), ("pass_len", ctypes.c_int32 * MAX_PASSES),
                ("group", ctypes.c_int32 * MAX_PASSES), ("elems_per_thread", ctypes.c_int32 * MAX_PASSES),
                ("tile_signals", ctypes.c_int32 * MAX_PASSES), ("stages", ctypes.c_int32 * MAX_PASSES),
                ("radices", (ctypes.c_int32 * 8) * MAX_PASSES), ("groups", ctypes.c_int64 * MAX_PASSES),
                ("workspace_bytes", ctypes.c_size_t), ("kappa", ctypes.c_double)]


class tfft_counts(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in
                ("groups_checked", "detected", "corrected", "uncorrectable", "benign", "n_records", "dropped")]


class tfft_record(ctypes.Structure):
    _fields_ = [("signal", ctypes.c_int64), ("sub", ctypes.c_int64), ("group", ctypes.c_int64),
                ("pass_", ctypes.c_int32), ("member", ctypes.c_int32), ("action", ctypes.c_int32),
                ("method", ctypes.c_int32), ("residual", ctypes.c_double), ("threshold", ctypes.c_double),
                ("ratio_re", ctypes.c_double), ("ratio_im", ctypes.c_double)]


class tfft_fault(ctypes.Structure):
    _fields_ = [("signal", ctypes.c_int64), ("pass_", ctypes.c_int32), ("stage", ctypes.c_int32),
                ("index", ctypes.c_int64), ("dre", ctypes.c_double), ("dim", ctypes.c_double),
                ("mode", ctypes.c_int32), ("bit", ctypes.c_int32)]


FAULT_ADD, FAULT_FLIP_RE, FAULT_FLIP_IM = 0, 1, 2


_P = ctypes.c_void_p
_sig = {
    "tfft_plan_create": ([ctypes.POINTER(_P), ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_uint32],
                         ctypes.c_int),
    "tfft_plan_create_with": ([ctypes.POINTER(_P), ctypes.c_int64, ctypes.c_int64, ctypes.c_int,
                               ctypes.POINTER(tfft_options)], ctypes.c_int),
    "tfft_plan_destroy": ([_P], ctypes.c_int),
    "tfft_exec_forward": ([_P, _P, _P, ctypes.c_int, _P], ctypes.c_int),
    "tfft_exec_inverse": ([_P, _P, _P, ctypes.c_int, _P], ctypes.c_int),
    "tfft_exec_noalloc": ([_P, _P, _P, ctypes.c_int, ctypes.c_int, _P], ctypes.c_int),
    "tfft_get_report": ([_P, ctypes.POINTER(tfft_counts), ctypes.POINTER(tfft_record), ctypes.c_int64],
                        ctypes.c_int),
    "tfft_set_faults": ([_P, ctypes.POINTER(tfft_fault), ctypes.c_int64], ctypes.c_int),
    "tfft_plan_info": ([_P, ctypes.POINTER(tfft_plan_desc)], ctypes.c_int),
    "tfft_set_timing": ([_P, ctypes.c_int], ctypes.c_int),
    "tfft_get_timings": ([_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "tfft_ragged_create": ([ctypes.POINTER(_P), ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                            ctypes.POINTER(ctypes.c_int64), ctypes.c_int, ctypes.POINTER(tfft_options)], ctypes.c_int),
    "tfft_ragged_destroy": ([_P], ctypes.c_int),
    "tfft_ragged_exec": ([_P, _P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int, _P], ctypes.c_int),
    "tfft_ragged_get_report": ([_P, ctypes.POINTER(tfft_counts), ctypes.POINTER(tfft_record), ctypes.c_int64],
                               ctypes.c_int),
    "tfft_ragged_set_faults": ([_P, ctypes.POINTER(tfft_fault), ctypes.c_int64], ctypes.c_int),
    "tfft_ragged_tune": ([_P, _P, _P, _P, ctypes.c_int], ctypes.c_int),
    "tfft_ragged_info": ([_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                          ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(tfft_plan_desc), ctypes.c_int64],
                         ctypes.c_int),
    "tfft_plan_describe": ([ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(tfft_options),
                            ctypes.POINTER(tfft_plan_desc)], ctypes.c_int),
    "tfft_host_root": ([ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "tfft_host_checksum_vector": ([ctypes.c_int64, ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_double)],
                                  ctypes.c_int),
    "tfft_stream_copy": ([_P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "tfft_status_string": ([ctypes.c_int], ctypes.c_char_p),
    "tfft_version": ([], ctypes.c_int),
}
for _name, (_args, _res) in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = _res
    globals()[_name] = _f

EXPORTED = tuple(_sig)


class TfftError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {tfft_status_string(status).decode()} ({status})")
        self.status = status


def _check(status: int, what: str) -> int:
    if status < 0:
        raise TfftError(status, what)
    return status


@dataclass
class Record:
    signal: int
    sub: int
    group: int
    pass_: int
    member: int
    action: str
    method: int
    residual: float
    threshold: float
    ratio: complex


def _dtype_code(dtype) -> int:
    s = str(dtype)
    if s in ("c64", "complex64", "torch.complex64"):
        return C64
    if s in ("c128", "complex128", "torch.complex128"):
        return C128
    raise ValueError(f"unsupported dtype {dtype!r}")


class Plan:
    """A plan for ``batch`` length-``n`` complex transforms on the current device."""

    def __init__(self, n: int, batch: int, dtype="c64", group: int = 0, kappa: float = 0.0,
                 inverse_unscaled: bool = False, passes: int = 0, grid_scale: int = 0, scheme="block",
                 chunk: int = 0, split: int = 0):
        """scheme: "block" (two-sided, per group of signals), "signal"
        (one-sided, per signal or sub-signal) or "thread" (per radix
        butterfly).  chunk: multi-pass plans run the batch in chunks of this
        many signals (a multiple of 64; 0 = the whole batch)."""
        self.n, self.batch = int(n), int(batch)
        self.dtype_code = _dtype_code(dtype)
        sch = _SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
        opt = tfft_options(flags=INVERSE_UNSCALED if inverse_unscaled else 0, group=int(group), kappa=float(kappa),
                           passes=int(passes), grid_scale=int(grid_scale), scheme=sch, chunk=int(chunk),
                           split=int(split))
        h = _P()
        _check(tfft_plan_create_with(ctypes.byref(h), self.n, self.batch, self.dtype_code, ctypes.byref(opt)),
               "tfft_plan_create_with")
        self._h = h
        self.last_status = OK

    def close(self):
        if getattr(self, "_h", None):
            tfft_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        d = tfft_plan_desc()
        _check(tfft_plan_info(self._h, ctypes.byref(d)), "tfft_plan_info")
        return _desc_dict(d)

    def _check_tensor(self, t, name):
        import torch
        want = torch.complex64 if self.dtype_code == C64 else torch.complex128
        if not t.is_cuda or t.dtype != want or not t.is_contiguous() or t.numel() != self.n * self.batch:
            raise ValueError(f"{name} must be a contiguous {want} CUDA tensor with {self.batch}x{self.n} elements")

    def _exec(self, fn, x, out, ft_mode, stream):
        import torch
        self._check_tensor(x, "input")
        if out is None:
            out = torch.empty_like(x)
        self._check_tensor(out, "output")
        mode = _MODES[ft_mode] if isinstance(ft_mode, str) else int(ft_mode)
        st = stream if stream is not None else torch.cuda.current_stream(x.device)
        _check(fn(self._h, x.data_ptr(), out.data_ptr(), mode, st.cuda_stream), fn.__name__)
        return out

    def forward(self, x, out=None, ft_mode="correct", stream=None):
        return self._exec(tfft_exec_forward, x, out, ft_mode, stream)

    def inverse(self, x, out=None, ft_mode="correct", stream=None):
        return self._exec(tfft_exec_inverse, x, out, ft_mode, stream)

    def execute_noalloc(self, x, out, ft_mode="correct", inverse=False, stream=None):
        """tfft_exec_noalloc: the transform with its report and workspace in
        the library's static device scratch; ``out`` must be given (nothing
        is allocated)."""
        import torch
        self._check_tensor(x, "input")
        self._check_tensor(out, "output")
        mode = _MODES[ft_mode] if isinstance(ft_mode, str) else int(ft_mode)
        st = stream if stream is not None else torch.cuda.current_stream(x.device)
        _check(tfft_exec_noalloc(self._h, x.data_ptr(), out.data_ptr(), mode, 1 if inverse else 0, st.cuda_stream),
               "tfft_exec_noalloc")
        return out

    def set_faults(self, faults):
        """faults: iterable of dicts with keys signal, pass_, stage, index and
        either value (complex, added) or flip ("re" | "im") with bit."""
        arr, n = _fault_array(faults)
        _check(tfft_set_faults(self._h, arr, n), "tfft_set_faults")

    def set_timing(self, enable: bool = True):
        _check(tfft_set_timing(self._h, 1 if enable else 0), "tfft_set_timing")

    def timings(self):
        """(pass_ms[passes], correct_ms[passes]) of the last timed execution."""
        a = (ctypes.c_double * MAX_PASSES)()
        b = (ctypes.c_double * MAX_PASSES)()
        _check(tfft_get_timings(self._h, a, b), "tfft_get_timings")
        p = self.info()["passes"]
        return list(a[:p]), list(b[:p])

    def report(self, cap: int | None = None):
        """(counts dict, [Record]) of the last execution; synchronises its stream."""
        c, out, self.last_status = _report(tfft_get_report, self._h, cap)
        return c, out


def _fault_array(faults):
    faults = list(faults)
    arr = (tfft_fault * max(1, len(faults)))()
    for i, f in enumerate(faults):
        v = complex(f.get("value", 0.0))
        mode = {None: FAULT_ADD, "re": FAULT_FLIP_RE, "im": FAULT_FLIP_IM}[f.get("flip")]
        arr[i] = tfft_fault(int(f["signal"]), int(f.get("pass_", 0)), int(f.get("stage", -1)),
                            int(f["index"]), v.real, v.imag, mode, int(f.get("bit", 0)))
    return arr, len(faults)


def _report(fn, h, cap):
    counts = tfft_counts()
    _check(fn(h, ctypes.byref(counts), None, 0), fn.__name__)
    n = counts.n_records if cap is None else min(cap, counts.n_records)
    recs = (tfft_record * max(1, n))()
    st = _check(fn(h, ctypes.byref(counts), recs, n), fn.__name__)
    if st == UNCORRECTABLE:
        warnings.warn("tfft: a flagged checksum group could not be corrected", RuntimeWarning, stacklevel=3)
    c = {k: getattr(counts, k) for k, _ in tfft_counts._fields_}
    out = [Record(r.signal, r.sub, r.group, r.pass_, r.member, ACTION_NAMES.get(r.action, str(r.action)),
                  r.method, r.residual, r.threshold, complex(r.ratio_re, r.ratio_im)) for r in recs[:n]]
    return c, out, st


class Ragged:
    """Signals of mixed power-of-two lengths in one flat buffer: signal i is
    elements [offsets[i], offsets[i] + lengths[i]) of the input and output
    (default offsets: packed back to back).  Each length class runs as one
    plan addressing its signals through a device offset table; ``use_graph``
    replays all launches of all classes as one captured HIP graph."""

    def __init__(self, lengths, offsets=None, dtype="c64", group: int = 0, kappa: float = 0.0,
                 persistent: bool = False, interleave: bool = False, one_queue: bool = False):
        """persistent: every pass of every class runs in one persistent kernel
        launch that drains a queue of work items (lengths 64..2^24);
        interleave: its items take every n-th checksum group of a block of
        signals instead of a range; one_queue: a single work queue instead of
        one per XCD (the tuner may change both)."""
        import numpy as np
        self.lengths = np.asarray(lengths, dtype=np.int64)
        if offsets is None:
            offsets = np.concatenate([[0], np.cumsum(self.lengths)[:-1]]) if len(self.lengths) else []
        self.offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        self.count = int(len(self.lengths))
        self.extent = int((self.offsets + self.lengths).max()) if self.count else 0
        self.dtype_code = _dtype_code(dtype)
        flags = ((PERSISTENT if persistent else 0) | (PERSIST_INTERLEAVE if interleave else 0) |
                 (PERSIST_ONE_QUEUE if one_queue else 0))
        opt = tfft_options(flags=flags, group=int(group), kappa=float(kappa))
        self.persistent = bool(persistent)
        ln = np.ascontiguousarray(self.lengths)
        h = _P()
        _check(tfft_ragged_create(ctypes.byref(h), self.count,
                                  ln.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  self.dtype_code, ctypes.byref(opt)), "tfft_ragged_create")
        self._h = h
        self._gstream = None
        self.last_status = OK

    def close(self):
        if getattr(self, "_h", None):
            tfft_ragged_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_tensor(self, t, name):
        import torch
        want = torch.complex64 if self.dtype_code == C64 else torch.complex128
        if not t.is_cuda or t.dtype != want or not t.is_contiguous() or t.numel() < self.extent:
            raise ValueError(f"{name} must be a contiguous {want} CUDA tensor of at least {self.extent} elements")

    def _stream(self, x, use_graph, stream):
        import torch
        st = stream if stream is not None else torch.cuda.current_stream(x.device)
        if use_graph and st.cuda_stream == 0:
            # graphs are captured on a stream of their own (the null stream cannot capture)
            if self._gstream is None:
                self._gstream = torch.cuda.Stream(x.device)
            return st, self._gstream
        return st, st

    def execute(self, x, out=None, ft_mode="correct", inverse=False, use_graph=False, stream=None):
        import torch
        self._check_tensor(x, "input")
        if out is None:
            out = torch.empty_like(x)
        self._check_tensor(out, "output")
        mode = _MODES[ft_mode] if isinstance(ft_mode, str) else int(ft_mode)
        caller, st = self._stream(x, use_graph, stream)
        if st is not caller:
            st.wait_stream(caller)
        _check(tfft_ragged_exec(self._h, x.data_ptr(), out.data_ptr(), mode, 1 if inverse else 0,
                                1 if use_graph else 0, st.cuda_stream), "tfft_ragged_exec")
        if st is not caller:
            caller.wait_stream(st)
            x.record_stream(st)
            out.record_stream(st)
        return out

    def forward(self, x, out=None, ft_mode="correct", use_graph=False, stream=None):
        return self.execute(x, out, ft_mode, False, use_graph, stream)

    def inverse(self, x, out=None, ft_mode="correct", use_graph=False, stream=None):
        return self.execute(x, out, ft_mode, True, use_graph, stream)

    def set_faults(self, faults):
        """As Plan.set_faults, with ``signal`` the ragged index."""
        arr, n = _fault_array(faults)
        _check(tfft_ragged_set_faults(self._h, arr, n), "tfft_ragged_set_faults")

    def tune(self, x, out, reps: int = 3, stream=None):
        import torch
        self._check_tensor(x, "input")
        self._check_tensor(out, "output")
        st = stream if stream is not None else torch.cuda.current_stream(x.device)
        _check(tfft_ragged_tune(self._h, x.data_ptr(), out.data_ptr(), st.cuda_stream, int(reps)),
               "tfft_ragged_tune")

    def info(self):
        """[(length, signals, plan description dict)] per length class."""
        nc = ctypes.c_int64()
        _check(tfft_ragged_info(self._h, ctypes.byref(nc), None, None, None, 0), "tfft_ragged_info")
        k = nc.value
        ln = (ctypes.c_int64 * max(1, k))()
        cn = (ctypes.c_int64 * max(1, k))()
        ds = (tfft_plan_desc * max(1, k))()
        _check(tfft_ragged_info(self._h, ctypes.byref(nc), ln, cn, ds, k), "tfft_ragged_info")
        return [(int(ln[i]), int(cn[i]), _desc_dict(ds[i])) for i in range(k)]

    def report(self, cap: int | None = None):
        """Merged (counts dict, [Record]) of the last execution; records carry the ragged index."""
        c, out, self.last_status = _report(tfft_ragged_get_report, self._h, cap)
        return c, out


def describe(n: int, batch: int, dtype="c64", group: int = 0, kappa: float = 0.0, passes: int = 0,
             grid_scale: int = 0, scheme="block", split: int = 0) -> dict:
    """The plan description (as ``Plan.info``) of a plan with these
    arguments, computed on the host without a device."""
    sch = _SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
    opt = tfft_options(group=int(group), kappa=float(kappa), passes=int(passes), grid_scale=int(grid_scale), scheme=sch,
                       split=int(split))
    d = tfft_plan_desc()
    _check(tfft_plan_describe(int(n), int(batch), _dtype_code(dtype), ctypes.byref(opt), ctypes.byref(d)),
           "tfft_plan_describe")
    return _desc_dict(d)


def host_root(t: int, n: int) -> complex:
    """w_n^t as the plans generate it (binary64, host)."""
    out = (ctypes.c_double * 2)()
    _check(tfft_host_root(int(t), int(n), out), "tfft_host_root")
    return complex(out[0], out[1])


def host_checksum_vector(m: int, inverse: bool = False, scale: float = 1.0):
    """The checksum vector c = scale (e^T W)^T a plan uploads (binary64,
    host), as a complex128 numpy array."""
    import numpy as np
    out = np.empty(2 * int(m), dtype=np.float64)
    _check(tfft_host_checksum_vector(int(m), 1 if inverse else 0, float(scale),
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "tfft_host_checksum_vector")
    return out.view(np.complex128)


def _desc_dict(d) -> dict:
    p = d.passes
    return dict(n=d.n, batch=d.batch, dtype=d.dtype, passes=p, pass_len=list(d.pass_len[:p]),
                group=list(d.group[:p]), elems_per_thread=list(d.elems_per_thread[:p]),
                tile_signals=list(d.tile_signals[:p]), stages=list(d.stages[:p]),
                radices=[list(d.radices[i][:d.stages[i]]) for i in range(p)], groups=list(d.groups[:p]),
                workspace_bytes=int(d.workspace_bytes), kappa=d.kappa)
