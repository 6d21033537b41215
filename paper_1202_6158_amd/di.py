"""ctypes binding of libdi.so (argument marshalling only).

Every step of a solve runs in the library's HIP kernels; this module converts
Python arguments into the C structures of include/di.h, passes torch device
tensors as raw pointers (with DI_DEVICE_PTRS) together with torch's current
HIP stream, and raises :class:`DiError` for a non-OK status.  There is no
fallback: if libdi.so is missing, importing this module fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdi.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libdi.so not built: run `python -c 'import __graft_entry__ as g; g.build()'` "
                      "or `python paper_1202_6158_amd/compile_lib.py` (expected at %s)" % LIB_PATH)

_lib = ctypes.CDLL(LIB_PATH)

# ------------------------------------------------------------------ constants
OK, EINVAL, ENOMEM, EDEVICE, ENOTCONV, EAGAIN, ECANCELED, EBUSY = 0, -1, -2, -3, -4, -5, -6, -7
FP32_FLUID, FP64 = 0, 1
DEVICE_PTRS, RESUME, TIMING, TRACE = 1, 2, 4, 8
SCHED_MEAN, SCHED_OP2, SCHED_OP = 0, 1, 2
PRECISION = {"fp32": FP32_FLUID, "fp64": FP64, FP32_FLUID: FP32_FLUID, FP64: FP64}
SCHEDULE = {"mean": SCHED_MEAN, "op2": SCHED_OP2, "op": SCHED_OP}
STATUS_NAMES = {OK: "DI_OK", EINVAL: "DI_EINVAL", ENOMEM: "DI_ENOMEM", EDEVICE: "DI_EDEVICE",
                ENOTCONV: "DI_ENOTCONV", EAGAIN: "DI_EAGAIN", ECANCELED: "DI_ECANCELED",
                EBUSY: "DI_EBUSY"}


class DiError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status
        self.message = message


class Tune(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_int32), ("c", ctypes.c_float),
                ("window_log2", ctypes.c_int32), ("check_every", ctypes.c_int32),
                ("threads", ctypes.c_int32), ("tables", ctypes.c_int32),
                ("persist", ctypes.c_int32)]


class TuneTrial(ctypes.Structure):
    _fields_ = [("tune", Tune), ("seconds", ctypes.c_double), ("status", ctypes.c_int32),
                ("pad", ctypes.c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [("d", ctypes.c_double), ("tol", ctypes.c_double), ("precision", ctypes.c_int32),
                ("normalize", ctypes.c_int32), ("max_rounds", ctypes.c_int64),
                ("tune", ctypes.POINTER(Tune)), ("flags", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("state_f", ctypes.c_void_p), ("state_h", ctypes.c_void_p),
                ("trace_sets", ctypes.c_void_p), ("trace_rounds", ctypes.c_int64)]


class Stats(ctypes.Structure):
    _fields_ = [("residual_l1", ctypes.c_double), ("err_bound_l1", ctypes.c_double),
                ("mass_drift", ctypes.c_double), ("seconds", ctypes.c_double),
                ("rounds", ctypes.c_int64), ("nodes_diffused", ctypes.c_int64),
                ("edges_diffused", ctypes.c_int64), ("kernel_seconds", ctypes.c_double),
                ("kernel_launches", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerOpts(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_int64), ("max_slots", ctypes.c_int32),
                ("topk", ctypes.c_int32), ("precision", ctypes.c_int32), ("pad", ctypes.c_int32),
                ("tune", ctypes.POINTER(Tune))]


class Result(ctypes.Structure):
    _fields_ = [("req_id", ctypes.c_uint64), ("status", ctypes.c_int32), ("k", ctypes.c_int32),
                ("top_ids", ctypes.c_int32 * 1024), ("top_x", ctypes.c_double * 1024),
                ("residual_l1", ctypes.c_double), ("err_bound_l1", ctypes.c_double),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("rounds", ctypes.c_int64),
                ("edges_diffused", ctypes.c_int64)]

    def as_dict(self):
        k = self.k
        return {"req_id": self.req_id, "status": self.status,
                "top_ids": np.array(self.top_ids[:k], dtype=np.int32),
                "top_x": np.array(self.top_x[:k]), "residual_l1": self.residual_l1,
                "err_bound_l1": self.err_bound_l1, "t_submit": self.t_submit,
                "t_admit": self.t_admit, "t_done": self.t_done, "rounds": self.rounds,
                "edges_diffused": self.edges_diffused}


class ServerMetrics(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("cancelled", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("active", ctypes.c_int64),
                ("hbm_in_use", ctypes.c_int64), ("hbm_budget", ctypes.c_int64),
                ("p50_latency_s", ctypes.c_double), ("p99_latency_s", ctypes.c_double),
                ("qps", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = ctypes.c_void_p
_SIGS = {
    "di_graph_create": [ctypes.c_int64, ctypes.c_int64, _P, _P, _P, _P, _P],
    "di_graph_destroy": [_P],
    "di_graph_info": [_P, _P, _P, _P],
    "di_window_layout": [ctypes.c_int64, ctypes.POINTER(Tune), _P, _P],
    "di_set_taken_list": [ctypes.c_int32],
    "di_set_persist_wait": [ctypes.c_double],
    "di_solve": [_P, _P, ctypes.POINTER(Opts), _P, ctypes.POINTER(Stats), _P],
    "di_power_solve": [_P, _P, ctypes.POINTER(Opts), _P, ctypes.POINTER(Stats), _P],
    "di_power_solve_noalloc": [_P, _P, ctypes.POINTER(Opts), _P, ctypes.POINTER(Stats), _P],
    "di_diffuse_round": [_P, ctypes.c_int32, ctypes.c_double, ctypes.c_double, _P, _P, _P, _P, _P],
    "di_solve_batch": [_P, ctypes.c_int32, _P, _P, _P, ctypes.POINTER(Opts), _P, _P, _P],
    "di_solve_batch_topk": [_P, ctypes.c_int32, _P, _P, _P, ctypes.POINTER(Opts), ctypes.c_int32,
                            _P, _P, _P, _P],
    "di_inject_update": [_P, _P, ctypes.c_int32, ctypes.c_double, _P, _P, _P],
    "di_autotune": [_P, ctypes.c_int32, ctypes.POINTER(Opts), ctypes.c_int32, _P, _P,
                    ctypes.POINTER(Tune), _P, ctypes.c_int32, _P, _P],
    "di_server_create": [ctypes.POINTER(ServerOpts), _P],
    "di_server_add_graph": [_P, _P, _P],
    "di_server_submit": [_P, ctypes.c_int32, ctypes.c_int32, _P, _P, ctypes.c_double,
                         ctypes.c_double, _P],
    "di_server_poll": [_P, ctypes.c_uint64, ctypes.POINTER(Result)],
    "di_server_wait": [_P, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(Result)],
    "di_server_cancel": [_P, ctypes.c_uint64],
    "di_server_stats": [_P, ctypes.POINTER(ServerMetrics)],
    "di_server_destroy": [_P],
}
for _name, _args in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_lib.di_last_error.restype = ctypes.c_char_p
_lib.di_last_error.argtypes = []
_lib.di_version.restype = ctypes.c_char_p
_lib.di_version.argtypes = []

EXPORTED = sorted(list(_SIGS) + ["di_last_error", "di_version"])


def last_error() -> str:
    return _lib.di_last_error().decode()


def version() -> str:
    return _lib.di_version().decode()


def set_taken_list(enable: bool):
    """di_set_taken_list: diagnostic, process-wide; False forces the round
    kernel's fallback of passes over consecutive nodes."""
    _check(_lib.di_set_taken_list(1 if enable else 0))


def set_persist_wait(seconds: float):
    """di_set_persist_wait: diagnostic, process-wide; the longest grid-barrier
    wait of the one-launch solve before it ends with DI_EDEVICE."""
    _check(_lib.di_set_persist_wait(float(seconds)))


def window_layout(n: int, tune=None):
    """di_window_layout: (window_log2, global_tables) that solves on an
    n-node graph get under the given knobs (host only)."""
    k = ctypes.c_int32()
    gt = ctypes.c_int32()
    _check(_lib.di_window_layout(int(n), ctypes.byref(tune) if tune is not None else None,
                                 ctypes.byref(k), ctypes.byref(gt)))
    return k.value, bool(gt.value)


def _check(rc: int, allow=()):
    if rc != OK and rc not in allow:
        raise DiError(rc, last_error())
    return rc


def _torch():
    import torch
    return torch


def _stream(stream):
    """hipStream_t for a torch stream, a raw handle, or None (torch's current stream)."""
    if stream is not None:
        return ctypes.c_void_p(int(getattr(stream, "cuda_stream", stream)))
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return ctypes.c_void_p(a.ctypes.data)
    return ctypes.c_void_p(a.data_ptr())


def _check_device_tensor(t, name, dtype, numel):
    """Raise ValueError unless t is a contiguous CUDA tensor of the given
    dtype and element count (checked before any library call, so a wrong
    tensor never reaches a kernel)."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise ValueError("%s must be a torch tensor (got %s)" % (name, type(t).__name__))
    if not t.is_cuda:
        raise ValueError("%s must be a CUDA tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s must have dtype %s (got %s)" % (name, dtype, t.dtype))
    if t.numel() != numel:
        raise ValueError("%s must have %d elements (got %d)" % (name, numel, t.numel()))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


def _check_host_array(a, name, numel):
    """Raise ValueError unless a is a C-contiguous float64 numpy array of numel
    elements."""
    if not isinstance(a, np.ndarray):
        raise ValueError("%s must be a numpy array with host=True" % name)
    if a.dtype != np.float64 or a.size != numel or not a.flags["C_CONTIGUOUS"]:
        raise ValueError("%s must be a C-contiguous float64 array of %d elements" % (name, numel))


def _fluid_dtype(precision):
    torch = _torch()
    return torch.float64 if PRECISION[precision] == FP64 else torch.float32


TABLES = {"auto": 0, "lds": 1, "global": 2}


def make_tune(schedule="mean", c=1.0, window_log2=0, check_every=0, threads=0,
              tables="auto", persist=False) -> Tune:
    return Tune(SCHEDULE.get(schedule, schedule), float(c), int(window_log2), int(check_every),
                int(threads), TABLES.get(tables, tables), int(persist))


def make_opts(d=0.85, tol=1e-8, precision="fp32", normalize=True, max_rounds=0, tune=None,
              flags=0) -> Opts:
    o = Opts()
    o.d = float(d)
    o.tol = float(tol)
    o.precision = PRECISION[precision]
    o.normalize = 1 if normalize else 0
    o.max_rounds = int(max_rounds)
    o.tune = ctypes.pointer(tune) if tune is not None else None
    o.flags = int(flags)
    return o


class Graph:
    """A device-resident graph (di_graph_create).  `g` is any object with n,
    row_ptr (int64[n+1]) and col_idx (int32[nnz]); w optional (double[nnz])."""

    def __init__(self, g=None, *, n=None, row_ptr=None, col_idx=None, w=None, stream=None):
        if g is not None:
            n, row_ptr, col_idx = g.n, g.row_ptr, g.col_idx
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
        self.w = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        self.n = int(n)
        self.nnz = int(self.row_ptr[-1]) if len(self.row_ptr) else 0
        self._h = ctypes.c_void_p()
        st = _stream(stream) if stream is not None else None
        _check(_lib.di_graph_create(self.n, len(self.col_idx), _ptr(self.row_ptr),
                                    _ptr(self.col_idx) if len(self.col_idx) else None,
                                    _ptr(self.w), st, ctypes.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def info(self):
        n, m, dg = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(_lib.di_graph_info(self._h, ctypes.byref(n), ctypes.byref(m), ctypes.byref(dg)))
        return {"n": n.value, "nnz": m.value, "dangling": dg.value}

    def close(self):
        if self._h:
            _check(_lib.di_graph_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            if self._h:
                _lib.di_graph_destroy(self._h)
        except Exception:
            pass


def _device_vec(v, n):
    """torch float64 device tensor for v (or None)."""
    if v is None:
        return None
    torch = _torch()
    if isinstance(v, np.ndarray):
        if v.size != n:
            raise ValueError("v must have %d elements (got %d)" % (n, v.size))
        v = torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).cuda()
    _check_device_tensor(v, "v", torch.float64, n)
    return v


def _host_vec(v, n):
    """Contiguous float64 host array for v (or None)."""
    if v is None:
        return None
    v = np.ascontiguousarray(v, dtype=np.float64)
    if v.shape != (n,):
        raise ValueError("v must have shape (%d,) (got %s)" % (n, v.shape))
    return v


def solve(graph: Graph, v=None, d=0.85, tol=1e-8, precision="fp32", normalize=True,
          max_rounds=0, tune=None, out=None, state=None, stream=None, allow_notconv=False,
          timing=False, trace=None, host=False):
    """D-iteration solve on the device.  v: None (uniform), numpy or torch cuda
    float64[n].  Returns (x: torch cuda float64[n], stats dict).  With
    state=(F, H) (torch cuda tensors, F float32/float64 per precision, H
    float64) the solve resumes from and updates that state.  trace: a zeroed
    torch cuda uint8[rounds, n] tensor that receives the set each round takes.
    host=True passes v and x as host arrays (the library copies them over the
    bus) and returns x as a numpy array."""
    torch = _torch()
    n = graph.n
    if precision not in PRECISION:
        raise ValueError("unknown precision %r" % (precision,))
    if state is not None:
        if len(state) != 2:
            raise ValueError("state must be a pair (F, H)")
        _check_device_tensor(state[0], "state F", _fluid_dtype(precision), n)
        _check_device_tensor(state[1], "state H", torch.float64, n)
    if trace is not None:
        if trace.dim() != 2:
            raise ValueError("trace must be a 2-d tensor [rounds, n]")
        _check_device_tensor(trace, "trace", torch.uint8, trace.shape[0] * n)
    if out is not None:
        if host:
            _check_host_array(out, "out", n)
        else:
            _check_device_tensor(out, "out", torch.float64, n)
    if host:
        x = out if out is not None else np.empty(n, dtype=np.float64)
        vd = _host_vec(v, n)
    else:
        x = out if out is not None else torch.empty(n, dtype=torch.float64, device="cuda")
        vd = _device_vec(v, n)
    flags = (0 if host else DEVICE_PTRS) | (TIMING if timing else 0)
    o = make_opts(d, tol, precision, normalize, max_rounds, tune, flags)
    if state is not None:
        o.flags |= RESUME
        o.state_f = state[0].data_ptr()
        o.state_h = state[1].data_ptr()
    if trace is not None:
        o.flags |= TRACE
        o.trace_sets = trace.data_ptr()
        o.trace_rounds = trace.shape[0]
    st = Stats()
    rc = _lib.di_solve(graph.handle, _ptr(vd), ctypes.byref(o), _ptr(x), ctypes.byref(st),
                       _stream(stream))
    _check(rc, allow=(ENOTCONV,) if allow_notconv else ())
    s = st.as_dict()
    s["status"] = rc
    return x, s


def power_solve(graph: Graph, v=None, d=0.85, tol=1e-8, precision="fp64", normalize=True,
                max_rounds=0, out=None, stream=None, allow_notconv=False, timing=False,
                host=False):
    """Power-iteration comparator (pull SpMV) on the device; host as in solve."""
    torch = _torch()
    n = graph.n
    if precision not in PRECISION:
        raise ValueError("unknown precision %r" % (precision,))
    if out is not None:
        if host:
            _check_host_array(out, "out", n)
        else:
            _check_device_tensor(out, "out", torch.float64, n)
    if host:
        x = out if out is not None else np.empty(n, dtype=np.float64)
        vd = _host_vec(v, n)
    else:
        x = out if out is not None else torch.empty(n, dtype=torch.float64, device="cuda")
        vd = _device_vec(v, n)
    o = make_opts(d, tol, precision, normalize, max_rounds, None,
                  (0 if host else DEVICE_PTRS) | (TIMING if timing else 0))
    st = Stats()
    rc = _lib.di_power_solve(graph.handle, _ptr(vd), ctypes.byref(o), _ptr(x), ctypes.byref(st),
                             _stream(stream))
    _check(rc, allow=(ENOTCONV,) if allow_notconv else ())
    s = st.as_dict()
    s["status"] = rc
    return x, s


def power_solve_noalloc(graph: Graph, out, v=None, d=0.85, tol=1e-8, precision="fp64",
                        normalize=True, max_rounds=0, stream=None, allow_notconv=False):
    """di_power_solve_noalloc: the power iteration on the library's fixed device
    scratch (no allocation inside the call).  out (and v, if given) are torch
    cuda tensors of n float64; returns (out, stats dict)."""
    torch = _torch()
    n = graph.n
    if precision not in PRECISION:
        raise ValueError("unknown precision %r" % (precision,))
    _check_device_tensor(out, "out", torch.float64, n)
    if v is not None:
        _check_device_tensor(v, "v", torch.float64, n)
    o = make_opts(d, tol, precision, normalize, max_rounds, None, DEVICE_PTRS)
    st = Stats()
    rc = _lib.di_power_solve_noalloc(graph.handle, _ptr(v), ctypes.byref(o), _ptr(out),
                                     ctypes.byref(st), _stream(stream))
    _check(rc, allow=(ENOTCONV,) if allow_notconv else ())
    s = st.as_dict()
    s["status"] = rc
    return out, s


def diffuse_round(graph: Graph, F, H, theta: float, d=0.85, stream=None):
    """One threshold round in place on device tensors F (float32 or float64)
    and H (float64).  Returns (taken_nodes, taken_edges)."""
    torch = _torch()
    if not isinstance(F, torch.Tensor) or F.dtype not in (torch.float32, torch.float64):
        raise ValueError("F must be a float32 or float64 torch tensor")
    prec = FP64 if F.dtype == torch.float64 else FP32_FLUID
    _check_device_tensor(F, "F", F.dtype, graph.n)
    _check_device_tensor(H, "H", torch.float64, graph.n)
    tn, te = ctypes.c_int64(), ctypes.c_int64()
    _check(_lib.di_diffuse_round(graph.handle, prec, float(d), float(theta), _ptr(F), _ptr(H),
                                 ctypes.byref(tn), ctypes.byref(te), _stream(stream)))
    return tn.value, te.value


def solve_batch(graph: Graph, seed_ptr, seeds, seed_w=None, d=0.85, tol=1e-6, precision="fp32",
                normalize=True, max_rounds=0, tune=None, out=None, stream=None,
                allow_notconv=False, host=False):
    """Batched personalised PageRank.  seed_ptr int64[B+1], seeds int32, seed_w
    float64 or None (host arrays).  Returns (x: torch cuda float64[B, n],
    list of per-vector stats dicts); host=True returns x as a numpy array
    (the library copies each group of vectors back)."""
    torch = _torch()
    seed_ptr = np.ascontiguousarray(seed_ptr, dtype=np.int64)
    seeds = np.ascontiguousarray(seeds, dtype=np.int32)
    sw = None if seed_w is None else np.ascontiguousarray(seed_w, dtype=np.float64)
    B = len(seed_ptr) - 1
    if precision not in PRECISION:
        raise ValueError("unknown precision %r" % (precision,))
    if out is not None:
        if host:
            _check_host_array(out, "out", B * graph.n)
        else:
            _check_device_tensor(out, "out", torch.float64, B * graph.n)
    if host:
        x = out if out is not None else np.empty((B, graph.n), dtype=np.float64)
    else:
        x = out if out is not None else torch.empty((B, graph.n), dtype=torch.float64,
                                                    device="cuda")
    o = make_opts(d, tol, precision, normalize, max_rounds, tune, 0 if host else DEVICE_PTRS)
    st = (Stats * max(B, 1))()
    rc = _lib.di_solve_batch(graph.handle, B, _ptr(seed_ptr), _ptr(seeds), _ptr(sw),
                             ctypes.byref(o), _ptr(x), st, _stream(stream))
    _check(rc, allow=(ENOTCONV,) if allow_notconv else ())
    return x, [st[b].as_dict() for b in range(B)]


def solve_batch_topk(graph: Graph, seed_ptr, seeds, k=100, seed_w=None, d=0.85, tol=1e-6,
                     precision="fp32", normalize=True, max_rounds=0, tune=None, stream=None,
                     allow_notconv=False):
    """Batched personalised PageRank keeping the k largest entries of each
    vector.  Returns (ids int32[B, k] with -1 padding, x float64[B, k], list of
    per-vector stats dicts) as numpy arrays."""
    seed_ptr = np.ascontiguousarray(seed_ptr, dtype=np.int64)
    seeds = np.ascontiguousarray(seeds, dtype=np.int32)
    sw = None if seed_w is None else np.ascontiguousarray(seed_w, dtype=np.float64)
    B = len(seed_ptr) - 1
    ids = np.empty((max(B, 0), k), dtype=np.int32)
    vals = np.empty((max(B, 0), k), dtype=np.float64)
    o = make_opts(d, tol, precision, normalize, max_rounds, tune, 0)
    st = (Stats * max(B, 1))()
    rc = _lib.di_solve_batch_topk(graph.handle, B, _ptr(seed_ptr), _ptr(seeds), _ptr(sw),
                                  ctypes.byref(o), int(k), _ptr(ids), _ptr(vals), st,
                                  _stream(stream))
    _check(rc, allow=(ENOTCONV,) if allow_notconv else ())
    return ids, vals, [st[b].as_dict() for b in range(B)]


def inject_update(old: Graph, new: Graph, F, H, d=0.85, stream=None):
    """di_inject_update: F += d (P_new - P_old) H on torch cuda tensors (F
    float32 or float64, H float64), in place."""
    torch = _torch()
    if old.n != new.n:
        raise ValueError("the two graphs must have the same number of nodes")
    if not isinstance(F, torch.Tensor) or F.dtype not in (torch.float32, torch.float64):
        raise ValueError("F must be a float32 or float64 torch tensor")
    prec = "fp64" if F.dtype == torch.float64 else "fp32"
    _check_device_tensor(F, "F", F.dtype, new.n)
    _check_device_tensor(H, "H", torch.float64, new.n)
    _check(_lib.di_inject_update(old.handle, new.handle, PRECISION[prec], float(d), _ptr(F),
                                 _ptr(H), _stream(stream)))


TUNE_SOLVE = 0
TUNE_BATCH = 1
_SCHED_NAME = {v: k for k, v in SCHEDULE.items()}


def tune_dict(t: Tune) -> dict:
    return {"schedule": _SCHED_NAME.get(t.schedule, t.schedule), "c": float(t.c),
            "window_log2": int(t.window_log2), "check_every": int(t.check_every),
            "threads": int(t.threads),
            "tables": {v: k for k, v in TABLES.items()}.get(int(t.tables), int(t.tables)),
            "persist": bool(t.persist)}


def autotune(graph: Graph, mode="solve", d=0.85, tol=1e-8, precision="fp32", seed_ptr=None,
             seeds=None, max_rounds=0, stream=None):
    """di_autotune: times trial solves (mode "solve": uniform V; "batch": the
    given seed sets) and caches the fastest knobs in the graph.  Returns
    (best Tune, list of trial dicts)."""
    m = {"solve": TUNE_SOLVE, "batch": TUNE_BATCH}[mode]
    o = make_opts(d, tol, precision, True, max_rounds, None, 0)
    B = 0
    if m == TUNE_BATCH:
        seed_ptr = np.ascontiguousarray(seed_ptr, dtype=np.int64)
        seeds = np.ascontiguousarray(seeds, dtype=np.int32)
        B = len(seed_ptr) - 1
    best = Tune()
    cap = 160  # more than the tuner runs on any graph
    trials = (TuneTrial * cap)()
    nt = ctypes.c_int32()
    _check(_lib.di_autotune(graph.handle, m, ctypes.byref(o), B, _ptr(seed_ptr), _ptr(seeds),
                            ctypes.byref(best), trials, cap, ctypes.byref(nt), _stream(stream)))
    out = [dict(tune_dict(trials[k].tune), seconds=trials[k].seconds, status=trials[k].status)
           for k in range(min(nt.value, cap))]
    return best, out


class Server:
    """Continuous-batching personalised PageRank server (di_server_*)."""

    def __init__(self, hbm_budget_bytes=0, max_slots=0, topk=0, precision="fp32", tune=None):
        o = ServerOpts()
        o.hbm_budget_bytes = int(hbm_budget_bytes)
        o.max_slots = int(max_slots)
        o.topk = int(topk)
        o.precision = PRECISION[precision]
        self._tune = tune
        o.tune = ctypes.pointer(tune) if tune is not None else None
        self._h = ctypes.c_void_p()
        _check(_lib.di_server_create(ctypes.byref(o), ctypes.byref(self._h)))
        self._graphs = []

    def add_graph(self, graph: Graph) -> int:
        gid = ctypes.c_int32()
        _check(_lib.di_server_add_graph(self._h, graph.handle, ctypes.byref(gid)))
        self._graphs.append(graph)
        return gid.value

    def submit(self, graph_id: int, seeds, w=None, d=0.85, tol=1e-6) -> int:
        seeds = np.ascontiguousarray(seeds, dtype=np.int32)
        w = None if w is None else np.ascontiguousarray(w, dtype=np.float64)
        rid = ctypes.c_uint64()
        _check(_lib.di_server_submit(self._h, int(graph_id), len(seeds), _ptr(seeds), _ptr(w),
                                     float(d), float(tol), ctypes.byref(rid)))
        return rid.value

    def poll(self, req_id: int):
        r = Result()
        rc = _lib.di_server_poll(self._h, req_id, ctypes.byref(r))
        if rc == EAGAIN:
            return None
        _check(rc)
        return r.as_dict()

    def wait(self, req_id: int, timeout_s: float = -1.0):
        r = Result()
        rc = _lib.di_server_wait(self._h, req_id, float(timeout_s), ctypes.byref(r))
        if rc == EAGAIN:
            return None
        _check(rc)
        return r.as_dict()

    def cancel(self, req_id: int):
        _check(_lib.di_server_cancel(self._h, req_id))

    def stats(self):
        m = ServerMetrics()
        _check(_lib.di_server_stats(self._h, ctypes.byref(m)))
        return m.as_dict()

    def close(self):
        if self._h:
            _check(_lib.di_server_destroy(self._h))
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
