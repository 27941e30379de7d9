"""ctypes binding of the C ABI in include/rd.h (argument marshalling only).

Every computation runs in the HIP library ``librd.so``; this module converts
Python arguments to pointers and sizes and raises on error codes. Arrays may
be numpy arrays (host memory) or torch CUDA tensors (device memory, passed
with RD_DEVICE_PTRS). If the library is missing the import of a function
fails with an error: there is no fallback implementation.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librd.so")

RD_OK = 0
RD_E_ARG = 1
RD_E_NOT_CONNECTED = 2
RD_E_OOM = 3
RD_E_DEVICE = 4
RD_E_NOT_CONVERGED = 5
RD_E_BREAKDOWN = 6

RD_DEVICE_PTRS = 0x1
RD_PROFILE = 0x2
RD_GENERAL_PATH = 0x4
RD_REORDER = 0x8
RD_NO_COMPACT = 0x10
RD_NO_SPARSE2 = 0x20
RD_F64 = 0
RD_F32 = 1

EXPORTED = [
    "rd_default_options", "rd_init_graph", "rd_set_weights", "rd_graph_info", "rd_query",
    "rd_query_trace", "rd_query_batch", "rd_grad_edges", "rd_free_graph", "rd_status_string",
    "rd_last_error", "rd_kernel_stats", "rd_tune_width", "rd_batch_schedule", "rd_power_method",
    "rd_potentials", "rd_ritz_bounds", "rd_lanczos_push",
]


class RdOptions(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("max_iters", ctypes.c_int32),
        ("fixed_k", ctypes.c_int32),
        ("delay", ctypes.c_int32),
        ("block_width", ctypes.c_int32),
        ("err_mode", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("refine", ctypes.c_int32),
        ("reorth", ctypes.c_int32),
        ("stream", ctypes.c_void_p),
    ]


class RdResult(ctypes.Structure):
    _fields_ = [
        ("r", ctypes.c_double),
        ("err_est", ctypes.c_double),
        ("iters", ctypes.c_int32),
        ("status", ctypes.c_int32),
    ]


RESULT_DTYPE = np.dtype([("r", "<f8"), ("err_est", "<f8"), ("iters", "<i4"), ("status", "<i4")])
assert RESULT_DTYPE.itemsize == ctypes.sizeof(RdResult) == 24


class RdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


_lib = None


def load(path: str = LIB_PATH):
    """Load librd.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint32
    P = ctypes.POINTER
    lib.rd_default_options.argtypes = [P(RdOptions)]
    lib.rd_default_options.restype = None
    lib.rd_init_graph.argtypes = [i32, i64, vp, vp, vp, i32, u32, P(vp)]
    lib.rd_set_weights.argtypes = [vp, vp, i32, u32]
    lib.rd_graph_info.argtypes = [vp, P(i32), P(i64), P(i64)]
    lib.rd_query.argtypes = [vp, i32, i32, dbl, P(RdOptions), P(RdResult)]
    lib.rd_query_trace.argtypes = [vp, i32, i32, i32, P(RdOptions), vp, vp, vp, P(i32)]
    lib.rd_query_batch.argtypes = [vp, i32, vp, vp, dbl, P(RdOptions), vp]
    lib.rd_grad_edges.argtypes = [vp, i32, vp, vp, vp, dbl, P(RdOptions), vp, vp]
    lib.rd_power_method.argtypes = [vp, i32, vp, vp, i32, P(RdOptions), vp]
    lib.rd_potentials.argtypes = [vp, i32, vp, vp, dbl, P(RdOptions), vp, vp]
    lib.rd_ritz_bounds.argtypes = [vp, i32, i32, i32, P(RdOptions), P(dbl), P(dbl), P(i32)]
    lib.rd_lanczos_push.argtypes = [vp, i32, vp, vp, i32, dbl, P(RdOptions), vp]
    for f in (lib.rd_init_graph, lib.rd_set_weights, lib.rd_graph_info, lib.rd_query,
              lib.rd_query_trace, lib.rd_query_batch, lib.rd_grad_edges, lib.rd_power_method,
              lib.rd_potentials, lib.rd_ritz_bounds, lib.rd_lanczos_push):
        f.restype = ctypes.c_int
    lib.rd_tune_width.argtypes = [vp, i32, i32, vp, P(i32)]
    lib.rd_tune_width.restype = ctypes.c_int
    lib.rd_batch_schedule.argtypes = [vp, P(i32), P(i32)]
    lib.rd_batch_schedule.restype = ctypes.c_int
    lib.rd_kernel_stats.argtypes = [vp, i32, P(dbl), P(i64), P(dbl)]
    lib.rd_kernel_stats.restype = ctypes.c_int
    lib.rd_free_graph.argtypes = [vp]
    lib.rd_free_graph.restype = None
    lib.rd_status_string.argtypes = [ctypes.c_int]
    lib.rd_status_string.restype = ctypes.c_char_p
    lib.rd_last_error.argtypes = [vp]
    lib.rd_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def rd_status_string(code: int) -> str:
    return load().rd_status_string(code).decode()


def rd_default_options(**kw) -> RdOptions:
    o = RdOptions()
    load().rd_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _ptr(x, dtype, count: Optional[int] = None):
    """(pointer, is_device, keepalive) for a numpy array or torch tensor."""
    if x is None:
        return None, False, None
    if _is_torch(x):
        import torch
        want = {np.int32: torch.int32, np.float64: torch.float64, np.float32: torch.float32}[dtype]
        if x.dtype != want or not x.is_contiguous():
            raise TypeError(f"tensor must be contiguous {want}")
        if count is not None and x.numel() != count:
            raise ValueError(f"expected {count} elements, got {x.numel()}")
        return x.data_ptr(), x.is_cuda, x
    a = np.ascontiguousarray(x, dtype=dtype)
    if count is not None and a.size != count:
        raise ValueError(f"expected {count} elements, got {a.size}")
    return a.ctypes.data, False, a


def _stream_of(opts: Optional[RdOptions], device: bool = False) -> RdOptions:
    o = opts if opts is not None else rd_default_options()
    if device:
        o = RdOptions.from_buffer_copy(o)
        o.flags |= RD_DEVICE_PTRS
    return o


class RDGraph:
    """Owning wrapper of an rd_graph handle."""

    def __init__(self, n: int, u, v, w=None, reorder: bool = False):
        """reorder: number the nodes internally by decreasing degree (RD_REORDER);
        node ids, pair lists and edge order seen by the caller do not change."""
        lib = load()
        m = int(len(u))
        pu, du, ku = _ptr(u, np.int32, m)
        pv, dv, kv = _ptr(v, np.int32, m)
        wdt = RD_F64
        pw = None
        dw = du
        kw_ = None
        if w is not None:
            is32 = (str(getattr(w, "dtype", "")).endswith("float32"))
            wdt = RD_F32 if is32 else RD_F64
            pw, dw, kw_ = _ptr(w, np.float32 if is32 else np.float64, m)
        if not (du == dv == dw):
            raise ValueError("edge arrays and weights must all be host or all be device memory")
        flags = (RD_DEVICE_PTRS if du else 0) | (RD_REORDER if reorder else 0)
        h = ctypes.c_void_p()
        rc = lib.rd_init_graph(int(n), m, pu, pv, pw, wdt, flags, ctypes.byref(h))
        if rc != RD_OK:
            msg = lib.rd_last_error(None).decode()
            raise RdError(rc, f"rd_init_graph: {rd_status_string(rc)}: {msg}")
        self._h = h
        self.n = int(n)
        self.m = m
        del ku, kv, kw_

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            load().rd_free_graph(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _raise(self, rc: int, what: str):
        msg = load().rd_last_error(self._h).decode()
        raise RdError(rc, f"{what}: {rd_status_string(rc)}: {msg}")

    def info(self):
        n, m, nnz = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        rc = load().rd_graph_info(self._h, ctypes.byref(n), ctypes.byref(m), ctypes.byref(nnz))
        if rc != RD_OK:
            self._raise(rc, "rd_graph_info")
        return n.value, m.value, nnz.value

    def tune_width(self, precision: int, npairs: int, stream=None) -> int:
        w = ctypes.c_int32()
        rc = load().rd_tune_width(self._h, int(precision), int(npairs), stream, ctypes.byref(w))
        if rc != RD_OK:
            self._raise(rc, "rd_tune_width")
        return w.value

    def batch_schedule(self):
        """(entries per wavefront work item, long-row threshold) of the
        batched product's row-bin schedule currently in effect."""
        wv, ld = ctypes.c_int32(), ctypes.c_int32()
        rc = load().rd_batch_schedule(self._h, ctypes.byref(wv), ctypes.byref(ld))
        if rc != RD_OK:
            self._raise(rc, "rd_batch_schedule")
        return wv.value, ld.value

    def kernel_stats(self, which: int):
        """(total ms, launches, algorithmic bytes per launch) of the sparse
        product launches timed under RD_PROFILE since the last call.
        which = 0: batched short-row product; 1: single-pair product;
        2: edge pass of grad_edges."""
        ms, n, b = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        rc = load().rd_kernel_stats(self._h, int(which), ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b))
        if rc != RD_OK:
            self._raise(rc, "rd_kernel_stats")
        return ms.value, n.value, b.value

    def set_weights(self, w):
        is32 = str(getattr(w, "dtype", "")).endswith("float32")
        p, dev, keep = _ptr(w, np.float32 if is32 else np.float64, self.m)
        rc = load().rd_set_weights(self._h, p, RD_F32 if is32 else RD_F64, RD_DEVICE_PTRS if dev else 0)
        if rc != RD_OK:
            self._raise(rc, "rd_set_weights")

    def query(self, s: int, t: int, eps: float = 1e-6, opts: Optional[RdOptions] = None) -> RdResult:
        res = RdResult()
        rc = load().rd_query(self._h, int(s), int(t), float(eps), ctypes.byref(_stream_of(opts)),
                             ctypes.byref(res))
        if rc != RD_OK:
            self._raise(rc, "rd_query")
        return res

    def query_trace(self, s: int, t: int, k: int, opts: Optional[RdOptions] = None):
        a = np.zeros(k)
        b = np.zeros(k)
        r = np.zeros(k)
        it = ctypes.c_int32()
        rc = load().rd_query_trace(self._h, int(s), int(t), int(k), ctypes.byref(_stream_of(opts)),
                                   a.ctypes.data, b.ctypes.data, r.ctypes.data, ctypes.byref(it))
        if rc != RD_OK:
            self._raise(rc, "rd_query_trace")
        i = it.value
        return a[:i], b[:i], r[:i]

    def query_batch(self, s, t, eps: float = 1e-4, opts: Optional[RdOptions] = None, out=None):
        """Host arrays -> numpy structured array of results; device tensors ->
        results written to `out` (a torch uint8 CUDA tensor of 24*npairs bytes)."""
        npairs = int(len(s))
        ps, ds, ks = _ptr(s, np.int32, npairs)
        pt, dt, kt = _ptr(t, np.int32, npairs)
        if ds != dt:
            raise ValueError("s and t must both be host or both be device memory")
        if ds:
            if out is None:
                raise ValueError("device pair lists need a device `out` buffer")
            pout = out.data_ptr()
            res = out
        else:
            res = np.zeros(npairs, dtype=RESULT_DTYPE)
            pout = res.ctypes.data
        rc = load().rd_query_batch(self._h, npairs, ps, pt, float(eps),
                                   ctypes.byref(_stream_of(opts, ds)), pout)
        if rc != RD_OK:
            self._raise(rc, "rd_query_batch")
        del ks, kt
        return res

    def power_method(self, s, t, l: int, opts: Optional[RdOptions] = None, out=None):
        """Power Method (Algorithm 1) with l products per pair. Host arrays ->
        numpy structured array of results; device tensors -> results written
        to `out` (a torch uint8 CUDA tensor of 24*npairs bytes)."""
        npairs = int(len(s))
        ps, ds, ks = _ptr(s, np.int32, npairs)
        pt, dt, kt = _ptr(t, np.int32, npairs)
        if ds != dt:
            raise ValueError("s and t must both be host or both be device memory")
        if ds:
            if out is None:
                raise ValueError("device pair lists need a device `out` buffer")
            pout = out.data_ptr()
            res = out
        else:
            res = np.zeros(npairs, dtype=RESULT_DTYPE)
            pout = res.ctypes.data
        rc = load().rd_power_method(self._h, npairs, ps, pt, int(l),
                                    ctypes.byref(_stream_of(opts, ds)), pout)
        if rc != RD_OK:
            self._raise(rc, "rd_power_method")
        del ks, kt
        return res

    def lanczos_push(self, s, t, k: int, eps: float, opts: Optional[RdOptions] = None):
        """Lanczos Push (Algorithm 4) for host pair arrays: numpy results."""
        npairs = int(len(s))
        ps, ds, ks = _ptr(s, np.int32, npairs)
        pt, dt, kt = _ptr(t, np.int32, npairs)
        if ds or dt:
            raise ValueError("lanczos_push() takes host pair lists")
        res = np.zeros(npairs, dtype=RESULT_DTYPE)
        rc = load().rd_lanczos_push(self._h, npairs, ps, pt, int(k), float(eps),
                                    ctypes.byref(_stream_of(opts, False)), res.ctypes.data)
        if rc != RD_OK:
            self._raise(rc, "rd_lanczos_push")
        del ks, kt
        return res

    def ritz_bounds(self, s: int, t: int, k: int, opts: Optional[RdOptions] = None):
        """(theta_min, theta_max, iters) of a k-step Lanczos run from the pair's
        start vector; kappa_hat = 2 / (1 - theta_max)."""
        lo, hi, it = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
        o = opts if opts is not None else rd_default_options()
        rc = load().rd_ritz_bounds(self._h, int(s), int(t), int(k), ctypes.byref(o), ctypes.byref(lo),
                                   ctypes.byref(hi), ctypes.byref(it))
        if rc != RD_OK:
            self._raise(rc, "rd_ritz_bounds")
        return lo.value, hi.value, it.value

    def potentials(self, s, t, eps: float = 1e-6, opts: Optional[RdOptions] = None, out=None, phi=None):
        """Electric potentials of the pairs: (results, phi) with phi float64
        [npairs, n] in the caller's node order, mean zero. Host arrays -> numpy
        outputs; device tensors -> results into `out` (torch uint8, 24*npairs
        bytes) and potentials into `phi` (torch float64 [npairs, n])."""
        npairs = int(len(s))
        ps, ds, ks = _ptr(s, np.int32, npairs)
        pt, dt, kt = _ptr(t, np.int32, npairs)
        if ds != dt:
            raise ValueError("s and t must both be host or both be device memory")
        if ds:
            if out is None or phi is None:
                raise ValueError("device pair lists need device `out` and `phi` buffers")
            if tuple(phi.shape) != (npairs, self.n) or phi.dtype != __import__("torch").float64:
                raise ValueError("phi must be a float64 tensor of shape [npairs, n]")
            res, pout, pphi = out, out.data_ptr(), phi.data_ptr()
        else:
            res = np.zeros(npairs, dtype=RESULT_DTYPE)
            phi = np.zeros((npairs, self.n), dtype=np.float64)
            pout, pphi = res.ctypes.data, phi.ctypes.data
        rc = load().rd_potentials(self._h, npairs, ps, pt, float(eps), ctypes.byref(_stream_of(opts, ds)),
                                  pout, pphi)
        if rc != RD_OK:
            self._raise(rc, "rd_potentials")
        del ks, kt
        return res, phi

    def grad_edges(self, s, t, grad_r=None, eps: float = 1e-6, opts: Optional[RdOptions] = None,
                   fwd=None, grad_w=None):
        """Host arrays -> (fwd results, grad_w float32[m]) as numpy; device
        tensors -> written into the given device `fwd` / `grad_w` tensors."""
        npairs = int(len(s))
        ps, ds, ks = _ptr(s, np.int32, npairs)
        pt, dt, kt = _ptr(t, np.int32, npairs)
        pg, dg, kg = _ptr(grad_r, np.float64, npairs)
        if ds:
            if grad_w is None:
                raise ValueError("device pair lists need a device grad_w tensor")
            pgw = grad_w.data_ptr()
            pf = fwd.data_ptr() if fwd is not None else None
            outs = (fwd, grad_w)
        else:
            gw = np.zeros(self.m, dtype=np.float32)
            fw = np.zeros(npairs, dtype=RESULT_DTYPE)
            pgw, pf = gw.ctypes.data, fw.ctypes.data
            outs = (fw, gw)
        rc = load().rd_grad_edges(self._h, npairs, ps, pt, pg, float(eps),
                                  ctypes.byref(_stream_of(opts, ds)), pf, pgw)
        if rc != RD_OK:
            self._raise(rc, "rd_grad_edges")
        del ks, kt, kg
        return outs
