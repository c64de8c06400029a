"""Binding of the library's serving loop (ata_server_* in include/ata.h).

Argument marshalling only: admission, batching, launches and timing all run
in libata's scheduler thread and kernels.
"""
from __future__ import annotations

import ctypes

from . import F32, F64, AtaError, load, tri

SRC_HOST = 0
SRC_DEVICE = 1
SRC_NORMAL = 2
SERVER_SIMULATE = 1
STATE_DONE = 3
EPENDING = 8


class Request(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("dtype", ctypes.c_int32),
                ("cutoff", ctypes.c_int32), ("max_depth", ctypes.c_int32), ("src", ctypes.c_int32),
                ("a", ctypes.c_void_p), ("seed", ctypes.c_uint64), ("keep_a", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class RequestInfo(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("status", ctypes.c_int32), ("m", ctypes.c_int64),
                ("n", ctypes.c_int64), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double), ("batched", ctypes.c_int32),
                ("stream", ctypes.c_int32), ("footprint", ctypes.c_int64), ("flops", ctypes.c_double),
                ("slabs", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "admitted", "completed", "rejected", "batches",
                                              "batched_requests", "pool_bytes", "pool_in_use", "pool_peak",
                                              "queued", "active")]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


_bound = False


def _bind():
    global _bound
    lib = load()
    if _bound:
        return lib
    vp, ci, i64, u64, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    lib.ata_server_create.argtypes = [ctypes.c_size_t, ci, ci, ci, dbl, ctypes.POINTER(vp)]
    lib.ata_server_submit.argtypes = [vp, ctypes.POINTER(Request), ctypes.POINTER(u64)]
    lib.ata_server_query.argtypes = [vp, u64, ctypes.POINTER(RequestInfo)]
    lib.ata_server_wait.argtypes = [vp, u64, dbl, ctypes.POINTER(RequestInfo)]
    lib.ata_server_take.argtypes = [vp, u64, vp, vp, ci]
    lib.ata_server_release.argtypes = [vp, u64]
    lib.ata_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    lib.ata_server_now.argtypes = [vp]
    lib.ata_server_now.restype = dbl
    lib.ata_server_destroy.argtypes = [vp]
    for f in ("ata_server_create", "ata_server_submit", "ata_server_query", "ata_server_wait", "ata_server_take",
              "ata_server_release", "ata_server_get_stats", "ata_server_destroy"):
        getattr(lib, f).restype = ci
    _bound = True
    return lib


class Server:
    """Continuous-batching server for A^t A requests on the current device.

    budget_bytes: device memory pool used for admission (A + packed C +
    workspace per request); max_active: requests in flight; streams: HIP
    streams the loop spreads requests over.  simulate_tflops: host-only mode
    (no GPU) where a request takes flops / (simulate_tflops 1e12) seconds."""

    def __init__(self, budget_bytes: int, max_active: int = 64, streams: int = 4, simulate_tflops=None):
        self._lib = _bind()
        h = ctypes.c_void_p()
        flags = SERVER_SIMULATE if simulate_tflops else 0
        rc = self._lib.ata_server_create(int(budget_bytes), int(max_active), int(streams), flags,
                                         float(simulate_tflops or 0.0), ctypes.byref(h))
        if rc:
            raise AtaError(rc, "ata_server_create")
        self._h = h
        self._keep = {}    # source buffers that must outlive admission
        self._dtypes = {}  # ticket -> dtype

    def submit(self, m: int, n: int, dtype: int = F32, a=None, seed: int = 0, cutoff: int = 0, max_depth=None,
               keep_a: bool = False) -> int:
        """a: None (N(0,1) drawn on the device from `seed`), a numpy array
        (copied from host memory) or a device tensor (copied on the device),
        row-major m x n with row stride n."""
        r = Request()
        r.m, r.n, r.dtype, r.cutoff = int(m), int(n), int(dtype), int(cutoff)
        r.max_depth = -2 if max_depth is None else int(max_depth)
        r.seed, r.keep_a, r.reserved = int(seed), 1 if keep_a else 0, 0
        keep = None
        if a is None:
            r.src, r.a = SRC_NORMAL, None
        elif hasattr(a, "is_cuda") and a.is_cuda:
            if not a.is_contiguous() or tuple(a.shape) != (m, n):
                raise ValueError("device A must be contiguous m x n")
            r.src, r.a, keep = SRC_DEVICE, a.data_ptr(), a
        else:
            import numpy as np
            want = np.float64 if dtype == F64 else np.float32
            keep = np.ascontiguousarray(a, dtype=want)
            if keep.shape != (m, n):
                raise ValueError("host A must be m x n")
            r.src, r.a = SRC_HOST, keep.ctypes.data
        t = ctypes.c_uint64()
        rc = self._lib.ata_server_submit(self._h, ctypes.byref(r), ctypes.byref(t))
        if rc:
            raise AtaError(rc, "ata_server_submit")
        if keep is not None:
            self._keep[t.value] = keep
        self._dtypes[t.value] = int(dtype)
        return t.value

    def query(self, ticket: int):
        info = RequestInfo()
        rc = self._lib.ata_server_query(self._h, ticket, ctypes.byref(info))
        if rc not in (0, EPENDING):
            raise AtaError(rc, "ata_server_query")
        return rc == 0, info.as_dict()

    def wait(self, ticket: int, timeout: float = 60.0) -> dict:
        info = RequestInfo()
        rc = self._lib.ata_server_wait(self._h, ticket, float(timeout), ctypes.byref(info))
        if rc:
            raise AtaError(rc, "ata_server_wait")
        self._keep.pop(ticket, None)
        if info.status:
            raise AtaError(info.status, "request %d" % ticket)
        return info.as_dict()

    def take(self, ticket: int, want_a: bool = False, device: bool = False):
        """Copy the packed result (and A if kept) out and release the request:
        host numpy arrays, or device tensors on the current device when
        `device` is set."""
        import numpy as np
        info = self.wait(ticket)
        m, n = info["m"], info["n"]
        f64 = self._dtypes.pop(ticket, F32) == F64
        if device:
            import torch
            dt = torch.float64 if f64 else torch.float32
            c = torch.empty(tri(n), dtype=dt, device="cuda")
            a = torch.empty((m, n), dtype=dt, device="cuda") if want_a else None
            cp, ap = c.data_ptr(), (a.data_ptr() if want_a else None)
        else:
            dt = np.float64 if f64 else np.float32
            c = np.empty(tri(n), dtype=dt)
            a = np.empty((m, n), dtype=dt) if want_a else None
            cp, ap = c.ctypes.data, (a.ctypes.data if want_a else None)
        rc = self._lib.ata_server_take(self._h, ticket, cp, ap, 1 if device else 0)
        if rc:
            raise AtaError(rc, "ata_server_take")
        return (c, a) if want_a else c

    def release(self, ticket: int) -> None:
        rc = self._lib.ata_server_release(self._h, ticket)
        self._keep.pop(ticket, None)
        self._dtypes.pop(ticket, None)
        if rc:
            raise AtaError(rc, "ata_server_release")

    def stats(self) -> dict:
        s = ServerStats()
        rc = self._lib.ata_server_get_stats(self._h, ctypes.byref(s))
        if rc:
            raise AtaError(rc, "ata_server_get_stats")
        return s.as_dict()

    def now(self) -> float:
        return self._lib.ata_server_now(self._h)

    def close(self) -> None:
        if self._h:
            self._lib.ata_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
