"""Python binding of the request-serving engine (include/rcm_server.h).

Marshalling only: the engine (queue, memory admission, batching, executors)
is native code in ``librcm.so`` and every ordering runs in the library's HIP
kernels.  The binding keeps each request's host arrays alive until the
request has been collected, as the C interface requires.
"""

from __future__ import annotations

import ctypes
from typing import Dict, Optional, Tuple

import numpy as np

from . import rcm

SERVER_EXPORTED = [
    "rcm_server_default_config",
    "rcm_server_request_bytes",
    "rcm_server_create",
    "rcm_server_submit",
    "rcm_server_poll",
    "rcm_server_wait",
    "rcm_server_counters_get",
    "rcm_server_destroy",
]


class ServerConfig(ctypes.Structure):
    _fields_ = [
        ("mem_budget_bytes", ctypes.c_uint64),
        ("max_batch", ctypes.c_int32),
        ("executors", ctypes.c_int32),
        ("batch_nnz_limit", ctypes.c_int64),
        ("order_options", rcm.Options),
    ]


class RequestResult(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("batch_size", ctypes.c_int32),
        ("stats", rcm.Stats),
        ("t_submit", ctypes.c_double),
        ("t_admit", ctypes.c_double),
        ("t_done", ctypes.c_double),
    ]

    def to_dict(self) -> Dict:
        return {
            "status": int(self.status),
            "batch_size": int(self.batch_size),
            "stats": self.stats.to_dict(),
            "t_submit": self.t_submit,
            "t_admit": self.t_admit,
            "t_done": self.t_done,
            "latency_s": self.t_done - self.t_submit,
            "queue_s": self.t_admit - self.t_submit,
        }


class ServerCounters(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64),
        ("completed", ctypes.c_int64),
        ("failed", ctypes.c_int64),
        ("batches", ctypes.c_int64),
        ("retried_alone", ctypes.c_int64),
        ("max_batch_seen", ctypes.c_int64),
        ("bytes_in_flight", ctypes.c_uint64),
        ("peak_bytes_in_flight", ctypes.c_uint64),
        ("mem_budget_bytes", ctypes.c_uint64),
    ]


_configured = False


def _lib() -> ctypes.CDLL:
    global _configured
    L = rcm.lib()
    if not _configured:
        vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        L.rcm_server_default_config.argtypes = [vp]
        L.rcm_server_default_config.restype = None
        L.rcm_server_request_bytes.argtypes = [i32, i64]
        L.rcm_server_request_bytes.restype = u64
        L.rcm_server_create.argtypes = [vp, ctypes.POINTER(vp)]
        L.rcm_server_create.restype = ctypes.c_int
        L.rcm_server_submit.argtypes = [vp, i32, i64, vp, vp, vp, ctypes.POINTER(i64)]
        L.rcm_server_submit.restype = ctypes.c_int
        L.rcm_server_poll.argtypes = [vp, i64, ctypes.POINTER(i32)]
        L.rcm_server_poll.restype = ctypes.c_int
        L.rcm_server_wait.argtypes = [vp, i64, i64, vp]
        L.rcm_server_wait.restype = ctypes.c_int
        L.rcm_server_counters_get.argtypes = [vp, vp]
        L.rcm_server_counters_get.restype = ctypes.c_int
        L.rcm_server_destroy.argtypes = [vp]
        L.rcm_server_destroy.restype = None
        _configured = True
    return L


def request_bytes(n: int, nnz: int) -> int:
    """Device bytes a request reserves while in flight when it runs alone."""
    return int(_lib().rcm_server_request_bytes(int(n), int(nnz)))


class Server:
    """An ordering server on the current GPU.

    >>> srv = Server(mem_budget_bytes=1 << 30)
    >>> t = srv.submit(rowptr, colidx)          # host int32 arrays
    >>> perm, info = srv.wait(t)
    """

    def __init__(self, *, mem_budget_bytes: int = 0, max_batch: int = 0, executors: int = 0,
                 batch_nnz_limit: int = 0, **order_opts):
        L = _lib()
        cfg = ServerConfig()
        L.rcm_server_default_config(ctypes.byref(cfg))
        cfg.mem_budget_bytes = int(mem_budget_bytes)
        cfg.max_batch = int(max_batch)
        cfg.executors = int(executors)
        cfg.batch_nnz_limit = int(batch_nnz_limit)
        cfg.order_options = rcm.make_options(**order_opts)
        h = ctypes.c_void_p()
        status = L.rcm_server_create(ctypes.byref(cfg), ctypes.byref(h))
        if status != rcm.OK:
            raise rcm.RcmError(status, rcm.status_string(status))
        self._h = h
        self._cfg = cfg
        self._held: Dict[int, Tuple[np.ndarray, np.ndarray, np.ndarray]] = {}

    def submit(self, rowptr, colidx) -> int:
        """Queue one ordering of the host CSR pattern; returns a ticket."""
        rp = np.ascontiguousarray(rowptr, dtype=np.int32)
        ci = np.ascontiguousarray(colidx, dtype=np.int32)
        n = rp.size - 1
        perm = np.empty(max(n, 0), dtype=np.int32)
        t = ctypes.c_int64()
        status = _lib().rcm_server_submit(
            self._h, int(n), int(ci.size), rp.ctypes.data if rp.size else None,
            ci.ctypes.data if ci.size else None, perm.ctypes.data if perm.size else None,
            ctypes.byref(t))
        if status != rcm.OK:
            raise rcm.RcmError(status, rcm.status_string(status))
        self._held[t.value] = (rp, ci, perm)
        return t.value

    def poll(self, ticket: int) -> bool:
        done = ctypes.c_int32()
        status = _lib().rcm_server_poll(self._h, int(ticket), ctypes.byref(done))
        if status != rcm.OK:
            raise rcm.RcmError(status, rcm.status_string(status))
        return bool(done.value)

    def wait(self, ticket: int, timeout_ms: int = -1) -> Tuple[Optional[np.ndarray], Dict]:
        """Block until the request is complete; returns (perm or None on a
        failed request, result dict)."""
        res = RequestResult()
        status = _lib().rcm_server_wait(self._h, int(ticket), int(timeout_ms), ctypes.byref(res))
        if status != rcm.OK:
            raise rcm.RcmError(status, rcm.status_string(status))
        _, _, perm = self._held.pop(int(ticket))
        info = res.to_dict()
        return (perm if info["status"] == rcm.OK else None), info

    def counters(self) -> Dict[str, int]:
        c = ServerCounters()
        status = _lib().rcm_server_counters_get(self._h, ctypes.byref(c))
        if status != rcm.OK:
            raise rcm.RcmError(status, rcm.status_string(status))
        return {name: int(getattr(c, name)) for name, _ in ServerCounters._fields_}

    def close(self) -> None:
        if self._h:
            _lib().rcm_server_destroy(self._h)
            self._h = None
            self._held.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
