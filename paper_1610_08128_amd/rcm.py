"""Python binding of ``librcm.so`` (the C ABI declared in include/rcm.h).

Argument marshalling only: tensors are handed to the library as raw device
pointers together with torch's current HIP stream; every step of the
ordering runs in the library's HIP kernels.  There is no fallback: if the
library is missing, the first call raises.
"""

from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence, Tuple

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "librcm.so")

STATUS = {
    0: "RCM_OK",
    1: "RCM_ERR_INVALID_ARGUMENT",
    2: "RCM_ERR_BAD_CSR",
    3: "RCM_ERR_NOT_SYMMETRIC",
    4: "RCM_ERR_WORKSPACE_TOO_SMALL",
    5: "RCM_ERR_OUT_OF_MEMORY",
    6: "RCM_ERR_ABORTED",
    7: "RCM_ERR_HIP",
}
OK, ERR_INVALID_ARGUMENT, ERR_BAD_CSR, ERR_NOT_SYMMETRIC = 0, 1, 2, 3
ERR_WORKSPACE_TOO_SMALL, ERR_OUT_OF_MEMORY, ERR_ABORTED, ERR_HIP = 4, 5, 6, 7

EXPORTED = [
    "rcm_status_string",
    "rcm_default_options",
    "rcm_workspace_bytes",
    "rcm_order",
    "rcm_order_ex",
    "rcm_batched_workspace_bytes",
    "rcm_order_batched",
    "rcm_last_timings",
    "rcm_order_noalloc",
    "rcm_tuning_options",
    "rcm_abort_flag_create",
    "rcm_abort_flag_destroy",
]

NOALLOC_SCRATCH_BYTES = 256 << 20  # RCM_NOALLOC_SCRATCH_BYTES in include/rcm.h


class RcmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


class Stats(ctypes.Structure):
    _fields_ = [
        ("bandwidth_before", ctypes.c_int64),
        ("profile_before", ctypes.c_int64),
        ("bandwidth_after", ctypes.c_int64),
        ("profile_after", ctypes.c_int64),
        ("edges_traversed", ctypes.c_int64),
        ("num_components", ctypes.c_int32),
        ("pseudo_diameter", ctypes.c_int32),
        ("num_bfs", ctypes.c_int32),
        ("num_levels", ctypes.c_int32),
    ]

    def to_dict(self) -> Dict[str, int]:
        return {f: int(getattr(self, f)) for f, _ in self._fields_}


class Options(ctypes.Structure):
    _fields_ = [
        ("pp_variant", ctypes.c_int32),
        ("reverse_mode", ctypes.c_int32),
        ("check_full", ctypes.c_int32),
        ("team_size", ctypes.c_int32),
        ("block_threads", ctypes.c_int32),
        ("small_cutoff", ctypes.c_int32),
        ("narrow_cutoff", ctypes.c_int32),
        ("small_threads", ctypes.c_int32),
        ("max_teams", ctypes.c_int32),
        ("rebalance_levels", ctypes.c_int32),
        ("label_mode", ctypes.c_int32),
        ("async_search", ctypes.c_int32),
        ("label_team", ctypes.c_int32),
        ("search_round", ctypes.c_int32),
        ("mode", ctypes.c_int32),
        ("shuffle_seed", ctypes.c_int32),
        ("tuning_file", ctypes.c_char_p),
        ("abort_flag", ctypes.c_void_p),
        ("relabel_levels", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class Timings(ctypes.Structure):
    _fields_ = [
        ("validate_ms", ctypes.c_float),
        ("components_ms", ctypes.c_float),
        ("order_ms", ctypes.c_float),
        ("after_ms", ctypes.c_float),
        ("total_ms", ctypes.c_float),
        ("small_kernel_ms", ctypes.c_float),
        ("team_kernel_ms", ctypes.c_float),
        ("team_pp_ms", ctypes.c_float),
        ("team_label_ms", ctypes.c_float),
        ("team_pp_levels", ctypes.c_int32),
        ("team_label_levels", ctypes.c_int32),
        ("used_mode", ctypes.c_int32),
        ("used_team_size", ctypes.c_int32),
        ("used_block_threads", ctypes.c_int32),
        ("used_label_team", ctypes.c_int32),
        ("used_search_round", ctypes.c_int32),
        ("used_small_cutoff", ctypes.c_int32),
        ("phase_ticks", ctypes.c_int64 * 28),
    ]


_lib = None


def lib() -> ctypes.CDLL:
    """Load librcm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1610_08128_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        L.rcm_status_string.argtypes = [ctypes.c_int]
        L.rcm_status_string.restype = ctypes.c_char_p
        L.rcm_default_options.argtypes = [ctypes.POINTER(Options)]
        L.rcm_default_options.restype = None
        L.rcm_workspace_bytes.argtypes = [i32, i64, ctypes.POINTER(Options)]
        L.rcm_workspace_bytes.restype = ctypes.c_size_t
        L.rcm_batched_workspace_bytes.argtypes = [i32, i64, i64, ctypes.POINTER(Options)]
        L.rcm_batched_workspace_bytes.restype = ctypes.c_size_t
        L.rcm_order.argtypes = [i32, P, P, P, ctypes.POINTER(Stats), P]
        L.rcm_order.restype = ctypes.c_int
        L.rcm_order_ex.argtypes = [i32, P, P, P, P, ctypes.POINTER(Stats),
                                   ctypes.POINTER(Options), P, ctypes.c_size_t, P]
        L.rcm_order_ex.restype = ctypes.c_int
        L.rcm_order_batched.argtypes = [i32, P, P, P, P, P, P, ctypes.POINTER(Options), P,
                                        ctypes.c_size_t, P]
        L.rcm_order_batched.restype = ctypes.c_int
        L.rcm_order_noalloc.argtypes = [i32, P, P, P, P, ctypes.POINTER(Stats),
                                        ctypes.POINTER(Options), P]
        L.rcm_order_noalloc.restype = ctypes.c_int
        L.rcm_tuning_options.argtypes = [ctypes.c_char_p, i32, i64, i64, ctypes.POINTER(Options)]
        L.rcm_tuning_options.restype = ctypes.c_int
        L.rcm_last_timings.argtypes = [ctypes.POINTER(Timings)]
        L.rcm_last_timings.restype = None
        L.rcm_abort_flag_create.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        L.rcm_abort_flag_create.restype = ctypes.c_int
        L.rcm_abort_flag_destroy.argtypes = [ctypes.c_void_p]
        L.rcm_abort_flag_destroy.restype = None
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().rcm_status_string(int(status)).decode()


def make_options(*, pp_variant=0, reverse_mode=0, check_full=False, team_size=0,
                 block_threads=0, small_cutoff=0, narrow_cutoff=0, small_threads=0,
                 max_teams=0, rebalance_levels=0, label_mode=0, async_search=0,
                 label_team=0, search_round=0, mode=0, tuning_file=None, shuffle_seed=0,
                 abort_flag=None, relabel_levels=0) -> Options:
    o = Options()
    o.pp_variant = int(pp_variant)
    o.reverse_mode = int(reverse_mode)
    o.check_full = int(bool(check_full))
    o.team_size = int(team_size)
    o.block_threads = int(block_threads)
    o.small_cutoff = int(small_cutoff)
    o.narrow_cutoff = int(narrow_cutoff)
    o.small_threads = int(small_threads)
    o.max_teams = int(max_teams)
    o.rebalance_levels = int(rebalance_levels)
    o.label_mode = int(label_mode)
    o.async_search = int(async_search)
    o.label_team = int(label_team)
    o.search_round = int(search_round)
    o.mode = int(mode)
    o.tuning_file = tuning_file.encode() if isinstance(tuning_file, str) else tuning_file
    o.shuffle_seed = int(shuffle_seed)
    o.relabel_levels = int(relabel_levels)
    o.abort_flag = abort_flag.address if isinstance(abort_flag, AbortFlag) else abort_flag
    return o


class AbortFlag:
    """rcm_abort_flag_create's flag: pass it as ``abort_flag=`` to a call and
    ``set()`` it, from any thread, to make that call return
    RCM_ERR_ABORTED; ``clear()`` it before the next call."""

    def __init__(self):
        p = ctypes.c_void_p()
        st = lib().rcm_abort_flag_create(ctypes.byref(p))
        if st != OK:
            raise RcmError(st, "rcm_abort_flag_create")
        self.address = p.value
        self._word = ctypes.c_int32.from_address(self.address)

    def set(self) -> None:
        self._word.value = 1

    def clear(self) -> None:
        self._word.value = 0

    @property
    def is_set(self) -> bool:
        return self._word.value != 0

    def close(self) -> None:
        if self.address:
            lib().rcm_abort_flag_destroy(self.address)
            self.address = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


TUNING_FIELDS = ("team_size", "block_threads", "small_cutoff", "narrow_cutoff", "small_threads",
                 "max_teams", "rebalance_levels", "async_search", "label_team", "search_round",
                 "mode", "relabel_levels")


def tuning_options(path: str, n: int, nnz: int, num_graphs: int = 1) -> Dict[str, int]:
    """The launch options the library takes from the tuning table at
    ``path`` for a call of this size (rcm_tuning_options); only the options
    the table sets."""
    o = Options()
    status = lib().rcm_tuning_options(path.encode(), int(num_graphs), int(n), int(nnz),
                                      ctypes.byref(o))
    if status != OK:
        raise RcmError(status, status_string(status))
    return {f: int(getattr(o, f)) for f in TUNING_FIELDS if getattr(o, f) != 0}


def workspace_bytes(n: int, nnz: int, **opts) -> int:
    return int(lib().rcm_workspace_bytes(int(n), int(nnz), ctypes.byref(make_options(**opts))))


def batched_workspace_bytes(num_graphs: int, total_vertices: int, total_nnz: int, **opts) -> int:
    return int(lib().rcm_batched_workspace_bytes(int(num_graphs), int(total_vertices),
                                                 int(total_nnz),
                                                 ctypes.byref(make_options(**opts))))


def last_timings() -> Dict[str, float]:
    t = Timings()
    lib().rcm_last_timings(ctypes.byref(t))
    out = {f: getattr(t, f) for f, _ in t._fields_}
    out["phase_ticks"] = list(t.phase_ticks)
    return out


def _stream_handle(stream) -> Optional[int]:
    import torch

    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _dev_i32(x, device):
    import numpy as np
    import torch

    if isinstance(x, torch.Tensor):
        if x.dtype != torch.int32 or not x.is_cuda or not x.is_contiguous():
            raise TypeError("expected a contiguous int32 CUDA tensor")
        return x
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.int32)).to(device)


def order_raw(n: int, rowptr_ptr: int, colidx_ptr: int, perm_ptr: int, iperm_ptr: int = 0,
              options: Optional[Options] = None, workspace_ptr: int = 0,
              workspace_size: int = 0, stream_ptr: int = 0) -> Tuple[int, Dict[str, int]]:
    """Direct call of rcm_order_ex with raw pointers (0 = NULL); returns
    (status, stats)."""
    st = Stats()
    opts = ctypes.byref(options) if options is not None else None
    status = lib().rcm_order_ex(int(n), rowptr_ptr or None, colidx_ptr or None, perm_ptr or None,
                                iperm_ptr or None, ctypes.byref(st), opts, workspace_ptr or None,
                                int(workspace_size), stream_ptr or None)
    return int(status), st.to_dict()


def order(rowptr, colidx, *, stream=None, return_iperm: bool = False, workspace=None,
          device=None, **opts):
    """Reverse Cuthill-McKee permutation of a symmetric CSR pattern.

    rowptr, colidx: int32 CUDA tensors (or arrays, copied to ``device``).
    Returns (perm, stats) or (perm, iperm, stats); perm[k] = original vertex
    placed at position k.  Raises RcmError on a non-OK status.
    """
    import torch

    device = device or torch.device("cuda", torch.cuda.current_device())
    rp = _dev_i32(rowptr, device)
    ci = _dev_i32(colidx, device)
    n = rp.numel() - 1
    if n < 0:
        raise ValueError("rowptr must have n+1 entries")
    perm = torch.empty(max(n, 0), dtype=torch.int32, device=rp.device)
    iperm = torch.empty(max(n, 0), dtype=torch.int32, device=rp.device) if return_iperm else None
    o = make_options(**opts)
    st = Stats()
    ws_ptr, ws_size = None, 0
    if workspace is not None:
        ws_ptr, ws_size = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    status = lib().rcm_order_ex(
        int(n), rp.data_ptr() if n >= 0 else None, ci.data_ptr() if ci.numel() else None,
        perm.data_ptr() if n > 0 else None, iperm.data_ptr() if (iperm is not None and n > 0)
        else None, ctypes.byref(st), ctypes.byref(o), ws_ptr, ws_size, _stream_handle(stream))
    if status != OK:
        raise RcmError(status, status_string(status))
    if return_iperm:
        return perm, iperm, st.to_dict()
    return perm, st.to_dict()


def order_batched(vtx_offsets, nnz_offsets, rowptr_cat, colidx_cat, *, stream=None,
                  workspace=None, device=None, **opts):
    """Order G graphs in one call.  vtx_offsets / nnz_offsets: host int64
    prefix sums (G+1); rowptr_cat / colidx_cat: the graphs' local CSR arrays
    concatenated (graph g's rowptr at rowptr_cat[vtx_offsets[g] + g]).
    Returns (perm_cat, [stats per graph])."""
    import numpy as np
    import torch

    device = device or torch.device("cuda", torch.cuda.current_device())
    vo = np.ascontiguousarray(vtx_offsets, dtype=np.int64)
    no = np.ascontiguousarray(nnz_offsets, dtype=np.int64)
    G = vo.size - 1
    rp = _dev_i32(rowptr_cat, device)
    ci = _dev_i32(colidx_cat, device)
    total = int(vo[-1]) if G >= 0 else 0
    perm = torch.empty(max(total, 1), dtype=torch.int32, device=rp.device)
    st = (Stats * max(G, 1))()
    o = make_options(**opts)
    ws_ptr, ws_size = None, 0
    if workspace is not None:
        ws_ptr, ws_size = workspace.data_ptr(), workspace.numel() * workspace.element_size()
    status = lib().rcm_order_batched(
        int(G), vo.ctypes.data_as(ctypes.c_void_p), no.ctypes.data_as(ctypes.c_void_p),
        rp.data_ptr(), ci.data_ptr() if ci.numel() else None, perm.data_ptr(),
        ctypes.cast(st, ctypes.c_void_p), ctypes.byref(o), ws_ptr, ws_size,
        _stream_handle(stream))
    if status != OK:
        raise RcmError(status, status_string(status))
    return perm[:total], [st[i].to_dict() for i in range(G)]
