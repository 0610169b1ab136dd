"""Python binding of include/rcm_apply.h: the permuted matrix B = P A P^T
and the sparse matrix-vector product (argument marshalling only; both run in
the library's HIP kernels)."""

from __future__ import annotations

import ctypes
from typing import Optional, Tuple

from . import rcm

APPLY_EXPORTED = ["rcm_permute_workspace_bytes", "rcm_permute", "rcm_spmv"]

_configured = False


def _lib() -> ctypes.CDLL:
    global _configured
    L = rcm.lib()
    if not _configured:
        P, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
        L.rcm_permute_workspace_bytes.argtypes = [i32, i64, i32]
        L.rcm_permute_workspace_bytes.restype = ctypes.c_size_t
        L.rcm_permute.argtypes = [i32, i64, P, P, P, P, P, P, P, P, P, ctypes.c_size_t, P]
        L.rcm_permute.restype = ctypes.c_int
        L.rcm_spmv.argtypes = [i32, P, P, P, P, P, P]
        L.rcm_spmv.restype = ctypes.c_int
        _configured = True
    return L


def permute_workspace_bytes(n: int, nnz: int, with_values: bool = False) -> int:
    return int(_lib().rcm_permute_workspace_bytes(int(n), int(nnz), 1 if with_values else 0))


def _ptr(t) -> Optional[int]:
    return t.data_ptr() if t is not None and t.numel() else None


def permute(rowptr, colidx, perm, iperm, vals=None, *, stream=None, workspace=None):
    """B = P A P^T for CUDA tensors (int32 CSR, int32 perm/iperm, optional
    float64 vals).  Returns (rowptr_out, colidx_out, vals_out or None)."""
    import torch

    n = rowptr.numel() - 1
    nnz = colidx.numel()
    dev = rowptr.device
    rp_out = torch.empty(n + 1, dtype=torch.int32, device=dev)
    ci_out = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
    v_out = torch.empty(max(nnz, 1), dtype=torch.float64, device=dev) if vals is not None else None
    if workspace is None:
        workspace = torch.empty(max(permute_workspace_bytes(n, nnz, vals is not None), 1),
                                dtype=torch.uint8, device=dev)
    status = _lib().rcm_permute(
        int(n), int(nnz), _ptr(rowptr), _ptr(colidx), _ptr(vals), _ptr(perm), _ptr(iperm),
        _ptr(rp_out), ci_out.data_ptr() if nnz else None,
        v_out.data_ptr() if (v_out is not None and nnz) else None, workspace.data_ptr(),
        workspace.numel(), rcm._stream_handle(stream))
    if status != rcm.OK:
        raise rcm.RcmError(status, rcm.status_string(status))
    return rp_out, ci_out[:nnz], (v_out[:nnz] if v_out is not None else None)


def spmv(rowptr, colidx, x, vals=None, *, out=None, stream=None):
    """y = A x (float64) for a CSR matrix held in CUDA tensors."""
    import torch

    n = rowptr.numel() - 1
    y = out if out is not None else torch.empty(max(n, 0), dtype=torch.float64, device=x.device)
    status = _lib().rcm_spmv(int(n), _ptr(rowptr), _ptr(colidx), _ptr(vals), _ptr(x), _ptr(y),
                             rcm._stream_handle(stream))
    if status != rcm.OK:
        raise rcm.RcmError(status, rcm.status_string(status))
    return y
