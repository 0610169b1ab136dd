"""CPU oracle for Reverse Cuthill-McKee ordering -- TEST INFRASTRUCTURE ONLY.

A thin ctypes wrapper over ``rcm_oracle.c`` (plain single-threaded C that
follows the paper's Algorithms 1-4 and Section II-A definitions step by
step).  Only the test suite, the smoke check and the benchmark's CPU-baseline
leg may import this package; the product library never does, and the two share
no code beyond the seeded input generators.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rcm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK = 0
ERR_INVALID_ARGUMENT = 1
ERR_BAD_CSR = 2
ERR_NOT_SYMMETRIC = 3
ERR_OUT_OF_MEMORY = 5


def build(force: bool = True) -> str:
    """Compile the oracle into ``oracle/liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Stats(ctypes.Structure):
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


STAT_FIELDS = [f for f, _ in _Stats._fields_]

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32 = ctypes.c_int32
        lib.orc_validate.argtypes = [i32, P, P, ctypes.c_int]
        lib.orc_validate.restype = ctypes.c_int
        lib.orc_degrees.argtypes = [i32, P, P, P]
        lib.orc_degrees.restype = None
        lib.orc_bw_profile.argtypes = [i32, P, P, P, P, P]
        lib.orc_bw_profile.restype = ctypes.c_int
        lib.orc_level_structure.argtypes = [P, P, i32, P, P, P]
        lib.orc_level_structure.restype = i32
        lib.orc_pseudo_peripheral.argtypes = [P, P, P, i32, ctypes.c_int, P, P, P, P]
        lib.orc_pseudo_peripheral.restype = i32
        lib.orc_cm_queue.argtypes = [P, P, P, i32, i32, P, P, P]
        lib.orc_cm_queue.restype = i32
        lib.orc_cm_levelsync.argtypes = [P, P, P, i32, i32, P, P, P, P]
        lib.orc_cm_levelsync.restype = i32
        lib.orc_rcm_ex.argtypes = [i32, P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, P, P, ctypes.POINTER(_Stats), P, P, P, P]
        lib.orc_rcm_ex.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _i32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.int32)


@dataclass
class OracleResult:
    status: int
    perm: np.ndarray
    iperm: np.ndarray
    stats: dict
    comp_offset: np.ndarray
    comp_root: np.ndarray
    comp_nbfs: np.ndarray
    comp_levels: np.ndarray


def validate(n, rowptr, colidx, full_check=False) -> int:
    lib = _load()
    rp = _i32(rowptr) if rowptr is not None else None
    ci = _i32(colidx) if colidx is not None else None
    return int(lib.orc_validate(int(n), _ptr(rp), _ptr(ci), int(bool(full_check))))


def degrees(n, rowptr, colidx) -> np.ndarray:
    lib = _load()
    rp, ci = _i32(rowptr), _i32(colidx)
    deg = np.zeros(n, np.int32)
    lib.orc_degrees(int(n), _ptr(rp), _ptr(ci), _ptr(deg))
    return deg


def bw_profile(n, rowptr, colidx, perm=None):
    """(bandwidth, profile) of P A P^T where perm[k] = old index at new k."""
    lib = _load()
    rp, ci = _i32(rowptr), _i32(colidx)
    p = _i32(perm) if perm is not None else None
    bw = np.zeros(1, np.int64)
    pr = np.zeros(1, np.int64)
    lib.orc_bw_profile(int(n), _ptr(rp), _ptr(ci), _ptr(p), _ptr(bw), _ptr(pr))
    return int(bw[0]), int(pr[0])


def level_structure(n, rowptr, colidx, root):
    """Distances from root (-1 outside its component) and eccentricity."""
    lib = _load()
    rp, ci = _i32(rowptr), _i32(colidx)
    level = np.full(n, -1, np.int32)
    order = np.zeros(n, np.int32)
    cnt = np.zeros(1, np.int32)
    ecc = lib.orc_level_structure(_ptr(rp), _ptr(ci), int(root), _ptr(level), _ptr(order),
                                  _ptr(cnt))
    return level, int(ecc), order[: int(cnt[0])].copy()


def pseudo_peripheral(n, rowptr, colidx, start, variant=0):
    """(vertex, number of level structures computed, component size)."""
    lib = _load()
    rp, ci = _i32(rowptr), _i32(colidx)
    deg = degrees(n, rp, ci)
    level = np.full(n, -1, np.int32)
    order = np.zeros(n, np.int32)
    nb = np.zeros(1, np.int32)
    cs = np.zeros(1, np.int32)
    r = lib.orc_pseudo_peripheral(_ptr(rp), _ptr(ci), _ptr(deg), int(start), int(variant),
                                  _ptr(level), _ptr(order), _ptr(nb), _ptr(cs))
    return int(r), int(nb[0]), int(cs[0])


def cm_from_root(n, rowptr, colidx, root, mode=0) -> np.ndarray:
    """Cuthill-McKee order (before reversal) of root's component, from the
    given root: mode 0 = Algorithm 1 queue, 1 = Algorithm 3."""
    lib = _load()
    rp, ci = _i32(rowptr), _i32(colidx)
    deg = degrees(n, rp, ci)
    label = np.full(n, -1, np.int32)
    cm = np.zeros(n, np.int32)
    nl = np.zeros(1, np.int32)
    if mode == 0:
        got = lib.orc_cm_queue(_ptr(rp), _ptr(ci), _ptr(deg), int(root), 0, _ptr(label),
                               _ptr(cm), _ptr(nl))
    else:
        parent = np.full(n, np.iinfo(np.int32).max, np.int32)
        got = lib.orc_cm_levelsync(_ptr(rp), _ptr(ci), _ptr(deg), int(root), 0, _ptr(label),
                                   _ptr(cm), _ptr(parent), _ptr(nl))
    return cm[:got].copy()


def rcm(n, rowptr, colidx, *, pp_variant=0, reverse_mode=0, full_check=False,
        cm_mode=0) -> OracleResult:
    """Whole ordering.  cm_mode 0 = Algorithm 1 queue, 1 = Algorithm 3
    level-synchronous labelling, 2 = level order by id (no sort), 3 = level
    order by (degree, id) (one global sort at the end); 2 and 3 are the
    alternatives to per-level sorting named as future work in Section VI."""
    lib = _load()
    n = int(n)
    rp = _i32(rowptr) if rowptr is not None else None
    ci = _i32(colidx) if colidx is not None else None
    cap = max(n, 1)
    perm = np.zeros(cap, np.int32)
    iperm = np.zeros(cap, np.int32)
    co = np.zeros(cap, np.int32)
    cr = np.zeros(cap, np.int32)
    cb = np.zeros(cap, np.int32)
    cl = np.zeros(cap, np.int32)
    st = _Stats()
    status = lib.orc_rcm_ex(n, _ptr(rp), _ptr(ci), int(pp_variant), int(reverse_mode),
                            int(bool(full_check)), int(cm_mode), _ptr(perm), _ptr(iperm),
                            ctypes.byref(st), _ptr(co), _ptr(cr), _ptr(cb), _ptr(cl))
    stats = {f: int(getattr(st, f)) for f in STAT_FIELDS}
    nc = stats["num_components"] if status == OK else 0
    nn = n if status == OK else 0
    return OracleResult(int(status), perm[:nn].copy(), iperm[:nn].copy(), stats,
                        co[:nc].copy(), cr[:nc].copy(), cb[:nc].copy(), cl[:nc].copy())


# ---------------------------------------------------------------------------
# Applying an ordering (the reordered matrix and the product an iterative
# solver spends its time in; the paper motivates the ordering by the data
# locality it gives such solvers, Section I).  Plain definitions, in numpy.
# ---------------------------------------------------------------------------

def permute_csr(n, rowptr, colidx, perm, vals=None):
    """B = P A P^T: row k of B is row perm[k] of A with every column j
    renamed iperm[j] (iperm the inverse of perm), entries sorted by column.
    Returns (rowptr_B, colidx_B, vals_B or None)."""
    n = int(n)
    rp = np.asarray(rowptr, dtype=np.int64)
    ci = np.asarray(colidx, dtype=np.int64)
    perm = np.asarray(perm, dtype=np.int64)
    iperm = np.empty(n, dtype=np.int64)
    iperm[perm] = np.arange(n, dtype=np.int64)
    out_rp = np.zeros(n + 1, dtype=np.int64)
    rows, vrows = [], []
    for k in range(n):
        v = perm[k]
        cols = iperm[ci[rp[v]:rp[v + 1]]]
        order = np.argsort(cols, kind="stable")
        rows.append(cols[order])
        if vals is not None:
            vrows.append(np.asarray(vals, dtype=np.float64)[rp[v]:rp[v + 1]][order])
        out_rp[k + 1] = out_rp[k] + cols.size
    out_ci = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    out_v = (np.concatenate(vrows) if vrows else np.zeros(0)) if vals is not None else None
    return out_rp.astype(np.int32), out_ci.astype(np.int32), out_v


def spmv(n, rowptr, colidx, x, vals=None):
    """y = A x in float64, each row summed in storage order (vals None:
    every stored entry is 1)."""
    n = int(n)
    x = np.asarray(x, dtype=np.float64)
    y = np.zeros(n, dtype=np.float64)
    for i in range(n):
        a, b = int(rowptr[i]), int(rowptr[i + 1])
        w = np.ones(b - a) if vals is None else np.asarray(vals[a:b], dtype=np.float64)
        s = 0.0
        for t in range(b - a):
            s += w[t] * x[int(colidx[a + t])]
        y[i] = s
    return y
