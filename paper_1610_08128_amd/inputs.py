"""Seeded synthetic inputs: symmetric sparsity patterns in int32 CSR form.

This module only *builds graphs*.  It holds none of the ordering method's
arithmetic (no degrees, no traversal, no bandwidth), so that both the CPU
oracle and the GPU library can be fed the very same bytes without sharing any
of the method's code.

Workload shapes follow the paper's experimental setting: symmetric matrices
(Section V, matrix suite) of mesh-like, medium and high pseudo-diameter
structure.  The paper's own matrices are not available, so seeded synthetic
stand-ins of the same kind are generated here:

* 2D 5-point and 3D 7-point stencil patterns (mesh problems such as nd24k);
* a long thin 2D strip with randomly dropped edges (high-diameter problems
  such as ldoor / Flan_1565, taken to the extreme);
* 2D random geometric graphs made of several disjoint patches (irregular,
  disconnected patterns; the paper handles several components by running the
  ordering once per component, Section III-B);
* batches and arrival streams of the above.

Every generator writes rows sorted by column with the diagonal present unless
asked otherwise; ``shuffle_rows`` puts each row's entries in a seeded random
order (the interface accepts rows in any order).  Vertex ids are randomly relabelled from a seed with
``numpy.random.default_rng(seed).permutation(n)`` applied to both endpoints.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

__all__ = [
    "Graph",
    "from_edges",
    "grid2d",
    "grid3d",
    "strip_drop",
    "rgg_patches",
    "relabel",
    "path",
    "cycle",
    "complete",
    "star",
    "erdos_renyi",
    "random_tree",
    "disjoint_union",
    "drop_diagonal",
    "add_random_self_loops",
    "shuffle_rows",
    "config",
    "CONFIG_NAMES",
    "batch_graphs",
    "concat_batch",
    "request_stream",
]


@dataclasses.dataclass
class Graph:
    """A symmetric sparsity pattern in CSR form (int32 arrays)."""

    n: int
    rowptr: np.ndarray  # int32[n+1]
    colidx: np.ndarray  # int32[nnz]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1]) if self.n > 0 else 0


# --------------------------------------------------------------------------
# CSR assembly
# --------------------------------------------------------------------------

def from_edges(n: int, u: np.ndarray, v: np.ndarray, *, diag: bool = True,
               perm: Optional[np.ndarray] = None, name: str = "") -> Graph:
    """Assemble a symmetric CSR pattern from an undirected edge list.

    ``u``/``v`` list each undirected edge once (u != v); both directions are
    stored.  Duplicate edges are merged.  ``perm`` (old id -> new id), if
    given, relabels both endpoints before assembly.  Rows come out sorted.
    """
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    if perm is not None:
        perm = np.asarray(perm, dtype=np.int64)
        u = perm[u]
        v = perm[v]
    parts_r = [u, v]
    parts_c = [v, u]
    if diag and n > 0:
        d = np.arange(n, dtype=np.int64)
        parts_r.append(d)
        parts_c.append(d)
    rows = np.concatenate(parts_r) if parts_r else np.zeros(0, np.int64)
    cols = np.concatenate(parts_c) if parts_c else np.zeros(0, np.int64)
    keys = rows * np.int64(max(n, 1)) + cols
    del rows, cols
    keys = np.unique(keys)
    rows = keys // max(n, 1)
    colidx = (keys - rows * max(n, 1)).astype(np.int32)
    counts = np.bincount(rows, minlength=n) if n > 0 else np.zeros(0, np.int64)
    del keys, rows
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if rowptr[-1] >= 2**31:
        raise ValueError("pattern too large for int32 CSR")
    return Graph(n, rowptr.astype(np.int32), colidx, name)


def _edges_of(g: Graph) -> Tuple[np.ndarray, np.ndarray, bool]:
    """Undirected off-diagonal edges (u < v) of a CSR pattern, and whether
    every diagonal entry is present."""
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.rowptr).astype(np.int64))
    cols = g.colidx.astype(np.int64)
    diag_count = int(np.count_nonzero(rows == cols))
    keep = rows < cols
    return rows[keep], cols[keep], diag_count == g.n


def relabel(g: Graph, seed: int) -> Tuple[Graph, np.ndarray]:
    """Randomly relabel a pattern: new_id = perm[old_id] with
    ``perm = default_rng(seed).permutation(n)``.  Self loops are kept
    exactly where they were (moved with their vertex)."""
    perm = np.random.default_rng(seed).permutation(g.n)
    rows = np.repeat(np.arange(g.n, dtype=np.int64), np.diff(g.rowptr).astype(np.int64))
    cols = g.colidx.astype(np.int64)
    pr = perm[rows]
    pc = perm[cols]
    keys = np.sort(pr * max(g.n, 1) + pc)
    r = keys // max(g.n, 1)
    c = (keys - r * max(g.n, 1)).astype(np.int32)
    rowptr = np.zeros(g.n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=g.n), out=rowptr[1:])
    return Graph(g.n, rowptr.astype(np.int32), c, g.name), perm


# --------------------------------------------------------------------------
# Structured generators
# --------------------------------------------------------------------------

def _grid2d_edges(k: int, m: int) -> Tuple[np.ndarray, np.ndarray]:
    idx = np.arange(k * m, dtype=np.int64).reshape(k, m)
    hu, hv = idx[:, :-1].ravel(), idx[:, 1:].ravel()
    vu, vv = idx[:-1, :].ravel(), idx[1:, :].ravel()
    return np.concatenate([hu, vu]), np.concatenate([hv, vv])


def grid2d(k: int, m: int, *, seed: Optional[int] = None, diag: bool = True) -> Graph:
    """k x m 2D 5-point stencil pattern; vertex (i, j) has id i*m + j before
    relabelling.  With ``seed`` the ids are randomly relabelled."""
    u, v = _grid2d_edges(k, m)
    n = k * m
    perm = np.random.default_rng(seed).permutation(n) if seed is not None else None
    return from_edges(n, u, v, diag=diag, perm=perm, name=f"grid2d_{k}x{m}")


def grid3d(a: int, b: int, c: int, *, seed: Optional[int] = None, diag: bool = True) -> Graph:
    """a x b x c 3D 7-point stencil pattern; (x, y, z) has id (x*b + y)*c + z
    before relabelling."""
    idx = np.arange(a * b * c, dtype=np.int64).reshape(a, b, c)
    us = [idx[:-1, :, :].ravel(), idx[:, :-1, :].ravel(), idx[:, :, :-1].ravel()]
    vs = [idx[1:, :, :].ravel(), idx[:, 1:, :].ravel(), idx[:, :, 1:].ravel()]
    n = a * b * c
    perm = np.random.default_rng(seed).permutation(n) if seed is not None else None
    return from_edges(n, np.concatenate(us), np.concatenate(vs), diag=diag, perm=perm,
                      name=f"grid3d_{a}x{b}x{c}")


def strip_drop(k: int, m: int, p: float, seed: int, *, relabel_ids: bool = True) -> Graph:
    """k x m 2D 5-point strip; every undirected edge is dropped independently
    with probability ``p`` (symmetry is kept because an edge is dropped in
    both directions); the diagonal is kept.  One generator stream drives both
    the drop mask and the relabelling."""
    rng = np.random.default_rng(seed)
    u, v = _grid2d_edges(k, m)
    keep = rng.random(u.shape[0]) >= p
    u, v = u[keep], v[keep]
    n = k * m
    perm = rng.permutation(n) if relabel_ids else None
    return from_edges(n, u, v, diag=True, perm=perm, name=f"strip_{k}x{m}_drop{p}")


def rgg_patches(n: int, seed: int, *, patches: Optional[int] = None,
                mean_degree: float = 12.0, relabel_ids: bool = True) -> Graph:
    """2D random geometric graph built from K disjoint patches.

    K ~ U{2..5} unless given.  Each patch holds about n/K points uniform in
    [0,1)^2 joined when closer than r = sqrt(mean_degree / (pi * n_patch)),
    which gives an expected degree close to ``mean_degree`` away from the
    patch border.  Patches share no edges, so the graph has at least K
    components (usually more: stray points near the border)."""
    from scipy.spatial import cKDTree

    rng = np.random.default_rng(seed)
    K = int(patches) if patches is not None else int(rng.integers(2, 6))
    K = max(1, min(K, n))
    sizes = np.full(K, n // K, dtype=np.int64)
    sizes[: n - int(sizes.sum())] += 1
    us, vs = [], []
    base = 0
    for s in sizes:
        s = int(s)
        pts = rng.random((s, 2))
        if s > 1:
            r = math.sqrt(mean_degree / (math.pi * s))
            pairs = cKDTree(pts).query_pairs(r, output_type="ndarray")
            if pairs.size:
                us.append(pairs[:, 0].astype(np.int64) + base)
                vs.append(pairs[:, 1].astype(np.int64) + base)
        base += s
    u = np.concatenate(us) if us else np.zeros(0, np.int64)
    v = np.concatenate(vs) if vs else np.zeros(0, np.int64)
    perm = rng.permutation(n) if relabel_ids else None
    return from_edges(n, u, v, diag=True, perm=perm, name=f"rgg_{n}_K{K}")


# --------------------------------------------------------------------------
# Small graphs for tests
# --------------------------------------------------------------------------

def path(n: int, *, seed: Optional[int] = None, diag: bool = True) -> Graph:
    u = np.arange(max(n - 1, 0), dtype=np.int64)
    perm = np.random.default_rng(seed).permutation(n) if seed is not None else None
    return from_edges(n, u, u + 1, diag=diag, perm=perm, name=f"path_{n}")


def cycle(n: int, *, seed: Optional[int] = None, diag: bool = True) -> Graph:
    u = np.arange(n, dtype=np.int64)
    v = (u + 1) % n
    perm = np.random.default_rng(seed).permutation(n) if seed is not None else None
    return from_edges(n, u, v, diag=diag, perm=perm, name=f"cycle_{n}")


def complete(n: int, *, diag: bool = True) -> Graph:
    iu = np.triu_indices(n, 1)
    return from_edges(n, iu[0], iu[1], diag=diag, name=f"complete_{n}")


def star(n: int, center: int = 0, *, diag: bool = True) -> Graph:
    leaves = np.array([i for i in range(n) if i != center], dtype=np.int64)
    return from_edges(n, np.full(leaves.shape, center, np.int64), leaves, diag=diag,
                      name=f"star_{n}_c{center}")


def erdos_renyi(n: int, p: float, seed: int, *, diag: bool = True) -> Graph:
    rng = np.random.default_rng(seed)
    iu = np.triu_indices(n, 1)
    keep = rng.random(iu[0].shape[0]) < p
    return from_edges(n, iu[0][keep], iu[1][keep], diag=diag, name=f"er_{n}_{p}_{seed}")


def random_tree(n: int, seed: int, *, diag: bool = True) -> Graph:
    rng = np.random.default_rng(seed)
    if n <= 1:
        return from_edges(n, np.zeros(0, np.int64), np.zeros(0, np.int64), diag=diag)
    parents = np.array([rng.integers(0, i) for i in range(1, n)], dtype=np.int64)
    return from_edges(n, parents, np.arange(1, n, dtype=np.int64), diag=diag,
                      name=f"tree_{n}_{seed}")


def disjoint_union(graphs: Sequence[Graph], *, seed: Optional[int] = None) -> Graph:
    """Disjoint union; graph g's vertices get ids offset by the sizes of the
    graphs before it.  With ``seed`` the union is randomly relabelled."""
    us, vs = [], []
    off = 0
    diag_all = True
    for g in graphs:
        u, v, has_diag = _edges_of(g)
        diag_all &= has_diag
        us.append(u + off)
        vs.append(v + off)
        off += g.n
    u = np.concatenate(us) if us else np.zeros(0, np.int64)
    v = np.concatenate(vs) if vs else np.zeros(0, np.int64)
    perm = np.random.default_rng(seed).permutation(off) if seed is not None else None
    return from_edges(off, u, v, diag=diag_all, perm=perm, name="union")


def drop_diagonal(g: Graph) -> Graph:
    u, v, _ = _edges_of(g)
    return from_edges(g.n, u, v, diag=False, name=g.name + "_nodiag")


def add_random_self_loops(g: Graph, frac: float, seed: int) -> Graph:
    """Pattern without diagonal except a random fraction of self loops."""
    rng = np.random.default_rng(seed)
    u, v, _ = _edges_of(g)
    loops = np.nonzero(rng.random(g.n) < frac)[0].astype(np.int64)
    rows = np.concatenate([u, v, loops])
    cols = np.concatenate([v, u, loops])
    keys = np.unique(rows * max(g.n, 1) + cols)
    r = keys // max(g.n, 1)
    c = (keys - r * max(g.n, 1)).astype(np.int32)
    rowptr = np.zeros(g.n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=g.n), out=rowptr[1:])
    return Graph(g.n, rowptr.astype(np.int32), c, g.name + "_loops")


def shuffle_rows(g: Graph, seed: int) -> Graph:
    """The same pattern with every row's entries in a random order: one
    random key per entry from ``default_rng(seed)``, then a stable sort of
    the entries by (row, key).  The set of entries of each row is unchanged,
    so this only exercises the "rows need not be sorted" promise."""
    rng = np.random.default_rng(seed)
    lens = np.diff(g.rowptr).astype(np.int64)
    rows = np.repeat(np.arange(g.n, dtype=np.int64), lens)
    keys = rng.random(rows.size)
    order = np.lexsort((keys, rows))
    return Graph(g.n, g.rowptr.copy(), g.colidx[order].astype(np.int32), g.name + "_shuf")


# --------------------------------------------------------------------------
# Named workloads
# --------------------------------------------------------------------------

CONFIG_NAMES = {
    0: "grid2d_64x64",          # 4,096 vertices, 20,224 nnz
    1: "grid3d_128x128x128",    # 2,097,152 vertices, 14,581,760 nnz
    2: "strip_32x500000_drop1pct",  # 16M vertices, ~78.4M nnz
    3: "batch_512",             # 512 independent graphs
    4: "serving_stream",        # Poisson arrivals
}

DEFAULT_SEEDS = {0: 1, 1: 2, 2: 3, 3: 4}


def config(i: int, seed: Optional[int] = None) -> Graph:
    """The single-graph workloads: 0 = 64x64 2D 5-point, 1 = 128^3 3D
    7-point, 2 = 32x500,000 strip with 1% of edges dropped; all randomly
    relabelled from ``seed``."""
    s = DEFAULT_SEEDS[i] if seed is None else seed
    if i == 0:
        g = grid2d(64, 64, seed=s)
    elif i == 1:
        g = grid3d(128, 128, 128, seed=s)
    elif i == 2:
        g = strip_drop(32, 500_000, 0.01, seed=s)
    else:
        raise ValueError("config(i) covers the single-graph workloads 0..2")
    g.name = CONFIG_NAMES[i]
    return g


def _loguniform_int(rng: np.random.Generator, lo: float, hi: float) -> int:
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def _shape_graph(kind: int, n_target: int, seed: int) -> Graph:
    """kind 0: near-square 2D grid, 1: near-cubic 3D grid, 2: RGG patches."""
    if kind == 0:
        k = max(2, int(round(math.sqrt(n_target))))
        m = max(2, int(round(n_target / k)))
        return grid2d(k, m, seed=seed)
    if kind == 1:
        a = max(2, int(round(n_target ** (1.0 / 3.0))))
        c = max(2, int(round(n_target / (a * a))))
        return grid3d(a, a, c, seed=seed)
    return rgg_patches(max(n_target, 2), seed)


def batch_graphs(num_graphs: int = 512, seed: int = 4, lo: float = 1e3, hi: float = 2e5) -> List[Graph]:
    """Batched workload: sizes log-uniform in [lo, hi] vertices, graph kinds in
    round-robin order {2D grid, 3D grid, RGG patches}, each relabelled with
    its own child seed."""
    rng = np.random.default_rng(seed)
    out = []
    for gi in range(num_graphs):
        n_t = _loguniform_int(rng, lo, hi)
        child = int(rng.integers(0, 2**31 - 1))
        out.append(_shape_graph(gi % 3, n_t, child))
    return out


def concat_batch(graphs: Sequence[Graph]):
    """Concatenate graphs for a batched call: returns (vtx_offsets int64[G+1],
    nnz_offsets int64[G+1], rowptr_cat int32[sum(n_g+1)], colidx_cat
    int32[sum nnz]).  Each graph's rowptr slice is local (starts at 0) and
    occupies n_g+1 entries starting at vtx_offsets[g] + g."""
    G = len(graphs)
    vtx = np.zeros(G + 1, np.int64)
    nz = np.zeros(G + 1, np.int64)
    for i, g in enumerate(graphs):
        vtx[i + 1] = vtx[i] + g.n
        nz[i + 1] = nz[i] + g.nnz
    rowptr_cat = np.concatenate([g.rowptr for g in graphs]) if G else np.zeros(0, np.int32)
    colidx_cat = np.concatenate([g.colidx for g in graphs]) if G else np.zeros(0, np.int32)
    return vtx, nz, rowptr_cat.astype(np.int32), colidx_cat.astype(np.int32)


def request_stream(num: int, rate: float, *, seed_sizes: int = 5, seed_arrivals: int = 6,
                   lo_nnz: float = 1e4, hi_nnz: float = 2e7):
    """Serving workload description: a list of (arrival_time_s, kind,
    n_target, graph_seed).  Sizes are log-uniform in nnz; kind is uniform over
    the three generators, and the vertex count is chosen so that the pattern
    has about the drawn nnz (5, 7 and ~13 entries per row respectively).
    Arrival gaps are exponential with mean 1/rate (a Poisson process)."""
    rs = np.random.default_rng(seed_sizes)
    ra = np.random.default_rng(seed_arrivals)
    per_row = {0: 5.0, 1: 7.0, 2: 13.0}
    t = 0.0
    out = []
    for _ in range(num):
        t += float(ra.exponential(1.0 / rate))
        nnz = _loguniform_int(rs, lo_nnz, hi_nnz)
        kind = int(rs.integers(0, 3))
        n_t = max(2, int(round(nnz / per_row[kind])))
        out.append((t, kind, n_t, int(rs.integers(0, 2**31 - 1))))
    return out


def request_graph(kind: int, n_target: int, graph_seed: int) -> Graph:
    """Materialise one serving request."""
    return _shape_graph(kind, n_target, graph_seed)
