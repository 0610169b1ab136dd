"""Pins for the oracle's level orders (cm_mode 2 and 3): the alternatives to
per-level sorting that the paper names as future work (Section VI), "no
sort" (each level in increasing id) and "one global sort at the end" by
(level, degree, id).

The expected orders are built here from scipy's BFS distances and numpy's
lexsort, not from the oracle's level structure or its comparison; the root of
each component comes from the oracle's pseudo-peripheral search, which
test_oracle_pins.py pins on its own.
"""

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components, shortest_path

import oracle
from paper_1610_08128_amd import inputs as I


def _sp(g):
    return sp.csr_matrix((np.ones(g.nnz), g.colidx, g.rowptr), shape=(g.n, g.n))


def _graphs():
    out = []
    out.append(I.grid2d(9, 13, seed=3))
    out.append(I.grid3d(4, 5, 6, seed=5, diag=False))
    out.append(I.strip_drop(4, 60, 0.1, seed=7))
    out.append(I.rgg_patches(400, seed=11))
    out.append(I.erdos_renyi(80, 0.04, seed=2))
    out.append(I.disjoint_union([I.grid2d(5, 7), I.path(9), I.star(6), I.complete(1),
                                 I.random_tree(30, 4)], seed=9))
    return out


def _expected(g, by_degree, pp_variant, reverse_mode):
    """Blocks of components in order of their lowest id; inside a block the
    vertices sorted by (distance from the root, degree or 0, id); then the
    reversal."""
    A = _sp(g)
    _, comp = connected_components(A, directed=False)
    deg = oracle.degrees(g.n, g.rowptr, g.colidx).astype(np.int64)
    order = []
    seen = set()
    for s in range(g.n):
        c = comp[s]
        if c in seen:
            continue
        seen.add(c)
        members = np.nonzero(comp == c)[0]
        root, _, size = oracle.pseudo_peripheral(g.n, g.rowptr, g.colidx, s, pp_variant)
        assert size == members.size
        dist = shortest_path(A, unweighted=True, indices=root)[members].astype(np.int64)
        key2 = deg[members] if by_degree else np.zeros(members.size, np.int64)
        idx = np.lexsort((members, key2, dist))
        block = members[idx]
        order.append(block[::-1] if reverse_mode == 0 else block)
    cm = np.concatenate(order)
    return cm if reverse_mode == 0 else cm[::-1]


@pytest.mark.parametrize("gi", range(6))
@pytest.mark.parametrize("cm_mode", [2, 3])
@pytest.mark.parametrize("pp_variant", [0, 1])
@pytest.mark.parametrize("reverse_mode", [0, 1])
def test_level_order_definition(gi, cm_mode, pp_variant, reverse_mode):
    g = _graphs()[gi]
    r = oracle.rcm(g.n, g.rowptr, g.colidx, pp_variant=pp_variant, reverse_mode=reverse_mode,
                   cm_mode=cm_mode)
    assert r.status == oracle.OK
    want = _expected(g, cm_mode == 3, pp_variant, reverse_mode)
    assert np.array_equal(r.perm, want)


@pytest.mark.parametrize("n", [2, 5, 17])
@pytest.mark.parametrize("seed", range(3))
def test_level_orders_equal_rcm_on_paths(n, seed):
    """Every level of a path rooted at an end holds one vertex, so no order
    inside a level can differ: all labelling modes agree."""
    g = I.path(n, seed=seed)
    want = oracle.rcm(g.n, g.rowptr, g.colidx).perm
    for cm_mode in (1, 2, 3):
        got = oracle.rcm(g.n, g.rowptr, g.colidx, cm_mode=cm_mode).perm
        assert np.array_equal(got, want)


@pytest.mark.parametrize("seed", range(5))
def test_level_order_bandwidth_bound(seed):
    """In any order that keeps levels contiguous, an edge joins two
    vertices of the same or adjacent levels, so it spans less than
    |L_i| + |L_(i+1)| positions; the bandwidth is below the largest sum of
    two adjacent level widths."""
    rng = np.random.default_rng(seed)
    a, b, c = (int(x) for x in rng.integers(3, 9, size=3))
    g = I.grid3d(a, b, c, seed=seed, diag=bool(seed % 2))
    A = _sp(g)
    _, comp = connected_components(A, directed=False)
    assert comp.max() == 0
    for cm_mode in (2, 3):
        r = oracle.rcm(g.n, g.rowptr, g.colidx, cm_mode=cm_mode)
        root = int(r.comp_root[0])
        dist = shortest_path(A, unweighted=True, indices=root).astype(np.int64)
        widths = np.bincount(dist)
        bound = int(np.max(widths[:-1] + widths[1:])) if widths.size > 1 else 1
        assert r.stats["bandwidth_after"] < bound


@pytest.mark.parametrize("pp_variant", [0, 1])
def test_level_order_stats(pp_variant):
    """edges_traversed counts the search's level structures, plus one more
    when the root is Algorithm 4's pick; num_levels is the root's
    eccentricity plus one."""
    g = I.disjoint_union([I.grid2d(6, 9, seed=1), I.random_tree(40, 3)], seed=2)
    A = _sp(g)
    deg = oracle.degrees(g.n, g.rowptr, g.colidx).astype(np.int64)
    _, comp = connected_components(A, directed=False)
    for cm_mode in (2, 3):
        r = oracle.rcm(g.n, g.rowptr, g.colidx, pp_variant=pp_variant, cm_mode=cm_mode)
        want_edges = 0
        want_levels = 0
        for c in range(r.stats["num_components"]):
            root = int(r.comp_root[c])
            members = np.nonzero(comp == comp[root])[0]
            ecc = int(shortest_path(A, unweighted=True, indices=root)[members].max())
            assert r.comp_levels[c] == ecc + 1
            want_levels += ecc + 1
            want_edges += (int(r.comp_nbfs[c]) + pp_variant) * int(deg[members].sum())
        assert r.stats["edges_traversed"] == want_edges
        assert r.stats["num_levels"] == want_levels


def test_level_orders_lose_quality_on_a_grid():
    """Dropping the parent key can only be judged against the exact order:
    on a relabelled square grid the exact RCM reaches the optimal bandwidth
    k, the level orders do not (they keep a level's vertices in id order, so
    neighbours in adjacent levels land up to two level widths apart)."""
    k = 24
    g = I.grid2d(k, k, seed=6)
    exact = oracle.rcm(g.n, g.rowptr, g.colidx).stats["bandwidth_after"]
    assert exact == k
    for cm_mode in (2, 3):
        bw = oracle.rcm(g.n, g.rowptr, g.colidx, cm_mode=cm_mode).stats["bandwidth_after"]
        assert k < bw < 2 * k
