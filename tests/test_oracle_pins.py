"""Pins for the CPU oracle: it is checked against things other than itself.

Each test states what fixes the expected value: a closed form derived from the
paper's rules, a library routine (scipy), brute force on tiny inputs, or a
published theorem.  A plausible mistake in the oracle (wrong tie-break, wrong
parent rule, off-by-one in the pseudo-peripheral loop, a transposed
permutation, a dropped term in the profile) fails at least one of them.
"""

import itertools
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components, shortest_path

import oracle
from paper_1610_08128_amd import inputs as I


def _sp(g):
    data = np.ones(g.nnz, dtype=np.float64)
    return sp.csr_matrix((data, g.colidx, g.rowptr), shape=(g.n, g.n))


def _dense_permuted(g, perm):
    A = _sp(g).toarray() != 0
    p = np.asarray(perm)
    return A[np.ix_(p, p)]


def _edge_bandwidth(g, perm):
    """Bandwidth in its edge form: max |new(u) - new(v)| over the edges."""
    ip = np.empty(g.n, np.int64)
    ip[np.asarray(perm)] = np.arange(g.n)
    rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    if rows.size == 0:
        return 0
    return int(np.max(np.abs(ip[rows] - ip[g.colidx])))


# ---------------------------------------------------------------------------
# Section II-A: bandwidth and profile
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(12))
def test_bandwidth_matches_scipy_linalg(seed):
    """beta(A) equals scipy.linalg.bandwidth's lower bandwidth of the dense
    permuted matrix (a library routine), for patterns with and without a
    diagonal."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 30))
    g = I.erdos_renyi(n, float(rng.uniform(0.02, 0.4)), seed, diag=bool(seed % 2))
    perm = rng.permutation(n)
    bw, _ = oracle.bw_profile(g.n, g.rowptr, g.colidx, perm)
    lower, upper = scipy.linalg.bandwidth(_dense_permuted(g, perm).astype(np.float64))
    assert bw == lower == upper
    assert bw == _edge_bandwidth(g, perm)


def test_profile_closed_forms():
    """Envelope sizes of matrices whose envelope is known by inspection."""
    n = 9
    # tridiagonal (a path in natural order): one entry per row below the diagonal
    g = I.path(n)
    assert oracle.bw_profile(n, g.rowptr, g.colidx) == (1, n - 1)
    # full matrix: the whole strict lower triangle
    g = I.complete(n)
    assert oracle.bw_profile(n, g.rowptr, g.colidx) == (n - 1, n * (n - 1) // 2)
    # arrow with the hub first: full first column, so again the whole triangle
    g = I.star(n, center=0)
    assert oracle.bw_profile(n, g.rowptr, g.colidx) == (n - 1, n * (n - 1) // 2)
    # arrow with the hub last: only the last row has an envelope (n-1 entries)
    g = I.star(n, center=n - 1)
    assert oracle.bw_profile(n, g.rowptr, g.colidx) == (n - 1, n - 1)
    # the same arrow, permuted hub-first by perm = [n-1, 0, 1, ...]
    perm = [n - 1] + list(range(n - 1))
    assert oracle.bw_profile(n, g.rowptr, g.colidx, perm) == (n - 1, n * (n - 1) // 2)
    # diagonal only / no entries at all
    g = I.from_edges(n, np.zeros(0), np.zeros(0))
    assert oracle.bw_profile(n, g.rowptr, g.colidx) == (0, 0)
    g = I.from_edges(n, np.zeros(0), np.zeros(0), diag=False)
    assert oracle.bw_profile(n, g.rowptr, g.colidx) == (0, 0)


@pytest.mark.parametrize("seed", range(6))
def test_profile_counts_envelope_pairs(seed):
    """|Env(A)| counted pair by pair from the dense matrix: (i, j) with j < i
    is in the envelope iff some nonzero of row i lies at column <= j."""
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 25))
    g = I.erdos_renyi(n, 0.15, 100 + seed)
    perm = rng.permutation(n)
    B = _dense_permuted(g, perm)
    count = 0
    for i in range(n):
        for j in range(i):
            if B[i, : j + 1].any():
                count += 1
    assert oracle.bw_profile(n, g.rowptr, g.colidx, perm)[1] == count


# ---------------------------------------------------------------------------
# Degrees (the vector D of Algorithms 3 and 4)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(5))
def test_degrees_match_scipy(seed):
    g = I.add_random_self_loops(I.erdos_renyi(40, 0.1, seed), 0.5, seed)
    A = _sp(g).tolil()
    A.setdiag(0)
    A = A.tocsr()
    A.eliminate_zeros()
    assert np.array_equal(oracle.degrees(g.n, g.rowptr, g.colidx), np.diff(A.indptr))


# ---------------------------------------------------------------------------
# Input checks
# ---------------------------------------------------------------------------

def test_validate_statuses():
    g = I.path(5)
    assert oracle.validate(5, g.rowptr, g.colidx, True) == oracle.OK
    assert oracle.validate(0, None, None) == oracle.OK
    assert oracle.validate(-1, g.rowptr, g.colidx) == oracle.ERR_INVALID_ARGUMENT
    assert oracle.validate(5, None, g.colidx) == oracle.ERR_INVALID_ARGUMENT
    bad = g.rowptr.copy(); bad[0] = 1
    assert oracle.validate(5, bad, g.colidx) == oracle.ERR_BAD_CSR
    bad = g.rowptr.copy(); bad[2], bad[3] = bad[3], bad[2]
    assert oracle.validate(5, bad, g.colidx) == oracle.ERR_BAD_CSR
    badc = g.colidx.copy(); badc[3] = 5
    assert oracle.validate(5, g.rowptr, badc) == oracle.ERR_BAD_CSR
    badc = g.colidx.copy(); badc[3] = -1
    assert oracle.validate(5, g.rowptr, badc) == oracle.ERR_BAD_CSR
    # duplicate entry: a pattern is a set of positions, so a repeated one is
    # malformed with or without the full check (reading R4)
    dup = g.colidx.copy(); dup[1] = dup[0]
    assert oracle.validate(5, g.rowptr, dup, False) == oracle.ERR_BAD_CSR
    assert oracle.validate(5, g.rowptr, dup, True) == oracle.ERR_BAD_CSR
    # symmetric as a set but with (0, 1) twice in row 0
    rp = np.array([0, 3, 6, 8], np.int32)
    ci = np.array([0, 1, 1, 0, 1, 2, 1, 2], np.int32)
    assert oracle.validate(3, rp, ci, False) == oracle.ERR_BAD_CSR
    # asymmetric pattern: row 0 -> 4 without 4 -> 0
    rp = np.array([0, 2, 3, 4, 5, 6], np.int32)
    ci = np.array([0, 4, 1, 2, 3, 4], np.int32)
    assert oracle.validate(5, rp, ci, False) == oracle.OK
    assert oracle.validate(5, rp, ci, True) == oracle.ERR_NOT_SYMMETRIC
    r = oracle.rcm(5, rp, ci, full_check=True)
    assert r.status == oracle.ERR_NOT_SYMMETRIC


@pytest.mark.parametrize("seed", range(6))
def test_validate_duplicates_against_row_sets(seed):
    """Duplicates anywhere in a row, rows in any order: the oracle's status
    equals the plain definition (some row has fewer distinct columns than
    entries), for short rows and for rows far longer than a register batch."""
    rng = np.random.default_rng(seed)
    g = I.shuffle_rows(I.erdos_renyi(120, 0.02 + 0.1 * (seed % 3), seed), seed)
    assert oracle.validate(g.n, g.rowptr, g.colidx) == oracle.OK
    ci = g.colidx.copy()
    lens = np.diff(g.rowptr)
    rows = np.nonzero(lens >= 2)[0]
    r = int(rows[rng.integers(0, rows.size)])
    a, b = int(g.rowptr[r]), int(g.rowptr[r + 1])
    i, j = rng.choice(np.arange(a, b), 2, replace=False)
    ci[j] = ci[i]
    distinct = all(np.unique(ci[g.rowptr[v]:g.rowptr[v + 1]]).size == lens[v]
                   for v in range(g.n))
    assert not distinct
    assert oracle.validate(g.n, g.rowptr, ci) == oracle.ERR_BAD_CSR
    assert oracle.rcm(g.n, g.rowptr, ci).status == oracle.ERR_BAD_CSR


# ---------------------------------------------------------------------------
# Level structures (Section II-A) against a library BFS
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(8))
def test_level_structure_matches_scipy_bfs(seed):
    rng = np.random.default_rng(seed)
    g = I.erdos_renyi(60, 0.05, seed, diag=bool(seed % 2))
    root = int(rng.integers(0, g.n))
    level, ecc, order = oracle.level_structure(g.n, g.rowptr, g.colidx, root)
    d = shortest_path(_sp(g), unweighted=True, indices=root)
    want = np.where(np.isinf(d), -1, d).astype(np.int64)
    assert np.array_equal(level.astype(np.int64), want)
    assert ecc == int(want.max())
    assert sorted(order.tolist()) == sorted(np.nonzero(want >= 0)[0].tolist())


# ---------------------------------------------------------------------------
# Algorithm 2 on paths: closed form of the returned vertex
# ---------------------------------------------------------------------------

def _path_endpoint_root(g_perm, n):
    """The vertex Algorithm 2 must return on a path (derived from its
    steps): start at vertex 0; if 0 is an endpoint the loop stops at the far
    endpoint after 2 level structures; otherwise the first BFS ends at the
    farther endpoint (the lower id if both are equally far), the second ends
    at the other endpoint and the third confirms it, so the result is the
    endpoint nearer to vertex 0 (the higher id on a tie)."""
    pos = np.empty(n, np.int64)  # pos[vertex] = position along the path
    pos[g_perm] = np.arange(n)
    inv = np.asarray(g_perm)      # inv[position] = vertex id
    if n == 1:
        return 0, 2
    p0 = pos[0]
    ends = (int(inv[0]), int(inv[n - 1]))
    if p0 == 0:
        return ends[1], 2
    if p0 == n - 1:
        return ends[0], 2
    d0, d1 = p0, (n - 1) - p0
    if d0 < d1:
        return ends[0], 3
    if d1 < d0:
        return ends[1], 3
    return max(ends), 3


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 7, 10, 13])
@pytest.mark.parametrize("seed", range(6))
def test_pseudo_peripheral_on_paths(n, seed):
    perm = np.random.default_rng(seed).permutation(n)  # perm[pos] = vertex
    u = perm[:-1]
    v = perm[1:]
    g = I.from_edges(n, u, v)
    want_root, want_bfs = _path_endpoint_root(perm, n)
    r, nbfs, size = oracle.pseudo_peripheral(g.n, g.rowptr, g.colidx, 0, variant=0)
    assert (r, nbfs, size) == (want_root, want_bfs, n)
    res = oracle.rcm(g.n, g.rowptr, g.colidx)
    # the RCM of a path walks it from end to end: bandwidth 1, profile n-1
    assert res.stats["bandwidth_after"] == (1 if n > 1 else 0)
    assert res.stats["profile_after"] == n - 1
    assert res.stats["num_bfs"] == want_bfs
    assert res.stats["pseudo_diameter"] == n - 1
    # the CM order starts at the root, so the reversed order ends there
    assert res.perm[-1] == want_root


# ---------------------------------------------------------------------------
# Complete graphs
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [2, 3, 6, 11])
def test_complete_graph(n):
    """K_n: the first BFS from 0 has one level below the root; its min
    (degree, id) vertex is 1; the BFS from 1 has the same length, so 1 is the
    root.  All other vertices have equal degree, so the CM order is
    1, 0, 2, ..., n-1 and the reversed order is n-1, ..., 2, 0, 1."""
    g = I.complete(n)
    res = oracle.rcm(g.n, g.rowptr, g.colidx)
    assert res.comp_root.tolist() == [1]
    want = list(range(n - 1, 1, -1)) + [0, 1]
    assert res.perm.tolist() == want
    assert res.stats["bandwidth_after"] == n - 1
    assert res.stats["profile_after"] == n * (n - 1) // 2
    assert res.stats["num_bfs"] == 2


# ---------------------------------------------------------------------------
# Square grids: bandwidth k and profile k(k-1)(4k+7)/6 for any relabelling
# ---------------------------------------------------------------------------

def square_grid_profile(k):
    """Closed form for the RCM of a k x k 5-point grid rooted at a corner.

    Level d holds the anti-diagonal i + j = d.  Each vertex takes the
    lower-labelled of its two previous-level neighbours as parent, and a
    boundary child (degree 3) precedes an interior one (degree 4), so every
    level is ordered along its anti-diagonal in the same direction.  In the
    reversed order the envelope of vertex (i, j) reaches its last
    next-level neighbour; summing these distances level by level gives
    sum_{u=1}^{k-1} u(u+1) + sum_{t=0}^{k-1} (t^2 + 2t) = k(k-1)(4k+7)/6, and
    the largest of them is k (Chvatalova: k is also the minimum bandwidth of
    the k x k grid, so the result is optimal)."""
    return k * (k - 1) * (4 * k + 7) // 6


@pytest.mark.parametrize("k", [2, 3, 4, 5, 8, 13])
@pytest.mark.parametrize("seed", [None, 1, 2, 3])
def test_square_grid_closed_form(k, seed):
    g = I.grid2d(k, k, seed=seed)
    res = oracle.rcm(g.n, g.rowptr, g.colidx)
    assert res.stats["bandwidth_after"] == k
    assert res.stats["profile_after"] == square_grid_profile(k)
    assert res.stats["pseudo_diameter"] == 2 * k - 2
    assert res.stats["num_levels"] == 2 * k - 1


def test_grid_64x64_any_seed():
    """The 64 x 64 workload has the same bandwidth and profile under every
    relabelling."""
    for seed in range(1, 6):
        g = I.config(0, seed=seed)
        st = oracle.rcm(g.n, g.rowptr, g.colidx).stats
        assert st["bandwidth_after"] == 64
        assert st["profile_after"] == square_grid_profile(64) == 176736


@pytest.mark.parametrize("k,m", [(3, 7), (4, 9), (5, 12), (7, 20)])
def test_rectangular_grid_row_major(k, m):
    """Row-major ids (id = i*m + j), k < m.  The start vertex 0 is a corner;
    its BFS ends at the opposite corner n-1, whose BFS has the same length, so
    Algorithm 2 returns n-1 and Algorithm 4 returns the last level of that BFS,
    vertex 0.  From n-1 the lower-id neighbour is n-1-m (a step along the
    short axis), from 0 it is 1 (a step along the long axis); the first gives
    bandwidth k, the second k+1."""
    g = I.grid2d(k, m)
    n = k * m
    base = k * (k - 1) * (4 * k + 7) // 6
    r2 = oracle.rcm(g.n, g.rowptr, g.colidx, pp_variant=0)
    assert r2.comp_root.tolist() == [n - 1]
    assert r2.stats["bandwidth_after"] == k
    assert r2.stats["profile_after"] == base + k * k * (m - k)
    r4 = oracle.rcm(g.n, g.rowptr, g.colidx, pp_variant=1)
    assert r4.comp_root.tolist() == [0]
    assert r4.stats["bandwidth_after"] == k + 1
    assert r4.stats["profile_after"] == base + (k * k + k - 1) * (m - k)
    assert r2.stats["num_bfs"] == r4.stats["num_bfs"] == 2


@pytest.mark.parametrize("seed", range(8))
def test_grid_root_is_a_corner(seed):
    """On a relabelled k x m grid the root is a corner and the level
    structure has k+m-1 levels of sizes min(d+1, k, m, k+m-1-d)."""
    k, m = 6, 11
    g = I.grid2d(k, m, seed=seed)
    res = oracle.rcm(g.n, g.rowptr, g.colidx)
    r = int(res.comp_root[0])
    deg = oracle.degrees(g.n, g.rowptr, g.colidx)
    assert deg[r] == 2
    level, ecc, _ = oracle.level_structure(g.n, g.rowptr, g.colidx, r)
    assert ecc == k + m - 2
    sizes = np.bincount(level)
    want = [min(d + 1, k, m, k + m - 1 - d) for d in range(k + m - 1)]
    assert sizes.tolist() == want


# ---------------------------------------------------------------------------
# Statistics of the search: how many level structures Algorithm 2 builds, and
# the edges those and the labelled BFS scan
# ---------------------------------------------------------------------------

def _george_liu_bfs_count(g, A, members):
    """Algorithm 2 on one component, with scipy's unweighted BFS distances
    in place of the oracle's own: start at the lowest id, and while the
    newest level structure is deeper than the one before, restart from the
    minimum-(degree, id) vertex of its last level.  Returns the number of
    level structures built."""
    deg = np.array([np.count_nonzero(g.colidx[g.rowptr[v]:g.rowptr[v + 1]] != v)
                    for v in range(g.n)])
    def last_level(root):
        d = shortest_path(A, method="D", unweighted=True, indices=root)
        ecc = int(np.max(d[members]))
        ring = members[d[members] == ecc]
        return ecc, int(min(ring, key=lambda v: (deg[v], v)))
    r = int(members.min())
    ecc, pick = last_level(r)
    count, nlvl = 1, ecc - 1
    while ecc > nlvl:
        nlvl = ecc
        r = pick
        ecc, pick = last_level(r)
        count += 1
    return count


@pytest.mark.parametrize("seed", range(10))
def test_edges_traversed_counts_search_and_labelling(seed):
    """edges_traversed = sum over components of (level structures of the
    search + 1 labelled BFS) x (directed off-diagonal entries of the
    component), with the search's count taken from scipy's BFS and the
    entries counted from the CSR, for both root variants (which build the
    same level structures)."""
    rng = np.random.default_rng(seed)
    parts = [I.erdos_renyi(int(rng.integers(2, 60)), 0.08, seed),
             I.grid2d(int(rng.integers(2, 9)), int(rng.integers(2, 9)), seed=seed),
             I.random_tree(int(rng.integers(1, 40)), seed), I.path(1)]
    g = I.disjoint_union(parts, seed=seed)
    A = _sp(g)
    _, lab = connected_components(A, directed=False)
    rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    off = rows != g.colidx
    want_bfs, want_edges = 0, 0
    for c in np.unique(lab):
        members = np.nonzero(lab == c)[0]
        k = _george_liu_bfs_count(g, A, members)
        m_c = int(np.count_nonzero(off & (lab[rows] == c)))
        want_bfs += k
        want_edges += (k + 1) * m_c
    for pp in (0, 1):
        st = oracle.rcm(g.n, g.rowptr, g.colidx, pp_variant=pp).stats
        assert st["num_bfs"] == want_bfs, (pp, st)
        assert st["edges_traversed"] == want_edges, (pp, st)


@pytest.mark.parametrize("seed", range(12))
def test_edges_traversed_grid_closed_form(seed):
    """On a relabelled k x m grid, Algorithm 2 started at a vertex that is
    not a corner builds 3 level structures (the start, the far corner it
    finds, the opposite corner, which is no deeper); started at a corner it
    builds 2.  With the labelled BFS: 4 (or 3) sweeps over the 2(k(m-1) +
    m(k-1)) directed edges."""
    k, m = 5 + seed % 3, 9 + seed
    g = I.grid2d(k, m, seed=seed)
    deg = oracle.degrees(g.n, g.rowptr, g.colidx)
    sweeps = 3 if deg[0] == 2 else 4
    st = oracle.rcm(g.n, g.rowptr, g.colidx).stats
    assert st["num_bfs"] == sweeps - 1
    assert st["edges_traversed"] == sweeps * 2 * (k * (m - 1) + m * (k - 1))


# ---------------------------------------------------------------------------
# Cubes: relabelling invariance (cross-check values from an independent script)
# ---------------------------------------------------------------------------

CUBE_VALUES = {3: (8, 153), 4: (14, 629), 5: (21, 1881), 6: (30, 4611)}


@pytest.mark.parametrize("a", sorted(CUBE_VALUES))
def test_cube_seed_invariance(a):
    vals = set()
    for seed in range(1, 5):
        g = I.grid3d(a, a, a, seed=seed)
        st = oracle.rcm(g.n, g.rowptr, g.colidx).stats
        vals.add((st["bandwidth_after"], st["profile_after"]))
    assert vals == {CUBE_VALUES[a]}


# ---------------------------------------------------------------------------
# Brute force: RCM never beats the minimum bandwidth; equal where expected
# ---------------------------------------------------------------------------

def _min_bandwidth(g):
    rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    u, v = rows[rows < g.colidx], g.colidx[rows < g.colidx]
    if u.size == 0:
        return 0
    perms = np.array(list(itertools.permutations(range(g.n))), dtype=np.int16)
    # perms[p, vertex] = position
    return int(np.min(np.max(np.abs(perms[:, u] - perms[:, v]), axis=1)))


@pytest.mark.parametrize("seed", range(15))
def test_rcm_bandwidth_at_least_brute_force_minimum(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 8))
    g = I.erdos_renyi(n, float(rng.uniform(0.2, 0.7)), 1000 + seed)
    res = oracle.rcm(g.n, g.rowptr, g.colidx)
    assert res.stats["bandwidth_after"] >= _min_bandwidth(g)
    assert res.stats["bandwidth_after"] == _edge_bandwidth(g, res.perm)


@pytest.mark.parametrize("shape", [(2, 3), (2, 4), (3, 3)])
def test_rcm_optimal_on_small_grids(shape):
    g = I.grid2d(*shape, seed=7)
    res = oracle.rcm(g.n, g.rowptr, g.colidx)
    assert res.stats["bandwidth_after"] == _min_bandwidth(g) == min(shape)


# ---------------------------------------------------------------------------
# Level invariants of the labelling
# ---------------------------------------------------------------------------

def _components_of(g):
    return connected_components(_sp(g), directed=False)[1]


@pytest.mark.parametrize("seed", range(10))
def test_labelling_invariants(seed):
    rng = np.random.default_rng(seed)
    parts = [I.erdos_renyi(int(rng.integers(1, 40)), 0.08, seed * 10 + i) for i in range(3)]
    g = I.disjoint_union(parts, seed=seed)
    res = oracle.rcm(g.n, g.rowptr, g.colidx)
    n = g.n
    perm = res.perm
    assert sorted(perm.tolist()) == list(range(n))                 # a permutation
    assert np.array_equal(res.iperm[perm], np.arange(n))
    comp = _components_of(g)
    offs = list(res.comp_offset) + [n]
    assert len(offs) - 1 == comp.max() + 1 == res.stats["num_components"]
    A = _sp(g)
    deg = oracle.degrees(n, g.rowptr, g.colidx)
    for c in range(len(offs) - 1):
        block = perm[offs[c]:offs[c + 1]]
        # components are contiguous blocks, in increasing order of min id
        assert len(set(comp[block].tolist())) == 1
        if c > 0:
            assert block.min() > perm[offs[c - 1]:offs[c]].min()
        cm = block[::-1]                                  # the CM order
        root = int(res.comp_root[c])
        assert cm[0] == root
        dist = shortest_path(A, unweighted=True, indices=root)[cm]
        assert np.all(np.diff(dist) >= 0)                 # blocks = distance shells
        assert int(dist[-1]) + 1 == res.comp_levels[c]
        pos = {int(v): t for t, v in enumerate(cm)}
        keys = []
        for t, v in enumerate(cm):
            if t == 0:
                keys.append((dist[t], -1, 0, int(v)))
                continue
            nb = [w for w in g.colidx[g.rowptr[v]:g.rowptr[v + 1]] if w != v]
            par = min(pos[int(w)] for w in nb)
            # the parent lies in the previous level
            assert dist[par] == dist[t] - 1
            keys.append((dist[t], par, int(deg[v]), int(v)))
        # within a level: (parent label, degree, id) strictly increasing
        assert keys == sorted(keys)
        assert len(set(keys)) == len(keys)


@pytest.mark.parametrize("seed", range(30))
def test_algorithm3_equals_algorithm1(seed):
    """The level-synchronous matrix form (Algorithm 3) labels exactly like
    the serial queue (Algorithm 1)."""
    rng = np.random.default_rng(seed)
    kind = seed % 5
    if kind == 0:
        g = I.erdos_renyi(int(rng.integers(1, 80)), float(rng.uniform(0.01, 0.2)), seed)
    elif kind == 1:
        g = I.random_tree(int(rng.integers(1, 80)), seed)
    elif kind == 2:
        g = I.grid2d(int(rng.integers(1, 9)), int(rng.integers(1, 12)), seed=seed)
    elif kind == 3:
        g = I.add_random_self_loops(I.erdos_renyi(50, 0.05, seed), 0.3, seed)
    else:
        g = I.disjoint_union([I.cycle(int(rng.integers(3, 20)), seed=seed),
                              I.star(int(rng.integers(2, 12))),
                              I.path(int(rng.integers(1, 15)))], seed=seed)
    for variant in (0, 1):
        a = oracle.rcm(g.n, g.rowptr, g.colidx, pp_variant=variant, cm_mode=0)
        b = oracle.rcm(g.n, g.rowptr, g.colidx, pp_variant=variant, cm_mode=1)
        assert np.array_equal(a.perm, b.perm)
        assert a.stats == b.stats


@pytest.mark.parametrize("seed", range(20))
def test_reversal_never_increases_profile(seed):
    """Liu & Sherman (1976): reversing a Cuthill-McKee order never increases
    the envelope size, and the bandwidth is unchanged."""
    rng = np.random.default_rng(seed)
    g = I.erdos_renyi(int(rng.integers(5, 70)), float(rng.uniform(0.03, 0.2)), 500 + seed)
    res = oracle.rcm(g.n, g.rowptr, g.colidx)
    cm = np.empty_like(res.perm)
    offs = list(res.comp_offset) + [g.n]
    for c in range(len(offs) - 1):
        cm[offs[c]:offs[c + 1]] = res.perm[offs[c]:offs[c + 1]][::-1]
    bw_cm, prof_cm = oracle.bw_profile(g.n, g.rowptr, g.colidx, cm)
    assert res.stats["profile_after"] <= prof_cm
    assert res.stats["bandwidth_after"] == bw_cm


@pytest.mark.parametrize("seed", range(6))
def test_global_and_per_component_reversal_same_quality(seed):
    g = I.disjoint_union([I.erdos_renyi(30, 0.1, seed), I.grid2d(4, 5, seed=seed),
                          I.path(7)], seed=seed)
    a = oracle.rcm(g.n, g.rowptr, g.colidx, reverse_mode=0)
    b = oracle.rcm(g.n, g.rowptr, g.colidx, reverse_mode=1)
    assert a.stats == b.stats
    if a.stats["num_components"] > 1:
        assert not np.array_equal(a.perm, b.perm)
    assert np.array_equal(np.sort(a.perm), np.sort(b.perm))


# ---------------------------------------------------------------------------
# Section III-B: one ordering per component; disjoint unions
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(5))
def test_union_of_blocks_is_concatenation(seed):
    rng = np.random.default_rng(seed)
    parts = [I.grid2d(int(rng.integers(2, 7)), int(rng.integers(2, 7)), seed=seed + i)
             for i in range(4)]
    parts.append(I.complete(int(rng.integers(1, 6))))
    u = I.disjoint_union(parts)  # block ids in order, no relabelling
    whole = oracle.rcm(u.n, u.rowptr, u.colidx)
    off = 0
    pieces = []
    for p in parts:
        r = oracle.rcm(p.n, p.rowptr, p.colidx)
        pieces.append(r.perm + off)
        off += p.n
    assert np.array_equal(whole.perm, np.concatenate(pieces))


def test_isolated_vertices_and_empty():
    g = I.from_edges(5, np.zeros(0), np.zeros(0), diag=False)
    r = oracle.rcm(5, g.rowptr, g.colidx)
    assert r.perm.tolist() == [0, 1, 2, 3, 4]
    assert r.stats["num_components"] == 5
    assert r.stats["num_bfs"] == 10          # two level structures per singleton
    assert r.stats["num_levels"] == 5
    r = oracle.rcm(0, np.zeros(1, np.int32), np.zeros(0, np.int32))
    assert r.status == oracle.OK and r.perm.size == 0


# ---------------------------------------------------------------------------
# Fig. 2: a child attaches to the lower-labelled of its frontier neighbours
# ---------------------------------------------------------------------------

def test_fig2_child_takes_lowest_labelled_parent():
    """Hand-built instance of the rule illustrated in Fig. 2.  Root a has
    frontier children e and b with label(e) < label(b) (e has the lower
    degree); c is adjacent to both.  The (select2nd, min) product gives c the
    parent e, so c is labelled before f, b's only other child, although c's
    degree (2) is larger than f's (1).  If c took b as parent the level would
    be ordered by degree as (f, c)."""
    a, b, c, e, f = 0, 1, 2, 3, 4
    edges = [(a, b), (a, e), (b, c), (e, c), (b, f)]
    g = I.from_edges(5, np.array([x for x, _ in edges]), np.array([y for _, y in edges]))
    golden = open(__file__.replace("test_oracle_pins.py", "golden/fig2_rule.txt")).read().split()
    want_cm = [int(x) for x in golden[golden.index("cm_order_from_a:") + 1:][:5]]
    for mode in (0, 1):
        # labelling from the given root a (Algorithm 1 and Algorithm 3)
        lab = oracle.cm_from_root(g.n, g.rowptr, g.colidx, a, mode)
        assert lab.tolist() == want_cm == [a, e, b, c, f]
