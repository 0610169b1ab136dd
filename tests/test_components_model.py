"""A CPU model of the component search in paper_1610_08128_amd/csrc/rcm_prep.hip,
run under adversarial interleavings, to check the argument its comments make
for why the search needs no locks.

The kernels are modelled step by step: k_cc_init, k_cc_compress (flatten),
four k_cc_round contraction rounds (the first two capped at four row
entries), k_cc_pick (with 8 samples instead of 64,
so that the marked set varies more between graphs) and the exact hooking of
k_cc_link.  Every thread is a generator that yields after each memory
operation, and a seeded scheduler interleaves them at random.  Loads that the
kernels make through workgroup-scope atomics (which a cache may serve from an
older line) return, half of the time, any value the location has held since
the kernel began; agent-scope loads and compare-and-swap see the current
value.  A kernel boundary makes every store visible.

The expected result is the definition the search must meet: every vertex of
a component ends pointing at the component's lowest id (scipy's connected
components), and the vertices of the skipped set are left alone.  An edge
into the skipped set is reported.
"""

import random

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

from paper_1610_08128_amd import inputs as I

ROUNDS = 4
CAPPED_ROUNDS = 2  # the first rounds look at the first ROUND_CAP entries of a row
ROUND_CAP = 4
SAMPLES = 8


class Memory:
    def __init__(self, values):
        self.cur = list(values)
        self.seen = [[v] for v in self.cur]

    def kernel_start(self):
        self.seen = [[v] for v in self.cur]

    def store(self, i, v):
        self.cur[i] = v
        self.seen[i].append(v)

    def load_cached(self, i, rng):
        return rng.choice(self.seen[i]) if rng.random() < 0.5 else self.cur[i]

    def cas(self, i, expected, new):
        if self.cur[i] == expected:
            self.store(i, new)
            return True, expected
        return False, self.cur[i]


def _interleave(threads, rng):
    live = list(threads)
    while live:
        k = rng.randrange(len(live))
        try:
            next(live[k])
        except StopIteration:
            live[k] = live[-1]
            live.pop()


def _root_cached(P, x, rng):
    while True:
        p = P.load_cached(x, rng)
        yield
        if p == x:
            return x
        x = p


def _root_current(P, x):
    while True:
        p = P.cur[x]
        yield
        if p == x:
            return x
        x = p


def search(n, rowptr, colidx, seg, skip, rng):
    """Returns (parent after the final flattening, edge-into-skip flag)."""
    nbrs = [[int(v) for v in colidx[rowptr[u]:rowptr[u + 1]]] for u in range(n)]
    P = Memory(range(n))
    done = [0] * n
    pick = [0] * n
    err = False
    for u in range(n):  # k_cc_init: plain stores, no races
        m = u
        if not skip[u]:
            for v in nbrs[u]:
                if skip[v]:
                    err = True
                elif v < m:
                    m = v
        P.store(u, m)

    def flatten():
        P.kernel_start()

        def thread(i):
            r = yield from _root_current(P, i)
            P.store(i, r)
            yield

        _interleave([thread(i) for i in range(n)], rng)

    def contraction_round(cap):
        P.kernel_start()

        def thread(u):
            if done[u] or skip[u]:
                return
            pu = P.load_cached(u, rng)
            yield
            look = nbrs[u][:cap] if cap else nbrs[u]
            m, inside = pu, len(look) == len(nbrs[u])
            for v in look:
                if skip[v]:
                    continue
                pv = P.load_cached(v, rng)
                yield
                inside = inside and pv == pu
                m = min(m, pv)
            if inside:
                done[u] = 1
            if m < pu:
                still_root = P.load_cached(pu, rng) == pu
                yield
                if still_root:
                    P.cas(pu, pu, m)
                    yield

        _interleave([thread(u) for u in range(n)], rng)

    def exact_hooking():
        P.kernel_start()

        def thread(u):
            if done[u] or skip[u]:
                return
            pu = P.load_cached(u, rng)
            yield
            if pick[pu] or not nbrs[u]:
                return
            a = yield from _root_cached(P, u, rng)
            for v in nbrs[u]:
                if skip[v]:
                    continue
                b = yield from _root_cached(P, v, rng)
                if a == b:
                    continue
                a = yield from _root_cached(P, a, rng)
                while a != b:
                    if a < b:
                        a, b = b, a
                    ok, current = P.cas(a, a, b)
                    yield
                    if ok:
                        break
                    a = yield from _root_cached(P, current, rng)
                    b = yield from _root_cached(P, b, rng)

        _interleave([thread(u) for u in range(n)], rng)

    flatten()
    for r in range(ROUNDS):
        contraction_round(ROUND_CAP if r < CAPPED_ROUNDS else 0)
        flatten()
    for b, e in zip(seg[:-1], seg[1:]):  # k_cc_pick
        roots = []
        for j in range(SAMPLES):
            x = b + (e - b) * (2 * j + 1) // (2 * SAMPLES) if e > b else -1
            if x >= 0 and not skip[x]:
                roots.append(P.cur[x])
        if roots:
            pick[max(set(roots), key=lambda r: (roots.count(r), -r))] = 1
    exact_hooking()
    flatten()
    return P.cur, err


def _union(parts):
    """Disjoint union in global ids, one segment per part."""
    rows, cols, seg, base, nz = [], [], [0], 0, 0
    for g in parts:
        rows.append(g.rowptr[:-1] + nz)
        cols.append(g.colidx + base)
        base += g.n
        nz += g.nnz
        seg.append(base)
    rowptr = np.concatenate(rows + [np.array([nz])]).astype(np.int64)
    return base, rowptr, np.concatenate(cols).astype(np.int64), seg


def _lowest_ids(n, rowptr, colidx, skip):
    keep = np.nonzero(~skip)[0]
    A = sp.csr_matrix((np.ones(colidx.size), colidx, rowptr), shape=(n, n))
    A = A[keep][:, keep]
    nc, lab = connected_components(A, directed=False)
    want = np.arange(n)
    for c in range(nc):
        members = keep[lab == c]
        want[members] = members.min()
    return want


def _parts(seed):
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(int(rng.integers(1, 5))):
        kind = int(rng.integers(0, 5))
        if kind == 0:
            parts.append(I.grid2d(int(rng.integers(2, 9)), int(rng.integers(2, 9)), seed=seed + i))
        elif kind == 1:
            parts.append(I.rgg_patches(int(rng.integers(20, 90)), seed + i))
        elif kind == 2:
            parts.append(I.random_tree(int(rng.integers(1, 60)), seed + i))
        elif kind == 3:
            parts.append(I.erdos_renyi(int(rng.integers(2, 60)), 0.06, seed + i))
        else:
            parts.append(I.grid3d(int(rng.integers(2, 5)), int(rng.integers(2, 5)),
                                  int(rng.integers(2, 5)), seed=seed + i))
    return parts


@pytest.mark.parametrize("seed", range(40))
def test_batch_components_under_interleavings(seed):
    n, rowptr, colidx, seg = _union(_parts(seed))
    skip = np.zeros(n, bool)
    want = _lowest_ids(n, rowptr, colidx, skip)
    for schedule in range(4):
        got, err = search(n, rowptr, colidx, seg, skip, random.Random(seed * 100 + schedule))
        assert not err
        assert np.array_equal(np.array(got), want), (seed, schedule)


@pytest.mark.parametrize("seed", range(20))
def test_components_outside_a_skipped_set(seed):
    """The single-graph path: vertex 0's component is ordered first and
    skipped; one segment covers the whole graph."""
    parts = _parts(1000 + seed)
    g = I.disjoint_union(parts, seed=seed)
    n, rowptr, colidx = g.n, g.rowptr.astype(np.int64), g.colidx.astype(np.int64)
    A = sp.csr_matrix((np.ones(colidx.size), colidx, rowptr), shape=(n, n))
    _, lab = connected_components(A, directed=False)
    skip = lab == lab[0]
    want = _lowest_ids(n, rowptr, colidx, skip)
    for schedule in range(4):
        got, err = search(n, rowptr, colidx, [0, n], skip, random.Random(seed * 100 + schedule))
        assert not err
        got = np.array(got)
        assert np.array_equal(got[~skip], want[~skip]), (seed, schedule)


def test_edge_into_the_skipped_set_is_reported():
    # 1 -> 0 without 0 -> 1; {0, 2} is the skipped (already ordered) set
    rowptr = np.array([0, 1, 3, 4, 5])
    colidx = np.array([2, 0, 3, 0, 1])
    skip = np.array([True, False, True, False])
    _, err = search(4, rowptr, colidx, [0, 4], skip, random.Random(0))
    assert err


@pytest.mark.parametrize("seed", range(16))
def test_shuffled_rows_under_interleavings(seed):
    """Rows in a random order: the capped contraction rounds then see an
    arbitrary subset of each row, which must not change the result."""
    parts = [I.shuffle_rows(p, seed + i) for i, p in enumerate(_parts(2000 + seed))]
    n, rowptr, colidx, seg = _union(parts)
    skip = np.zeros(n, bool)
    want = _lowest_ids(n, rowptr, colidx, skip)
    for schedule in range(3):
        got, err = search(n, rowptr, colidx, seg, skip, random.Random(seed * 100 + schedule))
        assert not err
        assert np.array_equal(np.array(got), want), (seed, schedule)
    g = I.shuffle_rows(I.disjoint_union(_parts(3000 + seed), seed=seed), seed)
    n, rowptr, colidx = g.n, g.rowptr.astype(np.int64), g.colidx.astype(np.int64)
    A = sp.csr_matrix((np.ones(colidx.size), colidx, rowptr), shape=(n, n))
    _, lab = connected_components(A, directed=False)
    skip = lab == lab[0]
    want = _lowest_ids(n, rowptr, colidx, skip)
    got, err = search(n, rowptr, colidx, [0, n], skip, random.Random(seed))
    assert not err
    assert np.array_equal(np.array(got)[~skip], want[~skip])
