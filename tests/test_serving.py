"""The request-serving engine: every served result equals the oracle's (and
so the single-call library's) for the same pattern alone; admission keeps
the device memory in flight within the budget; a malformed request fails
alone while the requests batched with it succeed."""

import sys
import threading

import numpy as np
import pytest

import oracle
from paper_1610_08128_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _mixed_requests(seed, count):
    """Requests of mixed kinds and sizes (several components, self loops)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        kind = int(rng.integers(0, 6))
        s = int(rng.integers(0, 2**31 - 1))
        if kind == 0:
            g = I.grid2d(int(rng.integers(2, 120)), int(rng.integers(2, 120)), seed=s)
        elif kind == 1:
            a = int(rng.integers(2, 24))
            g = I.grid3d(a, a, int(rng.integers(2, 30)), seed=s)
        elif kind == 2:
            g = I.rgg_patches(int(rng.integers(50, 6000)), s)
        elif kind == 3:
            g = I.disjoint_union([I.erdos_renyi(int(rng.integers(5, 300)), 0.02, s),
                                  I.random_tree(int(rng.integers(1, 300)), s + 1), I.path(1)],
                                 seed=s)
        elif kind == 4:
            g = I.add_random_self_loops(I.random_tree(int(rng.integers(2, 2000)), s), 0.3, s)
        else:
            g = I.path(int(rng.integers(1, 50)), seed=s)
        out.append(g)
    return out


def _expect(g):
    want = oracle.rcm(g.n, g.rowptr, g.colidx)
    assert want.status == oracle.OK
    return want


def test_served_results_equal_oracle_alone():
    from paper_1610_08128_amd.serve import Server

    graphs = _mixed_requests(11, 60)
    _say(f"serving {len(graphs)} mixed requests")
    with Server(mem_budget_bytes=256 << 20, max_batch=16, executors=2) as srv:
        tickets = [srv.submit(g.rowptr, g.colidx) for g in graphs]
        for g, t in zip(graphs, tickets):
            perm, info = srv.wait(t, timeout_ms=60000)
            want = _expect(g)
            assert info["status"] == 0, info
            assert np.array_equal(perm, want.perm), g.name
            assert info["stats"] == want.stats, (g.name, info["stats"], want.stats)
            assert info["t_submit"] <= info["t_admit"] <= info["t_done"]
        c = srv.counters()
    _say(f"counters {c}")
    assert c["completed"] == len(graphs) and c["failed"] == 0
    assert c["max_batch_seen"] > 1  # requests were batched
    assert c["bytes_in_flight"] == 0


def test_admission_respects_the_memory_budget():
    from paper_1610_08128_amd.serve import Server, request_bytes

    graphs = _mixed_requests(12, 24) + [I.grid2d(300, 300, seed=5)]
    big = max(request_bytes(g.n, g.nnz) for g in graphs)
    budget = int(big * 1.3)
    too_big = I.grid3d(80, 80, 80, seed=6)
    assert request_bytes(too_big.n, too_big.nnz) > budget
    _say(f"budget {budget} bytes, largest request {big} bytes")
    with Server(mem_budget_bytes=budget, max_batch=8, executors=3) as srv:
        tickets = [srv.submit(g.rowptr, g.colidx) for g in graphs]
        t_big = srv.submit(too_big.rowptr, too_big.colidx)
        perm, info = srv.wait(t_big, timeout_ms=60000)
        assert perm is None and info["status"] == 5  # RCM_ERR_OUT_OF_MEMORY, alone
        for g, t in zip(graphs, tickets):
            perm, info = srv.wait(t, timeout_ms=60000)
            assert info["status"] == 0
            assert np.array_equal(perm, _expect(g).perm), g.name
        c = srv.counters()
    _say(f"counters {c}")
    assert c["peak_bytes_in_flight"] <= budget
    assert c["failed"] == 1


def test_malformed_request_fails_alone():
    from paper_1610_08128_amd.serve import Server

    good = _mixed_requests(13, 12)
    # column out of range
    bad_col = (np.array([0, 2, 3, 4], np.int32), np.array([1, 7, 0, 1], np.int32))
    # edge 0 -> 1 without 1 -> 0
    asym = (np.array([0, 2, 3, 4], np.int32), np.array([0, 1, 1, 2], np.int32))
    # rowptr ends disagree with the entries handed over
    bad_ends = (np.array([0, 1, 5], np.int32), np.array([1, 0], np.int32))
    with Server(mem_budget_bytes=128 << 20, max_batch=32, executors=1) as srv:
        tickets = [srv.submit(g.rowptr, g.colidx) for g in good[:6]]
        t_col = srv.submit(*bad_col)
        t_asym = srv.submit(*asym)
        t_ends = srv.submit(*bad_ends)
        tickets += [srv.submit(g.rowptr, g.colidx) for g in good[6:]]
        for t, code in ((t_col, 2), (t_asym, 3), (t_ends, 2)):
            perm, info = srv.wait(t, timeout_ms=60000)
            assert perm is None and info["status"] == code, info
        for g, t in zip(good, tickets):
            perm, info = srv.wait(t, timeout_ms=60000)
            assert info["status"] == 0, (g.name, info)
            assert np.array_equal(perm, _expect(g).perm), g.name
        c = srv.counters()
    _say(f"counters {c}")
    assert c["failed"] == 3
    assert c["retried_alone"] > 0


def test_concurrent_submitters_and_repeated_requests():
    from paper_1610_08128_amd.serve import Server

    graphs = _mixed_requests(14, 16)
    wants = [_expect(g).perm for g in graphs]
    errors = []

    def client(k):
        try:
            for rep in range(3):
                i = (k * 5 + rep) % len(graphs)
                t = srv.submit(graphs[i].rowptr, graphs[i].colidx)
                perm, info = srv.wait(t, timeout_ms=60000)
                if info["status"] != 0 or not np.array_equal(perm, wants[i]):
                    errors.append((k, rep, i, info["status"]))
        except Exception as e:  # pragma: no cover - reported below
            errors.append(repr(e))

    with Server(mem_budget_bytes=256 << 20, executors=2) as srv:
        threads = [threading.Thread(target=client, args=(k,)) for k in range(6)]
        for th in threads:
            th.start()
        for th in threads:
            th.join()
        c = srv.counters()
    _say(f"counters {c}")
    assert not errors, errors
    assert c["completed"] == 18


def test_served_team_path_and_large_requests():
    """Requests above the batched small-component cutoff (teams of
    work-groups, cooperative launches from two executors' streams) and
    requests of the serving workload's large end (at least 5M entries),
    mixed with small ones; every result and its statistics equal the
    oracle's for the same pattern alone."""
    from paper_1610_08128_amd.serve import Server

    big = [I.grid3d(100, 100, 100, seed=21),                 # 6.9M entries
           I.shuffle_rows(I.grid2d(1100, 1000, seed=22), 3),  # 5.5M entries, rows shuffled
           I.rgg_patches(420_000, 23)]                       # about 5.5M entries
    team = [I.grid2d(300, 300, seed=24), I.grid3d(70, 70, 70, seed=25),
            I.rgg_patches(90_000, 26), I.grid2d(400, 260, seed=27)]
    small = _mixed_requests(15, 20)
    graphs = []
    for i in range(max(len(big), len(team), len(small))):
        for lst in (small, team, big, small):
            if i < len(lst):
                graphs.append(lst[i])
    assert any(g.nnz >= 5_000_000 for g in graphs)
    assert sum(g.n > 65536 for g in graphs) >= 4
    _say(f"serving {len(graphs)} requests, largest {max(g.nnz for g in graphs)} entries")
    wants = [_expect(g) for g in graphs]
    with Server(mem_budget_bytes=4 << 30, max_batch=8, executors=2) as srv:
        tickets = [srv.submit(g.rowptr, g.colidx) for g in graphs]
        for g, t, want in zip(graphs, tickets, wants):
            perm, info = srv.wait(t, timeout_ms=120000)
            assert info["status"] == 0, (g.name, info)
            assert np.array_equal(perm, want.perm), g.name
            assert info["stats"] == want.stats, (g.name, info["stats"], want.stats)
        c = srv.counters()
    _say(f"counters {c}")
    assert c["completed"] == len(graphs) and c["failed"] == 0
