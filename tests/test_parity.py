"""GPU parity: the HIP library's permutation and statistics equal the CPU
oracle's bit for bit (the ordering is integer work; every tie is broken by a
fixed rule, so the result is unique)."""

import os
import sys

import numpy as np
import pytest

import oracle
from paper_1610_08128_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# options that only the persistent team kernel reads: a test that sets them
# means that kernel (mode 1), not the one-work-group engine small graphs
# take by default
TEAM_OPTIONS = {"small_cutoff", "team_size", "narrow_cutoff", "block_threads", "label_team",
                "search_round", "async_search", "rebalance_levels", "max_teams",
                "small_threads"}


def _with_mode(opts):
    if "mode" not in opts and TEAM_OPTIONS & set(opts):
        opts = dict(opts, mode=1)
    return opts


def gpu_order(g, **opts):
    import torch
    from paper_1610_08128_amd import rcm

    opts = _with_mode(opts)

    rp = torch.from_numpy(g.rowptr).cuda()
    ci = torch.from_numpy(g.colidx if g.colidx.size else np.zeros(1, np.int32)).cuda()
    perm, iperm, st = rcm.order(rp, ci, return_iperm=True, **opts)
    torch.cuda.synchronize()
    return perm.cpu().numpy(), iperm.cpu().numpy(), st


# the library's label_mode and the oracle's cm_mode for the same order
CM_MODE = {0: 0, 1: 2, 2: 3}


def check(g, *, pp_variant=0, reverse_mode=0, label_mode=0, **gpu_opts):
    _say(f"case {g.name} n={g.n} nnz={g.nnz} pp={pp_variant} rev={reverse_mode} "
         f"label={label_mode} {gpu_opts}")
    want = oracle.rcm(g.n, g.rowptr, g.colidx, pp_variant=pp_variant, reverse_mode=reverse_mode,
                      cm_mode=CM_MODE[label_mode])
    assert want.status == oracle.OK
    perm, iperm, st = gpu_order(g, pp_variant=pp_variant, reverse_mode=reverse_mode,
                                label_mode=label_mode, **gpu_opts)
    if not np.array_equal(perm, want.perm):
        bad = np.nonzero(perm != want.perm)[0]
        raise AssertionError(f"perm differs at {bad.size} positions, first {bad[:10]}: "
                             f"gpu {perm[bad[:10]]} oracle {want.perm[bad[:10]]}")
    assert np.array_equal(iperm, want.iperm)
    assert st == want.stats, (st, want.stats)
    return st


def _tiny_graphs():
    gs = [I.path(1), I.path(2), I.path(3), I.path(7, seed=1), I.complete(2), I.complete(6),
          I.star(9, 4), I.cycle(8, seed=3), I.grid2d(3, 3, seed=2), I.grid2d(4, 9),
          I.grid2d(5, 12, seed=5), I.random_tree(40, 3), I.drop_diagonal(I.grid2d(4, 4, seed=1)),
          I.add_random_self_loops(I.erdos_renyi(30, 0.1, 4), 0.4, 4),
          I.from_edges(6, np.zeros(0), np.zeros(0), diag=False),
          I.disjoint_union([I.path(3), I.complete(4), I.path(1), I.cycle(5)], seed=9)]
    a, b, c, e, f = 0, 1, 2, 3, 4
    gs.append(I.from_edges(5, np.array([a, a, b, e, b]), np.array([b, e, c, c, f])))
    for i, g in enumerate(gs):
        g.name = g.name or f"tiny{i}"
    return gs


@pytest.mark.parametrize("idx", range(17))
@pytest.mark.parametrize("mode", [0, 1])
def test_tiny_graphs(idx, mode):
    """mode 0 takes the one-work-group LDS engine for graphs this small, mode
    1 the persistent team kernel."""
    g = _tiny_graphs()[idx]
    for pp in (0, 1):
        for rev in (0, 1):
            check(g, pp_variant=pp, reverse_mode=rev, mode=mode)


def _random_graph(seed):
    rng = np.random.default_rng(seed)
    parts = []
    for i in range(int(rng.integers(1, 5))):
        kind = int(rng.integers(0, 5))
        if kind == 0:
            parts.append(I.erdos_renyi(int(rng.integers(1, 300)), float(rng.uniform(0.003, 0.05)),
                                       seed * 7 + i))
        elif kind == 1:
            parts.append(I.grid2d(int(rng.integers(1, 30)), int(rng.integers(1, 30)),
                                  seed=seed + i))
        elif kind == 2:
            parts.append(I.random_tree(int(rng.integers(1, 200)), seed + i))
        elif kind == 3:
            parts.append(I.grid3d(int(rng.integers(1, 8)), int(rng.integers(1, 8)),
                                  int(rng.integers(1, 8)), seed=seed + i))
        else:
            parts.append(I.rgg_patches(int(rng.integers(20, 400)), seed + i))
    g = I.disjoint_union(parts, seed=seed)
    if seed % 3 == 1:
        g = I.add_random_self_loops(g, 0.2, seed)
    g.name = f"random{seed}"
    return g


@pytest.mark.parametrize("seed", range(24))
@pytest.mark.parametrize("mode", [0, 1])
def test_random_graphs_small_path(seed, mode):
    g = _random_graph(seed)
    check(g, pp_variant=seed % 2, reverse_mode=(seed // 2) % 2, mode=mode)


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("team,narrow", [(1, 0), (2, -1), (8, -1), (8, 16), (4, 4096)])
def test_random_graphs_team_path(seed, team, narrow):
    """small_cutoff=1 sends every non-isolated component to the team path;
    narrow_cutoff moves levels between the whole team and its first
    work-group."""
    g = _random_graph(100 + seed)
    check(g, small_cutoff=1, team_size=team, block_threads=256, narrow_cutoff=narrow)


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_grid_64x64(seed):
    g = I.config(0, seed=seed)
    st = check(g)
    assert st["bandwidth_after"] == 64 and st["profile_after"] == 176736
    check(g, mode=2)
    check(g, mode=1)
    check(g, small_cutoff=1)


@pytest.mark.parametrize("team,threads,narrow", [(32, 512, 0), (4, 512, -1), (16, 256, 1024),
                                                 (8, 512, 100000)])
def test_grid_128_cubed(team, threads, narrow):
    g = I.config(1)
    check(g, team_size=team, block_threads=threads, narrow_cutoff=narrow)


def test_strip_32x500000():
    """The strip at full size: renumbered after its first level structure
    and finished by the window engine (used_mode 4), both variants."""
    from paper_1610_08128_amd import rcm

    g = I.config(2)
    check(g)
    assert rcm.last_timings()["used_mode"] == 4
    check(g, pp_variant=1, reverse_mode=1)
    assert rcm.last_timings()["used_mode"] == 4


@pytest.mark.parametrize("case", range(4))
def test_head_component_shapes(case):
    """The component of vertex 0 is ordered before the component search;
    cover it being isolated, small, the largest, and the only component."""
    if case == 0:
        g = I.disjoint_union([I.path(1), I.grid2d(40, 50, seed=3), I.complete(5)])
    elif case == 1:
        g = I.disjoint_union([I.path(3), I.grid3d(12, 12, 12, seed=4), I.path(1), I.cycle(9)])
    elif case == 2:
        g = I.disjoint_union([I.grid2d(60, 70, seed=5), I.path(1), I.path(1), I.star(7)])
    else:
        g = I.grid2d(33, 65, seed=6)
    g.name = f"head{case}"
    check(g)
    check(g, reverse_mode=1, pp_variant=1)
    check(g, small_cutoff=1, team_size=4)


def test_repeated_runs_identical():
    g = I.config(0, seed=11)
    first = gpu_order(g)[0]
    for team in (1, 2, 3, 8):
        for _ in range(2):
            assert np.array_equal(gpu_order(g, small_cutoff=1, team_size=team)[0], first)
    assert np.array_equal(gpu_order(g, small_cutoff=1 << 20)[0], first)


def test_status_codes_on_gpu():
    import torch
    from paper_1610_08128_amd import rcm

    g = I.path(6)
    bad = g.colidx.copy()
    bad[2] = 6
    with pytest.raises(rcm.RcmError) as e:
        rcm.order(torch.from_numpy(g.rowptr).cuda(), torch.from_numpy(bad).cuda())
    assert e.value.status == rcm.ERR_BAD_CSR
    badr = g.rowptr.copy()
    badr[3] = badr[2] - 1
    with pytest.raises(rcm.RcmError) as e:
        rcm.order(torch.from_numpy(badr).cuda(), torch.from_numpy(g.colidx).cuda())
    assert e.value.status == rcm.ERR_BAD_CSR
    # a duplicated entry (0, 1) that keeps the pattern symmetric as a set:
    # malformed with or without the full check
    rp = np.array([0, 3, 6, 8], np.int32)
    ci = np.array([0, 1, 1, 0, 1, 2, 1, 2], np.int32)
    assert oracle.validate(3, rp, ci, False) == oracle.ERR_BAD_CSR
    for full in (False, True):
        with pytest.raises(rcm.RcmError) as e:
            rcm.order(torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(), check_full=full)
        assert e.value.status == rcm.ERR_BAD_CSR
    # an asymmetric pattern without the full check: the traversal notices that
    # it leaves a component and reports it instead of writing out of bounds
    # (row 0 of the path loses its entry (0, 1); no row repeats a column)
    rp = np.array([0, 1, 4, 6, 8, 10, 12], np.int32)
    ci = np.array([0, 0, 1, 2, 2, 3, 3, 4, 4, 5, 4, 5], np.int32)
    assert oracle.validate(6, rp, ci, False) == oracle.OK
    assert oracle.validate(6, rp, ci, True) == oracle.ERR_NOT_SYMMETRIC
    with pytest.raises(rcm.RcmError) as e:
        rcm.order(torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda())
    assert e.value.status == rcm.ERR_NOT_SYMMETRIC
    rp = np.array([0, 2, 3, 4, 5, 6], np.int32)
    ci = np.array([0, 4, 1, 2, 3, 4], np.int32)
    with pytest.raises(rcm.RcmError) as e:
        rcm.order(torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(), check_full=True)
    assert e.value.status == rcm.ERR_NOT_SYMMETRIC
    assert oracle.validate(5, rp, ci, True) == oracle.ERR_NOT_SYMMETRIC
    # vertex 1 points into vertex 0's component {0, 2} without the way back:
    # the ordering of that component never reaches 1, and the component
    # search of the rest reports the edge, without the full check
    rp = np.array([0, 1, 3, 4, 5], np.int32)
    ci = np.array([2, 0, 3, 0, 1], np.int32)
    assert oracle.validate(4, rp, ci, True) == oracle.ERR_NOT_SYMMETRIC
    with pytest.raises(rcm.RcmError) as e:
        rcm.order(torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda())
    assert e.value.status == rcm.ERR_NOT_SYMMETRIC


def test_caller_workspace_and_stream():
    import torch
    from paper_1610_08128_amd import rcm

    g = I.config(0, seed=3)
    want = oracle.rcm(g.n, g.rowptr, g.colidx)
    nbytes = rcm.workspace_bytes(g.n, g.nnz)
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    rp = torch.from_numpy(g.rowptr).cuda()
    ci = torch.from_numpy(g.colidx).cuda()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        perm, st = rcm.order(rp, ci, workspace=ws)
    s.synchronize()
    assert np.array_equal(perm.cpu().numpy(), want.perm)
    small = torch.empty(nbytes - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(rcm.RcmError) as e:
        rcm.order(rp, ci, workspace=small)
    assert e.value.status == rcm.ERR_WORKSPACE_TOO_SMALL


def _check_batch(graphs, **opts):
    import torch
    from paper_1610_08128_amd import rcm

    vo, no, rp, ci = I.concat_batch(graphs)
    opts = _with_mode(opts)
    _say(f"batch of {len(graphs)} graphs, {vo[-1]} vertices, {no[-1]} nnz {opts}")
    perm, stats = rcm.order_batched(vo, no, torch.from_numpy(rp).cuda(),
                                    torch.from_numpy(ci).cuda(), **opts)
    perm = perm.cpu().numpy()
    for i, g in enumerate(graphs):
        want = oracle.rcm(g.n, g.rowptr, g.colidx, pp_variant=opts.get("pp_variant", 0),
                          reverse_mode=opts.get("reverse_mode", 0),
                          cm_mode=CM_MODE[opts.get("label_mode", 0)])
        assert np.array_equal(perm[vo[i]:vo[i + 1]], want.perm), f"graph {i}"
        assert stats[i] == want.stats, (i, stats[i], want.stats)


def test_batched_small():
    graphs = [_random_graph(200 + i) for i in range(10)] + [I.path(1), I.complete(5)]
    _check_batch(graphs)
    _check_batch(graphs, reverse_mode=1, pp_variant=1)
    _check_batch(graphs, small_cutoff=1, team_size=4)


@pytest.mark.parametrize("where", ["past_end", "before_start"])
def test_batched_column_outside_its_graph(where):
    """A column index outside its own graph becomes, in the union's ids, a
    vertex of the neighbouring graph: still in range, so only the check that
    every row stays inside its graph rejects it."""
    import torch
    from paper_1610_08128_amd import rcm

    graphs = [I.grid2d(5, 6, seed=1), I.path(7, seed=3), I.grid2d(4, 4, seed=2)]
    vo, no, rp, ci = I.concat_batch(graphs)
    bad = ci.copy()
    if where == "past_end":
        bad[no[2] - 1] = graphs[1].n  # last entry of graph 1's last row
    else:
        bad[no[1]] = -1  # first entry of graph 1's first row
    _say(f"batch with a column outside graph 1 ({where})")
    with pytest.raises(rcm.RcmError) as e:
        rcm.order_batched(vo, no, torch.from_numpy(rp).cuda(), torch.from_numpy(bad).cuda())
    assert e.value.status == rcm.ERR_BAD_CSR


def test_batched_concurrent_teams():
    # several large-component teams in one cooperative launch, tasks taken
    # largest first; single-work-group teams with 512 threads
    graphs = [I.grid2d(20 + 3 * i, 30, seed=300 + i) for i in range(11)]
    graphs += [I.rgg_patches(3000, seed=77), I.path(2)]
    _check_batch(graphs, small_cutoff=500, team_size=4, max_teams=8)
    _check_batch(graphs, small_cutoff=500, team_size=32, max_teams=3, narrow_cutoff=16)
    _check_batch(graphs, small_threads=512)
    _check_batch(graphs, small_cutoff=1 << 30, small_threads=512)


def test_batched_512():
    graphs = I.batch_graphs(512, seed=4)
    _check_batch(graphs)


def test_batched_components_repeated():
    """The component search of a batch hooks roots from many work-groups at
    once; mid-size relabelled grids and random geometric patches give it many
    roots to merge.  Several calls on one workspace must all agree with the
    oracle (a union lost to a race splits a component, which the ordering
    reports as an unsymmetric pattern)."""
    import torch
    from paper_1610_08128_amd import rcm

    graphs = I.batch_graphs(64, seed=12, lo=2e4, hi=2e5)
    vo, no, rp, ci = I.concat_batch(graphs)
    want = [oracle.rcm(g.n, g.rowptr, g.colidx) for g in graphs]
    rpd, cid = torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda()
    ws = torch.empty(rcm.batched_workspace_bytes(len(graphs), int(vo[-1]), int(no[-1])),
                     dtype=torch.uint8, device="cuda")
    for call in range(4):
        _say(f"batch of {len(graphs)} graphs, {vo[-1]} vertices, call {call}")
        perm, stats = rcm.order_batched(vo, no, rpd, cid, workspace=ws)
        perm = perm.cpu().numpy()
        for i, w in enumerate(want):
            assert np.array_equal(perm[vo[i]:vo[i + 1]], w.perm), (call, i)
            assert stats[i] == w.stats, (call, i)


# ---------------------------------------------------------------------------
# Level orders (label_mode 1: no sort, 2: one global sort at the end)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("idx", range(17))
@pytest.mark.parametrize("label_mode", [1, 2])
def test_level_orders_tiny(idx, label_mode):
    g = _tiny_graphs()[idx]
    for pp in (0, 1):
        for rev in (0, 1):
            check(g, pp_variant=pp, reverse_mode=rev, label_mode=label_mode)


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("label_mode", [1, 2])
def test_level_orders_random(seed, label_mode):
    g = _random_graph(400 + seed)
    check(g, pp_variant=seed % 2, reverse_mode=(seed // 2) % 2, label_mode=label_mode)
    check(g, label_mode=label_mode, small_cutoff=1, team_size=1 + seed % 8, narrow_cutoff=16)


@pytest.mark.parametrize("label_mode", [1, 2])
def test_level_orders_grids(label_mode):
    check(I.config(0, seed=3), label_mode=label_mode)
    check(I.config(0, seed=3), label_mode=label_mode, small_cutoff=1)
    # the 128^3 grid at full size, in the benchmark's launch configuration
    check(I.config(1), label_mode=label_mode)
    check(I.config(1), label_mode=label_mode, pp_variant=1, reverse_mode=1)


def test_level_orders_batched():
    graphs = [_random_graph(500 + i) for i in range(8)] + [I.path(1), I.complete(5)]
    graphs += [I.grid2d(20 + 3 * i, 30, seed=600 + i) for i in range(4)]
    for label_mode in (1, 2):
        _check_batch(graphs, label_mode=label_mode)
        _check_batch(graphs, label_mode=label_mode, small_cutoff=500, team_size=4,
                     pp_variant=1, reverse_mode=1)


# ---------------------------------------------------------------------------
# Asynchronous (label-correcting) search passes: same results
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(10))
def test_async_search_random(seed):
    g = _random_graph(700 + seed)
    check(g, async_search=1, small_cutoff=1, team_size=2 + seed % 7, pp_variant=seed % 2,
          reverse_mode=(seed // 2) % 2)
    check(g, async_search=1, small_cutoff=1, team_size=8, search_round=1 + seed % 4,
          rebalance_levels=1 + seed % 3, narrow_cutoff=16, label_mode=seed % 3)


def test_async_search_grids():
    check(I.config(0, seed=4), async_search=1, small_cutoff=1)
    check(I.config(0, seed=4), async_search=1, small_cutoff=1, team_size=3, search_round=2)
    # the 128^3 grid at full size, in the benchmark's launch configuration
    check(I.config(1), async_search=1)
    check(I.config(1), async_search=1, label_mode=2)
    check(I.config(1), async_search=1, pp_variant=1, reverse_mode=1, search_round=3,
          team_size=200, label_team=40)


def test_async_search_batched():
    graphs = [_random_graph(800 + i) for i in range(6)] + [I.path(1), I.complete(5)]
    graphs += [I.grid2d(40 + 5 * i, 30, seed=900 + i) for i in range(3)]
    _check_batch(graphs, async_search=1, small_cutoff=500, team_size=4)
    _check_batch(graphs, async_search=1, small_cutoff=500, team_size=4, label_mode=1,
                 pp_variant=1, reverse_mode=1)


@pytest.mark.parametrize("seed", range(6))
def test_level_synchronous_search(seed):
    """The level-synchronous search passes (async_search=-1) on the team path."""
    g = _random_graph(1000 + seed)
    check(g, async_search=-1, small_cutoff=1, team_size=2 + seed, narrow_cutoff=16 * seed,
          pp_variant=seed % 2, label_mode=seed % 3)


@pytest.mark.parametrize("team,threads,narrow", [(64, 256, 0), (16, 512, 1024)])
def test_level_synchronous_grid_128_cubed(team, threads, narrow):
    check(I.config(1), async_search=-1, team_size=team, block_threads=threads,
          narrow_cutoff=narrow)


# ---------------------------------------------------------------------------
# The fixed-stride row copy of graphs whose rows have at most 8 entries: the
# asynchronous search passes load a reached neighbour's row with its atomic
# ---------------------------------------------------------------------------

def _king_graph(k, m, *, diag, seed):
    """k x m grid with the 8 king-move neighbours: rows of exactly 8 entries
    inside (9 with the diagonal), so the copy's width is met exactly or
    exceeded."""
    idx = np.arange(k * m, dtype=np.int64).reshape(k, m)
    us = [idx[:-1, :].ravel(), idx[:, :-1].ravel(), idx[:-1, :-1].ravel(), idx[:-1, 1:].ravel()]
    vs = [idx[1:, :].ravel(), idx[:, 1:].ravel(), idx[1:, 1:].ravel(), idx[1:, :-1].ravel()]
    perm = np.random.default_rng(seed).permutation(k * m)
    return I.from_edges(k * m, np.concatenate(us), np.concatenate(vs), diag=diag, perm=perm,
                        name=f"king_{k}x{m}_diag{int(diag)}")


def _with_hub(g, hub, degree, seed):
    """g plus edges from `hub` to `degree` random vertices: one row longer
    than the copy's width, so the copy is not used."""
    u, v, diag = I._edges_of(g)
    rng = np.random.default_rng(seed)
    others = rng.choice(np.setdiff1d(np.arange(g.n), [hub]), size=degree, replace=False)
    u = np.concatenate([u, np.full(degree, hub, dtype=np.int64)])
    v = np.concatenate([v, others.astype(np.int64)])
    return I.from_edges(g.n, u, v, diag=diag, name=f"{g.name}_hub{degree}")


def _row_copy_graphs():
    return [I.grid3d(24, 20, 18, seed=61), I.grid2d(90, 70, seed=62),
            I.drop_diagonal(I.grid3d(16, 16, 16, seed=63)), I.strip_drop(8, 3000, 0.02, 64),
            _king_graph(60, 50, diag=False, seed=65), _king_graph(40, 45, diag=True, seed=66),
            _with_hub(I.grid3d(20, 20, 20, seed=67), 5, 9, 68),
            I.shuffle_rows(I.grid3d(18, 22, 16, seed=69), 70)]


def _hub_graphs():
    """Hubs whose children outnumber what one thread ranks: a star of 20,001
    (its children sort outside LDS), 8,193 and 700, a wheel-like hub over a
    cycle, and a hub joined to a grid, each relabelled."""
    hub = np.zeros(3000, np.int64)
    rim = np.arange(1, 3001, dtype=np.int64)
    wheel = I.from_edges(3001, np.concatenate([hub, rim[:-1]]), np.concatenate([rim, rim[1:]]),
                         perm=np.random.default_rng(81).permutation(3001), name="wheel_3001")
    return [I.relabel(I.star(20001), 82)[0], I.relabel(I.star(8193), 83)[0],
            I.relabel(I.star(700), 84)[0], wheel,
            _with_hub(I.grid2d(60, 70, seed=85), 7, 2500, 86)]


@pytest.mark.parametrize("team", [1, 4, 64])
def test_hub_children_placed_by_the_work_group(team):
    """Parity where one parent has thousands of children on a long row, on
    a work-group alone and on teams, in both search variants."""
    for i, g in enumerate(_hub_graphs()):
        check(g, small_cutoff=1 if team > 1 else 1 << 30, team_size=team, pp_variant=i % 2)


def test_engine_hub_rows():
    """The one-work-group engine on graphs where one parent has thousands of
    children (the wave collects and sorts them in their label range): stars
    up to the engine's LDS limit, a wheel, a hub on a grid."""
    gs = [I.relabel(I.star(2000), 91)[0], I.relabel(I.star(8000), 92)[0]] + _hub_graphs()[2:]
    for g in gs:
        check(g, mode=2)
        check(g, mode=2, pp_variant=1, reverse_mode=1)


def test_batched_hub_rows():
    _check_batch([I.star(9000), I.grid2d(40, 50, seed=87), I.relabel(I.star(3000), 88)[0],
                  I.path(9)], small_cutoff=100)


@pytest.mark.parametrize("copy", ["1", "0"])
def test_row_copy_team_path(copy, monkeypatch):
    """Parity on the team path with the copy on and off (RCM_ELL): bounded
    rows (with and without the diagonal, rows of exactly 8 entries, a strip
    with dropped edges, rows in any order), rows too long for the copy, and
    launch shapes that make records superseded often (small teams, long
    rounds, the work-group shuffle)."""
    monkeypatch.setenv("RCM_ELL", copy)
    for i, g in enumerate(_row_copy_graphs()):
        check(g, async_search=1, small_cutoff=1, team_size=2 + i, search_round=1 + 3 * i,
              shuffle_seed=100 + i)
        check(g, async_search=1, small_cutoff=1, team_size=64, pp_variant=1, reverse_mode=1,
              label_mode=i % 3)


def test_row_copy_full_size_grid_both_ways(monkeypatch):
    """The 128^3 grid in the benchmark's launch configuration with and
    without the copy: the same ordering."""
    g = I.config(1)
    for copy in ("1", "0"):
        monkeypatch.setenv("RCM_ELL", copy)
        check(g, async_search=1)


# ---------------------------------------------------------------------------
# Rows in any order, rows without a diagonal (the interface promises both)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("idx", range(17))
def test_tiny_graphs_shuffled_rows(idx):
    g = I.shuffle_rows(_tiny_graphs()[idx], 50 + idx)
    check(g)
    check(g, pp_variant=1, reverse_mode=1)
    check(g, small_cutoff=1, team_size=3, narrow_cutoff=-1)


@pytest.mark.parametrize("seed", range(10))
def test_random_graphs_shuffled_rows(seed):
    """Shuffled rows on the single-work-group path and on the team path (the
    component search's capped contraction rounds read only the first row
    entries, whichever they are)."""
    g = I.shuffle_rows(_random_graph(1200 + seed), seed)
    check(g, pp_variant=seed % 2, reverse_mode=(seed // 2) % 2)
    check(g, small_cutoff=1, team_size=2 + seed % 7, narrow_cutoff=16 * (seed % 3),
          async_search=1 - 2 * (seed % 2))
    h = I.shuffle_rows(I.drop_diagonal(_random_graph(1300 + seed)), seed)
    check(h)
    check(h, small_cutoff=1, team_size=4, label_mode=seed % 3)


def test_grid_128_cubed_shuffled_rows():
    """The 3D grid at full size in the benchmark's launch configuration, with
    each row in a random order."""
    check(I.shuffle_rows(I.config(1), 7))


def test_grid_128_cubed_without_diagonal():
    """No row holds its diagonal entry (degree = row length), rows shuffled,
    at full size; also on teams of 64 with the level-synchronous search."""
    g = I.shuffle_rows(I.drop_diagonal(I.config(1)), 8)
    g.name = "grid3d_128_nodiag_shuf"
    check(g)
    check(g, async_search=-1, team_size=64)


def test_batched_shuffled_rows():
    graphs = [I.shuffle_rows(_random_graph(1400 + i), i) for i in range(8)]
    graphs += [I.shuffle_rows(I.drop_diagonal(I.grid2d(30 + 4 * i, 25, seed=i)), i)
               for i in range(4)]
    graphs += [I.path(1), I.shuffle_rows(I.complete(6), 1)]
    _check_batch(graphs)
    _check_batch(graphs, small_cutoff=500, team_size=4, pp_variant=1)
    _check_batch(graphs, small_cutoff=1 << 30, small_threads=256)


# ---------------------------------------------------------------------------
# rcm_order itself (the binding's order() goes through rcm_order_ex)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("which", ["grid64", "union", "grid128"])
def test_rcm_order_entry_point(which):
    import ctypes
    import torch
    from paper_1610_08128_amd import rcm

    if which == "grid64":
        g = I.config(0, seed=5)
    elif which == "union":
        g = I.shuffle_rows(_random_graph(1500), 3)
    else:
        g = I.config(1)
    _say(f"rcm_order on {g.name} n={g.n}")
    want = oracle.rcm(g.n, g.rowptr, g.colidx)
    rp = torch.from_numpy(g.rowptr).cuda()
    ci = torch.from_numpy(g.colidx).cuda()
    perm = torch.full((g.n,), -1, dtype=torch.int32, device="cuda")
    st = rcm.Stats()
    stream = torch.cuda.current_stream().cuda_stream
    status = rcm.lib().rcm_order(g.n, rp.data_ptr(), ci.data_ptr(), perm.data_ptr(),
                                 ctypes.byref(st), stream)
    assert status == rcm.OK, rcm.status_string(status)
    assert np.array_equal(perm.cpu().numpy(), want.perm)
    assert st.to_dict() == want.stats
    # stats is nullable
    status = rcm.lib().rcm_order(g.n, rp.data_ptr(), ci.data_ptr(), perm.data_ptr(), None, stream)
    assert status == rcm.OK
    assert np.array_equal(perm.cpu().numpy(), want.perm)


# ---------------------------------------------------------------------------
# Repeated columns are malformed on every path, rows of any length
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("row_len", [2, 7, 16, 17, 64, 65, 300, 2000, 40000])
def test_duplicates_rejected_without_full_check(row_len):
    """A column repeated within a row gives RCM_ERR_BAD_CSR whatever the row
    length (register check up to 16 entries, re-read up to 64, a work-group
    per row beyond), as the oracle's validation does."""
    import torch
    from paper_1610_08128_amd import rcm

    g = I.shuffle_rows(I.disjoint_union([I.star(row_len + 1), I.grid2d(5, 7, seed=1)], seed=4),
                       row_len)
    lens = np.diff(g.rowptr)
    r = int(np.nonzero(lens == row_len + 1)[0][0])  # the star's centre (diagonal included)
    ci = g.colidx.copy()
    a, b = int(g.rowptr[r]), int(g.rowptr[r + 1])
    ci[b - 1] = ci[a]
    assert oracle.validate(g.n, g.rowptr, ci) == oracle.ERR_BAD_CSR
    _say(f"duplicate in a row of {b - a} entries")
    for opts in ({}, {"small_cutoff": 1, "team_size": 4}, {"check_full": True}):
        with pytest.raises(rcm.RcmError) as e:
            rcm.order(torch.from_numpy(g.rowptr).cuda(), torch.from_numpy(ci).cuda(), **opts)
        assert e.value.status == rcm.ERR_BAD_CSR, opts
    graphs = [I.grid2d(4, 4, seed=2), g]
    vo, no, rpc, cic = I.concat_batch(graphs)
    cic = cic.copy()
    cic[no[1] + a:no[1] + b] = ci[a:b]
    with pytest.raises(rcm.RcmError) as e:
        rcm.order_batched(vo, no, torch.from_numpy(rpc).cuda(), torch.from_numpy(cic).cuda())
    assert e.value.status == rcm.ERR_BAD_CSR


# ---------------------------------------------------------------------------
# The one-work-group LDS engine (mode 2 requires it)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("idx", range(17))
def test_engine_tiny_graphs(idx):
    g = _tiny_graphs()[idx]
    for pp in (0, 1):
        for rev in (0, 1):
            check(g, pp_variant=pp, reverse_mode=rev, mode=2)
    check(I.shuffle_rows(g, idx), mode=2, check_full=True)


@pytest.mark.parametrize("seed", range(16))
def test_engine_random_graphs(seed):
    g = _random_graph(1600 + seed)
    check(g, pp_variant=seed % 2, reverse_mode=(seed // 2) % 2, mode=2)
    h = I.shuffle_rows(I.drop_diagonal(_random_graph(1700 + seed)), seed)
    check(h, mode=2)
    check(h, mode=2, pp_variant=1, reverse_mode=1)


def test_engine_near_its_lds_limit():
    """The largest meshes the engine takes, and one just past it: mode 2
    refuses that one, mode 0 gives it to the team kernel, same result."""
    import torch
    from paper_1610_08128_amd import rcm

    for g in (I.grid2d(80, 80, seed=41), I.grid3d(18, 18, 18, seed=42),
              I.shuffle_rows(I.rgg_patches(4000, 43), 3)):
        check(g, mode=2)
    big = I.grid2d(85, 85, seed=44)
    with pytest.raises(rcm.RcmError) as e:
        rcm.order(torch.from_numpy(big.rowptr).cuda(), torch.from_numpy(big.colidx).cuda(),
                  mode=2)
    assert e.value.status == rcm.ERR_INVALID_ARGUMENT
    check(big)
    with pytest.raises(rcm.RcmError) as e:
        rcm.order(torch.from_numpy(big.rowptr).cuda(), torch.from_numpy(big.colidx).cuda(),
                  mode=2, label_mode=1)
    assert e.value.status == rcm.ERR_INVALID_ARGUMENT


def test_engine_long_rows():
    """Rows longer than the per-lane duplicate check (64 entries) and parents
    with more children than the register ranking holds (8)."""
    graphs = [I.star(300, 17), I.complete(70), I.erdos_renyi(200, 0.3, 45),
              I.shuffle_rows(I.disjoint_union([I.star(90), I.complete(12), I.path(40)],
                                              seed=46), 4)]
    for g in graphs:
        check(g, mode=2)
        check(g, mode=2, pp_variant=1, reverse_mode=1)


def test_engine_status_codes():
    import torch
    from paper_1610_08128_amd import rcm

    def status(rp, ci, **opts):
        try:
            rcm.order(torch.from_numpy(np.asarray(rp, np.int32)).cuda(),
                      torch.from_numpy(np.asarray(ci, np.int32)).cuda(), mode=2, **opts)
            return rcm.OK
        except rcm.RcmError as e:
            return e.status

    g = I.path(6)
    bad = g.colidx.copy()
    bad[2] = 6
    assert status(g.rowptr, bad) == rcm.ERR_BAD_CSR
    badr = g.rowptr.copy()
    badr[3] = badr[2] - 1
    assert status(badr, g.colidx) == rcm.ERR_BAD_CSR
    # a repeated column in a short row and in a long one
    assert status([0, 3, 6, 8], [0, 1, 1, 0, 1, 2, 1, 2]) == rcm.ERR_BAD_CSR
    s = I.star(100, 0)
    ci = s.colidx.copy()
    ci[s.rowptr[1] - 1] = ci[s.rowptr[0] + 5]
    assert status(s.rowptr, ci) == rcm.ERR_BAD_CSR
    # vertex 1 points at vertex 0 without the way back: found by the
    # traversal, and by the full check
    rp = [0, 1, 4, 6, 8, 10, 12]
    ci = [0, 0, 1, 2, 2, 3, 3, 4, 4, 5, 4, 5]
    assert status(rp, ci) == rcm.ERR_NOT_SYMMETRIC
    assert status(rp, ci, check_full=True) == rcm.ERR_NOT_SYMMETRIC
    assert status([0, 2, 3, 4, 5, 6], [0, 4, 1, 2, 3, 4], check_full=True) == \
        rcm.ERR_NOT_SYMMETRIC


def _max_offdiag(g):
    rows = np.diff(g.rowptr)
    if g.n == 0:
        return 0
    r = np.repeat(np.arange(g.n), rows)
    off = np.bincount(r[g.colidx != r], minlength=g.n) if g.colidx.size else np.zeros(g.n)
    return int(off.max()) if off.size else 0


def _bounded_row_graphs():
    """Graphs whose rows hold at most 8 off-diagonal entries: the bounded-row
    variant of the engine takes them.  Levels of one vertex (paths) up to
    several wave-wide chunks (the 66 x 90 grid, the 3D grid), many
    components (enough for the search numbers to wrap), isolated vertices,
    self loops, shuffled rows, no diagonal."""
    gs = [g for g in _tiny_graphs() if _max_offdiag(g) <= 8]
    gs += [I.config(0),
           I.grid2d(66, 90, seed=11),
           I.grid3d(18, 18, 18, seed=42),
           I.shuffle_rows(I.drop_diagonal(I.grid2d(30, 41, seed=3)), 5),
           I.add_random_self_loops(I.grid3d(9, 10, 11, seed=4), 0.3, 4),
           I.disjoint_union([I.grid2d(10, 12), I.path(50), I.path(1), I.cycle(30),
                             I.grid3d(5, 6, 7), I.path(2)], seed=7),
           I.path(5000, seed=12),
           I.strip_drop(4, 1200, 0.02, seed=13),
           # 200 components of two or three searches each: the search
           # numbers wrap (every 126 searches) several times
           I.disjoint_union([I.path(4 + i % 9, seed=i) for i in range(200)], seed=15),
           I.rgg_patches(3000, 14)]
    return [g for g in gs if _max_offdiag(g) <= 8]


@pytest.mark.parametrize("idx", range(len(_bounded_row_graphs())))
def test_engine_bounded_rows_both_variants(idx, monkeypatch):
    """The bounded-row variant (8 waves, rows as sorted 16-byte records,
    token claims) and the general engine (RCM_SMALL_ELL=0) both give the
    oracle's ordering and statistics, and each call ran the variant asked
    for."""
    from paper_1610_08128_amd import rcm

    g = _bounded_row_graphs()[idx]
    assert _max_offdiag(g) <= 8
    for variant, threads in (("1", 512), ("0", 64)):
        monkeypatch.setenv("RCM_SMALL_ELL", variant)
        for pp, rev in ((0, 0), (1, 1), (0, 1)):
            check(g, pp_variant=pp, reverse_mode=rev, mode=2)
            tm = rcm.last_timings()
            assert tm["used_mode"] == 2 and tm["used_block_threads"] == threads, (variant, tm)
        check(I.shuffle_rows(g, idx + 1), mode=2, check_full=True)


def test_engine_bounded_rows_declines_long_rows():
    """A graph with one row of 9 off-diagonal entries goes to the general
    engine; a row of 8 stays in the bounded-row variant."""
    from paper_1610_08128_amd import rcm

    for k, threads in ((8, 512), (9, 64)):
        g = I.disjoint_union([I.star(k + 1), I.grid2d(12, 13, seed=k)], seed=k)
        assert _max_offdiag(g) == k
        check(g, mode=2)
        assert rcm.last_timings()["used_block_threads"] == threads


@pytest.mark.parametrize("seed", range(6))
def test_engine_equals_team_kernel(seed):
    """The two engines agree with each other on the same input (and with the
    oracle), including graphs with isolated vertices and self loops."""
    g = I.add_random_self_loops(_random_graph(1800 + seed), 0.3, seed)
    a = gpu_order(g, mode=2)
    b = gpu_order(g, mode=1)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]
    check(g, mode=2)


# Long graphs whose vertex-0 component is renumbered after its first level
# structure (relabel_levels; forced here with a threshold of 2 levels): the
# ordering must not change.  On a connected graph the renumbered path must
# have run; with several components it runs when vertex 0's is large enough
# for the asynchronous search, and the other components are then ordered in
# the caller's numbering.
def _relabel_graphs():
    return [
        I.grid2d(16, 4000, seed=1),
        I.path(30000, seed=2),
        I.strip_drop(8, 12000, 0.01, seed=3),
        I.shuffle_rows(I.drop_diagonal(I.grid2d(12, 5000, seed=4)), 5),
        I.grid3d(10, 10, 600, seed=6),
        I.add_random_self_loops(I.grid2d(20, 3000, seed=7), 0.3, 7),
        I.disjoint_union([I.grid2d(10, 3000, seed=8), I.path(500), I.star(6)], seed=9),
        # vertex 0 in the long component, other components beside it
        I.disjoint_union([I.grid2d(10, 3000, seed=10), I.path(700, seed=11), I.star(6),
                          I.path(1), I.grid2d(7, 9, seed=12)]),
        I.strip_drop(4, 20000, 0.02, seed=13),
    ]


@pytest.mark.parametrize("case", range(9))
@pytest.mark.parametrize("window", ["1", "0"])
def test_relabelled_long_graphs(case, window, monkeypatch):
    """With the window engine (rows of at most 4 off-diagonal entries; it
    declines the others, and the team kernel resumes) and without it
    (RCM_WINDOW=0: the team kernel on the renumbered copy)."""
    from paper_1610_08128_amd import rcm

    monkeypatch.setenv("RCM_WINDOW", window)
    g = _relabel_graphs()[case]
    g.name = g.name or f"long{case}"
    variants = [dict(), dict(pp_variant=1, reverse_mode=1), dict(team_size=16, narrow_cutoff=64),
                dict(team_size=256, label_team=32, search_round=4)]
    renumbered = (3, 4) if window == "1" else (3,)
    for v in variants:
        st = check(g, mode=1, relabel_levels=2, **v)
        used = rcm.last_timings()["used_mode"]
        assert used in renumbered if st["num_components"] == 1 else used in (1,) + renumbered, \
            (g.name, v, used)
    check(g, mode=1, relabel_levels=-1)
    assert rcm.last_timings()["used_mode"] == 1
    # the default threshold (4096 levels) and a level-synchronous first
    # search, which never renumbers
    check(g, mode=1)
    check(g, mode=1, relabel_levels=2, async_search=-1)
    assert rcm.last_timings()["used_mode"] == 1


def test_relabelled_tiny_graphs():
    """The renumbering at its smallest: vertex-0 components of two to a few
    vertices (eccentricity 1 and up), alone or beside other components.
    Every case must give the oracle's ordering; the smallest may not
    renumber at all (their first search's ring is so small that it can fall
    back to the level-synchronous pass), but most do."""
    from paper_1610_08128_amd import rcm

    gs = [I.path(2), I.path(3), I.star(5), I.complete(4), I.cycle(5, seed=1),
          I.disjoint_union([I.path(2), I.path(1), I.star(4)]),
          I.disjoint_union([I.cycle(7), I.grid2d(3, 4, seed=2)]),
          I.drop_diagonal(I.grid2d(2, 9, seed=3)), I.path(40, seed=4), I.grid2d(5, 7, seed=5)]
    renumbered = windowed = 0
    for idx, g in enumerate(gs):
        g.name = g.name or f"tinyrl{idx}"
        for v in (dict(), dict(pp_variant=1, reverse_mode=1)):
            for window in ("1", "0"):
                os.environ["RCM_WINDOW"] = window
                try:
                    check(g, mode=1, relabel_levels=2, team_size=4, **v)
                finally:
                    os.environ.pop("RCM_WINDOW")
                used = rcm.last_timings()["used_mode"]
                assert used in ((1, 3, 4) if window == "1" else (1, 3)), used
                renumbered += used in (3, 4)
                windowed += used == 4
    assert renumbered >= 12, renumbered
    assert windowed >= 4, windowed


def test_window_engine_runs_and_declines():
    """Long components with rows of at most 4 off-diagonal entries take the
    window engine (used_mode 4), also when it must slide its window many
    times (the path and the strips are far longer than the window) and when
    its levels take several passes of the wave; a
    component with longer rows (a 3D grid) goes back to the team kernel
    (used_mode 3); both give the oracle's ordering."""
    from paper_1610_08128_amd import rcm

    # (grid2d(100, 2000) in its natural numbering: vertex 0 at a corner, so
    # the later searches' levels -- up to 100 wide, two passes of the wave
    # -- each lie within one level of the renumbering)
    for g, want in ((I.path(30000, seed=2), 4), (I.strip_drop(8, 12000, 0.01, seed=3), 4),
                    (I.grid2d(40, 3000, seed=8), 4), (I.grid2d(100, 2000), 4),
                    (I.grid3d(10, 10, 600, seed=6), 3)):
        for v in (dict(), dict(pp_variant=1, reverse_mode=1)):
            check(g, mode=1, relabel_levels=2, **v)
            assert rcm.last_timings()["used_mode"] == want, (g.name, v)
