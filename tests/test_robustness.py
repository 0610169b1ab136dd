"""Failure handling and determinism on the GPU.

- The caller's abort flag (rcm_abort_flag_create): set before a call, every
  entry point returns RCM_ERR_ABORTED without launching; set by another host
  thread while a long ordering runs, the kernels see it at their next poll
  and end normally, and the call returns RCM_ERR_ABORTED well before the
  ordering would have finished; cleared, the next calls return the oracle's
  ordering again.
- The shuffle knob (rcm_options.shuffle_seed): seeded permutations of which
  work-group plays which team member and which component or graph each one
  takes, plus seeded delays at every team barrier.  The ordering is unique,
  so every seed must give the oracle's permutation and statistics."""

import ctypes
import sys
import threading
import time

import numpy as np
import pytest

import oracle
from paper_1610_08128_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(g):
    import torch

    rp = torch.from_numpy(g.rowptr).cuda()
    ci = torch.from_numpy(g.colidx if g.colidx.size else np.zeros(1, np.int32)).cuda()
    return rp, ci


def _expect_aborted(fn):
    from paper_1610_08128_amd import rcm

    with pytest.raises(rcm.RcmError) as e:
        fn()
    assert e.value.status == rcm.ERR_ABORTED, e.value


def test_abort_flag_set_before_the_call():
    import torch
    from paper_1610_08128_amd import rcm

    g = I.grid2d(30, 40, seed=3)          # fits the one-work-group engine
    h = I.grid2d(150, 160, seed=4)        # the team kernel
    gs = [g, I.path(9), I.grid2d(20, 25, seed=5)]
    vo, no, rpc, cic = I.concat_batch(gs)
    with rcm.AbortFlag() as flag:
        assert not flag.is_set
        flag.set()
        for graph, mode in ((g, 0), (g, 2), (h, 1), (g, 1)):
            _say(f"case abort-before {graph.name} mode={mode}")
            rp, ci = _dev(graph)
            _expect_aborted(lambda: rcm.order(rp, ci, mode=mode, abort_flag=flag))
        _expect_aborted(lambda: rcm.order_batched(vo, no, torch.from_numpy(rpc).cuda(),
                                                  torch.from_numpy(cic).cuda(), abort_flag=flag))
        # the allocation-free entry point
        rp, ci = _dev(g)
        perm = torch.empty(g.n, dtype=torch.int32, device="cuda")
        o = rcm.make_options(abort_flag=flag)
        st = rcm.lib().rcm_order_noalloc(g.n, rp.data_ptr(), ci.data_ptr(), perm.data_ptr(), None,
                                         None, ctypes.byref(o), None)
        assert st == rcm.ERR_ABORTED
        # cleared: the same calls order again
        flag.clear()
        for graph, mode in ((g, 0), (g, 2), (h, 1)):
            rp, ci = _dev(graph)
            p, s = rcm.order(rp, ci, mode=mode, abort_flag=flag)
            want = oracle.rcm(graph.n, graph.rowptr, graph.colidx)
            assert np.array_equal(p.cpu().numpy(), want.perm) and s == want.stats
        pb, _ = rcm.order_batched(vo, no, torch.from_numpy(rpc).cuda(),
                                  torch.from_numpy(cic).cuda(), abort_flag=flag)
        pb = pb.cpu().numpy()
        for i, x in enumerate(gs):
            assert np.array_equal(pb[vo[i]:vo[i + 1]], oracle.rcm(x.n, x.rowptr, x.colidx).perm)


def test_foreign_abort_pointer_is_rejected():
    from paper_1610_08128_amd import rcm

    g = I.path(5)
    rp, ci = _dev(g)
    word = ctypes.c_int32(0)
    with pytest.raises(rcm.RcmError) as e:
        rcm.order(rp, ci, abort_flag=ctypes.addressof(word))
    assert e.value.status == rcm.ERR_INVALID_ARGUMENT


def _timed(fn):
    import torch

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


# Long orderings: a path (one work-group walks every level alone) and a
# long 2D strip whose levels are wide enough for the whole team.
LONG_CASES = [
    ("path", lambda: I.path(1_500_000), dict(mode=1)),
    ("strip", lambda: I.grid2d(256, 25_000), dict(mode=1, narrow_cutoff=64)),
]


@pytest.mark.parametrize("name,make,opts", LONG_CASES, ids=[c[0] for c in LONG_CASES])
def test_abort_flag_set_while_the_kernel_runs(name, make, opts):
    from paper_1610_08128_amd import rcm

    g = make()
    rp, ci = _dev(g)
    _say(f"case abort-during {name} n={g.n} nnz={g.nnz} {opts}")
    with rcm.AbortFlag() as flag:
        # the whole ordering first (flag never set), for its time and result
        (perm, st), full = _timed(lambda: rcm.order(rp, ci, abort_flag=flag, **opts))
        _say(f"  full ordering {full * 1e3:.1f} ms")
        assert full > 0.2, "the case is too short to abort in flight"
        delay = full / 4
        timer = threading.Timer(delay, flag.set)
        timer.start()
        try:
            _, took = _timed(lambda: _expect_aborted(
                lambda: rcm.order(rp, ci, abort_flag=flag, **opts)))
        finally:
            timer.join()
        _say(f"  aborted after {took * 1e3:.1f} ms (flag set at {delay * 1e3:.1f} ms)")
        # the kernels stopped at their next poll, long before the end
        assert took < delay + 0.5 * (full - delay)
        flag.clear()
        (perm2, st2), _ = _timed(lambda: rcm.order(rp, ci, abort_flag=flag, **opts))
        assert np.array_equal(perm.cpu().numpy(), perm2.cpu().numpy()) and st == st2
    if g.n <= 2_000_000:
        want = oracle.rcm(g.n, g.rowptr, g.colidx)
        assert np.array_equal(perm.cpu().numpy(), want.perm) and st == want.stats


SEEDS = (1, 2, 3, 0xBEEF)


def _shuffle_graphs():
    return [
        I.grid2d(60, 70, seed=1),
        I.rgg_patches(20_000, 5),
        I.disjoint_union([I.grid2d(90, 95, seed=2), I.grid3d(20, 21, 22, seed=3),
                          I.rgg_patches(5000, 4), I.path(300), I.star(40)] +
                         [I.grid2d(6 + i % 5, 7, seed=i) for i in range(60)], seed=6),
        I.shuffle_rows(I.drop_diagonal(I.grid3d(24, 25, 26, seed=7)), 8),
    ]


@pytest.mark.parametrize("mode", [1, 2])
def test_shuffle_seed_keeps_the_ordering(mode):
    from paper_1610_08128_amd import rcm

    for g in _shuffle_graphs():
        if mode == 2 and g.n >= 6000:
            continue
        want = oracle.rcm(g.n, g.rowptr, g.colidx)
        rp, ci = _dev(g)
        for seed in (0,) + SEEDS:
            opts = dict(mode=mode, shuffle_seed=seed)
            if mode == 1:
                opts.update(team_size=16, small_cutoff=2000, label_team=8)
            _say(f"case shuffle {g.name} n={g.n} {opts}")
            perm, st = rcm.order(rp, ci, **opts)
            assert np.array_equal(perm.cpu().numpy(), want.perm), (g.name, seed)
            assert st == want.stats, (g.name, seed)


def test_shuffle_seed_keeps_renumbered_orderings():
    """The renumbering of long components (forced with a two-level
    threshold) under shuffled work-group roles and barrier delays."""
    from paper_1610_08128_amd import rcm

    for g in (I.grid2d(12, 3000, seed=21),
              I.disjoint_union([I.strip_drop(6, 4000, 0.01, seed=22), I.path(40), I.star(5)])):
        want = oracle.rcm(g.n, g.rowptr, g.colidx)
        rp, ci = _dev(g)
        for seed in (0,) + SEEDS:
            _say(f"case shuffle renumbered {g.name} n={g.n} seed={seed}")
            perm, st = rcm.order(rp, ci, mode=1, relabel_levels=2, team_size=32, shuffle_seed=seed)
            assert rcm.last_timings()["used_mode"] in (3, 4)
            assert np.array_equal(perm.cpu().numpy(), want.perm), (g.name, seed)
            assert st == want.stats, (g.name, seed)


def test_shuffle_seed_keeps_batched_orderings():
    import torch
    from paper_1610_08128_amd import rcm

    gs = [I.grid2d(40 + i, 30, seed=i) for i in range(6)] + \
         [I.rgg_patches(3000 + 500 * i, i) for i in range(6)] + [I.path(1), I.star(7)]
    vo, no, rpc, cic = I.concat_batch(gs)
    rp = torch.from_numpy(rpc).cuda()
    ci = torch.from_numpy(cic).cuda()
    wants = [oracle.rcm(g.n, g.rowptr, g.colidx) for g in gs]
    for seed in (0,) + SEEDS:
        for opts in (dict(), dict(team_size=4, small_cutoff=2500)):
            _say(f"case shuffle batch seed={seed} {opts}")
            pb, stats = rcm.order_batched(vo, no, rp, ci, shuffle_seed=seed, **opts)
            pb = pb.cpu().numpy()
            for i, w in enumerate(wants):
                assert np.array_equal(pb[vo[i]:vo[i + 1]], w.perm), (seed, i)
                assert stats[i] == w.stats, (seed, i)
