"""The allocation-free entry point rcm_order_noalloc (include/rcm.h), called
through the C ABI: the same permutation, inverse and statistics as
rcm_order_ex on the same input, over consecutive calls that reuse the
library's device array (each call smaller than the one before), and the
documented rejection of a graph whose workspace exceeds that array."""

import ctypes
import sys

import numpy as np
import pytest

from paper_1610_08128_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _noalloc(g, with_iperm=True, with_stats=True, **opts):
    import torch
    from paper_1610_08128_amd import rcm

    rp = torch.from_numpy(g.rowptr).cuda()
    ci = torch.from_numpy(g.colidx if g.colidx.size else np.zeros(1, np.int32)).cuda()
    perm = torch.full((max(g.n, 1),), -1, dtype=torch.int32, device="cuda")
    iperm = torch.full((max(g.n, 1),), -1, dtype=torch.int32, device="cuda")
    st = rcm.Stats()
    o = rcm.make_options(**opts)
    status = rcm.lib().rcm_order_noalloc(
        g.n, rp.data_ptr(), ci.data_ptr(), perm.data_ptr(),
        iperm.data_ptr() if with_iperm else None, ctypes.byref(st) if with_stats else None,
        ctypes.byref(o), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return status, perm.cpu().numpy()[:g.n], iperm.cpu().numpy()[:g.n], st.to_dict()


def _with_workspace(g, **opts):
    import torch
    from paper_1610_08128_amd import rcm

    perm, iperm, st = rcm.order(torch.from_numpy(g.rowptr).cuda(),
                                torch.from_numpy(g.colidx).cuda(), return_iperm=True, **opts)
    return perm.cpu().numpy(), iperm.cpu().numpy(), st


def _random_union(seed):
    rng = np.random.default_rng(seed)
    parts = [I.grid2d(int(rng.integers(3, 40)), int(rng.integers(3, 40)), seed=seed),
             I.rgg_patches(int(rng.integers(50, 900)), seed), I.path(1),
             I.random_tree(int(rng.integers(2, 300)), seed)]
    return I.shuffle_rows(I.disjoint_union(parts, seed=seed), seed)


def test_noalloc_matches_rcm_order_ex_on_shrinking_inputs():
    from paper_1610_08128_amd import rcm

    graphs = [I.grid3d(60, 60, 60, seed=31),  # a team of work-groups, about 50 MB of workspace
              I.config(0, seed=32),           # 64 x 64 grid
              _random_union(33),              # several components, rows in random order
              I.path(5, seed=34)]
    for i in range(len(graphs) - 1):
        assert graphs[i + 1].n < graphs[i].n
    for g in graphs:
        assert rcm.workspace_bytes(g.n, g.nnz) <= rcm.NOALLOC_SCRATCH_BYTES
        _say(f"noalloc call on {g.name} n={g.n} nnz={g.nnz}")
        status, perm, iperm, st = _noalloc(g)
        assert status == rcm.OK, rcm.status_string(status)
        want_perm, want_iperm, want_st = _with_workspace(g)
        assert np.array_equal(perm, want_perm), g.name
        assert np.array_equal(iperm, want_iperm), g.name
        assert st == want_st, (g.name, st, want_st)


def test_noalloc_options_and_nullable_outputs():
    from paper_1610_08128_amd import rcm

    g = _random_union(35)
    _say(f"noalloc call with options on {g.name} n={g.n}")
    for opts in ({"pp_variant": 1, "reverse_mode": 1}, {"small_cutoff": 1, "team_size": 4},
                 {"label_mode": 2}):
        status, perm, _, st = _noalloc(g, **opts)
        assert status == rcm.OK
        want_perm, _, want_st = _with_workspace(g, **opts)
        assert np.array_equal(perm, want_perm), opts
        assert st == want_st, opts
    status, perm, _, _ = _noalloc(g, with_iperm=False, with_stats=False)
    assert status == rcm.OK
    assert np.array_equal(perm, _with_workspace(g)[0])


def test_noalloc_rejects_a_graph_beyond_its_array():
    from paper_1610_08128_amd import rcm

    big = I.grid2d(1300, 1300, seed=36)
    assert rcm.workspace_bytes(big.n, big.nnz) > rcm.NOALLOC_SCRATCH_BYTES
    _say(f"noalloc call on {big.name} n={big.n}, beyond the array")
    status, _, _, _ = _noalloc(big)
    assert status == rcm.ERR_WORKSPACE_TOO_SMALL
    # the next call on the same array still works
    g = I.config(0, seed=37)
    status, perm, _, st = _noalloc(g)
    assert status == rcm.OK
    assert np.array_equal(perm, _with_workspace(g)[0])
