"""The autotuner's table logic (CPU) and a small tuning run (GPU) whose
chosen options still give the oracle's ordering."""

import numpy as np
import pytest

from paper_1610_08128_amd import inputs as I
from paper_1610_08128_amd.tune import TuningTable, autotune_batched, autotune_single, size_class


def test_size_class_and_lookup(tmp_path):
    assert size_class(4096, 20224) == "single:n2^12:d5"
    assert size_class(4096, 20224, graphs=3) == "batch:n2^12:d5"
    t = TuningTable(entries={"single:n2^12:d5": {"team_size": 8},
                             "single:n2^21:d7": {"team_size": 64, "block_threads": 256},
                             "batch:n2^24:d8": {"small_threads": 512}})
    assert t.options_for(4000, 20000) == {"team_size": 8}
    # nearest class of the same kind
    assert t.options_for(2_000_000, 14_000_000) == {"team_size": 64, "block_threads": 256}
    assert t.options_for(1 << 20, 7 << 20) == {"team_size": 64, "block_threads": 256}
    assert t.options_for(100, 500, graphs=2) == {"small_threads": 512}
    assert TuningTable().options_for(10, 10) == {}
    p = tmp_path / "t.txt"
    t.save(str(p))
    u = TuningTable.load(str(p))
    assert u.entries == t.entries


def test_library_reads_the_tuners_table(tmp_path):
    """The library's own lookup (rcm_tuning_options, no GPU) agrees with the
    tuner's for exact and nearest classes, fills only options left at 0,
    and rejects tables that set anything but launch options."""
    import ctypes

    from paper_1610_08128_amd import rcm

    t = TuningTable(entries={"single:n2^12:d5": {"team_size": 8, "mode": 1},
                             "single:n2^21:d7": {"team_size": 256, "label_team": 96,
                                                 "search_round": 12},
                             "batch:n2^24:d8": {"small_threads": 512, "max_teams": 32}},
                    timings={"single:n2^12:d5": {"{}": 1.5}})
    p = str(tmp_path / "t.txt")
    t.save(p, header="test table")
    for n, nnz, g in ((4096, 20224, 1), (4000, 20000, 1), (2_000_000, 14_000_000, 1),
                      (1 << 20, 7 << 20, 1), (100, 500, 2), (19_000_000, 160_000_000, 512),
                      (3, 2, 1)):
        assert rcm.tuning_options(p, n, nnz, g) == t.options_for(n, nnz, g), (n, nnz, g)
    # a caller's own setting wins over the table
    o = rcm.make_options(team_size=4)
    assert rcm.lib().rcm_tuning_options(p.encode(), 1, 4096, 20224, ctypes.byref(o)) == rcm.OK
    assert o.team_size == 4 and o.mode == 1
    # the engine comes only from the exact class, and never as mode 2
    t2 = TuningTable(entries={"single:n2^12:d5": {"mode": 2, "team_size": 8},
                              "single:n2^21:d7": {"mode": 1, "team_size": 256}})
    p2 = str(tmp_path / "t2.txt")
    t2.save(p2)
    assert rcm.tuning_options(p2, 4096, 20224) == {"team_size": 8} == t2.options_for(4096, 20224)
    assert rcm.tuning_options(p2, 1 << 15, 5 << 15) == {"team_size": 8}
    assert rcm.tuning_options(p2, 1 << 21, 7 << 21) == {"mode": 1, "team_size": 256}
    assert rcm.tuning_options(p2, 1 << 20, 7 << 20) == {"team_size": 256}
    # rounding half to even, as the tuner's round(): 2.5 -> 2, 3.5 -> 4
    assert size_class(1000, 2500) == "single:n2^9:d2" and size_class(1000, 3500) == "single:n2^9:d4"
    bad = tmp_path / "bad.txt"
    bad.write_text("single:n2^12:d5 pp_variant=1\n")
    import pytest as _pytest
    with _pytest.raises(rcm.RcmError):
        rcm.tuning_options(str(bad), 4096, 20224)
    with _pytest.raises(rcm.RcmError):
        rcm.tuning_options(str(tmp_path / "missing.txt"), 4096, 20224)
    # a bad table makes the ordering call itself fail before any device work
    status, _ = rcm.order_raw(5, 0, 0, 0, options=rcm.make_options(tuning_file=str(bad)))
    assert status == rcm.ERR_INVALID_ARGUMENT


@pytest.mark.gpu
def test_autotune_keeps_the_ordering():
    import oracle
    import torch
    from paper_1610_08128_amd import rcm

    graphs = [I.grid2d(40, 50, seed=3), I.rgg_patches(3000, 9)]
    cands = [dict(team_size=4, narrow_cutoff=64), dict(team_size=16, narrow_cutoff=-1),
             dict(team_size=32, block_threads=256)]
    table = autotune_single(graphs, candidates=cands, reps=1)
    assert set(table.entries) == {size_class(g.n, g.nnz) for g in graphs}
    for g in graphs:
        opts = table.options_for(g.n, g.nnz)
        assert opts in cands
        perm, _ = rcm.order(torch.from_numpy(g.rowptr).cuda(), torch.from_numpy(g.colidx).cuda(),
                            **opts)
        assert np.array_equal(perm.cpu().numpy(), oracle.rcm(g.n, g.rowptr, g.colidx).perm)
    bt = autotune_batched([graphs + [I.path(5)]], candidates=[dict(), dict(small_cutoff=100)],
                          reps=1)
    assert len(bt.entries) == 1


@pytest.mark.gpu
def test_tuning_table_changes_the_launch_and_keeps_the_result(tmp_path):
    """A table that maps a graph's size class to other launch settings: the
    call uses them (rcm_last_timings' used_* fields) and returns the
    oracle's ordering, alone and in a batch."""
    import oracle
    import torch
    from paper_1610_08128_amd import rcm

    g = I.grid2d(120, 130, seed=5)  # past the one-work-group engine's LDS
    t = TuningTable(entries={size_class(g.n, g.nnz): {"mode": 1, "team_size": 8,
                                                       "label_team": 4, "search_round": 3},
                             "batch:n2^15:d5": {"team_size": 4, "small_cutoff": 100}})
    p = str(tmp_path / "t.txt")
    t.save(p)
    rp = torch.from_numpy(g.rowptr).cuda()
    ci = torch.from_numpy(g.colidx).cuda()
    want = oracle.rcm(g.n, g.rowptr, g.colidx)
    perm, st = rcm.order(rp, ci)
    plain = rcm.last_timings()
    assert plain["used_team_size"] == 64 and plain["used_search_round"] == 16
    perm2, st2 = rcm.order(rp, ci, tuning_file=p)
    tuned = rcm.last_timings()
    assert (tuned["used_team_size"], tuned["used_label_team"], tuned["used_search_round"]) == \
        (8, 4, 3)
    for p_, s_ in ((perm, st), (perm2, st2)):
        assert np.array_equal(p_.cpu().numpy(), want.perm) and s_ == want.stats
    # the environment variable names a table too; options set by the caller win
    import os
    os.environ["RCM_TUNING_FILE"] = p
    try:
        perm3, _ = rcm.order(rp, ci, team_size=2)
        assert rcm.last_timings()["used_team_size"] == 2
        assert np.array_equal(perm3.cpu().numpy(), want.perm)
    finally:
        del os.environ["RCM_TUNING_FILE"]
    graphs = [g, I.path(7), I.grid2d(30, 40, seed=6)]
    vo, no, rpc, cic = I.concat_batch(graphs)
    pb, _ = rcm.order_batched(vo, no, torch.from_numpy(rpc).cuda(), torch.from_numpy(cic).cuda(),
                              tuning_file=p)
    assert rcm.last_timings()["used_small_cutoff"] == 100
    pb = pb.cpu().numpy()
    for i, h in enumerate(graphs):
        assert np.array_equal(pb[vo[i]:vo[i + 1]], oracle.rcm(h.n, h.rowptr, h.colidx).perm)
