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
    p = tmp_path / "t.json"
    t.save(str(p))
    u = TuningTable.load(str(p))
    assert u.entries == t.entries


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
