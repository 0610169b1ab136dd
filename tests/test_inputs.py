"""The seeded generators produce the workloads' exact shapes, symmetric,
with sorted rows, and the same bytes for the same seed."""

import hashlib

import numpy as np
import pytest
import scipy.sparse as sp

from paper_1610_08128_amd import inputs as I


def _check_csr(g, diag=True):
    assert g.rowptr.dtype == np.int32 and g.colidx.dtype == np.int32
    assert g.rowptr[0] == 0 and np.all(np.diff(g.rowptr) >= 0)
    assert g.colidx.min(initial=0) >= 0 and g.colidx.max(initial=-1) < g.n
    A = sp.csr_matrix((np.ones(g.nnz), g.colidx, g.rowptr), shape=(g.n, g.n))
    assert (A != A.T).nnz == 0
    for v in range(min(g.n, 200)):
        row = g.colidx[g.rowptr[v]:g.rowptr[v + 1]]
        assert np.all(np.diff(row) > 0)  # sorted, no duplicates
        if diag:
            assert v in row


def _sha(g):
    h = hashlib.sha256()
    h.update(g.rowptr.tobytes())
    h.update(g.colidx.tobytes())
    return h.hexdigest()


def test_config0_shape():
    g = I.config(0)
    assert (g.n, g.nnz) == (4096, 20224)
    _check_csr(g)
    assert _sha(g) == _sha(I.config(0))
    assert _sha(g) != _sha(I.config(0, seed=2))


def test_config1_shape():
    g = I.config(1)
    assert (g.n, g.nnz) == (2_097_152, 14_581_760)
    assert np.all(np.diff(g.rowptr) <= 7)


def test_config2_shape():
    g = I.config(2)
    assert g.n == 16_000_000
    undirected_full = 31 * 500_000 + 32 * 499_999
    dropped = undirected_full - (g.nnz - g.n) // 2
    # 1% drop: about 315k edges, within 5 standard deviations
    assert abs(dropped - 0.01 * undirected_full) < 5 * np.sqrt(undirected_full * 0.01)


@pytest.mark.parametrize("seed", range(3))
def test_rgg_patches(seed):
    g = I.rgg_patches(3000, seed)
    _check_csr(g)
    mean_deg = (g.nnz - g.n) / g.n
    assert 8 < mean_deg < 13


def test_batch_and_concat():
    gs = I.batch_graphs(12, seed=4, lo=100, hi=3000)
    assert len(gs) == 12
    vtx, nz, rp, ci = I.concat_batch(gs)
    assert vtx[-1] == sum(g.n for g in gs) and nz[-1] == sum(g.nnz for g in gs)
    for i, g in enumerate(gs):
        _check_csr(g)
        s = vtx[i] + i
        assert np.array_equal(rp[s:s + g.n + 1], g.rowptr)
        assert np.array_equal(ci[nz[i]:nz[i + 1]], g.colidx)


def test_request_stream_is_seeded():
    a = I.request_stream(50, rate=10.0)
    b = I.request_stream(50, rate=10.0)
    assert a == b
    t = [x[0] for x in a]
    assert all(t1 > t0 for t0, t1 in zip(t, t[1:]))


def test_small_graphs():
    for g in [I.path(1), I.path(6, seed=3), I.cycle(5), I.complete(4), I.star(5, 2),
              I.erdos_renyi(30, 0.1, 1), I.random_tree(20, 2), I.grid3d(2, 3, 4, seed=1)]:
        _check_csr(g)
    g = I.drop_diagonal(I.path(5))
    _check_csr(g, diag=False)
    assert g.nnz == 8
