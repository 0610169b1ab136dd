"""Applying an ordering: the oracle's B = P A P^T and y = A x are pinned to
library routines and to the ordering's own statistics (CPU); the GPU's
permuted matrix equals the oracle's exactly and its product agrees within
the float64 rounding bound (GPU)."""

import numpy as np
import pytest
import scipy.linalg
import scipy.sparse as sp

import oracle
from paper_1610_08128_amd import inputs as I


def _graphs():
    return [I.grid2d(9, 13, seed=3), I.rgg_patches(300, 5), I.path(7, seed=2),
            I.add_random_self_loops(I.random_tree(60, 4), 0.3, 4),
            I.disjoint_union([I.complete(5), I.grid3d(3, 4, 2, seed=1)], seed=9),
            # rows around and well past the register-sort limit of the
            # permutation (16 entries), and a very long star row
            I.disjoint_union([I.complete(16), I.complete(17), I.star(40), I.path(3)], seed=5),
            I.erdos_renyi(120, 0.2, 6)]


def _csr(g, vals=None):
    data = np.ones(g.nnz) if vals is None else vals
    return sp.csr_matrix((data, g.colidx, g.rowptr), shape=(g.n, g.n))


@pytest.mark.parametrize("gi", range(7))
def test_oracle_permute_matches_scipy_indexing(gi):
    g = _graphs()[gi]
    rng = np.random.default_rng(gi)
    vals = rng.standard_normal(g.nnz)
    perm = oracle.rcm(g.n, g.rowptr, g.colidx).perm
    rp, ci, v = oracle.permute_csr(g.n, g.rowptr, g.colidx, perm, vals)
    want = _csr(g, vals)[perm][:, perm].tocsr()
    want.sort_indices()
    assert np.array_equal(rp, want.indptr) and np.array_equal(ci, want.indices)
    assert np.array_equal(v, want.data)


@pytest.mark.parametrize("gi", range(7))
def test_oracle_permute_gives_the_reported_bandwidth(gi):
    # the bandwidth of the permuted pattern (library routine on the dense
    # matrix with the diagonal present) is the ordering's bandwidth_after
    g = _graphs()[gi]
    r = oracle.rcm(g.n, g.rowptr, g.colidx)
    rp, ci, _ = oracle.permute_csr(g.n, g.rowptr, g.colidx, r.perm)
    dense = sp.csr_matrix((np.ones(ci.size), ci, rp), shape=(g.n, g.n)).toarray()
    dense[np.arange(g.n), np.arange(g.n)] = 1.0
    lo, hi = scipy.linalg.bandwidth(dense)
    assert max(lo, hi) == r.stats["bandwidth_after"]


def test_oracle_permute_identity_and_round_trip():
    g = I.rgg_patches(200, 3)
    ident = np.arange(g.n, dtype=np.int32)
    rp, ci, _ = oracle.permute_csr(g.n, g.rowptr, g.colidx, ident)
    want = _csr(g)
    want.sort_indices()
    assert np.array_equal(rp, want.indptr) and np.array_equal(ci, want.indices)
    perm = np.random.default_rng(1).permutation(g.n).astype(np.int32)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(g.n, dtype=np.int32)
    rp1, ci1, _ = oracle.permute_csr(g.n, g.rowptr, g.colidx, perm)
    rp2, ci2, _ = oracle.permute_csr(g.n, rp1, ci1, inv)
    assert np.array_equal(rp2, want.indptr) and np.array_equal(ci2, want.indices)


def test_oracle_spmv_matches_scipy():
    g = I.grid3d(5, 6, 7, seed=2)
    rng = np.random.default_rng(0)
    vals = rng.standard_normal(g.nnz)
    x = rng.standard_normal(g.n)
    y = oracle.spmv(g.n, g.rowptr, g.colidx, x, vals)
    assert np.allclose(y, _csr(g, vals) @ x, rtol=1e-14, atol=1e-14)
    y1 = oracle.spmv(g.n, g.rowptr, g.colidx, x)
    assert np.allclose(y1, _csr(g) @ x, rtol=1e-14, atol=1e-14)


@pytest.mark.gpu
@pytest.mark.parametrize("gi", range(7))
def test_gpu_permute_and_spmv(gi):
    import torch
    from paper_1610_08128_amd import apply, rcm

    g = _graphs()[gi]
    rng = np.random.default_rng(10 + gi)
    vals = rng.standard_normal(g.nnz)
    x = rng.standard_normal(g.n)
    rp = torch.from_numpy(g.rowptr).cuda()
    ci = torch.from_numpy(g.colidx).cuda()
    perm, iperm, st = rcm.order(rp, ci, return_iperm=True)
    want_rp, want_ci, want_v = oracle.permute_csr(g.n, g.rowptr, g.colidx, perm.cpu().numpy(), vals)
    vd = torch.from_numpy(vals).cuda()
    brp, bci, bv = apply.permute(rp, ci, perm, iperm, vd)
    assert np.array_equal(brp.cpu().numpy(), want_rp)
    assert np.array_equal(bci.cpu().numpy(), want_ci)
    assert np.array_equal(bv.cpu().numpy(), want_v)  # values are moved, not computed
    brp2, bci2, _ = apply.permute(rp, ci, perm, iperm)
    assert np.array_equal(bci2.cpu().numpy(), want_ci)
    # product: each |y_i - y'_i| <= 2 * L_i * u * sum_j |a_ij x_j| for row length L_i
    # (two summation orders, each within L_i * u of the exact sum); u = 2^-53
    y = apply.spmv(brp, bci, torch.from_numpy(x).cuda(), bv).cpu().numpy()
    want_y = oracle.spmv(g.n, want_rp, want_ci, x, want_v)
    L = np.diff(want_rp).astype(np.float64)
    absum = oracle.spmv(g.n, want_rp, want_ci, np.abs(x), np.abs(want_v))
    assert np.all(np.abs(y - want_y) <= 2 * L * 2.0**-53 * absum + 1e-300)
    # the permuted pattern's bandwidth is the one the ordering reported
    rows = np.repeat(np.arange(g.n), np.diff(want_rp))
    bw = int(np.max(np.maximum(rows - want_ci, 0))) if want_ci.size else 0
    assert bw == st["bandwidth_after"]


def _check_gpu_permute(g, seed):
    import torch
    from paper_1610_08128_amd import apply, rcm

    rng = np.random.default_rng(seed)
    vals = rng.standard_normal(g.nnz)
    rp = torch.from_numpy(g.rowptr).cuda()
    ci = torch.from_numpy(g.colidx).cuda()
    perm, iperm, _ = rcm.order(rp, ci, return_iperm=True)
    want_rp, want_ci, want_v = oracle.permute_csr(g.n, g.rowptr, g.colidx, perm.cpu().numpy(),
                                                  vals)
    brp, bci, bv = apply.permute(rp, ci, perm, iperm, torch.from_numpy(vals).cuda())
    assert np.array_equal(brp.cpu().numpy(), want_rp)
    assert np.array_equal(bci.cpu().numpy(), want_ci)
    assert np.array_equal(bv.cpu().numpy(), want_v)


@pytest.mark.gpu
def test_gpu_permute_dense_rows():
    """About 60 entries per row: a block's 256 rows then hold more entries than
    its LDS stage, so the rows are written directly; rows in random order."""
    g = I.shuffle_rows(I.erdos_renyi(600, 0.1, 11), 2)
    assert int(g.rowptr[256]) > 256 * 16
    _check_gpu_permute(g, 1)


@pytest.mark.gpu
def test_gpu_permute_many_tiles():
    """More rows than one pass of the grid covers (8,192 blocks of 256 rows),
    so blocks take a second tile."""
    g = I.grid2d(1500, 1500, seed=12)
    assert g.n > 8192 * 256
    _check_gpu_permute(g, 2)


@pytest.mark.gpu
def test_gpu_permute_long_rows():
    """Rows longer than a register sort: rows of 17 to 300 entries, and hub
    rows of exactly the LDS sort's 8,192 entries, one more, and 20,001 (the
    last two sort in the scratch array), with rows in random order."""
    g = I.shuffle_rows(I.disjoint_union([I.star(20001), I.star(8192), I.star(8193),
                                         I.erdos_renyi(900, 0.15, 13), I.star(18), I.star(300)],
                                        seed=14), 3)
    lens = np.diff(g.rowptr)
    assert {8192, 8193, 20001} <= set(lens.tolist())
    _check_gpu_permute(g, 4)
