"""Input generators (no GPU): the sampled-row assembly of the five-point
operator used to check large-grid products on a few rows."""
import numpy as np
import scipy.sparse as sp

import instances


def test_stencil_csr_sampled_rows_equal_full_assembly():
    N = 9
    wx, wy = instances.varcoef_weights(N)
    rng = np.random.default_rng(0)
    wx = wx * rng.uniform(0.5, 1.5, size=wx.shape)
    wy = wy * rng.uniform(0.5, 1.5, size=wy.shape)
    full = instances.stencil_csr(N, wx, wy)
    A = sp.csr_matrix((full[2], full[1], full[0]), shape=(N * N, N * N))
    rows = np.array([0, 1, N - 1, N, 40, N * N - N, N * N - 1])
    part = instances.stencil_csr(N, wx, wy, rows)
    B = sp.csr_matrix((part[2], part[1], part[0]), shape=(N * N, N * N))
    assert part[0].dtype == np.int32 and part[1].dtype == np.int32
    assert (A[rows] != B[rows]).nnz == 0
    others = np.setdiff1d(np.arange(N * N), rows)
    assert B[others].nnz == 0
    v = rng.standard_normal(N * N)
    assert np.array_equal((B @ v)[rows], (A @ v)[rows])


def test_batch_member_equals_batch_entry():
    full = instances.batch512(0, count=16, nmin=8, nmax=24)
    for i in (0, 7, 15):
        one = instances.batch_member(0, i, count=16, nmin=8, nmax=24)
        assert one.name == full[i].name and one.N == full[i].N
        for k in ("b", "l", "u", "x0"):
            assert np.array_equal(getattr(one, k), getattr(full[i], k))
