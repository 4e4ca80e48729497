"""Checks on the seeded input generators (shapes, symmetry, value ranges)."""
import numpy as np

import synth


def test_dense_dd_shape_and_symmetry():
    A = synth.dense_dd(300, seed=1)
    assert A.shape == (300, 300) and A.flags.c_contiguous
    assert np.array_equal(A, A.T)
    d = np.diag(A) - 1.0 - 0.05 * np.arange(300)
    assert d.min() >= 0.0 and d.max() < 0.01
    off = A - np.diag(np.diag(A))
    assert abs(off.std() - 1e-3) < 1e-4
    assert np.array_equal(A, synth.dense_dd(300, seed=1))


def test_csr_banded_structure():
    n = 20000
    C = synth.csr_banded(n=n, seed=3, band=500, diag_slope=1e-3)
    S = C.to_scipy()
    assert (S - S.T).nnz == 0
    assert C.row_ptr.dtype == np.int32 and C.col.dtype == np.int32
    nnz_row = np.diff(C.row_ptr)
    assert 38 <= nnz_row.mean() <= 42
    r = np.repeat(np.arange(n), nnz_row)
    assert np.abs(C.col.astype(np.int64) - r).max() <= 500
    # columns sorted, no duplicates, diagonal present
    for i in (0, 1, 777, n - 1):
        cols = C.col[C.row_ptr[i]:C.row_ptr[i + 1]]
        assert np.all(np.diff(cols) > 0) and i in cols
    off = C.val[C.col != r]
    assert np.abs(off).max() <= 1e-3
    assert np.allclose(C.diag, S.diagonal())
    assert synth.array_digest(C.val) == synth.array_digest(synth.csr_banded(n=n, seed=3, band=500, diag_slope=1e-3).val)


def test_dense_hessian_not_dominant():
    A = synth.dense_hessian(600, seed=2, rank=16)
    assert np.array_equal(A, A.T)
    off = np.abs(A).sum(1) - np.abs(np.diag(A))
    assert np.mean(off > np.abs(np.diag(A))) > 0.5


def test_csr_family_ratio():
    C, rho = synth.csr_family(3, n=5000, band=300)
    assert 0.3 <= rho < 3.0
    S = C.to_scipy()
    assert (S - S.T).nnz == 0
    R = np.asarray(abs(S).sum(1)).ravel() - np.abs(C.diag)
    ratio = C.diag / R
    assert np.all(ratio >= rho - 1e-12) and np.all(ratio <= 2 * rho + 1e-12)


def test_kronsum_factors():
    A, V = synth.kronsum(na=64, seed=1)
    assert np.array_equal(A, A.T) and np.all(np.diff(np.diag(A)) >= 0)
    i = np.arange(64)
    assert np.allclose(V, 0.1 * np.cos((np.outer(i, i) % 97).astype(float)))
    assert np.array_equal(V, V.T)


def test_start_block_seeded():
    a = synth.start_block(100, 4, 7)
    assert a.shape == (100, 4) and np.array_equal(a, synth.start_block(100, 4, 7))
    assert not np.array_equal(a, synth.start_block(100, 4, 8))
