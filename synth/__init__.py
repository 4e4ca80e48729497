"""Seeded synthetic inputs for the block LOBPCG solver and its tests.

This module only *draws* matrices and starting blocks.  It contains none of
the eigensolver's arithmetic, so both the CPU oracle and the GPU path may use
it without sharing any solver code.

Conventions (the same for every generator):
  * indices are 0-based; ``U(a, b)`` is half-open; ``N(mu, s**2)`` takes the
    *variance* as its second argument, so ``N(0, 1e-3**2)`` has std 1e-3;
  * every symmetric random matrix draws its strict upper triangle, mirrors it,
    and draws the diagonal separately;
  * every generator takes an integer seed and uses numpy's PCG64, so the same
    seed always yields the same array on any machine.

Workload families (stand-ins for the paper's quantum-chemistry matrices,
Sec. 4: Full CI Hamiltonians, SCF orbital Hessians, CASSCF augmented
Hessians, none of which can be built without a quantum-chemistry code):
  * ``dense_dd``      dense, strongly diagonally dominant (SCF Hessian at
                      convergence), n = 2000 by default;
  * ``csr_banded``    sparse, diagonally dominant, random offsets inside a
                      band (Full-CI-like), n = 1e6 by default;
  * ``dense_hessian`` dense, not diagonally dominant: diagonal + rank-64
                      term + Wigner noise (Hueckel-guess / CASSCF Hessian);
  * ``csr_family``    sparse matrices with a drawn diagonal-dominance ratio
                      (preconditioner study, Sec. 4.4);
  * ``kronsum``       matrix-free A (x) I + I (x) A + diag(V) (CI-sigma-like).
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np

__all__ = [
    "rng",
    "CSR",
    "dense_dd",
    "csr_banded",
    "dense_hessian",
    "csr_family",
    "kronsum",
    "start_block",
    "laplacian_1d",
    "prescribed_spectrum",
    "random_symmetric",
    "csr_from_dense",
    "array_digest",
    "SEEDS",
]

# Matrix seed / start-block seed per workload.
SEEDS = {
    "dense_dd": (2305101, 2305201),
    "csr_banded": (2305102, 2305202),
    "dense_hessian": (2305103, 2305203),
    "kronsum": (2305105, 2305205),
}


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


@dataclasses.dataclass
class CSR:
    """Symmetric matrix in CSR form: int32 row pointers and columns, fp64 values.

    Columns are sorted within each row; the diagonal entry is always stored.
    ``diag`` is a copy of the diagonal (the Jacobi preconditioner's input).
    """

    n: int
    row_ptr: np.ndarray  # int32 (n+1)
    col: np.ndarray  # int32 (nnz)
    val: np.ndarray  # float64 (nnz)
    diag: np.ndarray  # float64 (n)

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        return self.to_scipy().toarray()


def _csr_from_triplets(n, rows, cols, vals) -> CSR:
    import scipy.sparse as sp

    m = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    m.sum_duplicates()
    m.sort_indices()
    if m.indptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("nnz does not fit int32 row pointers")
    diag = np.asarray(m.diagonal(), dtype=np.float64)
    return CSR(
        n=n,
        row_ptr=m.indptr.astype(np.int32),
        col=m.indices.astype(np.int32),
        val=m.data.astype(np.float64),
        diag=diag,
    )


def csr_from_dense(A: np.ndarray) -> CSR:
    """Exact CSR copy of a dense symmetric matrix (keeps the full diagonal)."""
    n = A.shape[0]
    r, c = np.nonzero(A)
    rows = np.concatenate([r, np.arange(n)])
    cols = np.concatenate([c, np.arange(n)])
    vals = np.concatenate([A[r, c], np.zeros(n)])
    out = _csr_from_triplets(n, rows, cols, vals)
    return out


def dense_dd(n: int = 2000, seed: int = 2305101) -> np.ndarray:
    """Dense, strongly diagonally dominant symmetric matrix (row-major fp64).

    d_i = 1 + 0.05 i + U(0, 0.01);  a_ij ~ N(0, (1e-3)^2) for i < j, mirrored.
    """
    g = rng(seed)
    d = 1.0 + 0.05 * np.arange(n, dtype=np.float64) + g.uniform(0.0, 0.01, n)
    E = g.normal(0.0, 1e-3, (n, n))
    A = np.triu(E, 1)
    A = A + A.T
    A[np.diag_indices(n)] = d
    return np.ascontiguousarray(A)


def csr_banded(
    n: int = 1_000_000,
    seed: int = 2305102,
    offsets_per_row: int = 20,
    band: int = 5000,
    offdiag: float = 1e-3,
    diag_slope: float = 1e-5,
    diag_noise: float = 0.1,
) -> CSR:
    """Sparse, diagonally dominant symmetric CSR matrix.

    Row i draws ``offsets_per_row`` offsets d ~ U{1..band}; repeated offsets
    are dropped and so are columns j = i + d >= n.  Values U(-offdiag,
    offdiag) are mirrored to (j, i).  Diagonal d_i = 1 + diag_slope * i +
    U(0, diag_noise).  About 2*offsets_per_row + 1 stored entries per row.
    """
    g = rng(seed)
    offs = g.integers(1, band + 1, size=(n, offsets_per_row), dtype=np.int64)
    vals = g.uniform(-offdiag, offdiag, size=(n, offsets_per_row))
    d = 1.0 + diag_slope * np.arange(n, dtype=np.float64) + g.uniform(0.0, diag_noise, n)
    order = np.argsort(offs, axis=1, kind="stable")
    offs = np.take_along_axis(offs, order, axis=1)
    vals = np.take_along_axis(vals, order, axis=1)
    keep = np.ones_like(offs, dtype=bool)
    keep[:, 1:] = offs[:, 1:] != offs[:, :-1]
    i = np.arange(n, dtype=np.int64)[:, None]
    j = i + offs
    keep &= j < n
    ii = np.broadcast_to(i, offs.shape)[keep]
    jj = j[keep]
    vv = vals[keep]
    del offs, vals, j, keep
    rows = np.concatenate([ii, jj, np.arange(n, dtype=np.int64)])
    cols = np.concatenate([jj, ii, np.arange(n, dtype=np.int64)])
    vv = np.concatenate([vv, vv, d])
    return _csr_from_triplets(n, rows, cols, vv)


def dense_hessian(n: int = 20000, seed: int = 2305103, rank: int = 64) -> np.ndarray:
    """Dense symmetric matrix that is *not* diagonally dominant.

    A = diag(D) + U diag(S) U^T + E with D ~ U(0.1, 10), U the Q factor of an
    n x rank N(0,1) matrix, S ~ U(-5, 5), E_ij ~ N(0, 0.05^2) for i <= j,
    mirrored.
    """
    g = rng(seed)
    D = g.uniform(0.1, 10.0, n)
    G = g.standard_normal((n, rank))
    U, _ = np.linalg.qr(G)
    S = g.uniform(-5.0, 5.0, rank)
    A = g.normal(0.0, 0.05, (n, n))
    A = np.triu(A)
    A = A + np.triu(A, 1).T
    A += (U * S) @ U.T
    A[np.diag_indices(n)] += D
    # exact symmetry (the low-rank product is symmetric only up to rounding)
    A = np.triu(A) + np.triu(A, 1).T
    return np.ascontiguousarray(A)


def csr_family(
    idx: int,
    n: int = 200_000,
    offsets_per_row: int = 15,
    band: int = 5000,
    ratio: float | None = None,
    base_seed: int = 2305400,
) -> tuple[CSR, float]:
    """One member of the preconditioner-study family.

    Off-diagonal pattern as in ``csr_banded`` with values U(-1, 1); with
    R_i = sum_{j != i} |a_ij| the diagonal is d_i = rho * R_i * (1 + U(0, 1))
    where the dominance ratio rho ~ U(0.3, 3) is drawn per matrix (rho >= 1
    is strictly dominant, rho < 1 is not).  Returns (matrix, rho).
    """
    g = rng(base_seed + idx)
    rho = float(g.uniform(0.3, 3.0)) if ratio is None else float(ratio)
    offs = g.integers(1, band + 1, size=(n, offsets_per_row), dtype=np.int64)
    vals = g.uniform(-1.0, 1.0, size=(n, offsets_per_row))
    jit = g.uniform(0.0, 1.0, n)
    order = np.argsort(offs, axis=1, kind="stable")
    offs = np.take_along_axis(offs, order, axis=1)
    vals = np.take_along_axis(vals, order, axis=1)
    keep = np.ones_like(offs, dtype=bool)
    keep[:, 1:] = offs[:, 1:] != offs[:, :-1]
    i = np.arange(n, dtype=np.int64)[:, None]
    j = i + offs
    keep &= j < n
    ii = np.broadcast_to(i, offs.shape)[keep]
    jj = j[keep]
    vv = vals[keep]
    rowsum = np.bincount(ii, weights=np.abs(vv), minlength=n) + np.bincount(
        jj, weights=np.abs(vv), minlength=n
    )
    d = rho * rowsum * (1.0 + jit)
    rows = np.concatenate([ii, jj, np.arange(n, dtype=np.int64)])
    cols = np.concatenate([jj, ii, np.arange(n, dtype=np.int64)])
    allv = np.concatenate([vv, vv, d])
    return _csr_from_triplets(n, rows, cols, allv), rho


def kronsum(na: int = 4096, seed: int = 2305105, potential: float = 0.1) -> tuple[np.ndarray, np.ndarray]:
    """Factors of H = A (x) I + I (x) A + diag(vec V), n = na^2.

    A_ii = sort(U(0, 20)), A_ij ~ N(0, 0.01^2) mirrored;
    V_ij = potential * cos((i * j) mod 97) (integer radians, int64 product).
    The vector index of entry (i, j) is i * na + j (row-major reshape).
    """
    g = rng(seed)
    diag = np.sort(g.uniform(0.0, 20.0, na))
    E = g.normal(0.0, 0.01, (na, na))
    A = np.triu(E, 1)
    A = A + A.T
    A[np.diag_indices(na)] = diag
    i = np.arange(na, dtype=np.int64)
    V = potential * np.cos(((i[:, None] * i[None, :]) % 97).astype(np.float64))
    return np.ascontiguousarray(A), np.ascontiguousarray(V)


def start_block(n: int, m: int, seed: int) -> np.ndarray:
    """Initial block X0 ~ N(0, 1)^{n x m}, row-major fp64."""
    return np.ascontiguousarray(rng(seed).standard_normal((n, m)))


def laplacian_1d(n: int) -> CSR:
    """tridiag(-1, 2, -1) of order n (Dirichlet 1-D Laplacian)."""
    i = np.arange(n, dtype=np.int64)
    rows = np.concatenate([i, i[:-1], i[1:]])
    cols = np.concatenate([i, i[1:], i[:-1]])
    vals = np.concatenate([np.full(n, 2.0), np.full(n - 1, -1.0), np.full(n - 1, -1.0)])
    return _csr_from_triplets(n, rows, cols, vals)


def prescribed_spectrum(evals: np.ndarray, seed: int) -> tuple[np.ndarray, np.ndarray]:
    """Dense Q diag(evals) Q^T with Q Haar-random orthogonal; returns (A, Q)."""
    evals = np.asarray(evals, dtype=np.float64)
    n = evals.shape[0]
    G = rng(seed).standard_normal((n, n))
    Q, R = np.linalg.qr(G)
    Q = Q * np.sign(np.diag(R))
    A = (Q * evals) @ Q.T
    A = 0.5 * (A + A.T)
    return np.ascontiguousarray(A), Q


def random_symmetric(n: int, seed: int, scale: float = 1.0) -> np.ndarray:
    """Dense symmetric with N(0, scale^2) upper triangle and diagonal."""
    g = rng(seed)
    E = g.normal(0.0, scale, (n, n))
    A = np.triu(E)
    A = A + np.triu(A, 1).T
    return np.ascontiguousarray(A)


def array_digest(*arrays: np.ndarray) -> str:
    """SHA-256 over the raw bytes of the arrays (for fixture bookkeeping)."""
    h = hashlib.sha256()
    for a in arrays:
        a = np.ascontiguousarray(a)
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()
