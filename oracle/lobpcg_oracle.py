"""Plain FP64 CPU oracle for the robust block LOBPCG of Nottoli, Gianni,
Levitt and Lipparini, "A robust, open-source implementation of the locally
optimal block preconditioned conjugate gradient for large eigenvalue problems
in quantum chemistry" (arXiv:2305.06668).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the GPU library: it uses numpy / scipy (LAPACK, OpenBLAS, scipy.sparse) for
every step, in float64, in the order the paper states them.

What is computed (paper Sec. 2 and Sec. 3):
  * ``ortho``          Alg. 2 (Cholesky orthonormalisation with repetition and
                       a diagonal shift when the factorisation fails, after
                       Fukaya et al.'s shifted CholeskyQR; Sec. 3.2);
  * ``ortho_against``  Alg. 3 (project out Y, re-orthonormalise, loop);
  * ``rayleigh_ritz``  the RR step of Sec. 2 on an orthonormal basis;
  * ``lobpcg``         Alg. 1 with the orthonormal (X, W, P) basis, P built
                       implicitly from the RR coefficients (eq. a_block and
                       neweigv), operator applications reused only through
                       orthonormal coefficient matrices, and locking
                       (Sec. 3.1, paragraphs "Basis selection", "Reuse of
                       applications", "Locking").

Readings taken where the paper is silent or ambiguous (each is also listed in
the design notes of the repository):
  R1  Alg. 1 writes the residual with the old iterate right after forming the
      new one; the residual is taken for the *new* Ritz pairs.
  R2  The initial RR of Alg. 1 needs an orthonormal X0, so X0 is passed
      through ``ortho`` first.
  R3  Alg. 3 is read as a do-while: normalise the columns, always project and
      orthonormalise once, then test ||Y^T X|| on the orthonormal X.
  R4  The norms in ||X^T X - I|| and ||Y^T X|| are max-abs entries; pass caps
      6 (Alg. 2) and 4 (Alg. 3); hitting a cap is counted as "stalled".
  R5  Shift: eps = 2^-52, ||X|| = ||X||_F = sqrt(trace(X^T X)) taken after
      column normalisation, sigma = alpha * eps * ||X||_F starting at
      alpha = 100 and growing 10x per retry, at most 20 retries, then the
      SVQB orthonormalisation of Stathopoulos and Wu as a last resort.
  R6  Columns are scaled to unit 2-norm before the first factorisation; a
      column of exact zeros is replaced by a deterministic SplitMix64 vector.
  R7  Jacobi preconditioner.  Sec. 2 gives T = (diag(A) - rho I)^-1 as an
      example for diagonally dominant A.  LOBPCG's convergence theory wants a
      positive definite T, and from a random start (rho in the middle of the
      diagonal) the indefinite form stalls, so the default is the absolute
      value T_j = |diag(A) - theta_j I|^-1, which equals the paper's form
      wherever diag(A) > theta_j.  The signed form is kept as an option
      ("diag_signed").  Either way a denominator x with |x| < delta_j =
      1e-8 max(1, |theta_j|) is replaced by copysign(delta_j, x), sign(0) = +.
  R8  Locking: m_conv is the number of *leading* columns whose residual
      2-norm is <= tol, never decreasing; locked columns stay in X and are
      still rotated by the RR; W and P are built for the active columns only.
  R9  Convergence is the per-column residual 2-norm ||A x - theta x|| <= tol
      with ||x|| = 1.  When the RR residuals say "converged", X is passed
      through ``ortho`` once more and the residual is recomputed from an
      explicit product A X (the true residual); if that check fails, the
      iteration restarts as Alg. 1 starts: Rayleigh-Ritz on [X] with the
      explicit product, P dropped, locking recounted, and the next
      convergence test only after one more iteration, which locks at most
      k - 1 columns (so it has an active column, and a check that fails
      again cannot repeat without progress).
  R10 The reduced matrix is symmetrised, a <- (a + a^T) / 2, before eigh.
  R17 Cheap exits (optional; Sec. 3.2 proposes them after Alg. 2 and Alg. 3
      without fixing a rule): Alg. 2 stops without a new overlap after an
      unshifted factor whose e = ||I - L||_F < 1/2 gives c(n) eps kappa^2 <=
      tau, kappa = (1 + e) / (1 - e); Alg. 3 stops without Y^T X when
      c(n) eps g <= tau, g the growth of the ortho call (normalisation scale
      times a bound on ||L^-1|| per factor).  c(n) = max(4, 0.02 sqrt(n)) is
      twice the loss measured on this oracle.
  R19 Tridiagonal preconditioner (Sec. 4.4): T_j = tridiag(e, t, e) with
      t_i = max(|d_i - theta_j|, |e_{i-1}| + |e_i| + delta_j), the positive
      definite counterpart of R7 (strictly diagonally dominant), solved by
      LAPACK's Gaussian elimination with partial pivoting (dgtsv).
  R22 Stalled recurrence: the residuals of Alg. 1's recurrence come from
      X and A X carried through the Rayleigh-Ritz coefficients ("Reuse of
      applications", Sec. 3.1), and rounding in those implicit products can
      leave them on a floor above tol while the true residuals are below
      it (or the reverse for a locked column), so that R9's check is never
      reached.  When the largest residual of the sought active columns
      (m_conv <= j < k) is within 100 tol and has not fallen below 0.99
      times its smallest value since the last check for ``stall_window``
      consecutive Rayleigh-Ritz steps, R9's check runs although m_conv < k:
      it ends the solve if the true residuals meet tol, else restarts as R9
      does.  (A plateau far above tol is slow convergence, which a restart,
      dropping P, would only slow down.)
  R16 Eigenvectors of the reduced matrix are oriented so that the diagonal
      entry u[j, j] is >= 0 (for the X block: the new Ritz vector continues
      the old one).  The "Basis selection" paragraph forms P from the
      coefficients of X^{k+1} - X^k by subtracting the identity from u_xx,
      which presumes that orientation; an eigensolver's signs are otherwise
      arbitrary, and a flipped column turns the small difference into
      2 x_j minus the difference, which the ortho against u_x then recovers
      only to eps / ||difference||.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Optional

import numpy as np
import scipy.linalg as sla

EPS = 2.0 ** -52  # double precision unit roundoff used for the shift (R5)
TAU_ORTHO = 1e-14  # Sec. 4: the only ortho parameter used in all experiments
SHIFT_ALPHA0 = 100.0  # Sec. 3.2: start at 100 x norm(X) x machine precision
SHIFT_GROWTH = 10.0  # R5
SHIFT_RETRIES = 20  # R5
ORTHO_MAX_PASSES = 6  # R4 (Alg. 2)
ORTHO_Y_MAX_PASSES = 4  # R4 (Alg. 3)
PRECOND_GUARD = 1e-8  # R7
# Cheap exits of Alg. 2 / Alg. 3 (the estimates Sec. 3.2 proposes after each
# algorithm; reading R17): one Cholesky-QR pass leaves X^T X - I at about
# c eps kappa^2, and one project + ortho pass leaves Y^T X at about c eps g,
# with c measured on this oracle at up to 1.5 (n = 1e4) .. 8.5 (n = 1e6),
# ~0.0085 sqrt(n); the exits use twice that.


def cheap_exit_factor(n: int) -> float:
    return max(4.0, 0.02 * math.sqrt(n))
ZERO_COLUMN_SEED = 0x2305066680000000  # R6

Operator = Callable[[np.ndarray], np.ndarray]


# ---------------------------------------------------------------------------
# bookkeeping


@dataclasses.dataclass
class OrthoStats:
    grams: int = 0  # overlap matrices formed (checks included)
    factorizations: int = 0  # Cholesky attempts, failed ones included
    failed_factorizations: int = 0
    shifted: int = 0  # successful factorisations that needed a shift
    updates: int = 0  # X <- X L^-T applications
    ortho_calls: int = 0
    against_calls: int = 0
    against_passes: int = 0  # project+ortho passes of Alg. 3
    stalled: int = 0
    svqb: int = 0
    zero_columns: int = 0
    cheap_exits: int = 0  # overlaps not formed thanks to a cheap exit (R17)

    def merge(self, o: "OrthoStats") -> None:
        for f in dataclasses.fields(self):
            setattr(self, f.name, getattr(self, f.name) + getattr(o, f.name))


class OrthoFailed(RuntimeError):
    pass


# ---------------------------------------------------------------------------
# a counter-based generator for the zero-column replacement (R6)

_MASK64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """SplitMix64 finaliser (Steele, Lea, Flood 2014) on a 64-bit counter."""
    z = (x + 0x9E3779B97F4A7C15) & _MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
    return z ^ (z >> 31)


def splitmix_column(n: int, col: int, seed: int = ZERO_COLUMN_SEED) -> np.ndarray:
    """Entry i is (splitmix64(seed + col*n + i) >> 11) * 2^-53 - 0.5."""
    out = np.empty(n, dtype=np.float64)
    base = seed + col * n
    for i in range(n):
        out[i] = (splitmix64((base + i) & _MASK64) >> 11) * (2.0 ** -53) - 0.5
    return out


# ---------------------------------------------------------------------------
# Sec. 3.2, Alg. 2 and Alg. 3


def max_abs(M: np.ndarray) -> float:
    return float(np.max(np.abs(M))) if M.size else 0.0


def normalize_columns(X: np.ndarray, stats: Optional[OrthoStats] = None) -> np.ndarray:
    """Scale every column to unit 2-norm (R6)."""
    X = np.array(X, dtype=np.float64, copy=True)
    norms = np.sqrt(np.einsum("ij,ij->j", X, X))
    for j in np.nonzero(norms == 0.0)[0]:
        X[:, j] = splitmix_column(X.shape[0], int(j))
        norms[j] = math.sqrt(float(X[:, j] @ X[:, j]))
        if stats is not None:
            stats.zero_columns += 1
    return X / norms


def _potrf(M: np.ndarray) -> Optional[np.ndarray]:
    """Lower Cholesky factor, or None when the factorisation breaks down."""
    try:
        L = np.linalg.cholesky(M)
    except np.linalg.LinAlgError:
        return None
    if not np.all(np.isfinite(L)):
        return None
    return L


def shifted_cholesky(
    M: np.ndarray, stats: OrthoStats, retries: int = SHIFT_RETRIES
) -> Optional[np.ndarray]:
    """Cholesky of M; on failure add alpha*eps*||X||_F to the diagonal and
    increase alpha until it succeeds (Sec. 3.2, Alg. 2; reading R5), at most
    ``retries`` shifted attempts.

    Returns None when every retry failed (the caller then uses SVQB)."""
    stats.factorizations += 1
    L = _potrf(M)
    if L is not None:
        return L
    stats.failed_factorizations += 1
    norm_x = math.sqrt(max(float(np.trace(M)), 0.0))
    alpha = SHIFT_ALPHA0
    eye = np.eye(M.shape[0])
    for _ in range(retries):
        sigma = alpha * EPS * norm_x
        stats.factorizations += 1
        L = _potrf(M + sigma * eye)
        if L is not None:
            stats.shifted += 1
            return L
        stats.failed_factorizations += 1
        alpha *= SHIFT_GROWTH
    return None


def svqb(X: np.ndarray, M: np.ndarray, stats: OrthoStats) -> np.ndarray:
    """Stathopoulos-Wu SVQB: X <- X U Sigma^-1/2 with small eigenvalues of
    the overlap clamped to eps * max(Sigma); no column is dropped."""
    stats.svqb += 1
    s, U = np.linalg.eigh(M)
    s = np.maximum(s, EPS * max(float(s.max()), 0.0))
    if not np.all(s > 0.0):
        raise OrthoFailed("overlap matrix has no positive eigenvalue")
    return (X @ U) / np.sqrt(s)


def inverse_factor_bound(L: np.ndarray):
    """Upper bound b >= ||L^-1||_2 for a lower-triangular factor, and
    e = ||I - L||_F: b = 1 / (1 - e) when e < 1/2 (Neumann series), else
    ||L^-1||_F."""
    m = L.shape[0]
    e = float(np.linalg.norm(np.eye(m) - L))
    if e < 0.5:
        return 1.0 / (1.0 - e), e
    Li = sla.solve_triangular(L, np.eye(m), lower=True, check_finite=False)
    return float(np.linalg.norm(Li)), e


def ortho(
    X: np.ndarray,
    tau: float = TAU_ORTHO,
    stats: Optional[OrthoStats] = None,
    max_passes: int = ORTHO_MAX_PASSES,
    shift_retries: int = SHIFT_RETRIES,
    cheap_exit: bool = False,
    growth: Optional[dict] = None,
) -> np.ndarray:
    """Alg. 2: while ||X^T X - I|| > tau, factor M = X^T X = L L^T (shifting
    the diagonal when the factorisation fails) and set X <- X L^-T.  When
    the plain factorisation and all ``shift_retries`` shifted ones fail, the
    pass uses SVQB instead (reading R5).

    ``cheap_exit`` (reading R17): after an unshifted factor with
    e = ||I - L||_F < 1/2, kappa(L) <= (1 + e) / (1 - e) bounds the
    conditioning the pass removed; when c(n) eps kappa^2 <= tau the new X is
    taken as orthonormal without forming its overlap.  ``growth`` (a dict,
    optional) receives "g": the amplification this call can apply to errors
    in its input, 1 / (smallest input column norm) times the bound on
    ||L^-1|| of every factor (infinite after an SVQB pass)."""
    st = stats if stats is not None else OrthoStats()
    st.ortho_calls += 1
    n = X.shape[0]
    cn = cheap_exit_factor(n)
    norms0 = np.sqrt(np.einsum("ij,ij->j", X, X)) if X.shape[1] else np.ones(0)
    g = (1.0 / float(norms0.min())) if X.shape[1] and norms0.min() > 0 else math.inf
    X = normalize_columns(X, st)
    if growth is not None:
        growth["g"] = g
    if X.shape[1] == 0:
        return X
    eye = np.eye(X.shape[1])
    for p in range(max_passes):
        M = X.T @ X
        M = 0.5 * (M + M.T)
        st.grams += 1
        if max_abs(M - eye) <= tau:
            break
        if p == max_passes - 1:
            st.stalled += 1
            g = math.inf  # a stalled call gives no bound
            break
        shifted_before = st.shifted
        L = shifted_cholesky(M, st, shift_retries)
        if L is None:
            X = svqb(X, M, st)
            g = math.inf
            st.updates += 1
            continue
        # X L^-T  ==  (L^-1 X^T)^T
        X = sla.solve_triangular(L, X.T, lower=True, check_finite=False).T
        st.updates += 1
        b, e = inverse_factor_bound(L)
        g *= b
        if cheap_exit and st.shifted == shifted_before and e < 0.5:
            kappa = (1.0 + e) / (1.0 - e)
            if cn * EPS * kappa * kappa <= tau:
                st.cheap_exits += 1
                break
    if growth is not None:
        growth["g"] = g
    return X


def ortho_against(
    X: np.ndarray,
    Y: np.ndarray,
    tau: float = TAU_ORTHO,
    stats: Optional[OrthoStats] = None,
    max_passes: int = ORTHO_Y_MAX_PASSES,
    shift_retries: int = SHIFT_RETRIES,
    cheap_exit: bool = False,
) -> np.ndarray:
    """Alg. 3 (reading R3): X <- X - Y (Y^T X); X <- ortho(X); repeat until
    ||Y^T X|| <= tau.  Y must have orthonormal columns.

    ``cheap_exit`` (reading R17): the projection leaves a Y-component of
    rounding size, which ortho(X) amplifies by at most its growth g; when
    c(n) eps g <= tau the loop ends without forming Y^T X (and the Alg. 2
    exits inside ortho apply)."""
    st = stats if stats is not None else OrthoStats()
    st.against_calls += 1
    X = normalize_columns(X, st)
    if Y is None or Y.shape[1] == 0:
        return ortho(X, tau, st, shift_retries=shift_retries, cheap_exit=cheap_exit)
    cn = cheap_exit_factor(X.shape[0])
    C = Y.T @ X
    for p in range(max_passes):
        st.against_passes += 1
        X = X - Y @ C
        gr = {}
        X = ortho(X, tau, st, shift_retries=shift_retries, cheap_exit=cheap_exit, growth=gr)
        if cheap_exit and cn * EPS * gr["g"] <= tau:
            st.cheap_exits += 1
            return X
        C = Y.T @ X
        if max_abs(C) <= tau:
            return X
    st.stalled += 1
    return X


# ---------------------------------------------------------------------------
# Sec. 2: Rayleigh-Ritz, residuals, the Jacobi preconditioner


def symmetrize(a: np.ndarray) -> np.ndarray:
    return 0.5 * (a + a.T)


def rayleigh_ritz(V: np.ndarray, AV: np.ndarray):
    """RR on an orthonormal basis V: eigen-decompose a = V^T A V (R10);
    returns all Ritz values (ascending) and the coefficient matrix, its
    columns oriented by R16."""
    a = symmetrize(V.T @ AV)
    theta, U = np.linalg.eigh(a)
    return theta, orient_columns(U)


def orient_columns(U: np.ndarray) -> np.ndarray:
    """R16: flip column j when U[j, j] < 0."""
    s = np.where(np.diag(U) < 0.0, -1.0, 1.0)
    return U * s


def precondition_diag(
    R: np.ndarray, diag: np.ndarray, theta: np.ndarray, signed: bool = False
) -> np.ndarray:
    """W~[:, j] = R[:, j] / g(|diag - theta_j|)  (Sec. 2, reading R7);
    ``signed=True`` drops the absolute value (the paper's literal example)."""
    out = np.empty_like(R)
    for j in range(R.shape[1]):
        delta = PRECOND_GUARD * max(1.0, abs(float(theta[j])))
        den = diag - theta[j]
        if not signed:
            den = np.abs(den)
        small = np.abs(den) < delta
        den = np.where(small, np.where(den < 0.0, -delta, delta), den)
        out[:, j] = R[:, j] / den
    return out


def tridiagonal_part(A) -> np.ndarray:
    """The off-diagonal of tridiag(A): e[i] = a_{i, i+1} (n - 1 values) of a
    dense array or a scipy sparse matrix."""
    if hasattr(A, "tocsr"):
        return np.asarray(A.tocsr().diagonal(1), dtype=np.float64)
    return np.asarray(np.diagonal(A, 1), dtype=np.float64).copy()


def precondition_tridiag(R: np.ndarray, diag: np.ndarray, off: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """Tridiagonal preconditioner (Sec. 4.4, Table 1: the diagonal plus the
    upper and lower diagonal elements, solved by LAPACK's Gaussian
    elimination with partial pivoting), reading R19: column j solves
    T_j w = r with T_j = tridiag(e, t, e), e the off-diagonal of A and
    t_i = max(|d_i - theta_j|, |e_{i-1}| + |e_i| + delta_j), delta_j the
    Jacobi guard of R7.  T_j is symmetric and strictly diagonally dominant
    with a positive diagonal (so positive definite, like R7's absolute
    Jacobi step, to which it reduces where e = 0)."""
    from scipy.linalg import lapack

    n = R.shape[0]
    e = np.asarray(off, dtype=np.float64)
    ae = np.abs(e)
    rowoff = np.zeros(n)
    rowoff[:-1] += ae
    rowoff[1:] += ae
    out = np.empty_like(R)
    for j in range(R.shape[1]):
        delta = PRECOND_GUARD * max(1.0, abs(float(theta[j])))
        t = np.maximum(np.abs(diag - theta[j]), rowoff + delta)
        _, _, _, x, info = lapack.dgtsv(e.copy(), t, e.copy(), R[:, j].copy())
        if info != 0:
            raise np.linalg.LinAlgError(f"dgtsv failed (info {info})")
        out[:, j] = x
    return out


def ritz_residual(AX: np.ndarray, X: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """R = A X - X diag(theta) for Ritz pairs (Sec. 2, reading R1)."""
    return AX - X * theta


def _stall_step(rnorm, m_conv, k, tol, best_act, since_best, window):
    """Reading R22's bookkeeping for one Rayleigh-Ritz step: (stalled,
    best_act, since_best)."""
    if window <= 0:
        return False, best_act, since_best
    ract = float(np.max(rnorm[m_conv:k])) if m_conv < k else 0.0
    if ract < 0.99 * best_act:
        best_act, since_best = ract, 0
    else:
        since_best += 1
    return since_best >= window and ract <= 100.0 * tol, best_act, since_best


def leading_converged(rnorm: np.ndarray, tol: float) -> int:
    c = 0
    for r in rnorm:
        if r <= tol:
            c += 1
        else:
            break
    return c


def true_residuals(op: Operator, X: np.ndarray):
    """Explicit A X, Rayleigh quotients x^T A x / x^T x and residual 2-norms."""
    AX = op(X)
    xx = np.einsum("ij,ij->j", X, X)
    theta = np.einsum("ij,ij->j", X, AX) / xx
    R = AX - X * theta
    return theta, np.linalg.norm(R, axis=0), AX


def lowest_eigenpairs_dense(A: np.ndarray, k: int):
    """The result the method approximates, by its plain definition (Sec. 2:
    the k lowest eigenpairs of a symmetric matrix): LAPACK's dense symmetric
    eigensolver restricted to eigenvalue indices 0..k-1 (syevr).  Returns
    the ascending eigenvalues and orthonormal eigenvectors (n x k)."""
    w, V = sla.eigh(A, subset_by_index=[0, k - 1], driver="evr", check_finite=False)
    return w, V


def normalize_signs(X: np.ndarray) -> np.ndarray:
    """Largest-|.| entry of each column made positive (first index on ties)."""
    X = np.array(X, copy=True)
    for j in range(X.shape[1]):
        i = int(np.argmax(np.abs(X[:, j])))
        if X[i, j] < 0:
            X[:, j] = -X[:, j]
    return X


# ---------------------------------------------------------------------------
# operators (the paper's method is matrix-free; these are its inputs)


def csr_operator(row_ptr, col, val, n: int) -> Operator:
    import scipy.sparse as sp

    A = sp.csr_matrix((np.asarray(val, np.float64), np.asarray(col), np.asarray(row_ptr)), shape=(n, n))

    def apply(X):
        return np.asarray(A @ X)

    return apply


def dense_operator(A: np.ndarray) -> Operator:
    def apply(X):
        return A @ X

    return apply


def kronsum_operator(A: np.ndarray, V: np.ndarray) -> Operator:
    """H = A (x) I + I (x) A + diag(vec V) on row-major vectorised na x na
    blocks: H vec(Z) = vec(A Z + Z A + V o Z)."""
    na = A.shape[0]

    def apply(X):
        out = np.empty_like(X)
        for b in range(X.shape[1]):
            Z = X[:, b].reshape(na, na)
            out[:, b] = (A @ Z + Z @ A + V * Z).reshape(-1)
        return out

    return apply


def kronsum_diagonal(A: np.ndarray, V: np.ndarray) -> np.ndarray:
    d = np.diag(A)
    return (d[:, None] + d[None, :] + V).reshape(-1)


# ---------------------------------------------------------------------------
# Alg. 1


@dataclasses.dataclass
class LobpcgResult:
    evals: np.ndarray
    evecs: np.ndarray
    resnorms: np.ndarray  # true residual 2-norms of the returned pairs
    converged: bool
    iterations: int
    matvec_columns: int
    ortho: OrthoStats
    history_theta: list  # Ritz values (first m) after every RR
    history_resid: list  # RR residual norms (all m) after every RR
    history_active: list  # m_act used for the matvec of every iteration
    true_checks: int
    rms: np.ndarray  # ||r||_2 / sqrt(n), the paper's RMS measure
    maxabs: np.ndarray  # max |r_i|, the paper's second measure
    X_all: np.ndarray = None  # the whole final block
    restarts: int = 0  # failed true-residual checks (reading R9)
    theta_all: np.ndarray = None
    stall_checks: int = 0  # true-residual checks started by reading R22


def lobpcg(
    op: Operator,
    X0: np.ndarray,
    k: int,
    tol: float = 1e-8,
    diag: Optional[np.ndarray] = None,
    precond="diag",
    tau: float = TAU_ORTHO,
    max_iter: int = 1000,
    callback: Optional[Callable[[dict], None]] = None,
    off: Optional[np.ndarray] = None,
    shift_retries: int = SHIFT_RETRIES,
    force_restarts: int = 0,
    cheap_exit: bool = False,
    stall_window: int = 20,
) -> LobpcgResult:
    """Alg. 1: the lowest k eigenpairs of the symmetric operator ``op``.

    X0 is the n x m initial block (m >= k, the block may hold extra vectors,
    Sec. 2).  ``precond`` is "diag" (|Jacobi|, needs ``diag``),
    "diag_signed" (the paper's signed Jacobi), "tridiag" (reading R19,
    needs ``diag`` and the off-diagonal ``off``), "none", or a callable
    f(R_act, theta_act, X_act) returning the preconditioned columns.
    ``shift_retries`` caps the shifted Cholesky retries of every ortho call
    (0 sends a failed factorisation straight to SVQB).  ``force_restarts``
    is a test hook: the first that many true-residual checks count as
    failed, which drives the restart branch of reading R9.  ``cheap_exit``
    turns on reading R17's exits in the orthonormalisations of n-vectors
    (X0, W, the re-orthonormalisation before a true check).
    ``stall_window`` is reading R22's window (0 turns the rule off)."""
    X0 = np.asarray(X0, dtype=np.float64)
    n, m = X0.shape
    if not (1 <= k <= m):
        raise ValueError("need 1 <= k <= block size")
    if isinstance(precond, str) and precond in ("diag", "diag_signed", "tridiag") and diag is None:
        raise ValueError("the Jacobi and tridiagonal preconditioners need diag(A)")
    if precond == "tridiag" and off is None:
        raise ValueError("the tridiagonal preconditioner needs the off-diagonal of A (off=)")
    st = OrthoStats()
    hist_theta, hist_resid, hist_active = [], [], []
    matvecs = 0
    true_checks = 0

    def tprec(R, theta, Xa):
        if callable(precond):
            return np.asarray(precond(R, theta, Xa), dtype=np.float64)
        if precond == "diag":
            return precondition_diag(R, diag, theta)
        if precond == "diag_signed":
            return precondition_diag(R, diag, theta, signed=True)
        if precond == "tridiag":
            return precondition_tridiag(R, diag, off, theta)
        if precond == "none":
            return R.copy()
        raise ValueError(precond)

    # Alg. 1 initial Rayleigh-Ritz (reading R2: orthonormalise X0 first)
    X = ortho(X0, tau, st, shift_retries=shift_retries, cheap_exit=cheap_exit)
    AX = op(X)
    matvecs += m
    theta_all, U = rayleigh_ritz(X, AX)
    X = X @ U
    AX = AX @ U
    theta = theta_all[:m]
    R = ritz_residual(AX, X, theta)  # reading R1
    rnorm = np.linalg.norm(R, axis=0)
    hist_theta.append(theta.copy())
    hist_resid.append(rnorm.copy())
    m_conv = 0
    P = AP = None
    it = 0
    converged = False
    restarts = 0
    just_restarted = False
    best_act, since_best, stall_checks = np.inf, 0, 0  # reading R22
    while True:
        lead = leading_converged(rnorm, tol)
        if just_restarted:
            # after a restart the convergence test waits one iteration, and
            # that iteration keeps at least the k-th column active
            m_conv = min(max(m_conv, lead), k - 1)
        else:
            m_conv = max(m_conv, lead)  # reading R8
        stalled = False
        if stall_window > 0:
            ract = float(np.max(rnorm[m_conv:k])) if m_conv < k else 0.0
            if ract < 0.99 * best_act:
                best_act, since_best = ract, 0
            else:
                since_best += 1
            stalled = since_best >= stall_window and ract <= 100.0 * tol
        if m_conv >= k or stalled:
            if m_conv < k:
                stall_checks += 1
            best_act, since_best = np.inf, 0
            # reading R9: re-orthonormalise X (Alg. 2; the implicit-P
            # recurrence lets X^T X drift from I by rounding), then judge with
            # the true residual of an explicit product
            X = ortho(X, tau, st, shift_retries=shift_retries, cheap_exit=cheap_exit)
            true_checks += 1
            th_t, r_t, AX_t = true_residuals(op, X)
            matvecs += m
            if float(np.max(r_t[:k])) <= tol and restarts >= force_restarts:
                converged = True
                break
            # restart: Rayleigh-Ritz on [X] with the explicit product (as at
            # the start of Alg. 1), P dropped, locking recomputed; the next
            # convergence test waits for one iteration
            restarts += 1
            theta_all, U = rayleigh_ritz(X, AX_t)
            X = X @ U
            AX = AX_t @ U
            theta = theta_all[:m]
            R = ritz_residual(AX, X, theta)
            rnorm = np.linalg.norm(R, axis=0)
            hist_theta.append(theta.copy())
            hist_resid.append(rnorm.copy())
            m_conv = leading_converged(rnorm, tol)
            P = AP = None
            just_restarted = True
            continue
        just_restarted = False
        if it >= max_iter:
            break
        it += 1
        act = np.arange(m_conv, m)
        # Alg. 1: preconditioned residuals, orthogonalised against (X, P)
        Wt = tprec(R[:, act], theta[act], X[:, act])
        Y = X if P is None else np.hstack([X, P])
        W = ortho_against(Wt, Y, tau, st, shift_retries=shift_retries, cheap_exit=cheap_exit)
        AW = op(W)
        matvecs += W.shape[1]
        hist_active.append(W.shape[1])
        if P is None:
            V = np.hstack([X, W])
            AV = np.hstack([AX, AW])
        else:
            V = np.hstack([X, W, P])
            AV = np.hstack([AX, AW, AP])
        # Rayleigh-Ritz in V
        theta_all, U = rayleigh_ritz(V, AV)
        ux = U[:, :m]
        theta = theta_all[:m]
        # eq. neweigv and "Reuse of applications": X and AX through u_x
        Xn = V @ ux
        AXn = AV @ ux
        R = ritz_residual(AXn, Xn, theta)  # reading R1
        rnorm = np.linalg.norm(R, axis=0)
        hist_theta.append(theta.copy())
        hist_resid.append(rnorm.copy())
        if callback is not None:
            callback(dict(it=it, theta=theta, rnorm=rnorm, m_conv=m_conv, X=Xn, AX=AXn))
        m_conv = max(m_conv, leading_converged(rnorm, tol))
        act = np.arange(m_conv, m)
        if m_conv < k:
            # P from u_x: subtract the identity on the X block from the
            # unconverged columns, orthonormalise against u_x in R^p, and
            # rotate V and AV with the orthonormal u_p
            p = V.shape[1]
            up_t = ux[:, act].copy()
            up_t[act, np.arange(act.size)] -= 1.0
            up = ortho_against(up_t, ux, tau, st, shift_retries=shift_retries)
            P = V @ up
            AP = AV @ up
        X, AX = Xn, AXn

    if not converged:
        X = ortho(X, tau, st, shift_retries=shift_retries, cheap_exit=cheap_exit)
        true_checks += 1
        th_t, r_t, AX_t = true_residuals(op, X)
    Rt = AX_t[:, :k] - X[:, :k] * th_t[:k]
    res = LobpcgResult(
        evals=th_t[:k].copy(),
        evecs=normalize_signs(X[:, :k]),
        resnorms=r_t[:k].copy(),
        converged=converged,
        iterations=it,
        matvec_columns=matvecs,
        ortho=st,
        history_theta=hist_theta,
        history_resid=hist_resid,
        history_active=hist_active,
        true_checks=true_checks,
        rms=r_t[:k] / math.sqrt(n),
        maxabs=np.max(np.abs(Rt), axis=0),
        X_all=X,
        theta_all=th_t,
        restarts=restarts,
        stall_checks=stall_checks,
    )
    return res


# ---------------------------------------------------------------------------
# Block Davidson with a history (Sec. 2, the recurrence X^{k+1} = RR(X^1,
# T^1 R^1, ..., T^k R^k); Sec. 4 runs it with 25 vectors per root and
# locking).  Reading R18: the history is truncated by a restart from the
# current Ritz vectors when adding the next block would exceed
# ``max_dim`` columns; every block is made orthonormal to the basis with
# Alg. 3; convergence, locking and the true-residual judgement are those of
# the LOBPCG above (R8, R9).


@dataclasses.dataclass
class DavidsonResult:
    evals: np.ndarray
    evecs: np.ndarray
    resnorms: np.ndarray
    converged: bool
    iterations: int
    matvec_columns: int
    restarts: int  # history truncations
    max_basis: int  # largest basis size reached
    true_checks: int
    check_restarts: int  # failed true-residual checks (R9)
    ortho: OrthoStats
    history_theta: list
    X_all: np.ndarray = None


def davidson(
    op: Operator,
    X0: np.ndarray,
    k: int,
    tol: float = 1e-8,
    diag: Optional[np.ndarray] = None,
    precond="diag",
    max_dim: Optional[int] = None,
    tau: float = TAU_ORTHO,
    max_iter: int = 1000,
    off: Optional[np.ndarray] = None,
    stall_window: int = 20,
) -> DavidsonResult:
    """Block Davidson for the lowest k eigenpairs of ``op`` (Sec. 2): the
    basis holds X^{[1]} and every preconditioned residual block since the
    last restart.  ``max_dim`` defaults to 25 m (Sec. 4's subspace of 25 per
    root).  The preconditioners are those of ``lobpcg``; R9's check also
    runs on reading R22's stall rule (``stall_window``, 0 = off)."""
    X0 = np.asarray(X0, dtype=np.float64)
    n, m = X0.shape
    if not (1 <= k <= m):
        raise ValueError("need 1 <= k <= block size")
    if max_dim is None:
        max_dim = 25 * m
    if max_dim < 2 * m:
        raise ValueError("max_dim must hold the Ritz block and one new block")
    st = OrthoStats()
    hist_theta = []
    V = ortho(X0, tau, st)
    AV = op(V)
    matvecs = m
    true_checks = 0
    restarts = 0
    max_basis = m
    m_conv = 0
    it = 0
    converged = False
    just_restarted = False
    best_act, since_best = np.inf, 0  # reading R22
    check_restarts = 0

    def tprec(R, theta):
        if precond == "diag":
            return precondition_diag(R, diag, theta)
        if precond == "diag_signed":
            return precondition_diag(R, diag, theta, signed=True)
        if precond == "tridiag":
            return precondition_tridiag(R, diag, off, theta)
        if precond == "none":
            return R.copy()
        return np.asarray(precond(R, theta, None), dtype=np.float64)

    while True:
        # Rayleigh-Ritz on the whole basis (R10, R16)
        theta_all, U = rayleigh_ritz(V, AV)
        ux = U[:, :m]
        theta = theta_all[:m]
        X = V @ ux
        AX = AV @ ux
        R = ritz_residual(AX, X, theta)
        rnorm = np.linalg.norm(R, axis=0)
        hist_theta.append(theta.copy())
        lead = leading_converged(rnorm, tol)
        # R9's rule after a restart: one iteration with at most k - 1 locked
        m_conv = min(max(m_conv, lead), k - 1) if just_restarted else max(m_conv, lead)
        just_restarted = False
        stalled, best_act, since_best = _stall_step(rnorm, m_conv, k, tol, best_act, since_best, stall_window)
        if m_conv >= k or stalled:
            best_act, since_best = np.inf, 0
            X = ortho(X, tau, st)
            true_checks += 1
            th_t, r_t, AX_t = true_residuals(op, X)
            matvecs += m
            if float(np.max(r_t[:k])) <= tol:
                converged = True
                break
            # restart from X with the explicit product (as in R9)
            V, AV = X, AX_t
            m_conv = 0
            check_restarts += 1
            just_restarted = True
            continue
        if it >= max_iter:
            break
        it += 1
        act = np.arange(m_conv, m)
        Wt = tprec(R[:, act], theta[act])
        if V.shape[1] + act.size > max_dim:
            # history truncation: restart from the current Ritz vectors
            V, AV = X, AX
            restarts += 1
        W = ortho_against(Wt, V, tau, st)
        AW = op(W)
        matvecs += W.shape[1]
        V = np.hstack([V, W])
        AV = np.hstack([AV, AW])
        max_basis = max(max_basis, V.shape[1])
    if not converged:
        X = ortho(X, tau, st)
        true_checks += 1
        th_t, r_t, AX_t = true_residuals(op, X)
    return DavidsonResult(
        evals=th_t[:k].copy(),
        evecs=normalize_signs(X[:, :k]),
        resnorms=r_t[:k].copy(),
        converged=converged,
        iterations=it,
        matvec_columns=matvecs,
        restarts=restarts,
        max_basis=max_basis,
        true_checks=true_checks,
        check_restarts=check_restarts,
        ortho=st,
        history_theta=hist_theta,
        X_all=X,
    )


# ---------------------------------------------------------------------------
# The generalized problem A x = lambda B x, B symmetric positive definite
# (Sec. 3.3).  Reading R21: the basis V = [X, W, P] is kept B-orthonormal
# with B V carried along.  W~ = T R (R = A X - B X Theta, the Jacobi
# preconditioner (diag A - theta diag B)^-1 with the guard of R7) goes through
# W^ = ortho(W~, (BX, BP)): Alg. 3 with the projection W <- W - [X P]
# ([BX BP]^T W) (the B-orthogonal projector, since [X P] is B-orthonormal)
# and Euclidean Alg. 2 passes, until ||[BX BP]^T W||_max <= tau; then one
# B-Cholesky with the reused application: B W^ once, M = W^T B W^ = L L^T
# (shifted if it fails, as in Alg. 2), W = W^ L^-T, BW = (B W^) L^-T.  X0
# is B-orthonormalised the same way.  The Rayleigh-Ritz matrix V^T A V is a
# standard symmetric eigenproblem on a B-orthonormal V.  Convergence:
# ||A x - theta B x||_2 <= tol for x with x^T B x = 1 (theta = x^T A x),
# judged on explicit products after one more B-orthonormalisation (R9).


def b_orthonormalize(X: np.ndarray, BX: np.ndarray, st: OrthoStats):
    """One Cholesky B-orthonormalisation reusing B X: X L^-T, BX L^-T."""
    M = symmetrize(X.T @ BX)
    st.grams += 1
    L = shifted_cholesky(M, st)
    if L is None:
        raise OrthoFailed("B-overlap not positive definite")
    X = sla.solve_triangular(L, X.T, lower=True, check_finite=False).T
    BX = sla.solve_triangular(L, BX.T, lower=True, check_finite=False).T
    st.updates += 1
    return X, BX


def b_ortho_against(Wt: np.ndarray, Y: np.ndarray, BY: np.ndarray, tau: float, st: OrthoStats,
                    max_passes: int = ORTHO_Y_MAX_PASSES) -> np.ndarray:
    """W^ = ortho(W~, (BX, BP)) of Sec. 3.3 (reading R21)."""
    W = normalize_columns(Wt, st)
    if Y is None or Y.shape[1] == 0:
        return ortho(W, tau, st)
    C = BY.T @ W
    for _ in range(max_passes):
        st.against_passes += 1
        W = W - Y @ C
        W = ortho(W, tau, st)
        C = BY.T @ W
        if max_abs(C) <= tau:
            return W
    st.stalled += 1
    return W


def precondition_diag_gen(R: np.ndarray, dA: np.ndarray, dB: np.ndarray, theta: np.ndarray) -> np.ndarray:
    """W~[:, j] = R[:, j] / g(|dA - theta_j dB|) (reading R21, R7's guard)."""
    out = np.empty_like(R)
    for j in range(R.shape[1]):
        delta = PRECOND_GUARD * max(1.0, abs(float(theta[j])))
        den = np.abs(dA - theta[j] * dB)
        out[:, j] = R[:, j] / np.maximum(den, delta)
    return out


def lobpcg_generalized(
    opA: Operator,
    opB: Operator,
    X0: np.ndarray,
    k: int,
    tol: float = 1e-8,
    dA: Optional[np.ndarray] = None,
    dB: Optional[np.ndarray] = None,
    precond="diag",
    tau: float = TAU_ORTHO,
    max_iter: int = 1000,
    stall_window: int = 20,
) -> LobpcgResult:
    """Alg. 1 for A x = lambda B x (Sec. 3.3, reading R21).  ``precond``:
    "diag" (needs dA, dB) or "none".  The returned vectors satisfy
    X^T B X = I.  R9's check also runs on reading R22's stall rule
    (``stall_window``, 0 = off)."""
    X0 = np.asarray(X0, dtype=np.float64)
    n, m = X0.shape
    if not (1 <= k <= m):
        raise ValueError("need 1 <= k <= block size")
    st = OrthoStats()
    hist_theta, hist_resid, hist_active = [], [], []
    matvecs = bmatvecs = 0
    true_checks = 0

    def tprec(R, theta):
        if precond == "diag":
            return precondition_diag_gen(R, dA, dB, theta)
        if precond == "none":
            return R.copy()
        raise ValueError(precond)

    X = ortho(X0, tau, st)
    BX = opB(X)
    bmatvecs += m
    X, BX = b_orthonormalize(X, BX, st)
    AX = opA(X)
    matvecs += m
    theta_all, U = rayleigh_ritz(X, AX)
    X, AX, BX = X @ U, AX @ U, BX @ U
    theta = theta_all[:m]
    R = AX - BX * theta
    rnorm = np.linalg.norm(R, axis=0)
    hist_theta.append(theta.copy())
    hist_resid.append(rnorm.copy())
    m_conv = 0
    P = AP = BP = None
    it = 0
    converged = False
    restarts = 0
    just_restarted = False
    best_act, since_best = np.inf, 0  # reading R22
    while True:
        lead = leading_converged(rnorm, tol)
        m_conv = min(max(m_conv, lead), k - 1) if just_restarted else max(m_conv, lead)
        just_restarted = False
        stalled, best_act, since_best = _stall_step(rnorm, m_conv, k, tol, best_act, since_best, stall_window)
        if m_conv >= k or stalled:
            best_act, since_best = np.inf, 0
            # R9 for the generalized problem: B-orthonormalise X once more
            # (explicit B X), then judge with explicit products
            BXt = opB(X)
            bmatvecs += m
            X, BXt = b_orthonormalize(X, BXt, st)
            AXt = opA(X)
            matvecs += m
            true_checks += 1
            th_t = np.einsum("ij,ij->j", X, AXt) / np.einsum("ij,ij->j", X, BXt)
            r_t = np.linalg.norm(AXt - BXt * th_t, axis=0)
            if float(np.max(r_t[:k])) <= tol:
                converged = True
                break
            restarts += 1
            theta_all, U = rayleigh_ritz(X, AXt)
            X, AX, BX = X @ U, AXt @ U, BXt @ U
            theta = theta_all[:m]
            R = AX - BX * theta
            rnorm = np.linalg.norm(R, axis=0)
            m_conv = 0
            P = AP = BP = None
            just_restarted = True
            continue
        if it >= max_iter:
            break
        it += 1
        act = np.arange(m_conv, m)
        Wt = tprec(R[:, act], theta[act])
        Y = X if P is None else np.hstack([X, P])
        BY = BX if P is None else np.hstack([BX, BP])
        W = b_ortho_against(Wt, Y, BY, tau, st)
        BW = opB(W)
        bmatvecs += W.shape[1]
        W, BW = b_orthonormalize(W, BW, st)
        AW = opA(W)
        matvecs += W.shape[1]
        hist_active.append(W.shape[1])
        if P is None:
            V, AV, BV = np.hstack([X, W]), np.hstack([AX, AW]), np.hstack([BX, BW])
        else:
            V, AV, BV = np.hstack([X, W, P]), np.hstack([AX, AW, AP]), np.hstack([BX, BW, BP])
        theta_all, U = rayleigh_ritz(V, AV)
        ux = U[:, :m]
        theta = theta_all[:m]
        Xn, AXn, BXn = V @ ux, AV @ ux, BV @ ux
        R = AXn - BXn * theta
        rnorm = np.linalg.norm(R, axis=0)
        hist_theta.append(theta.copy())
        hist_resid.append(rnorm.copy())
        m_conv = max(m_conv, leading_converged(rnorm, tol))
        act = np.arange(m_conv, m)
        if m_conv < k:
            up_t = ux[:, act].copy()
            up_t[act, np.arange(act.size)] -= 1.0
            up = ortho_against(up_t, ux, tau, st)
            P, AP, BP = V @ up, AV @ up, BV @ up
        X, AX, BX = Xn, AXn, BXn
    if not converged:
        BXt = opB(X)
        X, BXt = b_orthonormalize(X, BXt, st)
        AXt = opA(X)
        true_checks += 1
        th_t = np.einsum("ij,ij->j", X, AXt) / np.einsum("ij,ij->j", X, BXt)
        r_t = np.linalg.norm(AXt - BXt * th_t, axis=0)
    return LobpcgResult(
        evals=th_t[:k].copy(),
        evecs=normalize_signs(X[:, :k]),
        resnorms=r_t[:k].copy(),
        converged=converged,
        iterations=it,
        matvec_columns=matvecs,
        ortho=st,
        history_theta=hist_theta,
        history_resid=hist_resid,
        history_active=hist_active,
        true_checks=true_checks,
        rms=r_t[:k] / math.sqrt(n),
        maxabs=np.max(np.abs(AXt[:, :k] - BXt[:, :k] * th_t[:k]), axis=0),
        X_all=X,
        theta_all=th_t,
        restarts=restarts,
    )
