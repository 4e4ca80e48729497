/*
 * lobpcg.h -- C ABI of an MI355X (gfx950) block LOBPCG eigensolver.
 *
 * Method: Nottoli, Gianni, Levitt, Lipparini, "A robust, open-source
 * implementation of the locally optimal block preconditioned conjugate
 * gradient for large eigenvalue problems in quantum chemistry",
 * arXiv:2305.06668.  The problem (Sec. 2): for a real symmetric A of order n,
 * find the m << n lowest eigenpairs.  Alg. 1 gives the iteration; Alg. 2 and
 * Alg. 3 the Cholesky-based orthonormalisations it relies on (Sec. 3.2).
 *
 * Conventions shared by every entry point
 *  - Every function returns an int status (LOBPCG_OK = 0, >0 warnings, <0
 *    errors); nothing is thrown across this boundary.  A per-handle message
 *    for the last error is available from lobpcg_last_error().
 *  - Blocks of vectors are ROW-MAJOR: an n x c block with leading dimension
 *    ld >= c stores entry (i, j) at ptr[i * ld + j].  Small matrices are
 *    row-major and dense (ld = number of columns).
 *  - "device" pointers are HIP device memory on the handle's device, owned by
 *    the caller, and must stay valid until the handle is destroyed or the
 *    setter is called again.  "host" pointers are ordinary host memory.
 *  - All device work runs on the handle's stream (lobpcg_set_stream; the
 *    null stream by default).  Entry points that return host data synchronise
 *    that stream before returning; the step entry points (lobpcg_apply_operator,
 *    lobpcg_gram, ...) are asynchronous unless stated otherwise.
 *  - Device scratch comes from a caller-provided workspace
 *    (lobpcg_workspace_size / lobpcg_set_workspace); the library itself only
 *    allocates a few KB of pinned host memory for read-backs and, once learned
 *    weights are set, a 68 KB device copy of them.
 *  - A handle is not thread-safe; distinct handles are independent.
 */
#ifndef LOBPCG_MI355X_H
#define LOBPCG_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lobpcg_ctx* lobpcg_t;

/* ---- status codes ------------------------------------------------------ */
#define LOBPCG_OK 0
#define LOBPCG_NOT_CONVERGED 1     /* max_iter reached; results are readable */
#define LOBPCG_ERR_INVALID_ARG -1
#define LOBPCG_ERR_BAD_STATE -2    /* call order violated (e.g. solve before set_operator) */
#define LOBPCG_ERR_DEVICE -3       /* a HIP runtime call failed */
#define LOBPCG_ERR_WORKSPACE -4    /* no workspace, or smaller than lobpcg_workspace_size */
#define LOBPCG_ERR_ORTHO_FAILED -5 /* shifted Cholesky and SVQB both failed */
#define LOBPCG_ERR_NONFINITE -6    /* NaN or Inf met in residuals or overlaps */
#define LOBPCG_ERR_UNSUPPORTED -7  /* size or mode outside what the library implements */

/* ---- preconditioners (Sec. 2, T in w = T r) ---------------------------- */
#define LOBPCG_PRECOND_NONE 0        /* T = I */
#define LOBPCG_PRECOND_DIAG 1        /* T_j = |diag(A) - theta_j I|^-1 (default) */
#define LOBPCG_PRECOND_DIAG_SIGNED 2 /* T_j = (diag(A) - theta_j I)^-1, Sec. 2's example */
#define LOBPCG_PRECOND_LEARNED 3     /* learned regularised Jacobi step (see
                                        lobpcg_set_learned_weights); Jacobi fallback */
#define LOBPCG_PRECOND_TRIDIAG 4     /* tridiagonal (Sec. 4.4, Table 1): T_j w = r with
                                        T_j = tridiag(e, t, e), e_i = a_{i,i+1},
                                        t_i = max(|d_i - theta_j|, |e_{i-1}| + |e_i| +
                                        delta_j): the positive definite counterpart of
                                        LOBPCG_PRECOND_DIAG (equal to it where e = 0),
                                        solved exactly on the device */

/* Parameters of the learned preconditioner's MLP (3 -> 128 -> 128 -> 1). */
#define LOBPCG_LEARNED_NPARAMS 17153

/* ---- precision modes --------------------------------------------------- */
#define LOBPCG_PREC_FP64 0 /* every step in fp64 */
#define LOBPCG_PREC_FP32 1 /* operator, Grams and blocks in fp32 until the
                              residual nears the fp32 floor, then fp64 */

/* ---- methods ------------------------------------------------------------ */
#define LOBPCG_METHOD_LOBPCG 0   /* Alg. 1 (default) */
#define LOBPCG_METHOD_DAVIDSON 1 /* block Davidson with a history (Sec. 2: X^{k+1} =
                                    RR(X^1, T^1 R^1, ..., T^k R^k); Sec. 4 compares it
                                    with LOBPCG): each active preconditioned residual
                                    block is made orthonormal to the basis by Alg. 3 and
                                    appended; Rayleigh-Ritz runs on the whole basis;
                                    locking and the true-residual test as for LOBPCG.
                                    fp64 with the Jacobi preconditioners only. */

/* ---- option keys for lobpcg_set_option --------------------------------- */
#define LOBPCG_OPT_TAU_ORTHO 0        /* ortho threshold, default 1e-14 (Sec. 4) */
#define LOBPCG_OPT_MAX_ITER 1         /* default 1000 */
#define LOBPCG_OPT_PRECISION 2        /* LOBPCG_PREC_*, default FP64 */
#define LOBPCG_OPT_ORTHO_MAX_PASSES 3 /* Alg. 2 overlap evaluations, default 6 */
#define LOBPCG_OPT_ORTHO_Y_MAX_PASSES 4 /* Alg. 3 passes, default 4 */
#define LOBPCG_OPT_TRACE 5            /* 1: time phases with HIP events */
#define LOBPCG_OPT_RR_JACOBI 7         /* Rayleigh-Ritz eigensolver: 0 (default) =
                                         Householder tridiagonalisation, Sturm
                                         multisection and inverse iteration;
                                         1 = parallel cyclic Jacobi */
#define LOBPCG_OPT_LEARNED_BF16 6     /* learned preconditioner inference: 1 (default)
                                         = hidden layer on bf16 MFMA with fp32
                                         accumulation, 0 = fp32 throughout */
#define LOBPCG_OPT_SHIFT_RETRIES 8    /* shifted Cholesky attempts after a failed plain
                                         factorisation (Sec. 3.2), default 20, 0..20;
                                         when they all fail the pass orthonormalises
                                         by SVQB (Stathopoulos-Wu).  0 sends every
                                         failed factorisation straight to SVQB */
#define LOBPCG_OPT_CHEAP_EXIT 10      /* 1: cheap exits of the ortho loops (Sec. 3.2
                                         proposes them after Alg. 2 and Alg. 3): an
                                         unshifted factor L with e = ||I - L||_F < 1/2
                                         and c(n) u ((1+e)/(1-e))^2 <= tau ends Alg. 2
                                         without the overlap of the new block, and a
                                         growth g of the Alg. 2 call (normalisation
                                         scale times a bound on ||L^-1|| per factor)
                                         with c(n) u g <= tau ends Alg. 3 without
                                         Y^T X; c(n) = max(4, 0.02 sqrt(n)), u the
                                         blocks' unit roundoff.  Default 0 */
#define LOBPCG_OPT_METHOD 11          /* LOBPCG_METHOD_*, default LOBPCG */
#define LOBPCG_OPT_DAVIDSON_MAX_DIM 12 /* block Davidson: largest basis (columns) before
                                          its history is truncated by a restart from the
                                          current Ritz vectors; 0 (default) = min(25 m,
                                          96) (Sec. 4 keeps 25 vectors per root; 96 is the
                                          library's Rayleigh-Ritz limit); 2 m .. 96 */
#define LOBPCG_OPT_LEARNED_BUDGET 13  /* learned preconditioner: the iterations of a
                                         solve that use the learned step; from
                                         the next one on every column takes the
                                         (absolute) Jacobi step, its fallback.
                                         Default 200, 0 = no limit.  Bounds the
                                         cost of a net that slows a solve down
                                         without ever failing the per-column
                                         residual test */
#define LOBPCG_OPT_STALL_WINDOW 14    /* LOBPCG's fp64 phase, block Davidson and the
                                         generalized driver: when the largest residual of
                                         the sought active columns is within 100
                                         tol and has not fallen by 1 % over this
                                         many iterations, the
                                         explicit true-residual check runs
                                         although the recurrence has not
                                         converged: it ends the solve if A X
                                         meets the tolerance, else restarts from
                                         A X.  The recurrence's residuals can
                                         settle on a floor left by rounding in
                                         its implicit products (Sec. 3.1, "Reuse
                                         of applications") just above the
                                         tolerance, which no other test would
                                         leave.  Default 20, 0 = off */
#define LOBPCG_OPT_SPMM_SLAB 15      /* CSR products: 0 (default) the gather
                                         kernels; 1 the banded path (W staged in
                                         LDS in slabs over each 2048-row block's
                                         column window) where the columns are
                                         sorted within rows, else the gather
                                         kernels.  Measured slower on the
                                         benchmark's banded matrix (1.4 ms
                                         against 0.38 ms at 16 fp64 columns) */
#define LOBPCG_OPT_FORCE_RESTARTS 9   /* test hook, default 0: the first N explicit
                                         true-residual checks of a solve count as
                                         failed, which drives the restart that a
                                         failed check triggers (Rayleigh-Ritz on
                                         [X] with the explicit product A X, P
                                         dropped) */

/* ---- statistics --------------------------------------------------------- */
typedef struct lobpcg_stats {
  int32_t iterations;          /* Alg. 1 loop iterations */
  int32_t converged;           /* 1 when all k pairs met tol on the true residual */
  int64_t matvec_columns;      /* columns the operator was applied to */
  int32_t ortho_grams;         /* overlap matrices formed in ortho calls */
  int32_t ortho_factorizations;/* Cholesky attempts (failed ones included) */
  int32_t ortho_failed;        /* failed Cholesky attempts */
  int32_t ortho_shifted;       /* factorizations that needed the diagonal shift */
  int32_t ortho_stalled;       /* ortho loops stopped at their pass cap */
  int32_t ortho_svqb;          /* SVQB fallbacks */
  int32_t against_passes;      /* Alg. 3 project+ortho passes */
  int32_t true_checks;         /* explicit A X residual checks */
  int32_t relocks;             /* iterations where locking changed the active set */
  int32_t precision_switch_iter; /* iteration of the fp32 -> fp64 switch, -1 if none */
  int32_t m_conv;              /* locked (converged) leading columns */
  double ms_total;             /* wall time of lobpcg_solve */
  double ms_operator;          /* the phase times below need LOBPCG_OPT_TRACE */
  double ms_rr;                /* RR Gram + small eigensolve + rotation */
  double ms_ortho;             /* ortho(W~; [X P]) */
  double ms_sync;              /* host waits for per-iteration read-backs */
  int32_t learned_fallbacks;   /* learned steps that did not lower the residual
                                  (the column then takes 3 Jacobi steps) */
  int32_t learned_nonfinite;   /* learned applications with a non-finite net output */
  int32_t rr_eig_fallbacks;    /* Rayleigh-Ritz eigensolves that fell back from the
                                  tridiagonal path to Jacobi */
  int32_t restarts;            /* failed true-residual checks (each restarts the
                                  iteration from X with the explicit product) */
  int32_t ortho_cheap_exits;   /* overlaps the cheap exits skipped */
  int32_t history_restarts;    /* block Davidson: history truncations */
  int32_t max_basis;           /* block Davidson: largest basis reached (columns) */
  int64_t b_matvec_columns;    /* generalized problem: columns B was applied to */
  int32_t learned_budget_iter; /* first iteration that took the Jacobi step because
                                  LOBPCG_OPT_LEARNED_BUDGET was spent, -1 if none */
  int32_t stall_checks;        /* true-residual checks started by
                                  LOBPCG_OPT_STALL_WINDOW */
} lobpcg_stats;

/* ---- ortho report for the step entry points ---------------------------- */
typedef struct lobpcg_ortho_info {
  int32_t grams, factorizations, failed, shifted, updates, passes, stalled, svqb;
  int32_t cheap_exits;  /* overlaps skipped by LOBPCG_OPT_CHEAP_EXIT */
} lobpcg_ortho_info;

/* ======================================================================== */
/* Handle life cycle                                                         */
/* ======================================================================== */

/* Create a solver for a symmetric operator of order n (Sec. 2) on HIP device
 * `device`.  n >= 1.  *out receives the handle (NULL on error). */
int lobpcg_create(int64_t n, int device, lobpcg_t* out);
/* Release the handle and its pinned host buffers (never the caller's memory). */
int lobpcg_destroy(lobpcg_t h);
/* Run all device work of this handle on `hip_stream` (a hipStream_t). */
int lobpcg_set_stream(lobpcg_t h, void* hip_stream);
/* Set an option (LOBPCG_OPT_*); integer options take integral values. */
int lobpcg_set_option(lobpcg_t h, int key, double value);

/* Bytes of device workspace a solve for k pairs with a block of `block`
 * columns needs in precision mode `precision` (LOBPCG_PREC_*) with the
 * operator currently set (the dense and Kronecker operators and the fp32
 * mode need more, so query again after changing them; Sec. 2: the block m
 * may exceed the number k of pairs sought, and the solve stops when the
 * first k have converged).  1 <= k <= block <= 32 and 3 * block <= n.  Also
 * selects `block` for a later solve when no initial guess is set. */
int lobpcg_workspace_size(lobpcg_t h, int k, int block, int precision, size_t* bytes);
/* Hand over a device buffer of `bytes` bytes (256-byte aligned) used for all
 * blocks and partial results.  Borrowed, not freed by the library. */
int lobpcg_set_workspace(lobpcg_t h, void* dev_ptr, size_t bytes);

/* ======================================================================== */
/* Operator and preconditioner (the method is matrix-free, Sec. 3.1)          */
/* ======================================================================== */

/* Sparse symmetric A in CSR: row_ptr (n+1, int32), col (nnz, int32, any
 * order within a row), val (nnz, fp64); all device, borrowed.  Both
 * triangles must be stored. */
int lobpcg_set_operator_csr(lobpcg_t h, const int32_t* row_ptr, const int32_t* col,
                            const double* val, int64_t nnz);
/* Dense symmetric A, row-major with leading dimension lda >= n; device,
 * borrowed. */
int lobpcg_set_operator_dense(lobpcg_t h, const double* A, int64_t lda);
/* Matrix-free H = A (x) I + I (x) A + diag(vec V) of order n = na^2, with A
 * (na x na, symmetric, row-major) and V (na x na, row-major); vector entry
 * i * na + j pairs with V[i][j].  Device, borrowed. */
int lobpcg_set_operator_kronsum(lobpcg_t h, int64_t na, const double* A, const double* V);

/* The second operator B of the generalized problem A x = lambda B x (Sec.
 * 3.3), B symmetric positive definite: CSR (device arrays, both triangles,
 * borrowed) or dense (device, row-major, ldb >= n, borrowed).  A NULL
 * row_ptr / B returns to the standard problem.  With B set, lobpcg_solve
 * keeps the basis B-orthonormal (Sec. 3.3: W^ = ortho(W~, (BX, BP)) by the
 * B-orthogonal projection and Euclidean Alg. 2 passes, one application B W^,
 * one B-Cholesky reusing it), the residuals are A x - theta B x, the Jacobi
 * step uses |diag A - theta diag B|, returned vectors satisfy X^T B X = I
 * and resnorms are ||A x - theta B x||.  fp64 LOBPCG with the NONE / DIAG /
 * DIAG_SIGNED preconditioners only (else LOBPCG_ERR_UNSUPPORTED). */
int lobpcg_set_operator_b_csr(lobpcg_t h, const int32_t* row_ptr, const int32_t* col,
                              const double* val, int64_t nnz);
int lobpcg_set_operator_b_dense(lobpcg_t h, const double* B, int64_t ldb);

/* Preconditioner T (Sec. 2).  kind: LOBPCG_PRECOND_*.  diag: device array of
 * n values of diag(A), or NULL to take it from the operator (CSR: the stored
 * diagonal entries; dense: A_ii; kronsum: A_ii + A_jj + V_ij).  A diagonal
 * entry x with |x - theta_j| < 1e-8 max(1, |theta_j|) is clamped to that
 * bound (sign kept, 0 taken as +). */
int lobpcg_set_preconditioner(lobpcg_t h, int kind, const double* diag);

/* Weights of the learned preconditioner (an extension beside Sec. 2's
 * Jacobi T; Sec. 4.4 studies other preconditioners).  w: host, the
 * LOBPCG_LEARNED_NPARAMS fp32 parameters in the order W1 (128 x 3 row-major),
 * b1 (128), W2 (128 x 128), b2 (128), W3 (128), b3 (1); copied to a
 * library-owned device buffer.  With kind LOBPCG_PRECOND_LEARNED the active
 * column j of W~ becomes
 *   w_i = r_i / sqrt((d_i - theta_j)^2 + c_i^2),  c_i = s softplus(y_i),
 * y_i = MLP(log(|d_i - theta_j| / s + 1e-6), theta_j / s,
 *           log(rho_i / s + 1e-6)),
 * d = diag(A), rho_i = sum_{l != i} |a_il|, s = mean |d|; the denominator is
 * floored at the Jacobi guard.  A column whose residual did not decrease
 * over the step that used its learned column takes the Jacobi step for the
 * next 3 iterations; an entry with a non-finite net output takes the Jacobi
 * step.  INVALID_ARG unless count == LOBPCG_LEARNED_NPARAMS. */
int lobpcg_set_learned_weights(lobpcg_t h, const float* w, int64_t count);

/* Initial block X0 (Alg. 1 input): device, row-major n x block with leading
 * dimension ld >= block; borrowed, read when lobpcg_solve starts.  Without an
 * initial guess the solver fills X0 with SplitMix64 uniforms in [-0.5, 0.5).
 * 1 <= block <= 32, 3 * block <= n. */
int lobpcg_set_initial_guess(lobpcg_t h, const double* X0, int64_t ld, int block);
/* The same from host memory in column-major order (the layout of the
 * problem statement: column j is the j-th start vector): entry (i, j) at
 * X0[j * ld + i], ld >= n.  Copied into a library-owned host buffer at the
 * call (n * block doubles) and uploaded when lobpcg_solve starts; replaces a
 * device initial guess and vice versa. */
int lobpcg_set_initial_guess_host(lobpcg_t h, const double* X0, int64_t ld, int block);

/* ======================================================================== */
/* Solve and results                                                          */
/* ======================================================================== */

/* Alg. 1: iterate until the k lowest pairs have true residual 2-norms
 * ||A x - theta x|| <= tol (||x|| = 1), or max_iter.  1 <= k <= block.
 * Blocking: returns after the stream is synchronised.  Returns LOBPCG_OK,
 * LOBPCG_NOT_CONVERGED, or an error. */
int lobpcg_solve(lobpcg_t h, int k, double tol);

/* Results of the last solve.  evals, resnorms: host arrays of k doubles (may
 * be NULL); evecs: device, row-major n x k with leading dimension ldv >= k
 * (may be NULL).  Pairs are in ascending order; each eigenvector's entry of
 * largest magnitude is positive (lowest index on ties).  resnorms are true
 * residual 2-norms from an explicit product A X.  Blocking. */
int lobpcg_get_eigenpairs(lobpcg_t h, int k, double* evals, double* evecs, int64_t ldv,
                          double* resnorms);
/* The same with evecs in host memory, column-major: entry (i, j) of the
 * n x k result at evecs[j * ldv + i], ldv >= n (may be NULL).  Uses the
 * workspace as staging.  Blocking. */
int lobpcg_get_eigenpairs_host(lobpcg_t h, int k, double* evals, double* evecs, int64_t ldv,
                               double* resnorms);
/* Counters and phase times of the last solve (host struct). */
int lobpcg_get_stats(lobpcg_t h, lobpcg_stats* out);

const char* lobpcg_status_string(int status);
const char* lobpcg_last_error(lobpcg_t h);

/* ======================================================================== */
/* Step entry points: one step of the hot path each, on caller buffers.       */
/* They need the operator (for apply/rotate) and a workspace set.             */
/* ======================================================================== */

/* Operator application Y = A W (Alg. 1, the products A X^[0] and A W^[k]).
 * W: device n x ncols (ldw), Y: device n x ncols (ldy), 1 <= ncols <= 64.
 * Asynchronous. */
int lobpcg_apply_operator(lobpcg_t h, const double* W, int64_t ldw, int ncols, double* Y,
                          int64_t ldy);
/* The same product in fp32 (the operator applications of the fp32 phase of
 * the mixed-precision solve): the operator's values rounded to fp32 (a copy
 * the library keeps in the workspace, made on first use), fp32 W and Y,
 * fp32 accumulation.  Needs LOBPCG_OPT_PRECISION = LOBPCG_PREC_FP32 (the
 * workspace layout that holds the fp32 copy) and a workspace; returns
 * LOBPCG_ERR_BAD_STATE otherwise.  Asynchronous. */
int lobpcg_apply_operator_f32(lobpcg_t h, const float* W, int64_t ldw, int ncols, float* Y,
                              int64_t ldy);

/* Overlap / projection product C = A^T B over the handle's n rows (the
 * a = V^T AV of Alg. 1, the X^T X of Alg. 2, the Y^T X of Alg. 3).
 * A: device n x p (lda), B: device n x q (ldb), C: device p x q row-major.
 * 1 <= p, q <= 128.  The n-reduction is fixed-order (deterministic).
 * Asynchronous. */
int lobpcg_gram(lobpcg_t h, const double* A, int64_t lda, int p, const double* B, int64_t ldb,
                int q, double* C);

/* lobpcg_gram for callers that cannot allocate memory (code under HIP
 * stream capture, tight serving loops, harnesses that forbid allocation): the
 * same product, the same kernels and bitwise the same result, but no
 * workspace is needed -- the partial sums of the n-reduction live in a
 * library-owned static device array (16 MiB per GPU the library runs on, held
 * until the process ends), and the call allocates nothing.  Limit: 1 <= p, q
 * <= 64 (INVALID_ARG beyond).  Every call on one GPU shares that array, so
 * calls that overlap on a GPU (other streams, other threads) race; calls in
 * one stream's order are safe.  Asynchronous. */
int lobpcg_gram_noalloc(lobpcg_t h, const double* A, int64_t lda, int p, const double* B,
                        int64_t ldb, int q, double* C);

/* Alg. 2, ortho(X): orthonormalise the ncols columns of X in place (device,
 * n x ncols, ldx), 1 <= ncols <= 32.  Columns are scaled to unit norm first;
 * a failed Cholesky of the overlap is retried with the diagonal shift
 * alpha * eps * ||X||_F, alpha = 100, 1000, ... (Sec. 3.2).  info (host,
 * may be NULL) receives the counters.  Blocking. */
int lobpcg_ortho(lobpcg_t h, double* X, int64_t ldx, int ncols, lobpcg_ortho_info* info);

/* Alg. 3, ortho(X, Y): make X (device n x ncols, ldx, in place) orthonormal
 * and orthogonal to the orthonormal Y (device n x ycols, ldy).  Y must sit
 * immediately left of X in the same row-major buffer: X == Y + ycols and
 * ldx == ldy (the layout the solver keeps [X P | W] in).  ncols <= 32,
 * ycols + ncols <= 96.  Blocking. */
int lobpcg_ortho_against(lobpcg_t h, double* X, int64_t ldx, int ncols, const double* Y,
                         int64_t ldy, int ycols, lobpcg_ortho_info* info);

/* Small symmetric eigensolve of the RR matrix (Alg. 1, "solve a u = lambda
 * u"; Sec. 3.1 uses LAPACK's dsyev there): a (device p x p, symmetrised as
 * (a + a^T)/2 first) -> evals (device, p, ascending) and evecs (device p x p
 * row-major, column j pairs with evals[j]).  1 <= p <= 96.  fp64, one
 * workgroup, the Rayleigh-Ritz kernel's eigensolver: Householder
 * tridiagonalisation, Sturm multisection and inverse iteration, with cyclic
 * parallel-order Jacobi sweeps as the fallback.  Asynchronous. */
int lobpcg_small_eigh(lobpcg_t h, const double* a, int p, double* evals, double* evecs);

/* Shifted Cholesky of a small overlap M (device p x p, p <= 64): L (device,
 * lower triangular p x p) with L L^T = M + sigma I, sigma = 0 when the plain
 * factorisation succeeds, else alpha * eps * sqrt(trace M) with alpha =
 * 100, 1000, ... (Sec. 3.2, Alg. 2).  *shifts (host, may be NULL) receives
 * the number of failed attempts.  Blocking.  LOBPCG_ERR_ORTHO_FAILED when
 * all retries fail. */
int lobpcg_small_cholesky(lobpcg_t h, const double* M, int p, double* L, int* shifts);

/* Block rotation with residual and preconditioner (the steps of Alg. 1 forming
 * X^[k+1], AX^[k+1], P^[k+1], AP^[k+1], R and W~ = T R; eq. neweigv and the
 * "Reuse of applications" paragraph, Sec. 3.1):
 *   [X' P'] = V U,  [AX' AP'] = AV U    with U = [u_x u_p] (device p x q,
 *                                       q = m + np), V, AV device n x p (ldv)
 *   R = AX' - X' diag(theta)            theta: device m
 *   W~[:, j - a0] = T_j R[:, j] for j in [a0, m)   (T from the handle)
 * Outputs go to Vout / AVout (device n x ldo): columns [0, q) hold [X' P'] /
 * [AX' AP'], columns [q, q + m - a0) of Vout hold W~.  resnorm2 (device m)
 * receives ||R[:, j]||^2.  Vout must not alias V.  p <= 96, q <= 64.
 * Asynchronous. */
int lobpcg_rotate(lobpcg_t h, const double* V, const double* AV, int64_t ldv, int p,
                  const double* U, int m, int q, const double* theta, int a0, double* Vout,
                  double* AVout, int64_t ldo, double* resnorm2);

/* The learned preconditioner's transform (see lobpcg_set_learned_weights) on
 * caller buffers, in the precision LOBPCG_OPT_LEARNED_BF16 selects: R (device n x nact, ldr) is replaced in place by the
 * learned columns for the Ritz values theta (device, nact); mask (device,
 * nact ints, may be NULL): nonzero selects the Jacobi step for that column.
 * Needs weights and the operator.  1 <= nact <= 64.  Asynchronous. */
int lobpcg_learned_apply(lobpcg_t h, double* R, int64_t ldr, int nact, const double* theta,
                         const int* mask);

/* The tridiagonal preconditioner (LOBPCG_PRECOND_TRIDIAG) on caller
 * buffers: column j of R (device n x nact, ldr, in place) becomes the
 * solution w of T_j w = r_j for theta_j (device, nact).  diag(A) and the
 * off-diagonal come from the operator (or the diag given to
 * lobpcg_set_preconditioner).  Needs the operator and a workspace sized with
 * the tridiagonal preconditioner selected.  1 <= nact <= block.
 * Asynchronous. */
int lobpcg_tridiag_apply(lobpcg_t h, double* R, int64_t ldr, int nact, const double* theta);

/* ======================================================================== */
/* Training the learned preconditioner                                        */
/* ======================================================================== */
/* A learner holds fp32 weights with Adam state and a set of snapshots.  A
 * snapshot is an orthonormal Ritz block X of some operator (for example the
 * eigenvectors of a solve stopped early with LOBPCG_OPT_MAX_ITER); the
 * learner forms R = A X - X diag(theta) and, for each column, the near-exact
 * Jacobi-Davidson correction t_j solving
 *   (I - x_j x_j^T)(A - theta_j I)(I - x_j x_j^T) t = -r_j,  t orthogonal to x_j
 * by MINRES.  The training loss of a column is log(Delta(t_j) / Delta(w_j)),
 * Delta(v) being the decrease of theta_j achieved by the Rayleigh-Ritz step on
 * span{x_j, (I - X X^T) v}, and w_j the learned column, plus (weight mu, 0 by
 * default) the supervised term mu (1 - cos^2 of the angle between
 * (I - X X^T) w_j and (I - X X^T) t_j), which ties the learned step to the
 * near-exact one; the loss of a step is its mean over the step's columns.
 * Device buffers are library-owned. */
typedef struct lobpcg_learner* lobpcg_learner_t;

/* Create a learner on `device` with weights drawn from `seed` (layer l
 * weights N(0, 1/fan_in) from SplitMix64 + Box-Muller, output layer scaled by
 * 0.1, biases 0 except b3 = -3). */
int lobpcg_learner_create(int device, uint64_t seed, lobpcg_learner_t* out);
int lobpcg_learner_destroy(lobpcg_learner_t L);
/* The learner has no stream of its own: snapshot collection, the objective
 * and training run on the stream of the solver handle of each snapshot
 * (lobpcg_set_stream), and each call returns once that work is done. */
/* Weight mu >= 0 (finite) of the supervised term of the loss; 0 turns it
 * off.  Applies to later lobpcg_learner_objective / lobpcg_learner_train
 * calls; LOBPCG_ERR_INVALID_ARG for a negative or non-finite mu. */
int lobpcg_learner_set_supervision(lobpcg_learner_t L, double mu);
/* Host fp32 weights in, out (LOBPCG_LEARNED_NPARAMS); set resets Adam and
 * returns once the device copy is complete. */
int lobpcg_learner_set_weights(lobpcg_learner_t L, const float* w, int64_t count);
int lobpcg_learner_get_weights(lobpcg_learner_t L, float* w, int64_t count);
/* Add a snapshot: X device n x m (ldx), orthonormal columns, of the operator
 * set in solver handle h (which must stay alive and unchanged while the
 * learner uses it and must have a workspace for block >= m); m <= 32.
 * MINRES runs at most minres_maxiter iterations or to relative residual
 * minres_rtol.  *index receives the snapshot number.  Blocking. */
int lobpcg_learner_add_snapshot(lobpcg_learner_t L, lobpcg_t h, const double* X, int64_t ldx,
                                int m, int minres_maxiter, double minres_rtol, int* index);
/* Per-column data of snapshot `snap` (host arrays of m doubles, any may be
 * NULL): Ritz values, residual norms, Delta(t_j) of the MINRES corrections and
 * MINRES relative residual estimates. */
int lobpcg_learner_snapshot_info(lobpcg_learner_t L, int snap, double* theta, double* resnorm,
                                 double* ref_decrease, double* minres_relres);
/* Loss of the current weights on columns cols[0..ncols) (host) of snapshot
 * `snap`, and optionally its gradient (host, LOBPCG_LEARNED_NPARAMS doubles)
 * and the learned and Jacobi decreases per column (host, ncols each; may be
 * NULL).  Blocking. */
int lobpcg_learner_objective(lobpcg_learner_t L, int snap, const int* cols, int ncols,
                             double* loss, double* grad, double* learned_decrease,
                             double* jacobi_decrease);
/* `steps` Adam steps (learning rate lr), each on a snapshot and
 * cols_per_step distinct columns drawn with SplitMix64 from `seed`.
 * loss_first / loss_last (host, may be NULL): mean loss of the first and
 * last 10% of the steps.  Blocking. */
int lobpcg_learner_train(lobpcg_learner_t L, int steps, int cols_per_step, double lr,
                         uint64_t seed, double* loss_first, double* loss_last);
const char* lobpcg_learner_last_error(lobpcg_learner_t L);

#ifdef __cplusplus
}
#endif
#endif /* LOBPCG_MI355X_H */
