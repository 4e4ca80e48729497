"""Pins for the CPU oracle: each test checks the oracle against something other
than itself -- a library special case, a closed form, brute force on a tiny
input, an invariant the mathematics fixes, or a value the paper states.

The ``test_planted_*`` tests plant a plausible mistake in the oracle (on the
CPU) and show that one of the pins catches it.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.linalg as sla

import synth
from oracle import lobpcg_oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def graded(n, m, cond, seed):
    """n x m matrix with singular values logspaced over [1/cond, 1]."""
    g = synth.rng(seed)
    U, _ = np.linalg.qr(g.standard_normal((n, m)))
    V, _ = np.linalg.qr(g.standard_normal((m, m)))
    s = np.logspace(0, -math.log10(cond), m)
    return (U * s) @ V.T


def householder_q(X):
    Q, R = np.linalg.qr(X)
    return Q * np.sign(np.diag(R))


def projector_distance(A, B):
    """|| P_A - P_B ||_2 for column spaces (sine of largest principal angle)."""
    QA = np.linalg.qr(A)[0]
    QB = np.linalg.qr(B)[0]
    return float(np.linalg.norm(QA @ QA.T - QB @ QB.T, 2))


# ---------------------------------------------------------------------------
# paper-stated constants


def test_paper_constants():
    c = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    assert O.TAU_ORTHO == c["tau_ortho"]["value"]
    assert O.SHIFT_ALPHA0 == c["shift_alpha0"]["value"]


def test_splitmix64_published_sequence():
    # SplitMix64 seeded with 0: the first three outputs of the reference
    # generator (Steele, Lea, Flood 2014; also Vigna's splitmix64.c).
    gamma = 0x9E3779B97F4A7C15
    assert O.splitmix64(0) == 0xE220A8397B1DCDAF
    assert O.splitmix64(gamma) == 0x6E789E6AA1B965F4
    assert O.splitmix64((2 * gamma) % (1 << 64)) == 0x06C45D188009454F


# ---------------------------------------------------------------------------
# Alg. 2: ortho(X)


def check_ortho_vs_qr(ortho_fn):
    worst = 0.0
    for seed, cond in [(1, 10.0), (2, 1e3), (3, 1e3)]:
        X = graded(400, 8, cond, seed) * synth.rng(seed + 10).uniform(0.5, 50, 8)
        Q = ortho_fn(X)
        worst = max(worst, float(np.max(np.abs(Q - householder_q(X)))))
    return worst


def test_ortho_equals_householder_q():
    # Without a shift, Cholesky QR and Householder QR give the same Q once
    # R has a positive diagonal (a library special case of Alg. 2).
    assert check_ortho_vs_qr(O.ortho) < 1e-12


@pytest.mark.parametrize("cond", [1.0, 1e4, 1e7])
def test_ortho_orthonormal(cond):
    st = O.OrthoStats()
    Q = O.ortho(graded(1000, 12, cond, 7), stats=st)
    assert O.max_abs(Q.T @ Q - np.eye(12)) <= O.TAU_ORTHO
    assert st.stalled == 0


def test_cholesky_breakdown_near_1e8():
    # Sec. 3.2: the unshifted factorisation of the overlap fails once
    # cond(X) is past ~1e8; well below it, it succeeds.
    c = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    edge = c["cholesky_breakdown_condition"]["value"]
    ok = O._potrf(O.normalize_columns(graded(500, 6, edge / 1e3, 3)).T @ O.normalize_columns(graded(500, 6, edge / 1e3, 3)))
    assert ok is not None
    fails = 0
    for seed in range(5):
        X = O.normalize_columns(graded(500, 6, edge * 1e3, seed))
        if O._potrf(X.T @ X) is None:
            fails += 1
    assert fails >= 4


def test_ortho_forced_shift_at_most_four_factorizations():
    # Columns [x, x + 1e-10 y, z...]: cond ~ 1e10, the first Cholesky must
    # fail; Sec. 3.2 says one failed + one shifted + two unshifted suffice.
    g = synth.rng(5)
    x, y = g.standard_normal(800), g.standard_normal(800)
    Z = g.standard_normal((800, 3))
    X = np.column_stack([x, x + 1e-10 * y, Z])
    st = O.OrthoStats()
    Q = O.ortho(X, stats=st)
    c = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    assert st.failed_factorizations >= 1
    assert st.shifted == 1
    assert st.factorizations <= c["max_cholesky_factorizations"]["value"]
    assert O.max_abs(Q.T @ Q - np.eye(5)) <= O.TAU_ORTHO
    # the span keeps x, the part of y that survived rounding, and Z
    assert projector_distance(Q, np.column_stack([x, y, Z])) < 1e-5


def test_shift_value_is_alpha_eps_normX():
    # Force a failure and read the shift back from L L^T - M (Alg. 2).
    X = O.normalize_columns(np.column_stack([np.ones(50), np.ones(50), np.arange(50.0)]))
    M = X.T @ X
    st = O.OrthoStats()
    L = O.shifted_cholesky(M, st)
    assert st.failed_factorizations >= 1 and L is not None
    sigma = np.diag(L @ L.T - M).mean()
    k = st.factorizations - 2  # retries before the successful one
    expected = O.SHIFT_ALPHA0 * (O.SHIFT_GROWTH ** k) * O.EPS * math.sqrt(np.trace(M))
    # rounding in M + sigma I leaves sigma known to ~1e-16 absolute; a wrong
    # alpha (10x off) or norm (||X||^2 vs ||X||) would miss by far more
    assert abs(sigma - expected) <= 0.02 * expected


def test_zero_column_replaced():
    X = np.zeros((64, 3))
    X[:, 0] = 1.0
    X[:, 2] = np.arange(64.0)
    st = O.OrthoStats()
    Q = O.ortho(X, stats=st)
    assert st.zero_columns == 1
    assert O.max_abs(Q.T @ Q - np.eye(3)) <= O.TAU_ORTHO


# ---------------------------------------------------------------------------
# Alg. 3: ortho(X, Y)


def check_ortho_against(fn):
    g = synth.rng(11)
    n = 600
    Y = np.linalg.qr(g.standard_normal((n, 6)))[0]
    Xt = Y @ g.standard_normal((6, 4)) + 1e-10 * g.standard_normal((n, 4))
    st = O.OrthoStats()
    Q = fn(Xt, Y, stats=st)
    return Y, Xt, Q, st


def test_ortho_against_pins():
    Y, Xt, Q, st = check_ortho_against(O.ortho_against)
    assert O.max_abs(Y.T @ Q) <= O.TAU_ORTHO
    assert O.max_abs(Q.T @ Q - np.eye(4)) <= O.TAU_ORTHO
    # span([Y Q]) == span([Y X~]) up to what rounding left of the 1e-10 part
    assert projector_distance(np.hstack([Y, Q]), np.hstack([Y, Xt])) < 1e-5
    # Sec. 3.2: about two passes are usually enough
    assert st.against_passes <= 3


def test_ortho_against_single_projection_is_not_enough():
    # The paper's argument for the loop: one projection + ortho leaves
    # Y^T Q of order eps/delta.  Check the oracle really needed > 1 pass.
    Y, Xt, Q, st = check_ortho_against(O.ortho_against)
    one = O.ortho(Xt - Y @ (Y.T @ Xt))
    assert O.max_abs(Y.T @ one) > 1e3 * O.TAU_ORTHO
    assert st.against_passes >= 2


# ---------------------------------------------------------------------------
# Rayleigh-Ritz and the preconditioner


def test_rayleigh_ritz_interlacing():
    A = synth.random_symmetric(300, 4)
    lam = np.linalg.eigvalsh(A)
    V = np.linalg.qr(synth.rng(5).standard_normal((300, 12)))[0]
    theta, U = O.rayleigh_ritz(V, A @ V)
    # Cauchy interlacing: lam_j <= theta_j <= lam_{n-p+j}
    assert np.all(theta >= lam[:12] - 1e-12)
    assert np.all(theta <= lam[-12:] + 1e-12)
    assert np.all(np.diff(theta) >= 0)
    # U diagonalises the projected matrix
    a = V.T @ A @ V
    assert np.allclose(U.T @ (0.5 * (a + a.T)) @ U, np.diag(theta), atol=1e-12)


def test_rayleigh_ritz_orientation_and_p_accuracy():
    # R16: every coefficient column has a nonnegative diagonal entry and is
    # still an eigenvector; with it, u_x - E is the small update, and the
    # P coefficients built from it match those built from the flipped
    # column only up to eps / ||update|| (the cancellation R16 avoids)
    g = synth.rng(21)
    n, m = 400, 4
    A = synth.dense_dd(n, seed=21)
    w, V = np.linalg.eigh(A)
    X = np.linalg.qr(V[:, :m] + 1e-9 * g.standard_normal((n, m)))[0]
    W = np.linalg.qr(g.standard_normal((n, m)) - X @ (X.T @ g.standard_normal((n, m))))[0]
    W = np.linalg.qr(W - X @ (X.T @ W))[0]
    Vb = np.hstack([X, W])
    th, U = O.rayleigh_ritz(Vb, A @ Vb)
    a = O.symmetrize(Vb.T @ A @ Vb)
    assert np.all(np.diag(U) >= 0.0)
    assert np.abs(a @ U - U * th).max() <= 1e-12 * np.abs(a).max()
    # flipping basis vector k flips row k of every eigenvector and so the
    # sign of diagonal entry k: the oriented result is exactly D U D, with
    # u_xx ~ I, whatever signs the eigensolver picks
    for k in range(m):
        D = np.ones(2 * m)
        D[k] = -1.0
        th2, U2 = O.rayleigh_ritz(Vb * D, (A @ Vb) * D)
        assert np.all(np.diag(U2) >= 0.0)
        assert np.allclose(U2, D[:, None] * U * D[None, :], atol=1e-10)
        assert np.linalg.norm(U2[:, :m] - np.eye(2 * m)[:, :m], axis=0).max() < 1e-6
    ux = U[:, :m]
    upd = ux - np.eye(2 * m)[:, :m]
    assert np.linalg.norm(upd, axis=0).max() < 1e-6  # the update is small
    flip = ux * np.array([1.0, -1.0, 1.0, -1.0])
    upd_f = flip - np.eye(2 * m)[:, :m]
    # both project to the same direction; the flipped one loses digits
    def proj(Y):
        Y = Y - ux @ (ux.T @ Y)
        return Y / np.linalg.norm(Y, axis=0)
    p0, p1 = proj(upd), proj(upd_f)
    cos = np.abs(np.sum(p0 * p1, axis=0))
    assert np.all(cos > 0.99)
    assert np.max(1.0 - cos) > 1e-12  # measurable loss on the flipped columns


def test_preconditioner_guard_by_hand():
    R = np.array([[1.0, 2.0], [1.0, 2.0], [1.0, 2.0]])
    d = np.array([3.0, 1.0, 1.0 + 5e-9])
    theta = np.array([1.0, 2.0])
    W = O.precondition_diag(R, d, theta)
    # column 0: |3-1| = 2; |0| -> guard 1e-8 (positive); |5e-9| -> 1e-8
    assert np.allclose(W[:, 0], [0.5, 1e8, 1e8], rtol=1e-15)
    # column 1: |3-2| = 1, |1-2| = 1, |1+5e-9-2| ~ 1
    assert np.allclose(W[:, 1], [2.0, 2.0, 2.0 / (1.0 - 5e-9)], rtol=1e-15)
    Ws = O.precondition_diag(R, d, theta, signed=True)
    assert np.allclose(Ws[:, 1], [2.0, -2.0, -2.0 / (1.0 - 5e-9)], rtol=1e-15)
    assert Ws[1, 0] == 1e8  # sign(0) taken as +


# ---------------------------------------------------------------------------
# full solves against closed forms and brute force


def assert_eigs(res, lam, tol=1e-8, rel=1e-9):
    assert res.converged
    assert np.all(res.resnorms <= tol)
    scale = np.maximum(np.abs(lam), 1e-3 * max(1.0, float(np.max(np.abs(lam)))))
    assert np.all(np.abs(res.evals - lam) <= rel * scale), (res.evals, lam)


def test_closed_form_laplacian_1d():
    n, k = 120, 4
    L = synth.laplacian_1d(n)
    op = O.csr_operator(L.row_ptr, L.col, L.val, n)
    res = O.lobpcg(op, synth.start_block(n, 6, 1), k, 1e-9, diag=L.diag, max_iter=2000)
    j = np.arange(1, k + 1)
    lam = 2.0 - 2.0 * np.cos(j * np.pi / (n + 1))
    assert_eigs(res, lam, tol=1e-9)
    # eigenvectors sin(i j pi/(n+1)) (up to sign)
    i = np.arange(1, n + 1)[:, None]
    ex = np.sin(i * j[None, :] * np.pi / (n + 1))
    ex /= np.linalg.norm(ex, axis=0)
    assert np.all(np.abs(np.abs(np.sum(ex * res.evecs, axis=0)) - 1.0) < 1e-8)


def test_closed_form_diagonal():
    d = synth.rng(3).permutation(np.linspace(1.0, 9.0, 150))
    A = np.diag(d)
    res = O.lobpcg(O.dense_operator(A), synth.start_block(150, 5, 2), 5, 1e-9, diag=d)
    lam = np.sort(d)[:5]
    assert_eigs(res, lam, tol=1e-9)
    idx = np.argsort(d)[:5]
    for c in range(5):
        e = np.zeros(150)
        e[idx[c]] = 1.0
        assert np.allclose(res.evecs[:, c], e, atol=1e-8)


def test_closed_form_kronsum():
    na = 24
    A, _ = synth.kronsum(na=na, seed=9)
    V = np.zeros((na, na))
    alpha = np.linalg.eigvalsh(A)
    sums = np.sort((alpha[:, None] + alpha[None, :]).reshape(-1))
    k = 6
    assert sums[k] - sums[k - 1] > 1e-6  # the block does not cut a cluster
    op = O.kronsum_operator(A, V)
    res = O.lobpcg(op, synth.start_block(na * na, k, 3), k, 1e-9, diag=O.kronsum_diagonal(A, V))
    assert_eigs(res, sums[:k], tol=1e-9)


def test_kronsum_operator_matches_kron():
    na = 5
    A, V = synth.kronsum(na=na, seed=2)
    H = np.kron(A, np.eye(na)) + np.kron(np.eye(na), A) + np.diag(V.reshape(-1))
    X = synth.start_block(na * na, 3, 1)
    assert np.allclose(O.kronsum_operator(A, V)(X), H @ X, atol=1e-13)
    assert np.allclose(O.kronsum_diagonal(A, V), np.diag(H), atol=1e-15)


@pytest.mark.parametrize(
    "kind",
    ["random", "clustered", "degenerate"],
)
def test_brute_force_dense(kind):
    n = 160
    if kind == "random":
        A = synth.random_symmetric(n, 21)
    elif kind == "clustered":
        lam = np.concatenate([[1.0, 1.0 + 1e-6, 1.0 + 2e-6, 2.0], np.linspace(3.0, 10.0, n - 4)])
        A, _ = synth.prescribed_spectrum(lam, 22)
    else:
        lam = np.concatenate([[-1.0, 0.5, 0.5, 2.0], np.linspace(3.0, 10.0, n - 4)])
        A, _ = synth.prescribed_spectrum(lam, 23)
    k = 4
    w, Vx = np.linalg.eigh(A)
    res = O.lobpcg(O.dense_operator(A), synth.start_block(n, k, 5), k, 1e-9, diag=np.diag(A).copy(), max_iter=3000)
    assert_eigs(res, w[:k], tol=1e-9)
    # spectral projector of the whole computed block vs brute force
    assert projector_distance(res.evecs, Vx[:, :k]) < 1e-6


def test_invariants_and_ritz_monotone():
    n, m = 400, 6
    A = synth.dense_dd(n, seed=77)
    lam = np.linalg.eigvalsh(A)
    res = O.lobpcg(O.dense_operator(A), synth.start_block(n, m, 8), m, 1e-9, diag=np.diag(A).copy())
    assert res.converged
    X = res.X_all
    assert O.max_abs(X.T @ X - np.eye(m)) < 1e-12
    H = np.array(res.history_theta)
    # X^(k) is inside the next subspace, so Ritz values never increase
    assert np.all(np.diff(H, axis=0) <= 10 * np.finfo(float).eps * np.abs(lam).max())
    # Courant-Fischer: theta_j >= lambda_j at every iteration
    assert np.all(H >= lam[:m] - 1e-12)
    assert np.all(np.diff(res.evals) >= 0)


def test_reuse_keeps_ax_accurate():
    # Sec. 3.1 "Reuse of applications": AX reached through orthonormal
    # coefficients only stays within a few ulps of an explicit A X.
    n, m = 300, 4
    A = synth.dense_dd(n, seed=5)
    normA = np.abs(A).sum(1).max()
    worst = []

    def cb(d):
        worst.append(O.max_abs(d["AX"] - A @ d["X"]))

    res = O.lobpcg(O.dense_operator(A), synth.start_block(n, m, 1), m, 1e-10, diag=np.diag(A).copy(), callback=cb)
    assert res.converged and len(worst) > 5
    assert max(worst) <= 1e3 * np.finfo(float).eps * normA


def test_locking_matvec_count():
    # Widely separated leading eigenvalues converge one after another.
    n, m = 200, 4
    d = np.concatenate([[1.0, 2.0, 4.0, 8.0], np.linspace(20.0, 40.0, n - 4)])
    A = np.diag(d) + 1e-3 * synth.random_symmetric(n, 3)
    res = O.lobpcg(O.dense_operator(A), synth.start_block(n, m, 4), m, 1e-9, diag=np.diag(A).copy())
    assert res.converged
    act = res.history_active
    assert all(a >= b for a, b in zip(act, act[1:]))  # m_conv never decreases
    assert min(act) < m  # locking happened
    assert res.matvec_columns == m + sum(act) + m * res.true_checks


def test_extra_block_vectors():
    n = 300
    A = synth.dense_dd(n, seed=31)
    lam = np.linalg.eigvalsh(A)
    res = O.lobpcg(O.dense_operator(A), synth.start_block(n, 6, 2), 2, 1e-9, diag=np.diag(A).copy())
    assert_eigs(res, lam[:2], tol=1e-9)
    assert res.evecs.shape == (n, 2)


def test_max_iter_reports_not_converged():
    A = synth.dense_dd(300, seed=31)
    res = O.lobpcg(O.dense_operator(A), synth.start_block(300, 4, 2), 4, 1e-12, diag=np.diag(A).copy(), max_iter=2)
    assert not res.converged
    assert res.iterations == 2
    assert np.all(np.isfinite(res.evals)) and np.all(res.resnorms > 0)


def test_signed_preconditioner_also_converges_from_unit_guess():
    n, m = 400, 4
    A = synth.dense_dd(n, seed=12)
    d = np.diag(A).copy()
    X0 = np.zeros((n, m))
    X0[np.argsort(d)[:m], np.arange(m)] = 1.0
    X0 += 1e-3 * synth.start_block(n, m, 1)
    res = O.lobpcg(O.dense_operator(A), X0, m, 1e-9, diag=d, precond="diag_signed")
    assert_eigs(res, np.linalg.eigvalsh(A)[:m], tol=1e-9)


def test_output_signs_normalised():
    A = synth.dense_dd(200, seed=2)
    res = O.lobpcg(O.dense_operator(A), synth.start_block(200, 3, 9), 3, 1e-9, diag=np.diag(A).copy())
    for j in range(3):
        i = np.argmax(np.abs(res.evecs[:, j]))
        assert res.evecs[i, j] > 0


# ---------------------------------------------------------------------------
# planted mistakes (in the oracle, on the CPU): the pins above must catch them


def test_planted_transposed_triangular_factor():
    def bad_ortho(X):
        X = O.normalize_columns(X)
        for _ in range(3):
            M = X.T @ X
            L = np.linalg.cholesky(M)
            X = X @ np.linalg.inv(L)  # should be L^-T
        return X

    try:
        worst = check_ortho_vs_qr(bad_ortho)
    except np.linalg.LinAlgError:
        worst = np.inf
    assert worst > 1e-6


def test_planted_missing_projection():
    def bad_against(X, Y, stats=None):
        return O.ortho(X, stats=stats)

    Y, Xt, Q, st = check_ortho_against(bad_against)
    assert O.max_abs(Y.T @ Q) > O.TAU_ORTHO


def test_planted_residual_sign_error(monkeypatch):
    monkeypatch.setattr(O, "ritz_residual", lambda AX, X, th: AX + X * th)
    A = synth.dense_dd(150, seed=1)
    res = O.lobpcg(O.dense_operator(A), synth.start_block(150, 3, 1), 3, 1e-9, diag=np.diag(A).copy(), max_iter=60)
    with pytest.raises(AssertionError):
        assert_eigs(res, np.linalg.eigvalsh(A)[:3], tol=1e-9)


def test_planted_wrong_end_of_spectrum(monkeypatch):
    def rr_top(V, AV):
        th, U = np.linalg.eigh(O.symmetrize(V.T @ AV))
        return th[::-1].copy(), U[:, ::-1].copy()

    monkeypatch.setattr(O, "rayleigh_ritz", rr_top)
    A = synth.dense_dd(150, seed=1)
    res = O.lobpcg(O.dense_operator(A), synth.start_block(150, 3, 1), 3, 1e-9, diag=np.diag(A).copy(), max_iter=60)
    with pytest.raises(AssertionError):
        assert_eigs(res, np.linalg.eigvalsh(A)[:3], tol=1e-9)


def run_invariants(A, m, seed):
    res = O.lobpcg(O.dense_operator(A), synth.start_block(A.shape[0], m, seed), m, 1e-9, diag=np.diag(A).copy(), max_iter=200)
    X = res.X_all
    assert res.converged
    assert O.max_abs(X.T @ X - np.eye(m)) < 1e-12


def test_planted_unorthogonalised_p(monkeypatch):
    # u_p used without its ortho against u_x: V is no longer orthonormal and
    # the standard RR is invalid; the invariants catch it.
    A = synth.dense_dd(300, seed=6)
    run_invariants(A, 4, 1)
    orig = O.ortho_against

    def skip_small(X, Y, tau=O.TAU_ORTHO, stats=None, max_passes=O.ORTHO_Y_MAX_PASSES, **kw):
        if Y is not None and Y.shape[0] < 100:  # the R^p call that builds u_p
            return O.normalize_columns(X)
        return orig(X, Y, tau, stats, max_passes, **kw)

    monkeypatch.setattr(O, "ortho_against", skip_small)
    with pytest.raises(AssertionError):
        run_invariants(A, 4, 1)


# ---------------------------------------------------------------------------
# SVQB, the last resort after the shifted retries (reading R5; Stathopoulos
# and Wu's orthonormalisation from the eigen-decomposition of the overlap)


def svqb_pin(svqb_fn):
    """One SVQB pass on unit columns of condition 1e2 and 1e4: the columns
    must come out orthonormal to within what a one-pass method built on the
    overlap allows (about eps cond^2) and span the same space as the input.
    Returns the worst error relative to that allowance."""
    worst = 0.0
    for cond in (1e2, 1e4):
        Xn = O.normalize_columns(graded(600, 8, cond, 3))
        Q = svqb_fn(Xn, Xn.T @ Xn, O.OrthoStats())
        allow = 1e2 * O.EPS * cond**2
        worst = max(worst, O.max_abs(Q.T @ Q - np.eye(8)) / allow)
        assert projector_distance(Q, Xn) < 1e-12 * cond
    return worst


def test_svqb_one_pass():
    assert svqb_pin(O.svqb) <= 1.0


def test_planted_svqb_inverse_instead_of_inverse_sqrt():
    def bad(X, M, stats):
        s, U = np.linalg.eigh(M)
        s = np.maximum(s, O.EPS * s.max())
        return (X @ U) / s  # should be / sqrt(s)

    assert svqb_pin(bad) > 1.0


def test_ortho_reaches_svqb_without_shift_retries():
    # cond ~ 1e10: the plain factorisation fails (Sec. 3.2); with no
    # shifted retry allowed, that pass of Alg. 2 takes SVQB, and the next
    # pass's plain Cholesky finishes the job
    g = synth.rng(5)
    x, y = g.standard_normal(800), g.standard_normal(800)
    Z = g.standard_normal((800, 3))
    st = O.OrthoStats()
    Q = O.ortho(np.column_stack([x, x + 1e-10 * y, Z]), stats=st, shift_retries=0)
    assert st.svqb == 1 and st.failed_factorizations == 1 and st.shifted == 0
    assert O.max_abs(Q.T @ Q - np.eye(5)) <= O.TAU_ORTHO
    assert projector_distance(Q, np.column_stack([x, y, Z])) < 1e-5
    # an exactly repeated column: no column is dropped, the output is finite
    # and orthonormal (the clamped eigenvalue turns the copy into a new
    # direction)
    st = O.OrthoStats()
    Q = O.ortho(np.column_stack([x, x, Z]), stats=st, shift_retries=0)
    assert st.svqb == 1 and Q.shape == (800, 5) and np.all(np.isfinite(Q))
    assert O.max_abs(Q.T @ Q - np.eye(5)) <= O.TAU_ORTHO
    assert projector_distance(np.column_stack([x, Z]), Q @ (Q.T @ np.column_stack([x, Z]))) < 1e-10


def test_ortho_against_with_svqb():
    # Alg. 3 around an Alg. 2 that needs SVQB (an exactly repeated column
    # makes the overlap singular, so the plain factorisation must fail): the
    # same span and Y-orthogonality bars as with the shifted Cholesky
    g = synth.rng(8)
    Y = np.linalg.qr(g.standard_normal((700, 4)))[0]
    x = g.standard_normal(700)
    Z = g.standard_normal((700, 2))
    st = O.OrthoStats()
    Q = O.ortho_against(np.column_stack([x, x, Z]), Y, stats=st, shift_retries=0)
    assert st.svqb >= 1
    assert O.max_abs(Y.T @ Q) <= O.TAU_ORTHO
    assert O.max_abs(Q.T @ Q - np.eye(4)) <= O.TAU_ORTHO
    # x and Z, less their Y parts, lie in span(Q)
    B = np.column_stack([x, Z])
    B = B - Y @ (Y.T @ B)
    assert np.linalg.norm(B - Q @ (Q.T @ B)) <= 1e-12 * np.linalg.norm(B)


# ---------------------------------------------------------------------------
# reading R9: a failed true-residual check restarts the iteration


def _drifted_solve(plant, tol=1e-9, force_restarts=0):
    n, k = 400, 4
    A = synth.dense_dd(n, seed=7)
    noise = 1e-6 * synth.start_block(n, k, 99)
    planted = {}

    def cb(d):
        # once the recurrence's residuals meet tol, move X away from the
        # vectors they were measured on (in place: this is the block the
        # true check will judge)
        if plant and not planted and np.max(d["rnorm"][:k]) <= tol:
            d["X"] += noise
            planted["it"] = d["it"]

    res = O.lobpcg(O.dense_operator(A), synth.start_block(n, k, 8), k, tol, diag=np.diag(A).copy(), callback=cb,
                   force_restarts=force_restarts)
    return A, res, planted


def test_restart_after_failed_true_check():
    A, res0, _ = _drifted_solve(False)
    assert res0.converged and res0.true_checks == 1 and res0.restarts == 0
    A, res, planted = _drifted_solve(True)
    assert planted
    assert res.true_checks >= 2 and res.restarts >= 1
    assert res.converged and np.max(res.resnorms) <= 1e-9
    assert_eigs(res, np.linalg.eigvalsh(A)[:4], tol=1e-9)
    # the restart costs iterations: it drops P and re-enters the loop
    assert res.iterations > res0.iterations
    X = res.X_all
    assert O.max_abs(X.T @ X - np.eye(4)) < 1e-12


def test_forced_restart_hook_matches_a_real_one():
    # the test hook that rejects the first true check takes the same branch
    A, res, _ = _drifted_solve(False, force_restarts=1)
    assert res.restarts == 1 and res.true_checks == 2
    assert res.converged
    assert_eigs(res, np.linalg.eigvalsh(A)[:4], tol=1e-9)


# ---------------------------------------------------------------------------
# reading R22: a stalled recurrence still reaches the true-residual check


def _floor_solve(window, plant):
    n, k = 400, 4
    A = synth.dense_dd(n, seed=7)
    e = synth.start_block(n, 1, 98)[:, 0]
    E = 3e-8 * e / np.linalg.norm(e)
    planted = {}

    def cb(d):
        # once the last sought column is on its way, add a fixed error to its
        # A x: the recurrence carries it on (A X from [AX AW AP] U), so the
        # residuals it reports for that column stay near 3e-8 (30 tol)
        if plant and not planted and d["rnorm"][k - 1] < 1e-4:
            d["AX"][:, k - 1] += E
            planted["it"] = d["it"]

    res = O.lobpcg(O.dense_operator(A), synth.start_block(n, k, 8), k, 1e-9, diag=np.diag(A).copy(), callback=cb,
                   max_iter=300, stall_window=window)
    return A, res, planted


def test_stalled_recurrence_reaches_the_true_check():
    A, res0, planted = _floor_solve(0, True)
    assert planted
    # without the rule R9's check is never reached: the iterations run out
    assert not res0.converged and res0.iterations == 300
    assert res0.stall_checks == 0 and res0.true_checks == 1
    A, res, _ = _floor_solve(20, True)
    assert res.converged and res.stall_checks >= 1 and res.restarts >= 1
    assert np.max(res.resnorms) <= 1e-9
    assert_eigs(res, np.linalg.eigvalsh(A)[:4], tol=1e-9)
    X = res.X_all
    assert O.max_abs(X.T @ X - np.eye(4)) < 1e-12


def test_stall_rule_silent_on_a_converging_solve():
    A, res, _ = _floor_solve(20, False)
    assert res.converged and res.stall_checks == 0 and res.restarts == 0 and res.true_checks == 1


# ---------------------------------------------------------------------------
# the exact dense eigensolve that the full-size dense goldens come from


def test_lowest_eigenpairs_dense_closed_forms():
    # 1-D Laplacian: lambda_j = 2 - 2 cos(j pi / (n + 1)), j = 1..k
    n, k = 300, 9
    L = synth.laplacian_1d(n).to_dense()
    w, V = O.lowest_eigenpairs_dense(L, k)
    j = np.arange(1, k + 1)
    assert np.allclose(w, 2 - 2 * np.cos(j * np.pi / (n + 1)), rtol=0, atol=1e-13)
    assert np.abs(V.T @ V - np.eye(k)).max() < 1e-13
    # prescribed spectrum Q diag(lam) Q^T, with a cluster and a negative end
    lam = np.concatenate([[-3.0, -1.0, -1.0 + 1e-9, 0.5], np.linspace(2.0, 9.0, 196)])
    A, Q = synth.prescribed_spectrum(lam, 12)
    w, V = O.lowest_eigenpairs_dense(A, 5)
    assert np.allclose(w, lam[:5], rtol=0, atol=1e-13)
    assert np.linalg.norm(A @ V - V * w, axis=0).max() < 1e-13


def test_planted_eigh_off_by_one_index():
    lam = np.linspace(1.0, 2.0, 50)
    A, _ = synth.prescribed_spectrum(lam, 3)
    w = sla.eigh(A, subset_by_index=[1, 4], eigvals_only=True)  # skips the lowest
    with pytest.raises(AssertionError):
        assert np.allclose(w, lam[:4], atol=1e-13)


def subspace_sine(A, B):
    """Sine of the largest principal angle between the column spaces of A
    and B (equal dimensions), ||Q_B - Q_A Q_A^T Q_B||_2, for tall blocks."""
    QA = np.linalg.qr(A)[0]
    QB = np.linalg.qr(B)[0]
    return float(np.linalg.norm(QB - QA @ (QA.T @ QB), 2))


# ---------------------------------------------------------------------------
# reading R17: cheap exits of Alg. 2 and Alg. 3 (Sec. 3.2 proposes a norm
# estimate of L^-T and the growth factor of ortho(X); the exit rules are
# this oracle's reading)


@pytest.mark.parametrize("n", [20000, 200000])
def test_cheap_exit_alg2(n):
    I = np.eye(16)
    for cond in (1.0 + 1e-3, 3.0, 1e3, 1e7):
        X = graded(n, 16, cond, 3) * synth.rng(5).uniform(0.5, 2.0, 16)
        st0, st1 = O.OrthoStats(), O.OrthoStats()
        Q0 = O.ortho(X, stats=st0)
        Q1 = O.ortho(X, stats=st1, cheap_exit=True)
        assert O.max_abs(Q1.T @ Q1 - I) <= O.TAU_ORTHO, cond
        assert subspace_sine(Q1, Q0) < 1e-13 * cond
        assert st1.grams <= st0.grams and st1.updates == st0.updates
        if cond == 1e3:
            # Cholesky-QR twice, then the exit replaces the third overlap
            assert st0.updates == 2 and st1.cheap_exits == 1 and st1.grams == st0.grams - 1


def test_cheap_exit_alg3():
    n = 100000
    g = synth.rng(14)
    Y = np.linalg.qr(g.standard_normal((n, 16)))[0]
    exits = 0
    for delta in (1e-1, 1e-4, 1e-10):
        Xt = Y @ g.standard_normal((16, 8)) + delta * g.standard_normal((n, 8))
        st0, st1 = O.OrthoStats(), O.OrthoStats()
        Q0 = O.ortho_against(Xt, Y, stats=st0)
        Q1 = O.ortho_against(Xt, Y, stats=st1, cheap_exit=True)
        assert O.max_abs(Y.T @ Q1) <= O.TAU_ORTHO, delta
        assert O.max_abs(Q1.T @ Q1 - np.eye(8)) <= O.TAU_ORTHO, delta
        assert subspace_sine(np.hstack([Y, Q1]), np.hstack([Y, Q0])) < 1e-12 / delta
        assert st1.against_passes <= st0.against_passes
        exits += st1.cheap_exits
    assert exits >= 3


def test_planted_cheap_exit_ignoring_kappa(monkeypatch):
    # an exit that trusts any unshifted pass (the bound on ||L^-1|| taken as
    # 1 and ||I - L|| as 0) stops after one Cholesky-QR of a cond 1e3 block,
    # whose orthogonality is only ~eps cond^2
    monkeypatch.setattr(O, "inverse_factor_bound", lambda L: (1.0, 0.0))
    Q = O.ortho(graded(20000, 16, 1e3, 3), cheap_exit=True)
    assert O.max_abs(Q.T @ Q - np.eye(16)) > O.TAU_ORTHO


def test_cheap_exit_solve_matches_eigh():
    n, k = 600, 6
    A = synth.dense_dd(n, seed=17)
    lam = np.linalg.eigvalsh(A)[:k]
    X0 = synth.start_block(n, k, 3)
    r0 = O.lobpcg(O.dense_operator(A), X0, k, 1e-9, diag=np.diag(A).copy())
    r1 = O.lobpcg(O.dense_operator(A), X0, k, 1e-9, diag=np.diag(A).copy(), cheap_exit=True)
    assert_eigs(r1, lam, tol=1e-9)
    assert O.max_abs(r1.X_all.T @ r1.X_all - np.eye(k)) < 1e-12
    assert r1.ortho.cheap_exits > 0 and r1.ortho.grams < r0.ortho.grams
    assert abs(r1.iterations - r0.iterations) <= 2


# ---------------------------------------------------------------------------
# block Davidson (Sec. 2's recurrence, Sec. 4's history; reading R18)


def _davidson_by_definition(A, X0, steps, diag):
    """X^{j+1} = RR(X^1, T^1 R^1, ..., T^j R^j) written out directly: the
    span of the blocks by Householder QR, the RR by eigh, no locking."""
    m = X0.shape[1]
    Q = np.linalg.qr(X0)[0]
    th, U = np.linalg.eigh(Q.T @ A @ Q)
    X = Q @ U[:, :m]
    blocks = [X]
    out = [th[:m]]
    for _ in range(steps):
        th_x = out[-1]
        R = A @ X - X * th_x
        den = np.abs(diag[:, None] - th_x[None, :])
        den = np.maximum(den, O.PRECOND_GUARD * np.maximum(1.0, np.abs(th_x)))
        blocks.append(R / den)
        Q = np.linalg.qr(np.hstack(blocks))[0]
        th, U = np.linalg.eigh(Q.T @ A @ Q)
        X = Q @ U[:, :m]
        out.append(th[:m])
    return out


def test_davidson_is_rr_on_the_history():
    n, m = 300, 3
    A = synth.dense_dd(n, seed=41)
    X0 = synth.start_block(n, m, 5)
    d = np.diag(A).copy()
    res = O.davidson(O.dense_operator(A), X0, m, 1e-30, diag=d, max_iter=4)
    ref = _davidson_by_definition(A, X0, 4, d)
    assert res.restarts == 0 and res.max_basis == 5 * m
    # the two roundings (Cholesky-QR of the growing basis vs Householder QR
    # of the stacked blocks) separate to ~1e-12 relative over the steps,
    # since each step's residuals carry the previous step's rounding
    for j in range(5):
        assert np.allclose(res.history_theta[j], ref[j], rtol=1e-10, atol=0), j
    # the subspace only grows between restarts: Ritz values never increase
    H = np.array(res.history_theta)
    assert np.all(np.diff(H, axis=0) <= 1e-13)


@pytest.mark.parametrize("max_dim", [8, 24, None])
def test_davidson_vs_eigh(max_dim):
    n, k = 600, 4
    A = synth.dense_dd(n, seed=2)
    lam = np.linalg.eigvalsh(A)[:k]
    res = O.davidson(O.dense_operator(A), synth.start_block(n, k, 3), k, 1e-9, diag=np.diag(A).copy(), max_dim=max_dim)
    assert_eigs(res, lam, tol=1e-9)
    assert O.max_abs(res.X_all.T @ res.X_all - np.eye(k)) < 1e-12
    if max_dim == 8:
        assert res.restarts > 0 and res.max_basis <= 8


def test_davidson_closed_form_laplacian():
    n, k = 150, 3
    L = synth.laplacian_1d(n)
    op = O.csr_operator(L.row_ptr, L.col, L.val, n)
    res = O.davidson(op, synth.start_block(n, 5, 1), k, 1e-9, diag=L.diag, max_dim=40, max_iter=3000)
    j = np.arange(1, k + 1)
    assert_eigs(res, 2 - 2 * np.cos(j * np.pi / (n + 1)), tol=1e-9)


def test_planted_davidson_without_projection(monkeypatch):
    # each new block orthonormalised only among itself (no Alg. 3 against
    # the basis): the basis stops being orthonormal and the standard RR on it
    # goes wrong
    monkeypatch.setattr(O, "ortho_against", lambda X, Y, tau=O.TAU_ORTHO, stats=None, **kw: O.ortho(X, tau, stats))
    n, m = 300, 3
    A = synth.dense_dd(n, seed=41)
    X0 = synth.start_block(n, m, 5)
    res = O.davidson(O.dense_operator(A), X0, m, 1e-30, diag=np.diag(A).copy(), max_iter=4)
    ref = _davidson_by_definition(A, X0, 4, np.diag(A).copy())
    assert not all(np.allclose(res.history_theta[j], ref[j], rtol=1e-10, atol=0) for j in range(5))


# ---------------------------------------------------------------------------
# tridiagonal preconditioner (Sec. 4.4, Table 1; reading R19)


def _tri_dense(d, e, theta):
    ae = np.abs(e)
    rowoff = np.zeros(d.size)
    rowoff[:-1] += ae
    rowoff[1:] += ae
    delta = O.PRECOND_GUARD * max(1.0, abs(theta))
    t = np.maximum(np.abs(d - theta), rowoff + delta)
    return np.diag(t) + np.diag(e, 1) + np.diag(e, -1)


def test_tridiag_preconditioner_definition():
    n = 400
    A = synth.dense_dd(n, seed=9) + np.diag(np.full(n - 1, 0.3), 1) + np.diag(np.full(n - 1, 0.3), -1)
    d, e = np.diag(A).copy(), O.tridiagonal_part(A)
    assert np.array_equal(e, np.diagonal(A, 1))
    R = synth.start_block(n, 3, 1)
    theta = np.array([1.2, 3.01, 11.0])  # below, inside and far inside the diagonal's range
    W = O.precondition_tridiag(R, d, e, theta)
    for j in range(3):
        T = _tri_dense(d, e, theta[j])
        assert np.all(np.linalg.eigvalsh(T) > 0)  # positive definite
        assert np.allclose(W[:, j], np.linalg.solve(T, R[:, j]), rtol=0, atol=1e-12 * np.abs(W[:, j]).max())
    # sparse and dense inputs give the same off-diagonal
    Cs = synth.csr_from_dense(A).to_scipy()
    assert np.array_equal(O.tridiagonal_part(Cs), e)


def test_tridiag_reduces_to_jacobi_without_offdiagonal():
    n = 300
    d = synth.rng(3).uniform(0.5, 5.0, n)
    d[7] = 2.0  # an entry right at theta: the guard decides
    R = synth.start_block(n, 2, 4)
    theta = np.array([2.0, 0.1])
    W = O.precondition_tridiag(R, d, np.zeros(n - 1), theta)
    assert np.array_equal(W, O.precondition_diag(R, d, theta))


def test_planted_tridiag_subdiagonal_shift():
    # the sub-diagonal taken one row off (e shifted by one) is caught by the
    # dense solve of the definition
    n = 200
    g = synth.rng(8)
    d, e = g.uniform(2.0, 4.0, n), g.uniform(-0.5, 0.5, n - 1)
    R = g.standard_normal((n, 1))
    from scipy.linalg import lapack

    ae = np.abs(e)
    rowoff = np.zeros(n)
    rowoff[:-1] += ae
    rowoff[1:] += ae
    t = np.maximum(np.abs(d - 1.0), rowoff + 1e-8)
    _, _, _, bad, _ = lapack.dgtsv(np.roll(e, 1), t, e.copy(), R[:, 0].copy())
    good = np.linalg.solve(_tri_dense(d, e, 1.0), R[:, 0])
    assert np.allclose(O.precondition_tridiag(R, d, e, np.array([1.0]))[:, 0], good, atol=1e-13)
    assert not np.allclose(bad, good, atol=1e-8)


def test_tridiag_solve_matches_eigh():
    n, k = 600, 4
    A = synth.dense_dd(n, seed=4) + np.diag(np.full(n - 1, 0.02), 1) + np.diag(np.full(n - 1, 0.02), -1)
    lam = np.linalg.eigvalsh(A)[:k]
    X0 = synth.start_block(n, k, 2)
    d, e = np.diag(A).copy(), O.tridiagonal_part(A)
    r0 = O.lobpcg(O.dense_operator(A), X0, k, 1e-9, diag=d)
    r1 = O.lobpcg(O.dense_operator(A), X0, k, 1e-9, diag=d, precond="tridiag", off=e)
    assert_eigs(r1, lam, tol=1e-9)
    # the tridiagonal part is a better model of A here than its diagonal
    assert r1.iterations < r0.iterations
    rd = O.davidson(O.dense_operator(A), X0, k, 1e-9, diag=d, precond="tridiag", off=e)
    assert_eigs(rd, lam, tol=1e-9)


# ---------------------------------------------------------------------------
# the generalized problem A x = lambda B x (Sec. 3.3; reading R21)


def _gen_problem(n=400, seed=5):
    A = synth.dense_dd(n, seed=seed)
    g = synth.rng(seed + 4)
    B = np.diag(g.uniform(1.0, 2.0, n)) + synth.random_symmetric(n, seed + 1, 1e-3)
    return A, B


def test_generalized_vs_scipy_eigh():
    n, k = 400, 4
    A, B = _gen_problem(n)
    lam = sla.eigh(A, B, eigvals_only=True)[:k]
    res = O.lobpcg_generalized(O.dense_operator(A), O.dense_operator(B), synth.start_block(n, k, 2), k, 1e-9,
                               dA=np.diag(A).copy(), dB=np.diag(B).copy())
    assert_eigs(res, lam, tol=1e-9)
    X = res.X_all
    assert O.max_abs(X.T @ B @ X - np.eye(k)) < 1e-12  # B-orthonormal output
    r = np.linalg.norm(A @ X - (B @ X) * res.theta_all, axis=0)
    assert np.all(r[:k] <= 1e-9)
    # Courant-Fischer for the pencil: Ritz values never below the eigenvalues
    assert np.all(np.array(res.history_theta) >= lam - 1e-12)


def test_generalized_with_identity_is_the_standard_method():
    n, k = 400, 4
    A = synth.dense_dd(n, seed=5)
    X0 = synth.start_block(n, k, 2)
    rI = O.lobpcg_generalized(O.dense_operator(A), lambda X: X.copy(), X0, k, 1e-9, dA=np.diag(A).copy(), dB=np.ones(n))
    rs = O.lobpcg(O.dense_operator(A), X0, k, 1e-9, diag=np.diag(A).copy())
    assert rI.iterations == rs.iterations
    assert np.allclose(rI.evals, rs.evals, rtol=0, atol=1e-13)


def test_generalized_closed_form_diagonal():
    n, k = 300, 5
    g = synth.rng(12)
    a = g.uniform(1.0, 50.0, n)
    b = g.uniform(0.5, 3.0, n)
    res = O.lobpcg_generalized(lambda X: a[:, None] * X, lambda X: b[:, None] * X, synth.start_block(n, 8, 1), k, 1e-10,
                               dA=a, dB=b)
    assert_eigs(res, np.sort(a / b)[:k], tol=1e-10)


def test_planted_euclidean_projection_in_generalized(monkeypatch):
    # projecting W against [X P] with Y^T W instead of (B Y)^T W leaves W
    # B-nonorthogonal to X: the standard RR on V is then invalid
    n, k = 400, 4
    A, B = _gen_problem(n)
    lam = sla.eigh(A, B, eigvals_only=True)[:k]
    orig = O.b_ortho_against
    monkeypatch.setattr(O, "b_ortho_against", lambda Wt, Y, BY, tau, st, max_passes=4: orig(Wt, Y, Y, tau, st, max_passes))
    res = O.lobpcg_generalized(O.dense_operator(A), O.dense_operator(B), synth.start_block(n, k, 2), k, 1e-9,
                               dA=np.diag(A).copy(), dB=np.diag(B).copy(), max_iter=200)
    with pytest.raises(AssertionError):
        assert_eigs(res, lam, tol=1e-9)
