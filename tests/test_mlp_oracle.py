"""Pins for the CPU oracle of the learned preconditioner (oracle/mlp_oracle.py)."""
import numpy as np

import synth
from oracle import lobpcg_oracle as O
from oracle import mlp_oracle as M


def small_net(seed=1, H=16, out_bias=-1.0):
    p = M.init_params(seed, H=H, out_bias=out_bias)
    p.W3 *= 10.0  # undo the small output init so every layer matters
    return p


def block_problem(n=40, m=3, seed=5):
    """An orthonormal Ritz block X of a dense diagonally dominant A with its
    Ritz values and residuals."""
    A = synth.dense_dd(n, seed=seed)
    g = synth.rng(seed + 1)
    X = np.linalg.qr(g.standard_normal((n, m)))[0]
    th, U = np.linalg.eigh(X.T @ A @ X)
    X = X @ U
    R = A @ X - X * th
    d = np.diag(A).copy()
    rho = np.abs(A).sum(1) - np.abs(d)
    return A, X, th, R, d, rho, M.scale_of(d)


def test_backward_dy_matches_central_differences():
    H = 16
    p = small_net(H=H)
    g = synth.rng(2)
    X = g.standard_normal((50, M.NFEAT))
    dy = g.standard_normal(50)
    gr = M.backward_dy(p, M.forward(p, X)[1], dy).flat()
    v = p.flat()
    h = 1e-6
    for i in np.linspace(0, v.size - 1, 60).astype(int):
        vp, vm = v.copy(), v.copy()
        vp[i] += h
        vm[i] -= h
        fp = dy @ M.forward(M.Params.from_flat(vp, H=H), X)[0]
        fm = dy @ M.forward(M.Params.from_flat(vm, H=H), X)[0]
        fd = (fp - fm) / (2 * h)
        assert abs(fd - gr[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, gr[i])


def test_objective_gradient_matches_central_differences():
    H = 16
    A, X, th, R, d, rho, s = block_problem()
    p = small_net(H=H)
    cols = [0, 2]
    L, gr = M.objective(p, A, X, R, th, cols, d, rho, s)
    v = p.flat()
    h = 1e-6
    checked = 0
    for i in np.linspace(0, v.size - 1, 50).astype(int):
        vp, vm = v.copy(), v.copy()
        vp[i] += h
        vm[i] -= h
        lp = M.objective(M.Params.from_flat(vp, H=H), A, X, R, th, cols, d, rho, s)[0]
        lm = M.objective(M.Params.from_flat(vm, H=H), A, X, R, th, cols, d, rho, s)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gr[i]) <= 1e-6 * max(1e-3, abs(fd)), (i, fd, gr[i])
        checked += abs(fd) > 1e-6
    assert checked > 20


def test_alignment_closed_forms():
    g = np.random.default_rng(5)
    tau = g.standard_normal(40)
    assert abs(M.alignment(3.0 * tau, tau)[0]) <= 1e-15  # same direction: 0
    assert abs(M.alignment(-0.5 * tau, tau)[0]) <= 1e-15  # sign does not matter
    e1, e2 = np.eye(40)[0], np.eye(40)[1]
    assert M.alignment(e2, e1)[0] == 1.0  # orthogonal: 1
    assert abs(M.alignment(e1 + e2, e1)[0] - 0.5) <= 1e-15  # 45 degrees: sin^2 = 1/2
    u = g.standard_normal(40)
    v0 = M.alignment(u, tau)[0]
    assert abs(M.alignment(7.0 * u, 0.01 * tau)[0] - v0) <= 1e-14  # scale-free in both
    v, gz = M.alignment(u, np.zeros(40))  # no target: no term
    assert v == 0.0 and not gz.any()


def test_alignment_gradient_matches_central_differences():
    g = np.random.default_rng(6)
    u, tau = g.standard_normal(30), g.standard_normal(30)
    _, gr = M.alignment(u, tau)
    h = 1e-6
    for i in range(30):
        up, um = u.copy(), u.copy()
        up[i] += h
        um[i] -= h
        fd = (M.alignment(up, tau)[0] - M.alignment(um, tau)[0]) / (2 * h)
        assert abs(fd - gr[i]) <= 1e-7 * max(1.0, abs(fd)), (i, fd, gr[i])


def test_objective_with_supervision_gradient_matches_central_differences():
    H = 16
    A, X, th, R, d, rho, s = block_problem()
    p = small_net(H=H)
    cols = [0, 2]
    T = M.jd_targets(A, X, th, R, rtol=1e-10, maxiter=400)
    L, gr = M.objective(p, A, X, R, th, cols, d, rho, s, T=T, mu=0.7)
    L0, _ = M.objective(p, A, X, R, th, cols, d, rho, s)
    assert L > L0  # the term is >= 0 and the learned step is not the near-exact one
    v = p.flat()
    h = 1e-6
    checked = 0
    for i in np.linspace(0, v.size - 1, 50).astype(int):
        vp, vm = v.copy(), v.copy()
        vp[i] += h
        vm[i] -= h
        lp = M.objective(M.Params.from_flat(vp, H=H), A, X, R, th, cols, d, rho, s, T=T, mu=0.7)[0]
        lm = M.objective(M.Params.from_flat(vm, H=H), A, X, R, th, cols, d, rho, s, T=T, mu=0.7)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gr[i]) <= 1e-6 * max(1e-3, abs(fd)), (i, fd, gr[i])
        checked += abs(fd) > 1e-6
    assert checked > 20


def test_supervision_sees_only_the_complement_of_the_block():
    # the target enters through (I - X X^T) t: parts of t inside span(X)
    # change nothing; mu = 0 is the unsupervised objective exactly
    H = 16
    A, X, th, R, d, rho, s = block_problem()
    p = small_net(H=H)
    cols = [1, 2]
    T = M.jd_targets(A, X, th, R, rtol=1e-10, maxiter=400)
    Tx = T + X @ np.random.default_rng(8).standard_normal((X.shape[1], T.shape[1]))
    La, ga = M.objective(p, A, X, R, th, cols, d, rho, s, T=T, mu=1.3)
    Lb, gb = M.objective(p, A, X, R, th, cols, d, rho, s, T=Tx, mu=1.3)
    assert abs(La - Lb) <= 1e-12 * abs(La)
    assert np.linalg.norm(ga - gb) <= 1e-10 * np.linalg.norm(ga)
    L0, g0 = M.objective(p, A, X, R, th, cols, d, rho, s)
    Lz, gz = M.objective(p, A, X, R, th, cols, d, rho, s, T=T, mu=0.0)
    assert Lz == L0 and np.array_equal(gz, g0)


def test_decrease_is_two_dimensional_rayleigh_ritz():
    # independent: Rayleigh-Ritz on an orthonormal basis of span{x_j, (I - X X^T) w}
    A, X, th, R, d, rho, s = block_problem(n=50, m=4, seed=9)
    g = synth.rng(4)
    for j in range(4):
        w = g.standard_normal(50)
        u = w - X @ (X.T @ w)
        Q = np.linalg.qr(np.column_stack([X[:, j], u]))[0]
        lam = np.linalg.eigvalsh(Q.T @ A @ Q)[0]
        D = M.decrease(A, X, X[:, j], R[:, j], th[j], w)
        assert abs(D - (th[j] - lam)) <= 1e-12 * np.abs(A).max()
        # Courant-Fischer: the step never raises the Ritz value and cannot go
        # below the smallest eigenvalue
        assert -1e-14 <= D <= th[j] - np.linalg.eigvalsh(A)[0] + 1e-12


def test_vanishing_regulariser_is_absolute_jacobi():
    # c -> 0 reduces the learned column to the guarded absolute Jacobi step,
    # computed by the independent LOBPCG oracle function
    A, X, th, R, d, rho, s = block_problem()
    p = small_net()
    p.W3[:] = 0.0
    p.b3[:] = -80.0
    d2 = d.copy()
    d2[3] = th[1]  # exercise the guard
    for j in range(3):
        w, _ = M.precondition(p, R[:, j], d2, th[j], rho, s)
        ref = O.precondition_diag(R[:, [j]], d2, th[[j]])[:, 0]
        assert np.allclose(w, ref, rtol=1e-12, atol=0)


def test_regulariser_closed_form():
    # with a constant output y the regulariser is c = s log(1 + e^y) inside
    # the window |d - theta| <= 16 rho and 0 outside it
    p = small_net()
    p.W3[:] = 0.0
    p.b3[:] = 0.7
    r = np.array([1.0, -2.0, 0.5, 3.0])
    d = np.array([2.0, 1.0, 1.5, 9.0])
    rho = np.array([0.1, 0.2, 0.3, 0.1])  # the last entry is outside (7.8 > 1.6)
    s = M.scale_of(d)
    w, aux = M.precondition(p, r, d, 1.2, rho, s)
    c = s * np.log1p(np.exp(0.7))
    ref = r / np.sqrt((d - 1.2) ** 2 + np.array([c, c, c, 0.0]) ** 2)
    assert np.allclose(w, ref, rtol=1e-14)
    assert list(aux["inside"]) == [True, True, True, False]


def test_activation_closed_forms():
    assert M.silu(np.array([0.0]))[0] == 0.0
    assert abs(M.silu(np.array([40.0]))[0] - 40.0) < 1e-12
    z = np.linspace(-5, 5, 21)
    h = 1e-6
    assert np.allclose(M.dsilu(z), (M.silu(z + h) - M.silu(z - h)) / (2 * h), atol=1e-8)
    assert np.allclose(M.sigmoid(z), 1 / (1 + np.exp(-z)), rtol=1e-14)
    assert abs(M.softplus(np.array([0.0]))[0] - np.log(2.0)) < 1e-15
    assert M.softplus(np.array([800.0]))[0] == 800.0


def test_adam_first_step_is_signed_lr():
    g = np.array([3.0, -0.5, 1e-3])
    th, m, v = M.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=1e-2)
    assert np.allclose(th, -1e-2 * np.sign(g), rtol=1e-4)


def test_param_count_and_roundtrip():
    p = M.init_params(3)
    assert p.flat().size == M.n_params() == 128 * 3 + 128 + 128 * 128 + 128 + 128 + 1
    q = M.Params.from_flat(p.flat())
    assert np.array_equal(q.flat(), p.flat())


def test_features_definition():
    d = np.array([2.0, 1.0, 1.5, 4.0])
    rho = np.array([0.5, 0.0, 1.0, 2.0])
    f = M.features(d, 1.0, rho, 2.0)
    assert np.allclose(f[:, 0], np.log(np.abs(d - 1.0) / 2.0 + 1e-6))
    assert np.allclose(f[:, 1], 0.5)
    assert np.allclose(f[:, 2], np.log(rho / 2.0 + 1e-6))


def test_jd_targets_solve_projected_system():
    # independent check: solve in an orthonormal basis Q of x-perp by a dense
    # factorisation and compare with the MINRES answer
    n = 60
    A = synth.dense_dd(n, seed=4)
    w, V = np.linalg.eigh(A)
    x = V[:, 0] + 1e-3 * synth.rng(2).standard_normal(n)
    x /= np.linalg.norm(x)
    th = x @ A @ x
    r = A @ x - th * x
    T = M.jd_targets(A, x[:, None], np.array([th]), r[:, None], rtol=1e-12, maxiter=2000)
    Q = np.linalg.qr(np.column_stack([x, synth.rng(3).standard_normal((n, n - 1))]))[0][:, 1:]
    t_ref = Q @ np.linalg.solve(Q.T @ (A - th * np.eye(n)) @ Q, -(Q.T @ r))
    assert abs(T[:, 0] @ x) < 1e-10
    assert np.allclose(T[:, 0], t_ref, atol=1e-7 * np.abs(t_ref).max())


def test_decrease_formula_has_no_cancellation():
    # Delta = sqrt(h^2 + b^2) - h: for b << h it is b^2 / (2h) to first order
    # (the smaller root of the 2 x 2 problem), never 0 for b != 0
    for h, b in [(1.0, 1e-9), (3.0, 1e-12), (1e3, 1e-5)]:
        D, S = M._delta(h, b)
        assert D > 0.0
        assert abs(D - b * b / (2 * h)) <= 1e-6 * b * b / (2 * h)
    for h, b in [(-2.0, 0.5), (0.3, 0.4), (0.0, 1.0)]:
        D, S = M._delta(h, b)
        lam = np.linalg.eigvalsh(np.array([[0.0, b], [b, 2 * h]]))[0]
        assert abs(D - (0.0 - lam)) <= 1e-14 * max(1.0, abs(lam))
