"""GPU parity of the learned preconditioner against its CPU fp64 oracle
(oracle/mlp_oracle.py), through the C ABI.

Bars: the learned column (fp32 MLP, fp64 epilogue) within 1e-4 relative of
the oracle per entry (the net runs in fp32: features and activations carry
about 1e-6 relative error, amplified at most by c^2 / q <= 1 in w); the
training loss within 1e-5 relative and its gradient within 1e-4 relative in
norm (fp32 products, fp64 accumulation across tiles); the MINRES corrections'
decreases within 1e-6 relative of scipy's MINRES on the same projected
systems solved to 1e-12.  Solves with the learned preconditioner are judged
on their eigenpairs, like any other preconditioner.
"""
import numpy as np
import pytest

import synth
from oracle import lobpcg_oracle as O
from oracle import mlp_oracle as M

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2305_06668_amd as P

    return P


def cu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def say(*a):
    print(*a, flush=True)


def f32_params(seed, out_bias=-1.0, w3_scale=10.0):
    """Oracle parameters rounded to fp32 (what the GPU holds)."""
    p = M.init_params(seed, out_bias=out_bias)
    p.W3 *= w3_scale
    w = p.flat().astype(np.float32)
    return w, M.Params.from_flat(w.astype(np.float64))


def family_problem(n=3000, idx=3, seed=11, m=6):
    C, _ = synth.csr_family(idx, n=n, band=400)
    A = O.csr_operator(C.row_ptr, C.col, C.val, n)
    import scipy.sparse as sp

    As = sp.csr_matrix((C.val, C.col, C.row_ptr), shape=(n, n))
    rho = np.asarray(abs(As).sum(1)).ravel() - np.abs(C.diag)
    # an orthonormal Ritz block after a few oracle iterations
    X0 = synth.start_block(n, m, seed)
    r = O.lobpcg(A, X0, m, 1e-8, diag=C.diag, max_iter=3)
    X = r.X_all
    return C, As, X, rho


def solver_for(P, C, block):
    s = P.Solver(C.n)
    s.set_operator_csr(cu(C.row_ptr), cu(C.col), cu(C.val))
    s.ensure_workspace(block)
    return s


def test_learned_apply_matches_oracle(P):
    C, As, X, rho = family_problem()
    n, m = X.shape
    d = C.diag
    s_ = M.scale_of(d)
    w32, p = f32_params(5)
    s = solver_for(P, C, m)
    s.set_learned_weights(w32)
    s.set_option(P.OPT_LEARNED_BF16, 0)
    g = synth.rng(7)
    R = g.standard_normal((n, m))
    theta = np.sort(d)[[0, 3, 10, 50, 200, 999]] + np.array([0.0, 1e-3, -2e-3, 0.1, 0.0, 5.0])
    theta[4] = d[17]  # an exact hit of a diagonal entry: the guard floor
    mask = np.array([0, 1, 0, 0, 1, 0], dtype=np.int32)
    Rd = cu(R)
    P.lobpcg_learned_apply(s.h, Rd, cu(theta), cu(mask))
    Wg = Rd.cpu().numpy()
    for j in range(m):
        if mask[j]:
            ref = O.precondition_diag(R[:, [j]], d, theta[[j]])[:, 0]
            assert np.allclose(Wg[:, j], ref, rtol=1e-14, atol=0), j
        else:
            ref, _ = M.precondition(p, R[:, j], d, theta[j], rho, s_)
            err = np.abs(Wg[:, j] - ref) / np.abs(ref)
            say(f"col {j}: max rel err {err.max():.2e}")
            assert err.max() <= 1e-4, j


def test_learned_apply_screened_tiles_match_oracle(P):
    """fp32 net where most 64-entry tiles have no entry inside the window
    |d - theta| <= 16 rho (d_i = i + 1, couplings 0.5, so rho <= 1): those
    tiles take the guarded Jacobi step in the kernel's screening pass, the
    others run the net; every column against the oracle's definition,
    n = 3001 (ragged last tile), one theta hitting a diagonal entry."""
    import scipy.sparse as sp

    n, m = 3001, 6
    d = np.arange(n, dtype=np.float64) + 1.0
    off = np.full(n - 1, 0.5)
    As = sp.diags([off, d, off], [-1, 0, 1], format="csr")
    rho = np.asarray(abs(As).sum(1)).ravel() - np.abs(d)
    C = synth.CSR(n=n, row_ptr=As.indptr.astype(np.int32), col=As.indices.astype(np.int32),
                  val=As.data.astype(np.float64), diag=d)
    theta = np.array([5.5, 100.0, 1500.25, 2990.0, 17.0, 700.0])  # 17.0 = d[16]
    inside = (np.abs(d[:, None] - theta[None, :]) <= 16 * rho[:, None]).ravel()
    act = [inside[t : t + 64].any() for t in range(0, inside.size, 64)]
    assert 0 < sum(act) < len(act) // 4  # both kinds of tiles, mostly screened out
    s_ = M.scale_of(d)
    w32, p = f32_params(5)
    s = solver_for(P, C, m)
    s.set_learned_weights(w32)
    s.set_option(P.OPT_LEARNED_BF16, 0)
    R = synth.rng(8).standard_normal((n, m))
    Rd = cu(R)
    P.lobpcg_learned_apply(s.h, Rd, cu(theta), cu(np.zeros(m, dtype=np.int32)))
    Wg = Rd.cpu().numpy()
    for j in range(m):
        ref, _ = M.precondition(p, R[:, j], d, theta[j], rho, s_)
        err = np.abs(Wg[:, j] - ref) / np.abs(ref)
        out = ~inside.reshape(n, m)[:, j]
        say(f"col {j}: max rel err {err.max():.2e}, outside the window {err[out].max():.2e}")
        assert err.max() <= 1e-4, j
        assert err[out].max() <= 1e-14, j  # the Jacobi step: fp64 on both sides


@pytest.mark.parametrize("n", [3000, 1777])
def test_learned_apply_bf16_matches_oracle(P, n):
    # the solver's inference path: layer 2 on bf16 MFMA.  bf16 rounding of
    # h1 and W2 (2^-9 relative) moves y by O(1e-3 |y|); w moves by at most the
    # relative change of c, so entries agree to 3e-2 and typically to 1e-3
    C, As, X, rho = family_problem(n=n)
    d = C.diag
    m = 5
    w32, p = f32_params(5)
    s = solver_for(P, C, 6)
    s.set_learned_weights(w32)
    R = synth.rng(17).standard_normal((n, m))
    theta = np.sort(d)[[0, 2, 9, 40, 300]] + np.array([0.0, 1e-3, -2e-3, 0.1, 0.0])
    Rd = cu(R)
    P.lobpcg_learned_apply(s.h, Rd, cu(theta))
    Wg = Rd.cpu().numpy()
    errs = []
    for j in range(m):
        ref, _ = M.precondition(p, R[:, j], d, theta[j], rho, M.scale_of(d))
        errs.append(np.abs(Wg[:, j] - ref) / np.abs(ref))
    errs = np.concatenate(errs)
    say(f"bf16 apply: max rel err {errs.max():.2e}, median {np.median(errs):.2e}")
    assert errs.max() <= 3e-2
    assert np.median(errs) <= 2e-3


@pytest.mark.parametrize("bf16", [0, 1])
def test_learned_apply_nonfinite_weights_fall_back(P, bf16):
    # NaN weights: every entry takes the guarded Jacobi step (the bf16 path
    # forms the fallback denominator in fp32)
    C, As, X, rho = family_problem(n=1200)
    n, m = X.shape
    w32, _ = f32_params(5)
    w32[M.n_params() - 1] = np.nan
    s = solver_for(P, C, m)
    s.set_learned_weights(w32)
    s.set_option(P.OPT_LEARNED_BF16, bf16)
    R = synth.rng(8).standard_normal((n, 4))
    theta = np.sort(C.diag)[:4] + 1e-3
    Rd = cu(R)
    P.lobpcg_learned_apply(s.h, Rd, cu(theta))
    ref = O.precondition_diag(R, C.diag, theta)
    assert np.allclose(Rd.cpu().numpy(), ref, rtol=1e-14 if bf16 == 0 else 1e-6, atol=0)


@pytest.mark.parametrize("n", [3000, 20011])
def test_learner_objective_and_gradient_match_oracle(P, n):
    """n = 3000: one 64-entry tile per workgroup; n = 20011: 938 tiles over
    the 256 workgroups (several per workgroup, fp64 sums across them) and a
    ragged last tile of one entry."""
    C, As, X, rho = family_problem(n=n)
    n, m = X.shape
    s = solver_for(P, C, m)
    L = P.lobpcg_learner_create(0, 3)
    try:
        w32, p = f32_params(9)
        P.lobpcg_learner_set_weights(L, w32)
        snap = P.lobpcg_learner_add_snapshot(L, s.h, cu(X), minres_maxiter=50, minres_rtol=1e-6)
        info = P.lobpcg_learner_snapshot_info(L, snap, m)
        th = np.einsum("ij,ij->j", X, As @ X)
        assert np.allclose(info["theta"], th, rtol=1e-13)
        # the oracle takes the snapshot's own theta (a sum over n terms whose
        # order differs from numpy's by ~1e-14 relative): the Jacobi step
        # r / (d - theta) amplifies that ~1e5-fold in Delta where some
        # |d_i - theta| ~ 1e-5
        th = np.asarray(info["theta"], dtype=np.float64)
        R = As @ X - X * th
        assert np.allclose(info["resnorm"], np.linalg.norm(R, axis=0), rtol=1e-10)
        cols = [0, 2, 5]
        out = P.lobpcg_learner_objective(L, snap, cols, want_grad=True, want_decreases=True)
        ref = info["ref_decrease"][cols]
        Lo, go = M.objective(p, As, X, R, th, cols, C.diag, rho, M.scale_of(C.diag), ref=ref)
        gg = out["grad"]
        rel_l = abs(out["loss"] - Lo) / abs(Lo)
        rel_g = np.linalg.norm(gg - go) / np.linalg.norm(go)
        say(f"loss gpu {out['loss']:.10f} oracle {Lo:.10f} rel {rel_l:.2e}; grad rel {rel_g:.2e}")
        assert rel_l <= 1e-5
        assert rel_g <= 1e-4
        # per-block agreement (every layer's gradient, not only the dominant one)
        gp, op = M.Params.from_flat(gg), M.Params.from_flat(go)
        for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
            a, b = getattr(gp, name), getattr(op, name)
            assert np.linalg.norm(a - b) <= 1e-3 * np.linalg.norm(b) + 1e-12 * np.linalg.norm(go), name
        # decreases: learned and Jacobi, against the oracle's definition
        for k, j in enumerate(cols):
            w, _ = M.precondition(p, R[:, j], C.diag, th[j], rho, M.scale_of(C.diag))
            Dl = M.decrease(As, X, X[:, j], R[:, j], th[j], w)
            wj = O.precondition_diag(R[:, [j]], C.diag, th[[j]])[:, 0]
            Dj = M.decrease(As, X, X[:, j], R[:, j], th[j], wj)
            assert abs(out["learned_decrease"][k] - Dl) <= 1e-4 * Dl
            assert abs(out["jacobi_decrease"][k] - Dj) <= 1e-9 * Dj
    finally:
        P.lobpcg_learner_destroy(L)


def test_learner_gradient_screened_tiles_match_oracle(P):
    """Loss and gradient where 139 of 141 tiles have no entry inside the
    net's window (tridiagonal, d_i = i + 1, couplings 0.5, a block near the
    lowest eigenvectors): the gradient kernel skips those tiles, whose dL/dy
    is zero by definition; every layer against the oracle."""
    import scipy.linalg as sl
    import scipy.sparse as sp

    n, m = 3001, 4
    d = np.arange(n, dtype=np.float64) + 1.0
    off = np.full(n - 1, 0.5)
    As = sp.diags([off, d, off], [-1, 0, 1], format="csr")
    rho = np.asarray(abs(As).sum(1)).ravel() - np.abs(d)
    C = synth.CSR(n=n, row_ptr=As.indptr.astype(np.int32), col=As.indices.astype(np.int32),
                  val=As.data.astype(np.float64), diag=d)
    V = sl.eigh_tridiagonal(d, off, select="i", select_range=(0, m - 1))[1]
    Xb = np.linalg.qr(V + 1e-3 * synth.rng(13).standard_normal((n, m)))[0]
    X = Xb @ np.linalg.eigh(Xb.T @ (As @ Xb))[1]
    s = solver_for(P, C, m)
    L = P.lobpcg_learner_create(0, 3)
    try:
        w32, p = f32_params(9)
        P.lobpcg_learner_set_weights(L, w32)
        snap = P.lobpcg_learner_add_snapshot(L, s.h, cu(X), minres_maxiter=50, minres_rtol=1e-6)
        info = P.lobpcg_learner_snapshot_info(L, snap, m)
        th = np.asarray(info["theta"], dtype=np.float64)
        R = As @ X - X * th
        cols = [0, 1, 3]
        inside = (np.abs(d[:, None] - th[None, cols]) <= 16 * rho[:, None]).ravel()
        act = [inside[t : t + 64].any() for t in range(0, inside.size, 64)]
        assert 0 < sum(act) <= 4 and len(act) == 141
        out = P.lobpcg_learner_objective(L, snap, cols, want_grad=True)
        Lo, go = M.objective(p, As, X, R, th, cols, d, rho, M.scale_of(d), ref=info["ref_decrease"][cols])
        rel_l = abs(out["loss"] - Lo) / abs(Lo)
        rel_g = np.linalg.norm(out["grad"] - go) / np.linalg.norm(go)
        say(f"active tiles {sum(act)} of {len(act)}: loss rel {rel_l:.2e}, grad rel {rel_g:.2e}")
        assert rel_l <= 1e-5
        assert rel_g <= 1e-4
        gp, op = M.Params.from_flat(out["grad"]), M.Params.from_flat(go)
        for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
            a, b = getattr(gp, name), getattr(op, name)
            assert np.linalg.norm(b) > 0, name
            assert np.linalg.norm(a - b) <= 1e-3 * np.linalg.norm(b), name
    finally:
        P.lobpcg_learner_destroy(L)


def test_learner_supervised_objective_matches_oracle(P):
    """The loss with the supervised term mu (1 - cos^2 angle(u, (I - X X^T) t))
    and its gradient against the oracle, the corrections t solved tightly on
    both sides (GPU block MINRES to 1e-10, scipy's MINRES to 1e-12) on a
    block near the lowest eigenvectors, where the projected systems are well
    enough conditioned for that."""
    n, m = 500, 4
    A = synth.dense_dd(n, seed=12)
    V = np.linalg.eigh(A)[1]
    Xb = np.linalg.qr(V[:, :m] + 1e-2 * synth.rng(13).standard_normal((n, m)))[0]
    X = Xb @ np.linalg.eigh(Xb.T @ A @ Xb)[1]
    d = np.diag(A).copy()
    rho = np.abs(A).sum(1) - np.abs(d)
    s = P.Solver(n)
    s.set_operator_dense(cu(A))
    s.ensure_workspace(m)
    L = P.lobpcg_learner_create(0, 3)
    try:
        w32, p = f32_params(9)
        P.lobpcg_learner_set_weights(L, w32)
        snap = P.lobpcg_learner_add_snapshot(L, s.h, cu(X), minres_maxiter=600, minres_rtol=1e-10)
        info = P.lobpcg_learner_snapshot_info(L, snap, m)
        assert np.all(info["minres_relres"] <= 1e-10)
        th = np.einsum("ij,ij->j", X, A @ X)
        R = A @ X - X * th
        T = M.jd_targets(A, X, th, R, rtol=1e-12, maxiter=2000)
        cols = [0, 1, 3]
        ref = info["ref_decrease"][cols]
        base = P.lobpcg_learner_objective(L, snap, cols, want_grad=True)
        Lb, _ = M.objective(p, A, X, R, th, cols, d, rho, M.scale_of(d), ref=ref)
        assert abs(base["loss"] - Lb) <= 1e-5 * abs(Lb)
        for mu in (0.8, 3.0):
            P.lobpcg_learner_set_supervision(L, mu)
            out = P.lobpcg_learner_objective(L, snap, cols, want_grad=True)
            Lo, go = M.objective(p, A, X, R, th, cols, d, rho, M.scale_of(d), ref=ref, T=T, mu=mu)
            rel_l = abs(out["loss"] - Lo) / abs(Lo)
            rel_g = np.linalg.norm(out["grad"] - go) / np.linalg.norm(go)
            say(f"mu {mu}: loss gpu {out['loss']:.10f} oracle {Lo:.10f} rel {rel_l:.2e}; grad rel {rel_g:.2e}")
            assert rel_l <= 1e-5
            assert rel_g <= 1e-4
            assert out["loss"] > base["loss"]  # the term is positive here
        P.lobpcg_learner_set_supervision(L, 0.0)
        off = P.lobpcg_learner_objective(L, snap, cols, want_grad=True)
        assert off["loss"] == base["loss"] and np.array_equal(off["grad"], base["grad"])
        with pytest.raises(P.LobpcgError):
            P.lobpcg_learner_set_supervision(L, -1.0)
    finally:
        P.lobpcg_learner_destroy(L)


def test_minres_corrections_match_oracle(P):
    # a Ritz block near the lowest eigenvectors: the projected systems are
    # then well enough conditioned for MINRES to reach 1e-10 in a few hundred
    # steps (from a random block theta sits mid-spectrum and it needs > 700)
    n, m = 500, 4
    A = synth.dense_dd(n, seed=12)
    V = np.linalg.eigh(A)[1]
    Xb = np.linalg.qr(V[:, :m] + 1e-2 * synth.rng(13).standard_normal((n, m)))[0]
    th0, U = np.linalg.eigh(Xb.T @ A @ Xb)
    X = Xb @ U
    s = P.Solver(n)
    s.set_operator_dense(cu(A))
    s.ensure_workspace(m)
    L = P.lobpcg_learner_create(0, 1)
    try:
        snap = P.lobpcg_learner_add_snapshot(L, s.h, cu(X), minres_maxiter=600, minres_rtol=1e-10)
        info = P.lobpcg_learner_snapshot_info(L, snap, m)
        th = np.einsum("ij,ij->j", X, A @ X)
        R = A @ X - X * th
        T = M.jd_targets(A, X, th, R, rtol=1e-12, maxiter=2000)
        say("minres relres", info["minres_relres"])
        assert np.all(info["minres_relres"] <= 1e-10)
        for j in range(m):
            D = M.decrease(A, X, X[:, j], R[:, j], th[j], T[:, j])
            assert abs(info["ref_decrease"][j] - D) <= 1e-6 * D, (j, info["ref_decrease"][j], D)
    finally:
        P.lobpcg_learner_destroy(L)


def test_training_lowers_loss(P):
    C, As, X, rho = family_problem(n=4000, m=8)
    s = solver_for(P, C, 8)
    L = P.lobpcg_learner_create(0, 4)
    try:
        for it in (2, 6):
            Xs = O.lobpcg(O.csr_operator(C.row_ptr, C.col, C.val, C.n), synth.start_block(C.n, 8, it), 8, 1e-8,
                          diag=C.diag, max_iter=it).X_all
            P.lobpcg_learner_add_snapshot(L, s.h, cu(Xs), minres_maxiter=60)
        first, last = P.lobpcg_learner_train(L, 120, 4, 3e-3, seed=2)
        say(f"training loss {first:.4f} -> {last:.4f}")
        assert np.isfinite(first) and np.isfinite(last)
        assert last < first
        # with the supervised term as well
        P.lobpcg_learner_set_supervision(L, 1.0)
        first, last = P.lobpcg_learner_train(L, 120, 4, 3e-3, seed=3)
        say(f"supervised training loss {first:.4f} -> {last:.4f}")
        assert np.isfinite(first) and np.isfinite(last)
        assert last < first
    finally:
        P.lobpcg_learner_destroy(L)


def test_training_and_learned_solve_on_a_caller_stream(P):
    """Snapshot collection, training and a learned mixed-precision solve
    whose solver handles were created under a caller's stream (default
    priority) give the default stream's weights and bits."""
    C, As, X, rho = family_problem(n=4000, m=8)
    op = O.csr_operator(C.row_ptr, C.col, C.val, C.n)
    Xs = O.lobpcg(op, synth.start_block(C.n, 8, 2), 8, 1e-8, diag=C.diag, max_iter=2).X_all
    X0 = synth.start_block(C.n, 8, 5)

    def run():
        s = solver_for(P, C, 8)
        L = P.lobpcg_learner_create(0, 4)
        try:
            P.lobpcg_learner_add_snapshot(L, s.h, cu(Xs), minres_maxiter=60)
            first, last = P.lobpcg_learner_train(L, 40, 4, 3e-3, seed=2)
            w = P.lobpcg_learner_get_weights(L)
        finally:
            P.lobpcg_learner_destroy(L)
        s.set_learned_weights(w)
        s.set_preconditioner(P.PRECOND_LEARNED)
        s.set_option(P.OPT_PRECISION, P.PREC_FP32)
        s.set_initial_guess(cu(X0))
        res = s.solve(8, 1e-8)
        return first, last, w, res.status, res.evals, res.evecs.cpu().numpy(), res.stats["iterations"]

    a = run()
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        b = run()
    torch.cuda.synchronize()
    say("caller stream: loss", a[0], "->", a[1], "status", a[3], "iterations", a[6])
    assert np.isfinite(a[0]) and np.isfinite(a[1])
    assert a[0] == b[0] and a[1] == b[1]
    assert np.array_equal(a[2], b[2])
    assert a[3] == b[3] and a[6] == b[6]
    assert np.array_equal(a[4], b[4])
    assert np.array_equal(a[5], b[5])


def _eig_ref(A, k):
    w, V = np.linalg.eigh(A)
    return w, V[:, :k]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_learned_solve_eigenpairs(P, precision):
    n, k = 1500, 6
    A = synth.dense_dd(n, seed=21)
    w_all, V = _eig_ref(A, k)
    X0 = synth.start_block(n, k, 22)
    w32, _ = f32_params(3, out_bias=-2.0, w3_scale=1.0)
    s = P.Solver(n)
    s.set_operator_dense(cu(A))
    s.set_learned_weights(w32)
    s.set_preconditioner(P.PRECOND_LEARNED)
    if precision == "mixed":
        s.set_option(P.OPT_PRECISION, P.PREC_FP32)
    s.set_initial_guess(cu(X0))
    res = s.solve(k, 1e-8)
    say(precision, res.stats["iterations"], res.stats["learned_fallbacks"], res.resnorms.max())
    assert res.status == 0
    X = res.evecs.cpu().numpy()
    AX = A @ X
    th = np.einsum("ij,ij->j", X, AX)
    assert np.all(np.linalg.norm(AX - X * th, axis=0) <= 1e-8 * 1.0001)
    assert np.all(np.abs(res.evals - w_all[:k]) <= 1e-9 * np.maximum(np.abs(w_all[:k]), 1e-3 * 101))
    assert np.abs(X.T @ X - np.eye(k)).max() < 1e-12


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_learned_budget_switches_to_jacobi(P, precision):
    """LOBPCG_OPT_LEARNED_BUDGET: after that many iterations every column
    takes the Jacobi step; the solve still meets the eigenpair bar, and with
    the budget at 0 (no limit) or above the iteration count nothing switches."""
    n, k = 1500, 6
    A = synth.dense_dd(n, seed=21)
    w_all, _ = _eig_ref(A, k)
    X0 = synth.start_block(n, k, 22)
    w32, _ = f32_params(3, out_bias=-2.0, w3_scale=1.0)
    s = P.Solver(n)
    s.set_operator_dense(cu(A))
    s.set_learned_weights(w32)
    s.set_preconditioner(P.PRECOND_LEARNED)
    if precision == "mixed":
        s.set_option(P.OPT_PRECISION, P.PREC_FP32)
    out = {}
    for budget in (0, 3, 10000):
        s.set_option(P.OPT_LEARNED_BUDGET, budget)
        s.set_initial_guess(cu(X0))
        res = s.solve(k, 1e-8)
        say(precision, "budget", budget, res.stats["iterations"], "switch", res.stats["learned_budget_iter"])
        assert res.status == 0
        X = res.evecs.cpu().numpy()
        AX = A @ X
        th = np.einsum("ij,ij->j", X, AX)
        assert np.all(np.linalg.norm(AX - X * th, axis=0) <= 1e-8 * 1.0001)
        assert np.all(np.abs(res.evals - w_all[:k]) <= 1e-9 * np.maximum(np.abs(w_all[:k]), 1e-3 * 101))
        out[budget] = res.stats
    assert out[0]["learned_budget_iter"] == -1
    assert out[10000]["learned_budget_iter"] == -1
    assert out[3]["learned_budget_iter"] == 4
    # budget 0 and a budget above the iteration count are the same solve
    assert out[0]["iterations"] == out[10000]["iterations"]
    with pytest.raises(P.LobpcgError):
        s.set_option(P.OPT_LEARNED_BUDGET, -1)


def test_learned_solve_with_nan_weights_still_converges(P):
    # diagonal slope 1e-3: gaps wide enough that the Jacobi-preconditioned
    # solve converges in tens of iterations (with the default slope at this n
    # the lowest pairs sit inside the U(0, 0.1) noise and take hundreds)
    n, k = 1200, 4
    C = synth.csr_banded(n=n, band=200, seed=31, diag_slope=1e-3)
    X0 = synth.start_block(n, k, 32)
    w32, _ = f32_params(3)
    w32[:] = np.nan
    s = P.Solver(n)
    s.set_operator_csr(cu(C.row_ptr), cu(C.col), cu(C.val))
    s.set_learned_weights(w32)
    s.set_preconditioner(P.PRECOND_LEARNED)
    s.set_initial_guess(cu(X0))
    res = s.solve(k, 1e-8)
    say("nan weights:", res.stats["iterations"], res.stats["learned_nonfinite"])
    assert res.status == 0
    assert res.stats["learned_nonfinite"] > 0
    op = O.csr_operator(C.row_ptr, C.col, C.val, n)
    ref = O.lobpcg(op, X0, k, 1e-8, diag=C.diag)
    assert np.all(np.abs(res.evals - ref.evals) <= 1e-9 * np.abs(ref.evals))
