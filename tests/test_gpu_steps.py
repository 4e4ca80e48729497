"""GPU parity of the individual steps (through the C ABI) against the CPU
oracle or against the plain mathematical definition of the step.

Tolerances: every step here is fp64.  A product or overlap over n rows is
compared entry-wise within 1e-13 of the scale sum_k |a_ik| |b_kj| (the
standard forward error bound ~ n eps times that scale, with the tree
reduction's log2(n) factor well inside it for the sizes used); small dense
results within 1e-12 of their norm.
"""
import math

import numpy as np
import pytest

import synth
from oracle import lobpcg_oracle as O

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


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def say(*a):
    print(*a, flush=True)


def make_solver(P, n, block=8):
    s = P.Solver(n)
    s.ensure_workspace(block)
    return s


@pytest.mark.parametrize("n,p,q", [(1000, 1, 1), (4097, 5, 17), (100003, 48, 48), (20011, 96, 32), (7, 3, 2), (333, 128, 128)])
def test_gram(P, n, p, q):
    say("gram", n, p, q)
    g = synth.rng(n + p + q)
    A = g.standard_normal((n, p))
    B = g.standard_normal((n, q))
    s = make_solver(P, max(n, 24))
    # operate on the handle's n: pad to the handle size if needed
    nn = s.n
    Ap = np.zeros((nn, p)); Ap[:n] = A
    Bp = np.zeros((nn, q)); Bp[:n] = B
    C = torch.zeros((p, q), dtype=torch.float64, device="cuda")
    P.lobpcg_gram(s.h, cu(Ap), cu(Bp), C)
    ref = A.T @ B
    scale = np.abs(A).T @ np.abs(B)
    assert np.all(np.abs(host(C) - ref) <= 1e-13 * scale + 1e-300)


def test_gram_strided_views(P):
    n = 5003
    g = synth.rng(3)
    Vb = g.standard_normal((n, 40))
    s = make_solver(P, n)
    V = cu(Vb)
    C = torch.zeros((30, 10), dtype=torch.float64, device="cuda")
    P.lobpcg_gram(s.h, V[:, :30], V[:, 30:], C)
    ref = Vb[:, :30].T @ Vb[:, 30:]
    assert np.allclose(host(C), ref, rtol=0, atol=1e-11)


def test_gram_deterministic(P):
    n = 65537
    g = synth.rng(9)
    A = cu(g.standard_normal((n, 24)))
    s = make_solver(P, n)
    C1 = torch.zeros((24, 24), dtype=torch.float64, device="cuda")
    C2 = torch.zeros_like(C1)
    P.lobpcg_gram(s.h, A, A, C1)
    P.lobpcg_gram(s.h, A, A, C2)
    assert torch.equal(C1, C2)


@pytest.mark.parametrize("m", [1, 3, 4, 8, 9, 12, 16, 17, 32, 40])
def test_apply_csr(P, m):
    say("apply_csr", m)
    n = 30011
    C = synth.csr_banded(n=n, seed=5, band=700, diag_slope=1e-3)
    S = C.to_scipy()
    W = synth.start_block(n, m, 7)
    s = P.Solver(n)
    s.set_operator_csr(cu(C.row_ptr), cu(C.col), cu(C.val))
    s.ensure_workspace(1)
    Y = torch.zeros((n, m), dtype=torch.float64, device="cuda")
    P.lobpcg_apply_operator(s.h, cu(W), Y)
    ref = S @ W
    scale = abs(S) @ np.abs(W)
    assert np.all(np.abs(host(Y) - ref) <= 1e-14 * scale + 1e-300)


def test_apply_csr_strided_and_empty_rows(P):
    n = 4099
    A = np.zeros((n, n))
    idx = np.arange(0, n, 3)
    A[idx, idx] = 1.0 + idx
    A[idx[:-1], idx[1:]] = 0.5
    A[idx[1:], idx[:-1]] = 0.5
    C = synth.csr_from_dense(A)
    # rows with only an explicit zero diagonal exist (csr_from_dense keeps them)
    s = P.Solver(n)
    s.set_operator_csr(cu(C.row_ptr), cu(C.col), cu(C.val))
    s.ensure_workspace(1)
    Wb = synth.start_block(n, 12, 1)
    W = cu(Wb)
    Y = torch.zeros((n, 20), dtype=torch.float64, device="cuda")
    P.lobpcg_apply_operator(s.h, W[:, 2:9], Y[:, 5:12])
    out = host(Y)
    assert np.allclose(out[:, 5:12], A @ Wb[:, 2:9], atol=1e-13)
    assert np.all(out[:, :5] == 0) and np.all(out[:, 12:] == 0)


def _heavy_csr(n, seed):
    """Banded CSR (~41 stored entries per row, band +-700) plus four rows of
    1500-3100 entries: a 64-row block then holds more entries than one LDS
    pass of the vector kernel takes, and a pass boundary falls inside a row."""
    import scipy.sparse as sp

    C = synth.csr_banded(n=n, seed=seed, band=700, diag_slope=1e-3)
    g = np.random.default_rng(seed)
    rows, cols = [], []
    for r, cnt in ((100, 3100), (101, 1500), (4000, 2200), (n - 1, 1800)):
        c = np.unique(g.integers(0, n, size=cnt))
        rows.append(np.full(c.size, r))
        cols.append(c)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    H = sp.csr_matrix((g.uniform(-1e-3, 1e-3, rows.size), (rows, cols)), shape=(n, n))
    S = (C.to_scipy() + H).tocsr()
    S.sort_indices()
    return S


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize(
    "m,ldw,q",
    [
        (16, 16, 0),  # 16-byte loads: 8 (fp64) / 4 (fp32) lanes per row
        (16, 48, 32),  # the solver's layout: W at column 32 of a 48-wide basis
        (16, 48, 17),  # misaligned start: one column per lane
        (15, 48, 18),  # 16-byte loads with a partial last lane (fp64)
        (6, 8, 2),  # fp64: 3 lanes in a group of 4; fp32: narrow kernel
        (12, 12, 0),
        (9, 10, 0),  # fp64: 5 lanes; fp32: ldw not a multiple of 4
        (24, 24, 0),
        (32, 40, 8),  # fp64: 16 lanes per row; fp32: 8
        (40, 40, 0),  # fp64: 32 + 8 columns (two launches); fp32: 10 lanes
        (64, 64, 0),  # fp64: two launches of 32; fp32: 16 lanes
    ],
)
def test_apply_csr_paths(P, prec, m, ldw, q):
    """Both CSR kernels (16-byte loads from LDS-staged (col, val), and one
    column per lane) in fp64 and fp32 against the definition, entry by entry,
    within the summation bound (row length + 2) u sum_j |a_ij| |w_j|."""
    say("csr paths", prec, m, ldw, q)
    n = 20011
    S = _heavy_csr(n, 11)
    s = P.Solver(n)
    s.set_operator_csr(
        cu(S.indptr.astype(np.int32)), cu(S.indices.astype(np.int32)), cu(S.data.astype(np.float64))
    )
    f32 = prec == "f32"
    if f32:
        s.set_option(P.OPT_PRECISION, P.PREC_FP32)
    s.ensure_workspace(1)
    ldy = ldw + 3
    Wb = synth.start_block(n, ldw, 3)
    dt = torch.float32 if f32 else torch.float64
    Wd = torch.from_numpy(Wb).to(dt).cuda()
    Y = torch.full((n, ldy), 5.0, dtype=dt, device="cuda")
    (P.lobpcg_apply_operator_f32 if f32 else P.lobpcg_apply_operator)(s.h, Wd[:, q : q + m], Y[:, q : q + m])
    Yh = Y.cpu().numpy().astype(np.float64)
    if f32:
        Sv = S.copy()
        Sv.data = S.data.astype(np.float32).astype(np.float64)
        Wv = Wb.astype(np.float32).astype(np.float64)[:, q : q + m]
        u = 2.0**-24
    else:
        Sv, Wv, u = S, Wb[:, q : q + m], 2.0**-53
    ref = Sv @ Wv
    scale = abs(Sv) @ np.abs(Wv)
    lens = np.diff(S.indptr)[:, None]
    assert np.all(np.abs(Yh[:, q : q + m] - ref) <= (lens + 2) * u * scale + 1e-300)
    assert np.all(Yh[:, :q] == 5.0) and np.all(Yh[:, q + m :] == 5.0)  # other columns untouched
    s.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("m,ldw,q", [(16, 16, 0), (12, 40, 5), (3, 3, 0), (20, 24, 2)])
def test_apply_csr_banded_path(P, prec, m, ldw, q):
    """The opt-in banded path (LOBPCG_OPT_SPMM_SLAB = 1: W staged in LDS in
    slabs over each 2048-row block's column window) against the definition
    within the summation bound, on the heavy-row banded matrix: 20011 rows
    (ten blocks, a ragged last one), rows whose columns span the whole
    matrix (every slab), widths below 16, a 16-column slice plus a 4-column
    one, strided W and Y.  A matrix with unsorted columns takes the gather
    kernels under the same option, with the same result."""
    say("csr banded path", prec, m, ldw, q)
    n = 20011
    S = _heavy_csr(n, 11)
    f32 = prec == "f32"
    dt = torch.float32 if f32 else torch.float64
    Wb = synth.start_block(n, ldw, 3)
    if f32:
        Sv = S.copy()
        Sv.data = S.data.astype(np.float32).astype(np.float64)
        Wv = Wb.astype(np.float32).astype(np.float64)[:, q : q + m]
        u = 2.0**-24
    else:
        Sv, Wv, u = S, Wb[:, q : q + m], 2.0**-53
    ref = Sv @ Wv
    bound = (np.diff(S.indptr)[:, None] + 2) * u * (abs(Sv) @ np.abs(Wv)) + 1e-300
    # the same matrix with each row's columns reversed: not sorted
    Su = S.copy()
    for r in range(n):
        a, z = Su.indptr[r], Su.indptr[r + 1]
        Su.indices[a:z] = Su.indices[a:z][::-1].copy()
        Su.data[a:z] = Su.data[a:z][::-1].copy()
    for M in (S, Su):
        s = P.Solver(n)
        s.set_operator_csr(
            cu(M.indptr.astype(np.int32)), cu(M.indices.astype(np.int32)), cu(M.data.astype(np.float64))
        )
        if f32:
            s.set_option(P.OPT_PRECISION, P.PREC_FP32)
        s.ensure_workspace(1)
        s.set_option(P.OPT_SPMM_SLAB, 1)
        Wd = torch.from_numpy(Wb).to(dt).cuda()
        Y = torch.full((n, ldw + 3), 5.0, dtype=dt, device="cuda")
        (P.lobpcg_apply_operator_f32 if f32 else P.lobpcg_apply_operator)(s.h, Wd[:, q : q + m], Y[:, q : q + m])
        Yh = Y.cpu().numpy().astype(np.float64)
        assert np.all(np.abs(Yh[:, q : q + m] - ref) <= bound)
        assert np.all(Yh[:, :q] == 5.0) and np.all(Yh[:, q + m :] == 5.0)
        s.close()
    with pytest.raises(P.LobpcgError):
        P.Solver(n).set_option(P.OPT_SPMM_SLAB, 2)


def test_apply_csr_f32_needs_fp32_layout(P):
    n = 1000
    C = synth.csr_banded(n=n, seed=2, band=50)
    s = P.Solver(n)
    s.set_operator_csr(cu(C.row_ptr), cu(C.col), cu(C.val))
    s.ensure_workspace(1)
    W = torch.zeros((n, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(P.LobpcgError):
        P.lobpcg_apply_operator_f32(s.h, W, W.clone())
    s.close()


@pytest.mark.parametrize(
    "n,m,ldw",
    [
        (777, 1, 1),  # odd sizes: value-by-value kernel
        (2000, 4, 4),  # 16-byte vector kernel, 4 columns, ragged column tail
        (1031, 8, 8),
        (515, 11, 11),
        (1030, 8, 8),  # vector kernel, 8 columns, ragged row group and tail
        (1030, 6, 10),  # vector kernel on a strided block
        (2050, 12, 12),  # two launches (8 + 4 columns), both vector
        (1030, 5, 6),  # even but too narrow for whole-row W vectors
    ],
)
def test_apply_dense(P, n, m, ldw):
    say("dense", n, m, ldw)
    A = synth.dense_dd(n, seed=n)
    W = synth.start_block(n, ldw, 2)
    s = P.Solver(n)
    s.set_operator_dense(cu(A))
    s.ensure_workspace(1)
    Wd = cu(W)
    Y = torch.full((n, ldw), 5.0, dtype=torch.float64, device="cuda")
    P.lobpcg_apply_operator(s.h, Wd[:, :m], Y[:, :m])
    ref = A @ W[:, :m]
    scale = np.abs(A) @ np.abs(W[:, :m])
    Yh = host(Y)
    assert np.all(np.abs(Yh[:, :m] - ref) <= 1e-13 * scale)
    assert np.all(Yh[:, m:] == 5.0)


@pytest.mark.parametrize("na,m,ldw", [(19, 5, 5), (64, 8, 8), (45, 13, 16), (96, 17, 20)])
def test_apply_kronsum(P, na, m, ldw):
    # tiles of 32 x 32 x 8 with ragged i/j/column edges and strided blocks
    say("kronsum", na, m, ldw)
    A, V = synth.kronsum(na=na, seed=4)
    W = synth.start_block(na * na, ldw, 1)
    s = P.Solver(na * na)
    s.set_operator_kronsum(cu(A), cu(V))
    s.ensure_workspace(1)
    Wd = cu(W)
    Y = torch.full((na * na, ldw), 7.0, dtype=torch.float64, device="cuda")
    P.lobpcg_apply_operator(s.h, Wd[:, :m], Y[:, :m])
    H = np.kron(A, np.eye(na)) + np.kron(np.eye(na), A) + np.diag(V.reshape(-1))
    ref = H @ W[:, :m]
    scale = np.abs(H) @ np.abs(W[:, :m])
    Yh = host(Y)
    assert np.all(np.abs(Yh[:, :m] - ref) <= 1e-13 * scale + 1e-300)
    assert np.all(Yh[:, m:] == 7.0)  # columns past ncols untouched


@pytest.mark.parametrize("p", [2, 7, 24, 48, 96])
def test_small_eigh(P, p):
    say("small_eigh", p)
    a = synth.random_symmetric(p, p) + 3.0 * np.diag(np.arange(p))
    a[0, 1] += 1e-9  # not exactly symmetric: the kernel symmetrises
    s = make_solver(P, 300)
    ev = torch.zeros(p, dtype=torch.float64, device="cuda")
    U = torch.zeros((p, p), dtype=torch.float64, device="cuda")
    P.lobpcg_small_eigh(s.h, cu(a), ev, U)
    lam, Uh = host(ev), host(U)
    asym = 0.5 * (a + a.T)
    ref = np.linalg.eigvalsh(asym)
    nrm = np.linalg.norm(asym, 2)
    assert np.all(np.abs(lam - ref) <= 1e-13 * nrm)
    assert np.all(np.diff(lam) >= 0)
    assert np.abs(Uh.T @ Uh - np.eye(p)).max() <= 1e-13
    assert np.abs(asym @ Uh - Uh * lam).max() <= 1e-13 * nrm


def test_small_eigh_degenerate(P):
    p = 12
    lam = np.array([1.0, 1.0, 1.0, 2.0, 2.0] + list(np.linspace(3, 9, p - 5)))
    a, _ = synth.prescribed_spectrum(lam, 3)
    s = make_solver(P, 300)
    ev = torch.zeros(p, dtype=torch.float64, device="cuda")
    U = torch.zeros((p, p), dtype=torch.float64, device="cuda")
    P.lobpcg_small_eigh(s.h, cu(a), ev, U)
    assert np.allclose(host(ev), lam, atol=1e-13 * 9)
    Uh = host(U)
    assert np.abs(Uh.T @ Uh - np.eye(p)).max() <= 1e-13


def test_small_cholesky(P):
    g = synth.rng(1)
    G = g.standard_normal((50, 20))
    M = G.T @ G
    s = make_solver(P, 300)
    L = torch.zeros((20, 20), dtype=torch.float64, device="cuda")
    shifts = P.lobpcg_small_cholesky(s.h, cu(M), L)
    Lh = host(L)
    assert shifts == 0
    assert np.allclose(Lh, np.linalg.cholesky(M), atol=1e-12)
    # singular overlap: the plain factorisation fails, the shifted one works
    X = O.normalize_columns(np.column_stack([np.ones(50), np.ones(50), np.arange(50.0)]))
    M2 = X.T @ X
    L2 = torch.zeros((3, 3), dtype=torch.float64, device="cuda")
    shifts = P.lobpcg_small_cholesky(s.h, cu(M2), L2)
    st = O.OrthoStats()
    Lo = O.shifted_cholesky(M2, st)
    assert shifts == st.failed_factorizations >= 1
    # same shift as the oracle: L L^T - M is sigma I on both sides; entries
    # below a pivot of size sqrt(sigma) carry rounding of order eps/sqrt(sigma)
    Lg = host(L2)
    sig_g = np.diag(Lg @ Lg.T - M2)
    sig_o = np.diag(Lo @ Lo.T - M2)
    assert np.allclose(sig_g, sig_o, rtol=0.02)
    assert np.abs(Lg @ Lg.T - M2 - np.diag(sig_g)).max() <= 1e-15
    assert np.abs(Lg - Lo).max() <= 8 * np.finfo(float).eps / np.sqrt(sig_o.mean())


def graded(n, m, cond, seed):
    g = synth.rng(seed)
    U, _ = np.linalg.qr(g.standard_normal((n, m)))
    V, _ = np.linalg.qr(g.standard_normal((m, m)))
    return (U * np.logspace(0, -math.log10(cond), m)) @ V.T


@pytest.mark.parametrize("n,m,cond", [(5000, 8, 10.0), (20011, 16, 1e3), (3001, 32, 1e5), (1000, 1, 1.0)])
def test_ortho_vs_oracle(P, n, m, cond):
    say("ortho", n, m, cond)
    X = graded(n, m, cond, 3) * synth.rng(4).uniform(0.5, 10, m)
    s = make_solver(P, n)
    Xd = cu(X)
    info = P.lobpcg_ortho(s.h, Xd)
    Q = host(Xd)
    Qo = O.ortho(X)
    assert np.abs(Q.T @ Q - np.eye(m)).max() <= 1e-14
    assert np.abs(Q - Qo).max() <= 1e-15 * cond * 50
    assert info["stalled"] == 0


@pytest.mark.parametrize("n,m,cond", [(20011, 16, 1e3), (200003, 16, 1.001), (5000, 8, 1e5), (3001, 32, 10.0)])
def test_ortho_cheap_exit_vs_oracle(P, n, m, cond):
    """Cheap exit of Alg. 2 (the ||L^-T|| estimate Sec. 3.2 proposes): the
    GPU takes the oracle's decisions (same overlaps formed, same exits) and
    gives its Q; the overlap it skips would only have confirmed tau."""
    say("ortho cheap exit", n, m, cond)
    X = graded(n, m, cond, 3) * synth.rng(4).uniform(0.5, 10, m)
    s = make_solver(P, n)
    P.lobpcg_set_option(s.h, P.OPT_CHEAP_EXIT, 1)
    Xd = cu(X)
    info = P.lobpcg_ortho(s.h, Xd)
    Q = host(Xd)
    st = O.OrthoStats()
    Qo = O.ortho(X, stats=st, cheap_exit=True)
    say(info, st)
    assert np.abs(Q.T @ Q - np.eye(m)).max() <= 1e-14
    assert np.abs(Q - Qo).max() <= 1e-15 * cond * 50
    assert info["cheap_exits"] == st.cheap_exits and info["grams"] == st.grams
    assert info["updates"] == st.updates and info["stalled"] == 0
    # the same call without the exit forms one overlap more when it exits
    s2 = make_solver(P, n)
    Xd = cu(X)
    info0 = P.lobpcg_ortho(s2.h, Xd)
    assert info0["cheap_exits"] == 0 and info0["grams"] == info["grams"] + info["cheap_exits"]


@pytest.mark.parametrize("delta", [1e-1, 1e-4, 1e-9])
def test_ortho_against_cheap_exit_vs_oracle(P, delta):
    """Cheap exit of Alg. 3 (the growth factor of ortho(X)): Y^T W is not
    formed once the growth of the last Alg. 2 call bounds it below tau."""
    g = synth.rng(21)
    n, ny, nw = 100003, 16, 8
    Y = np.linalg.qr(g.standard_normal((n, ny)))[0]
    Xt = Y @ g.standard_normal((ny, nw)) + delta * g.standard_normal((n, nw))
    buf = cu(np.hstack([Y, Xt]))
    s = make_solver(P, n)
    P.lobpcg_set_option(s.h, P.OPT_CHEAP_EXIT, 1)
    info = P.lobpcg_ortho_against(s.h, buf[:, ny:], buf[:, :ny])
    out = host(buf)
    Q = out[:, ny:]
    st = O.OrthoStats()
    Qo = O.ortho_against(Xt, Y, stats=st, cheap_exit=True)
    say(delta, info, st)
    assert np.abs(Y.T @ Q).max() <= 1e-14
    assert np.abs(Q.T @ Q - np.eye(nw)).max() <= 1e-14
    assert info["cheap_exits"] >= 1 and st.cheap_exits >= 1
    assert info["passes"] == st.against_passes
    Qa = np.linalg.qr(np.hstack([Y, Q]))[0]
    Qb = np.linalg.qr(np.hstack([Y, Qo]))[0]
    assert np.linalg.norm(Qb - Qa @ (Qa.T @ Qb), 2) < 1e-12 / delta


def test_ortho_forced_shift(P):
    g = synth.rng(5)
    n = 800
    x, y = g.standard_normal(n), g.standard_normal(n)
    Z = g.standard_normal((n, 3))
    X = np.column_stack([x, x + 1e-10 * y, Z])
    s = make_solver(P, n)
    Xd = cu(X)
    info = P.lobpcg_ortho(s.h, Xd)
    Q = host(Xd)
    assert info["failed"] >= 1 and info["shifted"] == 1 and info["factorizations"] <= 4
    assert np.abs(Q.T @ Q - np.eye(5)).max() <= 1e-14


def test_ortho_svqb_without_shift_retries(P):
    """Sec. 3.2's fallback chain with the shifted retries switched off: the
    failed plain factorisation of a cond ~ 1e10 block goes straight to SVQB
    (Stathopoulos-Wu), as in the oracle with shift_retries=0, and the next
    pass finishes with a plain Cholesky."""
    say("ortho svqb")
    g = synth.rng(5)
    n = 800
    x, y = g.standard_normal(n), g.standard_normal(n)
    Z = g.standard_normal((n, 3))
    X = np.column_stack([x, x + 1e-10 * y, Z])
    s = make_solver(P, n)
    P.lobpcg_set_option(s.h, P.OPT_SHIFT_RETRIES, 0)
    Xd = cu(X)
    info = P.lobpcg_ortho(s.h, Xd)
    Q = host(Xd)
    st = O.OrthoStats()
    Qo = O.ortho(X, stats=st, shift_retries=0)
    say(info, st)
    assert st.svqb == 1 and st.failed_factorizations == 1
    assert info["svqb"] == st.svqb and info["failed"] == st.failed_factorizations
    assert info["shifted"] == 0 and info["stalled"] == 0
    assert np.abs(Q.T @ Q - np.eye(5)).max() <= 1e-14
    # the span is fixed to ~ eps cond: x, y and Z as the oracle keeps them
    dist = lambda A, B: np.linalg.norm(np.linalg.qr(A)[0] @ np.linalg.qr(A)[0].T - np.linalg.qr(B)[0] @ np.linalg.qr(B)[0].T, 2)
    assert dist(Q, Qo) < 1e-5 and dist(Q, np.column_stack([x, y, Z])) < 1e-5
    # an exactly repeated column: every column kept, finite and orthonormal
    s2 = make_solver(P, n)
    P.lobpcg_set_option(s2.h, P.OPT_SHIFT_RETRIES, 0)
    Xd = cu(np.column_stack([x, x, Z]))
    info = P.lobpcg_ortho(s2.h, Xd)
    Q = host(Xd)
    assert np.all(np.isfinite(Q)) and np.abs(Q.T @ Q - np.eye(5)).max() <= 1e-14
    B = np.column_stack([x, Z])
    assert np.linalg.norm(B - Q @ (Q.T @ B)) <= 1e-12 * np.linalg.norm(B)
    # the default (20 shifted retries) never needs SVQB here
    s3 = make_solver(P, n)
    Xd = cu(X)
    info = P.lobpcg_ortho(s3.h, Xd)
    assert info["svqb"] == 0 and info["shifted"] == 1


def test_ortho_against_svqb(P):
    """Alg. 3 around an Alg. 2 whose first factorisation fails, with SVQB as
    the only fallback: the oracle's bars (Y-orthogonality, orthonormality,
    span) hold."""
    g = synth.rng(8)
    n, ny = 7000, 4
    Y = np.linalg.qr(g.standard_normal((n, ny)))[0]
    x, y = g.standard_normal(n), g.standard_normal(n)
    Xt = np.column_stack([x, x + 1e-10 * y, g.standard_normal((n, 2))])
    buf = cu(np.hstack([Y, Xt]))
    s = make_solver(P, n)
    P.lobpcg_set_option(s.h, P.OPT_SHIFT_RETRIES, 0)
    info = P.lobpcg_ortho_against(s.h, buf[:, ny:], buf[:, :ny])
    out = host(buf)
    Q = out[:, ny:]
    st = O.OrthoStats()
    Qo = O.ortho_against(Xt, Y, stats=st, shift_retries=0)
    say(info, st)
    assert info["svqb"] >= 1 and st.svqb >= 1
    assert np.array_equal(out[:, :ny], Y)
    assert np.abs(Y.T @ Q).max() <= 1e-14
    assert np.abs(Q.T @ Q - np.eye(4)).max() <= 1e-14
    PQ = Q @ Q.T
    PO = Qo @ Qo.T
    assert np.linalg.norm(PQ - PO, 2) < 1e-5


def test_ortho_against_vs_oracle(P):
    g = synth.rng(11)
    n = 6000
    Y = np.linalg.qr(g.standard_normal((n, 6)))[0]
    Xt = Y @ g.standard_normal((6, 4)) + 1e-10 * g.standard_normal((n, 4))
    buf = cu(np.hstack([Y, Xt]))
    s = make_solver(P, n)
    info = P.lobpcg_ortho_against(s.h, buf[:, 6:], buf[:, :6])
    out = host(buf)
    Q = out[:, 6:]
    assert np.array_equal(out[:, :6], Y)
    assert np.abs(Y.T @ Q).max() <= 1e-14
    assert np.abs(Q.T @ Q - np.eye(4)).max() <= 1e-14
    assert info["passes"] <= 3
    Qo = O.ortho_against(Xt, Y)
    PQ = Q @ Q.T
    PO = Qo @ Qo.T
    assert np.linalg.norm(PQ - PO, 2) < 1e-5  # the 1e-10 part survives to ~1e-6


def test_ortho_zero_column(P):
    n = 1000
    X = synth.start_block(n, 3, 2)
    X[:, 1] = 0.0
    s = make_solver(P, n)
    Xd = cu(X)
    P.lobpcg_ortho(s.h, Xd)
    Q = host(Xd)
    assert np.abs(Q.T @ Q - np.eye(3)).max() <= 1e-14
    # the replacement is the oracle's SplitMix64 column, orthonormalised
    Qo = O.ortho(X)
    assert np.abs(Q - Qo).max() < 1e-12


@pytest.mark.parametrize("precond", [0, 1, 2])
def test_rotate_definition(P, precond):
    n, m, a0 = 10007, 6, 2
    p = m + 2 * 4
    q = m + (m - a0)
    g = synth.rng(precond)
    V = g.standard_normal((n, p))
    AV = g.standard_normal((n, p))
    U = g.standard_normal((p, q))
    theta = np.sort(g.uniform(0.5, 2.0, m))
    d = g.uniform(0.0, 3.0, n)
    d[:5] = theta[a0]  # exercise the guard
    s = P.Solver(n)
    s.ensure_workspace(m)
    s.set_preconditioner(precond, cu(d))
    ldo = q + (m - a0) + 3
    Vo = torch.zeros((n, ldo), dtype=torch.float64, device="cuda")
    AVo = torch.zeros((n, ldo), dtype=torch.float64, device="cuda")
    r2 = torch.zeros(m, dtype=torch.float64, device="cuda")
    P.lobpcg_rotate(s.h, cu(V), cu(AV), p, cu(U), m, q, cu(theta), a0, Vo, AVo, r2)
    Xn = V @ U
    AXn = AV @ U
    R = AXn[:, :m] - Xn[:, :m] * theta
    if precond == 0:
        Wt = R[:, a0:]
    else:
        Wt = O.precondition_diag(R[:, a0:], d, theta[a0:], signed=(precond == 2))
    vo, avo = host(Vo), host(AVo)
    scale = np.abs(V) @ np.abs(U)
    assert np.all(np.abs(vo[:, :q] - Xn) <= 1e-13 * scale)
    assert np.all(np.abs(avo[:, :q] - AXn) <= 1e-13 * (np.abs(AV) @ np.abs(U)))
    assert np.allclose(vo[:, q:q + m - a0], Wt, rtol=1e-12, atol=1e-12 * np.abs(Wt).max())
    assert np.allclose(host(r2), (R ** 2).sum(0), rtol=1e-12)


@pytest.mark.parametrize(
    "n,m,a0,npw,off",
    [
        (200003, 16, 0, 16, 0),  # the benchmark's shape: p = 48, q = 32; ~3 chunks per block, ragged tail
        (200003, 16, 5, 11, 2),  # p = 38 at a 16-byte aligned column offset
        (70001, 7, 1, 3, 0),  # odd p: staged path, 1-2 chunks per block
        (70001, 16, 3, 13, 1),  # misaligned base: staged path
    ],
)
def test_rotate_chunks(P, n, m, a0, npw, off):
    """The rotation over many 64-row chunks per workgroup (the register
    prefetch of the next chunk, and the staged path) against V U and AV U."""
    say("rotate chunks", n, m, a0, npw, off)
    p = m + 2 * npw
    q = m + (m - a0)
    g = synth.rng(n + off)
    Vf = g.standard_normal((n, p + off))
    AVf = g.standard_normal((n, p + off))
    U = g.standard_normal((p, q))
    theta = np.sort(g.uniform(0.5, 2.0, m))
    s = P.Solver(n)
    s.ensure_workspace(m)
    s.set_preconditioner(0)
    ldo = q + (m - a0)
    Vo = torch.zeros((n, ldo), dtype=torch.float64, device="cuda")
    AVo = torch.zeros((n, ldo), dtype=torch.float64, device="cuda")
    r2 = torch.zeros(m, dtype=torch.float64, device="cuda")
    P.lobpcg_rotate(s.h, cu(Vf)[:, off:], cu(AVf)[:, off:], p, cu(U), m, q, cu(theta), a0, Vo, AVo, r2)
    V, AV = Vf[:, off:], AVf[:, off:]
    Xn = V @ U
    AXn = AV @ U
    R = AXn[:, :m] - Xn[:, :m] * theta
    vo, avo = host(Vo), host(AVo)
    assert np.all(np.abs(vo[:, :q] - Xn) <= 1e-13 * (np.abs(V) @ np.abs(U)))
    assert np.all(np.abs(avo[:, :q] - AXn) <= 1e-13 * (np.abs(AV) @ np.abs(U)))
    assert np.allclose(vo[:, q:], R[:, a0:], rtol=1e-12, atol=1e-12 * np.abs(R).max())
    assert np.allclose(host(r2), (R ** 2).sum(0), rtol=1e-12)
    s.close()


def test_apply_dense_column_slice_at_buffer_end(P):
    # W is columns 2..6 of an (n, 8) buffer (16-byte aligned, vector path):
    # the operator must read no W column past the block's own (those of the
    # last row would lie past the buffer's end)
    n, ld, off, m = 1030, 8, 2, 5
    A = synth.dense_dd(n, seed=11)
    Wb = synth.start_block(n, ld, 4)
    s = P.Solver(n)
    s.set_operator_dense(cu(A))
    s.ensure_workspace(1)
    Wd = cu(Wb)
    Y = torch.zeros((n, m), dtype=torch.float64, device="cuda")
    P.lobpcg_apply_operator(s.h, Wd[:, off : off + m], Y)
    ref = A @ Wb[:, off : off + m]
    scale = np.abs(A) @ np.abs(Wb[:, off : off + m])
    assert np.all(np.abs(host(Y) - ref) <= 1e-13 * scale)
