"""Pins for the CPU oracle of the learned preconditioner (oracle/mlp_oracle.py)."""
import numpy as np
import pytest

import synth
from oracle import mlp_oracle as M


def small_problem(seed=1, B=64, H=16):
    g = synth.rng(seed)
    p = M.init_params(seed, H=H)
    X = g.standard_normal((B, M.NFEAT))
    t = g.standard_normal(B)
    return p, X, t


def test_backward_matches_central_differences():
    p, X, t = small_problem(H=16)
    y, cache = M.forward(p, X)
    gr = M.backward(p, cache, y, t).flat()
    v = p.flat()
    h = 1e-6
    idx = np.linspace(0, v.size - 1, 60).astype(int)
    for i in idx:
        vp, vm = v.copy(), v.copy()
        vp[i] += h
        vm[i] -= h
        lp = M.loss(M.forward(M.Params.from_flat(vp, H=16), X)[0], t)
        lm = M.loss(M.forward(M.Params.from_flat(vm, H=16), X)[0], t)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gr[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, gr[i])


def test_zero_output_layer_is_bias():
    p, X, t = small_problem()
    p.W3[:] = 0.0
    p.b3[:] = 0.25
    y, _ = M.forward(p, X)
    assert np.all(y == 0.25)


def test_silu_closed_forms():
    assert M.silu(np.array([0.0]))[0] == 0.0
    assert abs(M.silu(np.array([40.0]))[0] - 40.0) < 1e-12
    z = np.linspace(-5, 5, 21)
    h = 1e-6
    assert np.allclose(M.dsilu(z), (M.silu(z + h) - M.silu(z - h)) / (2 * h), atol=1e-8)


def test_adam_first_step_is_signed_lr():
    g = np.array([3.0, -0.5, 1e-3])
    th, m, v = M.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=1e-2)
    assert np.allclose(th, -1e-2 * np.sign(g), rtol=1e-4)


def test_param_count_and_roundtrip():
    p = M.init_params(3)
    assert p.flat().size == M.n_params() == 128 * 4 + 128 + 128 * 128 + 128 + 128 + 1
    q = M.Params.from_flat(p.flat())
    assert np.array_equal(q.flat(), p.flat())


def test_features_definition():
    r = np.array([1.0, -2.0, 0.5, 0.0])
    d = np.array([2.0, 1.0, 1.5, 4.0])
    f = M.features(r, d, 1.0, 2.0)
    rms = np.sqrt(np.mean(r * r))
    assert np.allclose(f[:, 0], r / rms)
    assert np.allclose(f[:, 1], (d - 1.0) / 2.0)
    assert np.allclose(f[:, 2], 0.5)
    assert np.allclose(f[:, 3], (r / rms) / (np.abs((d - 1.0) / 2.0) + 1e-3))


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
    t_ref /= np.sqrt(np.mean(t_ref**2))
    assert abs(T[:, 0] @ x) < 1e-10
    assert np.allclose(T[:, 0], t_ref, atol=1e-7)
