"""What the trained network gains over the method without it (Jacobi), on
held-out matrices of the preconditioner-study family, with everything --
snapshot solves, MINRES corrections, forward/backward, Adam, inference --
running in the library.

The gain is parity unpinned by nature (a measurement, not a value any oracle
fixes); the test asserts a clear margin that the measured gain exceeds
(about 3x fewer iterations at this size) and that every learned solve meets
the eigenpair bar.  It also solves with the untrained initial weights (the
regularised Jacobi step with c = s softplus(-3) ~ 0.05 s wherever the net
acts): measured, they take 161 iterations in all against Jacobi's 436 and
the trained weights' 151, so most of the gain at this size is the
regularised form and training adds ~6 %; the bar there is that training
does not make it worse (5 % slack for rounding-level iteration noise).
"""
import numpy as np
import pytest

import synth
from oracle import lobpcg_oracle as O

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

N, K = 20_000, 8


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2305_06668_amd as P

    return P


def say(*a):
    print(*a, flush=True)


def family_solver(P, idx):
    C, rho = synth.csr_family(idx, n=N)
    s = P.Solver(N)
    s.set_operator_csr(*(torch.from_numpy(a).cuda() for a in (C.row_ptr, C.col, C.val)))
    s.set_preconditioner(P.PRECOND_DIAG)
    s.set_initial_guess(torch.from_numpy(synth.start_block(N, K, 99 + idx)).cuda())
    return s, C, rho


def test_learned_beats_jacobi_on_held_out_matrices(P):
    from paper_2305_06668_amd import learn

    trainers = [family_solver(P, i)[0] for i in range(8)]
    val, _, _ = family_solver(P, 191)

    def validate(w):
        val.set_learned_weights(w)
        val.set_preconditioner(P.PRECOND_LEARNED)
        r = val.solve(K, 1e-8, want_vectors=False)
        return r.stats["iterations"] if r.status == P.OK else 10**6

    rep = learn.train(trainers, K, steps=300, cols_per_step=K, lr=1e-3, chunks=3, validate=validate)
    say(f"trained: loss {rep.loss_first:.3f} -> {rep.loss_last:.3f}, validation {[c['score'] for c in rep.log]}")
    # the weights training starts from (learn.train's learner seed, 1)
    L0 = P.lobpcg_learner_create(0, 1)
    try:
        w0 = P.lobpcg_learner_get_weights(L0)
    finally:
        P.lobpcg_learner_destroy(L0)
    it_d, it_l, it_0 = [], [], []
    for idx in (192, 193, 194, 195):
        s, C, rho = family_solver(P, idx)
        s.set_learned_weights(rep.weights)
        out = {}
        for name, kind in (("diag", P.PRECOND_DIAG), ("learned", P.PRECOND_LEARNED)):
            s.set_preconditioner(kind)
            res = s.solve(K, 1e-8)
            assert res.status == P.OK, (idx, name)
            out[name] = res
        say(f"matrix {idx} (rho {rho:.2f}): jacobi {out['diag'].stats['iterations']} iterations, "
            f"learned {out['learned'].stats['iterations']} ({out['learned'].stats['learned_fallbacks']} fallbacks)")
        it_d.append(out["diag"].stats["iterations"])
        it_l.append(out["learned"].stats["iterations"])
        s.set_learned_weights(w0)
        r0 = s.solve(K, 1e-8, want_vectors=False)
        assert r0.status == P.OK, (idx, "untrained")
        it_0.append(r0.stats["iterations"])
        say(f"   untrained weights: {it_0[-1]} iterations")
        s.set_learned_weights(rep.weights)
        # both solves return the same pairs (each certified by its residuals)
        op = O.csr_operator(C.row_ptr, C.col, C.val, N)
        X = out["learned"].evecs.cpu().numpy()
        AX = op(X)
        th = np.einsum("ij,ij->j", X, AX)
        assert np.all(np.linalg.norm(AX - X * th, axis=0) <= 1e-8 * 1.0001)
        scale = np.maximum(np.abs(out["diag"].evals), 1e-3 * np.abs(C.val).max())
        assert np.all(np.abs(out["learned"].evals - out["diag"].evals) <= 1e-9 * scale)
    say(f"total iterations: jacobi {sum(it_d)}, untrained {sum(it_0)}, learned {sum(it_l)}")
    assert sum(it_l) <= 0.7 * sum(it_d)
    assert sum(it_l) <= 1.05 * sum(it_0)
