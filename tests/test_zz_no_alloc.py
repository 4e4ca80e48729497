"""lobpcg_gram_noalloc, the Gram entry point that allocates nothing (its
partial sums live in the library's static device array): it must give
exactly lobpcg_gram's result, on consecutive calls that share that array
(the second with a smaller input), and reject sizes beyond its limit."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2305_06668_amd as P

    return P


def test_gram_noalloc_matches_gram(P):
    # (n, p, q): the second call is smaller, so it runs over what the first
    # left in the shared array; the third is the single-column edge
    cases = [(200003, 64, 48), (20011, 17, 5), (7, 1, 1)]
    for n, p, q in cases:
        print("gram_noalloc", n, p, q, flush=True)
        g = synth.rng(n + p + q)
        A = g.standard_normal((n, p))
        B = g.standard_normal((n, q))
        s = P.Solver(n)  # no workspace: the no-alloc form needs none
        Ad = torch.from_numpy(A).cuda()
        Bd = torch.from_numpy(B).cuda()
        C0 = torch.full((p, q), np.nan, dtype=torch.float64, device="cuda")
        P.lobpcg_gram_noalloc(s.h, Ad, Bd, C0)
        torch.cuda.synchronize()
        Cn = C0.cpu().numpy()
        # the workspace form on the same handle
        s.ensure_workspace(1)
        C1 = torch.full((p, q), np.nan, dtype=torch.float64, device="cuda")
        P.lobpcg_gram(s.h, Ad, Bd, C1)
        torch.cuda.synchronize()
        Cw = C1.cpu().numpy()
        assert np.array_equal(Cn, Cw), np.abs(Cn - Cw).max()
        ref = A.T @ B
        scale = np.abs(A).T @ np.abs(B)
        assert np.all(np.abs(Cn - ref) <= 1e-13 * scale)
        s.close()


def test_gram_noalloc_rejects_large(P):
    n = 1000
    s = P.Solver(n)
    A = torch.zeros((n, 65), dtype=torch.float64, device="cuda")
    C = torch.zeros((65, 65), dtype=torch.float64, device="cuda")
    with pytest.raises(P.LobpcgError) as e:
        P.lobpcg_gram_noalloc(s.h, A, A, C)
    assert e.value.status == P.ERR_INVALID_ARG
    assert "64" in str(e.value)
