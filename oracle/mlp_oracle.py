"""CPU fp64 oracle for the learned preconditioner (test infrastructure only).

The learned preconditioner is an extension beside the paper's method (the
paper's own study of better preconditioners is Sec. 4.4; its default is the
Jacobi preconditioner of Sec. 2).  Reading used here:

  * a per-entry MLP 4 -> 128 -> 128 -> 1 with SiLU activations maps, for an
    active residual column r (Ritz value theta) and the operator diagonal d,
    the features
        f1 = r_i / rms(r)
        f2 = (d_i - theta) / s
        f3 = theta / s
        f4 = r_i / (rms(r) (|d_i - theta| / s + 1e-3))
    (s = mean |d|) to a correction c_i; the preconditioned column is c;
  * training targets are the Jacobi-Davidson corrections t solving
        (I - x x^T)(A - theta I)(I - x x^T) t = -r,  t orthogonal to x
    (MINRES, relative residual 1e-6), scaled to unit RMS per column;
  * loss: mean squared error over the sampled entries; Adam.

Functions: ``features``, ``forward``, ``backward`` (analytic gradients),
``loss``, ``adam_step``, ``jd_targets`` (scipy MINRES on the projected
operator).  Everything in float64.
"""
from __future__ import annotations

import dataclasses

import numpy as np

HIDDEN = 128
NFEAT = 4
FEAT_EPS = 1e-3


@dataclasses.dataclass
class Params:
    W1: np.ndarray  # (H, F)
    b1: np.ndarray  # (H,)
    W2: np.ndarray  # (H, H)
    b2: np.ndarray  # (H,)
    W3: np.ndarray  # (1, H)
    b3: np.ndarray  # (1,)

    def flat(self) -> np.ndarray:
        return np.concatenate([self.W1.ravel(), self.b1, self.W2.ravel(), self.b2, self.W3.ravel(), self.b3])

    @staticmethod
    def from_flat(v: np.ndarray, H: int = HIDDEN, F: int = NFEAT) -> "Params":
        v = np.asarray(v, dtype=np.float64)
        o = 0

        def take(shape):
            nonlocal o
            size = int(np.prod(shape))
            out = v[o : o + size].reshape(shape)
            o += size
            return out.copy()

        p = Params(take((H, F)), take((H,)), take((H, H)), take((H,)), take((1, H)), take((1,)))
        assert o == v.size
        return p


def n_params(H: int = HIDDEN, F: int = NFEAT) -> int:
    return H * F + H + H * H + H + H + 1


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def features(r: np.ndarray, d: np.ndarray, theta: float, s: float) -> np.ndarray:
    """Per-entry features of one residual column (n x 4)."""
    rms = np.sqrt(np.mean(r * r))
    rn = r / rms
    dm = (d - theta) / s
    return np.column_stack([rn, dm, np.full_like(r, theta / s), rn / (np.abs(dm) + FEAT_EPS)])


def forward(p: Params, X: np.ndarray):
    """Returns (y, cache) for inputs X (B x F)."""
    z1 = X @ p.W1.T + p.b1
    h1 = silu(z1)
    z2 = h1 @ p.W2.T + p.b2
    h2 = silu(z2)
    y = (h2 @ p.W3.T + p.b3)[:, 0]
    return y, (X, z1, h1, z2, h2)


def loss(y: np.ndarray, t: np.ndarray) -> float:
    return float(np.mean((y - t) ** 2))


def backward(p: Params, cache, y: np.ndarray, t: np.ndarray) -> Params:
    """Analytic gradient of the mean squared error."""
    X, z1, h1, z2, h2 = cache
    B = X.shape[0]
    dy = (2.0 / B) * (y - t)  # (B,)
    dW3 = dy[None, :] @ h2  # (1, H)
    db3 = np.array([dy.sum()])
    dh2 = dy[:, None] * p.W3  # (B, H)
    dz2 = dh2 * dsilu(z2)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(0)
    dh1 = dz2 @ p.W2
    dz1 = dh1 * dsilu(z1)
    dW1 = dz1.T @ X
    db1 = dz1.sum(0)
    return Params(dW1, db1, dW2, db2, dW3, db3)


def adam_step(theta: np.ndarray, g: np.ndarray, m: np.ndarray, v: np.ndarray, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) on flat arrays; returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1**t)
    vh = v / (1 - b2**t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed: int, H: int = HIDDEN, F: int = NFEAT) -> Params:
    g = np.random.Generator(np.random.PCG64(seed))
    return Params(
        g.normal(0, 1 / np.sqrt(F), (H, F)),
        np.zeros(H),
        g.normal(0, 1 / np.sqrt(H), (H, H)),
        np.zeros(H),
        g.normal(0, 1 / np.sqrt(H), (1, H)),
        np.zeros(1),
    )


def jd_targets(A, X: np.ndarray, theta: np.ndarray, R: np.ndarray, rtol: float = 1e-6, maxiter: int = 500) -> np.ndarray:
    """Jacobi-Davidson corrections t_j: (I - x x^T)(A - theta_j I)(I - x x^T) t = -r_j,
    t orthogonal to x_j, by MINRES; each column scaled to unit RMS."""
    import scipy.sparse.linalg as spla

    n = X.shape[0]
    out = np.empty_like(R)
    for j in range(R.shape[1]):
        x = X[:, j] / np.linalg.norm(X[:, j])
        th = float(theta[j])

        def mv(v, x=x, th=th):
            v = v - x * (x @ v)
            w = A @ v - th * v
            return w - x * (x @ w)

        op = spla.LinearOperator((n, n), matvec=mv, dtype=np.float64)
        b = -(R[:, j] - x * (x @ R[:, j]))
        t, _ = spla.minres(op, b, rtol=rtol, maxiter=maxiter)
        t = t - x * (x @ t)
        out[:, j] = t / np.sqrt(np.mean(t * t))
    return out
