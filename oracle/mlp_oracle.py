"""CPU fp64 oracle for the learned preconditioner (test infrastructure only:
imported by tests, the smoke check and the CPU baseline, never by the GPU
library).

The learned preconditioner is an extension beside the paper's method; the
paper's default preconditioner is the Jacobi one of Sec. 2 and its study of
better preconditioners is Sec. 4.4.  Reading used here:

Preconditioned column.  For an active residual column r (Ritz value theta)
of an operator with diagonal d and off-diagonal absolute row sums
rho_i = sum_{l != i} |a_il|, with s = mean_i |d_i|,

    w_i = r_i / sqrt((d_i - theta)^2 + c_i^2),     c_i = s * softplus(y_i)
                                                    if |d_i - theta| <= 16 rho_i,
                                                    c_i = 0 otherwise,

where y_i is the output of a per-entry MLP 3 -> 128 -> 128 -> 1 (SiLU) on
the features
    phi_1 = log(|d_i - theta| / s + 1e-6),
    phi_2 = theta / s,
    phi_3 = log(rho_i / s + 1e-6).
c -> 0 gives the absolute Jacobi preconditioner; the net learns how much to
regularise it where d_i is close to theta relative to the coupling rho_i.
Outside the window |d_i - theta| <= 16 rho_i the step is the Jacobi one (a
regulariser of the size of the coupling changes w there by less than
(1/16)^2 / 2), so only the entries near theta need the net.
The denominator is floored at delta = 1e-8 max(1, |theta|), the Jacobi guard.

Training objective.  For a column j with Ritz vector x_j in the orthonormal
block X, let u = (I - X X^T) w.  The Rayleigh-Ritz step on span{x_j, u}
lowers the Ritz value by
    Delta(w) = sqrt(h^2 + b^2) - h,   b = r^T u / |u|,  h = (u^T A u / |u|^2 - theta) / 2
(theta minus the smaller eigenvalue of the 2 x 2 projected matrix
[[theta, b], [b, 2h + theta]]), evaluated as b^2 / (S + h) with
S = sqrt(h^2 + b^2) when h > 0, where the difference form cancels.
The loss is the mean over columns of log(Delta(t) / Delta(w)), where t is
the near-exact Jacobi-Davidson correction of the same column (``jd_targets``):
it is the log of the factor by which the learned step falls short of the
near-exact solve's step.  Its gradient does not depend on t, so a second,
supervised term ties the learned step to the near-exact one itself: with
tau = (I - X X^T) t, the column adds mu (1 - cos^2 angle(u, tau)) (``alignment``),
zero when the learned direction is the near-exact one, one when it is
orthogonal to it, blind to the scale of w (which the Rayleigh-Ritz step
ignores too).  mu = 0 leaves the first term alone.

Functions: ``features``, ``forward``, ``backward_dy`` (generic MLP backward
for an output gradient), ``precondition``, ``decrease`` (Delta),
``alignment`` (the supervised term and its gradient), ``objective`` (loss and
analytic gradient with respect to the flat parameters), ``adam_step``,
``init_params``, ``jd_targets``.  Everything in
float64.
"""
from __future__ import annotations

import dataclasses

import numpy as np

HIDDEN = 128
NFEAT = 3
FEAT_FLOOR = 1e-6
GUARD = 1e-8  # Jacobi guard, relative to max(1, |theta|)
WINDOW = 16.0  # the net acts where |d - theta| <= WINDOW * rho


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


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def silu(z):
    return z * sigmoid(z)


def dsilu(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def softplus(y):
    return np.logaddexp(0.0, y)


def scale_of(d: np.ndarray) -> float:
    return float(np.mean(np.abs(d)))


def features(d: np.ndarray, theta: float, rho: np.ndarray, s: float) -> np.ndarray:
    """Per-entry features of one column (n x 3)."""
    return np.column_stack(
        [
            np.log(np.abs(d - theta) / s + FEAT_FLOOR),
            np.full(d.shape, theta / s),
            np.log(rho / s + FEAT_FLOOR),
        ]
    )


def forward(p: Params, X: np.ndarray):
    """Returns (y, cache) for inputs X (B x F)."""
    z1 = X @ p.W1.T + p.b1
    h1 = silu(z1)
    z2 = h1 @ p.W2.T + p.b2
    h2 = silu(z2)
    y = (h2 @ p.W3.T + p.b3)[:, 0]
    return y, (X, z1, h1, z2, h2)


def backward_dy(p: Params, cache, dy: np.ndarray) -> Params:
    """Gradient of sum_i dy_i * y_i with respect to the parameters."""
    X, z1, h1, z2, h2 = cache
    dW3 = dy[None, :] @ h2
    db3 = np.array([dy.sum()])
    dz2 = (dy[:, None] * p.W3) * dsilu(z2)
    dW2 = dz2.T @ h1
    db2 = dz2.sum(0)
    dz1 = (dz2 @ p.W2) * dsilu(z1)
    dW1 = dz1.T @ X
    db1 = dz1.sum(0)
    return Params(dW1, db1, dW2, db2, dW3, db3)


def precondition(p: Params, r: np.ndarray, d: np.ndarray, theta: float, rho: np.ndarray, s: float):
    """The learned preconditioned column w (and the pieces the gradient needs)."""
    F = features(d, theta, rho, s)
    y, cache = forward(p, F)
    dm = d - theta
    inside = np.abs(dm) <= WINDOW * rho
    c = np.where(inside, s * softplus(y), 0.0)
    delta = GUARD * max(1.0, abs(theta))
    q = np.maximum(dm * dm + c * c, delta * delta)
    w = r / np.sqrt(q)
    return w, dict(y=y, c=c, q=q, floored=(dm * dm + c * c) < delta * delta, inside=inside, cache=cache)


def _delta(h: float, b: float):
    """(Delta, S) for Delta = sqrt(h^2 + b^2) - h without cancellation."""
    S = float(np.hypot(h, b))
    D = b * b / (S + h) if h > 0.0 else S - h
    return D, S


def decrease(A, X: np.ndarray, x: np.ndarray, r: np.ndarray, theta: float, w: np.ndarray) -> float:
    """Delta(w): how far the Rayleigh-Ritz step on span{x, (I - X X^T) w}
    lowers theta."""
    u = w - X @ (X.T @ w)
    nu2 = float(u @ u)
    b = float(r @ u) / np.sqrt(nu2)
    h = (float(u @ (A @ u)) / nu2 - theta) / 2.0
    return _delta(h, b)[0]


def alignment(u: np.ndarray, tau: np.ndarray):
    """1 - cos^2 of the angle between u and tau, and its gradient in u:
    with c = u.tau, a = u.u, e = tau.tau the value is 1 - c^2 / (a e) and
    d/du = -2 c / (a e) tau + 2 c^2 / (a^2 e) u.  (0, 0) when tau = 0."""
    a = float(u @ u)
    e = float(tau @ tau)
    if e == 0.0 or a == 0.0:
        return 0.0, np.zeros_like(u)
    c = float(u @ tau)
    return 1.0 - c * c / (a * e), -2.0 * c / (a * e) * tau + 2.0 * c * c / (a * a * e) * u


def objective(p: Params, A, X: np.ndarray, R: np.ndarray, theta: np.ndarray, cols, d, rho, s, ref=None,
              T=None, mu=0.0):
    """Mean over the columns `cols` of log(ref_j / Delta_j(w_j)) (ref_j = 1
    when None), plus mu (1 - cos^2 angle(u_j, (I - X X^T) T[:, j])) when the
    near-exact corrections T (n x m, all columns of the block) are given, and
    its gradient with respect to the flat parameters."""
    g = np.zeros(n_params(p.W2.shape[0], p.W1.shape[1]))
    L = 0.0
    nc = len(cols)
    for k, j in enumerate(cols):
        r = R[:, j]
        th = float(theta[j])
        w, aux = precondition(p, r, d, th, rho, s)
        u = w - X @ (X.T @ w)
        Au = A @ u
        nu2 = float(u @ u)
        nu = np.sqrt(nu2)
        b = float(r @ u) / nu
        cq = float(u @ Au) / nu2
        h = (cq - th) / 2.0
        D, S = _delta(h, b)
        L += (np.log(1.0 if ref is None else ref[k]) - np.log(D)) / nc
        # dD/db = b / S, dD/dcq = (h / S - 1) / 2 = -D / (2 S); the products
        # with dL/dD = -1 / (D nc) are formed without dividing by a tiny D
        cb = -b / (S * D * nc)
        cc = 1.0 / (2.0 * S * nc)
        gu = cb * (r / nu - b * u / nu2) + cc * 2.0 * (Au - cq * u) / nu2
        if T is not None and mu != 0.0:
            tau = T[:, j] - X @ (X.T @ T[:, j])
            la, ga = alignment(u, tau)
            L += mu * la / nc
            gu = gu + (mu / nc) * ga
        gw = gu - X @ (X.T @ gu)
        # w = r q^-1/2, q = dm^2 + c^2 (not floored), c = s softplus(y)
        dq = gw * r * (-0.5) * aux["q"] ** -1.5
        dq = np.where(aux["floored"] | ~aux["inside"], 0.0, dq)
        dy = dq * 2.0 * aux["c"] * s * sigmoid(aux["y"])
        g += backward_dy(p, aux["cache"], dy).flat()
    return L, g


def adam_step(theta: np.ndarray, g: np.ndarray, m: np.ndarray, v: np.ndarray, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba) on flat arrays; returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1**t)
    vh = v / (1 - b2**t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(seed: int, H: int = HIDDEN, F: int = NFEAT, out_bias: float = -3.0) -> Params:
    g = np.random.Generator(np.random.PCG64(seed))
    return Params(
        g.normal(0, 1 / np.sqrt(F), (H, F)),
        np.zeros(H),
        g.normal(0, 1 / np.sqrt(H), (H, H)),
        np.zeros(H),
        0.1 * g.normal(0, 1 / np.sqrt(H), (1, H)),
        np.full(1, out_bias),
    )


def jd_targets(A, X: np.ndarray, theta: np.ndarray, R: np.ndarray, rtol: float = 1e-6, maxiter: int = 500) -> np.ndarray:
    """Jacobi-Davidson corrections t_j: (I - x x^T)(A - theta_j I)(I - x x^T) t = -r_j,
    t orthogonal to x_j, by MINRES from a zero start."""
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
        out[:, j] = t - x * (x @ t)
    return out
