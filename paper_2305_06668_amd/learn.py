"""Training pipeline of the learned preconditioner, driven through the C ABI.

Every computation runs in the HIP library: the solver produces Ritz blocks
(solves stopped early at the given iteration counts), the learner turns each
into a snapshot (residuals, near-exact Jacobi-Davidson corrections by block
MINRES) and trains the MLP with its own forward, backward and Adam kernels.
This module only sequences those calls, and keeps the weights that did best
on a caller-supplied validation solve (the objective is a one-step decrease,
so its value is a noisy guide to the iteration count of whole solves).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import (
    OPT_MAX_ITER,
    lobpcg_learner_add_snapshot,
    lobpcg_learner_create,
    lobpcg_learner_destroy,
    lobpcg_learner_get_weights,
    lobpcg_learner_snapshot_info,
    lobpcg_learner_set_supervision,
    lobpcg_learner_train,
)


@dataclass
class TrainReport:
    weights: np.ndarray
    snapshots: int
    loss_first: float
    loss_last: float
    seconds_collect: float
    seconds_train: float
    minres_relres_max: float
    log: list = field(default_factory=list)
    best_chunk: int = -1
    best_score: float = float("nan")


def train(
    solvers,
    block: int,
    snapshot_iters=(1, 3, 8, 20, 50),
    minres_maxiter: int = 100,
    minres_rtol: float = 1e-6,
    steps: int = 300,
    cols_per_step: int = 8,
    lr: float = 1e-3,
    seed: int = 1,
    device: int = 0,
    chunks: int = 1,
    validate=None,
    supervision: float = 1.0,
    progress=None,
    lr_schedule: str = "constant",
) -> TrainReport:
    """Train on the operators held by `solvers` (paper_2305_06668_amd.Solver
    objects with an operator, a preconditioner and an initial block of
    `block` columns set).  Each solver is run up to every count in
    `snapshot_iters` (stopping early) and its Ritz block becomes a snapshot.

    The `steps` Adam steps run in `chunks` equal parts; with `validate`
    (weights -> score, lower is better) the weights after each part are
    scored and the best are returned.  `supervision` is the weight of the
    loss term that aligns the learned step with the MINRES correction;
    `progress(i, snapshots)`, when given, is called after solver i's
    snapshots are taken.  `lr_schedule` "cosine" runs chunk c at
    lr (1 + cos(pi c / chunks)) / 2 (the late chunks settle instead of
    moving at the full rate); "constant" keeps lr."""
    if lr_schedule not in ("constant", "cosine"):
        raise ValueError(f"lr_schedule: {lr_schedule!r}")
    L = lobpcg_learner_create(device, seed)
    lobpcg_learner_set_supervision(L, supervision)
    log = []
    relres = 0.0
    try:
        t0 = time.perf_counter()
        nsnap = 0
        for si, s in enumerate(solvers):
            for it in snapshot_iters:
                s.set_option(OPT_MAX_ITER, it)
                res = s.solve(block, 1e-300)
                idx = lobpcg_learner_add_snapshot(L, s.h, res.evecs, minres_maxiter, minres_rtol)
                info = lobpcg_learner_snapshot_info(L, idx, block)
                relres = max(relres, float(info["minres_relres"].max()))
                nsnap += 1
            s.set_option(OPT_MAX_ITER, 1000)
            if progress is not None:
                progress(si, nsnap)
        t1 = time.perf_counter()
        per = max(1, steps // max(1, chunks))
        best_w, best_score, best_chunk = None, float("inf"), -1
        first = last = float("nan")
        nch = max(1, chunks)
        for c in range(nch):
            lr_c = lr if lr_schedule == "constant" else lr * 0.5 * (1.0 + math.cos(math.pi * c / nch))
            a, b = lobpcg_learner_train(L, per, cols_per_step, lr_c, seed * 1000003 + c)
            if c == 0:
                first = a
            last = b
            w = lobpcg_learner_get_weights(L)
            score = float(validate(w)) if validate is not None else float(c)
            log.append(dict(chunk=c, steps=per * (c + 1), loss_first=a, loss_last=b, score=score))
            if validate is None or score < best_score:
                best_w, best_score, best_chunk = w, score, c
        t2 = time.perf_counter()
        return TrainReport(best_w, nsnap, first, last, t1 - t0, t2 - t1, relres, log, best_chunk, best_score)
    finally:
        lobpcg_learner_destroy(L)
