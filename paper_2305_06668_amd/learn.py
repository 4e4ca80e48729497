"""Training pipeline of the learned preconditioner, driven through the C ABI.

Every computation runs in the HIP library: the solver produces Ritz blocks
(solves stopped early at the given iteration counts), the learner turns each
into a snapshot (residuals, near-exact Jacobi-Davidson corrections by block
MINRES) and trains the MLP with its own forward, backward and Adam kernels.
This module only sequences those calls.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import (
    OPT_MAX_ITER,
    lobpcg_learner_add_snapshot,
    lobpcg_learner_create,
    lobpcg_learner_destroy,
    lobpcg_learner_get_weights,
    lobpcg_learner_set_stream,
    lobpcg_learner_snapshot_info,
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


def train(
    solvers,
    block: int,
    snapshot_iters=(2, 5, 10, 20, 40),
    minres_maxiter: int = 100,
    minres_rtol: float = 1e-6,
    steps: int = 400,
    cols_per_step: int = 8,
    lr: float = 3e-3,
    seed: int = 1,
    device: int = 0,
) -> TrainReport:
    """Train on the operators held by `solvers` (paper_2305_06668_amd.Solver
    objects with an operator, a preconditioner and an initial block of
    `block` columns set).  Each solver is run up to every count in
    `snapshot_iters` (stopping early) and its Ritz block becomes a snapshot."""
    L = lobpcg_learner_create(device, seed)
    lobpcg_learner_set_stream(L)
    log = []
    relres = 0.0
    try:
        t0 = time.perf_counter()
        nsnap = 0
        for s in solvers:
            for it in snapshot_iters:
                s.set_option(OPT_MAX_ITER, it)
                res = s.solve(block, 1e-300)
                idx = lobpcg_learner_add_snapshot(L, s.h, res.evecs, minres_maxiter, minres_rtol)
                info = lobpcg_learner_snapshot_info(L, idx, block)
                relres = max(relres, float(info["minres_relres"].max()))
                nsnap += 1
            s.set_option(OPT_MAX_ITER, 1000)
        t1 = time.perf_counter()
        first, last = lobpcg_learner_train(L, steps, cols_per_step, lr, seed)
        t2 = time.perf_counter()
        w = lobpcg_learner_get_weights(L)
        log.append(dict(snapshots=nsnap, loss_first=first, loss_last=last))
        return TrainReport(w, nsnap, first, last, t1 - t0, t2 - t1, relres, log)
    finally:
        lobpcg_learner_destroy(L)
