"""Autotuner of the batched form.

Chooses the number of concurrent graph branches and the Kalman batch size
(the K extent of the covariance products P -= V V^T and of the Cholesky of
S) by timing graph replays of a plan over a sample of the patches. The cost
of a run does not depend on the values in (w, P), so replays that keep
updating the sample's state time the same work.
"""
from __future__ import annotations

import itertools
import time

import torch

from . import api


def time_plan(ctx: api.Context, params: api.Params, patches: list, streams: int,
              batch: int, reps: int = 2, **kw) -> float:
    """Seconds per graph replay of one plan (after the capturing run)."""
    for q in patches:
        q["batch"] = 0
    plan = api.Batched(ctx, params, patches, streams=streams, default_batch=batch, **kw)
    try:
        plan.run()  # capture + first run
        plan.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            plan.run()
        plan.sync()
        return (time.perf_counter() - t0) / reps
    finally:
        plan.close()


def tune_batched(ctx: api.Context, params: api.Params, sample: list,
                 streams=(1, 2, 4, 8), batches=(512, 1024, 2048), reps: int = 2, **kw):
    """Return ((streams, batch), {(streams, batch): seconds}) over the grid."""
    table = {}
    for s, b in itertools.product(streams, batches):
        table[(s, b)] = time_plan(ctx, params, sample, s, b, reps=reps, **kw)
    best = min(table, key=table.get)
    return best, table
