"""Autotuner of the batched form.

Chooses the tile shape of the FP64 covariance products ("auto", "128" or
"sub") and the Kalman batch (the K extent of the covariance products and
the size of S, whose Cholesky is the latency-bound stage) by timing graph
replays of a plan over a sample of the patches. The cost of a run does not
depend on the values in (w, P), so replays that keep updating the sample's
state time the same work.
"""
from __future__ import annotations

import itertools
import time

import torch

from . import api


def time_plan(ctx: api.Context, params: api.Params, patches: list, tile: str,
              batch: int, reps: int = 2, **kw) -> float:
    """Seconds per graph replay of one plan (after the capturing run)."""
    for q in patches:
        q["batch"] = 0
    plan = api.Batched(ctx, params, patches, tile=tile, default_batch=batch, **kw)
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
                 tiles=("auto", "128", "sub"), batches=(512, 1024, 2048), reps: int = 2,
                 **kw):
    """Return ((tile, batch), {(tile, batch): seconds}) over the grid."""
    table = {}
    for t, b in itertools.product(tiles, batches):
        table[(t, b)] = time_plan(ctx, params, sample, t, b, reps=reps, **kw)
    best = min(table, key=table.get)
    return best, table
