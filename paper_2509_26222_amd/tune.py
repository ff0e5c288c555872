"""Autotuner of the batched form.

Chooses the number of concurrent patch chains (1, 2 or 4), the tile shape of
the FP64 covariance products ("auto", "128" or "sub") and the Kalman batch (the K extent of the covariance products and
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


def time_plan(ctx: api.Context, params: api.Params, patches: list, chains: int, tile: str,
              batch: int, reps: int = 2, **kw) -> float:
    """Seconds per graph replay of one plan (after the capturing run)."""
    for q in patches:
        q["batch"] = 0
    plan = api.Batched(ctx, params, patches, tile=tile, chains=chains, default_batch=batch,
                       **kw)
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


def tune_batched(ctx: api.Context, params: api.Params, sample: list, chains=(1, 2, 4),
                 tiles=("auto", "128", "sub"), batches=(512, 1024, 2048), reps: int = 2,
                 **kw):
    """Return ((chains, tile, batch), {(chains, tile, batch): seconds})."""
    table = {}
    for c, t, b in itertools.product(chains, tiles, batches):
        table[(c, t, b)] = time_plan(ctx, params, sample, c, t, b, reps=reps, **kw)
    best = min(table, key=table.get)
    return best, table
