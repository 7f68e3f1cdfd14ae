"""Launch-shape and schedule tuner for the batched persistent Newton launch.

md_newton_batch takes a launch shape (threads per workgroup, number of
persistent workgroups, waves per workgroup that evaluate terms) and a job
order.  Every shape gives the same bits; only the time changes.  The tuner
measures on the device:

  * the job order: longest first by the analytic operation count (Table 1
    weights of the md operations of one Newton step), or longest first by
    the duration of every path measured with the device wall clock in a
    first run (list scheduling of the longest jobs first, the paper's job
    queue with a better order);
  * the shape: block in {256, 512}, grid in multiples of the compute units,
    eval_waves among the values whose LDS fits.

It keeps the fastest and leaves that order set on the batch.  Results are
cached per batch structure and iteration count for the process.
"""
from __future__ import annotations

import hashlib

import numpy as np
import torch

from . import binding as B

_cache: dict = {}


def signature(batch: B.BatchedPaths, iters: int) -> str:
    h = hashlib.sha256(batch.table.tobytes())
    h.update(str(iters).encode())
    return h.hexdigest()


def _time(batch, iters, stream, reps, **shape) -> float:
    best = float("inf")
    for _ in range(reps):
        batch.restore()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        B.md_newton_batch(batch, iters, stream=stream, **shape)
        e1.record(stream)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def eval_wave_choices(batch, block):
    limit = B.md_device_lds_bytes()
    fits = [ew for ew in range(1, block // 64 + 1)
            if B.md_batch_lds_bytes(batch.max_m, batch.max_d, batch.max_deg, ew) <= limit]
    if not fits:
        return [1]
    top = fits[-1]
    return sorted({top, max(1, top // 2)})


def measured_durations(batch, iters, stream=None, **shape) -> np.ndarray:
    """Device wall-clock duration (seconds) of every path in one run."""
    clk = torch.zeros((batch.npaths, 2), dtype=torch.int64, device=batch.reals.device)
    batch.restore()
    B.md_newton_batch(batch, iters, stream=stream, path_clock=clk, **shape)
    torch.cuda.synchronize()
    c = clk.cpu().numpy()
    hz = B.md_wall_clock_hz(batch.reals.device.index or 0)
    return (c[:, 1] - c[:, 0]) / hz


def tune_batch(batch: B.BatchedPaths, iters: int, blocks=(256, 512), grid_factors=(1, 2, 4),
               reps: int = 1, stream=None, use_cache: bool = True) -> dict:
    """Measure the candidates and set the fastest order on the batch;
    returns {"best": {...}, "trials": [...]}.  The batch's series are
    restored to their start values."""
    key = signature(batch, iters)
    if use_cache and key in _cache:
        res = _cache[key]
        batch.set_order(res["order"])
        batch.restore()
        return res
    stream = stream or torch.cuda.current_stream()
    cus = torch.cuda.get_device_properties(batch.reals.device).multi_processor_count
    orders = {"analytic": np.argsort(-batch.cost, kind="stable")}
    dur = measured_durations(batch, iters, stream)
    orders["measured"] = np.argsort(-dur, kind="stable")
    trials = []
    for oname, order in orders.items():
        batch.set_order(order)
        for block in blocks:
            for gf in grid_factors:
                grid = max(1, gf * cus * 256 // block)
                for ew in eval_wave_choices(batch, block):
                    ms = _time(batch, iters, stream, reps, grid=grid, block=block, eval_waves=ew)
                    trials.append({"order": oname, "block": block, "grid": grid,
                                   "eval_waves": ew, "ms": round(ms, 3)})
    best = min(trials, key=lambda t: t["ms"])
    batch.set_order(orders[best["order"]])
    batch.restore()
    res = {"best": best, "trials": trials, "order": orders[best["order"]],
           "path_seconds": {"max": float(dur.max()), "sum": float(dur.sum())}}
    _cache[key] = res
    return res
