"""Launch-shape and schedule tuner for the batched persistent Newton launch.

md_newton_batch takes a launch shape (threads per workgroup, number of
persistent workgroups, waves per workgroup that evaluate terms) and a job
schedule.  Every choice gives the same bits; only the time changes.  The
tuner measures on the device:

  * the job order of one queue: longest first by the analytic operation
    count (Table 1 weights of the md operations of one Newton step), or
    longest first by the duration of every path measured with the device
    wall clock in a first run (list scheduling of the longest jobs first:
    the paper's job queue with a better order);
  * one queue per accelerator die, the paths spread over the dies by their
    measured durations, and the longest paths split into gangs of 2 or 4
    workgroups of one die (so that no single path outlasts the rest);
  * the shape: 256 threads with one or two workgroups per compute unit, or
    512 threads with one, and as many evaluating waves as the LDS allows.

It keeps the fastest and leaves that schedule set on the batch.  Results are
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
    return [fits[-1]]


def measured_durations(batch, iters, stream=None, **shape) -> np.ndarray:
    """Device wall-clock duration (seconds) of every path in one run."""
    clk = torch.zeros((batch.npaths, 2), dtype=torch.int64, device=batch.reals.device)
    batch.restore()
    B.md_newton_batch(batch, iters, stream=stream, path_clock=clk, **shape)
    torch.cuda.synchronize()
    c = clk.cpu().numpy()
    hz = B.md_wall_clock_hz(batch.reals.device.index or 0)
    return (c[:, 1] - c[:, 0]) / hz


def gang_sizes(dur: np.ndarray, workers: int, factor: float) -> np.ndarray:
    """2 workgroups for a path longer than `factor` times the mean load per
    workgroup, 4 beyond twice that."""
    mean = dur.sum() / workers
    G = np.ones(dur.shape[0], dtype=np.int64)
    G[dur > factor * mean] = 2
    G[dur > 2 * factor * mean] = 4
    return G


def tune_batch(batch: B.BatchedPaths, iters: int, shapes=((256, 1), (256, 2), (512, 1)),
               gang_factors=(0.5, 0.7, 0.9, 1.2), reps: int = 1, stream=None,
               use_cache: bool = True) -> dict:
    """Measure the candidates and set the fastest schedule on the batch;
    returns {"best": {...}, "trials": [...]}.  The batch's series are
    restored to their start values."""
    key = signature(batch, iters)
    if use_cache and key in _cache:
        res = _cache[key]
        batch.set_schedule(**res["schedule"])
        batch.restore()
        return res
    stream = stream or torch.cuda.current_stream()
    cus = torch.cuda.get_device_properties(batch.reals.device).multi_processor_count
    dur = measured_durations(batch, iters, stream, block=512, grid=cus)
    schedules = {
        "analytic": {"order": np.argsort(-batch.cost, kind="stable")},
        "measured": {"order": np.argsort(-dur, kind="stable")},
    }
    dies = B.md_device_dies(batch.reals.device.index or 0)
    for f in gang_factors:
        schedules[f"dies+gangs{f}"] = {"nq": dies, "weights": dur,
                                       "gangs": gang_sizes(dur, cus, f)}
    trials = []
    for sname, sched in schedules.items():
        batch.set_schedule(**sched)
        for block, per_cu in shapes:
            grid = per_cu * cus
            if grid < batch.nq * int(batch.gangs.max(initial=1)):
                continue
            for ew in eval_wave_choices(batch, block):
                ms = _time(batch, iters, stream, reps, grid=grid, block=block, eval_waves=ew)
                st = int(batch.status.max().item())
                trials.append({"schedule": sname, "block": block, "grid": grid,
                               "eval_waves": ew, "ms": round(ms, 3), "status": st})
    good = [t for t in trials if t["status"] == 0] or trials
    best = min(good, key=lambda t: t["ms"])
    sched = schedules[best["schedule"]]
    batch.set_schedule(**sched)
    batch.restore()
    res = {"best": best, "trials": trials, "schedule": sched,
           "gangs": {int(g): int((batch.gangs == g).sum()) for g in np.unique(batch.gangs)},
           "path_seconds": {"max": float(dur.max()), "sum": float(dur.sum())}}
    _cache[key] = res
    return res
