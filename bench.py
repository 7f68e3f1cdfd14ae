#!/usr/bin/env python3
"""Throughput of the multiple-double series Newton path on one MI355X.

Headline workload (one "step" = one pass over one batch of paths): 1024
independent paths, n uniform in {8, 16, ..., 64}, d uniform in 8..32, half
double double and half quad double, each a system of n equations with 8
monomials of degree <= 3, a constant and a t-term per equation and a root
at t = 0, 4 Newton steps per path (evaluation and differentiation, QR of
A_0, staggered solve, update), all in one persistent launch captured in a
graph.  Inputs are seeded, synthetic and resident in HBM before timing.
The value is Newton steps per second (paths x 4 per launch / launch time).

The same JSON line also carries: the roofline of the launch's only kernel
(Table 1 operations per launch against the FP64 vector peak, and its HBM
traffic from hardware counters), the per-path launch loop on the same
paths, the single 32-unknown quad-double step (eval + QR + solve), the
adjoint of a converged 32-unknown quad-double series, and the CPU oracle
timed on a sample of the same paths.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "multiple-double series Newton steps/s and % of FP64 vector peak"
ITERS = 4
WORKLOAD = ("1024 paths, n in {8,...,64}, d in 8..32, half double double / half quad double, "
            "8 monomials of degree <= 3 + constant + t-term per equation, 4 Newton steps per "
            "path, one persistent launch in a graph")
M1, N1, D1 = 4, 32, 16    # the single-path step

# HBM traffic of one launch from two rocprofv3 --pmc runs of this script
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch), each scaled by what the
# same counter reads for a plain 256 MiB device copy in the same run
# (--copy-mib 256).  Valid only for the kernel sources the counters were
# taken on: dropped (null) when their hash differs.
TRAFFIC = {
    "k_newton_batch": {"fetch_kib": 67959790.292, "fetch_scale": 262144 / 131088.1875,
                       "write_kib": 31923831.896, "write_scale": 262144 / 262144.0,
                       "sha256": "b9b1149694b5c75d377144884ac50a33f96673b82af69c672ee5c76795e76a75",
                       "sources": ('batch.hip', 'batch_kernel.hpp', 'gang.hpp', 'internal.hpp', 'common.hpp', 'md.hpp', 'wg.hpp', 'layout.hpp', 'series.hpp')},
    "k_qr": {"fetch_kib": 106.0625, "fetch_scale": 262144 / 131088.625, "write_kib": 67.0,
             "write_scale": 262144 / 262145.125,
             "sha256": "4c94538ad3b2f3cc03c2db639b07175c83e56dcce9dd25e55e71355aa08d3fde",
             "sources": ('qr.hip', 'gang.hpp', 'internal.hpp', 'common.hpp', 'md.hpp', 'wg.hpp', 'layout.hpp', 'series.hpp')},
}


def traffic_bytes(kernel: str):
    """Measured HBM bytes per launch, or None once the kernel's sources changed."""
    t = TRAFFIC[kernel]
    if t["fetch_kib"] is None:
        return None
    h = hashlib.sha256()
    for name in t["sources"]:
        with open(os.path.join(ROOT, "paper_2012_06607_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != t["sha256"]:
        return None
    return int(round(1024 * (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"])))


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed launches (graph replays)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--paths", type=int, default=1024)
    ap.add_argument("--cpu-seconds", type=float, default=12.0,
                    help="wall time budget of the CPU oracle baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=min(16, os.cpu_count() or 1),
                    help="oracle worker processes of the CPU baseline (default: the host's "
                         "cores, at most 16)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the launch-shape tuner (512 threads, one workgroup per CU)")
    ap.add_argument("--gang-factor", type=float, default=None,
                    help="skip the tuner's trials: one queue per die, gangs for paths longer "
                         "than this factor times the mean load per CU (durations measured in "
                         "one run), 512 threads, one workgroup per CU")
    ap.add_argument("--no-loop", action="store_true", help="skip the per-path launch loop")
    ap.add_argument("--no-single", action="store_true",
                    help="skip the single-path step (32 unknowns, d = 16, quad double)")
    ap.add_argument("--single-steps", type=int, default=50)
    ap.add_argument("--no-high-precision", action="store_true",
                    help="skip the octo / deca double step at 64 unknowns, d = 32")
    ap.add_argument("--hp-reps", type=int, default=3)
    ap.add_argument("--no-next", action="store_true",
                    help="skip the least-squares, protocol, division and Pade measurements")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="skip the adjoint measurement (32 unknowns, d = 16, quad double)")
    ap.add_argument("--adj-reps", type=int, default=20)
    ap.add_argument("--efficiency", action="store_true",
                    help="instead of the headline: the efficiency study of Section 7 (64 "
                         "polynomials with 64 monomials each, degrees 8, 16, 32, seven "
                         "precisions), one Newton step of one system on a gang of G = 1, 2, "
                         "4, 8, 16, 32 workgroups; prints one JSON line")
    ap.add_argument("--eff-reps", type=int, default=3)
    ap.add_argument("--eff-precisions", type=str, default="1,2,3,4,5,8,10")
    ap.add_argument("--eff-degrees", type=str, default="8,16,32")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="before timing, run one plain device copy of this many MiB (a "
                         "reference of known traffic for hardware byte counters)")
    return ap.parse_args()


def make_paths(count):
    from paper_2012_06607_amd import inputs as I
    specs = I.batch_specs((4, 0), count)
    paths = []
    for sp in specs:
        sysm, x0 = I.newton_system((4, sp.path), sp.n, sp.m)
        paths.append((sysm, I.series_start(x0, sp.d)))
    return paths


_POOL = {}


def _oracle_worker(w: int):
    """One worker of the CPU baseline: take the next job from the shared
    counter (job j is path 37 j mod the batch size), run ITERS oracle Newton
    steps on it, until the time budget is spent; returns (steps, seconds,
    paths done)."""
    import oracle
    paths, counter, budget, stride = (_POOL[k] for k in ("paths", "counter", "budget", "stride"))
    t0 = time.perf_counter()
    steps, done = 0, []
    while time.perf_counter() - t0 < budget:
        with counter.get_lock():
            j = counter.value
            counter.value += 1
        q = (j * stride) % len(paths)
        sysm, x = paths[q]
        oracle.newton(sysm, x, ITERS)
        steps += ITERS
        done.append(q)
    return steps, time.perf_counter() - t0, done


def cpu_baseline(paths, budget_s: float, workers: int) -> dict:
    """The oracle on a sample of the same paths: `workers` processes take
    paths from one shared job counter (the job queue of Section 5), each
    path ITERS Newton steps, until the time budget is spent.  The rate is
    the sum of the workers' own rates (steps over each worker's busy time).
    Runs before anything touches the GPU: the workers are forked."""
    import multiprocessing as mp

    import oracle
    oracle.build()
    oracle.lib()
    ctx = mp.get_context("fork")
    _POOL.update(paths=paths, counter=ctx.Value("i", 0), budget=budget_s, stride=37)
    t0 = time.perf_counter()
    with ctx.Pool(workers) as pool:
        res = pool.map(_oracle_worker, range(workers), chunksize=1)
    wall = time.perf_counter() - t0
    steps = sum(r[0] for r in res)
    rate = sum(r[0] / r[1] for r in res if r[1] > 0)
    done = sorted({q for r in res for q in r[2]})
    ns = sorted({paths[q][0].n for q in done})
    ms = sorted({paths[q][0].m for q in done})
    return {"value": round(rate, 3), "unit": "Newton steps/s", "cores": workers, "kind": "oracle",
            "sample": f"{len(done)} paths of the batch (job j = path 37 j mod {len(paths)}; n in "
                      f"{ns}, m in {ms}), {ITERS} Newton steps each, {steps} steps in {wall:.1f} s "
                      f"wall on {workers} worker processes sharing one job counter; gcc -O2 C "
                      f"oracle; rate = sum of per-worker steps/busy seconds"}


def batched(args, B, OC, paths):
    import numpy as np
    import torch
    batch = B.BatchedPaths(paths)
    stream = torch.cuda.current_stream()
    ops = sum(ITERS * OC.newton_step(sysm, x.shape[2] - 1, sysm.m).table_ops(sysm.m)
              for sysm, x in paths)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    if args.no_tune or args.gang_factor is not None:
        shape = {"grid": cus, "block": 512, "eval_waves": 8}
        while shape["eval_waves"] > 1 and B.md_batch_lds_bytes(
                batch.max_m, batch.max_d, batch.max_deg, shape["eval_waves"]) > B.md_device_lds_bytes():
            shape["eval_waves"] -= 1
        tuned = None
        if args.gang_factor is not None:
            from paper_2012_06607_amd.tune import gang_sizes, measured_durations
            dur = measured_durations(batch, ITERS, stream, **shape)
            batch.set_schedule(nq=B.md_device_dies(), weights=dur,
                               gangs=gang_sizes(dur, cus, args.gang_factor))
    else:
        from paper_2012_06607_amd.tune import tune_batch
        tuned = tune_batch(batch, ITERS, stream=stream)
        shape = {k: tuned["best"][k] for k in ("grid", "block", "eval_waves")}
    B.md_newton_batch(batch, ITERS, stream=stream, **shape)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        B.md_newton_batch(batch, ITERS, **shape)
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        batch.restore()
        g.replay()
    torch.cuda.synchronize()
    times = []
    for _ in range(args.steps):
        batch.restore()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g.replay()
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = float(np.mean(times))
    phases = phase_breakdown(B, batch, ITERS, shape, stream)
    res = {"ms": ms, "ops": ops, "shape": shape, "times": times, "phases": phases,
           "status": int(batch.status.max().item()), "tuned": tuned, "batch": batch,
           "qd_share": sum(ITERS * OC.newton_step(s, x.shape[2] - 1, s.m).table_ops(s.m)
                           for s, x in paths if s.m == 4) / ops}
    if not args.no_loop:
        sds = [B.DeviceSystem(sysm) for sysm, _ in paths]
        xs = [torch.as_tensor(x, device="cuda") for _, x in paths]
        wss = [B.workspace(B.MD_FN_NEWTON, sysm.m, sysm.N, sysm.n, x.shape[2] - 1, sysm.M,
                           sysm.max_deg) for sysm, x in paths]
        stat = torch.zeros(1, dtype=torch.int32, device="cuda")
        nrm = [torch.empty((sysm.m, 2), dtype=torch.float64, device="cuda") for sysm, _ in paths]

        def loop():
            for p in range(len(paths)):
                for _ in range(ITERS):
                    B.md_newton_step(sds[p], xs[p], nrm[p], wss[p], stat, stream)
        loop()
        torch.cuda.synchronize()
        for p, (_, x) in enumerate(paths):
            xs[p].copy_(torch.as_tensor(x))
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        loop()
        e1.record(stream)
        torch.cuda.synchronize()
        res["loop_ms"] = e0.elapsed_time(e1)
        # largest difference between the two, per coefficient, relative to
        # the coefficient vector's size, in units of 2^-(53m-8)
        worst = 0.0
        for p, (sysm, _) in enumerate(paths):
            a, b = xs[p].cpu().numpy(), batch.x(p).cpu().numpy()
            diff = np.abs((a - b).sum(axis=1)).max(axis=(0, 2))     # per k, limb sums
            size = np.maximum(np.abs(a[:, 0]).max(axis=(0, 2)), 1e-300)
            worst = max(worst, float((diff / size).max()) / 2.0 ** -(53 * sysm.m - 8))
        res["diff_units"] = worst
    return res


PHASES = ("evaluation", "sums into f and A", "QR", "R^-1 Q^H", "stages", "update")


def phase_breakdown(B, batch, iters, shape, stream) -> dict:
    """One more launch (outside any timed region) with the kernel's phase
    clocks on: the device wall-clock seconds each phase took, summed over
    the paths (member 0 of each path measures; a phase ends at a barrier),
    split by precision."""
    import numpy as np
    import torch
    clk = torch.zeros((batch.npaths, 8), dtype=torch.int64, device="cuda")
    batch.restore()
    B.md_newton_batch(batch, iters, stream=stream, phase_clock=clk, **shape)
    torch.cuda.synchronize()
    hz = B.md_wall_clock_hz()
    c = clk.cpu().numpy()[:, :len(PHASES)] / hz
    ms_ = np.array([m for (m, _, _, _) in batch.meta])
    out = {"total_s": {ph: round(float(c[:, i].sum()), 4) for i, ph in enumerate(PHASES)}}
    for m in sorted(set(ms_.tolist())):
        out[f"m{m}_s"] = {ph: round(float(c[ms_ == m, i].sum()), 4) for i, ph in enumerate(PHASES)}
    return out


def solve_eval(B, OC, m: int, n: int, d: int, key: int, reps: int, warm: int) -> dict:
    """One path's linear-algebra step at m limbs: md_poly_eval_diff on an
    n x n system (16 monomials of degree <= 4 per equation) at a unit
    series point, md_qr_gang of an n x n A_0 with condition number 1e3 (the
    QR spread over several workgroups, as md_newton_step runs it), and
    md_series_solve at degree d; mean of `reps` timed repetitions.  The
    one-workgroup md_qr of the same A_0 is timed apart (dur["md_qr"])."""
    import numpy as np
    import torch
    from paper_2012_06607_amd import inputs as I
    sysm = I.eval_system((key, 0), n, n, m, 16, 4)
    x = torch.as_tensor(I.unit_series((key, 1), m, d, n), device="cuda")
    A_h, b_h = I.toeplitz_system((key, n), n, d, m)
    A = torch.as_tensor(A_h, device="cuda")
    b = torch.as_tensor(b_h, device="cuda")
    sd = B.DeviceSystem(sysm)
    A0 = A[:, :, 0].contiguous()
    f = torch.empty((2, m, d + 1, n), dtype=torch.float64, device="cuda")
    Aev = torch.empty((2, m, d + 1, n, n), dtype=torch.float64, device="cuda")
    dx = torch.empty((2, m, d + 1, n), dtype=torch.float64, device="cuda")
    ws_eval = B.workspace(B.MD_FN_EVAL, m, n, n, d, sysm.M, sysm.max_deg)
    ws_solve = B.workspace(B.MD_FN_SOLVE, m, n, n, d, 0, 0)
    QRb = torch.empty_like(A0)
    vdb = torch.empty((2, m, n), dtype=torch.float64, device="cuda")
    betab = torch.empty((m, n), dtype=torch.float64, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    sync = torch.zeros(1, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        B.md_poly_eval_diff(sd, x, f, Aev, ws_eval, stream)
        if ev is not None:
            ev[1].record(stream)
        QR, vd, beta, _ = B.md_qr_gang(A0, status, stream, QRb, vdb, betab, sync)
        if ev is not None:
            ev[2].record(stream)
        B.md_series_solve(QR, vd, beta, A, b, dx, ws_solve, status, stream)
        if ev is not None:
            ev[3].record(stream)

    for _ in range(warm):
        step()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(reps)]
    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    for r in range(reps):
        step(evs[r])
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / reps
    names = ("md_poly_eval_diff", "md_qr_gang", "md_series_solve")
    dur = {nm: float(np.mean([evs[r][i].elapsed_time(evs[r][i + 1]) for r in range(reps)]))
           for i, nm in enumerate(names)}
    # the one-workgroup factorisation of the same matrix
    q0, q1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    q0.record(stream)
    for _ in range(reps):
        B.md_qr(A0, status, stream, QRb, vdb, betab)
    q1.record(stream)
    torch.cuda.synchronize()
    dur["md_qr"] = q0.elapsed_time(q1) / reps
    ops = {"md_poly_eval_diff": OC.eval_diff(sysm, d).table_ops(m),
           "md_qr_gang": OC.qr(n, n, m).table_ops(m),
           "md_series_solve": OC.series_solve(n, n, d).table_ops(m)}
    return {"ms": ms, "dur": dur, "ops": ops, "status": int(status.item())}


def single_path(args, B, OC) -> dict:
    """The 32-unknown quad-double step on one path (d = 16)."""
    r = solve_eval(B, OC, M1, N1, D1, 2, args.single_steps, 5)
    ms, dur, ops = r["ms"], r["dur"], r["ops"]
    qr_tf = ops["md_qr_gang"] / (dur["md_qr"] * 1e-3) / 1e12
    gang_tf = ops["md_qr_gang"] / (dur["md_qr_gang"] * 1e-3) / 1e12
    return {
        "workload": "qd, n = N = 32, d = 16: eval/diff of a 32x32 system (16 monomials of "
                    "degree <= 4 per equation) + QR of A_0 (cond 1e3) + staggered solve",
        "steps_per_s": round(1000.0 / ms, 3), "ms_per_step": round(ms, 4),
        "pct_fp64_vector_peak": round(100.0 * sum(ops.values()) / (ms * 1e-3)
                                      / OC.FP64_VECTOR_PEAK, 4),
        "kernels_ms": {k: round(v, 4) for k, v in dur.items()},
        "evals_per_s": round(1000.0 / dur["md_poly_eval_diff"], 2),
        "solves_per_s": round(1000.0 / (dur["md_qr_gang"] + dur["md_series_solve"]), 2),
        "k_qr_roofline": {"bound": "alu", "achieved": round(qr_tf, 5), "peak": 78.6,
                          "unit": "TFLOP/s", "frac": round(qr_tf / 78.6, 6),
                          "traffic": traffic_bytes("k_qr")},
        # the spread form md_newton_step uses (the look-ahead column on
        # four waves); traffic: the profile's counters, not taken here
        "k_qr_gang4_roofline": {"bound": "alu", "achieved": round(gang_tf, 5), "peak": 78.6,
                                "unit": "TFLOP/s", "frac": round(gang_tf / 78.6, 6),
                                "workgroups": B.md_qr_gang_size(M1, N1, N1), "traffic": None},
        "status": r["status"],
    }


def high_precision(args, B, OC) -> dict:
    """Octo and deca double at n = 64, d = 32: the eval + QR + solve of one
    path, the 2-norm of 64 unit complex numbers (Section 2: exactly 8) and
    64 series products of 33 coefficients."""
    import torch
    from paper_2012_06607_amd import inputs as I
    out = {"workload": "od and da, n = N = 64, d = 32: eval/diff of a 64x64 system (16 "
                       "monomials of degree <= 4 per equation) + QR of A_0 (cond 1e3) + "
                       "staggered solve; 2-norm of 64 unit complex numbers; 64 convolutions "
                       "of 33-coefficient series"}
    stream = torch.cuda.current_stream()
    for m, name in ((8, "od"), (10, "da")):
        r = solve_eval(B, OC, m, 64, 32, 3, args.hp_reps, 1)
        ms, dur, ops = r["ms"], r["dur"], r["ops"]
        xs = torch.as_tensor(I.unit_complex(I.rng(3, m, 1), m, 64, 33), device="cuda")
        ys = torch.as_tensor(I.unit_complex(I.rng(3, m, 2), m, 64, 33), device="cuda")
        z = B.md_series_convolve(xs, ys)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(10):
            B.md_series_convolve(xs, ys, z)
        e1.record(stream)
        torch.cuda.synchronize()
        conv_ms = e0.elapsed_time(e1) / 10
        conv_ops = OC.convolve(32, 64).table_ops(m)
        nrm = B.md_norm2(torch.as_tensor(I.unit_complex(I.rng(951, m), m, 64), device="cuda"))
        torch.cuda.synchronize()
        gang = gang_step(B, OC, m, args.hp_reps)
        out[name] = {
            "ms_per_step": round(ms, 3),
            "kernels_ms": {k: round(v, 3) for k, v in dur.items()},
            "evals_per_s": round(1000.0 / dur["md_poly_eval_diff"], 2),
            "solves_per_s": round(1000.0 / (dur["md_qr_gang"] + dur["md_series_solve"]), 2),
            "pct_fp64_vector_peak": round(100.0 * sum(ops.values()) / (ms * 1e-3)
                                          / OC.FP64_VECTOR_PEAK, 4),
            "qr_workgroups": B.md_qr_gang_size(m, 64, 64),
            "convolve_64x33_ms": round(conv_ms, 4),
            "convolve_pct_fp64_vector_peak": round(100.0 * conv_ops / (conv_ms * 1e-3)
                                                   / OC.FP64_VECTOR_PEAK, 3),
            "norm2_of_64_unit_numbers_limb0": float(nrm[0, 0].item()),
            "gang_newton_step": gang,
            "status": r["status"],
        }
    return out


HP_GANG = 32


def gang_step(B, OC, m: int, reps: int) -> dict:
    """One whole Newton step (eval/diff, QR, R^{-1} Q^H, staggered solve,
    update) of the same 64 x 64 system at the same unit series point (d =
    32), as one path on a gang of HP_GANG workgroups of the persistent
    kernel (the members split terms, Jacobian rows, QR columns, columns of
    R^{-1} Q^H and right-hand-side updates); mean of `reps` launches."""
    import numpy as np
    import torch
    from paper_2012_06607_amd import inputs as I
    sysm = I.eval_system((3, 0), 64, 64, m, 16, 4)
    x = I.unit_series((3, 1), m, 32, 64)
    batch = B.BatchedPaths([(sysm, x)])
    batch.set_schedule(gangs=np.array([HP_GANG]))
    stream = torch.cuda.current_stream()
    times = []
    for rep in range(reps + 1):
        batch.restore()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        B.md_newton_batch(batch, 1, grid=HP_GANG, block=256, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        if rep:
            times.append(e0.elapsed_time(e1))
    ms = float(np.mean(times))
    ops = OC.newton_step(sysm, 32, m).table_ops(m)
    ph = phase_breakdown(B, batch, 1, {"grid": HP_GANG, "block": 256}, stream)["total_s"]
    return {"gang": HP_GANG, "ms_per_step": round(ms, 3),
            "phases_ms": {k: round(v * 1e3, 3) for k, v in ph.items()},
            "pct_fp64_vector_peak": round(100.0 * ops / (ms * 1e-3) / OC.FP64_VECTOR_PEAK, 4),
            "status": int(batch.status.max().item())}


def next_rows(args, B, OC) -> dict:
    """The rows beyond the Newton step, each on a stated synthetic workload:
    least squares (one quad-double step of a consistent 39 x 32 system, the
    square system of 32 equations plus 7 sums of pairs of them, d = 16);
    Section 6's protocol in the persistent launch (1024 paths shaped as the
    headline batch's, degrees 8, 16, 24, 32 with at most 8, 8, 12, 16 steps,
    stop at |dx_d| <= 1e-32, longest first by operation count, one queue);
    series division (64 octo-double series of 33
    coefficients) and [16/16] Pade approximants (64 quad-double series)."""
    import numpy as np
    import torch
    from paper_2012_06607_amd import inputs as I
    stream = torch.cuda.current_stream()

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {}
    # least squares: N = n + 7
    m, n, d = 4, 32, 16
    sq, x0 = I.newton_system((6, 0), n, m)
    sysm = I.augmented_system((6, 1), sq)
    sd = B.DeviceSystem(sysm)
    x = torch.as_tensor(I.series_start(x0, d), device="cuda")
    ws = B.workspace(B.MD_FN_NEWTON, m, sysm.N, n, d, sysm.M, sysm.max_deg)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    nrm = torch.zeros((m, 2), dtype=torch.float64, device="cuda")
    ms = timed(lambda: B.md_newton_step(sd, x, nrm, ws, st, stream), 5)
    ops = OC.newton_step(sysm, d, m).table_ops(m)
    out["least_squares"] = {"workload": f"qd, N = {sysm.N} equations (32 + 7 sums of pairs), "
                                        f"n = {n}, d = {d}: one md_newton_step",
                            "ms_per_step": round(ms, 4),
                            "pct_fp64_vector_peak": round(100.0 * ops / (ms * 1e-3)
                                                          / OC.FP64_VECTOR_PEAK, 4)}
    # Section 6's protocol, batched
    specs = I.batch_specs((7, 0), 1024, d_range=(32, 32))
    paths = []
    for sp in specs:
        sy, xs = I.newton_system((7, sp.path), sp.n, sp.m)
        paths.append((sy, I.series_start(xs, 32)))
    batch = B.BatchedPaths(paths, protocol=True)
    B.md_newton_batch_protocol(batch, stream=stream)
    torch.cuda.synchronize()
    batch.restore()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    its, _ = B.md_newton_batch_protocol(batch, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    pms = e0.elapsed_time(e1)
    it = its.cpu().numpy()
    stt = batch.status.cpu().numpy()
    steps = int(it.sum())
    out["protocol"] = {"workload": "1024 paths (n in 8..64, half dd / half qd, 8 monomials of "
                                   "degree <= 3 + constant + t-term per equation), degrees 8, 16, "
                                   "24, 32 with at most 8, 8, 12, 16 steps, stop at "
                                   "|dx_d| <= 1e-32, one persistent launch",
                       "ms_per_launch": round(pms, 3), "newton_steps": steps,
                       "newton_steps_per_s": round(steps / (pms * 1e-3), 1),
                       "steps_per_degree": [int(v) for v in it.sum(axis=0)],
                       "paths_flagged_diverged": int(((stt & B.MD_ST_DIVERGED) != 0).sum()),
                       "other_status_bits": int((stt & ~B.MD_ST_DIVERGED).max())}
    # series division and Pade approximants
    g = I.rng(8, 0)
    xd = torch.as_tensor(I.unit_complex(g, 8, 64, 33), device="cuda")
    yd = torch.as_tensor(I.unit_complex(g, 8, 64, 33), device="cuda")
    yd[:, :, :, 0] *= 4.0   # y_0 away from zero
    out["series_division"] = {"workload": "64 od series of 33 coefficients",
                              "ms": round(timed(lambda: B.md_series_divide(xd, yd, stream=stream),
                                                10), 4)}
    cp = torch.as_tensor(I.unit_complex(g, 4, 64, 33), device="cuda")
    out["pade"] = {"workload": "[16/16] approximants of 64 qd series of 33 coefficients",
                   "ms": round(timed(lambda: B.md_series_pade(cp, 16, 16, stream=stream), 10), 4)}
    return out


def adjoint_measure(args, B, OC) -> dict:
    """Quad double series Newton on a 32-unknown system (8 monomials of degree
    <= 3, a constant and a t-term per equation: 320 coefficients), d = 16,
    8 steps from the root at t = 0; then the coefficient gradient of
    L = sum |x_k|^2 by md_newton_adjoint with the monomial series stored and
    recomputed, each against the forward Newton step on the same GPU."""
    import numpy as np
    import torch
    from paper_2012_06607_amd import inputs as I
    m, n, d, iters = 4, 32, 16, 8
    sysm, x0 = I.newton_system((5, 0), n, m, terms=8, max_deg=3)
    sd = B.DeviceSystem(sysm)
    x = torch.as_tensor(I.series_start(x0, d), device="cuda")
    stream = torch.cuda.current_stream()
    ws_n = B.workspace(B.MD_FN_NEWTON, m, n, n, d, sysm.M, sysm.max_deg)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    # zero: each step's update is not compared with an earlier one (the
    # growth bit MD_ST_DIVERGED is expected while the series converges)
    nrm = torch.zeros((m, 2), dtype=torch.float64, device="cuda")

    def step():
        nrm.zero_()
        B.md_newton_step(sd, x, nrm, ws_n, st, stream)

    def timed(fn, reps):
        out = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            out.append(e0.elapsed_time(e1))
        return float(np.median(out))

    step()                      # one untimed step (first launches of the step's kernels)
    torch.cuda.synchronize()
    x.copy_(torch.as_tensor(I.series_start(x0, d)))
    ms_fwd = timed(lambda: [step() for _ in range(iters)], 1) / iters
    G = 2 * x
    res, grads = {}, {}
    for store in (True, False):
        fn = B.MD_FN_ADJOINT_STORE if store else B.MD_FN_ADJOINT
        ws = B.workspace(fn, m, n, n, d, sysm.M, sysm.max_deg)
        g = torch.empty((2, 2, sysm.M, sysm.dc + 1), dtype=torch.float64, device="cuda")
        B.md_newton_adjoint(sd, x, G, store, g, ws, st, stream)
        torch.cuda.synchronize()
        ms = timed(lambda: B.md_newton_adjoint(sd, x, G, store, g, ws, st, stream), args.adj_reps)
        key = "store" if store else "recompute"
        res[key] = {"ms": round(ms, 4), "workspace_bytes": int(ws.numel())}
        grads[key] = g.clone()
    ops = OC.adjoint(sysm, d, m).table_ops(m)
    return {
        "workload": "qd, n=32, d=16, 256 monomials of degree <= 3 + 32 constants + 32 t-terms "
                    "(320 coefficients), gradient of sum |x_k|^2 in double double",
        "newton_step_ms": round(ms_fwd, 4),
        "adjoint": res,
        "adjoint_over_newton_step": round(res["store"]["ms"] / ms_fwd, 3),
        "table_ops_per_adjoint": ops,
        "pct_fp64_vector_peak_store": round(
            100.0 * ops / (res["store"]["ms"] * 1e-3) / OC.FP64_VECTOR_PEAK, 4),
        "store_equals_recompute": bool(torch.equal(grads["store"], grads["recompute"])),
        "status": int(st.item()),
    }


EFF_GANGS = (1, 2, 4, 8, 16, 32)


def efficiency_study(args, B, OC) -> dict:
    """Section 7's efficiency experiment on the GPU.  The paper runs one
    Newton step of a random system of 64 polynomials with 64 monomials per
    polynomial (power series truncated at degree 8, 16, 32; double, double
    double, triple, quad, penta, octo and deca double) on p worker threads
    taking jobs from a queue, and reports efficiency = speedup / p for
    p = 2, 4, 8, 16, 32, 40.  Here the workers are the workgroups of a gang
    (one workgroup per CU) splitting the path's jobs (terms, Jacobian rows,
    columns of R^{-1} Q^H, right-hand-side updates) in the persistent
    kernel: efficiency(G) = T(1) / (G T(G)) for G = 1 .. 32 workgroups.
    Each time is the mean of `reps` launches of one Newton step (HIP events
    on the launch stream), inputs restored outside the timed region."""
    import numpy as np
    import torch
    from paper_2012_06607_amd import inputs as I
    stream = torch.cuda.current_stream()
    ms_list = [int(v) for v in args.eff_precisions.split(",")]
    ds = [int(v) for v in args.eff_degrees.split(",")]
    rows = []
    for m in ms_list:
        sysm, x0 = I.newton_system((7, 64, m), 64, m, terms=64, max_deg=3)
        for d in ds:
            x = I.series_start(x0, d)
            ops = OC.newton_step(sysm, d, m).table_ops(m)
            batch = B.BatchedPaths([(sysm, x)])
            block = 512 if m <= 4 else 256
            row = {"m": m, "d": d, "table_ops": ops, "ms": {}, "status": 0}
            for G in EFF_GANGS:
                batch.set_schedule(gangs=np.array([G]))
                times = []
                for rep in range(args.eff_reps + 1):
                    batch.restore()
                    torch.cuda.synchronize()
                    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    B.md_newton_batch(batch, 1, grid=G, block=block, stream=stream)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    if rep:
                        times.append(e0.elapsed_time(e1))
                row["status"] |= int(batch.status.max().item())
                row["ms"][G] = float(np.mean(times))
            t1 = row["ms"][1]
            row["speedup"] = {G: t1 / row["ms"][G] for G in EFF_GANGS}
            row["efficiency"] = {G: t1 / (G * row["ms"][G]) for G in EFF_GANGS}
            row["pct_peak_one_cu"] = ops / (t1 * 1e-3) / (78.6e12 / 256) * 100
            print(json.dumps({"efficiency_row": {k: row[k] for k in ("m", "d", "ms", "efficiency",
                                                                    "status")}}), flush=True)
            rows.append(row)
            del batch
            torch.cuda.empty_cache()
    return {"workload": "one Newton step of one random system: 64 polynomials in 64 "
                        "unknowns, 64 monomials of degree <= 3 per polynomial plus a constant "
                        "and a t-term, at a unit start point",
            "workers": "workgroups of one gang (one per CU), G = " + ", ".join(map(str, EFF_GANGS)),
            "rows": rows}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); this build has no "
              f"multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import torch
    if torch.cuda.device_count() < 1:   # counts devices without initialising one
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.efficiency:
        from paper_2012_06607_amd import binding as B
        from paper_2012_06607_amd import opcount as OC
        if not torch.cuda.is_available():
            print("bench.py needs a GPU", file=sys.stderr)
            sys.exit(1)
        B.lib()
        print(json.dumps({"efficiency_study": efficiency_study(args, B, OC)}), flush=True)
        return
    paths = make_paths(args.paths)
    cpu = None
    if not args.no_cpu_baseline:
        # before the GPU is initialised, so that the oracle workers can be forked
        cpu = cpu_baseline(paths, args.cpu_seconds, args.cpu_workers)

    from paper_2012_06607_amd import binding as B
    from paper_2012_06607_amd import opcount as OC
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    B.lib()
    if args.copy_mib > 0:
        src = torch.ones(args.copy_mib << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.neg(src, out=dst)   # reads and writes copy_mib MiB each
        torch.cuda.synchronize()
        del src, dst
    r = batched(args, B, OC, paths)
    ms = r["ms"]
    steps_per_launch = len(paths) * ITERS
    value = steps_per_launch / (ms * 1e-3)
    achieved = r["ops"] / (ms * 1e-3) / 1e12
    peak = OC.FP64_VECTOR_PEAK / 1e12
    line = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "Newton steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "paths": len(paths), "newton_steps_per_path": ITERS,
                   "newton_steps_per_launch": steps_per_launch,
                   "precisions": "double double (m=2) and quad double (m=4), 50/50",
                   "launch": r["shape"]},
        "pct_fp64_vector_peak": round(100.0 * achieved / peak, 3),
        "table_ops_per_step": r["ops"],
        "roofline": {"kernel": "k_newton_batch", "bound": "alu", "achieved": round(achieved, 4),
                     "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 5),
                     "traffic": traffic_bytes("k_newton_batch"),
                     "basis": "Table 1 hardware-double operations of the md operations of "
                              "every Newton step of the launch / mean launch time (HIP "
                              "events on the launch stream); traffic: HBM bytes per launch "
                              "from FETCH_SIZE + WRITE_SIZE, copy-scaled"},
        "qd_share_of_ops": round(r["qd_share"], 4),
        "phases_s": r["phases"],
        "status": r["status"],
    }
    if r.get("tuned"):
        t = r["tuned"]
        line["tuner"] = {"trials": len(t["trials"]), "best": t["best"], "gangs": t["gangs"],
                         "slowest_path_ms": round(1e3 * t["path_seconds"]["max"], 3),
                         "sum_path_ms": round(1e3 * t["path_seconds"]["sum"], 1)}
    if "loop_ms" in r:
        line["per_path_loop"] = {"ms": round(r["loop_ms"], 3),
                                 "speedup_of_batched": round(r["loop_ms"] / ms, 2),
                                 "max_diff_vs_batched_in_2^-(53m-8)_units":
                                     round(r["diff_units"], 3)}
    if not args.no_single:
        line["single_path"] = single_path(args, B, OC)
    if not args.no_adjoint:
        line["adjoint"] = adjoint_measure(args, B, OC)
    if not args.no_high_precision:
        line["high_precision"] = high_precision(args, B, OC)
    if not args.no_next:
        line["next_rows"] = next_rows(args, B, OC)
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
