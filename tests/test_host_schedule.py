"""Host logic of the batched launch, on the CPU: the job lists that
BatchedPaths.set_schedule builds (queues, gangs, members), the tuner's gang
rule, and the benchmark's CPU-baseline pool (the job queue of Section 5 on
worker processes)."""
import numpy as np
import pytest

from paper_2012_06607_amd import binding as B
from paper_2012_06607_amd import inputs as I
from paper_2012_06607_amd.tune import gang_sizes


def tiny_paths(count=6):
    specs = I.batch_specs((993, 0), count, n_choices=(3, 5, 8), d_range=(1, 4), m_choices=(1, 2))
    out = []
    for s in specs:
        sysm, x0 = I.newton_system((994, s.path), s.n, s.m, terms=3, max_deg=2)
        out.append((sysm, I.series_start(x0, s.d)))
    return out


def job_table(batch):
    jobs = batch.jobs.cpu().numpy().reshape(-1, 2)[:batch.njobs]
    qb = batch.qbegin.cpu().numpy()
    return jobs, qb


def test_default_schedule_is_one_queue_longest_first():
    paths = tiny_paths()
    batch = B.BatchedPaths(paths, device="cpu")
    jobs, qb = job_table(batch)
    assert batch.nq == 1 and list(qb) == [0, len(paths)]
    assert sorted(jobs[:, 0].tolist()) == list(range(len(paths)))
    assert np.all(jobs[:, 1] == (1 << 8))            # gangs of one, member 0
    cost = batch.cost[jobs[:, 0]]
    assert np.all(np.diff(cost) <= 0)                # longest first


def test_queues_and_gangs():
    paths = tiny_paths(9)
    batch = B.BatchedPaths(paths, device="cpu")
    G = np.array([1, 2, 1, 4, 1, 1, 2, 1, 1])
    w = np.arange(1, 10, dtype=float)[::-1].copy()
    batch.set_schedule(nq=3, gangs=G, weights=w)
    jobs, qb = job_table(batch)
    assert batch.nq == 3 and len(qb) == 4 and qb[0] == 0 and qb[-1] == len(jobs)
    assert np.all(np.diff(qb) >= 0)
    assert len(jobs) == G.sum()
    load = np.zeros(3)
    for q in range(3):
        qj = jobs[qb[q]:qb[q + 1]]
        i = 0
        while i < len(qj):
            p, code = int(qj[i, 0]), int(qj[i, 1])
            g = code >> 8
            assert g == G[p] and (code & 0xff) == 0
            # a gang's members follow one another in one queue, numbered 0..G-1
            for r in range(g):
                assert int(qj[i + r, 0]) == p and int(qj[i + r, 1]) == (g << 8) | r
            load[q] += w[p]
            i += g
        # each queue runs its paths longest first
        firsts = [int(qj[k, 0]) for k in range(len(qj)) if (int(qj[k, 1]) & 0xff) == 0]
        assert all(w[a] >= w[b] for a, b in zip(firsts, firsts[1:]))
    # longest first onto the least loaded queue: within one largest weight
    assert load.max() - load.min() <= w.max()
    # every path is in exactly one queue
    assert sorted(int(p) for p, c in jobs if (c & 0xff) == 0) == list(range(len(paths)))


def test_explicit_order_and_errors():
    paths = tiny_paths(5)
    batch = B.BatchedPaths(paths, device="cpu")
    order = [3, 1, 4, 0, 2]
    batch.set_order(order)
    jobs, qb = job_table(batch)
    assert jobs[:, 0].tolist() == order and list(qb) == [0, 5]
    with pytest.raises(B.MdError):
        batch.set_order([0, 1, 2, 3, 3])
    with pytest.raises(B.MdError):
        batch.set_schedule(order=order, nq=2)
    with pytest.raises(B.MdError):
        batch.set_schedule(gangs=[1, 1, 33, 1, 1])
    with pytest.raises(B.MdError):
        batch.set_schedule(gangs=[1, 1, 1])
    with pytest.raises(B.MdError):
        batch.set_schedule(nq=65)


def test_gang_rule():
    dur = np.array([1.0, 1.0, 1.0, 1.0, 9.0, 20.0])   # total 33, mean per worker 11 on 3 workers
    G = gang_sizes(dur, workers=3, factor=0.5)       # > 5.5: gang of 2, > 11: gang of 4
    assert G.tolist() == [1, 1, 1, 1, 2, 4]
    assert gang_sizes(dur, workers=3, factor=2.0).tolist() == [1, 1, 1, 1, 1, 1]


def test_cpu_baseline_pool():
    import sys, os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    paths = tiny_paths(4)
    r = bench.cpu_baseline(paths, 0.3, 2)
    assert r["kind"] == "oracle" and r["cores"] == 2 and r["unit"] == "Newton steps/s"
    assert r["value"] > 0 and "2 worker processes" in r["sample"]


def test_batch_refuses_paths_the_kernel_does_not_carry():
    """BatchedPaths refuses, on the host, a path above 64 equations, with
    N < n, with a limb count no batched kernel carries, or of both classes
    of precision at once, so that md_newton_batch is never given one (its
    kernel would only flag it MD_ST_BADPATH)."""
    paths = tiny_paths(3)
    m, n = 2, 70
    one = ([1.0] + [0.0] * (m - 1), [0.0] * m)
    mone = ([-1.0] + [0.0] * (m - 1), [0.0] * m)
    big = I.build_system(n, n, m, 0, [[((i,), [one]), ((), [mone])] for i in range(n)])
    with pytest.raises(B.MdError, match="N <= 64"):
        B.BatchedPaths(paths + [(big, np.zeros((2, m, 3, n)))], device="cpu")
    # fewer equations than unknowns
    under = I.build_system(2, 3, m, 0, [[((0,), [one]), ((), [mone])],
                                        [((1, 2), [one]), ((), [mone])]])
    with pytest.raises(B.MdError, match="n <= N"):
        B.BatchedPaths([(under, np.zeros((2, m, 3, 3)))], device="cpu")
    # penta double next to double-double paths: the two classes of
    # precision run in separate launches
    sys5, x5 = I.newton_system((995, 0), 3, 5, terms=3, max_deg=2)
    with pytest.raises(B.MdError, match="separate launches"):
        B.BatchedPaths(paths + [(sys5, I.series_start(x5, 2))], device="cpu")
    # penta and octo double have a kernel each: not in one batch; two octo
    # double paths are
    sys8, x8 = I.newton_system((995, 1), 3, 8, terms=3, max_deg=2)
    with pytest.raises(B.MdError, match="separate launches"):
        B.BatchedPaths([(sys5, I.series_start(x5, 2)), (sys8, I.series_start(x8, 3))],
                       device="cpu")
    hb = B.BatchedPaths([(sys8, I.series_start(x8, 2)), (sys8, I.series_start(x8, 3))],
                        device="cpu")
    assert hb.max_m == 8
    # a limb count no kernel carries
    sys6, x6 = I.newton_system((995, 2), 3, 6, terms=3, max_deg=2)
    with pytest.raises(B.MdError, match="m=6"):
        B.BatchedPaths([(sys6, I.series_start(x6, 2))], device="cpu")
    # the largest accepted shapes pass, and the batch records its maxima
    batch = B.BatchedPaths(paths, device="cpu")
    assert batch.max_N == max(s.N for s, _ in paths) and batch.max_m <= 4
