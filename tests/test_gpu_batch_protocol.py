"""Section 6's protocol in the batched persistent launch
(md_newton_batch_protocol): per-path step counts and series against the
oracle's protocol, the same bits under other schedules and gang splits
(the decisions of a gang are shared through the path's workspace), and
the later degrees skipped after a divergence."""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from exact import fval, planes_rel_err_per_k as rel_err_per_k
from paper_2012_06607_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEG, MAXIT, TOL = (4, 8, 16), (8, 8, 8), 1e-32


@pytest.fixture(scope="module")
def B():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2012_06607_amd import binding
    binding.lib()
    return binding


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def paths_for(count=8, seed=0):
    specs = I.batch_specs((1600, seed), count, n_choices=(3, 5, 8, 12, 17), d_range=(16, 16),
                          m_choices=(2, 4))
    out = []
    for s in specs:
        sysm, x0 = I.newton_system((1601, s.path), s.n, s.m, terms=4, max_deg=3)
        out.append((sysm, x0, I.series_start(x0, 16)))
    return out


def borderline(sysm, x0, iters, bits=10):
    for d, it in zip(DEG, iters):
        if it == 0:
            continue
        _, nl, _ = oracle.newton(sysm, I.series_start(x0, d), it)
        for v in nl[1:]:
            val = abs(float(fval(v[:, 0])))
            if val > 0 and abs(math.log2(val / TOL)) <= bits:
                return True
    return False


def test_batch_protocol_against_oracle_and_schedules(B):
    sample = paths_for()
    batch = B.BatchedPaths([(s, x) for s, _, x in sample], protocol=True)
    it1, nr1 = B.md_newton_batch_protocol(batch, DEG, MAXIT)
    st = host(batch.status)
    # a double-double path whose series grows fast ends degree 16 above the
    # bound (as in Table 2's rows); nothing else may be flagged
    assert not (st & ~B.MD_ST_DIVERGED).any(), st
    it1, nr1 = host(it1), host(nr1)
    x1 = [host(batch.x(p)).copy() for p in range(len(sample))]
    # another schedule: per-die queues, the two longest paths as gangs of 2
    batch.restore()
    gangs = np.ones(len(sample), dtype=np.int64)
    gangs[np.argsort(-batch.cost)[:2]] = 2
    batch.set_schedule(nq=B.md_device_dies(), gangs=gangs)
    it2, nr2 = B.md_newton_batch_protocol(batch, DEG, MAXIT, block=256)
    assert np.array_equal(host(batch.status), st)
    assert np.array_equal(host(it2), it1) and np.array_equal(host(nr2), nr1)
    for p in range(len(sample)):
        assert np.array_equal(host(batch.x(p)), x1[p]), p
    # against the oracle's protocol
    for p, (sysm, x0, _) in enumerate(sample):
        xo, ito, no, sto = oracle.newton_protocol(sysm, x0, DEG, MAXIT, TOL, 1.0)
        print(f"path {p} m={sysm.m} n={sysm.n}: gpu steps {list(it1[p])}, oracle {ito}, "
              f"status {st[p]} / {sto}", flush=True)
        assert st[p] == sto, p
        if not borderline(sysm, x0, ito):
            assert list(it1[p]) == ito, p
        if list(it1[p]) == ito:
            cond = sysm.meta["cond_A0_double"]
            e = rel_err_per_k(x1[p], xo)
            for k in range(17):
                assert e[k] <= 2.0 ** -(53 * sysm.m - 8 - math.log2(cond) - math.log2(k + 1) - 4), (p, k, e)


def test_batch_protocol_divergence(B):
    """A divergence bound below what degree 4 ends with for every path: the
    later degrees are not run, each path is flagged MD_ST_DIVERGED, and x
    holds degree 4's series."""
    sample = paths_for(count=4, seed=1)
    batch = B.BatchedPaths([(s, x) for s, _, x in sample], protocol=True)
    it, nr = B.md_newton_batch_protocol(batch, DEG, MAXIT, diverge=1e-300)
    st = host(batch.status)
    it = host(it)
    for p, (sysm, x0, _) in enumerate(sample):
        if it[p, 0] == 0 or not host(nr)[p, 0].any():
            continue  # degree 4 ended with an update of exactly zero (not above the bound)
        assert st[p] == B.MD_ST_DIVERGED, (p, st[p])
        assert it[p, 1] == 0 and it[p, 2] == 0
        xw, _, _, _ = oracle.newton_protocol(sysm, x0, DEG, MAXIT, TOL, 1e-300)
        xg = host(batch.x(p))
        assert not xg[:, :, 5:].any()
        e = rel_err_per_k(xg[:, :, :5], xw[:, :, :5])
        assert e.max() <= 2.0 ** -(53 * sysm.m - 30), (p, e)
