"""The Newton protocol of Section 6 on the GPU (md_newton_protocol): every
degree from the start point until |dx_d| <= tol or the step limit, later
degrees skipped after one ends above the divergence bound, all decisions on
the device.  Checked against the oracle's protocol (step counts, series)
and against md_newton_step called in a host loop (the same kernels: the
same bits)."""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from exact import fval, planes_rel_err_per_k as rel_err_per_k
from paper_2012_06607_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEGREES, MAXIT, TOL = (8, 16, 24, 32), (8, 8, 12, 16), 1e-32


@pytest.fixture(scope="module")
def B():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2012_06607_amd import binding
    binding.lib()
    return binding


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def step_loop(B, sysm, x0, d, steps):
    """md_newton_step `steps` times from series_start(x0, d); (x, last norms)."""
    sd = B.DeviceSystem(sysm)
    xg = dev(I.series_start(x0, d))
    nrm = torch.zeros((sysm.m, 2), dtype=torch.float64, device="cuda")
    for _ in range(steps):
        nrm = torch.zeros((sysm.m, 2), dtype=torch.float64, device="cuda")
        B.md_newton_step(sd, xg, dx_norm=nrm)
    return host(xg), host(nrm)


def borderline(sysm, x0, degrees, iters, tol, bits=10):
    """True when the oracle's |dx_d| at some step that could decide a stop
    lies within 2^bits of tol (then the two sides may round to different
    decisions and the step counts are not compared)."""
    for d, it in zip(degrees, iters):
        _, nl, _ = oracle.newton(sysm, I.series_start(x0, d), it)
        for v in nl[1:]:
            val = abs(float(fval(v[:, 0])))
            if val > 0 and abs(math.log2(val / tol)) <= bits:
                return True
    return False


@pytest.mark.parametrize("m", (4, 8))
def test_protocol_sqrt_series(B, m):
    """x^2 - (1+t) = 0 from 1: each degree stops after ceil(log2(d+1)) + 1
    steps with the exact binomial series, as in the oracle."""
    sysm, x = I.sqrt_system(m, 16)
    xg, iters, norms, st = B.md_newton_protocol(B.DeviceSystem(sysm), dev(x[:, :, 0, :]),
                                                (4, 8, 16), (8, 8, 8))
    assert int(host(st)[0]) == 0
    assert list(host(iters)) == [4, 5, 6]
    assert not host(norms).any()
    xo, _, _, _ = oracle.newton_protocol(sysm, x[:, :, 0, :], (4, 8, 16), (8, 8, 8), 1e-32, 1.0)
    assert np.array_equal(host(xg), xo)


@pytest.mark.parametrize("m,n", ((2, 8), (4, 8), (8, 6), (10, 4)))
def test_protocol_against_oracle_and_step_loop(B, m, n):
    """A random system (the config-1 generator) through degrees 8, 16, 24,
    32 with 8, 8, 12, 16 steps at most and tolerance 1e-32: the step counts
    of the oracle's protocol, the last degree's series equal (bit for bit)
    to md_newton_step applied that many times, and within the agreement
    tolerance of the oracle's series."""
    sysm, x0 = I.newton_system((1400, m, n), n, m)
    print(f"protocol m={m} n={n}", flush=True)
    xg, iters, norms, st = B.md_newton_protocol(B.DeviceSystem(sysm), dev(x0))
    xg, iters, norms = host(xg), list(host(iters)), host(norms)
    assert int(host(st)[0]) == 0
    xo, it_o, norms_o, st_o = oracle.newton_protocol(sysm, x0, DEGREES, MAXIT, TOL, 1.0)
    print(f"  gpu steps {iters}, oracle steps {it_o}", flush=True)
    assert st_o == 0
    if not borderline(sysm, x0, DEGREES, it_o, TOL):
        assert iters == it_o
    assert all(1 <= it <= mi for it, mi in zip(iters, MAXIT))
    xs, ns = step_loop(B, sysm, x0, DEGREES[-1], iters[-1])
    assert np.array_equal(xg, xs)
    assert np.array_equal(norms[:, -1], ns[:, 0])
    if iters == it_o:
        e = rel_err_per_k(xg, xo)
        cond = sysm.meta["cond_A0_double"]
        for k in range(DEGREES[-1] + 1):
            assert e[k] <= 2.0 ** -(53 * m - 8 - math.log2(cond) - math.log2(k + 1) - 4), (k, e)


def test_protocol_divergence_skips_later_degrees(B):
    """A divergence bound below what degree 8 ends with: degrees 16, 24, 32
    are not run, MD_ST_DIVERGED is set, and x holds degree 8's series."""
    m = 2
    sysm, x0 = I.newton_system((922, 0), 6, m)
    sd = B.DeviceSystem(sysm)
    _, _, norms, _ = B.md_newton_protocol(sd, dev(x0))
    bound = float(host(norms)[0, 0]) / 2
    xg, iters, norms2, st = B.md_newton_protocol(sd, dev(x0), diverge=bound)
    assert int(host(st)[0]) == B.MD_ST_DIVERGED
    assert list(host(iters)) == [8, 0, 0, 0]
    n2 = host(norms2)
    assert np.array_equal(n2[:, 0], host(norms)[:, 0]) and not n2[:, 1:].any()
    xs, _ = step_loop(B, sysm, x0, 8, 8)
    xg = host(xg)
    assert np.array_equal(xg[:, :, :9], xs) and not xg[:, :, 9:].any()


def test_protocol_graph_replays(B):
    """The whole protocol captured in one graph (the decisions are on the
    device, nothing synchronises): every replay gives the eager result."""
    m = 4
    sysm, x0 = I.newton_system((1401, 0), 8, m)
    sd = B.DeviceSystem(sysm)
    x0g = dev(x0)
    eager = [host(t).copy() for t in B.md_newton_protocol(sd, x0g)[:3]]
    ws = B.workspace(B.MD_FN_PROTOCOL, m, sysm.N, sysm.n, 32, sysm.M, sysm.max_deg)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            st.zero_()
            out = B.md_newton_protocol(sd, x0g, ws=ws, status=st, stream=s)
    torch.cuda.synchronize()
    for rep in range(3):
        out[0].zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(host(st)[0]) == 0
        for a, b in zip(out[:3], eager):
            assert np.array_equal(host(a), b), rep
