"""GPU parity of the adjoint of the converged series solution
(md_newton_adjoint and its torch.autograd wrapper) against the oracle's
adjoint, which is pinned to finite differences on the CPU.

Both sides evaluate in m limbs and round the gradient to double double.
The HIP path sums in other orders (segment trees, W = R^{-1} Q^H formed
once), so the two agree within 2^-(53m-8) relative to the largest gradient,
widened by log2 of the condition number of A_0 and of the d+1 stages, and
never tighter than 2^-100 (the double-double output).  The stored and the
recomputed monomial series take the same products in the same order: those
two modes agree bit for bit.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from paper_2012_06607_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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


def converged(key, n, m, d, terms, max_deg=3, iters=8):
    sysm, x0 = I.newton_system(key, n, m, terms=terms, max_deg=max_deg)
    xs, norms, st = oracle.newton(sysm, I.series_start(x0, d), iters)
    assert st == 0
    return sysm, xs


def dd_rel_err(got, want):
    """max |got - want| / max |want| over double-double planes (2, 2, ...)."""
    diff = (got[:, 0] - want[:, 0]) + (got[:, 1] - want[:, 1])
    return float(np.max(np.abs(diff)) / np.max(np.abs(want[:, 0])))


def bound(m, sysm, d):
    extra = math.log2(max(2.0, sysm.meta["cond_A0_double"])) + math.log2(d + 1)
    return max(2.0 ** -(53 * m - 8 - extra), 2.0 ** -100)


def run_adjoint(B, sysm, xs, store):
    sysd = B.DeviceSystem(sysm)
    x = dev(xs)
    g, st = B.md_newton_adjoint(sysd, x, 2 * x, store_monomials=store)
    return host(g), int(host(st)[0])


@pytest.mark.parametrize("m", (1, 2, 3, 4, 5, 8, 10))
def test_adjoint_matches_oracle(B, m):
    d = 6
    sysm, xs = converged((1201, m), 6, m, d, terms=4)
    want, st = oracle.newton_adjoint(sysm, xs, 2 * xs)
    assert st == 0
    print(f"adjoint m={m} n=6 d={d} M={sysm.M}", flush=True)
    got_s, st_s = run_adjoint(B, sysm, xs, True)
    got_r, st_r = run_adjoint(B, sysm, xs, False)
    assert st_s == 0 and st_r == 0
    assert np.array_equal(got_s, got_r)
    err = dd_rel_err(got_s, want)
    assert err <= bound(m, sysm, d), (m, err)
    if m == 1:
        assert np.all(got_s[:, 1] == 0)


@pytest.mark.parametrize("store", (True, False))
def test_adjoint_quad_double_32_unknowns(B, store):
    """n = 32, 256 monomials of degree <= 3 plus a constant and a t-term
    per equation (M = 320), d = 16, quad double: every gradient entry."""
    m, d = 4, 16
    sysm, xs = converged((1202, 0), 32, m, d, terms=8)
    assert sysm.M == 320
    want, st = oracle.newton_adjoint(sysm, xs, 2 * xs)
    assert st == 0
    print(f"adjoint m={m} n=32 d={d} M=320 store={store}", flush=True)
    got, stg = run_adjoint(B, sysm, xs, store)
    assert stg == 0
    err = dd_rel_err(got, want)
    assert err <= bound(m, sysm, d), err


def test_adjoint_general_upstream_gradient(B):
    """An upstream gradient that is not 2x (random unit complex series)."""
    m, d = 2, 8
    sysm, xs = converged((1203, 0), 8, m, d, terms=6)
    G = I.unit_complex(I.rng(1203, 1), m, d + 1, 8)
    want, _ = oracle.newton_adjoint(sysm, xs, G)
    sysd = B.DeviceSystem(sysm)
    got, st = B.md_newton_adjoint(sysd, dev(xs), dev(G))
    assert int(host(st)[0]) == 0
    assert dd_rel_err(host(got), want) <= bound(m, sysm, d)


def test_adjoint_degree_zero(B):
    """d = 0: one stage, lambda = A_0^{-H} G_0."""
    m, d = 3, 0
    sysm, xs = converged((1204, 0), 5, m, d, terms=4)
    want, _ = oracle.newton_adjoint(sysm, xs, 2 * xs)
    got, st = run_adjoint(B, sysm, xs, True)
    assert st == 0 and dd_rel_err(got, want) <= bound(m, sysm, d)


def test_adjoint_deterministic(B):
    m, d = 4, 8
    sysm, xs = converged((1205, 0), 10, m, d, terms=5)
    a, _ = run_adjoint(B, sysm, xs, False)
    b, _ = run_adjoint(B, sysm, xs, False)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("store", (True, False))
def test_autograd_newton_solve(B, store):
    """coef.grad of sum |x|^2 through newton_solve equals the oracle's
    adjoint at the oracle's converged x; limbs above the second are zero."""
    from paper_2012_06607_amd.autograd import newton_solve, sum_abs2
    m, d, n, iters = 4, 8, 8, 8
    sysm, x0 = I.newton_system((1206, 0), n, m, terms=6)
    xs, _, _ = oracle.newton(sysm, I.series_start(x0, d), iters)
    want, _ = oracle.newton_adjoint(sysm, xs, 2 * xs)
    sysd = B.DeviceSystem(sysm)
    coef = dev(sysm.coef).requires_grad_()
    x, st = newton_solve(coef, sysd, dev(I.series_start(x0, d)), iters, store_monomials=store)
    L = sum_abs2(x)
    L.backward()
    g = host(coef.grad)
    assert int(host(st)[0]) == 0
    assert np.all(g[:, 2:] == 0)
    assert dd_rel_err(g[:, :2], want) <= bound(m, sysm, d)
    want_L = float(np.sum(xs[:, 0] ** 2))
    assert abs(float(L.detach()) - want_L) <= 1e-13 * want_L


def test_sum_abs2_backward_keeps_every_limb(B):
    """SumAbs2's backward is 2 g z formed in the library (md x double per
    plane): with an upstream g = 3 (not a power of two) it equals the
    oracle's md x double product by 6 bit for bit, in all m limbs."""
    from paper_2012_06607_amd.autograd import sum_abs2
    m = 4
    z = I.unit_complex(I.rng(1207, 0), m, 5, 7)
    zt = dev(z).requires_grad_()
    L = 3.0 * sum_abs2(zt)
    L.backward()
    got = host(zt.grad)
    six = np.zeros((m, 35))
    six[0] = 6.0
    for part in range(2):
        want = oracle.elementwise("muld", z[part].reshape(m, -1), six).reshape(m, 5, 7)
        assert np.array_equal(got[part], want)
    assert np.any(got[:, 1:] != 0)     # the lower limbs are there


def test_autograd_upstream_three(B):
    """coef.grad of 3 sum |x|^2 through newton_solve: the upstream 3 reaches
    the adjoint as G = 6 x with every limb, so the gradient is the oracle's
    adjoint for G = 6 x (formed by the oracle's md x double product)."""
    from paper_2012_06607_amd.autograd import newton_solve, sum_abs2
    m, d, n, iters = 4, 8, 8, 8
    sysm, x0 = I.newton_system((1206, 0), n, m, terms=6)
    xs, _, _ = oracle.newton(sysm, I.series_start(x0, d), iters)
    G = np.empty_like(xs)
    six = np.zeros((m, xs[0].size // m))
    six[0] = 6.0
    for part in range(2):
        G[part] = oracle.elementwise("muld", xs[part].reshape(m, -1), six).reshape(xs[part].shape)
    want, _ = oracle.newton_adjoint(sysm, xs, G)
    sysd = B.DeviceSystem(sysm)
    coef = dev(sysm.coef).requires_grad_()
    x, st = newton_solve(coef, sysd, dev(I.series_start(x0, d)), iters)
    (3.0 * sum_abs2(x)).backward()
    g = host(coef.grad)
    assert int(host(st)[0]) == 0
    assert dd_rel_err(g[:, :2], want) <= bound(m, sysm, d)
