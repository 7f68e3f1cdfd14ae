"""Series division and Pade approximants on the GPU against the oracle.
Division runs the oracle's operations in the oracle's order (bit-exact);
the Pade denominators come from the GPU's Householder QR (another summation
order), so they agree within the precision times the conditioning."""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from exact import fval, planes_rel_err_per_k as rel_err_per_k
from paper_2012_06607_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ALL_M = (1, 2, 3, 4, 5, 8, 10)


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


@pytest.mark.parametrize("m", ALL_M)
@pytest.mark.parametrize("count,d", ((64, 32), (3, 0), (70, 9)))
def test_divide_bit_exact(B, m, count, d):
    g = I.rng(1510, m, count, d)
    x = I.unit_complex(g, m, count, d + 1)
    y = I.unit_complex(g, m, count, d + 1)
    want, stw = oracle.series_divide(x, y)
    z, st = B.md_series_divide(dev(x), dev(y))
    assert int(host(st)[0]) == stw == 0
    assert np.array_equal(host(z), want)


@pytest.mark.parametrize("m,count,d", ((2, 5, 100), (4, 2, 70), (10, 1, 600)))
def test_divide_long_series(B, m, count, d):
    # more products per coefficient than lanes (d > 64), and deca double at
    # d = 600, whose products do not fit in LDS (one lane per series)
    g = I.rng(1512, m, count, d)
    x = I.unit_complex(g, m, count, d + 1)
    y = I.unit_complex(g, m, count, d + 1)
    y[:, :, :, 0] *= 4.0
    want, stw = oracle.series_divide(x, y)
    z, st = B.md_series_divide(dev(x), dev(y))
    assert int(host(st)[0]) == stw == 0
    assert np.array_equal(host(z), want)


def test_divide_flags_zero_constant(B):
    m = 2
    x = I.unit_complex(I.rng(1511), m, 4, 5)
    y = x.copy()
    y[:, :, 2, 0] = 0.0
    _, st = B.md_series_divide(dev(x), dev(y))
    assert int(host(st)[0]) == B.MD_ST_SINGULAR


@pytest.mark.parametrize("m", (2, 4, 8, 10))
@pytest.mark.parametrize("L,M", ((2, 2), (4, 4), (6, 3), (2, 5)))
def test_pade_of_exp(B, m, L, M):
    """exp(t): the closed-form approximants (ratios of factorials)."""
    f = math.factorial
    c = I.real_rational(m, [(1, f(k)) for k in range(L + M + 1)])[:, :, None, :]
    p, q, st = B.md_series_pade(dev(c), L, M)
    assert int(host(st)[0]) == 0
    p, q = host(p), host(q)
    for k in range(L + 1):
        want = Fraction(f(L + M - k) * f(L), f(L + M) * f(k) * f(L - k))
        assert abs(fval(p[0, :, 0, k]) - want) <= Fraction(2) ** -(53 * m - 16), k
    for k in range(M + 1):
        want = Fraction((-1) ** k * f(L + M - k) * f(M), f(L + M) * f(k) * f(M - k))
        assert abs(fval(q[0, :, 0, k]) - want) <= Fraction(2) ** -(53 * m - 16), k


@pytest.mark.parametrize("m", (2, 4, 8))
def test_pade_of_newton_series_against_oracle(B, m):
    """Pade approximants of the components of a computed solution series
    (the config-1 generator, 8 steps at degree 16, [8/8] per component),
    against the oracle's on the same series."""
    n, d = 8, 16
    sysm, x0 = I.newton_system((1512, m), n, m)
    x, _, _ = oracle.newton(sysm, I.series_start(x0, d), 8)
    c = np.ascontiguousarray(np.transpose(x, (0, 1, 3, 2)))  # (2, m, n, d+1)
    L, M = 8, 8
    pw, qw, stw = oracle.pade(c, L, M)
    p, q, st = B.md_series_pade(dev(c), L, M)
    assert int(host(st)[0]) == stw == 0
    p, q = host(p), host(q)
    # per series: the relative difference of the coefficient vectors
    for s in range(n):
        eq = rel_err_per_k(q[:, :, s:s + 1, :].transpose(0, 1, 3, 2),
                           qw[:, :, s:s + 1, :].transpose(0, 1, 3, 2))
        ep = rel_err_per_k(p[:, :, s:s + 1, :].transpose(0, 1, 3, 2),
                           pw[:, :, s:s + 1, :].transpose(0, 1, 3, 2))
        print(f"pade m={m} series {s}: log2 max diff q {math.log2(max(eq.max(), 1e-300)):.1f} "
              f"p {math.log2(max(ep.max(), 1e-300)):.1f}", flush=True)
        # agreement rule: within 2^-(53m-8) times the condition number of
        # the Toeplitz system (from the leading limbs), times 2^4
        cl = c[0, 0, s] + 1j * c[1, 0, s]
        T = np.array([[cl[L + i - j] if L + i - j >= 0 else 0 for j in range(1, M + 1)]
                      for i in range(1, M + 1)])
        kappa = np.linalg.cond(T)
        bound = 2.0 ** -(53 * m - 8) * kappa * 16
        assert eq.max() <= bound and ep.max() <= bound, (s, kappa, eq.max(), ep.max())


def test_pade_without_denominator(B):
    m = 4
    c = I.unit_complex(I.rng(1513), m, 5, 7)
    p, q, st = B.md_series_pade(dev(c), 6, 0)
    assert int(host(st)[0]) == 0
    assert np.array_equal(host(p), c)
    qh = host(q)
    assert np.all(qh[0, 0] == 1.0) and not qh[0, 1:].any() and not qh[1].any()
