"""Series division and Pade approximants in the oracle (Section 3: a series
with a nonzero constant term has an inverse, series divide like numbers,
and computed series give rational approximations), pinned to closed forms
and exact rational arithmetic."""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from exact import fval
from paper_2012_06607_amd import inputs as I

ALL_M = (1, 2, 3, 4, 5, 8, 10)


def real_series(m, coefs, count=1):
    """Planes (2, m, count, len) of real rational coefficients (P, Q)."""
    a = I.real_rational(m, coefs)  # (2, m, len)
    return np.repeat(a[:, :, None, :], count, axis=2)


def cval(planes, s, k):
    return (fval(planes[0, :, s, k]), fval(planes[1, :, s, k]))


@pytest.mark.parametrize("m", ALL_M)
def test_divide_geometric_series(m):
    """1 / (1 - t) = 1 + t + t^2 + ... exactly."""
    d = 20
    one = real_series(m, [(1, 1)] + [(0, 1)] * d)
    y = real_series(m, [(1, 1), (-1, 1)] + [(0, 1)] * (d - 1))
    z, st = oracle.series_divide(one, y)
    assert st == 0
    assert np.all(z[0, 0, 0] == 1.0) and not z[0, 1:].any() and not z[1].any()


@pytest.mark.parametrize("m", (2, 4, 8))
@pytest.mark.parametrize("a,b", ((5, 2), (2, 5)))
def test_divide_binomials(m, a, b):
    """(1+t)^a / (1+t)^b = (1+t)^(a-b): binomial coefficients, exact."""
    d = 16
    x = real_series(m, [(math.comb(a, k), 1) for k in range(d + 1)])
    y = real_series(m, [(math.comb(b, k), 1) for k in range(d + 1)])
    z, st = oracle.series_divide(x, y)
    assert st == 0
    e = a - b
    for k in range(d + 1):
        want = math.comb(e, k) if e >= 0 else (-1) ** k * math.comb(k - e - 1, k)
        assert cval(z, 0, k) == (Fraction(want), 0), k


@pytest.mark.parametrize("m", (1, 2, 3, 4))
def test_divide_against_exact_rationals(m):
    """Random unit-complex series: the quotient against the exact
    recurrence on the rounded inputs (Fractions), and x = y (x / y)."""
    d, count = 8, 6
    g = I.rng(1500, m)
    x = I.unit_complex(g, m, count, d + 1)
    y = I.unit_complex(g, m, count, d + 1)
    z, st = oracle.series_divide(x, y)
    assert st == 0
    for s in range(count):
        xs = [cval(x, s, k) for k in range(d + 1)]
        ys = [cval(y, s, k) for k in range(d + 1)]
        zs = []

        def cmul(u, v):
            return (u[0] * v[0] - u[1] * v[1], u[0] * v[1] + u[1] * v[0])
        y0n = ys[0][0] ** 2 + ys[0][1] ** 2
        for k in range(d + 1):
            r = xs[k]
            for i in range(1, k + 1):
                p = cmul(ys[i], zs[k - i])
                r = (r[0] - p[0], r[1] - p[1])
            q = cmul(r, (ys[0][0], -ys[0][1]))
            zs.append((q[0] / y0n, q[1] / y0n))
        scale = max(abs(complex(float(v[0]), float(v[1]))) for v in zs)
        for k in range(d + 1):
            got = cval(z, s, k)
            err = abs(complex(float(got[0] - zs[k][0]), float(got[1] - zs[k][1])))
            assert err <= 2.0 ** -(53 * m - 8) * (k + 1) ** 2 * scale, (s, k, err)
    # the product of divisor and quotient gives the dividend back
    xb = oracle.convolve(y, z)
    for s in range(count):
        for k in range(d + 1):
            got, want = cval(xb, s, k), cval(x, s, k)
            err = abs(complex(float(got[0] - want[0]), float(got[1] - want[1])))
            assert err <= 2.0 ** -(53 * m - 12) * (k + 1) ** 2, (s, k, err)


def test_divide_flags_a_zero_constant_term():
    x = real_series(2, [(1, 1), (1, 1)], count=2)
    y = real_series(2, [(1, 1), (1, 1)], count=2)
    y[:, :, 1, 0] = 0.0
    _, st = oracle.series_divide(x, y)
    assert st == oracle.ST_SINGULAR


def pade_exp(L, M):
    """Closed form of the [L/M] Pade approximant of exp(t)."""
    f = math.factorial
    p = [Fraction(f(L + M - k) * f(L), f(L + M) * f(k) * f(L - k)) for k in range(L + 1)]
    q = [Fraction((-1) ** k * f(L + M - k) * f(M), f(L + M) * f(k) * f(M - k)) for k in range(M + 1)]
    return p, q


@pytest.mark.parametrize("m", (2, 4, 8, 10))
@pytest.mark.parametrize("L,M", ((2, 2), (3, 3), (4, 4), (6, 3), (2, 5)))
def test_pade_of_exp(m, L, M):
    """The Pade approximants of exp(t) have a closed form (coefficients
    of ratios of factorials); from the rounded Taylor coefficients 1/k! the
    oracle reproduces them to the precision."""
    c = real_series(m, [(1, math.factorial(k)) for k in range(L + M + 1)])
    p, q, st = oracle.pade(c, L, M)
    assert st == 0
    pw, qw = pade_exp(L, M)
    for k in range(L + 1):
        assert abs(fval(p[0, :, 0, k]) - pw[k]) <= Fraction(2) ** -(53 * m - 16), (k, p[0, 0, 0, k])
        assert not p[1, :, 0, k].any()
    for k in range(M + 1):
        assert abs(fval(q[0, :, 0, k]) - qw[k]) <= Fraction(2) ** -(53 * m - 16), (k, q[0, 0, 0, k])


@pytest.mark.parametrize("m", (2, 4, 8))
def test_pade_recovers_a_rational_function(m):
    """c = P/Q with deg P = 2, deg Q = 3 (series by exact division):
    its [2/3] approximant is P/Q, and every approximant satisfies the
    defining property q c - p = O(t^{L+M+1}) (checked exactly)."""
    P = [Fraction(1), Fraction(2), Fraction(-1)]
    Q = [Fraction(1), Fraction(-1, 2), Fraction(1, 4), Fraction(1, 8)]
    K = 12
    cs = []
    for k in range(K):
        v = (P[k] if k < len(P) else 0) - sum(Q[i] * cs[k - i] for i in range(1, min(k, 3) + 1))
        cs.append(v)
    c = real_series(m, [(v.numerator, v.denominator) for v in cs])
    L, M = 2, 3
    p, q, st = oracle.pade(c[:, :, :, :L + M + 1], L, M)
    assert st == 0
    for k in range(L + 1):
        assert abs(fval(p[0, :, 0, k]) - P[k]) <= Fraction(2) ** -(53 * m - 12)
    for k in range(M + 1):
        assert abs(fval(q[0, :, 0, k]) - Q[k]) <= Fraction(2) ** -(53 * m - 12)
    for L, M in ((4, 4), (5, 2), (1, 6)):
        p, q, st = oracle.pade(c[:, :, :, :L + M + 1], L, M)
        qv = [fval(q[0, :, 0, j]) for j in range(M + 1)]
        pv = [fval(p[0, :, 0, k]) for k in range(L + 1)]
        cv = [fval(c[0, :, 0, k]) for k in range(L + M + 1)]
        for k in range(L + M + 1):
            r = sum(qv[j] * cv[k - j] for j in range(min(k, M) + 1)) - (pv[k] if k <= L else 0)
            assert abs(r) <= Fraction(2) ** -(53 * m - 16) * 64, (L, M, k, float(r))


def test_pade_with_no_denominator_is_the_truncated_series():
    m = 4
    c = I.unit_complex(I.rng(1501, m), m, 3, 6)
    p, q, st = oracle.pade(c, 5, 0)
    assert st == 0 and np.array_equal(p, c)
    assert np.all(q[0, 0] == 1.0) and not q[0, 1:].any() and not q[1].any()
