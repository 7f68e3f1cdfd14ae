"""Pins of the oracle's multiple-double arithmetic (Section 2) against exact
rational arithmetic, the paper's operation counts (Table 1) and its 2-norm
example."""
from __future__ import annotations

import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from exact import fval
from paper_2012_06607_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden")
ALL_M = (1, 2, 3, 4, 5, 8, 10)
C_BITS = 4  # per-operation error allowance: 2^-(53m - 4) of the scale


def rand_md(g, m, count, spread=20, allow_zero=False):
    """Normalised random expansions with exponents in [-spread, spread]."""
    out = np.zeros((m, count))
    for e in range(count):
        if allow_zero and g.random() < 0.05:
            continue
        P = int(g.integers(1, 2**62)) * (1 << 700) + int.from_bytes(g.bytes(88), "little")
        Q = 1 << (762 - int(g.integers(-spread, spread + 1)))
        if g.random() < 0.5:
            P = -P
        out[:, e] = I.limbs_of_ratio(P, Q, m)
    return out


def _limbs_of_fraction(v: Fraction, m: int):
    return I.limbs_of_ratio(v.numerator, v.denominator, m)


def adversarial_pairs(g, m, count):
    """Pairs with cancellation, equal and opposite operands, powers of two
    and short (exact) operands; every operand is a normalised expansion."""
    a = rand_md(g, m, count)
    b = rand_md(g, m, count)
    k = count // 6
    for e in range(count):
        A = fval(a[:, e])
        grp = e // k
        if grp == 0:                      # exact cancellation
            b[:, e] = -a[:, e]
        elif grp == 1:                    # cancellation down to the last limbs
            b[:, e] = _limbs_of_fraction(-A + A * Fraction(int(g.integers(1, 2**30)), 2 ** (53 * m - 10)), m)
        elif grp == 2:                    # a = b
            b[:, e] = a[:, e]
        elif grp == 3:                    # powers of two
            a[:, e] = 0.0
            a[0, e] = 2.0 ** int(g.integers(-40, 40))
        elif grp == 4:                    # b a plain double
            b[1:, e] = 0.0
        else:                             # leading limbs cancel
            b[:, e] = _limbs_of_fraction(-A + A * Fraction(int(g.integers(1, 2**50)), 2**70), m)
    return a, b


def normwise_err(z, exact, scale):
    return abs(fval(z) - exact) / scale if scale != 0 else abs(fval(z) - exact)


@pytest.mark.parametrize("m", ALL_M)
def test_real_ops_against_exact_rationals(m):
    g = I.rng(900, m)
    a, b = rand_md(g, m, 240), rand_md(g, m, 240)
    aa, bb = adversarial_pairs(g, m, 120)
    a = np.concatenate([a, aa], axis=1)
    b = np.concatenate([b, bb], axis=1)
    bound = Fraction(2) ** -(53 * m - C_BITS)
    z_add = oracle.elementwise("add", a, b)
    z_sub = oracle.elementwise("sub", a, b)
    z_mul = oracle.elementwise("mul", a, b)
    for e in range(a.shape[1]):
        A, B = fval(a[:, e]), fval(b[:, e])
        scale = max(abs(A), abs(B))
        assert normwise_err(z_add[:, e], A + B, scale) <= bound, ("add", e)
        assert normwise_err(z_sub[:, e], A - B, scale) <= bound, ("sub", e)
        assert normwise_err(z_mul[:, e], A * B, abs(A * B)) <= bound, ("mul", e)
    nz = np.abs(b[0]) > 0
    z_div = oracle.elementwise("div", a[:, nz], b[:, nz])
    for e, (x, y) in enumerate(zip(a[:, nz].T, b[:, nz].T)):
        q = fval(x) / fval(y)
        assert normwise_err(z_div[:, e], q, abs(q)) <= bound, ("div", e)


@pytest.mark.parametrize("m", ALL_M)
def test_sqrt_and_rsqrt_against_exact(m):
    g = I.rng(901, m)
    a = rand_md(g, m, 200, spread=40)
    a = a * np.sign(a[0])[None, :]
    a[:, :3] = 0.0
    a[0, 1] = 4.0
    a[0, 2] = 2.0 ** -30
    s = oracle.elementwise("sqrt", a)
    r = oracle.elementwise("rsqrt", a[:, 1:])
    assert np.all(s[:, 0] == 0.0)
    assert s[0, 1] == 2.0 and np.all(s[1:, 1] == 0.0)
    bound = Fraction(2) ** -(53 * m - C_BITS)
    for e in range(1, a.shape[1]):
        A, S = fval(a[:, e]), fval(s[:, e])
        # sqrt(A)(1 + delta): S^2 = A (1 + 2 delta + delta^2)
        assert abs(S * S - A) / A <= 2 * bound + bound * bound, ("sqrt", e)
        R = fval(r[:, e - 1])
        assert abs(R * R * A - 1) <= 2 * bound + bound * bound, ("rsqrt", e)


@pytest.mark.parametrize("m", ALL_M)
def test_complex_ops_against_exact(m):
    g = I.rng(902, m)
    x = I.unit_complex(g, m, 150) * np.asarray([1.0, 1.0])[:, None, None]
    y = I.unit_complex(g, m, 150)
    bound = Fraction(2) ** -(53 * m - C_BITS - 1)
    zm = oracle.elementwise("cmul", x, y)
    zd = oracle.elementwise("cdiv", x, y)
    za = oracle.elementwise("cadd", x, y)
    z2 = oracle.elementwise("cabs2", x)
    for e in range(x.shape[2]):
        xr, xi = fval(x[0, :, e]), fval(x[1, :, e])
        yr, yi = fval(y[0, :, e]), fval(y[1, :, e])
        pr, pi = xr * yr - xi * yi, xr * yi + xi * yr
        assert abs(fval(zm[0, :, e]) - pr) <= 2 * bound and abs(fval(zm[1, :, e]) - pi) <= 2 * bound
        den = yr * yr + yi * yi
        qr, qi = (xr * yr + xi * yi) / den, (xi * yr - xr * yi) / den
        assert abs(fval(zd[0, :, e]) - qr) <= 4 * bound and abs(fval(zd[1, :, e]) - qi) <= 4 * bound
        assert abs(fval(za[0, :, e]) - (xr + yr)) <= 2 * bound
        assert abs(fval(za[1, :, e]) - (xi + yi)) <= 2 * bound
        assert abs(fval(z2[:, e]) - (xr * xr + xi * xi)) <= 2 * bound


@pytest.mark.parametrize("m", ALL_M)
def test_results_are_normalised(m):
    """Each limb is below the unit in the last place of the one before
    (up to one bit), so the m limbs carry about 53m bits."""
    g = I.rng(903, m)
    a, b = rand_md(g, m, 200), rand_md(g, m, 200)
    for op in ("add", "mul", "div"):
        z = oracle.elementwise(op, a, b)
        for e in range(z.shape[1]):
            for i in range(m - 1):
                if z[i, e] != 0.0:
                    assert abs(z[i + 1, e]) <= math.ulp(z[i, e]), (op, e, i)


def test_double_precision_is_plain_ieee():
    g = np.random.default_rng(5)
    a = g.standard_normal((1, 500))
    b = g.standard_normal((1, 500))
    assert np.array_equal(oracle.elementwise("add", a, b)[0], a[0] + b[0])
    assert np.array_equal(oracle.elementwise("mul", a, b)[0], a[0] * b[0])
    assert np.array_equal(oracle.elementwise("div", a, b)[0], a[0] / b[0])
    assert np.array_equal(oracle.elementwise("sqrt", np.abs(a))[0], np.sqrt(np.abs(a[0])))


def test_table1_double_double_add_count():
    """Table 1: a double double addition is 8 additions and 12 subtractions."""
    counts = json.load(open(os.path.join(GOLD, "table1_opcounts.json")))["counts"]
    g = I.rng(904)
    a, b = rand_md(g, 2, 1), rand_md(g, 2, 1)
    oracle.reset_counters()
    oracle.elementwise("add", a, b)
    c = oracle.counters()
    assert [c["add"], c["sub"], c["mul"], c["div"]] == counts["2"]["add"]
    assert c["md_add"] == 1


@pytest.mark.parametrize("m", (2, 3, 4, 5, 8, 10))
def test_table1_division_takes_m_plus_one_quotients(m):
    """Table 1's '/' column is m+1 for every precision: the division is a
    long division with m+1 hardware quotient digits."""
    counts = json.load(open(os.path.join(GOLD, "table1_opcounts.json")))["counts"]
    g = I.rng(905, m)
    a, b = rand_md(g, m, 1), rand_md(g, m, 1)
    oracle.reset_counters()
    oracle.elementwise("div", a, b)
    c = oracle.counters()
    assert c["div"] == counts[str(m)]["div"][3] == m + 1
    assert c["md_div"] == 1 and c["md_add"] == 0 and c["md_mul"] == 0


@pytest.mark.parametrize("m", (2, 3, 4, 5, 8, 10))
def test_two_norm_of_64_unit_complex_numbers(m):
    """Section 2: the 2-norm of 64 numbers cos(theta) + i sin(theta) is 8; the
    leading limb is 8 and the second limb is at the precision's level.  The
    paper's printed second limbs (other random angles) obey the same bound."""
    gold = json.load(open(os.path.join(GOLD, "two_norm_paper.json")))
    x = I.unit_complex(I.rng(906, m), m, 64)
    nrm = oracle.norm2(x)
    assert nrm[0] == 8.0
    level = 8.0 * 2.0 ** -(53 * m)
    assert abs(nrm[1]) <= 2**8 * level
    assert abs(gold["second_limb"][str(m)]) <= level
    # exact: sum of |x_j|^2 of the rounded inputs, then the square root
    s = sum(fval(x[0, :, j]) ** 2 + fval(x[1, :, j]) ** 2 for j in range(64))
    got = fval(nrm)
    assert abs(got * got - s) / s <= Fraction(2) ** -(53 * m - C_BITS - 1)
