"""Pin of the oracle's adjoint: the coefficient gradient of L = sum |x_k|^2
through the converged series solution agrees with central finite
differences taken in quad double (h = 2^-66, truncation O(h^2) ~ 1e-40,
cancellation ~ 2^-212 / h ~ 1e-44, both far below double-double)."""
from __future__ import annotations

from fractions import Fraction

import numpy as np
import pytest

import oracle
from exact import fval
from paper_2012_06607_amd import inputs as I


def loss(x):
    return sum(fval(x[0, :, k, i]) ** 2 + fval(x[1, :, k, i]) ** 2
               for k in range(x.shape[2]) for i in range(x.shape[3]))


@pytest.mark.parametrize("key,n,d", (((995, 0), 3, 6), ((996, 1), 2, 4)))
def test_adjoint_against_central_differences(key, n, d):
    m, iters = 4, 8
    sysm, x0 = I.newton_system(key, n, m, terms=3, max_deg=3)
    x = I.series_start(x0, d)
    xs, norms, st = oracle.newton(sysm, x, iters)
    assert st == 0 and norms[-1][0, 0] < 1e-50
    g, st = oracle.newton_adjoint(sysm, xs, 2 * xs)
    assert st == 0
    h = Fraction(1, 2**66)
    for tau in range(sysm.M):
        for j in range(sysm.dc + 1):
            for part in (0, 1):
                vals = []
                for sgn in (1, -1):
                    coef = sysm.coef.copy()
                    v = fval(coef[part, :, tau, j]) + sgn * h
                    coef[part, :, tau, j] = I.limbs_of_ratio(v.numerator, v.denominator, m)
                    s2 = I.System(sysm.N, sysm.n, m, sysm.dc, sysm.eq_ptr, sysm.term_ptr,
                                  sysm.factors, coef, sysm.meta)
                    xp, _, _ = oracle.newton(s2, x, iters)
                    vals.append(loss(xp))
                fd = (vals[0] - vals[1]) / (2 * h)
                got = Fraction(g[part, 0, tau, j]) + Fraction(g[part, 1, tau, j])
                assert abs(float(fd - got)) <= 1e-30 * max(1.0, abs(float(fd))), (tau, j, part)


def test_adjoint_of_a_linear_equation():
    """x - c0 - c1 t = 0: x = c0 + c1 t exactly, so for L = |x_0|^2 + |x_1|^2
    the gradient (dL/dRe c + i dL/dIm c) is 2 c."""
    m, d = 2, 1
    g = I.rng(997)
    c = I.unit_complex(g, m, 2)
    one = ([1.0, 0.0], [0.0, 0.0])
    mone = ([-1.0, 0.0], [0.0, 0.0])
    sysm = I.build_system(1, 1, m, 1, [[((0,), [one]), ((), [(-c[0, :, 0], -c[1, :, 0]),
                                                              (-c[0, :, 1], -c[1, :, 1])])]])
    x = np.zeros((2, m, d + 1, 1))
    xs, _, _ = oracle.newton(sysm, x, 3)
    assert np.allclose(xs[0, 0, :, 0], c[0, 0]) and np.allclose(xs[1, 0, :, 0], c[1, 0])
    gr, _ = oracle.newton_adjoint(sysm, xs, 2 * xs)
    # the constant term's coefficient series is -c(t): its gradient is -2 c
    assert np.allclose(gr[0, 0, 1, :], -2 * c[0, 0], rtol=1e-14)
    assert np.allclose(gr[1, 0, 1, :], -2 * c[1, 0], rtol=1e-14)
    # the coefficient of x is 1; d/d(1) of x = c/coef: -2 |x|^2 summed
    want = -2 * (abs(c[0, 0] + 1j * c[1, 0]) ** 2).sum()
    assert np.allclose(gr[0, 0, 0, 0], want, rtol=1e-14) and abs(gr[1, 0, 0, 0]) < 1e-14
