"""Pins of the oracle's series layer: convolution (Section 3), evaluation and
differentiation, Householder QR, the block Toeplitz solve and Newton's
method (Section 4), against closed forms, the paper's printed example,
operation counts, exact rational arithmetic and 2000-bit references."""
from __future__ import annotations

import json
import math
import os
from fractions import Fraction

import mpmath
import numpy as np
import pytest

import oracle
from exact import cfrac, frac_of_mpf, fval, mpf_of, mp_array, mp_eval_diff, mp_newton_step, mp_toeplitz_solve, \
    rel_err_per_k, smul
from paper_2012_06607_amd import inputs as I

GOLD = os.path.join(os.path.dirname(__file__), "golden")
mpmath.mp.prec = 2000


def tol(m: int, extra_bits: float = 0.0) -> float:
    """2^-(53m - 8), the per-coefficient tolerance, widened by extra_bits."""
    return 2.0 ** -(53 * m - 8 - extra_bits)


# ----------------------------------------------------------------------------
# convolution


@pytest.mark.parametrize("case", json.load(open(os.path.join(GOLD, "convolution_counts.json")))["cases"])
def test_convolution_operation_counts(case):
    """Section 3: (d+2)(d+1)/2 coefficient products and (d+1)d/2 additions;
    each complex product is 4 real products and 2 real additions, each
    complex addition 2 real additions."""
    d = case["d"]
    assert (d + 2) * (d + 1) // 2 == case["mul"] and (d + 1) * d // 2 == case["add"]
    x = I.unit_complex(I.rng(910, d), 2, 1, d + 1)
    oracle.reset_counters()
    oracle.convolve(x, x)
    c = oracle.counters()
    assert c["md_mul"] == 4 * case["mul"]
    assert c["md_add"] == 2 * case["mul"] + 2 * case["add"]


@pytest.mark.parametrize("m", (1, 2, 4, 10))
def test_convolution_closed_forms(m):
    d = 32
    ones = np.zeros((2, m, 1, d + 1))
    ones[0, 0] = 1.0
    z = oracle.convolve(ones, ones)  # (1/(1-t))^2 = sum (k+1) t^k
    assert np.array_equal(z[0, 0, 0], np.arange(1, d + 2, dtype=float))
    assert not np.any(z[0, 1:]) and not np.any(z[1])
    # (1+t)^5 (1+t)^7 = (1+t)^12
    a = np.zeros((2, m, 1, d + 1))
    b = np.zeros((2, m, 1, d + 1))
    a[0, 0, 0, :6] = [math.comb(5, k) for k in range(6)]
    b[0, 0, 0, :8] = [math.comb(7, k) for k in range(8)]
    z = oracle.convolve(a, b)
    want = [math.comb(12, k) if k <= 12 else 0 for k in range(d + 1)]
    assert np.array_equal(z[0, 0, 0], np.asarray(want, dtype=float))
    # i t series times itself: (i/(1-t))^2 = -(k+1)
    ii = np.zeros((2, m, 1, d + 1))
    ii[1, 0] = 1.0
    z = oracle.convolve(ii, ii)
    assert np.array_equal(z[0, 0, 0], -np.arange(1, d + 2, dtype=float))


@pytest.mark.parametrize("m", (2, 4, 8))
def test_convolution_against_exact(m):
    d = 8
    g = I.rng(911, m)
    x = I.unit_complex(g, m, 3, d + 1)
    y = I.unit_complex(g, m, 3, d + 1)
    z = oracle.convolve(x, y)
    X, Y = mp_array(x), mp_array(y)
    for c in range(3):
        ref = smul(list(X[c]), list(Y[c]), d)
        for k in range(d + 1):
            got = mpmath.mpc(mpf_of(z[0, :, c, k]), mpf_of(z[1, :, c, k]))
            # |z_k - exact| <= (k+1) products of unit numbers, each 2^-(53m-5)
            assert abs(got - ref[k]) <= (k + 1) * tol(m, -3), (c, k)


# ----------------------------------------------------------------------------
# evaluation and differentiation


def small_system(m, dc=1):
    """Three equations in three unknowns with repeated variables, constants,
    t-terms and a coefficient series of degree dc."""
    g = I.rng(912, m, dc)
    uc = lambda: I.unit_complex(g, m, dc + 1)
    def ser():
        c = uc()
        return [(c[0, :, k], c[1, :, k]) for k in range(dc + 1)]
    eqs = [
        [((0, 0, 1), ser()), ((2,), ser()), ((), ser())],
        [((0, 1, 1, 2), ser()), ((1, 1), ser()), ((0, 2), ser()), ((), ser())],
        [((2, 2, 2), ser()), ((0, 1, 2), ser()), ((1,), ser())],
    ]
    return I.build_system(3, 3, m, dc, eqs)


@pytest.mark.parametrize("m", (1, 2, 4))
@pytest.mark.parametrize("dc", (0, 1, 3))
def test_eval_diff_against_power_rule(m, dc):
    d = 6
    sysm = small_system(m, dc)
    x = I.unit_complex(I.rng(913, m), m, d + 1, 3)
    f, A = oracle.eval_diff(sysm, x)
    fr, Ar = mp_eval_diff(sysm, mp_array(x), d)
    ef = rel_err_per_k(f, fr)
    eA = rel_err_per_k(A, Ar)
    assert np.all(ef <= tol(m, 6)), ef
    assert np.all(eA <= tol(m, 6)), eA


def test_eval_diff_single_variable_power():
    """x^3 at x(t) = 1 + t: value (1+t)^3, derivative 3 (1+t)^2, exactly."""
    m, d = 4, 5
    one = ([1.0] + [0.0] * (m - 1), [0.0] * m)
    sysm = I.build_system(1, 1, m, 0, [[((0, 0, 0), [one])]])
    x = np.zeros((2, m, d + 1, 1))
    x[0, 0, 0, 0] = 1.0
    x[0, 0, 1, 0] = 1.0
    f, A = oracle.eval_diff(sysm, x)
    assert np.array_equal(f[0, 0, :, 0], [1, 3, 3, 1, 0, 0])
    assert np.array_equal(A[0, 0, :, 0, 0], [3, 6, 3, 0, 0, 0])
    assert not np.any(f[:, 1:]) and not np.any(A[1])


# ----------------------------------------------------------------------------
# Householder QR


def qr_reconstruct(QR, vd, beta):
    """Q (from the reflectors) and R as mpmath matrices."""
    Qm = mp_array(QR)
    V = mp_array(vd)
    B = [mpf_of(beta[:, j]) for j in range(beta.shape[1])]
    N, n = Qm.shape
    Q = mpmath.eye(N)
    for j in reversed(range(n)):
        v = mpmath.matrix(N, 1)
        v[j] = V[j]
        for i in range(j + 1, N):
            v[i] = Qm[i, j]
        H = mpmath.eye(N) - B[j] * v * v.transpose_conj()
        Q = H * Q
    R = mpmath.matrix(N, n)
    for i in range(n):
        for l in range(i, n):
            R[i, l] = Qm[i, l]
    return Q, R


@pytest.mark.parametrize("m", (2, 4))
@pytest.mark.parametrize("shape", ((5, 5), (7, 4)))
def test_qr_invariants(m, shape):
    N, n = shape
    A0 = I.unit_complex(I.rng(914, m, N, n), m, N, n)
    QR, vd, beta, st = oracle.qr(A0)
    assert st == 0
    Q, R = qr_reconstruct(QR, vd, beta)
    Am = mp_array(A0)
    eps = mpmath.mpf(2) ** -(53 * m - 10)
    I_N = mpmath.eye(N)
    QhQ = Q.transpose_conj() * Q
    for i in range(N):
        for j in range(N):
            assert abs(QhQ[i, j] - I_N[i, j]) <= eps * N
    QRm = Q * R
    for i in range(N):
        for j in range(n):
            assert abs(QRm[i, j] - Am[i, j]) <= eps * N
    # the diagonal convention R_jj = -phi sigma: R_jj / |R_jj| = -x0/|x0| where
    # x0 is the column's diagonal entry after the previous reflections
    work = mpmath.matrix([[Am[i, j] for j in range(n)] for i in range(N)])
    for j in range(n):
        x0 = work[j, j]
        assert abs(R[j, j] / abs(R[j, j]) + x0 / abs(x0)) <= eps * 10
        sigma = mpmath.sqrt(sum(abs(work[i, j]) ** 2 for i in range(j, N)))
        assert abs(abs(R[j, j]) - sigma) <= eps * 10 * sigma
        # apply H_j to the remaining columns
        v = mpmath.matrix(N, 1)
        phi = x0 / abs(x0)
        v[j] = phi * (abs(x0) + sigma)
        for i in range(j + 1, N):
            v[i] = work[i, j]
        bet = 1 / (sigma * (sigma + abs(x0)))
        work = work - bet * v * (v.transpose_conj() * work)


def test_qr_flags_a_zero_column():
    m = 2
    A0 = I.unit_complex(I.rng(915), m, 4, 4)
    A0[:, :, :, 1] = 0.0
    _, _, beta, st = oracle.qr(A0)
    assert st & oracle.ST_SINGULAR
    assert np.all(beta[:, 1] == 0.0)


# ----------------------------------------------------------------------------
# block Toeplitz solve


@pytest.mark.parametrize("m", (2, 4))
def test_toeplitz_solve_against_dense(m):
    """Well conditioned A_0 (cond 1e3), unit complex A_k and b_k; the result
    does not depend on the method, so mpmath's dense solve at 2000 bits is
    the reference.  Tolerance: 2^-(53m-8) widened by log2(cond) + log2(k+1)."""
    n, d = 6, 6
    A, b = I.toeplitz_system((916, m), n, d, m)
    dx, st = oracle.solve_toeplitz(A, b)
    assert st == 0
    ref = mp_toeplitz_solve(mp_array(A), mp_array(b))
    e = rel_err_per_k(dx, ref)
    for k in range(d + 1):
        assert e[k] <= tol(m, math.log2(1e3) + math.log2(k + 1)), (k, e)


@pytest.mark.parametrize("m", (2, 4))
def test_toeplitz_solve_residual_and_transposition(m):
    """A(t) dx(t) = b(t) holds coefficient by coefficient; a transposed A_j
    or a wrong stage index would break the residual."""
    n, d = 5, 4
    A, b = I.toeplitz_system((917, m), n, d, m)
    dx, _ = oracle.solve_toeplitz(A, b)
    Am, bm, xm = mp_array(A), mp_array(b), mp_array(dx)
    for k in range(d + 1):
        for i in range(n):
            s = sum(Am[j, i, l] * xm[k - j, l] for j in range(k + 1) for l in range(n))
            scale = max(abs(xm[kk, l]) for kk in range(k + 1) for l in range(n)) * n * (k + 1)
            assert abs(s - bm[k, i]) <= tol(m, 10) * scale


@pytest.mark.parametrize("m", (2, 4))
def test_toeplitz_least_squares_consistent(m):
    """N > n: for b(t) = A(t) x(t) the least squares solution is x(t)."""
    N, n, d = 7, 4, 3
    g = I.rng(918, m)
    A = I.unit_complex(g, m, d + 1, N, n)
    xs = I.unit_complex(g, m, d + 1, n)
    Am, Xm = mp_array(A), mp_array(xs)
    b = np.zeros((2, m, d + 1, N))
    for k in range(d + 1):
        for i in range(N):
            s = sum(Am[j, i, l] * Xm[k - j, l] for j in range(k + 1) for l in range(n))
            re, im = frac_of_mpf(s.real), frac_of_mpf(s.imag)
            b[0, :, k, i] = I.limbs_of_ratio(re.numerator, re.denominator, m)
            b[1, :, k, i] = I.limbs_of_ratio(im.numerator, im.denominator, m)
    dx, st = oracle.solve_toeplitz(A, b)
    e = rel_err_per_k(dx, Xm)
    assert np.all(e <= tol(m, 14)), e


# ----------------------------------------------------------------------------
# Newton's method


def test_circle_example_double_precision():
    """Section 3: in double precision, 8 as truncation degree, from x = 1,
    y = 0, the x series holds the Taylor coefficients of cos(t); the printed
    x_8 = 2.48015873015868E-05 is off from 1/40320 by 2^-45.5 relative, and
    the oracle's double run stays at that level."""
    gold = json.load(open(os.path.join(GOLD, "circle_double_output.json")))
    sysm, x = I.circle_system(1, 8)
    xo, norms, st = oracle.newton(sysm, x, 8)
    assert st == 0
    for k, (p, q) in gold["exact"].items():
        k = int(k)
        exact = p / q
        printed = gold["printed"][str(k)]
        got = xo[0, 0, k, 0]
        paper_err = abs(printed - exact) / abs(exact)
        assert abs(got - exact) / abs(exact) <= max(2 * paper_err, 2.0**-50)
    for k in (1, 3, 5, 7):
        assert abs(xo[0, 0, k, 0]) <= 2.0**-50
    # y = sin(t) up to t^7, and y_8 = 0
    ys = [0, 1, 0, -1 / 6, 0, 1 / 120, 0, -1 / 5040, 0]
    assert np.allclose(xo[0, 0, :, 1], ys, rtol=2.0**-45, atol=2.0**-50)


@pytest.mark.parametrize("m", (2, 3, 4, 8))
def test_circle_example_multiple_double(m):
    sysm, x = I.circle_system(m, 8)
    xo, norms, st = oracle.newton(sysm, x, 6)
    assert st == 0
    for k in range(9):
        want = Fraction(0) if k % 2 else Fraction((-1) ** (k // 2), math.factorial(k))
        assert abs(fval(xo[0, :, k, 0]) - want) <= tol(m) * abs(want) + Fraction(2) ** (-53 * m)
        assert not np.any(xo[1, :, k, 0])
    assert abs(norms[-1][0, 0]) <= 2.0 ** -(53 * m - 8)


@pytest.mark.parametrize("m", (2, 4, 8))
def test_sqrt_one_plus_t(m):
    """x^2 - (1+t) = 0 from x = 1: the series of sqrt(1+t), binom(1/2, k)."""
    d = 16
    sysm, x = I.sqrt_system(m, d)
    xo, _, st = oracle.newton(sysm, x, 6)
    assert st == 0
    c = Fraction(1)
    for k in range(d + 1):
        assert abs(fval(xo[0, :, k, 0]) - c) <= tol(m) * abs(c)
        c = c * (Fraction(1, 2) - k) / (k + 1)


@pytest.mark.parametrize("m", (2, 4))
def test_newton_steps_against_2000_bit_reference(m):
    """Each step from the oracle's current x against the exact step (power
    rule evaluation, dense 2000-bit solve) from the same x."""
    n, d = 4, 8
    sysm, x0 = I.newton_system((919, m), n, m)
    x = I.series_start(x0, d)
    for it in range(5):
        xo, nrm, st = oracle.newton_step(sysm, x)
        assert st == 0
        ref, dx = mp_newton_step(sysm, mp_array(x))
        e = rel_err_per_k(xo, ref)
        cond = sysm.meta["cond_A0_double"]
        for k in range(d + 1):
            assert e[k] <= tol(m, math.log2(cond) + math.log2(k + 1) + 2), (it, k, e)
        # the reported update: modulus of the last coefficient of dx
        dmax = max(abs(v) for v in dx[d])
        assert abs(nrm[0, 0] - float(dmax)) <= 1e-12 * float(dmax) + 2.0 ** -(53 * m - 10)
        x = xo
    # converged: the update to the last coefficient is at the noise level
    assert nrm[0, 0] <= 2.0 ** -(53 * m - 12)


@pytest.mark.parametrize("m", (2, 4))
def test_least_squares_newton_on_a_consistent_overdetermined_system(m):
    """N = n + 7 (Section 4: N >= n, least squares by the QR of A_0; the
    experiment of Section 6 augments a square system with 7 equations): the
    appended equations are exact combinations of the first n, so the exact
    least-squares step equals the exact step of the square system, and the
    oracle's least-squares Newton converges to the square system's series."""
    n, d = 6, 8
    sysm, x0 = I.newton_system((920, m), n, m)
    aug = I.augmented_system((921, m), sysm, 7)
    assert (aug.N, aug.n) == (n + 7, n)
    x = I.series_start(x0, d)
    for it in range(6):
        xo, nrm, st = oracle.newton_step(aug, x)
        assert st == 0
        ref_sq, _ = mp_newton_step(sysm, mp_array(x))
        ref_ls, _ = mp_newton_step(aug, mp_array(x))
        # consistency: the two exact steps agree far below the precision
        for k in range(d + 1):
            for i in range(n):
                assert abs(ref_sq[k, i] - ref_ls[k, i]) <= mpmath.mpf(2) ** -1500 * (1 + abs(ref_sq[k, i]))
        e = rel_err_per_k(xo, ref_sq)
        cond = sysm.meta["cond_A0_double"]
        for k in range(d + 1):
            assert e[k] <= tol(m, math.log2(cond) + math.log2(k + 1) + 2), (it, k, e)
        x = xo
    # converged: the update to the last coefficient is at the precision's
    # level relative to that coefficient
    xd = np.abs(x[0, 0, d] + 1j * x[1, 0, d]).max()
    assert nrm[0, 0] <= 2.0 ** -(53 * m - 12) * max(1.0, xd)
    # the same series as Newton on the square system
    xs, _, _ = oracle.newton(sysm, I.series_start(x0, d), 6)
    e = rel_err_per_k(x, mp_array(xs))
    assert np.all(e <= tol(m, 12)), e


# ----------------------------------------------------------------------------
# the protocol of Section 6 over increasing truncation degrees


@pytest.mark.parametrize("m", (2, 4, 8))
def test_protocol_iteration_counts_on_sqrt_series(m):
    """x^2 - (1 + t) = 0 from x = 1: Newton on series doubles the number of
    correct coefficients per step (t-adic quadratic convergence), and the
    coefficients binom(1/2, k) are dyadic, so after ceil(log2(d+1)) steps
    the series is exact and the next update is exactly zero.  Each degree
    therefore stops after ceil(log2(d+1)) + 1 steps (Section 6's counts at
    degrees 8 and 16 in penta, octo and deca double are 5 and 6, the same
    numbers), with the exact series."""
    degrees = (4, 8, 16)
    sysm, x = I.sqrt_system(m, 16)
    xo, iters, norms, st = oracle.newton_protocol(sysm, x[:, :, 0, :], degrees, (8, 8, 8),
                                                  1e-32, 1.0)
    assert st == 0
    assert iters == [math.ceil(math.log2(d + 1)) + 1 for d in degrees] == [4, 5, 6]
    assert not norms.any()
    c = Fraction(1)
    for k in range(17):
        assert fval(xo[0, :, k, 0]) == c
        c = c * (Fraction(1, 2) - k) / (k + 1)


def test_protocol_stops_at_the_step_limit_and_after_divergence():
    """A random double-double system: its updates stay above 1e-32 (the
    double-double rounding level), so every degree takes its full 8, 8,
    12, 16 steps (as quad double does in Section 6 at degree 8); with a
    divergence bound below what degree 8 ends with, the later degrees are
    not done and the status says so."""
    m = 2
    sysm, x0 = I.newton_system((922, 0), 6, m)
    x, iters, norms, st = oracle.newton_protocol(sysm, x0, (8, 16, 24, 32), (8, 8, 12, 16),
                                                 1e-32, 1.0)
    assert st == 0 and iters == [8, 8, 12, 16]
    assert np.all(norms[0] > 1e-32) and np.all(norms[0] < 1.0)
    # the last degree's series is 16 plain Newton steps from x0 at degree 32
    xs, nl, _ = oracle.newton(sysm, I.series_start(x0, 32), 16)
    assert np.array_equal(x, xs) and np.array_equal(norms[:, 3], nl[-1][:, 0])
    bound = float(norms[0, 0]) / 2
    x, iters, norms2, st = oracle.newton_protocol(sysm, x0, (8, 16, 24, 32), (8, 8, 12, 16),
                                                  1e-32, bound)
    assert st == oracle.ST_DIVERGED and iters == [8, 0, 0, 0]
    assert np.array_equal(norms2[:, 0], norms[:, 0]) and not norms2[:, 1:].any()
    xs, _, _ = oracle.newton(sysm, I.series_start(x0, 8), 8)
    assert np.array_equal(x[:, :, :9], xs) and not x[:, :, 9:].any()


def test_protocol_quad_double_converges_in_few_steps():
    """In quad double the same kind of system converges: each degree stops
    at the first step whose update to the last coefficient is at most 1e-32,
    after the ceil(log2(d+1)) steps that reach that coefficient."""
    m = 4
    sysm, x0 = I.newton_system((922, 1), 6, m)
    degrees = (8, 16, 24, 32)
    x, iters, norms, st = oracle.newton_protocol(sysm, x0, degrees, (8, 8, 12, 16), 1e-32, 1.0)
    assert st == 0
    for j, d in enumerate(degrees):
        xs, nl, _ = oracle.newton(sysm, I.series_start(x0, d), iters[j])
        vals = [float(fval(v[:, 0])) for v in nl]
        # the stop is at the first step from the second on at or below 1e-32
        assert vals[-1] <= 1e-32 and all(v > 1e-32 for v in vals[1:-1])
        assert iters[j] >= math.ceil(math.log2(d + 1))
    assert np.array_equal(x, xs)
