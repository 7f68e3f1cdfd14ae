"""Exact (rational) and 2000-bit references that pin the oracle.

Test infrastructure only.  Nothing here follows the oracle's algorithms:
series products are the plain definition, derivatives come from the power
rule on each monomial, and the linearised systems are solved with mpmath's
own dense solver at 2000 bits, so an error in the oracle's arithmetic, term
order, signs or indexing shows up as a mismatch.
"""
from __future__ import annotations

from fractions import Fraction

import mpmath
import numpy as np

PREC = 2000


def fval(limbs) -> Fraction:
    """Exact value of a limb sum."""
    return sum((Fraction(float(v)) for v in limbs), Fraction(0))


def cfrac(planes: np.ndarray, *idx) -> tuple[Fraction, Fraction]:
    return fval(planes[(0, slice(None), *idx)]), fval(planes[(1, slice(None), *idx)])


def mpf_of(limbs) -> mpmath.mpf:
    s = mpmath.mpf(0)
    for v in limbs:
        s += mpmath.mpf(float(v))
    return s


def mp_array(planes: np.ndarray) -> np.ndarray:
    """Object array of mpc with the logical shape of complex planes."""
    shape = planes.shape[2:]
    out = np.empty(shape, dtype=object)
    for idx in np.ndindex(*shape):
        out[idx] = mpmath.mpc(mpf_of(planes[(0, slice(None), *idx)]),
                              mpf_of(planes[(1, slice(None), *idx)]))
    return out


def smul(a, b, d: int):
    """Product of two series (lists of length >= d+1, missing = 0) mod t^{d+1}."""
    out = []
    for k in range(d + 1):
        s = mpmath.mpc(0)
        for i in range(k + 1):
            if i < len(a) and k - i < len(b):
                s += a[i] * b[k - i]
        out.append(s)
    return out


def mp_eval_diff(sysm, X: np.ndarray, d: int):
    """f (d+1, N) and A (d+1, N, n) as object arrays, by the power rule."""
    N, n = sysm.N, sysm.n
    C = mp_array(sysm.coef)  # (M, dc+1)
    f = np.empty((d + 1, N), dtype=object)
    A = np.empty((d + 1, N, n), dtype=object)
    f[...] = mpmath.mpc(0)
    A[...] = mpmath.mpc(0)
    one = [mpmath.mpc(1)] + [mpmath.mpc(0)] * d
    for i in range(N):
        for j, fac in sysm.terms(i):
            c = [C[j, k] for k in range(sysm.dc + 1)]
            prod = one
            for v in fac:
                prod = smul(prod, [X[k, v] for k in range(d + 1)], d)
            val = smul(c, prod, d)
            for k in range(d + 1):
                f[k, i] += val[k]
            for l in sorted(set(fac)):
                a = fac.count(l)
                rest = list(fac)
                rest.remove(l)
                pr = one
                for v in rest:
                    pr = smul(pr, [X[k, v] for k in range(d + 1)], d)
                der = smul(c, pr, d)
                for k in range(d + 1):
                    A[k, i, l] += a * der[k]
    return f, A


def mp_toeplitz_solve(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """dx (d+1, n) with A(t) dx(t) = b(t) mod t^{d+1}, dense solves of A_0
    at the current precision (least squares through the normal equations
    when N > n)."""
    L, N, n = A.shape
    A0 = mpmath.matrix(N, n)
    for i in range(N):
        for l in range(n):
            A0[i, l] = A[0, i, l]
    if N == n:
        A0inv = mpmath.inverse(A0)
    else:
        AH = A0.transpose_conj()
        A0inv = mpmath.inverse(AH * A0) * AH
    dx = np.empty((L, n), dtype=object)
    for k in range(L):
        r = [b[k, i] for i in range(N)]
        for j in range(1, k + 1):
            for i in range(N):
                s = mpmath.mpc(0)
                for l in range(n):
                    s += A[j, i, l] * dx[k - j, l]
                r[i] -= s
        for l in range(n):
            s = mpmath.mpc(0)
            for i in range(N):
                s += A0inv[l, i] * r[i]
            dx[k, l] = s
    return dx


def mp_newton_step(sysm, X: np.ndarray):
    d = X.shape[0] - 1
    f, A = mp_eval_diff(sysm, X, d)
    dx = mp_toeplitz_solve(A, -f)
    return X + dx, dx


def rel_err_per_k(planes: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Per coefficient k: max_i |x_{k,i} - ref_{k,i}| / max(||ref_k||, 2^-40 max_j ||ref_j||)."""
    got = mp_array(planes)
    L = ref.shape[0]
    nk = [max(abs(v) for v in np.ravel(ref[k])) for k in range(L)]
    floor = max(nk) * mpmath.mpf(2) ** -40
    out = np.zeros(L)
    for k in range(L):
        e = max(abs(g - r) for g, r in zip(np.ravel(got[k]), np.ravel(ref[k])))
        den = max(nk[k], floor)
        out[k] = float(e / den) if den != 0 else float(e)
    return out


def log2_or_floor(v: float) -> float:
    return float(np.log2(v)) if v > 0 else -4000.0


def frac_of_mpf(x) -> Fraction:
    """Exact rational value of an mpf."""
    sign, man, exp, _ = mpmath.mpf(x)._mpf_
    v = Fraction(man) * Fraction(2) ** exp if man else Fraction(0)
    return -v if sign else v


def _limb_sum_diff(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Exact (a - b) limb sums along axis 0, rounded to double at the end."""
    m = a.shape[0]
    flat_a = a.reshape(m, -1)
    flat_b = b.reshape(m, -1)
    out = np.empty(flat_a.shape[1])
    for e in range(flat_a.shape[1]):
        s = Fraction(0)
        for l in range(m):
            s += Fraction(float(flat_a[l, e])) - Fraction(float(flat_b[l, e]))
        out[e] = float(s)
    return out.reshape(a.shape[1:])


def cdiff(got: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """|got - ref| per element of complex planes (2, m, ...), from exact limb
    sums (a difference of limb-by-limb doubles would lose the tail)."""
    dr = _limb_sum_diff(got[0], ref[0])
    di = _limb_sum_diff(got[1], ref[1])
    return np.hypot(dr, di)


def rdiff(got: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """|got - ref| per element of real planes (m, ...)."""
    return np.abs(_limb_sum_diff(got, ref))


def planes_rel_err_per_k(got: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Per coefficient k of series planes (2, m, d+1, ...): max_i |got - ref| /
    max(max_i |ref_k|, 2^-40 max |ref|), all from exact limb sums."""
    d = cdiff(got, ref)
    r = np.hypot(ref[0].sum(axis=0), ref[1].sum(axis=0))
    L = d.shape[0]
    nk = np.array([r[k].max() for k in range(L)])
    floor = max(nk.max() * 2.0**-40, 1e-300)
    return np.array([d[k].max() / max(nk[k], floor) for k in range(L)])
