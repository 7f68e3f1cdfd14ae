"""CPU oracle for the multiple-double series Newton step (test infrastructure).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The arithmetic lives in
``mdoracle.c`` (plain C, built with gcc -O2 -ffp-contract=off); this module
builds it and marshals numpy arrays.  It shares no code with the HIP path.

Array layout: complex planes (2, m, *S) float64, real planes (m, *S)
(limb 0 most significant).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading
from fractions import Fraction

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mdoracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB = os.path.join(_BUILD, "liboracle.so")
_lock = threading.Lock()
_lib = None

# operation codes of orc_elementwise
OPS = {"add": 0, "sub": 1, "mul": 2, "div": 3, "sqrt": 4, "rsqrt": 5, "muld": 6,
       "cadd": 7, "csub": 8, "cmul": 9, "cdiv": 10, "cabs2": 11}
REAL_OPS = ("add", "sub", "mul", "div", "sqrt", "rsqrt", "muld")

# counter slots of orc_get_counters
COUNTERS = ("add", "sub", "mul", "div", "fma", "sqrt", "md_add", "md_mul", "md_div", "md_muld")

ST_SINGULAR = 1
ST_NONFINITE = 2
ST_DIVERGED = 32

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc into oracle/_build/liboracle.so."""
    os.makedirs(_BUILD, exist_ok=True)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib() -> ctypes.CDLL:
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            i32, i64 = ctypes.c_int32, ctypes.c_int64
            L.orc_elementwise.argtypes = [i32, i32, i64, P, P, P]
            L.orc_norm2.argtypes = [i32, i64, P, P]
            L.orc_convolve.argtypes = [i32, i32, i64, P, P, P]
            L.orc_series_divide.argtypes = [i32, i32, i64, P, P, P, P]
            L.orc_eval_diff.argtypes = [i32, i32, i32, i32, i32, i32, P, P, P, P, P, P, P]
            L.orc_qr.argtypes = [i32, i32, i32, P, P, P, P, P]
            L.orc_series_solve.argtypes = [i32, i32, i32, i32, P, P, P, P, P, P, P]
            L.orc_newton_step.argtypes = [i32, i32, i32, i32, i32, i32, P, P, P, P, P, P, P]
            L.orc_newton_adjoint.argtypes = [i32, i32, i32, i32, i32, i32, P, P, P, P, P, P, P, P]
            L.orc_get_counters.argtypes = [P]
            L.orc_reset_counters.argtypes = []
            _lib = L
    return _lib


def _c(a: np.ndarray, dtype=np.float64) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=dtype)


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def reset_counters():
    lib().orc_reset_counters()


def counters() -> dict:
    out = np.zeros(len(COUNTERS), dtype=np.int64)
    lib().orc_get_counters(_p(out))
    return dict(zip(COUNTERS, (int(v) for v in out)))


def elementwise(op: str, a: np.ndarray, b: np.ndarray | None = None) -> np.ndarray:
    """One multiple-double operation per element.  Real ops take planes
    (m, count); complex ops (2, m, count); 'muld' multiplies by b's leading
    limb; 'cabs2' returns real planes."""
    a = _c(a)
    if op in REAL_OPS:
        m, count = a.shape
        out = np.zeros((m, count))
    else:
        _, m, count = a.shape
        out = np.zeros((m, count)) if op == "cabs2" else np.zeros((2, m, count))
    bb = _c(b) if b is not None else np.zeros_like(a)
    _check(lib().orc_elementwise(m, OPS[op], count, _p(a), _p(bb), _p(out)), op)
    return out


def norm2(x: np.ndarray) -> np.ndarray:
    """2-norm of a complex vector, planes (2, m, count) -> real limbs (m,)."""
    x = _c(x)
    _, m, count = x.shape
    out = np.zeros((m, 1))
    _check(lib().orc_norm2(m, count, _p(x), _p(out)), "norm2")
    return out[:, 0]


def convolve(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Truncated series products; planes (2, m, count, d+1)."""
    x, y = _c(x), _c(y)
    _, m, count, L = x.shape
    z = np.zeros_like(x)
    _check(lib().orc_convolve(m, L - 1, count, _p(x), _p(y), _p(z)), "convolve")
    return z


def series_divide(x: np.ndarray, y: np.ndarray):
    """z = x / y mod t^{d+1} per series, planes (2, m, count, d+1); returns
    (z, status) with ST_SINGULAR when some y_0 is zero."""
    x, y = _c(x), _c(y)
    assert x.shape == y.shape
    _, m, count, L = x.shape
    z = np.zeros_like(x)
    st = np.zeros(1, dtype=np.int32)
    _check(lib().orc_series_divide(m, L - 1, count, _p(x), _p(y), _p(z), _p(st)), "series_divide")
    return z, int(st[0])


def pade(c: np.ndarray, L: int, M: int):
    """[L/M] Pade approximants p(t)/q(t) of the series c (planes
    (2, m, count, L+M+1)), the rational approximations of Section 3 built
    from a computed series: q(t) = 1 + q_1 t + ... + q_M t^M and p(t) of
    degree L with q(t) c(t) - p(t) = O(t^{L+M+1}).  The coefficients of
    t^{L+1} .. t^{L+M} of q c vanish:
        sum_{j=1..M} c_{L+i-j} q_j = -c_{L+i},   i = 1..M  (c_k = 0, k < 0),
    an M x M Toeplitz system, solved by Householder QR (qr and
    series_solve at degree 0); then p_k = sum_{j=0..min(k,M)} q_j c_{k-j},
    k = 0..L (a truncated series product).  Returns (p planes
    (2, m, count, L+1), q planes (2, m, count, M+1), status)."""
    c = _c(c)
    _, m, count, K = c.shape
    assert K == L + M + 1 and L >= 0 and M >= 0
    p = np.zeros((2, m, count, L + 1))
    q = np.zeros((2, m, count, M + 1))
    status = 0
    for s in range(count):
        q[0, 0, s, 0] = 1.0
        if M > 0:
            T = np.zeros((2, m, M, M))
            rhs = np.zeros((2, m, M))
            for i in range(1, M + 1):
                for j in range(1, M + 1):
                    if L + i - j >= 0:
                        T[:, :, i - 1, j - 1] = c[:, :, s, L + i - j]
                rhs[:, :, i - 1] = -c[:, :, s, L + i]
            QR, vd, beta, st1 = qr(T)
            qs, st2 = series_solve(QR, vd, beta, T[:, :, None], rhs[:, :, None])
            q[:, :, s, 1:] = qs[:, :, 0, :]
            status |= st1 | st2
        qq = np.zeros((2, m, 1, L + 1))
        top = min(L, M)
        qq[:, :, 0, :top + 1] = q[:, :, s, :top + 1]
        p[:, :, s, :] = convolve(qq, c[:, :, s:s + 1, :L + 1])[:, :, 0, :]
    return p, q, status


def _sys_args(sysm):
    return (_c(sysm.eq_ptr, np.int32), _c(sysm.term_ptr, np.int32),
            _c(sysm.factors if sysm.factors.size else np.zeros(1, np.int32), np.int32),
            _c(sysm.coef))


def eval_diff(sysm, x: np.ndarray):
    """f(x(t)) (2, m, d+1, N) and A(t) (2, m, d+1, N, n) at x: (2, m, d+1, n)."""
    x = _c(x)
    _, m, L, n = x.shape
    N = sysm.N
    f = np.zeros((2, m, L, N))
    A = np.zeros((2, m, L, N, n))
    ep, tp, fa, co = _sys_args(sysm)
    _check(lib().orc_eval_diff(m, L - 1, N, n, sysm.M, sysm.dc, _p(ep), _p(tp), _p(fa), _p(co),
                               _p(x), _p(f), _p(A)), "eval_diff")
    return f, A


def qr(A0: np.ndarray):
    """Householder QR of A0 (2, m, N, n) -> (QR, vdiag, beta, status)."""
    A0 = _c(A0)
    _, m, N, n = A0.shape
    QR = np.zeros_like(A0)
    vd = np.zeros((2, m, n))
    beta = np.zeros((m, n))
    st = np.zeros(1, dtype=np.int32)
    _check(lib().orc_qr(m, N, n, _p(A0), _p(QR), _p(vd), _p(beta), _p(st)), "qr")
    return QR, vd, beta, int(st[0])


def series_solve(QR, vd, beta, A, b):
    """Staggered solve of A(t) dx(t) = b(t); returns (dx, status)."""
    QR, vd, beta, A, b = map(_c, (QR, vd, beta, A, b))
    _, m, L, N, n = A.shape
    dx = np.zeros((2, m, L, n))
    st = np.zeros(1, dtype=np.int32)
    _check(lib().orc_series_solve(m, N, n, L - 1, _p(QR), _p(vd), _p(beta), _p(A), _p(b), _p(dx),
                                  _p(st)), "series_solve")
    return dx, int(st[0])


def solve_toeplitz(A, b):
    """QR of A_0 then the staggered solve."""
    A = _c(A)
    QR, vd, beta, st1 = qr(A[:, :, 0])
    dx, st2 = series_solve(QR, vd, beta, A, b)
    return dx, st1 | st2


def newton_step(sysm, x: np.ndarray):
    """One Newton step; returns (new x, dx_norm (m, 2), status)."""
    x = _c(x).copy()
    _, m, L, n = x.shape
    nrm = np.zeros((m, 2))
    st = np.zeros(1, dtype=np.int32)
    ep, tp, fa, co = _sys_args(sysm)
    _check(lib().orc_newton_step(m, L - 1, sysm.N, n, sysm.M, sysm.dc, _p(ep), _p(tp), _p(fa),
                                 _p(co), _p(x), _p(nrm), _p(st)), "newton_step")
    return x, nrm, int(st[0])


def newton(sysm, x: np.ndarray, iters: int):
    """iters Newton steps from x; returns (x, list of dx_norm, status)."""
    norms = []
    status = 0
    for _ in range(iters):
        x, nrm, st = newton_step(sysm, x)
        norms.append(nrm)
        status |= st
    return x, norms, status


def _value(limbs) -> Fraction:
    """Exact value of a limb expansion."""
    return sum((Fraction(float(v)) for v in limbs), Fraction(0))


def newton_protocol(sysm, x0: np.ndarray, degrees, maxit, tol: float, diverge: float,
                    min_steps: int = 2):
    """Newton's method over increasing truncation degrees (Section 6): for
    each degree d_j, start from x(t) = x0 (higher coefficients zero) and
    take Newton steps until the modulus of the update to the last
    coefficient is at most tol (tested from step min_steps on: the first
    step from a constant series reaches only x_1 when t enters linearly), or
    maxit[j] steps are done; a degree that
    ends with that modulus above `diverge` ends the computations (the later
    degrees are not done).  The decisions compare exact values of the
    multiple-double norms with the double thresholds.

    x0: planes (2, m, n).  Returns (x planes (2, m, dmax+1, n): the series of
    the last degree done, zero above it; iters: steps per degree (0 when not
    done); norms: real planes (m, ndeg), the last modulus per degree (0 when
    not done); status: OR of the steps' status words, and ST_DIVERGED when a
    degree ended above the bound)."""
    x0 = _c(x0)
    _, m, n = x0.shape
    dmax = int(degrees[-1])
    x_out = np.zeros((2, m, dmax + 1, n))
    iters = [0] * len(degrees)
    norms = np.zeros((m, len(degrees)))
    status = 0
    tol_q, div_q = Fraction(tol), Fraction(diverge)
    for j, (d, mi) in enumerate(zip(degrees, maxit)):
        x = np.zeros((2, m, int(d) + 1, n))
        x[:, :, 0, :] = x0
        nrm = np.zeros((m, 2))
        for _ in range(int(mi)):
            x, nrm, st = newton_step(sysm, x)
            status |= st
            iters[j] += 1
            if iters[j] >= min_steps and _value(nrm[:, 0]) <= tol_q:
                break
        norms[:, j] = nrm[:, 0]
        x_out[:] = 0.0
        x_out[:, :, :int(d) + 1, :] = x
        if _value(nrm[:, 0]) > div_q:
            status |= ST_DIVERGED
            break
    return x_out, iters, norms, status


def newton_adjoint(sysm, x: np.ndarray, grad_x: np.ndarray):
    """Coefficient gradient (planes (2, 2, M, dc+1), double double) of a real
    loss with upstream gradient grad_x (planes like x) through the converged
    series x; returns (grad, status)."""
    x, grad_x = _c(x), _c(grad_x)
    _, m, L, n = x.shape
    g = np.zeros((2, 2, sysm.M, sysm.dc + 1))
    st = np.zeros(1, dtype=np.int32)
    ep, tp, fa, co = _sys_args(sysm)
    _check(lib().orc_newton_adjoint(m, L - 1, sysm.N, n, sysm.M, sysm.dc, _p(ep), _p(tp), _p(fa),
                                    _p(co), _p(x), _p(grad_x), _p(g), _p(st)), "newton_adjoint")
    return g, int(st[0])
