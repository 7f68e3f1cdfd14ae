"""Seeded synthetic inputs for the series Newton path, shared by the tests,
the benchmark and the CPU baseline.

This module holds no multiple-double arithmetic.  Every value it produces is
built in exact rational arithmetic (Python integers) and then rounded to m
limbs by greedy extraction: limb_i = RN(v - (limb_0 + ... + limb_{i-1})),
each rounding done by Python's correctly rounded int/int division.  The
limbs therefore form a non-overlapping expansion of v (Section 2: a
multiple double is an unevaluated sum of hardware doubles).

Random unit complex numbers, the paper's test data cos(theta) + i sin(theta)
with random theta (Section 2, the 2-norm example), are made exactly on the
unit circle through the rational parametrisation
    s = tan(theta/2),  cos = (1 - s^2)/(1 + s^2),  sin = 2 s/(1 + s^2),
with s the double nearest tan(theta/2); the point lies exactly on the circle
and its angle is theta up to one rounding of s.

Layout of every array returned here: a complex multiple-double tensor of
logical shape S is a float64 numpy array of shape (2, m, *S); index 0 of the
first axis is the real part, 1 the imaginary part, limb 0 is the most
significant.  Series vectors are coefficient-major, shape (d+1, n), and
Jacobian series are (d+1, N, n) (Section 4: power series with vector and
matrix coefficients).

A polynomial system (Section 4: f = (f_1..f_N) in x = (x_1..x_n) with power
series coefficients in t) is held in compressed form:
    eq_ptr[N+1]   terms of equation i are eq_ptr[i] .. eq_ptr[i+1]-1
    term_ptr[M+1] factors of term j are factors[term_ptr[j] .. term_ptr[j+1]-1]
    factors[F]    variable indices with repetition, non-decreasing per term
    coef          planes (2, m, M, dc+1): the coefficient series of each term
A term with no factors is a constant (or, with a t coefficient, a t-term).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 201206607

# -----------------------------------------------------------------------------
# seeding


def rng(*key: int) -> np.random.Generator:
    """Generator for a (config, path, stream...) key."""
    return np.random.default_rng(np.random.SeedSequence([SEED_BASE, *[int(k) for k in key]]))


# -----------------------------------------------------------------------------
# exact rationals -> limbs


def limbs_of_ratio(P: int, Q: int, m: int) -> list[float]:
    """Greedy m-limb expansion of the rational P/Q (Q > 0)."""
    out: list[float] = []
    for _ in range(m):
        if P == 0:
            out.append(0.0)
            continue
        x = P / Q
        out.append(x)
        if x == 0.0:  # below the double range: the rest stays zero
            P = 0
            continue
        a, b = x.as_integer_ratio()
        P, Q = P * b - a * Q, Q * b
    return out


def dyadic_of_limbs(limbs) -> tuple[int, int]:
    """Exact value of a limb sum as (N, K) meaning N / 2**K."""
    K = 0
    parts = []
    for v in limbs:
        v = float(v)
        if v == 0.0:
            continue
        a, b = v.as_integer_ratio()
        k = b.bit_length() - 1
        parts.append((a, k))
        K = max(K, k)
    N = sum(a << (K - k) for a, k in parts)
    return N, K


class CDy:
    """Exact complex dyadic rational (R + i I) / 2**K, used only to build
    inputs (constant terms that make a chosen point a root)."""

    __slots__ = ("R", "I", "K")

    def __init__(self, R: int, I: int, K: int):
        self.R, self.I, self.K = R, I, K

    @staticmethod
    def from_limbs(re_limbs, im_limbs) -> "CDy":
        R, KR = dyadic_of_limbs(re_limbs)
        I, KI = dyadic_of_limbs(im_limbs)
        K = max(KR, KI)
        return CDy(R << (K - KR), I << (K - KI), K)

    def __mul__(self, o: "CDy") -> "CDy":
        return CDy(self.R * o.R - self.I * o.I, self.R * o.I + self.I * o.R, self.K + o.K)

    def __add__(self, o: "CDy") -> "CDy":
        K = max(self.K, o.K)
        return CDy((self.R << (K - self.K)) + (o.R << (K - o.K)),
                   (self.I << (K - self.K)) + (o.I << (K - o.K)), K)

    def __neg__(self) -> "CDy":
        return CDy(-self.R, -self.I, self.K)

    def limbs(self, m: int) -> tuple[list[float], list[float]]:
        return limbs_of_ratio(self.R, 1 << self.K, m), limbs_of_ratio(self.I, 1 << self.K, m)


# -----------------------------------------------------------------------------
# planes


def zeros(m: int, *shape: int) -> np.ndarray:
    return np.zeros((2, m, *shape), dtype=np.float64)


def leading(planes: np.ndarray) -> np.ndarray:
    """Leading limbs as complex128 (for conditioning checks and display)."""
    return planes[0, 0] + 1j * planes[1, 0]


def unit_complex(g: np.random.Generator, m: int, *shape: int) -> np.ndarray:
    """Planes (2, m, *shape) of random points exactly on the unit circle,
    angle theta ~ U[0, 2 pi), rounded to m limbs."""
    count = int(np.prod(shape)) if shape else 1
    theta = g.uniform(0.0, 2.0 * math.pi, size=count)
    out = np.zeros((2, m, count), dtype=np.float64)
    for e, th in enumerate(theta):
        s = math.tan(0.5 * float(th))
        a, b = s.as_integer_ratio()
        a2, b2 = a * a, b * b
        den = a2 + b2
        out[0, :, e] = limbs_of_ratio(b2 - a2, den, m)
        out[1, :, e] = limbs_of_ratio(2 * a * b, den, m)
    return out.reshape((2, m, *shape))


def real_rational(m: int, values) -> np.ndarray:
    """Planes (2, m, len(values)) of real rationals given as (P, Q) pairs."""
    out = np.zeros((2, m, len(values)), dtype=np.float64)
    for e, (P, Q) in enumerate(values):
        out[0, :, e] = limbs_of_ratio(P, Q, m)
    return out


def cdy_at(planes: np.ndarray, *idx) -> CDy:
    return CDy.from_limbs(planes[(0, slice(None), *idx)], planes[(1, slice(None), *idx)])


# -----------------------------------------------------------------------------
# polynomial systems


@dataclass
class System:
    """A polynomial system with truncated power series coefficients."""

    N: int
    n: int
    m: int
    dc: int
    eq_ptr: np.ndarray  # int32 [N+1]
    term_ptr: np.ndarray  # int32 [M+1]
    factors: np.ndarray  # int32 [F]
    coef: np.ndarray  # float64 planes (2, m, M, dc+1)
    meta: dict = field(default_factory=dict)

    @property
    def M(self) -> int:
        return int(self.term_ptr.shape[0] - 1)

    @property
    def max_deg(self) -> int:
        if self.M == 0:
            return 0
        return int(np.max(np.diff(self.term_ptr)))

    def terms(self, i: int):
        """(term index, factor tuple) for equation i."""
        for j in range(int(self.eq_ptr[i]), int(self.eq_ptr[i + 1])):
            yield j, tuple(int(v) for v in self.factors[self.term_ptr[j]:self.term_ptr[j + 1]])


def build_system(N: int, n: int, m: int, dc: int, equations) -> System:
    """equations: list over i of lists of (factor tuple, coefficient series)
    where each coefficient series is a list (length <= dc+1) of (re limbs,
    im limbs) pairs or None for zero."""
    eq_ptr = [0]
    term_ptr = [0]
    factors: list[int] = []
    coefs = []
    for terms in equations:
        for fac, cser in terms:
            fac = tuple(sorted(int(v) for v in fac))
            factors.extend(fac)
            term_ptr.append(len(factors))
            coefs.append(cser)
        eq_ptr.append(len(term_ptr) - 1)
    M = len(coefs)
    coef = np.zeros((2, m, M, dc + 1), dtype=np.float64)
    for j, cser in enumerate(coefs):
        for k, c in enumerate(cser):
            if c is None:
                continue
            coef[0, :, j, k] = c[0]
            coef[1, :, j, k] = c[1]
    return System(N, n, m, dc,
                  np.asarray(eq_ptr, dtype=np.int32), np.asarray(term_ptr, dtype=np.int32),
                  np.asarray(factors, dtype=np.int32), coef)


def random_monomials(g: np.random.Generator, n: int, count: int, max_deg: int, min_deg: int = 1):
    """count distinct monomials in n variables; degree D ~ U{min_deg..max_deg},
    D variable indices drawn uniformly with replacement and sorted."""
    seen = set()
    out = []
    while len(out) < count:
        D = int(g.integers(min_deg, max_deg + 1))
        fac = tuple(sorted(int(v) for v in g.integers(0, n, size=D)))
        if fac in seen:
            continue
        seen.add(fac)
        out.append(fac)
    return out


def _jacobian_at(n: int, mons_per_eq, coefs_per_eq, x0: np.ndarray) -> np.ndarray:
    """Double-precision Jacobian at t = 0, used only to reject badly
    conditioned seeds."""
    J = np.zeros((len(mons_per_eq), n), dtype=np.complex128)
    for i, (mons, cs) in enumerate(zip(mons_per_eq, coefs_per_eq)):
        for fac, c in zip(mons, cs):
            for v in set(fac):
                a = fac.count(v)
                rest = list(fac)
                rest.remove(v)
                J[i, v] += c * a * np.prod([x0[u] for u in rest])
    return J


def newton_system(key, n: int, m: int, terms: int = 8, max_deg: int = 3,
                  cond_max: float = 1e3, max_tries: int = 1000):
    """Random square system with a known root at t = 0.

    Each of the n equations holds `terms` distinct monomials of degree
    1..max_deg with unit complex coefficients, a constant term chosen so
    that a random unit complex vector x0 solves the system at t = 0
    (computed exactly from the rounded coefficients and x0, then rounded to
    m limbs), and a term c*t with |c| = 1.  Seeds whose Jacobian at x0 has
    2-norm condition number above cond_max are redrawn.

    Returns (System with dc = 1, x0 planes (2, m, n))."""
    for attempt in range(max_tries):
        g = rng(*key, attempt)
        x0 = unit_complex(g, m, n)
        mons = [random_monomials(g, n, terms, max_deg) for _ in range(n)]
        cmono = [unit_complex(g, m, terms) for _ in range(n)]
        ct = unit_complex(g, m, n)
        x0l = leading(x0)
        J = _jacobian_at(n, mons, [leading(c) for c in cmono], x0l)
        s = np.linalg.svd(J, compute_uv=False)
        if s[-1] == 0 or s[0] / s[-1] > cond_max:
            continue
        xd = [cdy_at(x0, v) for v in range(n)]
        equations = []
        for i in range(n):
            eq = []
            acc = CDy(0, 0, 0)
            for j, fac in enumerate(mons[i]):
                c = cdy_at(cmono[i], j)
                val = c
                for v in fac:
                    val = val * xd[v]
                acc = acc + val
                eq.append((fac, [(cmono[i][0, :, j], cmono[i][1, :, j])]))
            c0 = (-acc).limbs(m)
            eq.append(((), [c0]))
            eq.append(((), [None, (ct[0, :, i], ct[1, :, i])]))
            equations.append(eq)
        sysm = build_system(n, n, m, 1, equations)
        sysm.meta = {"cond_A0_double": float(s[0] / s[-1]), "attempt": attempt}
        return sysm, x0
    raise RuntimeError("no well conditioned system found")


def augmented_system(key, sysm: System, extra: int = 7) -> System:
    """N = n + extra equations in n unknowns that are consistent exactly:
    the first n equations are those of the square system `sysm`, and each
    appended one is 2^a f_i + 2^b f_j for a random pair i != j and
    a, b in {-1, 0, 1}, written as the two equations' terms side by side
    with their coefficients scaled (powers of two scale exactly, and the
    terms are not merged).  Every solution series of the square system
    solves the augmented one with zero residual, so the least-squares
    Newton step (QR of the N x n matrix A_0) has the square system's
    solution as its fixed point (Section 4, N >= n; Section 6 augments a
    square system with extra equations in the same way in spirit)."""
    g = rng(*key)
    equations = []
    for i in range(sysm.N):
        eq = []
        for j, fac in sysm.terms(i):
            eq.append((fac, [(sysm.coef[0, :, j, k], sysm.coef[1, :, j, k])
                             for k in range(sysm.dc + 1)]))
        equations.append(eq)
    pairs = []
    for _ in range(extra):
        i, j = (int(v) for v in g.choice(sysm.N, size=2, replace=False))
        a, b = (int(v) for v in g.integers(-1, 2, size=2))
        pairs.append((i, j, a, b))
        eq = []
        for src, e in ((i, a), (j, b)):
            sc = math.ldexp(1.0, e)
            for t, fac in sysm.terms(src):
                eq.append((fac, [(sysm.coef[0, :, t, k] * sc, sysm.coef[1, :, t, k] * sc)
                                 for k in range(sysm.dc + 1)]))
        equations.append(eq)
    out = build_system(sysm.N + extra, sysm.n, sysm.m, sysm.dc, equations)
    out.meta = dict(sysm.meta)
    out.meta["appended"] = pairs
    return out


def series_start(x0: np.ndarray, d: int) -> np.ndarray:
    """x(t) = x0 + 0 t + ... as planes (2, m, d+1, n)."""
    two, m, n = x0.shape
    x = np.zeros((2, m, d + 1, n), dtype=np.float64)
    x[:, :, 0, :] = x0
    return x


def eval_system(key, N: int, n: int, m: int, terms: int = 16, max_deg: int = 4):
    """N equations in n variables, `terms` distinct monomials of degree
    1..max_deg per equation, unit complex coefficients (dc = 0)."""
    g = rng(*key)
    equations = []
    for i in range(N):
        mons = random_monomials(g, n, terms, max_deg)
        c = unit_complex(g, m, terms)
        equations.append([(fac, [(c[0, :, j], c[1, :, j])]) for j, fac in enumerate(mons)])
    return build_system(N, n, m, 0, equations)


def unit_series(key, m: int, d: int, n: int) -> np.ndarray:
    """Series point with unit complex coefficients, planes (2, m, d+1, n)."""
    return unit_complex(rng(*key), m, d + 1, n)


# -----------------------------------------------------------------------------
# block Toeplitz systems A(t) dx(t) = b(t)


def _haar_unitary_double(g: np.random.Generator, n: int) -> np.ndarray:
    Z = (g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))) / math.sqrt(2.0)
    Q, R = np.linalg.qr(Z)
    ph = np.diag(R) / np.abs(np.diag(R))
    return Q * ph[None, :]


def conditioned_matrix(g: np.random.Generator, n: int, m: int, cond: float = 1e3) -> np.ndarray:
    """A = U diag(s) U^H with U a double-precision Haar unitary and
    s_j = cond**(j/(n-1)); the product is formed exactly from the doubles
    and rounded to m limbs.  Planes (2, m, n, n)."""
    U = _haar_unitary_double(g, n)
    s = [cond ** (j / (n - 1)) if n > 1 else 1.0 for j in range(n)]
    # exact fixed point: every double here is an integer multiple of 2**-1100
    SH = 1100

    def fx(v: float) -> int:
        a, b = float(v).as_integer_ratio()
        return (a << SH) // b  # exact: b divides 2**SH for these magnitudes

    Ur = [[fx(U[i, l].real) for l in range(n)] for i in range(n)]
    Ui = [[fx(U[i, l].imag) for l in range(n)] for i in range(n)]
    S = [fx(v) for v in s]
    out = np.zeros((2, m, n, n), dtype=np.float64)
    den = 1 << (3 * SH)
    for i in range(n):
        for j in range(n):
            re = 0
            im = 0
            for l in range(n):
                # U_il * s_l * conj(U_jl)
                ar, ai = Ur[i][l], Ui[i][l]
                br, bi = Ur[j][l], -Ui[j][l]
                pr = ar * br - ai * bi
                pi = ar * bi + ai * br
                re += pr * S[l]
                im += pi * S[l]
            out[0, :, i, j] = limbs_of_ratio(re, den, m)
            out[1, :, i, j] = limbs_of_ratio(im, den, m)
    return out


def toeplitz_system(key, n: int, d: int, m: int, cond: float = 1e3):
    """A(t) = A_0 + ... + A_d t^d with A_0 = U diag U^H (condition number
    `cond`) and A_k (k >= 1), b_k with unit complex entries.
    Returns (A planes (2, m, d+1, n, n), b planes (2, m, d+1, n))."""
    g = rng(*key)
    A = np.zeros((2, m, d + 1, n, n), dtype=np.float64)
    A[:, :, 0] = conditioned_matrix(g, n, m, cond)
    if d > 0:
        A[:, :, 1:] = unit_complex(g, m, d, n, n)
    b = unit_complex(g, m, d + 1, n)
    return A, b


# -----------------------------------------------------------------------------
# the paper's fixed examples


def circle_system(m: int, d: int = 8):
    """Section 3: { t - t^3/6 + t^5/120 - t^7/5040 - y = 0, x^2 + y^2 - 1 = 0 }
    in the unknowns (x, y) = (x_0, x_1), started at x = 1, y = 0.
    Returns (System, start series planes (2, m, d+1, 2))."""
    dc = 7
    sin_coefs = [None, (1, 1), None, (-1, 6), None, (1, 120), None, (-1, 5040)]

    def real(P, Q):
        return (limbs_of_ratio(P, Q, m), [0.0] * m)

    cser = [None if c is None else real(*c) for c in sin_coefs]
    eq1 = [((), cser), ((1,), [real(-1, 1)])]
    eq2 = [((0, 0), [real(1, 1)]), ((1, 1), [real(1, 1)]), ((), [real(-1, 1)])]
    sysm = build_system(2, 2, m, dc, [eq1, eq2])
    x = np.zeros((2, m, d + 1, 2))
    x[0, 0, 0, 0] = 1.0
    return sysm, x


def sqrt_system(m: int, d: int):
    """x^2 - (1 + t) = 0 started at x = 1: the solution series is sqrt(1+t)."""
    def real(P, Q):
        return (limbs_of_ratio(P, Q, m), [0.0] * m)

    eq = [((0, 0), [real(1, 1)]), ((), [real(-1, 1), real(-1, 1)])]
    sysm = build_system(1, 1, m, 1, [eq])
    x = np.zeros((2, m, d + 1, 1))
    x[0, 0, 0, 0] = 1.0
    return sysm, x


# -----------------------------------------------------------------------------
# batched workload: many independent paths of uneven size and precision


@dataclass
class PathSpec:
    path: int
    n: int
    d: int
    m: int


def batch_specs(key, count: int = 1024, n_choices=(8, 16, 24, 32, 40, 48, 56, 64),
                d_range=(8, 32), m_choices=(2, 4)) -> list[PathSpec]:
    """n uniform in n_choices, d uniform in d_range (inclusive), precision
    exactly half and half over m_choices, shuffled by the seed."""
    g = rng(*key)
    ns = g.choice(np.asarray(n_choices), size=count)
    ds = g.integers(d_range[0], d_range[1] + 1, size=count)
    ms = np.asarray([m_choices[i * len(m_choices) // count] for i in range(count)])
    g.shuffle(ms)
    return [PathSpec(i, int(ns[i]), int(ds[i]), int(ms[i])) for i in range(count)]
