"""Algorithmic work of the series Newton path, in the units of Table 1.

Table 1 gives the hardware double operations (+, -, *, /) of one
multiple-double add, mul and div for m = 2, 3, 4, 5, 8, 10; a plain double
operation counts 1.  The functions below count the multiple-double
operations that each step of the method performs by definition (Section 3's
series product: (d+2)(d+1)/2 products and (d+1)d/2 additions; a complex
product is 4 real products and 2 additions, a complex addition 2 additions;
Section 4's evaluation / differentiation, Householder QR and staggered
solve) and weight them with Table 1.  The result is the algorithmic
operation count against which achieved throughput is compared with the
FP64 vector peak; it does not depend on how a kernel schedules the work.
"""
from __future__ import annotations

from dataclasses import dataclass, field

# Table 1 totals (+, -, *, / summed) per multiple-double add, mul, div
TABLE1 = {
    1: {"add": 1, "mul": 1, "div": 1},
    2: {"add": 20, "mul": 23, "div": 70},
    3: {"add": 35, "mul": 209, "div": 394},
    4: {"add": 89, "mul": 336, "div": 893},
    5: {"add": 122, "mul": 554, "div": 1553},
    8: {"add": 269, "mul": 1742, "div": 5126},
    10: {"add": 397, "mul": 3089, "div": 9208},
}

FP64_VECTOR_PEAK = 78.6e12   # MI355X, FMA counted as 2 flops
HBM_PEAK = 8.0e12            # bytes/s


@dataclass
class Ops:
    """Counts of multiple-double operations (md_muld counted apart)."""

    add: int = 0
    mul: int = 0
    div: int = 0
    muld: int = 0
    extra: dict = field(default_factory=dict)

    def __iadd__(self, o: "Ops"):
        self.add += o.add
        self.mul += o.mul
        self.div += o.div
        self.muld += o.muld
        return self

    def scaled(self, k: int) -> "Ops":
        return Ops(self.add * k, self.mul * k, self.div * k, self.muld * k)

    def table_ops(self, m: int) -> int:
        """Hardware double operations by Table 1 (a multiple double times a
        double is weighted as a multiplication)."""
        t = TABLE1[m]
        return self.add * t["add"] + (self.mul + self.muld) * t["mul"] + self.div * t["div"]


def _cmul(k=1):
    return Ops(add=2 * k, mul=4 * k)


def _cadd(k=1):
    return Ops(add=2 * k)


def _cabs2(k=1):
    return Ops(add=k, mul=2 * k)


def _cdiv(k=1):
    return Ops(add=3 * k, mul=6 * k, div=2 * k)


def rsqrt_iterations(m: int) -> int:
    it, p = 1, 1
    while p < m:
        p *= 2
        it += 1
    return it


def sqrt_ops(m: int) -> Ops:
    """1/sqrt by Newton steps (3 products, 2 additions each), then one product."""
    if m == 1:
        return Ops()
    it = rsqrt_iterations(m)
    return Ops(add=2 * it, mul=3 * it + 1)


def series_product(d: int, dx: int | None = None) -> Ops:
    """Product of a degree-dx series by a degree-d series, truncated at d."""
    dx = d if dx is None else min(dx, d)
    prods = sum(1 + min(k, dx) for k in range(d + 1))
    adds = sum(min(k, dx) for k in range(d + 1))
    o = _cmul(prods)
    o += _cadd(adds)
    return o


def convolve(d: int, count: int) -> Ops:
    return series_product(d).scaled(count)


def eval_diff(sysm, d: int) -> Ops:
    """Forward, backward and cross products, coefficient products,
    multiplicities and the accumulation into f and A (from zero)."""
    o = Ops()
    L = d + 1
    dcu = min(sysm.dc, d)
    for i in range(sysm.N):
        for _, fac in sysm.terms(i):
            D = len(fac)
            o += _cadd(L)  # f_i += value
            if D == 0:
                continue
            distinct = sorted(set(fac))
            o += _cadd(L * len(distinct))  # A_{i,l} += derivative
            o += series_product(d, dcu)    # value = c P_D
            if D == 1:
                continue
            o += series_product(d).scaled(D - 1)          # forward
            o += series_product(d).scaled(max(D - 2, 0))  # backward
            firsts = [j for j in range(2, D) if fac[j - 1] != fac[j - 2]]
            o += series_product(d).scaled(len(firsts))    # cross
            o += series_product(d, dcu).scaled(len(distinct))  # c * cross
            reps = sum(1 for v in distinct if fac.count(v) > 1)
            o.muld += 2 * L * reps
    return o


def qr(N: int, n: int, m: int) -> Ops:
    """Householder QR of an N x n matrix (nonzero diagonal entries and
    columns assumed)."""
    o = Ops()
    sq = sqrt_ops(m)
    for j in range(n):
        rows = N - j
        o += _cabs2(rows)
        o += Ops(add=rows - 1)
        o += sq.scaled(2)
        o += Ops(div=2)                       # phi
        o += Ops(add=1, mul=2 + 1 + 2, div=1)  # sp, v0, sigma*sp, beta, R_jj
        cols = n - 1 - j
        o += _cmul(rows).scaled(cols)         # w = v^H a
        o += _cadd(rows - 1).scaled(cols)
        o += Ops(mul=2 * cols)                # beta w
        o += _cmul(rows).scaled(cols)         # a -= (beta w) v
        o += _cadd(rows).scaled(cols)
    return o


def series_solve(N: int, n: int, d: int) -> Ops:
    """Staggered substitution: per stage Q^H r_k, back substitution, and the
    updates r_{k+j} -= A_j dx_k (Section 4)."""
    o = Ops()
    per_stage = Ops()
    for j in range(n):
        rows = N - j
        per_stage += _cmul(rows)
        per_stage += _cadd(rows - 1)
        per_stage += Ops(mul=2)
        per_stage += _cmul(rows)
        per_stage += _cadd(rows)
    for i in range(n):
        per_stage += _cmul(n - 1 - i)
        per_stage += _cadd(n - 1 - i)
        per_stage += _cdiv(1)
    o += per_stage.scaled(d + 1)
    upd = Ops()
    upd += _cmul(n)
    upd += _cadd(n - 1)
    upd += _cadd(1)
    o += upd.scaled(N * (d * (d + 1) // 2))
    return o


def newton_step(sysm, d: int, m: int) -> Ops:
    o = eval_diff(sysm, d)
    o += qr(sysm.N, sysm.n, m)
    o += series_solve(sysm.N, sysm.n, d)
    L = d + 1
    o += _cadd(L * sysm.n)     # x += dx
    o += _cabs2(L * sysm.n)    # |dx|^2
    o += sqrt_ops(m).scaled(2)
    return o


def adjoint(sysm, d: int, m: int) -> Ops:
    """Coefficient gradient through the converged series: evaluation and
    differentiation at x, the QR of A_0, the transposed staggered
    substitution (per stage A_0^H lambda_k = rhs_k through R^H and Q, and the
    updates rhs_{k-j} -= A_j^H lambda_k: the same counts as the forward
    solve), then per term and coefficient degree j the contraction
    sum_{k=j}^{d} conj(m_{k-j}) lambda_k (the monomial series m are the
    forward products, already counted in the evaluation)."""
    o = eval_diff(sysm, d)
    o += qr(sysm.N, sysm.n, m)
    o += series_solve(sysm.N, sysm.n, d)
    dcu = min(sysm.dc, d)
    for j in range(dcu + 1):
        o += _cmul(d + 1 - j).scaled(sysm.M)
        o += _cadd(d - j).scaled(sysm.M)
    return o
