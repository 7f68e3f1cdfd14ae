"""The library's fused complex multiply-add (c_fmadd: the four real products
as level sums, then s + p1 - p2 and s + p3 + p4 with one renormalisation
each, from three limbs on), compiled for the host from the device source
md.hpp, against exact rational arithmetic: never less accurate than the two
separate operations c_add(s, c_mul(a, b)) in the worst case over seeded
inputs, no worse on average, and md_mul (whose level sums it shares) bit for
bit the oracle's product.  Inputs: unit complex numbers at mixed scales,
and near-cancellation (s = -a b up to the last limb)."""
import os
import shutil
import subprocess
import tempfile
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_2012_06607_amd import inputs as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def driver():
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = os.path.join(tempfile.mkdtemp(prefix="md_host_"), "fused")
    subprocess.run([gxx, "-std=c++17", "-O2", "-ffp-contract=off",
                    "-I", os.path.join(HERE, "md_host"),
                    "-I", os.path.join(ROOT, "paper_2012_06607_amd", "csrc"),
                    os.path.join(HERE, "md_host", "fused_driver.cpp"), "-o", out], check=True)
    return out


def value(limbs) -> Fraction:
    return sum((Fraction(float(x)) for x in limbs), Fraction(0))


def cases(m: int, count: int, seed: int):
    """(s, a, b) as complex planes (2, m, count): scales 2^-20..2^20 for s and
    2^-10..2^10 for a; every fifth s is -(a b) with its last limb changed."""
    g = I.rng(971, m, seed)
    a = I.unit_complex(g, m, count)
    b = I.unit_complex(g, m, count)
    s = I.unit_complex(g, m, count)
    es = g.integers(-20, 21, count)
    ea = g.integers(-10, 11, count)
    s = s * np.ldexp(1.0, es)[None, None, :]
    a = a * np.ldexp(1.0, ea)[None, None, :]
    ab = oracle.elementwise("cmul", a, b)
    for t in range(0, count, 5):
        s[:, :, t] = -ab[:, :, t]
        s[0, m - 1, t] *= 1.5
    return s, a, b


@pytest.mark.parametrize("m,count", ((2, 200), (3, 300), (4, 300), (5, 200), (8, 120), (10, 100)))
def test_fused_multiply_add_against_exact(driver, m, count):
    s, a, b = cases(m, count, m)
    lines = [f"{m} {count}"]
    for t in range(count):
        vals = [s[0, :, t], s[1, :, t], a[0, :, t], a[1, :, t], b[0, :, t], b[1, :, t]]
        lines.append(" ".join(float(x).hex() for v in vals for x in v))
    r = subprocess.run([driver], input="\n".join(lines) + "\n", capture_output=True, text=True,
                       check=True)
    rows = [list(map(float.fromhex, ln.split())) for ln in r.stdout.strip().splitlines()]
    assert len(rows) == count
    prod = np.array([row[4 * m:5 * m] for row in rows]).T      # md_mul(a.re, b.re)
    assert np.array_equal(prod, oracle.elementwise("mul", a[0], b[0]))
    worst_f = worst_u = -10000.0
    sum_f = sum_u = 0.0
    for t, row in enumerate(rows):
        sr, si, ar, ai, br, bi = (value(v[:, t]) for v in (s[0], s[1], a[0], a[1], b[0], b[1]))
        er, ei = sr + ar * br - ai * bi, si + ar * bi + ai * br
        scale = max(abs(sr), abs(si), abs(ar * br), abs(ai * bi), abs(ar * bi), abs(ai * br))

        def lg(x):
            return float(np.log2(float(x / scale))) if x != 0 else -2000.0
        ef = max(lg(abs(value(row[0:m]) - er)), lg(abs(value(row[m:2 * m]) - ei)))
        eu = max(lg(abs(value(row[2 * m:3 * m]) - er)), lg(abs(value(row[3 * m:4 * m]) - ei)))
        worst_f, worst_u = max(worst_f, ef), max(worst_u, eu)
        sum_f += max(ef, -60.0 * m)
        sum_u += max(eu, -60.0 * m)
    print(f"m={m}: worst log2 error fused {worst_f:.1f}, separate {worst_u:.1f}; "
          f"mean {sum_f / count:.1f} / {sum_u / count:.1f}")
    assert worst_f <= worst_u + 0.5
    assert sum_f / count <= sum_u / count + 0.25
    assert worst_f <= -(53 * m - 6)
