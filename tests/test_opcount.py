"""The analytic operation counts used for the roofline agree exactly with
the oracle's instrumented counters on the same inputs."""
from __future__ import annotations

import pytest

import oracle
from paper_2012_06607_amd import inputs as I
from paper_2012_06607_amd import opcount as OC


def oracle_ops():
    c = oracle.counters()
    return (c["md_add"], c["md_mul"], c["md_div"], c["md_muld"])


def analytic(o: OC.Ops):
    return (o.add, o.mul, o.div, o.muld)


def test_table1_totals_match_the_fixture():
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "table1_opcounts.json")))
    for m, row in gold["counts"].items():
        for op in ("add", "mul", "div"):
            assert OC.TABLE1[int(m)][op] == sum(row[op])


@pytest.mark.parametrize("d", (0, 5, 16))
def test_convolve_counts(d):
    x = I.unit_complex(I.rng(970, d), 2, 3, d + 1)
    oracle.reset_counters()
    oracle.convolve(x, x)
    assert oracle_ops() == analytic(OC.convolve(d, 3))


@pytest.mark.parametrize("key", ((0, 0), (1, 0)))
def test_eval_and_newton_counts(key):
    m, d = 2, 6
    sysm, x0 = I.newton_system(key, 6, m, terms=5, max_deg=4)
    x = I.series_start(x0, d)
    x[:, :, 1:] = I.unit_complex(I.rng(971), m, d, 6)  # nonzero higher coefficients
    oracle.reset_counters()
    oracle.eval_diff(sysm, x)
    assert oracle_ops() == analytic(OC.eval_diff(sysm, d))
    oracle.reset_counters()
    oracle.newton_step(sysm, x)
    got, want = oracle_ops(), analytic(OC.newton_step(sysm, d, m))
    # phi = alpha/|alpha| is skipped (2 divisions) where a diagonal entry of
    # the sparse Jacobian is exactly zero; the analytic count assumes none is
    assert got[:2] == want[:2] and got[3] == want[3]
    assert want[2] - 2 * sysm.n <= got[2] <= want[2] and (want[2] - got[2]) % 2 == 0


def test_eval_counts_with_coefficient_series_and_powers():
    m, d, dc = 3, 5, 3
    g = I.rng(972)

    def ser():
        c = I.unit_complex(g, m, dc + 1)
        return [(c[0, :, k], c[1, :, k]) for k in range(dc + 1)]
    sysm = I.build_system(2, 3, m, dc, [
        [((0, 0, 1), ser()), ((2,), ser()), ((), ser()), ((1, 1, 1, 2), ser())],
        [((0, 1, 2), ser()), ((0, 0, 0, 0), ser())]])
    x = I.unit_complex(g, m, d + 1, 3)
    oracle.reset_counters()
    oracle.eval_diff(sysm, x)
    assert oracle_ops() == analytic(OC.eval_diff(sysm, d))


@pytest.mark.parametrize("m,N,n,d", ((2, 6, 6, 4), (4, 9, 5, 3), (1, 4, 4, 2)))
def test_qr_and_solve_counts(m, N, n, d):
    g = I.rng(973, m, N)
    A = I.unit_complex(g, m, d + 1, N, n)
    b = I.unit_complex(g, m, d + 1, N)
    oracle.reset_counters()
    QR, vd, beta, _ = oracle.qr(A[:, :, 0])
    assert oracle_ops() == analytic(OC.qr(N, n, m))
    oracle.reset_counters()
    oracle.series_solve(QR, vd, beta, A, b)
    assert oracle_ops() == analytic(OC.series_solve(N, n, d))
