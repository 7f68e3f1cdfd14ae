"""Accuracy of the HIP path against a high-precision reference, next to the
oracle's accuracy on the same inputs.

Rule (per coefficient vector k of a series): with eps_X,k the relative error
max_i |x_{k,i} - ref_{k,i}| / max(||ref_k||, 2^-40 max_j ||ref_j||) of result
X against the reference,

    eps_GPU,k <= 2 eps_oracle,k + 2^-(53m-8).

The GPU may sum in other orders than the oracle, but it may not lose more
than a bit beyond the oracle's own error plus a few units of the precision.
The reference is the exact Newton step (or solve) at 2000 bits (mpmath's
dense solves, tests/exact.py) where that finishes in seconds; for the
64-unknown, degree-32 paths of the batched workload it is the oracle run in
octo double (424 bits) on the same inputs, whose own error lies about 200
bits below the quad-double level being judged.  Every test prints the
measured log2 errors.
"""
from __future__ import annotations

import concurrent.futures as cf
import math

import mpmath
import numpy as np
import pytest

import oracle
from exact import mp_array, mp_newton_step, mp_toeplitz_solve, planes_rel_err_per_k, \
    rel_err_per_k as mp_rel_err_per_k
from paper_2012_06607_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2012_06607_amd import binding
    binding.lib()
    return binding


@pytest.fixture(autouse=True)
def _prec():
    old = mpmath.mp.prec
    mpmath.mp.prec = 2000
    yield
    mpmath.mp.prec = old


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def lg(v):
    return [round(math.log2(e), 1) if e > 0 else -9999 for e in v]


def check_t2(eg, eo, m, what):
    bound = 2.0 * np.asarray(eo) + 2.0 ** -(53 * m - 8)
    print(f"{what}: log2 eps gpu {lg(eg)}", flush=True)
    print(f"{what}: log2 eps oracle {lg(eo)}", flush=True)
    bad = [k for k in range(len(eg)) if not eg[k] <= bound[k]]
    assert not bad, (what, bad, lg(eg), lg(eo))


def pad_limbs(a: np.ndarray, m: int, axis: int) -> np.ndarray:
    """The same values with m limbs (zeros appended)."""
    shape = list(a.shape)
    shape[axis] = m
    out = np.zeros(shape)
    idx = [slice(None)] * a.ndim
    idx[axis] = slice(0, a.shape[axis])
    out[tuple(idx)] = a
    return out


def padded_system(sysm, m):
    s = I.System(sysm.N, sysm.n, m, sysm.dc, sysm.eq_ptr, sysm.term_ptr, sysm.factors,
                 pad_limbs(sysm.coef, m, 1), dict(sysm.meta))
    return s


def newton_t2(B, sysm, x, steps, what):
    """For each listed step: the oracle's iterate is the common input, the
    reference is the exact Newton step from it at 2000 bits."""
    m = sysm.m
    sd = B.DeviceSystem(sysm)
    it = 0
    for it in range(max(steps) + 1):
        xw, _, stw = oracle.newton_step(sysm, x)
        assert stw == 0
        if it in steps:
            xg = dev(x)
            _, _, st = B.md_newton_step(sd, xg)
            assert int(host(st)[0]) == 0
            ref, _ = mp_newton_step(sysm, mp_array(x))
            check_t2(mp_rel_err_per_k(host(xg), ref), mp_rel_err_per_k(xw, ref), m,
                     f"{what} step {it}")
        x = xw


def test_t2_config1_plain_double_double(B):
    """n = 8, d = 8, double double: every one of the 8 steps."""
    m, d = 2, 8
    sysm, x0 = I.newton_system((0, 0), 8, m)
    newton_t2(B, sysm, I.series_start(x0, d), set(range(8)), "cfg1 dd n=8 d=8")


def test_t2_config5_quad_double_newton(B):
    """n = 32, d = 16, quad double (the adjoint's forward system): the first,
    a middle and the last of its 8 steps."""
    m, d = 4, 16
    sysm, x0 = I.newton_system((1202, 0), 32, m, terms=8)
    newton_t2(B, sysm, I.series_start(x0, d), {0, 3, 7}, "cfg5 qd n=32 d=16")


def solve_t2(B, A, b, what):
    m = A.shape[1]
    dxw, stw = oracle.solve_toeplitz(A, b)
    QR, vd, beta, st = B.md_qr(dev(A[:, :, 0]))
    dx, st2 = B.md_series_solve(QR, vd, beta, dev(A), dev(b))
    assert int(host(st)[0]) == 0 and int(host(st2)[0]) == 0 and stw == 0
    ref = mp_toeplitz_solve(mp_array(A), mp_array(b))
    check_t2(mp_rel_err_per_k(host(dx), ref), mp_rel_err_per_k(dxw, ref), m, what)


@pytest.mark.parametrize("m", (2, 4))
def test_t2_config2_solve(B, m):
    """n = 32, d = 16, A_0 = U diag U^H with condition number 1e3."""
    A, b = I.toeplitz_system((2, 32), 32, 16, m)
    solve_t2(B, A, b, f"cfg2 solve m={m} n=32 d=16 cond=1e3")


@pytest.mark.parametrize("m", (2, 4))
def test_t2_solve_condition_1e5(B, m):
    """The conditioning of the paper's cyclic 128-roots experiment (the
    inverse condition number of A_0 near 4.6e-6, Section 6): the GPU's
    stages (dx_k = W r_k with W = R^{-1} Q^H formed once) against the
    oracle's per-stage Q^H and back substitution."""
    A, b = I.toeplitz_system((2, 32, 5), 32, 16, m, cond=2e5)
    solve_t2(B, A, b, f"solve m={m} n=32 d=16 cond=2e5")


# ----------------------------------------------------------------------------
# the batched workload at its own sizes


def config4_sample():
    """A seeded sample of the benchmark's 1024 paths (n in {8..64}, d in
    8..32, half dd / half qd, config-1 systems): the largest quad-double
    path (n = 64, d = 32), the double-double paths of 64 unknowns at
    d >= 31 and a smaller quad-double path at d >= 31 (series products
    take the kernel's one-product-at-a-time branch at d >= 32 and its paired
    branch below)."""
    specs = I.batch_specs((4, 0), 1024)
    big_qd = [s for s in specs if s.m == 4 and s.n == 64 and s.d == 32]
    dd64 = ([s for s in specs if s.m == 2 and s.n == 64 and s.d == 32][:1]
            + [s for s in specs if s.m == 2 and s.n == 64 and s.d == 31][:1])
    qd_small = [s for s in specs if s.m == 4 and s.n <= 24 and s.d >= 31]
    pick = big_qd[:1] + dd64 + qd_small[:1]
    out = []
    for s in pick:
        sysm, x0 = I.newton_system((4, s.path), s.n, s.m)
        out.append((s, sysm, I.series_start(x0, s.d)))
    return out


def test_config4_sample_batched_against_oracle(B):
    """The sampled paths in one batched launch (4 Newton steps, one queue
    per accelerator die, the largest path as a gang of 2 workgroups) against
    oracle.newton after 4 steps, coefficient by coefficient (T2 rule, the
    reference being each path's 4 steps in octo double by the oracle)."""
    sample = config4_sample()
    assert sample[0][0].n == 64 and sample[0][0].d == 32 and sample[0][0].m == 4
    assert any(s.d == 32 and s.m == 2 for s, _, _ in sample)
    paths = [(sysm, x) for _, sysm, x in sample]
    iters = 4
    print("config-4 sample:", [(s.path, s.n, s.d, s.m) for s, _, _ in sample], flush=True)

    def ref_run(i):
        sysm, x = paths[i]
        mr = 8
        xr, _, st = oracle.newton(padded_system(sysm, mr), pad_limbs(x, mr, 1), iters)
        return xr, st

    def orc_run(i):
        sysm, x = paths[i]
        return oracle.newton(sysm, x, iters)

    with cf.ThreadPoolExecutor(max_workers=2 * len(paths)) as ex:
        refs = [ex.submit(ref_run, i) for i in range(len(paths))]
        orcs = [ex.submit(orc_run, i) for i in range(len(paths))]
        batch = B.BatchedPaths(paths)
        gangs = np.ones(len(paths), dtype=np.int64)
        gangs[0] = 2
        batch.set_schedule(nq=B.md_device_dies(), gangs=gangs)
        B.md_newton_batch(batch, iters, block=512)
        torch.cuda.synchronize()
        st = host(batch.status)
        got = [host(batch.x(p)).copy() for p in range(len(paths))]
        refs = [f.result() for f in refs]
        orcs = [f.result() for f in orcs]
    assert not st.any(), st
    for p, (s, sysm, _) in enumerate(sample):
        xr, str_ = refs[p]
        xw, _, stw = orcs[p]
        assert str_ == 0 and stw == 0
        m = sysm.m
        # the reference rounded to nothing: compare its m-limb planes' values
        # exactly against both results (limb sums, exact differences)
        eg = planes_rel_err_per_k(pad_limbs(got[p], 8, 1), xr)
        eo = planes_rel_err_per_k(pad_limbs(xw, 8, 1), xr)
        check_t2(eg, eo, m, f"cfg4 path {s.path} n={s.n} d={s.d} m={m} (4 steps, batched)")


# ----------------------------------------------------------------------------
# least squares: N = n + 7 equations (Section 4, N >= n; Section 6 augments a
# square system with 7 equations)


@pytest.mark.parametrize("m,n,d,steps", ((4, 32, 16, (0, 3, 7)), (2, 64, 8, (4,))))
def test_t2_overdetermined_newton(B, m, n, d, steps):
    """md_newton_step on a consistent system of n + 7 equations in n
    unknowns (the least-squares QR of an (n+7) x n A_0), against the exact
    least-squares step at 2000 bits, next to the oracle."""
    sysm, x0 = I.newton_system((1300, m, n), n, m)
    aug = I.augmented_system((1301, m, n), sysm, 7)
    assert aug.N == n + 7
    newton_t2(B, aug, I.series_start(x0, d), set(steps), f"N={n + 7} n={n} m={m} d={d}")


def test_batched_overdetermined_paths_against_oracle(B):
    """Paths of n + 7 equations in n unknowns (N up to 47) next to a square
    path in one batched launch, 4 Newton steps, against each path's 4 steps
    by the oracle in octo double (T2 rule), a gang of 2 on the largest."""
    cases = ((12, 10, 2), (24, 16, 4), (40, 12, 2), (17, 20, 4), (20, 9, 2))
    paths = []
    for idx, (n, d, m) in enumerate(cases):
        sysm, x0 = I.newton_system((1310, idx), n, m)
        if idx < 4:
            sysm = I.augmented_system((1311, idx), sysm, 7)
        paths.append((sysm, I.series_start(x0, d)))
    iters = 4
    print("overdetermined batch:", [(s.N, s.n, s.m, x.shape[2] - 1) for s, x in paths], flush=True)

    def ref_run(i):
        sysm, x = paths[i]
        return oracle.newton(padded_system(sysm, 8), pad_limbs(x, 8, 1), iters)

    def orc_run(i):
        sysm, x = paths[i]
        return oracle.newton(sysm, x, iters)

    with cf.ThreadPoolExecutor(max_workers=2 * len(paths)) as ex:
        refs = [ex.submit(ref_run, i) for i in range(len(paths))]
        orcs = [ex.submit(orc_run, i) for i in range(len(paths))]
        batch = B.BatchedPaths(paths)
        gangs = np.ones(len(paths), dtype=np.int64)
        gangs[int(np.argmax(batch.cost))] = 2
        batch.set_schedule(gangs=gangs)
        B.md_newton_batch(batch, iters, block=512)
        st = host(batch.status)
        got = [host(batch.x(p)).copy() for p in range(len(paths))]
        refs = [f.result() for f in refs]
        orcs = [f.result() for f in orcs]
    assert not st.any(), st
    for p, (sysm, _) in enumerate(paths):
        xr, _, str_ = refs[p]
        xw, _, stw = orcs[p]
        assert str_ == 0 and stw == 0
        eg = planes_rel_err_per_k(pad_limbs(got[p], 8, 1), xr)
        eo = planes_rel_err_per_k(pad_limbs(xw, 8, 1), xr)
        check_t2(eg, eo, sysm.m, f"batched N={sysm.N} n={sysm.n} m={sysm.m}")
