"""GPU parity: the HIP path through the C ABI against the oracle.

Single multiple-double operations and the series product entry point run
the same operation sequence on both sides and must agree bit for bit.  The
evaluation kernel splits each coefficient's products over lanes, and QR,
the staggered solve and the Newton step sum in a different (tree) order on
the GPU, so they are compared within the per-coefficient tolerance
2^-(53m-8), widened for the solves by log2 of the condition number of A_0
and log2(k+1) for coefficient k (the paper's accuracy-loss argument,
Section 4).
"""
from __future__ import annotations

import math

import numpy as np
import pytest

import oracle
from exact import cdiff, planes_rel_err_per_k as rel_err_per_k, rdiff
from paper_2012_06607_amd import inputs as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ALL_M = (1, 2, 3, 4, 5, 8, 10)


@pytest.fixture(scope="module")
def B():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2012_06607_amd import binding
    binding.lib()
    return binding


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def tol(m, extra_bits=0.0):
    return 2.0 ** -(53 * m - 8 - extra_bits)


def rand_md(g, m, count):
    out = np.zeros((m, count))
    for e in range(count):
        P = int(g.integers(1, 2**62)) * (1 << 700) + int.from_bytes(g.bytes(88), "little")
        Q = 1 << (762 - int(g.integers(-30, 31)))
        out[:, e] = I.limbs_of_ratio(-P if g.random() < 0.5 else P, Q, m)
    return out


# ----------------------------------------------------------------------------
# single operations


def test_hardware_division_and_sqrt_are_correctly_rounded(B):
    """The quotient digits and square root seeds use the hardware double
    division and square root; they must round like the host's IEEE ones."""
    g = np.random.default_rng(7)
    a = g.standard_normal((1, 200000)) * 2.0 ** g.integers(-300, 300, size=(1, 200000))
    b = g.standard_normal((1, 200000)) * 2.0 ** g.integers(-300, 300, size=(1, 200000))
    a[0, :100] = 2.0 ** -1070 * g.random(100)   # subnormal operands
    assert np.array_equal(host(B.md_elementwise("div", dev(a), dev(b)))[0], a[0] / b[0])
    assert np.array_equal(host(B.md_elementwise("sqrt", dev(np.abs(a))))[0], np.sqrt(np.abs(a[0])))
    assert np.array_equal(host(B.md_elementwise("rsqrt", dev(np.abs(a))))[0],
                          1.0 / np.sqrt(np.abs(a[0])))


@pytest.mark.parametrize("m", ALL_M)
def test_operations_bit_exact(B, m):
    g = I.rng(950, m)
    n = 3000
    a, b = rand_md(g, m, n), rand_md(g, m, n)
    b[:, :300] = -a[:, :300]                 # exact cancellation
    b[:, 300:600] = a[:, 300:600]
    b[1:, 600:900] = 0.0                     # b a plain double
    a[:, 900:1000] = 0.0                     # zero operands
    for op in ("add", "sub", "mul", "div", "muld"):
        want = oracle.elementwise(op, a, b)
        got = host(B.md_elementwise(op, dev(a), dev(b)))
        same = (want == got) | (np.isnan(want) & np.isnan(got))
        assert same.all(), (op, np.argwhere(~same)[:5])
    pa = a * np.sign(a[0])[None, :]
    for op in ("sqrt", "rsqrt"):
        want = oracle.elementwise(op, pa)
        got = host(B.md_elementwise(op, dev(pa)))
        same = (want == got) | (np.isnan(want) & np.isnan(got))
        assert same.all(), (op, np.argwhere(~same)[:5])
    x = np.stack([a, b])
    y = np.stack([b[:, ::-1], a[:, ::-1]]).copy()
    for op in ("cadd", "csub", "cmul", "cdiv", "cabs2"):
        want = oracle.elementwise(op, x, y)
        got = host(B.md_elementwise(op, dev(x), dev(y)))
        same = (want == got) | (np.isnan(want) & np.isnan(got))
        assert same.all(), (op, np.argwhere(~same)[:5])


@pytest.mark.parametrize("m", (2, 3, 4, 5, 8, 10))
def test_two_norm_example(B, m):
    """Section 2: the 2-norm of 64 unit complex numbers is 8."""
    x = I.unit_complex(I.rng(951, m), m, 64)
    got = host(B.md_norm2(dev(x)))[:, 0]
    want = oracle.norm2(x)
    assert got[0] == 8.0
    assert abs(got[1]) <= 8.0 * tol(m)
    assert rdiff(got[:, None], want[:, None]).max() <= 8.0 * 2.0 ** -(53 * m - 4)
    # a ragged count above one workgroup
    x = I.unit_complex(I.rng(952, m), m, 300)
    got = host(B.md_norm2(dev(x)))[:, 0]
    assert abs(got[0] - math.sqrt(300.0)) < 1e-12


# ----------------------------------------------------------------------------
# series products


@pytest.mark.parametrize("m", ALL_M)
@pytest.mark.parametrize("count,d", ((64, 32), (3, 0), (5, 1), (7, 8), (130, 17)))
def test_convolve_bit_exact(B, m, count, d):
    if m == 10 and count == 130:
        pytest.skip("covered by the 64 x 32 case")
    g = I.rng(953, m, count, d)
    x = I.unit_complex(g, m, count, d + 1)
    y = I.unit_complex(g, m, count, d + 1)
    want = oracle.convolve(x, y)
    got = host(B.md_series_convolve(dev(x), dev(y)))
    assert np.array_equal(got, want)


@pytest.mark.parametrize("m,count,d", ((10, 1, 400), (2, 2, 400), (2, 70000, 0), (4, 1, 1)))
def test_convolve_long_series_and_many_tasks(B, m, count, d):
    # deca double at d = 400 does not fit in LDS (the one-thread-per-pair
    # form); 70000 one-coefficient series are more workgroup tasks than the
    # grid holds (the workgroups loop)
    g = I.rng(954, m, count, d)
    x = I.unit_complex(g, m, count, d + 1)
    y = I.unit_complex(g, m, count, d + 1)
    want = oracle.convolve(x, y)
    got = host(B.md_series_convolve(dev(x), dev(y)))
    assert np.array_equal(got, want)


def test_convolve_empty(B):
    x = torch.zeros((2, 2, 0, 9), dtype=torch.float64, device="cuda")
    z = B.md_series_convolve(x, x)
    assert z.shape == x.shape


# ----------------------------------------------------------------------------
# evaluation and differentiation


def small_system(m, dc):
    g = I.rng(954, m, dc)

    def ser():
        c = I.unit_complex(g, m, dc + 1)
        return [(c[0, :, k], c[1, :, k]) for k in range(dc + 1)]
    eqs = [
        [((0, 0, 1), ser()), ((2,), ser()), ((), ser())],
        [((0, 1, 1, 2), ser()), ((1, 1), ser()), ((0, 2), ser()), ((), ser())],
        [((2, 2, 2), ser()), ((0, 1, 2), ser()), ((1,), ser()), ((0, 0, 0, 0, 0), ser())],
    ]
    return I.build_system(3, 3, m, dc, eqs)


def eval_close(got, want, m, bits=4):
    """Per coefficient: |gpu - oracle| <= 2^-(53m - 8 - bits) of the
    coefficient's largest entry (products summed in another order)."""
    e = rel_err_per_k(got, want)
    assert np.all(e <= tol(m, bits)), e


@pytest.mark.parametrize("m", ALL_M)
@pytest.mark.parametrize("dc,d", ((0, 6), (3, 6), (7, 4), (1, 0)))
def test_eval_diff_small(B, m, dc, d):
    sysm = small_system(m, dc)
    x = I.unit_complex(I.rng(955, m, d), m, d + 1, 3)
    fw, Aw = oracle.eval_diff(sysm, x)
    sd = B.DeviceSystem(sysm)
    f, A = B.md_poly_eval_diff(sd, dev(x))
    eval_close(host(f), fw, m)
    eval_close(host(A), Aw, m)


def test_eval_diff_32x32_quad_double(B):
    """The 32 x 32 system of 16 monomials of degree <= 4 per equation, d = 16,
    quad double, at a unit-coefficient series point: the full output."""
    m, N, d = 4, 32, 16
    sysm = I.eval_system((2, 0), N, N, m, 16, 4)
    x = I.unit_series((2, 1), m, d, N)
    fw, Aw = oracle.eval_diff(sysm, x)
    f, A = B.md_poly_eval_diff(B.DeviceSystem(sysm), dev(x))
    eval_close(host(f), fw, m)
    eval_close(host(A), Aw, m)


@pytest.mark.parametrize("m", (8, 10))
def test_eval_diff_64x64_sampled_equations(B, m):
    """64 x 64, 16 monomials of degree <= 4, d = 32: the oracle evaluates a
    sample of equations on its own and the GPU rows must agree."""
    N, d = 64, 32
    sysm = I.eval_system((3, 0), N, N, m, 16, 4)
    x = I.unit_series((3, 1), m, d, N)
    f, A = B.md_poly_eval_diff(B.DeviceSystem(sysm), dev(x))
    f, A = host(f), host(A)
    for i in (0, 29, 63):
        sub = I.build_system(1, N, m, sysm.dc, [[
            (fac, [(sysm.coef[0, :, j, k], sysm.coef[1, :, j, k]) for k in range(sysm.dc + 1)])
            for j, fac in sysm.terms(i)]])
        fw, Aw = oracle.eval_diff(sub, x)
        eval_close(np.ascontiguousarray(f[:, :, :, i:i + 1]), fw, m)
        eval_close(np.ascontiguousarray(A[:, :, :, i:i + 1, :]), Aw, m)


# ----------------------------------------------------------------------------
# QR and the staggered solve


def compare_qr(got, want, m, cond):
    QRg, vdg, bg = got
    QRw, vdw, bw = want
    N, n = QRw.shape[2:]
    scale = np.abs(QRw[0, 0] + 1j * QRw[1, 0]).max()
    iu = np.triu_indices(n)
    dR = cdiff(QRg[:, :, :n], QRw[:, :, :n])[iu]
    assert dR.max() <= tol(m, math.log2(cond) + 4) * scale
    assert cdiff(vdg, vdw).max() <= tol(m, math.log2(cond) + 4) * scale
    assert (rdiff(bg, bw) / np.abs(bw[0])).max() <= tol(m, math.log2(cond) + 4)


@pytest.mark.parametrize("m", (2, 4, 8))
@pytest.mark.parametrize("shape", ((32, 32), (1, 1), (3, 2), (70, 24)))
def test_qr_within_tolerance(B, m, shape):
    N, n = shape
    A0 = I.unit_complex(I.rng(956, m, N, n), m, N, n)
    QRw, vdw, bw, stw = oracle.qr(A0)
    QR, vd, beta, st = B.md_qr(dev(A0))
    assert int(host(st)[0]) == stw == 0
    s = np.linalg.svd(A0[0, 0] + 1j * A0[1, 0], compute_uv=False)
    compare_qr((host(QR), host(vd), host(beta)), (QRw, vdw, bw), m, s[0] / s[-1])


@pytest.mark.parametrize("m", (2, 4))
def test_qr_tall_four_rows_per_lane(B, m):
    """N above 128 takes four rows per lane in md_qr, the form that reads
    the reflector and column rows where they are used instead of holding
    them (the batched kernel's QR form)."""
    N, n = 140, 60
    A0 = I.unit_complex(I.rng(958, m, N, n), m, N, n)
    QRw, vdw, bw, stw = oracle.qr(A0)
    QR, vd, beta, st = B.md_qr(dev(A0))
    assert int(host(st)[0]) == stw == 0
    s = np.linalg.svd(A0[0, 0] + 1j * A0[1, 0], compute_uv=False)
    compare_qr((host(QR), host(vd), host(beta)), (QRw, vdw, bw), m, s[0] / s[-1])


@pytest.mark.parametrize("m,N,n", ((8, 64, 64), (10, 64, 64), (4, 32, 32), (2, 70, 24),
                                   (4, 140, 60), (5, 9, 9), (1, 1, 1), (3, 3, 2), (3, 5, 3),
                                   (4, 17, 12), (5, 33, 20), (8, 40, 33), (4, 64, 64)))
def test_qr_gang_same_bits_as_one_workgroup(B, m, N, n):
    """md_qr_gang spreads each step's column updates over several
    workgroups with device barriers (from three limbs on and 5 <= N <= 64
    with the look-ahead column on four waves of one workgroup, its complex
    products one real product a lane); the factors are md_qr's bit for bit
    (the oracle comparison of md_qr covers their accuracy), also on a
    second call that reuses the synchronisation word."""
    A0 = dev(I.unit_complex(I.rng(959, m, N, n), m, N, n))
    QR, vd, beta, st = B.md_qr(A0)
    sync = torch.zeros(1, dtype=torch.int32, device="cuda")
    for _ in range(2):
        QRg, vdg, bg, stg = B.md_qr_gang(A0, sync=sync)
        assert int(host(stg)[0]) == int(host(st)[0]) == 0
        assert np.array_equal(host(QRg), host(QR))
        assert np.array_equal(host(vdg), host(vd))
        assert np.array_equal(host(bg), host(beta))
    if m >= 3 and 5 <= N <= 64 and n >= 3:
        assert B.md_qr_gang_size(m, N, n) > 1    # the four-wave look-ahead form


def test_qr_flags_singular_column(B):
    m = 2
    A0 = I.unit_complex(I.rng(957), m, 5, 5)
    A0[:, :, :, 2] = 0.0
    _, _, beta, st = B.md_qr(dev(A0))
    assert int(host(st)[0]) & B.MD_ST_SINGULAR
    assert np.all(host(beta)[:, 2] == 0.0)


@pytest.mark.parametrize("m", (4, 8))
def test_qr_gang_flags_singular_column_like_one_workgroup(B, m):
    """A zero column in the four-wave look-ahead form of md_qr_gang: the
    same status bit, zero beta and the same factors bit for bit as md_qr;
    a NaN entry sets MD_ST_NONFINITE in both."""
    N = n = 9
    A0 = I.unit_complex(I.rng(960, m), m, N, n)
    A0[:, :, :, 4] = 0.0
    assert B.md_qr_gang_size(m, N, n) > 1
    QR, vd, beta, st = B.md_qr(dev(A0))
    QRg, vdg, bg, stg = B.md_qr_gang(dev(A0), sync=torch.zeros(1, dtype=torch.int32, device="cuda"))
    assert int(host(st)[0]) == int(host(stg)[0])
    assert int(host(st)[0]) & B.MD_ST_SINGULAR
    assert np.all(host(bg)[:, 4] == 0.0)
    assert np.array_equal(host(QRg), host(QR))
    assert np.array_equal(host(vdg), host(vd))
    assert np.array_equal(host(bg), host(beta))
    A0 = I.unit_complex(I.rng(961, m), m, N, n)
    A0[0, 0, 6, 2] = np.nan
    _, _, _, st = B.md_qr(dev(A0))
    _, _, _, stg = B.md_qr_gang(dev(A0), sync=torch.zeros(1, dtype=torch.int32, device="cuda"))
    assert int(host(st)[0]) & B.MD_ST_NONFINITE
    assert int(host(stg)[0]) & B.MD_ST_NONFINITE


def solve_case(B, m, N, n, d, key):
    if N == n:
        A, b = I.toeplitz_system(key, n, d, m)
    else:
        g = I.rng(*key)
        A = I.unit_complex(g, m, d + 1, N, n)
        b = I.unit_complex(g, m, d + 1, N)
    dxw, stw = oracle.solve_toeplitz(A, b)
    QR, vd, beta, st = B.md_qr(dev(A[:, :, 0]))
    dx, st2 = B.md_series_solve(QR, vd, beta, dev(A), dev(b))
    assert int(host(st)[0]) == 0 and int(host(st2)[0]) == 0 and stw == 0
    A0 = A[0, 0, 0] + 1j * A[1, 0, 0]
    s = np.linalg.svd(A0, compute_uv=False)
    e = rel_err_per_k(host(dx), dxw)
    for k in range(d + 1):
        assert e[k] <= tol(m, math.log2(s[0] / s[-1]) + math.log2(k + 1) + 2), (k, e)


@pytest.mark.parametrize("m", (2, 4))
def test_solve_32_quad_double_config(B, m):
    """n = 32, d = 16, A_0 = U diag U^H with condition number 1e3."""
    solve_case(B, m, 32, 32, 16, (2, 32))


@pytest.mark.parametrize("m,N,n,d", ((2, 1, 1, 0), (3, 5, 5, 3), (5, 9, 9, 2), (2, 70, 70, 3),
                                     (4, 12, 7, 4)))
def test_solve_edge_shapes(B, m, N, n, d):
    solve_case(B, m, N, n, d, (960, N, n, d))


@pytest.mark.parametrize("m", (8, 10))
def test_solve_64_octo_deca_double(B, m):
    """n = 64, d = 32 at octo and deca double (the oracle takes ~10 s)."""
    solve_case(B, m, 64, 64, 32, (2, 64))


# ----------------------------------------------------------------------------
# Newton steps


def newton_compare(B, sysm, x, iters, m):
    sd = B.DeviceSystem(sysm)
    xg = dev(x)
    cond = sysm.meta.get("cond_A0_double", 10.0)
    for it in range(iters):
        xw, nrmw, stw = oracle.newton_step(sysm, x)
        _, nrm, st = B.md_newton_step(sd, xg)
        xh = host(xg)
        e = rel_err_per_k(xh, xw)
        for k in range(xw.shape[2]):
            assert e[k] <= tol(m, math.log2(cond) + math.log2(k + 1) + 4), (it, k, e)
        assert int(host(st)[0]) == stw == 0
        nh = host(nrm)
        # |dx_d| is the difference of x_d between two steps, so the two sides
        # may differ by what their x_d may differ by (the bound above at
        # k = d), relative to the larger of |x_d|, the update and 1
        d = xw.shape[2] - 1
        scale = max(1.0, np.abs(xw[0, 0, -1] + 1j * xw[1, 0, -1]).max(), nrmw[0, 0])
        dn = abs(nh[0, 0] - nrmw[0, 0])
        assert dn <= tol(m, math.log2(cond) + math.log2(d + 1) + 4) * scale, (it, dn, scale)
        x = xw  # continue both from the oracle's iterate
        xg = dev(x)
    return x, nh


def test_newton_plain_double_double_config(B):
    """n = 8, 8 monomials of degree <= 3 per equation, d = 8, 8 iterations."""
    m, d = 2, 8
    sysm, x0 = I.newton_system((0, 0), 8, m)
    x, nrm = newton_compare(B, sysm, I.series_start(x0, d), 8, m)
    # converged: the last update is at the precision's level relative to x_d
    xd = np.abs(x[0, 0, d] + 1j * x[1, 0, d]).max()
    assert nrm[0, 0] <= 2.0 ** -(53 * m - 16) * max(1.0, xd)


@pytest.mark.parametrize("m", (2, 4))
def test_circle_example(B, m):
    sysm, x = I.circle_system(m, 8)
    newton_compare(B, sysm, x, 6, m)


def test_sqrt_series_exact(B):
    m, d = 4, 16
    sysm, x = I.sqrt_system(m, d)
    xg = dev(x)
    B.newton(B.DeviceSystem(sysm), xg, 6)
    xw, _, _ = oracle.newton(sysm, x, 6)
    assert np.array_equal(host(xg), xw)  # dyadic coefficients: both exact


def test_newton_deterministic(B):
    m, d = 4, 12
    sysm, x0 = I.newton_system((5, 0), 12, m)
    sd = B.DeviceSystem(sysm)
    outs = []
    for _ in range(2):
        xg = dev(I.series_start(x0, d))
        B.newton(sd, xg, 3)
        outs.append(host(xg))
    assert np.array_equal(outs[0], outs[1])


def test_newton_diverged_flag(B):
    """MD_ST_DIVERGED: dx_norm carries the previous step's |dx_d| in; the bit
    is set when the new |dx_d| is larger, and not when the input is zero
    (no previous step) or larger than the new one."""
    m, d = 2, 6
    sysm, x0 = I.newton_system((6, 1), 5, m)
    sd = B.DeviceSystem(sysm)
    # the first step from a constant series leaves coefficients 2..d alone
    # (A(t) = A_0), so the flag is exercised from the second step's input
    xg = dev(I.series_start(x0, d))
    B.md_newton_step(sd, xg)
    x = host(xg).copy()
    _, nrm, st = B.md_newton_step(sd, dev(x))
    first = host(nrm).copy()
    assert int(host(st)[0]) == 0 and first[0, 0] > 0
    for prev, want in ((0.0, 0), (first[0, 0] * 0.5, B.MD_ST_DIVERGED),
                       (first[0, 0] * 2.0, 0)):
        nin = torch.zeros((m, 2), dtype=torch.float64, device="cuda")
        nin[0, 0] = prev
        _, nout, st = B.md_newton_step(sd, dev(x), dx_norm=nin)
        assert (int(host(st)[0]) & B.MD_ST_DIVERGED) == want, (prev, first[0, 0])
        assert np.array_equal(host(nout), first)   # the output norms do not depend on the input
    # equal values are not growth
    nin = torch.as_tensor(first, device="cuda").clone()
    _, _, st = B.md_newton_step(sd, dev(x), dx_norm=nin)
    assert int(host(st)[0]) == 0


def test_newton_nonfinite_flag(B):
    m, d = 2, 4
    sysm, x0 = I.newton_system((6, 0), 4, m)
    x = I.series_start(x0, d)
    x[0, 0, 0, 1] = np.nan
    _, _, st = B.md_newton_step(B.DeviceSystem(sysm), dev(x))
    assert int(host(st)[0]) & B.MD_ST_NONFINITE


# ----------------------------------------------------------------------------
# batched persistent launch


def small_batch(count=14, seed=0):
    specs = I.batch_specs((990, seed), count, n_choices=(3, 5, 8, 12, 17), d_range=(0, 9),
                          m_choices=(1, 2, 3, 4))
    paths = []
    for s in specs:
        sysm, x0 = I.newton_system((991, s.path), s.n, s.m, terms=4, max_deg=3)
        paths.append((sysm, I.series_start(x0, s.d)))
    return paths


def test_batch_agrees_with_per_path(B):
    """One persistent launch over paths of uneven n, d and precision agrees
    with md_newton_step applied to each path.  The batched kernel sums its
    dot products in its own fixed order (more products per lane), so the
    two agree within the solve tolerance rather than bit for bit."""
    paths = small_batch()
    batch = B.BatchedPaths(paths)
    B.md_newton_batch(batch, 3)
    torch.cuda.synchronize()
    assert not host(batch.status).any()
    for p, (sysm, x) in enumerate(paths):
        xg = dev(x)
        sd = B.DeviceSystem(sysm)
        for _ in range(3):
            _, nrm, st = B.md_newton_step(sd, xg)
        xb, xs = host(batch.x(p)), host(xg)
        e = rel_err_per_k(xb, xs)
        cond = sysm.meta["cond_A0_double"]
        for k in range(xs.shape[2]):
            assert e[k] <= tol(sysm.m, math.log2(cond) + math.log2(k + 1) + 4), (p, k, e)


def test_batch_against_oracle_and_reruns(B):
    paths = small_batch(count=6, seed=1)
    batch = B.BatchedPaths(paths)
    B.md_newton_batch(batch, 2, grid=3)
    first = [host(batch.x(p)).copy() for p in range(len(paths))]
    batch.reset(paths)
    B.md_newton_batch(batch, 2, grid=7, eval_waves=1)
    second = [host(batch.x(p)).copy() for p in range(len(paths))]
    batch.restore()
    batch.set_order(np.arange(len(paths))[::-1])
    clk = torch.zeros((len(paths), 2), dtype=torch.int64, device="cuda")
    B.md_newton_batch(batch, 2, grid=5, block=512, eval_waves=8, path_clock=clk)
    c = host(clk)
    assert np.all(c[:, 0] > 0) and np.all(c[:, 1] >= c[:, 0])
    for p, (sysm, x) in enumerate(paths):
        # neither the launch shape nor the job order changes the bits
        assert np.array_equal(second[p], first[p]) and np.array_equal(host(batch.x(p)), first[p])
        xw = x
        for _ in range(2):
            xw, _, _ = oracle.newton_step(sysm, xw)
        m = sysm.m
        e = rel_err_per_k(first[p], xw)
        cond = sysm.meta["cond_A0_double"]
        for k in range(xw.shape[2]):
            assert e[k] <= tol(m, math.log2(cond) + math.log2(k + 1) + 4), (p, k, e)


def test_batch_gangs_and_die_queues(B):
    """One queue per accelerator die, and the longest paths split over gangs
    of 2 and 4 workgroups (of one die, or of any die with one queue), give
    the bits of the one-queue launch."""
    paths = small_batch(count=14, seed=3)
    batch = B.BatchedPaths(paths)
    B.md_newton_batch(batch, 2, block=512)
    torch.cuda.synchronize()
    ref = [host(batch.x(p)).copy() for p in range(len(paths))]
    assert not host(batch.status).any()
    dies = B.md_device_dies()
    gangs = np.ones(len(paths), dtype=np.int64)
    order = np.argsort(-batch.cost)
    gangs[order[:2]] = 4
    gangs[order[2:5]] = 2
    for nq, g in ((dies, None), (dies, gangs), (1, gangs)):
        batch.set_schedule(nq=nq, gangs=g)
        batch.restore()
        cus = torch.cuda.get_device_properties(0).multi_processor_count
        print(f"batch gangs nq={nq} gangs={None if g is None else g.tolist()}", flush=True)
        B.md_newton_batch(batch, 2, block=512, grid=cus)
        torch.cuda.synchronize()
        assert not host(batch.status).any(), host(batch.status)
        for p in range(len(paths)):
            assert np.array_equal(host(batch.x(p)), ref[p]), (nq, p)


def test_batch_graph_replays(B):
    """The batched launch captured in a graph: three replays, with eager work
    (restoring the start series) and a synchronisation between them, each
    give the bits of the eager launch."""
    paths = small_batch(count=10, seed=4)
    batch = B.BatchedPaths(paths)
    B.md_newton_batch(batch, 2, block=512)
    torch.cuda.synchronize()
    eager = [host(batch.x(p)).copy() for p in range(len(paths))]
    g = torch.cuda.CUDAGraph()
    batch.restore()
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        B.md_newton_batch(batch, 2, block=512)
    torch.cuda.synchronize()
    for rep in range(3):
        batch.restore()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert not host(batch.status).any(), rep
        for p in range(len(paths)):
            assert np.array_equal(host(batch.x(p)), eager[p]), (rep, p)


def test_batch_flags_refused_paths(B):
    """A path table that breaks the kernel's limits anyway (the host refuses
    such paths, so the table is altered on the device after construction):
    a path that claims 70 equations and one that claims penta double get
    MD_ST_BADPATH and are not run; the others run as in a batch without
    them, and the launch ends (every workgroup leaves the job loop)."""
    paths = small_batch(count=5, seed=2)
    ref = B.BatchedPaths(paths)
    B.md_newton_batch(ref, 2, block=512)
    batch = B.BatchedPaths(paths)
    t = batch.table.copy()
    t[3]["N"] = 70
    t[1]["m"] = 5
    batch.paths_dev.copy_(torch.as_tensor(t.view(np.uint8).copy(), device="cuda"))
    print("refused-path launch: paths 1 (m=5) and 3 (N=70) of 5", flush=True)
    B.md_newton_batch(batch, 2, block=512)
    st = host(batch.status)
    assert st[1] == B.MD_ST_BADPATH | B.MD_ST_NOTRUN and st[3] == B.MD_ST_BADPATH | B.MD_ST_NOTRUN, st
    assert not st[[0, 2, 4]].any(), st
    assert not host(ref.status).any()
    for p in (0, 2, 4):
        assert np.array_equal(host(batch.x(p)), host(ref.x(p))), p
    for p in (1, 3):
        assert np.array_equal(host(batch.x(p)), paths[p][1]), p     # untouched


def hp_batch(count=6, seed=0, m=8):
    specs = I.batch_specs((996, seed), count, n_choices=(3, 5, 8, 12), d_range=(0, 9),
                          m_choices=(m,))
    paths = []
    for s in specs:
        sysm, x0 = I.newton_system((997, s.path), s.n, s.m, terms=4, max_deg=3)
        paths.append((sysm, I.series_start(x0, s.d)))
    return paths


@pytest.mark.parametrize("m", (5, 8, 10))
def test_batch_high_precision_against_oracle_and_per_path(B, m):
    """Penta, octo or deca double paths in one launch of their 256-thread
    kernel: against the oracle and md_newton_step after 2 steps (agreement
    rule), and the same bits under another launch shape, job order and a
    gang split."""
    paths = hp_batch(m=m)
    batch = B.BatchedPaths(paths)
    print("high-precision batch:", [(s.m, s.n, x.shape[2] - 1) for s, x in paths], flush=True)
    B.md_newton_batch(batch, 2)
    st = host(batch.status)
    assert not st.any(), st
    first = [host(batch.x(p)).copy() for p in range(len(paths))]
    batch.restore()
    gangs = np.ones(len(paths), dtype=np.int64)
    gangs[int(np.argmax(batch.cost))] = 3
    batch.set_schedule(gangs=gangs)
    B.md_newton_batch(batch, 2, grid=7, eval_waves=2)
    assert not host(batch.status).any()
    for p, (sysm, x) in enumerate(paths):
        assert np.array_equal(host(batch.x(p)), first[p]), p
        m = sysm.m
        xw, _, _ = oracle.newton(sysm, x, 2)
        xg = dev(x)
        sd = B.DeviceSystem(sysm)
        for _ in range(2):
            B.md_newton_step(sd, xg)
        cond = sysm.meta["cond_A0_double"]
        for ref in (xw, host(xg)):
            e = rel_err_per_k(first[p], ref)
            for k in range(x.shape[2]):
                assert e[k] <= tol(m, math.log2(cond) + math.log2(k + 1) + 4), (p, k, e)


def test_batch_high_precision_refuses_mixed_and_512(B):
    paths = hp_batch(count=2, seed=1)
    lo = small_batch(count=2, seed=4)
    with pytest.raises(B.MdError, match="separate launches"):
        B.BatchedPaths(paths + lo)
    batch = B.BatchedPaths(paths)
    with pytest.raises(B.MdError, match="block=256"):
        B.md_newton_batch(batch, 1, block=512, eval_waves=4)
