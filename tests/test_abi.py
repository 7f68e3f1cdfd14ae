"""The C-ABI library loads and exports every entry point declared in
include/mdseries.h; host-side argument checks return their error codes
without touching a GPU."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mdseries.h")
LIB = os.path.join(ROOT, "paper_2012_06607_amd", "libmdseries.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|size_t|const char \*)\s*(md_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} not built: run paper_2012_06607_amd.build.build()")
    return ctypes.CDLL(LIB)


def test_header_declares_the_five_entry_points():
    names = declared_functions()
    for name in ("md_series_convolve", "md_poly_eval_diff", "md_qr", "md_series_solve",
                 "md_newton_step"):
        assert name in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_workspace_sizes(lib):
    f = lib.md_workspace_bytes
    f.restype = ctypes.c_size_t
    f.argtypes = [ctypes.c_int] * 7
    assert f(1, 4, 32, 32, 16, 512, 4) > 0
    assert f(2, 4, 32, 32, 16, 0, 0) > 0
    assert f(3, 2, 8, 8, 8, 80, 3) >= f(1, 2, 8, 8, 8, 80, 3) + f(2, 2, 8, 8, 8, 0, 0)
    assert f(1, 6, 8, 8, 8, 80, 3) == 0      # m = 6 is not supported
    assert f(9, 2, 8, 8, 8, 80, 3) == 0      # unknown entry point
    assert f(2, 2, 8, 8, -1, 0, 0) == 0      # negative degree
    # workspace grows linearly in the number of terms and quadratically in N
    assert f(1, 2, 8, 8, 8, 160, 3) > f(1, 2, 8, 8, 8, 80, 3)
    assert f(2, 2, 64, 64, 8, 0, 0) > f(2, 2, 32, 32, 8, 0, 0)
    # adjoint: the Newton workspace plus lambda; storing the monomial series
    # adds at least M (d+1) complex md numbers
    assert f(4, 4, 32, 32, 16, 320, 3) > f(3, 4, 32, 32, 16, 320, 3)
    assert f(5, 4, 32, 32, 16, 320, 3) >= f(4, 4, 32, 32, 16, 320, 3) + 2 * 4 * 8 * 320 * 17


def test_argument_errors_return_codes(lib):
    P = ctypes.c_void_p
    lib.md_last_error.restype = ctypes.c_char_p
    lib.md_series_convolve.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, P, P, P, P]
    lib.md_qr.argtypes = [ctypes.c_int] * 3 + [P] * 6
    lib.md_elementwise.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, P, P, P, P]
    lib.md_norm2.argtypes = [ctypes.c_int, ctypes.c_int64, P, P, P]
    lib.md_newton_step.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, P, ctypes.c_size_t, P, P]
    fake = P(4096)
    assert lib.md_series_convolve(2, -1, 4, fake, fake, fake, None) == 1          # MD_EINVAL
    assert lib.md_series_convolve(2, 8, 4, None, fake, fake, None) == 3           # MD_ENULL
    assert lib.md_series_convolve(6, 8, 4, fake, fake, fake, None) == 1           # bad m
    assert b"m=6" in lib.md_last_error()
    assert lib.md_series_convolve(2, 8, 0, fake, fake, fake, None) == 0           # nothing to do
    assert lib.md_series_convolve(2, 8, 0, None, None, None, None) == 0           # empty: no pointers needed
    assert lib.md_qr(2, 3, 4, fake, fake, fake, fake, None, None) == 2            # MD_ESHAPE (N < n)
    lib.md_qr_gang.argtypes = [ctypes.c_int] * 3 + [P] * 7
    assert lib.md_qr_gang(4, 8, 8, fake, fake, fake, fake, None, None, None) == 3  # no sync word
    assert lib.md_qr_gang(4, 3, 4, fake, fake, fake, fake, fake, None, None) == 2  # N < n
    lib.md_qr_gang_size.argtypes = [ctypes.c_int] * 3
    # from three limbs on, N <= 64: workgroup 0 takes the look-ahead column
    # on four waves, the others the n - 2 columns after it
    assert lib.md_qr_gang_size(8, 64, 64) == 17      # 1 + 62 columns / 4 one-wave segments
    assert lib.md_qr_gang_size(4, 32, 32) == 3       # 1 + 30 columns / 16 segments
    assert lib.md_qr_gang_size(3, 5, 3) == 2         # the smallest such column (8-lane segments)
    assert lib.md_qr_gang_size(4, 4, 4) == 1         # N < 5: one workgroup
    assert lib.md_qr_gang_size(2, 32, 32) == 1       # double double: 31 columns, 32 segments
    assert lib.md_qr_gang_size(4, 140, 60) == 8      # N > 64: 59 columns, 8 four-row segments
    assert lib.md_qr_gang_size(2, 1, 1) == 1
    assert lib.md_qr_gang_size(6, 8, 8) == 0
    assert lib.md_elementwise(2, 99, 4, fake, fake, fake, None) == 1              # unknown op
    assert lib.md_norm2(2, 0, fake, fake, None) == 1                              # empty vector
    assert lib.md_newton_step(2, 8, None, fake, None, fake, 1 << 20, None, None) == 3
    lib.md_newton_adjoint.argtypes = [ctypes.c_int, ctypes.c_int, P, P, P, ctypes.c_int, P, P,
                                      ctypes.c_size_t, P, P]
    assert lib.md_newton_adjoint(2, 8, None, fake, fake, 1, fake, fake, 1 << 20, None, None) == 3


class _System(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("n", ctypes.c_int32), ("M", ctypes.c_int32),
                ("dc", ctypes.c_int32), ("max_deg", ctypes.c_int32),
                ("eq_ptr", ctypes.c_void_p), ("term_ptr", ctypes.c_void_p),
                ("factors", ctypes.c_void_p), ("coef", ctypes.c_void_p)]


def test_adjoint_host_checks(lib):
    P = ctypes.c_void_p
    lib.md_newton_adjoint.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(_System), P, P,
                                      ctypes.c_int, P, P, ctypes.c_size_t, P, P]
    lib.md_workspace_bytes.restype = ctypes.c_size_t
    lib.md_workspace_bytes.argtypes = [ctypes.c_int] * 7
    fake = P(4096)
    sysd = _System(8, 8, 80, 1, 3, 4096, 4096, 4096, 4096)
    need = lib.md_workspace_bytes(5, 2, 8, 8, 8, 80, 3)
    call = lambda m, d, s, ws, nb, store=1: lib.md_newton_adjoint(  # noqa: E731
        m, d, ctypes.byref(s), fake, fake, store, fake, ws, nb, None, None)
    assert call(2, -1, sysd, fake, need) == 1                       # negative degree
    assert call(6, 8, sysd, fake, need) == 1                        # m = 6
    assert call(2, 8, _System(4, 8, 80, 1, 3, 4096, 4096, 4096, 4096), fake, need) == 2  # N < n
    assert call(2, 8, _System(300, 8, 80, 1, 3, 4096, 4096, 4096, 4096), fake, need) == 2
    assert call(2, 8, sysd, P(4096), need - 1) == 4                 # workspace too small
    assert call(2, 8, sysd, P(4096 + 8), need) == 4                 # misaligned workspace
    assert lib.md_newton_adjoint(2, 8, ctypes.byref(sysd), None, fake, 1, fake, fake, need,
                                 None, None) == 3                   # x missing


def test_batch_host_checks(lib):
    P = ctypes.c_void_p
    i = ctypes.c_int
    lib.md_newton_batch.argtypes = [i, P, i, P, i, P, P, P, P, i, P, P, P, i, i, i, i, i, i, i,
                                    P, P, P]
    lib.md_batch_lds_bytes.argtypes = [i] * 4
    lib.md_batch_lds_bytes.restype = ctypes.c_size_t
    fake = P(4096)

    def call(npaths=4, njobs=4, nq=1, iters=1, max_m=4, max_N=64, max_d=8, max_deg=3, grid=16,
             block=256, ew=4, paths=fake):
        return lib.md_newton_batch(npaths, paths, njobs, fake, nq, fake, fake, fake, fake, iters,
                                   fake, fake, fake, max_m, max_N, max_d, max_deg, grid, block, ew,
                                   None, None, None)
    # limb counts outside both batched kernels are rejected on the host, and
    # the penta to deca double kernel runs 256-thread workgroups only
    assert call(max_m=6) == 1
    assert call(max_m=9) == 1
    assert call(max_m=0) == 1
    assert call(max_m=8, block=512, ew=4) == 1
    # neither are paths of more than 64 equations
    assert call(max_N=65) == 2
    assert b"max_N=65" in lib.md_last_error()
    assert call(max_N=70, npaths=0) == 2      # refused before the empty-batch early return
    assert call(max_N=0) == 2
    assert call(grid=0) == 1
    assert call(ew=5) == 1                      # more evaluation waves than the block has
    assert call(block=512, ew=9) == 1
    assert call(block=384) == 1
    assert call(nq=0) == 1
    assert call(njobs=-1) == 1
    assert call(paths=None) == 3
    assert call(npaths=0) == 0                  # empty batch
    # evaluation LDS above the device limit is refused (deca-size series on 4 waves)
    assert lib.md_batch_lds_bytes(4, 200, 4, 4) > 64 * 1024
    assert call(max_d=200, max_deg=4) == 2
    assert lib.md_batch_lds_bytes(6, 8, 3, 4) == 0
    assert lib.md_batch_lds_bytes(10, 8, 3, 4) == 10 * lib.md_batch_lds_bytes(1, 8, 3, 4)
    # never less than one dx_k of 64 unknowns (kept in LDS during the stages)
    assert lib.md_batch_lds_bytes(4, 0, 0, 1) == 8 * 2 * 4 * 64
    assert lib.md_batch_lds_bytes(2, 1, 1, 1) == 8 * 2 * 2 * 64
    lib.md_device_dies.argtypes = [P, i, P]
    assert lib.md_device_dies(None, 4, None) == 3
    assert lib.md_device_dies(fake, 0, None) == 1


def test_noalloc_host_checks(lib):
    """md_newton_step_noalloc refuses, before any device call, a step whose
    scratch would not fit the fixed per-GPU array, and bad arguments."""
    P = ctypes.c_void_p
    lib.md_newton_step_noalloc.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(_System),
                                           P, P, P, P]
    lib.md_workspace_bytes.restype = ctypes.c_size_t
    lib.md_workspace_bytes.argtypes = [ctypes.c_int] * 7
    lib.md_last_error.restype = ctypes.c_char_p
    fake = P(4096)
    limit = 32 << 20
    big = _System(64, 64, 1024, 1, 4, 4096, 4096, 4096, 4096)
    assert lib.md_workspace_bytes(3, 10, 64, 64, 32, 1024, 4) > limit
    assert lib.md_newton_step_noalloc(10, 32, ctypes.byref(big), fake, None, None, None) == 4
    assert b"above the fixed 33554432" in lib.md_last_error()
    small = _System(8, 8, 80, 1, 3, 4096, 4096, 4096, 4096)
    assert lib.md_workspace_bytes(3, 2, 8, 8, 8, 80, 3) <= limit
    assert lib.md_newton_step_noalloc(2, -1, ctypes.byref(small), fake, None, None, None) == 1
    assert lib.md_newton_step_noalloc(6, 8, ctypes.byref(small), fake, None, None, None) == 1
    assert lib.md_newton_step_noalloc(2, 8, None, fake, None, None, None) == 3
    assert lib.md_newton_step_noalloc(2, 8, ctypes.byref(small), None, None, None, None) == 3
    bad = _System(4, 8, 80, 1, 3, 4096, 4096, 4096, 4096)
    assert lib.md_newton_step_noalloc(2, 8, ctypes.byref(bad), fake, None, None, None) == 2


def test_batch_protocol_host_checks(lib):
    import paper_2012_06607_amd.binding as Bd
    P = ctypes.c_void_p
    i = ctypes.c_int
    lib.md_newton_batch_protocol.argtypes = [i, P, i, P, i, P, P, P, P,
                                             ctypes.POINTER(Bd.md_protocol), P, P, P, i, i, i, i,
                                             i, i, i, P, P, P]
    lib.md_last_error.restype = ctypes.c_char_p
    fake = P(4096)

    def proto(degrees=(8, 16), maxit=(8, 8), min_steps=2, tol=1e-32, diverge=1.0):
        pr = Bd.md_protocol()
        pr.ndeg, pr.min_steps, pr.tol, pr.diverge = len(degrees), min_steps, tol, diverge
        for j, (d, mi) in enumerate(zip(degrees, maxit)):
            pr.degrees[j], pr.maxit[j] = d, mi
        return pr

    def call(pr, max_m=4, npaths=2, out=fake):
        return lib.md_newton_batch_protocol(npaths, fake, 2, fake, 1, fake, fake, fake, fake,
                                            ctypes.byref(pr) if pr is not None else None, fake,
                                            fake, fake, max_m, 16, 16, 3, 16, 256, 4, out, out,
                                            None)
    assert call(None) == 3
    assert call(proto(degrees=(16, 8))) == 1          # not increasing
    assert call(proto(min_steps=0)) == 1
    assert call(proto(tol=-1.0)) == 1
    assert call(proto(diverge=0.0)) == 1
    assert call(proto(), max_m=8) == 1                # double to quad double only
    assert b"quad double" in lib.md_last_error()
    assert call(proto(), out=None) == 3               # outputs needed
    assert call(proto(), npaths=0) == 0               # empty batch
