"""Python binding of libmdseries.so: argument marshalling only.

Every function here has the name of the C entry point it calls (see
include/mdseries.h), checks the torch tensors it is given (float64 limb
planes on the GPU, contiguous), passes their device pointers and torch's
current HIP stream, and raises MdError when the library returns an error.
All arithmetic runs in the library's HIP kernels; PyTorch supplies device
memory and streams.  If the library is missing or cannot be loaded this
module raises at import of the first call: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmdseries.so")

MD_FN_EVAL, MD_FN_SOLVE, MD_FN_NEWTON, MD_FN_ADJOINT, MD_FN_ADJOINT_STORE = 1, 2, 3, 4, 5
MD_FN_PROTOCOL = 6
MD_FN_PADE = 7
MD_PROTOCOL_MAX_DEGREES = 16
MD_ST_SINGULAR, MD_ST_NONFINITE, MD_ST_BADPATH, MD_ST_GANG, MD_ST_NOTRUN = 1, 2, 4, 8, 16
MD_ST_DIVERGED = 32
OPS = {"add": 0, "sub": 1, "mul": 2, "div": 3, "sqrt": 4, "rsqrt": 5, "muld": 6,
       "cadd": 7, "csub": 8, "cmul": 9, "cdiv": 10, "cabs2": 11}
REAL_OPS = ("add", "sub", "mul", "div", "sqrt", "rsqrt", "muld")
LIMBS = (1, 2, 3, 4, 5, 8, 10)


class MdError(RuntimeError):
    pass


class md_system(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("n", ctypes.c_int32), ("M", ctypes.c_int32),
                ("dc", ctypes.c_int32), ("max_deg", ctypes.c_int32),
                ("eq_ptr", ctypes.c_void_p), ("term_ptr", ctypes.c_void_p),
                ("factors", ctypes.c_void_p), ("coef", ctypes.c_void_p)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise MdError(f"{LIB_PATH} is missing: build it with paper_2012_06607_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, i32, i64, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t
        L.md_series_convolve.argtypes = [i32, i32, i64, P, P, P, P]
        L.md_poly_eval_diff.argtypes = [i32, i32, ctypes.POINTER(md_system), P, P, P, P, sz, P]
        L.md_qr.argtypes = [i32, i32, i32, P, P, P, P, P, P]
        L.md_qr_gang.argtypes = [i32, i32, i32, P, P, P, P, P, P, P]
        L.md_qr_gang_size.argtypes = [i32, i32, i32]
        L.md_series_solve.argtypes = [i32, i32, i32, i32, P, P, P, P, P, P, P, sz, P, P]
        L.md_newton_step.argtypes = [i32, i32, ctypes.POINTER(md_system), P, P, P, sz, P, P]
        L.md_newton_step_noalloc.argtypes = [i32, i32, ctypes.POINTER(md_system), P, P, P, P]
        L.md_series_divide.argtypes = [i32, i32, i64, P, P, P, P, P]
        L.md_series_pade.argtypes = [i32, i32, i32, i64, P, P, P, P, sz, P, P]
        L.md_newton_protocol.argtypes = [i32, ctypes.POINTER(md_system), P, i32, P, P, i32,
                                         ctypes.c_double, ctypes.c_double, P, P, P, P, sz, P, P]
        L.md_newton_adjoint.argtypes = [i32, i32, ctypes.POINTER(md_system), P, P, i32, P, P, sz,
                                        P, P]
        L.md_workspace_bytes.argtypes = [i32, i32, i32, i32, i32, i32, i32]
        L.md_workspace_bytes.restype = sz
        L.md_elementwise.argtypes = [i32, i32, i64, P, P, P, P]
        L.md_norm2.argtypes = [i32, i64, P, P, P]
        L.md_last_error.restype = ctypes.c_char_p
        for name in ("md_series_convolve", "md_poly_eval_diff", "md_qr", "md_series_solve",
                     "md_newton_step", "md_elementwise", "md_norm2"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(rc: int, name: str):
    if rc != 0:
        msg = lib().md_last_error().decode(errors="replace")
        raise MdError(f"{name} returned {rc}: {msg}")


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _ptr(t: torch.Tensor | None, dtype=torch.float64):
    if t is None:
        return None
    if not t.is_cuda:
        raise MdError("expected a GPU tensor")
    if t.dtype != dtype:
        raise MdError(f"expected {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise MdError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _limbs(t: torch.Tensor, complex_planes: bool = True) -> int:
    if complex_planes:
        if t.dim() < 2 or t.shape[0] != 2:
            raise MdError(f"expected planes (2, m, ...), got {tuple(t.shape)}")
        return int(t.shape[1])
    return int(t.shape[0])


def workspace(fn: int, m: int, N: int, n: int, d: int, M: int = 0, max_deg: int = 0,
              device=None) -> torch.Tensor:
    """A device workspace for an entry point (uint8 tensor)."""
    nbytes = lib().md_workspace_bytes(fn, m, N, n, d, M, max_deg)
    if nbytes == 0:
        raise MdError("md_workspace_bytes: invalid sizes")
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=device or "cuda")
    off = (-ws.data_ptr()) % 256
    return ws[off:off + nbytes]


def validate_system(sysm):
    """Host-side checks of the compressed structure, so that no kernel can
    index outside the arrays it is given."""
    ep = np.asarray(sysm.eq_ptr)
    tp = np.asarray(sysm.term_ptr)
    fa = np.asarray(sysm.factors)
    if sysm.N < 1 or sysm.n < 1 or sysm.dc < 0:
        raise MdError(f"bad system sizes N={sysm.N} n={sysm.n} dc={sysm.dc}")
    if ep.shape != (sysm.N + 1,) or ep[0] != 0 or np.any(np.diff(ep) < 0):
        raise MdError("eq_ptr must have N+1 non-decreasing entries from 0")
    Mt = tp.shape[0] - 1
    if Mt < 0 or ep[-1] != Mt or tp[0] != 0 or np.any(np.diff(tp) < 0) or tp[-1] != fa.shape[0]:
        raise MdError("term_ptr must have M+1 non-decreasing entries from 0 to len(factors)")
    if fa.size and (fa.min() < 0 or fa.max() >= sysm.n):
        raise MdError("factor indices must lie in [0, n)")
    for j in range(Mt):
        f = fa[tp[j]:tp[j + 1]]
        if np.any(np.diff(f) < 0):
            raise MdError(f"factors of term {j} are not sorted")
    if sysm.max_deg != (int(np.max(np.diff(tp))) if Mt else 0):
        raise MdError("max_deg must be the largest number of factors of a term")
    if sysm.coef.shape != (2, sysm.m, Mt, sysm.dc + 1):
        raise MdError(f"coef must have shape (2, m, M, dc+1), got {sysm.coef.shape}")


class DeviceSystem:
    """A polynomial system (paper_2012_06607_amd.inputs.System) copied to the
    GPU, with its md_system descriptor."""

    def __init__(self, sysm, device="cuda"):
        validate_system(sysm)
        self.host = sysm
        self.m = sysm.m
        dev = torch.device(device)
        self.eq_ptr = torch.as_tensor(np.asarray(sysm.eq_ptr, dtype=np.int32), device=dev)
        self.term_ptr = torch.as_tensor(np.asarray(sysm.term_ptr, dtype=np.int32), device=dev)
        fac = np.asarray(sysm.factors, dtype=np.int32)
        self.factors = torch.as_tensor(fac if fac.size else np.zeros(1, np.int32), device=dev)
        self.coef = torch.as_tensor(np.ascontiguousarray(sysm.coef), device=dev)
        self.desc = md_system(sysm.N, sysm.n, sysm.M, sysm.dc, sysm.max_deg,
                              self.eq_ptr.data_ptr(), self.term_ptr.data_ptr(),
                              self.factors.data_ptr(), self.coef.data_ptr())

    def with_coef(self, coef: torch.Tensor) -> "DeviceSystem":
        """The same structure with the coefficients read from `coef`
        (planes (2, m, M, dc+1) on the device; kept alive by the result)."""
        h = self.host
        if tuple(coef.shape) != (2, h.m, h.M, h.dc + 1):
            raise MdError(f"coef must have shape (2, m, M, dc+1), got {tuple(coef.shape)}")
        _ptr(coef)
        other = object.__new__(DeviceSystem)
        other.__dict__.update(self.__dict__)
        other.coef = coef
        other.desc = md_system(h.N, h.n, h.M, h.dc, h.max_deg, self.eq_ptr.data_ptr(),
                               self.term_ptr.data_ptr(), self.factors.data_ptr(), coef.data_ptr())
        return other

    @property
    def N(self):
        return self.host.N

    @property
    def n(self):
        return self.host.n


# -----------------------------------------------------------------------------
# entry points


def md_series_convolve(x: torch.Tensor, y: torch.Tensor, z: torch.Tensor | None = None,
                       stream=None) -> torch.Tensor:
    """z = x y mod t^{d+1}; planes (2, m, count, d+1)."""
    m = _limbs(x)
    _, _, count, L = x.shape
    if y.shape != x.shape:
        raise MdError("x and y shapes differ")
    z = torch.empty_like(x) if z is None else z
    _check(lib().md_series_convolve(m, L - 1, count, _ptr(x), _ptr(y), _ptr(z), _stream(stream)),
           "md_series_convolve")
    return z


def md_series_divide(x: torch.Tensor, y: torch.Tensor, status=None, stream=None):
    """z = x / y mod t^{d+1} per series (planes (2, m, count, d+1)); returns
    (z, status) with MD_ST_SINGULAR set when some y_0 is zero."""
    m = _limbs(x)
    if tuple(x.shape) != tuple(y.shape) or x.dim() != 4:
        raise MdError("md_series_divide: x and y must be equal planes (2, m, count, d+1)")
    _, _, count, L = x.shape
    z = torch.empty_like(x)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=x.device)
    _check(lib().md_series_divide(m, L - 1, count, _ptr(x), _ptr(y), _ptr(z),
                                  _ptr(status, torch.int32), _stream(stream)), "md_series_divide")
    return z, status


def md_series_pade(c: torch.Tensor, L: int, M: int, status=None, stream=None):
    """[L/M] Pade approximants p/q of the series c (planes (2, m, count,
    L+M+1)); returns (p (2, m, count, L+1), q (2, m, count, M+1), status)."""
    m = _limbs(c)
    if c.dim() != 4 or c.shape[3] != L + M + 1:
        raise MdError("md_series_pade: c must be planes (2, m, count, L+M+1)")
    count = c.shape[2]
    p = torch.empty((2, m, count, L + 1), dtype=torch.float64, device=c.device)
    q = torch.empty((2, m, count, M + 1), dtype=torch.float64, device=c.device)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=c.device)
    ws = None
    if M > 0 and count > 0:
        nbytes = lib().md_workspace_bytes(MD_FN_PADE, m, M, L, 0, count, 0)
        if nbytes == 0:
            raise MdError("md_series_pade: unsupported sizes")
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=c.device)
        off = (-raw.data_ptr()) % 256
        ws = raw[off:off + nbytes]
    _check(lib().md_series_pade(m, L, M, count, _ptr(c), _ptr(p), _ptr(q),
                                _ptr(ws, torch.uint8) if ws is not None else None,
                                ws.numel() if ws is not None else 0, _ptr(status, torch.int32),
                                _stream(stream)), "md_series_pade")
    return p, q, status


def md_poly_eval_diff(sysd: DeviceSystem, x: torch.Tensor, f=None, A=None, ws=None,
                      stream=None):
    """f (2, m, d+1, N) and A (2, m, d+1, N, n) at x (2, m, d+1, n)."""
    m = _limbs(x)
    _, _, L, n = x.shape
    N = sysd.N
    f = torch.empty((2, m, L, N), dtype=torch.float64, device=x.device) if f is None else f
    A = torch.empty((2, m, L, N, n), dtype=torch.float64, device=x.device) if A is None else A
    if ws is None:
        ws = workspace(MD_FN_EVAL, m, N, n, L - 1, sysd.host.M, sysd.host.max_deg, x.device)
    _check(lib().md_poly_eval_diff(m, L - 1, ctypes.byref(sysd.desc), _ptr(x), _ptr(f), _ptr(A),
                                   _ptr(ws, torch.uint8), ws.numel(), _stream(stream)),
           "md_poly_eval_diff")
    return f, A


def md_qr(A0: torch.Tensor, status: torch.Tensor | None = None, stream=None, QR=None,
          vdiag=None, beta=None):
    """Householder QR of A0 (2, m, N, n) -> (QR, vdiag, beta, status)."""
    m = _limbs(A0)
    _, _, N, n = A0.shape
    QR = torch.empty_like(A0) if QR is None else QR
    vd = torch.empty((2, m, n), dtype=torch.float64, device=A0.device) if vdiag is None else vdiag
    beta = torch.empty((m, n), dtype=torch.float64, device=A0.device) if beta is None else beta
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=A0.device)
    _check(lib().md_qr(m, N, n, _ptr(A0), _ptr(QR), _ptr(vd), _ptr(beta), _ptr(status, torch.int32),
                       _stream(stream)), "md_qr")
    return QR, vd, beta, status


def md_qr_gang(A0: torch.Tensor, status: torch.Tensor | None = None, stream=None, QR=None,
               vdiag=None, beta=None, sync: torch.Tensor | None = None):
    """md_qr with the column updates spread over md_qr_gang_size workgroups
    (same bits) -> (QR, vdiag, beta, status)."""
    m = _limbs(A0)
    _, _, N, n = A0.shape
    QR = torch.empty_like(A0) if QR is None else QR
    vd = torch.empty((2, m, n), dtype=torch.float64, device=A0.device) if vdiag is None else vdiag
    beta = torch.empty((m, n), dtype=torch.float64, device=A0.device) if beta is None else beta
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=A0.device)
    if sync is None:
        sync = torch.zeros(1, dtype=torch.int32, device=A0.device)
    _check(lib().md_qr_gang(m, N, n, _ptr(A0), _ptr(QR), _ptr(vd), _ptr(beta),
                            _ptr(sync, torch.int32), _ptr(status, torch.int32), _stream(stream)),
           "md_qr_gang")
    return QR, vd, beta, status


def md_qr_gang_size(m: int, N: int, n: int) -> int:
    return int(lib().md_qr_gang_size(m, N, n))


def md_series_solve(QR, vdiag, beta, A, b, dx=None, ws=None, status=None, stream=None):
    """Staggered solve of A(t) dx(t) = b(t); returns (dx, status)."""
    m = _limbs(A)
    _, _, L, N, n = A.shape
    dx = torch.empty((2, m, L, n), dtype=torch.float64, device=A.device) if dx is None else dx
    if ws is None:
        ws = workspace(MD_FN_SOLVE, m, N, n, L - 1, 0, 0, A.device)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=A.device)
    _check(lib().md_series_solve(m, N, n, L - 1, _ptr(QR), _ptr(vdiag), _ptr(beta), _ptr(A),
                                 _ptr(b), _ptr(dx), _ptr(ws, torch.uint8), ws.numel(),
                                 _ptr(status, torch.int32), _stream(stream)), "md_series_solve")
    return dx, status


def md_newton_step(sysd: DeviceSystem, x: torch.Tensor, dx_norm=None, ws=None, status=None,
                   stream=None):
    """One Newton step in place on x (2, m, d+1, n); returns (x, dx_norm (m, 2), status)."""
    m = _limbs(x)
    _, _, L, n = x.shape
    if dx_norm is None:
        # zero: no previous step to compare the update with (MD_ST_DIVERGED)
        dx_norm = torch.zeros((m, 2), dtype=torch.float64, device=x.device)
    if ws is None:
        ws = workspace(MD_FN_NEWTON, m, sysd.N, n, L - 1, sysd.host.M, sysd.host.max_deg, x.device)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=x.device)
    _check(lib().md_newton_step(m, L - 1, ctypes.byref(sysd.desc), _ptr(x), _ptr(dx_norm),
                                _ptr(ws, torch.uint8), ws.numel(), _ptr(status, torch.int32),
                                _stream(stream)), "md_newton_step")
    return x, dx_norm, status


def md_newton_protocol(sysd: DeviceSystem, x0: torch.Tensor, degrees=(8, 16, 24, 32),
                       maxit=(8, 8, 12, 16), tol: float = 1e-32, diverge: float = 1.0,
                       min_steps: int = 2, ws=None, status=None, stream=None):
    """Newton's method over increasing truncation degrees from the point x0
    (planes (2, m, n)), each degree from x0, until |dx_d| <= tol (tested
    from step min_steps on) or maxit steps; a degree ending above `diverge`
    stops the later ones.  Returns
    (x planes (2, m, dmax+1, n), iters int32 (ndeg,), norms (m, ndeg),
    status); all decisions are taken on the device."""
    m = _limbs(x0)
    if x0.dim() != 3 or x0.shape[2] != sysd.n:
        raise MdError("md_newton_protocol: x0 must have shape (2, m, n)")
    deg = np.ascontiguousarray(degrees, dtype=np.int32)
    mit = np.ascontiguousarray(maxit, dtype=np.int32)
    if deg.ndim != 1 or deg.shape != mit.shape or deg.size < 1:
        raise MdError("md_newton_protocol: degrees and maxit must be equal-length lists")
    dmax = int(deg[-1])
    h = sysd.host
    if ws is None:
        ws = workspace(MD_FN_PROTOCOL, m, sysd.N, sysd.n, dmax, h.M, h.max_deg, x0.device)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=x0.device)
    x = torch.empty((2, m, dmax + 1, sysd.n), dtype=torch.float64, device=x0.device)
    iters = torch.empty(deg.size, dtype=torch.int32, device=x0.device)
    norms = torch.empty((m, deg.size), dtype=torch.float64, device=x0.device)
    _check(lib().md_newton_protocol(m, ctypes.byref(sysd.desc), _ptr(x0), int(deg.size),
                                    deg.ctypes.data_as(ctypes.c_void_p),
                                    mit.ctypes.data_as(ctypes.c_void_p), int(min_steps),
                                    float(tol),
                                    float(diverge), _ptr(x), _ptr(iters, torch.int32),
                                    _ptr(norms), _ptr(ws, torch.uint8), ws.numel(),
                                    _ptr(status, torch.int32), _stream(stream)),
           "md_newton_protocol")
    return x, iters, norms, status


MD_NOALLOC_SCRATCH_BYTES = 32 << 20


def md_newton_step_noalloc(sysd: DeviceSystem, x: torch.Tensor, dx_norm: torch.Tensor,
                           status: torch.Tensor, stream=None):
    """md_newton_step with the library's fixed per-GPU scratch instead of a
    workspace: the caller passes every buffer (x, dx_norm (m, 2), status
    int32[1]) and nothing is allocated here or in the library."""
    m = _limbs(x)
    _, _, L, n = x.shape
    if tuple(dx_norm.shape) != (m, 2) or dx_norm.dtype != torch.float64:
        raise MdError("md_newton_step_noalloc: dx_norm must be float64 (m, 2)")
    if status.dtype != torch.int32 or status.numel() < 1:
        raise MdError("md_newton_step_noalloc: status must be int32 with one element")
    _check(lib().md_newton_step_noalloc(m, L - 1, ctypes.byref(sysd.desc), _ptr(x),
                                        _ptr(dx_norm), _ptr(status, torch.int32),
                                        _stream(stream)), "md_newton_step_noalloc")
    return x, dx_norm, status


def md_newton_adjoint(sysd: DeviceSystem, x: torch.Tensor, grad_x: torch.Tensor,
                      store_monomials: bool = True, grad_coef=None, ws=None, status=None,
                      stream=None):
    """Coefficient gradient of a real loss through the converged series x
    (2, m, d+1, n) given grad_x = dL/dRe x + i dL/dIm x (same planes);
    returns (grad_coef planes (2, 2, M, dc+1) in double double, status)."""
    m = _limbs(x)
    _, _, L, n = x.shape
    if tuple(grad_x.shape) != tuple(x.shape):
        raise MdError(f"md_newton_adjoint: grad_x shape {tuple(grad_x.shape)} != x {tuple(x.shape)}")
    h = sysd.host
    if grad_coef is None:
        grad_coef = torch.empty((2, 2, h.M, h.dc + 1), dtype=torch.float64, device=x.device)
    elif tuple(grad_coef.shape) != (2, 2, h.M, h.dc + 1):
        raise MdError(f"md_newton_adjoint: grad_coef shape {tuple(grad_coef.shape)}")
    if ws is None:
        fn = MD_FN_ADJOINT_STORE if store_monomials else MD_FN_ADJOINT
        ws = workspace(fn, m, sysd.N, n, L - 1, h.M, h.max_deg, x.device)
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=x.device)
    _check(lib().md_newton_adjoint(m, L - 1, ctypes.byref(sysd.desc), _ptr(x), _ptr(grad_x),
                                   int(bool(store_monomials)), _ptr(grad_coef),
                                   _ptr(ws, torch.uint8), ws.numel(), _ptr(status, torch.int32),
                                   _stream(stream)), "md_newton_adjoint")
    return grad_coef, status


def md_elementwise(op: str, a: torch.Tensor, b: torch.Tensor | None = None, stream=None):
    """One multiple-double operation per element (real planes (m, count) or
    complex planes (2, m, count))."""
    if op in REAL_OPS:
        m, count = a.shape
        out = torch.empty((m, count), dtype=torch.float64, device=a.device)
    else:
        _, m, count = a.shape
        out = torch.empty((m, count) if op == "cabs2" else (2, m, count), dtype=torch.float64,
                          device=a.device)
    _check(lib().md_elementwise(m, OPS[op], count, _ptr(a), _ptr(b), _ptr(out), _stream(stream)),
           "md_elementwise")
    return out


def md_norm2(x: torch.Tensor, stream=None) -> torch.Tensor:
    """2-norm of a complex vector (2, m, count) -> real limbs (m, 1)."""
    m = _limbs(x)
    count = x.shape[2]
    out = torch.empty((m, 1), dtype=torch.float64, device=x.device)
    _check(lib().md_norm2(m, count, _ptr(x), _ptr(out), _stream(stream)), "md_norm2")
    return out


def newton(sysd: DeviceSystem, x: torch.Tensor, iters: int, stream=None):
    """iters Newton steps in place, one workspace; returns (x, list of dx_norm, status)."""
    m = _limbs(x)
    _, _, L, n = x.shape
    ws = workspace(MD_FN_NEWTON, m, sysd.N, n, L - 1, sysd.host.M, sysd.host.max_deg, x.device)
    status = torch.zeros(1, dtype=torch.int32, device=x.device)
    norms = []
    for _ in range(iters):
        _, nrm, _ = md_newton_step(sysd, x, ws=ws, status=status, stream=stream)
        norms.append(nrm)
    return x, norms, status


# -----------------------------------------------------------------------------
# batched paths

MD_PATH_DTYPE = np.dtype([("m", "<i4"), ("N", "<i4"), ("n", "<i4"), ("d", "<i4"),
                          ("M", "<i4"), ("dc", "<i4"), ("max_deg", "<i4"), ("reserved", "<i4"),
                          ("eq_ptr", "<i8"), ("term_ptr", "<i8"), ("factors", "<i8"),
                          ("coef", "<i8"), ("x", "<i8"), ("dx_norm", "<i8"), ("ws", "<i8")])
assert MD_PATH_DTYPE.itemsize == 88
BATCH_MAX_M, BATCH_MAX_N = 4, 64
BATCH_LO_M, BATCH_HI_M = (1, 2, 3, 4), (5, 8, 10)


def sysm_class(m: int) -> bool:
    """True for the penta to deca double kernel."""
    return m in BATCH_HI_M


class BatchedPaths:
    """Device arenas for md_newton_batch: every path's system structure (one
    int32 arena), coefficients, series and update norms (one float64 arena),
    and private workspaces (one float64 arena, 256-byte aligned slices).
    `paths` is a list of (System, x planes (2, m, d+1, n)); `order` (job
    order) defaults to longest first by the analytic operation count;
    protocol: size the workspaces for md_newton_batch_protocol."""

    def __init__(self, paths, device="cuda", order=None, protocol: bool = False):
        from . import opcount as OC
        ints, reals = [], []
        n_int, n_real, n_ws = 0, 0, 0
        table = np.zeros(len(paths), dtype=MD_PATH_DTYPE)
        cost = np.zeros(len(paths))
        self.meta = []
        for p, (sysm, x) in enumerate(paths):
            validate_system(sysm)
            m = sysm.m
            d = x.shape[2] - 1
            if x.shape != (2, m, d + 1, sysm.n):
                raise MdError(f"path {p}: x must have shape (2, m, d+1, n)")
            # the batched kernels carry double to quad double, or penta, octo
            # and deca double (one launch holds one of the two classes), and
            # at most 64 equations (one lane per row of the QR and of the
            # R^{-1} Q^H segments)
            if m not in BATCH_LO_M + BATCH_HI_M:
                raise MdError(f"path {p}: m={m} is not carried by the batched kernels")
            m0 = paths[0][0].m
            if (m in BATCH_HI_M) != sysm_class(m0) or (m in BATCH_HI_M and m != m0):
                raise MdError(f"path {p}: m={m} and m={m0} in one batch (double to quad double "
                              "run in one launch, and penta, octo and deca double each in "
                              "separate launches)")
            if not 1 <= sysm.n <= sysm.N <= BATCH_MAX_N:
                raise MdError(f"path {p}: needs 1 <= n <= N <= {BATCH_MAX_N} "
                              f"(n={sysm.n}, N={sysm.N})")
            t = table[p]
            t["m"], t["N"], t["n"], t["d"] = m, sysm.N, sysm.n, d
            t["M"], t["dc"], t["max_deg"] = sysm.M, sysm.dc, sysm.max_deg
            for name in ("eq_ptr", "term_ptr", "factors"):
                arr = np.asarray(getattr(sysm, name), dtype=np.int32)
                t[name] = n_int
                ints.append(arr)
                n_int += arr.size
            for name, arr in (("coef", sysm.coef), ("x", x), ("dx_norm", np.zeros((m, 2)))):
                arr = np.ascontiguousarray(arr, dtype=np.float64).ravel()
                t[name] = n_real
                reals.append(arr)
                n_real += arr.size
            wsb = lib().md_workspace_bytes(MD_FN_PROTOCOL if protocol else MD_FN_NEWTON, m, sysm.N,
                                           sysm.n, d, sysm.M, sysm.max_deg)
            if wsb == 0:
                raise MdError(f"path {p}: unsupported sizes")
            t["ws"] = n_ws
            n_ws += (wsb + 255) // 256 * 32
            cost[p] = OC.newton_step(sysm, d, m).table_ops(m)
            self.meta.append((m, sysm.N, sysm.n, d))
        dev = torch.device(device)
        self.protocol = protocol
        self.npaths = len(paths)
        self.table = table
        self.cost = cost
        self.max_m = int(table["m"].max()) if len(paths) else 1
        self.max_N = int(table["N"].max()) if len(paths) else 1
        self.max_d = int(table["d"].max()) if len(paths) else 0
        self.max_deg = int(table["max_deg"].max()) if len(paths) else 0
        self.paths_dev = torch.as_tensor(table.view(np.uint8).copy(), device=dev)
        self.ints = torch.as_tensor(np.concatenate(ints) if ints else np.zeros(1, np.int32), device=dev)
        self.reals = torch.as_tensor(np.concatenate(reals) if reals else np.zeros(1), device=dev)
        self.reals0 = self.reals.clone()  # start values, for restore()
        ws = torch.empty(n_ws + 32, dtype=torch.float64, device=dev)
        off = ((-ws.data_ptr()) % 256) // 8
        self.ws = ws[off:off + max(n_ws, 1)]
        self.device = dev
        self.counters = torch.zeros(64, dtype=torch.int32, device=dev)
        self.gang_ctr = torch.zeros(max(len(paths), 1), dtype=torch.int32, device=dev)
        self.status = torch.zeros(max(len(paths), 1), dtype=torch.int32, device=dev)
        self.set_schedule(order=order)

    def x(self, p: int) -> torch.Tensor:
        m, N, n, d = self.meta[p]
        o = int(self.table[p]["x"])
        return self.reals[o:o + 2 * m * (d + 1) * n].view(2, m, d + 1, n)

    def dx_norm(self, p: int) -> torch.Tensor:
        m = self.meta[p][0]
        o = int(self.table[p]["dx_norm"])
        return self.reals[o:o + 2 * m].view(m, 2)

    def restore(self):
        """Put the start series back from the device copy taken at
        construction and clear the status (device work only)."""
        self.reals.copy_(self.reals0)
        self.status.zero_()

    def set_order(self, order):
        """One queue, one workgroup per path, jobs in the given order (a
        permutation of the paths)."""
        self.set_schedule(order=order)

    def set_schedule(self, order=None, gangs=None, nq: int = 1, weights=None):
        """Job lists for md_newton_batch.  order: job order for one queue
        (default: longest first by the analytic cost).  nq > 1: the paths are
        spread over nq queues (one per accelerator die), longest first onto
        the least loaded queue by `weights` (default the analytic cost), and
        each queue runs its paths longest first; gangs (G per path) split a
        path over G workgroups (of one die when nq > 1)."""
        npaths = self.npaths
        w = np.asarray(self.cost if weights is None else weights, dtype=np.float64)
        G = np.ones(npaths, dtype=np.int64) if gangs is None else np.asarray(gangs, dtype=np.int64)
        if G.shape != (npaths,) or G.min(initial=1) < 1 or G.max(initial=1) > 32:
            raise MdError("gangs must give 1..32 workgroups per path")
        if nq < 1 or nq > 64:
            raise MdError("nq must be in 1..64")
        if order is not None:
            order = np.asarray(order, dtype=np.int64)
            if sorted(order.tolist()) != list(range(npaths)):
                raise MdError("order must be a permutation of the paths")
            if nq != 1:
                raise MdError("an explicit order is for one queue")
            queues = [order]
        else:
            by_w = np.argsort(-w, kind="stable")
            if nq == 1:
                queues = [by_w]
            else:
                load = np.zeros(nq)
                qs = [[] for _ in range(nq)]
                for p in by_w:
                    q = int(np.argmin(load))
                    qs[q].append(int(p))
                    load[q] += w[p]
                queues = [np.asarray(qp, dtype=np.int64) for qp in qs]
        jobs, qbegin = [], [0]
        for qp in queues:
            for p in qp:
                for r in range(int(G[p])):
                    jobs.append((int(p), (int(G[p]) << 8) | r))
            qbegin.append(len(jobs))
        self.nq = nq
        self.gangs = G
        self.njobs = len(jobs)
        self.jobs = torch.as_tensor(np.asarray(jobs, dtype=np.int32).reshape(-1) if jobs
                                    else np.zeros(2, np.int32), device=self.device)
        self.qbegin = torch.as_tensor(np.asarray(qbegin, dtype=np.int32), device=self.device)

    def reset(self, paths):
        """Put the start series back (same structure as at construction)."""
        for p, (_, x) in enumerate(paths):
            self.x(p).copy_(torch.as_tensor(np.ascontiguousarray(x)))
        self.status.zero_()


def md_batch_lds_bytes(max_m: int, max_d: int, max_deg: int, eval_waves: int) -> int:
    L = lib()
    L.md_batch_lds_bytes.argtypes = [ctypes.c_int] * 4
    L.md_batch_lds_bytes.restype = ctypes.c_size_t
    return int(L.md_batch_lds_bytes(max_m, max_d, max_deg, eval_waves))


def md_newton_batch(batch: BatchedPaths, iters: int, grid: int | None = None,
                    eval_waves: int | None = None, stream=None, block: int = 256,
                    path_clock: torch.Tensor | None = None,
                    phase_clock: torch.Tensor | None = None):
    """`iters` Newton steps on every path of the batch in one persistent
    launch, with the batch's job schedule (BatchedPaths.set_schedule; the
    library resets the counters on the stream first).  path_clock: optional
    int64 device tensor (npaths, 2) that receives each path's start and end
    on the device wall clock; phase_clock: optional int64 (npaths, 8),
    zeroed, receives the ticks each path spent per phase (evaluation, sums,
    QR, R^{-1} Q^H, stages, update)."""
    L = lib()
    P, i32 = ctypes.c_void_p, ctypes.c_int
    L.md_newton_batch.argtypes = [i32, P, i32, P, i32, P, P, P, P, i32, P, P, P, i32, i32, i32,
                                  i32, i32, i32, i32, P, P, P]
    L.md_newton_batch.restype = ctypes.c_int
    if batch.max_m >= 5 and block != 256:
        if block == 512 and eval_waves is None:
            block = 256  # penta to deca double run 256-thread workgroups
        else:
            raise MdError("md_newton_batch: penta to deca double paths run with block=256")
    if eval_waves is None:
        eval_waves = block // 64
        while eval_waves > 1 and md_batch_lds_bytes(batch.max_m, batch.max_d, batch.max_deg,
                                                     eval_waves) > md_device_lds_bytes():
            eval_waves -= 1
    if grid is None:
        props = torch.cuda.get_device_properties(batch.reals.device)
        grid = props.multi_processor_count
    if path_clock is not None and tuple(path_clock.shape) != (batch.npaths, 2):
        raise MdError("path_clock must have shape (npaths, 2)")
    if phase_clock is not None and tuple(phase_clock.shape) != (batch.npaths, 8):
        raise MdError("phase_clock must have shape (npaths, 8)")
    if grid < batch.nq * int(batch.gangs.max(initial=1)):
        raise MdError(f"grid={grid} too small for {batch.nq} queues with gangs of "
                      f"{int(batch.gangs.max(initial=1))}")
    _check(L.md_newton_batch(batch.npaths, _ptr(batch.paths_dev, torch.uint8), batch.njobs,
                             _ptr(batch.jobs, torch.int32), batch.nq,
                             _ptr(batch.qbegin, torch.int32), _ptr(batch.ints, torch.int32),
                             _ptr(batch.reals), _ptr(batch.ws), iters,
                             _ptr(batch.counters, torch.int32), _ptr(batch.gang_ctr, torch.int32),
                             _ptr(batch.status, torch.int32), batch.max_m, batch.max_N,
                             batch.max_d, batch.max_deg, grid, block, eval_waves,
                             _ptr(path_clock, torch.int64), _ptr(phase_clock, torch.int64),
                             _stream(stream)), "md_newton_batch")
    return batch


class md_protocol(ctypes.Structure):
    _fields_ = [("ndeg", ctypes.c_int32), ("min_steps", ctypes.c_int32),
                ("degrees", ctypes.c_int32 * MD_PROTOCOL_MAX_DEGREES),
                ("maxit", ctypes.c_int32 * MD_PROTOCOL_MAX_DEGREES),
                ("tol", ctypes.c_double), ("diverge", ctypes.c_double)]


def md_newton_batch_protocol(batch: BatchedPaths, degrees=(8, 16, 24, 32), maxit=(8, 8, 12, 16),
                             tol: float = 1e-32, diverge: float = 1.0, min_steps: int = 2,
                             grid: int | None = None, block: int = 512,
                             eval_waves: int | None = None, stream=None):
    """Section 6's protocol on every path of the batch in one persistent
    launch (per-path decisions on the device).  The batch must have been
    built with protocol=True.  Returns (iters int32 (npaths, ndeg), norms
    float64 (npaths, ndeg, 10): |dx_d| per degree as limbs)."""
    if not batch.protocol:
        raise MdError("md_newton_batch_protocol: build the batch with protocol=True")
    if batch.max_m > 4:
        raise MdError("md_newton_batch_protocol: double to quad double paths only")
    deg, mit = list(degrees), list(maxit)
    if not 1 <= len(deg) <= MD_PROTOCOL_MAX_DEGREES or len(deg) != len(mit):
        raise MdError("md_newton_batch_protocol: degrees and maxit must be equal-length lists")
    pr = md_protocol()
    pr.ndeg, pr.min_steps, pr.tol, pr.diverge = len(deg), int(min_steps), float(tol), float(diverge)
    for j, (dj, mj) in enumerate(zip(deg, mit)):
        pr.degrees[j], pr.maxit[j] = int(dj), int(mj)
    L = lib()
    P, i32 = ctypes.c_void_p, ctypes.c_int
    L.md_newton_batch_protocol.argtypes = [i32, P, i32, P, i32, P, P, P, P,
                                           ctypes.POINTER(md_protocol), P, P, P, i32, i32, i32,
                                           i32, i32, i32, i32, P, P, P]
    L.md_newton_batch_protocol.restype = ctypes.c_int
    if eval_waves is None:
        eval_waves = block // 64
        while eval_waves > 1 and md_batch_lds_bytes(batch.max_m, batch.max_d, batch.max_deg,
                                                     eval_waves) > md_device_lds_bytes():
            eval_waves -= 1
    if grid is None:
        grid = torch.cuda.get_device_properties(batch.reals.device).multi_processor_count
    if grid < batch.nq * int(batch.gangs.max(initial=1)):
        raise MdError(f"grid={grid} too small for {batch.nq} queues with gangs of "
                      f"{int(batch.gangs.max(initial=1))}")
    iters = torch.zeros((batch.npaths, len(deg)), dtype=torch.int32, device=batch.device)
    norms = torch.zeros((batch.npaths, len(deg), 10), dtype=torch.float64, device=batch.device)
    _check(L.md_newton_batch_protocol(batch.npaths, _ptr(batch.paths_dev, torch.uint8),
                                      batch.njobs, _ptr(batch.jobs, torch.int32), batch.nq,
                                      _ptr(batch.qbegin, torch.int32),
                                      _ptr(batch.ints, torch.int32), _ptr(batch.reals),
                                      _ptr(batch.ws), ctypes.byref(pr),
                                      _ptr(batch.counters, torch.int32),
                                      _ptr(batch.gang_ctr, torch.int32),
                                      _ptr(batch.status, torch.int32), batch.max_m, batch.max_N,
                                      batch.max_d, batch.max_deg, grid, block, eval_waves,
                                      _ptr(iters, torch.int32), _ptr(norms), _stream(stream)),
           "md_newton_batch_protocol")
    return iters, norms


_dies = {}


def md_device_dies(device: int = 0) -> int:
    """Number of accelerator dies the queues of md_newton_batch map to
    (distinct die ids over a small launch)."""
    if device not in _dies:
        L = lib()
        L.md_device_dies.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]
        ids = torch.full((256,), -1, dtype=torch.int32, device=f"cuda:{device}")
        _check(L.md_device_dies(_ptr(ids, torch.int32), 256, _stream(None)), "md_device_dies")
        v = ids.cpu().numpy()
        _dies[device] = int(v.max()) + 1
    return _dies[device]


def md_device_lds_bytes() -> int:
    L = lib()
    L.md_device_lds_bytes.argtypes = []
    L.md_device_lds_bytes.restype = ctypes.c_size_t
    return int(L.md_device_lds_bytes())


def md_wall_clock_hz(device: int = 0) -> int:
    L = lib()
    L.md_wall_clock_hz.argtypes = [ctypes.c_int, ctypes.c_void_p]
    hz = ctypes.c_int64(0)
    _check(L.md_wall_clock_hz(device, ctypes.byref(hz)), "md_wall_clock_hz")
    return int(hz.value)
