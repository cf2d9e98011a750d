"""Quantization-based bounds on the Wasserstein metric, MI355X-native.

Python binding of libqbw (include/qbw.h): argument marshalling only - every
step runs in the library (host network simplex for the coarse problem, HIP
kernels for gfx950 for everything on the fine grid).  PyTorch supplies device
memory and streams.  Measures are float64 CUDA tensors of shape (N,)*d.

    lower, upper = wasserstein_bounds(a, b, k=8, p=2)      # differentiable
    res = bounds(a, b, k=8, p=2)                            # dict, no autograd
"""
from __future__ import annotations

import ctypes as C
import threading

import numpy as np
import torch

from . import _lib
from ._lib import (QBW_BATCH_AUTOTUNE, QBW_BATCH_BACKWARD, QBW_BATCH_GRAPH, QBW_INTERP_CUBIC,
                   QBW_INTERP_NEAREST, QBW_SAVE_FOR_BWD, QBW_SEPARABLE, QBW_SEPARABLE_EXACT, QBW_WANT_ARGMIN, QBW_WARN_IPF_NOT_CONVERGED, QBW_WARN_LB_CLIPPED, QbwCoarse,
                   QbwError, QbwGrid, QbwJob, QbwOpts, QbwResult, check, load)

__all__ = ["Context", "Coarse", "Batch", "bounds", "wasserstein_bounds", "BoundsFunction",
           "sumpool", "coarse_cost", "cbar", "coarse_solve", "upscale_potential", "ctransform",
           "ctransform_separable", "ctransform_exact",
           "ipf", "plan_cost", "tv", "upper_kernel", "upper_kernel_bound", "UpperKernelFunction",
           "plan_kernel_gaussian", "autotune_ctransform", "weighted_cost_upper", "min_cost_lower",
           "bounds_with_grads", "QbwError", "load"]

_tls = threading.local()


class Context:
    """A libqbw context (per host thread and device)."""

    def __init__(self, device: int = 0):
        lib = load()
        h = C.c_void_p()
        check(lib.qbw_create(C.byref(h), int(device)), "qbw_create")
        self.handle = h
        self.device = int(device)
        self._lib = lib   # held for __del__: module globals may be gone at exit

    def __del__(self):
        h = getattr(self, "handle", None)
        lib = getattr(self, "_lib", None)
        if h is not None and h.value and lib is not None:
            lib.qbw_destroy(h)
            self.handle = None


def context(device: int | None = None) -> Context:
    if device is None:
        device = torch.cuda.current_device()
    cache = getattr(_tls, "ctx", None)
    if cache is None:
        cache = _tls.ctx = {}
    if device not in cache:
        cache[device] = Context(device)
    return cache[device]


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t, dtype=torch.float64):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise QbwError("inputs must be CUDA tensors (the library has no CPU path)")
    if t.dtype != dtype:
        raise QbwError(f"expected {dtype}, got {t.dtype}")
    return t.contiguous()


def _sized(t, count: int, what: str):
    """The library reads and writes exactly `count` elements behind each
    pointer: a shorter tensor would be overrun on the device."""
    if t.numel() != count:
        raise QbwError(f"{what} must hold {count} elements, got {t.numel()}")
    return t


def _pair(a, b):
    """Both measures as contiguous float64 device tensors of one shape."""
    a, b = _dev(a), _dev(b)
    if a.shape != b.shape:
        raise QbwError(f"a and b must have the same shape, got {tuple(a.shape)} and {tuple(b.shape)}")
    return a, b


def _out(t, like, what: str):
    """A caller-given output buffer: written in place through its pointer, so it
    must be a contiguous float64 device tensor with as many elements as `like`."""
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64:
        raise QbwError(f"{what} must be a float64 CUDA tensor")
    if not t.is_contiguous():
        raise QbwError(f"{what} must be contiguous (the library writes through its pointer)")
    return _sized(t, like.numel(), what)


def _grid(a, k, p) -> QbwGrid:
    if a.dim() not in (2, 3) or len(set(a.shape)) != 1:
        raise QbwError(f"measures must have shape (N,)*d with d in {{2,3}}, got {tuple(a.shape)}")
    return QbwGrid(a.dim(), a.shape[0], int(k), int(p))


def _opts(xi, max_ipf_iter, flags) -> QbwOpts:
    return QbwOpts(float(xi), int(max_ipf_iter), int(flags))


_INTERP = {"linear": 0, "nearest": QBW_INTERP_NEAREST, "cubic": QBW_INTERP_CUBIC}


def _interp(interp: str) -> int:
    """Flag bits of the interpolation R of the coarse potential (Section 3.5)."""
    if interp not in _INTERP:
        raise QbwError(f"interp must be one of {sorted(_INTERP)}, got {interp!r}")
    return _INTERP[interp]


class Coarse:
    """A coarse solution (coupling pi~ as COO, potential f~), held in host memory."""

    def __init__(self, rows, cols, vals, f, g=None, objective=None):
        self.rows = np.ascontiguousarray(rows, dtype=np.int32)
        self.cols = np.ascontiguousarray(cols, dtype=np.int32)
        self.vals = np.ascontiguousarray(vals, dtype=np.float64)
        self.f = np.ascontiguousarray(f, dtype=np.float64)
        self.g = None if g is None else np.ascontiguousarray(g, dtype=np.float64)
        self.objective = objective

    @property
    def Q(self):
        return len(self.f)

    def struct(self) -> QbwCoarse:
        return QbwCoarse(self.Q, len(self.vals),
                         self.rows.ctypes.data_as(C.POINTER(C.c_int32)),
                         self.cols.ctypes.data_as(C.POINTER(C.c_int32)),
                         self.vals.ctypes.data_as(C.POINTER(C.c_double)),
                         self.f.ctypes.data_as(C.POINTER(C.c_double)))


def coarse_solve(a_t, b_t, N: int, d: int, k: int, p: int) -> Coarse:
    """Exact coarse problem on the centre cost (host network simplex)."""
    a_t = np.ascontiguousarray(a_t, dtype=np.float64).reshape(-1)
    b_t = np.ascontiguousarray(b_t, dtype=np.float64).reshape(-1)
    Q = len(a_t)
    rows = np.zeros(2 * Q, np.int32)
    cols = np.zeros(2 * Q, np.int32)
    vals = np.zeros(2 * Q, np.float64)
    f = np.zeros(Q)
    g = np.zeros(Q)
    nnz = C.c_int32()
    obj = C.c_double()
    grid = QbwGrid(d, N, k, p)
    check(load().qbw_coarse_solve_host(C.byref(grid), a_t.ctypes.data, b_t.ctypes.data,
                                       rows.ctypes.data, cols.ctypes.data, vals.ctypes.data,
                                       C.byref(nnz), f.ctypes.data, g.ctypes.data, C.byref(obj)),
          "qbw_coarse_solve_host")
    n = nnz.value
    return Coarse(rows[:n], cols[:n], vals[:n], f, g, obj.value)


def _sep_flag(separable) -> int:
    """separable=False: all-pairs c-transforms; True: axis by axis with float32
    rounding per axis (QBW_SEPARABLE); "exact": axis by axis in float64 with the
    all-pairs values and arg-mins (QBW_SEPARABLE_EXACT).  p = 1 jobs ignore it."""
    if separable is False or separable is None:
        return 0
    if separable is True:
        return QBW_SEPARABLE
    if separable == "exact":
        return QBW_SEPARABLE_EXACT
    raise ValueError(f"separable must be False, True or 'exact' (got {separable!r})")


def bounds(a, b, k: int, p: int, coarse: Coarse | None = None, xi: float = 1e-12,
           max_ipf_iter: int = 50, want_argmin: bool = False, separable: bool = False,
           interp: str = "linear") -> dict:
    """Lower and upper bound of W_p(a, b) (no autograd).  Returns the qbw_result fields.
    separable=True evaluates the p = 2 c-transforms axis by axis (QBW_SEPARABLE),
    separable="exact" axis by axis with the all-pairs results (QBW_SEPARABLE_EXACT);
    interp picks the interpolation of the coarse potential ("linear", "nearest", "cubic")."""
    a, b = _pair(a, b)
    grid = _grid(a, k, p)
    opts = _opts(xi, max_ipf_iter, (QBW_WANT_ARGMIN if want_argmin else 0) | _sep_flag(separable) |
                 _interp(interp))
    res = QbwResult()
    lib = load()
    ctx = context(a.device.index)
    if coarse is None:
        rc = lib.qbw_bounds(ctx.handle, C.byref(grid), _ptr(a), _ptr(b), C.byref(opts), C.byref(res),
                            None, _stream())
    else:
        cs = coarse.struct()
        rc = lib.qbw_bounds_with_coarse(ctx.handle, C.byref(grid), _ptr(a), _ptr(b), C.byref(cs),
                                        C.byref(opts), C.byref(res), None, _stream())
    check(rc, "qbw_bounds")
    return res.as_dict()


class _Saved:
    def __init__(self, handle):
        self.handle = handle
        self._lib = load()   # held for __del__: module globals may be gone at exit

    def __del__(self):
        if self.handle is not None and self.handle.value:
            self._lib.qbw_saved_free(self.handle)
            self.handle = None


class BoundsFunction(torch.autograd.Function):
    """(lower, upper) = f(a, b); backward runs the library's gradient kernels with
    the coarse solution frozen (see qbw_bounds_backward)."""

    @staticmethod
    def forward(ctx, a, b, k, p, coarse, xi, max_ipf_iter, want_argmin, separable=False, interp="linear"):
        a, b = _pair(a, b)
        grid = _grid(a, k, p)
        flags = QBW_SAVE_FOR_BWD | (QBW_WANT_ARGMIN if want_argmin else 0) | _sep_flag(separable) | \
            _interp(interp)
        opts = _opts(xi, max_ipf_iter, flags)
        res = QbwResult()
        saved = C.c_void_p()
        lib = load()
        qctx = context(a.device.index)
        if coarse is None:
            rc = lib.qbw_bounds(qctx.handle, C.byref(grid), _ptr(a), _ptr(b), C.byref(opts),
                                C.byref(res), C.byref(saved), _stream())
        else:
            cs = coarse.struct()
            rc = lib.qbw_bounds_with_coarse(qctx.handle, C.byref(grid), _ptr(a), _ptr(b), C.byref(cs),
                                            C.byref(opts), C.byref(res), C.byref(saved), _stream())
        check(rc, "qbw_bounds")
        ctx.saved_handle = _Saved(saved)
        ctx.save_for_backward(a, b)
        ctx.result = res.as_dict()
        lower = torch.tensor(res.lower, dtype=torch.float64, device=a.device)
        upper = torch.tensor(res.upper, dtype=torch.float64, device=a.device)
        return lower, upper

    @staticmethod
    def backward(ctx, dlower, dupper):
        a, b = ctx.saved_tensors
        ga = torch.zeros_like(a)
        gb = torch.zeros_like(b)
        dl = 0.0 if dlower is None else float(dlower)
        du = 0.0 if dupper is None else float(dupper)
        check(load().qbw_bounds_backward(context(a.device.index).handle, ctx.saved_handle.handle,
                                         dl, du, _ptr(ga), _ptr(gb), None, _stream()),
              "qbw_bounds_backward")
        return ga, gb, None, None, None, None, None, None, None, None


def wasserstein_bounds(a, b, k: int, p: int, coarse: Coarse | None = None, xi: float = 1e-12,
                       max_ipf_iter: int = 50, want_argmin: bool = False, separable: bool = False,
                       interp: str = "linear"):
    """Differentiable (lower, upper) bounds on W_p(a, b)."""
    return BoundsFunction.apply(a, b, k, p, coarse, xi, max_ipf_iter, want_argmin, separable, interp)


def bounds_with_grads(a, b, k: int, p: int, coarse: Coarse | None = None, dlower: float = 1.0,
                      dupper: float = 1.0, want_fhat_grad: bool = False, xi: float = 1e-12,
                      max_ipf_iter: int = 50, separable: bool = False, interp: str = "linear"):
    """Forward + backward in one call: returns (result dict, grad_a, grad_b, grad_fhat or None)."""
    a, b = _pair(a, b)
    grid = _grid(a, k, p)
    opts = _opts(xi, max_ipf_iter, QBW_SAVE_FOR_BWD | (QBW_WANT_ARGMIN if want_fhat_grad else 0) |
                 _sep_flag(separable) | _interp(interp))
    res = QbwResult()
    saved = C.c_void_p()
    lib = load()
    qctx = context(a.device.index)
    if coarse is None:
        rc = lib.qbw_bounds(qctx.handle, C.byref(grid), _ptr(a), _ptr(b), C.byref(opts), C.byref(res),
                            C.byref(saved), _stream())
    else:
        cs = coarse.struct()
        rc = lib.qbw_bounds_with_coarse(qctx.handle, C.byref(grid), _ptr(a), _ptr(b), C.byref(cs),
                                        C.byref(opts), C.byref(res), C.byref(saved), _stream())
    check(rc, "qbw_bounds")
    holder = _Saved(saved)
    ga, gb = torch.zeros_like(a), torch.zeros_like(b)
    gf = torch.zeros(a.numel(), dtype=torch.float64, device=a.device) if want_fhat_grad else None
    check(lib.qbw_bounds_backward(qctx.handle, holder.handle, float(dlower), float(dupper), _ptr(ga),
                                  _ptr(gb), _ptr(gf), _stream()), "qbw_bounds_backward")
    del holder
    return res.as_dict(), ga, gb, gf


# ------------------------------------------------------------------ stages

def sumpool(m, k: int):
    m = _dev(m)
    grid = _grid(m, k, 2)
    n = m.shape[0] // k
    out = torch.empty(n ** m.dim(), dtype=torch.float64, device=m.device)
    check(load().qbw_sumpool(context(m.device.index).handle, C.byref(grid), _ptr(m), _ptr(out),
                             _stream()), "qbw_sumpool")
    return out


def coarse_cost(N: int, d: int, k: int, p: int) -> np.ndarray:
    Q = (N // k) ** d
    out = np.zeros((Q, Q))
    grid = QbwGrid(d, N, k, p)
    check(load().qbw_coarse_cost(C.byref(grid), out.ctypes.data), "qbw_coarse_cost")
    return out


def cbar(a, b, k: int, p: int):
    a, b = _pair(a, b)
    grid = _grid(a, k, p)
    Q = (a.shape[0] // k) ** a.dim()
    out = torch.empty((Q, Q), dtype=torch.float64, device=a.device)
    check(load().qbw_cbar(context(a.device.index).handle, C.byref(grid), _ptr(a), _ptr(b), _ptr(out),
                          _stream()), "qbw_cbar")
    return out


def upscale_potential(ftil, N: int, d: int, k: int, interp: str = "linear"):
    ftil = _dev(ftil)
    if 1 <= k <= N and N % k == 0:   # other shapes are the library's QBW_E_GRID
        _sized(ftil, (N // k) ** d, "ftil")
    grid = QbwGrid(d, N, k, 2)
    out = torch.empty(N ** d, dtype=torch.float32, device=ftil.device)
    check(load().qbw_upscale_potential_interp(context(ftil.device.index).handle, C.byref(grid),
                                              _interp(interp), _ptr(ftil), _ptr(out), _stream()),
          "qbw_upscale_potential_interp")
    return out


def ctransform(src, N: int, d: int, p: int, want_argmin: bool = False):
    src = _sized(_dev(src, torch.float32), N ** d, "src")
    grid = QbwGrid(d, N, 1, p)
    dst = torch.empty_like(src)
    arg = torch.empty(src.shape, dtype=torch.int32, device=src.device) if want_argmin else None
    check(load().qbw_ctransform(context(src.device.index).handle, C.byref(grid), _ptr(src), _ptr(dst),
                                _ptr(arg), _stream()), "qbw_ctransform")
    return (dst, arg) if want_argmin else dst


def ctransform_noalloc(src, N: int, d: int, p: int, dst=None, argmin=None):
    """qbw_ctransform_noalloc: the c-transform of ``ctransform`` computed in the
    library's static device scratch.  ``dst`` (float32) and ``argmin`` (int32,
    optional) are caller-owned N^d buffers; ``dst`` is created here when None.
    Returns dst, or (dst, argmin) when argmin is given."""
    src = _sized(_dev(src, torch.float32), N ** d, "src")
    if dst is None:
        dst = torch.empty_like(src)
    elif not (isinstance(dst, torch.Tensor) and dst.is_cuda and dst.dtype == torch.float32
              and dst.is_contiguous()):
        raise QbwError("dst must be a contiguous float32 CUDA tensor")
    _sized(dst, N ** d, "dst")
    if argmin is not None:
        if not (isinstance(argmin, torch.Tensor) and argmin.is_cuda and argmin.dtype == torch.int32
                and argmin.is_contiguous()):
            raise QbwError("argmin must be a contiguous int32 CUDA tensor")
        _sized(argmin, N ** d, "argmin")
    grid = QbwGrid(d, N, 1, p)
    check(load().qbw_ctransform_noalloc(context(src.device.index).handle, C.byref(grid), _ptr(src), _ptr(dst),
                                        _ptr(argmin), _stream()), "qbw_ctransform_noalloc")
    return (dst, argmin) if argmin is not None else dst


def ctransform_separable(src, N: int, d: int, want_argmin: bool = False):
    """p = 2 c-transform as d nested 1-D transforms (qbw_ctransform_separable)."""
    src = _sized(_dev(src, torch.float32), N ** d, "src")
    grid = QbwGrid(d, N, 1, 2)
    dst = torch.empty_like(src)
    arg = torch.empty(src.shape, dtype=torch.int32, device=src.device) if want_argmin else None
    check(load().qbw_ctransform_separable(context(src.device.index).handle, C.byref(grid), _ptr(src),
                                          _ptr(dst), _ptr(arg), _stream()), "qbw_ctransform_separable")
    return (dst, arg) if want_argmin else dst


def ctransform_exact(src, N: int, d: int, want_argmin: bool = False, return_fallback: bool = False):
    """p = 2 c-transform with the all-pairs values and arg-mins, from exact
    per-axis minima (qbw_ctransform_exact); return_fallback also returns how
    many targets needed the brute-force evaluation."""
    src = _sized(_dev(src, torch.float32), N ** d, "src")
    grid = QbwGrid(d, N, 1, 2)
    dst = torch.empty_like(src)
    arg = torch.empty(src.shape, dtype=torch.int32, device=src.device) if want_argmin else None
    nfb = C.c_int32(0)
    check(load().qbw_ctransform_exact(context(src.device.index).handle, C.byref(grid), _ptr(src), _ptr(dst),
                                      _ptr(arg), C.byref(nfb), _stream()), "qbw_ctransform_exact")
    out = (dst, arg) if want_argmin else (dst,)
    if return_fallback:
        out = out + (nfb.value,)
    return out if len(out) > 1 else out[0]


def ipf(a, b, k: int, coarse: Coarse, xi: float = 1e-12, max_ipf_iter: int = 50):
    a, b = _pair(a, b)
    grid = _grid(a, k, 2)
    opts = _opts(xi, max_ipf_iter, 0)
    a_s = torch.empty(a.numel(), dtype=torch.float64, device=a.device)
    b_s = torch.empty_like(a_s)
    it = C.c_int32()
    res = C.c_double()
    cs = coarse.struct()
    check(load().qbw_ipf(context(a.device.index).handle, C.byref(grid), _ptr(a), _ptr(b), C.byref(cs),
                         C.byref(opts), _ptr(a_s), _ptr(b_s), C.byref(it), C.byref(res), _stream()),
          "qbw_ipf")
    return a_s, b_s, it.value, res.value


def plan_cost(a_s, b_s, N: int, d: int, k: int, p: int, coarse: Coarse) -> float:
    a_s, b_s = _sized(_dev(a_s), N ** d, "a_s"), _sized(_dev(b_s), N ** d, "b_s")
    grid = QbwGrid(d, N, k, p)
    out = C.c_double()
    cs = coarse.struct()
    check(load().qbw_plan_cost(context(a_s.device.index).handle, C.byref(grid), C.byref(cs), _ptr(a_s),
                               _ptr(b_s), C.byref(out), _stream()), "qbw_plan_cost")
    return out.value


def tv(a, b, k: int, p: int, coarse: Coarse, a_s, b_s):
    (a, b), a_s, b_s = _pair(a, b), _dev(a_s), _dev(b_s)
    grid = _grid(a, k, p)
    _sized(a_s, a.numel(), "a_s"), _sized(b_s, a.numel(), "b_s")
    tm, tn = C.c_double(), C.c_double()
    cs = coarse.struct()
    check(load().qbw_tv(context(a.device.index).handle, C.byref(grid), _ptr(a), _ptr(b), C.byref(cs),
                        _ptr(a_s), _ptr(b_s), C.byref(tm), C.byref(tn), _stream()), "qbw_tv")
    return tm.value, tn.value


def plan_kernel_gaussian(k: int, d: int, sigma: float) -> np.ndarray:
    """(k^d, k^d) kernel for upper_kernel: Gaussian in the in-block offset
    difference, normalised to total 1 (qbw_plan_kernel_gaussian)."""
    m = k ** d
    out = np.empty((m, m), dtype=np.float64)
    check(load().qbw_plan_kernel_gaussian(int(k), int(d), float(sigma), out.ctypes.data),
          "qbw_plan_kernel_gaussian")
    return out


def upper_kernel(a, b, k: int, p: int, kernel, coarse: Coarse | None = None, xi: float = 1e-12,
                 max_ipf_iter: int = 50, return_scalings: bool = False, dupper: float | None = None,
                 grad_a=None, grad_b=None):
    """Upper bound of Algorithm 4 with the coarse coupling upscaled by ``kernel``
    ((k^d, k^d) float64, nonnegative, total 1; entry [s, t] weighs in-block
    offset s of the source block against offset t of the target block).
    Returns the result dict (plus the final scalings a_s, b_s on request).
    With ``dupper``, dupper * d upper / d(a, b) is added into ``grad_a`` /
    ``grad_b`` (float64 tensors shaped like a; created as zeros when None and
    returned in the dict)."""
    a, b = _pair(a, b)
    if coarse is None:
        coarse = coarse_solve(sumpool(a, k).cpu().numpy(), sumpool(b, k).cpu().numpy(),
                              a.shape[0], a.dim(), k, p)
    grid = _grid(a, k, p)
    opts = _opts(xi, max_ipf_iter, 0)
    kern = np.ascontiguousarray(kernel, dtype=np.float64)
    if kern.size != (k ** a.dim()) ** 2:
        raise ValueError(f"kernel must have (k^d)^2 = {(k ** a.dim()) ** 2} entries, got {kern.size}")
    res = QbwResult()
    a_s = b_s = None
    if return_scalings:
        a_s = torch.empty(a.numel(), dtype=torch.float64, device=a.device)
        b_s = torch.empty_like(a_s)
    if dupper is not None:
        grad_a = torch.zeros_like(a) if grad_a is None else _out(grad_a, a, "grad_a")
        grad_b = torch.zeros_like(b) if grad_b is None else _out(grad_b, b, "grad_b")
    cs = coarse.struct()
    check(load().qbw_upper_kernel(context(a.device.index).handle, C.byref(grid), _ptr(a), _ptr(b),
                                  C.byref(cs), kern.ctypes.data, C.byref(opts), C.byref(res),
                                  _ptr(a_s), _ptr(b_s), float(dupper or 0.0),
                                  _ptr(grad_a) if dupper is not None else None,
                                  _ptr(grad_b) if dupper is not None else None, _stream()),
          "qbw_upper_kernel")
    out = res.as_dict()
    if return_scalings:
        out["a_s"], out["b_s"] = a_s, b_s
    if dupper is not None:
        out["grad_a"], out["grad_b"] = grad_a, grad_b
    return out


class UpperKernelFunction(torch.autograd.Function):
    """upper = f(a, b) for the kernel-upscaled upper bound; backward re-runs the
    library's forward with every fitting iterate kept, then its reverse pass
    (qbw_upper_kernel with gradient outputs)."""

    @staticmethod
    def forward(ctx, a, b, k, p, kernel, coarse, xi, max_ipf_iter):
        a, b = _pair(a, b)
        if coarse is None:
            coarse = coarse_solve(sumpool(a, k).cpu().numpy(), sumpool(b, k).cpu().numpy(),
                                  a.shape[0], a.dim(), k, p)
        res = upper_kernel(a, b, k, p, kernel, coarse=coarse, xi=xi, max_ipf_iter=max_ipf_iter)
        ctx.save_for_backward(a, b)
        ctx.args = (k, p, kernel, coarse, xi, max_ipf_iter)
        ctx.result = res
        return torch.tensor(res["upper"], dtype=torch.float64, device=a.device)

    @staticmethod
    def backward(ctx, dupper):
        a, b = ctx.saved_tensors
        k, p, kernel, coarse, xi, max_ipf_iter = ctx.args
        res = upper_kernel(a, b, k, p, kernel, coarse=coarse, xi=xi, max_ipf_iter=max_ipf_iter,
                           dupper=float(dupper))
        return res["grad_a"], res["grad_b"], None, None, None, None, None, None


def upper_kernel_bound(a, b, k: int, p: int, kernel, coarse: Coarse | None = None, xi: float = 1e-12,
                       max_ipf_iter: int = 50):
    """Differentiable kernel-upscaled upper bound on W_p(a, b) (a 0-d tensor)."""
    return UpperKernelFunction.apply(a, b, k, p, kernel, coarse, xi, max_ipf_iter)


def weighted_cost_upper(a, b, k: int, p: int):
    """Weighted-cost upper bound (Algorithm 3): (bound, coarse objective on C-bar)."""
    a, b = _pair(a, b)
    grid = _grid(a, k, p)
    ub, obj = C.c_double(), C.c_double()
    check(load().qbw_weighted_cost_upper(context(a.device.index).handle, C.byref(grid), _ptr(a), _ptr(b),
                                         C.byref(ub), C.byref(obj), _stream()), "qbw_weighted_cost_upper")
    return ub.value, obj.value


def min_cost_lower(a, b, k: int, p: int):
    """Min-cost lower bound (Section 3.3): (bound, coarse objective on C^min)."""
    a, b = _pair(a, b)
    grid = _grid(a, k, p)
    lb, obj = C.c_double(), C.c_double()
    check(load().qbw_min_cost_lower(context(a.device.index).handle, C.byref(grid), _ptr(a), _ptr(b),
                                    C.byref(lb), C.byref(obj), _stream()), "qbw_min_cost_lower")
    return lb.value, obj.value


def autotune_ctransform(N: int, d: int, p: int, device: int | None = None):
    grid = QbwGrid(d, N, 1, p)
    R, Sp, ms = C.c_int32(), C.c_int32(), C.c_double()
    check(load().qbw_autotune_ctransform(context(device).handle, C.byref(grid), C.byref(R), C.byref(Sp),
                                         C.byref(ms), _stream()), "qbw_autotune_ctransform")
    return R.value, Sp.value, ms.value


# ------------------------------------------------------------------ batches

class Batch:
    """Many pairs of uneven sizes behind one persistent launch per stage
    (optionally captured in a hipGraph and autotuned)."""

    def __init__(self, jobs, coarse=None, backward: bool = False, graph: bool = False,
                 autotune: bool = False, xi: float = 1e-12, max_ipf_iter: int = 50,
                 separable: bool = False, interp: str = "linear"):
        """jobs: list of (a, b, k, p) or (a, b, k, p, grad_a, grad_b) with CUDA tensors."""
        lib = load()
        self._keep = []
        arr = (QbwJob * len(jobs))()
        dev = None
        for i, jb in enumerate(jobs):
            a, b, k, p = jb[:4]
            a, b = _pair(a, b)
            ga = gb = None
            if backward:
                ga = _out(jb[4], a, "grad_a") if len(jb) > 4 else torch.zeros_like(a)
                gb = _out(jb[5], b, "grad_b") if len(jb) > 5 else torch.zeros_like(b)
            self._keep += [a, b, ga, gb]
            arr[i] = QbwJob(_grid(a, k, p), a.data_ptr(), b.data_ptr(),
                            ga.data_ptr() if ga is not None else None,
                            gb.data_ptr() if gb is not None else None)
            dev = a.device.index
        self.grads = [(self._keep[4 * i + 2], self._keep[4 * i + 3]) for i in range(len(jobs))]
        cs = None
        if coarse is not None:
            cs = (QbwCoarse * len(jobs))(*[c.struct() for c in coarse])
            self._keep.append(coarse)
        flags = (QBW_BATCH_BACKWARD if backward else 0) | (QBW_BATCH_GRAPH if graph else 0) | \
                (QBW_BATCH_AUTOTUNE if autotune else 0)
        opts = _opts(xi, max_ipf_iter, _sep_flag(separable) | _interp(interp))
        h = C.c_void_p()
        self.n = len(jobs)
        self.ctx = context(dev)
        check(lib.qbw_batch_create(self.ctx.handle, arr, len(jobs), cs, C.byref(opts), flags, C.byref(h),
                                   _stream()), "qbw_batch_create")
        self.handle = h
        self._lib = lib   # held for __del__: module globals may be gone at exit
        self._jobs = arr

    def run(self, dlower=None, dupper=None):
        lib = load()
        dl = np.ascontiguousarray(dlower, dtype=np.float64) if dlower is not None else None
        du = np.ascontiguousarray(dupper, dtype=np.float64) if dupper is not None else None
        check(lib.qbw_batch_run(self.handle, dl.ctypes.data if dl is not None else None,
                                du.ctypes.data if du is not None else None, _stream()), "qbw_batch_run")

    def results(self):
        out = (QbwResult * self.n)()
        check(load().qbw_batch_results(self.handle, out, _stream()), "qbw_batch_results")
        return [r.as_dict() for r in out]

    def tiling(self, j: int):
        R, Sp = C.c_int32(), C.c_int32()
        check(load().qbw_batch_tiling(self.handle, j, C.byref(R), C.byref(Sp)), "qbw_batch_tiling")
        return R.value, Sp.value

    def set_timing(self, enable: bool):
        check(load().qbw_batch_set_timing(self.handle, int(bool(enable))), "qbw_batch_set_timing")

    def ctransform_time(self):
        """(mean c-transform launch duration in ms, launches) since the last call."""
        ms, n = C.c_double(), C.c_int32()
        check(load().qbw_batch_ctransform_time(self.handle, C.byref(ms), C.byref(n)),
              "qbw_batch_ctransform_time")
        return ms.value, n.value

    def ctransform_pairs(self) -> float:
        out = C.c_double()
        check(load().qbw_batch_ctransform_pairs(self.handle, C.byref(out)), "qbw_batch_ctransform_pairs")
        return out.value

    def __del__(self):
        h = getattr(self, "handle", None)
        lib = getattr(self, "_lib", None)
        if h is not None and h.value and lib is not None:
            lib.qbw_batch_destroy(h)
            self.handle = None
