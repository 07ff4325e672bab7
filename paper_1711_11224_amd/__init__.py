"""MI355X (gfx950) n-dimensional full convolution, its transpose and the
projected-gradient deconvolution of "Properties on n-dimensional convolution
for image deconvolution" (arXiv 1711.11224).

The functions named like the C ABI (conv_full_nd, conv_adjoint_nd,
conv_dH_nd, deconv_iterate) take torch tensors that already live on the GPU
and only marshal pointers, extents and the current stream into
libndconv.so; torch provides device memory and streams, nothing else.
"""
import torch

from . import _native
from ._native import (NDC_F32, NDC_F64, NDC_PREC_BF16, NDC_PREC_NATIVE, NDC_PREC_SPLIT_BF16, NdcError,
                      check, i64_array, lib, strerror)

PRECISIONS = {"native": NDC_PREC_NATIVE, "fp32": NDC_PREC_NATIVE, "fp64": NDC_PREC_NATIVE,
              "bf16": NDC_PREC_BF16, "split_bf16": NDC_PREC_SPLIT_BF16}

__all__ = ["conv_full_nd", "conv_adjoint_nd", "conv_dH_nd", "deconv_iterate", "deconv_workspace_bytes",
           "deconv_workspace_bytes_ex", "rl_iterate", "richardson_lucy",
           "conv_full", "conv_adjoint", "deconv", "NdcError", "strerror", "PRECISIONS"]


def _dtype_code(t):
    if t.dtype == torch.float32:
        return NDC_F32
    if t.dtype == torch.float64:
        return NDC_F64
    raise TypeError("ndconv supports float32 and float64 tensors, got %s" % t.dtype)


def _prec(precision):
    if isinstance(precision, int):
        return precision
    try:
        return PRECISIONS[precision]
    except KeyError:
        raise ValueError("precision must be one of %s" % sorted(PRECISIONS)) from None


def _dev(t, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a GPU tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous (C order)" % name)
    return t


def _half_widths(h):
    p = []
    for e in h.shape:
        if e % 2 != 1:
            raise ValueError("PSF extents must be odd (2p+1), got %s" % (tuple(h.shape),))
        p.append((e - 1) // 2)
    return p


def _stream(stream):
    if stream is None:
        return ctypes_void(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes_void(stream.cuda_stream)
    return ctypes_void(int(stream))


def ctypes_void(v):
    import ctypes
    return ctypes.c_void_p(v)


def conv_full_nd(X, H, Y=None, precision="native", stream=None):
    """Y = X (x) H (Property 1, Eq. 4): extent m_i + 2p_i."""
    _dev(X, "X")
    _dev(H, "H")
    if X.dim() != H.dim() or H.dtype != X.dtype:
        raise ValueError("X and H must have the same rank and dtype")
    p = _half_widths(H)
    shape = [a + 2 * b for a, b in zip(X.shape, p)]
    if Y is None:
        Y = torch.empty(shape, dtype=X.dtype, device=X.device)
    _dev(Y, "Y")
    if list(Y.shape) != shape or Y.dtype != X.dtype:
        raise ValueError("Y must have shape %s and dtype %s" % (shape, X.dtype))
    check(lib.conv_full_nd(X.dim(), i64_array(X.shape), i64_array(p), X.data_ptr(), H.data_ptr(), Y.data_ptr(),
                           _dtype_code(X), _prec(precision), _stream(stream)), "conv_full_nd")
    return Y


def conv_adjoint_nd(R, H, X=None, precision="native", stream=None):
    """(A^h)^T R = M_{2p}(R (x) H~) (Property 2, Eq. 2): extent r_i - 2p_i."""
    _dev(R, "R")
    _dev(H, "H")
    if R.dim() != H.dim() or H.dtype != R.dtype:
        raise ValueError("R and H must have the same rank and dtype")
    p = _half_widths(H)
    m = [a - 2 * b for a, b in zip(R.shape, p)]
    if min(m) < 1:
        raise ValueError("R must exceed the PSF's 2p on every axis")
    if X is None:
        X = torch.empty(m, dtype=R.dtype, device=R.device)
    _dev(X, "X")
    if list(X.shape) != m or X.dtype != R.dtype:
        raise ValueError("X must have shape %s and dtype %s" % (m, R.dtype))
    check(lib.conv_adjoint_nd(R.dim(), i64_array(m), i64_array(p), R.data_ptr(), H.data_ptr(), X.data_ptr(),
                              _dtype_code(R), _prec(precision), _stream(stream)), "conv_adjoint_nd")
    return X


def conv_dH_nd(X, G, psf_shape, dH=None, stream=None):
    """dH[j] = sum_k X[k] G[k+j]: gradient of 1/2||X(x)H - Y||^2 in H for the
    residual G, extent psf_shape (2p+1 per axis)."""
    _dev(X, "X")
    _dev(G, "G")
    p = []
    for e in psf_shape:
        if e % 2 != 1:
            raise ValueError("PSF extents must be odd")
        p.append((e - 1) // 2)
    if list(G.shape) != [a + 2 * b for a, b in zip(X.shape, p)] or G.dtype != X.dtype:
        raise ValueError("G must have extent m+2p and X's dtype")
    if dH is None:
        dH = torch.empty(list(psf_shape), dtype=X.dtype, device=X.device)
    _dev(dH, "dH")
    n, mm, pp, dt = X.dim(), i64_array(X.shape), i64_array(p), _dtype_code(X)
    nbytes = lib.conv_dH_workspace_bytes(n, mm, pp, dt)
    ws = torch.empty(max(1, nbytes), dtype=torch.uint8, device=X.device)
    check(lib.conv_dH_nd(n, mm, pp, X.data_ptr(), G.data_ptr(), dH.data_ptr(), dt, ws.data_ptr(), nbytes,
                         _stream(stream)), "conv_dH_nd")
    return dH


def deconv_workspace_bytes(shape, psf_shape, dtype=torch.float32, precision="native"):
    p = [(e - 1) // 2 for e in psf_shape]
    dt = NDC_F64 if dtype == torch.float64 else NDC_F32
    return int(lib.deconv_workspace_bytes(len(shape), i64_array(shape), i64_array(p), dt, _prec(precision)))


def deconv_workspace_bytes_ex(shape, psf_shape, dtype=torch.float32, precision="native", regularised=1):
    """Workspace of deconv_iterate with the Laplacian term (mu > 0)."""
    p = [(e - 1) // 2 for e in psf_shape]
    dt = NDC_F64 if dtype == torch.float64 else NDC_F32
    return int(lib.deconv_workspace_bytes_ex(len(shape), i64_array(shape), i64_array(p), dt, _prec(precision),
                                             int(regularised)))


STEP_RULES = {"fixed": 0, "cauchy": 1, "bb": 2}


def _check_out_buffer(t, name, dtype, min_numel):
    """Caller-supplied device output of the deconvolution: checked before the
    library writes min_numel elements of `dtype` through its pointer."""
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch tensor" % name)
    if t.dtype != dtype:
        raise ValueError("%s must have dtype %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.numel() < min_numel:
        raise ValueError("%s needs at least %d elements, got %d" % (name, min_numel, t.numel()))
    if not t.is_cuda:
        raise TypeError("%s must be a GPU tensor" % name)


def deconv_iterate(Y, H, X, iters, lam=0.0, precision="native", ws=None, stats=None, info=None, stream=None,
                   rule="fixed", mu=0.0, max_trials=0):
    """Run `iters` accepted projected-gradient steps in place on X (Steps 1-3,
    delta accepted by f(X^{k+1}) < f(X^k)).  `rule` picks the first trial of
    each iteration: "fixed" (delta_0), "cauchy" or "bb"; `mu` weights the
    Laplacian (Tikhonov-Miller) term mu/2 ||L X||^2; `max_trials` bounds the
    trial slots the call enqueues (0: 2*iters + 30; see ndconv.h).  Nothing
    waits on the host.  Returns (X, stats, info) with stats (iters+1, 4)
    float64 and info (2,) int32 = (iters_done, status) on the device."""
    if rule not in STEP_RULES:
        raise ValueError("rule must be one of %s" % sorted(STEP_RULES))
    iters, max_trials = int(iters), int(max_trials)
    if not 0 <= iters <= _native.NDC_MAX_ITERS:
        raise ValueError("iters must be in [0, %d]" % _native.NDC_MAX_ITERS)
    for t, nm in ((Y, "Y"), (H, "H"), (X, "X")):
        _dev(t, nm)
    if not (Y.dtype == H.dtype == X.dtype):
        raise ValueError("Y, H and X must share a dtype")
    p = _half_widths(H)
    if list(Y.shape) != [a + 2 * b for a, b in zip(X.shape, p)]:
        raise ValueError("Y must have extent m+2p")
    n, mm, pp, dt, pr = X.dim(), i64_array(X.shape), i64_array(p), _dtype_code(X), _prec(precision)
    need = lib.deconv_workspace_bytes_ex(n, mm, pp, dt, pr, 1 if mu > 0 else 0)
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=X.device)
    _check_out_buffer(ws, "ws", torch.uint8, need)
    if stats is None:
        stats = torch.full((iters + 1, 4), float("nan"), dtype=torch.float64, device=X.device)
    _check_out_buffer(stats, "stats", torch.float64, 4 * (iters + 1))
    if info is None:
        info = torch.zeros(2, dtype=torch.int32, device=X.device)
    _check_out_buffer(info, "info", torch.int32, 2)
    if rule == "fixed" and mu == 0 and max_trials == 0:
        check(lib.deconv_iterate(n, mm, pp, Y.data_ptr(), H.data_ptr(), X.data_ptr(), iters, float(lam), dt, pr,
                                 ws.data_ptr(), ws.numel() * ws.element_size(), stats.data_ptr(), info.data_ptr(),
                                 _stream(stream)), "deconv_iterate")
    else:
        check(lib.deconv_iterate_ex(n, mm, pp, Y.data_ptr(), H.data_ptr(), X.data_ptr(), iters, float(lam),
                                    float(mu), dt, pr, STEP_RULES[rule], max_trials, ws.data_ptr(),
                                    ws.numel() * ws.element_size(), stats.data_ptr(), info.data_ptr(),
                                    _stream(stream)), "deconv_iterate_ex")
    return X, stats, info


def rl_iterate(Y, H, X, iters, precision="native", ws=None, stats=None, info=None, stream=None):
    """`iters` Richardson-Lucy iterations in place on X (rl_iterate in
    ndconv.h): X <- X * A^T(Y / A X) / sum H.  Nothing waits on the host.
    Returns (X, stats, info): stats (iters+1,) float64 = D(Y || A X^k),
    info (2,) int32 = (last k recorded, status) on the device."""
    iters = int(iters)
    if not 0 <= iters <= _native.NDC_MAX_ITERS:
        raise ValueError("iters must be in [0, %d]" % _native.NDC_MAX_ITERS)
    for t, nm in ((Y, "Y"), (H, "H"), (X, "X")):
        _dev(t, nm)
    if not (Y.dtype == H.dtype == X.dtype):
        raise ValueError("Y, H and X must share a dtype")
    p = _half_widths(H)
    if list(Y.shape) != [a + 2 * b for a, b in zip(X.shape, p)]:
        raise ValueError("Y must have extent m+2p")
    n, mm, pp, dt, pr = X.dim(), i64_array(X.shape), i64_array(p), _dtype_code(X), _prec(precision)
    need = lib.rl_workspace_bytes(n, mm, pp, dt, pr)
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=X.device)
    _check_out_buffer(ws, "ws", torch.uint8, need)
    if stats is None:
        stats = torch.full((iters + 1,), float("nan"), dtype=torch.float64, device=X.device)
    _check_out_buffer(stats, "stats", torch.float64, iters + 1)
    if info is None:
        info = torch.zeros(2, dtype=torch.int32, device=X.device)
    _check_out_buffer(info, "info", torch.int32, 2)
    check(lib.rl_iterate(n, mm, pp, Y.data_ptr(), H.data_ptr(), X.data_ptr(), iters, dt, pr, ws.data_ptr(),
                         ws.numel() * ws.element_size(), stats.data_ptr(), info.data_ptr(), _stream(stream)),
          "rl_iterate")
    return X, stats, info


# Friendlier names ------------------------------------------------------------
def conv_full(x, h, precision="native"):
    return conv_full_nd(x.contiguous(), h.contiguous(), precision=precision)


def conv_adjoint(r, h, precision="native"):
    return conv_adjoint_nd(r.contiguous(), h.contiguous(), precision=precision)


def deconv(y, h, x0=None, iters=100, lam=0.0, precision="native", rule="fixed", mu=0.0, max_trials=0):
    """Projected-gradient deconvolution; x0 defaults to the flux-matching flat
    start max(sum Y, 0)/(N sum H).  Returns (x, stats, info)."""
    y, h = y.contiguous(), h.contiguous()
    p = _half_widths(h)
    m = [a - 2 * b for a, b in zip(y.shape, p)]
    if x0 is None:
        n = 1
        for v in m:
            n *= v
        val = torch.clamp(y.sum(dtype=torch.float64), min=0) / (n * h.sum(dtype=torch.float64))
        x = torch.empty(m, dtype=y.dtype, device=y.device)
        x.fill_(float(val))
    else:
        x = x0.clone().contiguous()
    return deconv_iterate(y, h, x, iters, lam=lam, precision=precision, rule=rule, mu=mu, max_trials=max_trials)


def richardson_lucy(y, h, x0=None, iters=100, precision="native"):
    """Richardson-Lucy deconvolution; x0 defaults to the flux-matching flat
    start max(sum Y, 0)/(N sum H).  Returns (x, stats, info)."""
    y, h = y.contiguous(), h.contiguous()
    p = _half_widths(h)
    m = [a - 2 * b for a, b in zip(y.shape, p)]
    if x0 is None:
        n = 1
        for v in m:
            n *= v
        val = torch.clamp(y.sum(dtype=torch.float64), min=0) / (n * h.sum(dtype=torch.float64))
        x = torch.empty(m, dtype=y.dtype, device=y.device)
        x.fill_(float(val))
    else:
        x = x0.clone().contiguous()
    return rl_iterate(y, h, x, iters, precision=precision)
