"""Batched form: many independent 3-D volumes with their own extents and
PSFs through persistent launches and a hipGraph-captured deconvolution step
(C ABI ndc_batch_*).  Marshalling only."""
import ctypes

import torch

from ._native import check, i64_array, lib


def _ptrs(tensors):
    arr = (ctypes.c_void_p * len(tensors))(*[t.data_ptr() for t in tensors])
    return arr


class BatchPlan:
    """A plan for `shapes[v]` = (z, y, x) extents of X and `psf_shapes[v]` =
    odd PSF extents.  tuning: None or (planes per tile 2|4, or 0 for the
    deconvolution on each volume's own kernels; work-groups per CU 1|2,
    order 0|1|2, use_graph 0|1)."""

    def __init__(self, shapes, psf_shapes, tuning=None):
        if len(shapes) != len(psf_shapes) or not shapes:
            raise ValueError("need one PSF shape per volume")
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.psf_shapes = [tuple(int(v) for v in s) for s in psf_shapes]
        for s, h in zip(self.shapes, self.psf_shapes):
            if len(s) != 3 or len(h) != 3 or any(e % 2 != 1 for e in h):
                raise ValueError("3-D volumes with odd PSF extents expected")
        self.half = [tuple((e - 1) // 2 for e in h) for h in self.psf_shapes]
        m = i64_array([v for s in self.shapes for v in s])
        p = i64_array([v for s in self.half for v in s])
        tun = None if tuning is None else (ctypes.c_int * 4)(*[int(v) for v in tuning])
        self.tuning = None if tuning is None else tuple(int(v) for v in tuning)
        handle = ctypes.c_void_p()
        check(lib.ndc_batch_plan_create(len(self.shapes), m, p, 0, 0, tun, ctypes.byref(handle)),
              "ndc_batch_plan_create")
        self._h = handle
        info = i64_array([0, 0, 0, 0])
        check(lib.ndc_batch_plan_info(self._h, info), "ndc_batch_plan_info")
        self.forward_tiles, self.transpose_tiles, self.grid, self.lds_bytes = [int(v) for v in info]
        self.workspace_bytes = int(lib.ndc_batch_workspace_bytes(self._h))
        self._ws = None

    def close(self):
        if getattr(self, "_h", None):
            lib.ndc_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _check_list(self, ts, shapes, name):
        if len(ts) != len(self.shapes):
            raise ValueError("%s: one tensor per volume" % name)
        for t, s in zip(ts, shapes):
            if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous() or tuple(t.shape) != tuple(s):
                raise ValueError("%s: contiguous float32 GPU tensors of shape %s expected" % (name, s))

    def _yshapes(self):
        return [tuple(a + 2 * b for a, b in zip(s, p)) for s, p in zip(self.shapes, self.half)]

    def conv_full(self, xs, hs, ys=None, stream=None):
        self._check_list(xs, self.shapes, "X")
        self._check_list(hs, self.psf_shapes, "H")
        ys = ys or [torch.empty(s, device=xs[0].device) for s in self._yshapes()]
        st = torch.cuda.current_stream().cuda_stream if stream is None else stream
        check(lib.ndc_batch_conv_full(self._h, _ptrs(xs), _ptrs(hs), _ptrs(ys), ctypes.c_void_p(st)),
              "ndc_batch_conv_full")
        return ys

    def conv_adjoint(self, rs, hs, xs=None, stream=None):
        self._check_list(rs, self._yshapes(), "R")
        self._check_list(hs, self.psf_shapes, "H")
        xs = xs or [torch.empty(s, device=rs[0].device) for s in self.shapes]
        st = torch.cuda.current_stream().cuda_stream if stream is None else stream
        check(lib.ndc_batch_conv_adjoint(self._h, _ptrs(rs), _ptrs(hs), _ptrs(xs), ctypes.c_void_p(st)),
              "ndc_batch_conv_adjoint")
        return xs

    def deconv(self, ys, hs, xs, iters, lam=0.0, stream=None):
        """`iters` accepted projected-gradient steps on every volume, X in
        place.  Returns (xs, stats list of (iters+1, 4), info (count, 2))."""
        self._check_list(ys, self._yshapes(), "Y")
        self._check_list(hs, self.psf_shapes, "H")
        self._check_list(xs, self.shapes, "X")
        dev = xs[0].device
        if self._ws is None or self._ws.device != dev:
            self._ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=dev)
        stats = [torch.full((iters + 1, 4), float("nan"), dtype=torch.float64, device=dev) for _ in xs]
        info = torch.zeros((len(xs), 2), dtype=torch.int32, device=dev)
        st = torch.cuda.current_stream().cuda_stream if stream is None else stream
        check(lib.ndc_batch_deconv(self._h, _ptrs(ys), _ptrs(hs), _ptrs(xs), int(iters), float(lam),
                                   ctypes.c_void_p(self._ws.data_ptr()), self._ws.numel(), _ptrs(stats),
                                   ctypes.c_void_p(info.data_ptr()), ctypes.c_void_p(st)), "ndc_batch_deconv")
        return xs, stats, info


def plan_for(shapes, psf_shapes, tuning="auto", table=None):
    """A BatchPlan whose tuning comes from the autotuner's table (tuning the
    batch first if the table has no entry for it) or is given explicitly;
    with "auto" the volumes' stored kernel forms are installed first, so the
    plan's per-volume kernels are the tuned ones."""
    if tuning == "auto":
        from .autotune import best_tuning, install_batch_forms
        tuning = best_tuning(shapes, psf_shapes, table=table)
        install_batch_forms(shapes, psf_shapes, table=table)
    return BatchPlan(shapes, psf_shapes, tuning=tuning)
