"""C-ABI checks that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

from tests.conftest import ROOT

nd = pytest.importorskip("paper_1711_11224_amd._native", exc_type=ImportError)
lib = nd.lib
I = nd.i64_array
F32, F64 = nd.NDC_F32, nd.NDC_F64


def header_symbols():
    src = open(os.path.join(ROOT, "include", "ndconv.h")).read()
    src = src.split("extern \"C\" {", 1)[1]
    return re.findall(r"NDC_API\s+[\w\s\*]*?\b(\w+)\s*\(", src)


def test_exports_every_header_symbol():
    syms = header_symbols()
    assert set(syms) == set(nd.EXPORTS)
    for s in syms:
        assert hasattr(lib, s), s


def test_version_and_strerror():
    assert lib.ndc_version() >> 16 == 1
    for code in (0, -1, -2, -3, -4, -5, -6, 99):
        assert isinstance(nd.strerror(code), str) and nd.strerror(code)
    assert nd.strerror(99) == "unknown status"


def _full(n, m, p, X=0x1000, H=0x100000, Y=0x10000000, dt=F32, pr=0):
    return lib.conv_full_nd(n, I(m), I(p), ctypes.c_void_p(X), ctypes.c_void_p(H), ctypes.c_void_p(Y), dt, pr, None)


def _adj(n, m, p, R=0x1000, H=0x100000000, X=0x10000000, dt=F32, pr=0):
    return lib.conv_adjoint_nd(n, I(m), I(p), ctypes.c_void_p(R), ctypes.c_void_p(H), ctypes.c_void_p(X), dt, pr,
                               None)


@pytest.mark.parametrize("fn", [_full, _adj])
def test_rank_extent_and_halfwidth_checks(fn):
    assert fn(0, [4], [1]) == nd.NDC_EINVAL
    assert fn(4, [2, 2, 2, 2], [0, 0, 0, 0]) == nd.NDC_EUNSUPPORTED
    assert fn(2, [0, 4], [1, 1]) == nd.NDC_EINVAL
    assert fn(2, [4, 4], [1, -1]) == nd.NDC_EINVAL
    assert fn(1, [1 << 30], [0]) == nd.NDC_EUNSUPPORTED


@pytest.mark.parametrize("fn", [_full, _adj])
def test_dtype_precision_checks(fn):
    assert fn(2, [4, 4], [1, 1], dt=7) == nd.NDC_EINVAL
    assert fn(2, [4, 4], [1, 1], pr=9) == nd.NDC_EINVAL
    assert fn(2, [4, 4], [1, 1], dt=F64, pr=nd.NDC_PREC_BF16) == nd.NDC_EUNSUPPORTED
    assert fn(2, [4, 4], [1, 1], dt=F64, pr=nd.NDC_PREC_SPLIT_BF16) == nd.NDC_EUNSUPPORTED


def test_null_and_alias_checks():
    assert _full(2, [4, 4], [1, 1], X=0) == nd.NDC_EINVAL
    assert _full(2, [4, 4], [1, 1], H=0) == nd.NDC_EINVAL
    assert _full(2, [4, 4], [1, 1], Y=0) == nd.NDC_EINVAL
    # Y (6x6 floats = 144 B) overlapping X
    assert _full(2, [4, 4], [1, 1], X=0x1000, Y=0x1000 + 32) == nd.NDC_EALIAS  # X is 64 B
    # Y overlapping H
    assert _full(2, [4, 4], [1, 1], H=0x2000, Y=0x2000 - 100) == nd.NDC_EALIAS
    assert _adj(2, [4, 4], [1, 1], R=0x1000, X=0x1000 + 140) == nd.NDC_EALIAS


def test_workspace_queries():
    assert lib.deconv_workspace_bytes(3, I([8, 9, 10]), I([1, 2, 3]), F32, 0) > 0
    assert lib.deconv_workspace_bytes(3, I([8, 9, 10]), I([1, 2, -3]), F32, 0) == 0
    assert lib.deconv_workspace_bytes(3, I([8, 9, 10]), I([1, 2, 3]), F64, nd.NDC_PREC_BF16) == 0
    a = lib.deconv_workspace_bytes(3, I([8, 9, 10]), I([1, 2, 3]), F32, 0)
    b = lib.deconv_workspace_bytes(3, I([8, 9, 10]), I([1, 2, 3]), F64, 0)
    assert b > a  # double buffers
    assert lib.conv_dH_workspace_bytes(3, I([8, 9, 10]), I([1, 2, 3]), F32) >= 0


def _deconv(iters=3, lam=0.0, ws=0x40000000, wsb=None, stats=0, info=0, X=0x1000):
    m, p = [4, 5, 6], [1, 1, 1]
    need = lib.deconv_workspace_bytes(3, I(m), I(p), F32, 0)
    return lib.deconv_iterate(3, I(m), I(p), ctypes.c_void_p(0x10000000), ctypes.c_void_p(0x20000000),
                              ctypes.c_void_p(X), iters, lam, F32, 0, ctypes.c_void_p(ws),
                              need if wsb is None else wsb, ctypes.c_void_p(stats) if stats else None,
                              ctypes.c_void_p(info) if info else None, None)


def test_deconv_argument_checks():
    assert _deconv(iters=-1) == nd.NDC_EINVAL
    assert _deconv(lam=-1.0) == nd.NDC_EINVAL
    assert _deconv(lam=float("nan")) == nd.NDC_EINVAL
    assert _deconv(lam=float("inf")) == nd.NDC_EINVAL
    assert _deconv(ws=0) == nd.NDC_EWORKSPACE
    assert _deconv(wsb=16) == nd.NDC_EWORKSPACE
    assert _deconv(X=0) == nd.NDC_EINVAL
    # X overlapping the workspace, stats overlapping Y
    assert _deconv(X=0x40000000 + 8) == nd.NDC_EALIAS
    assert _deconv(stats=0x10000000 + 8) == nd.NDC_EALIAS


def test_dH_workspace_check():
    m, p = [16, 64, 64], [3, 4, 5]
    need = lib.conv_dH_workspace_bytes(3, I(m), I(p), F32)
    assert need > 0  # split-K partial outputs
    rc = lib.conv_dH_nd(3, I(m), I(p), ctypes.c_void_p(0x1000), ctypes.c_void_p(0x10000000),
                        ctypes.c_void_p(0x20000000), F32, None, 0, None)
    assert rc == nd.NDC_EWORKSPACE


def _plan(count, m, p, dt=F32, pr=0, tuning=None):
    h = ctypes.c_void_p()
    tun = None if tuning is None else (ctypes.c_int * 4)(*tuning)
    rc = lib.ndc_batch_plan_create(count, I(m), I(p), dt, pr, tun, ctypes.byref(h))
    return rc, h


def test_batch_plan_argument_checks():
    assert _plan(0, [4, 4, 4], [1, 1, 1])[0] == nd.NDC_EINVAL
    assert _plan(1, [4, 0, 4], [1, 1, 1])[0] == nd.NDC_EINVAL
    assert _plan(1, [4, 4, 4], [1, -1, 1])[0] == nd.NDC_EINVAL
    assert _plan(1, [4, 4, 4], [1, 1, 1], dt=F64)[0] == nd.NDC_EUNSUPPORTED
    assert _plan(1, [4, 4, 4], [1, 1, 1], pr=nd.NDC_PREC_BF16)[0] == nd.NDC_EUNSUPPORTED
    assert _plan(1, [4, 4, 4], [1, 1, 17])[0] == nd.NDC_EUNSUPPORTED  # 2p_x+1 = 35 > 33
    assert _plan(1, [4, 4, 4], [1, 1, 0])[0] == nd.NDC_EUNSUPPORTED   # 2p_x+1 = 1 < 3
    assert _plan(2, [4, 4, 4, 5, 5, 5], [1, 1, 1, 1, 17, 1])[0] == nd.NDC_EUNSUPPORTED
    assert _plan(1, [4, 4, 4], [1, 1, 1], tuning=[3, 2, 0, 1])[0] == nd.NDC_EINVAL
    assert _plan(1, [4, 4, 4], [1, 1, 1], tuning=[4, 3, 0, 1])[0] == nd.NDC_EINVAL
    assert _plan(1, [4, 4, 4], [1, 1, 1], tuning=[4, 2, 5, 1])[0] == nd.NDC_EINVAL
    assert lib.ndc_batch_plan_create(1, I([4, 4, 4]), I([1, 1, 1]), F32, 0, None, None) == nd.NDC_EINVAL
    assert lib.ndc_batch_workspace_bytes(None) == 0
    lib.ndc_batch_plan_destroy(None)  # no-op


def test_deconv_ex_rejects_bad_rule_or_weight():
    """An unknown step rule or a negative / non-finite Laplacian weight is
    refused before any pointer is looked at."""
    for rule, mu in ((7, 0.0), (0, -1.0), (1, float("nan")), (2, float("inf"))):
        rc = lib.deconv_iterate_ex(3, I([4, 4, 4]), I([1, 1, 1]), None, None, None, 1, 0.0, mu, F32, 0, rule, 0,
                                   None, 0, None, None, None)
        assert rc == -1


def test_deconv_rejects_iteration_and_trial_counts_out_of_range():
    """iters and max_trials are bounded (the schedule is enqueued up front);
    both are checked before any pointer is looked at."""
    big = nd.NDC_MAX_ITERS + 1
    for iters, trials in ((-1, 0), (big, 0), (1, -1), (1, 2 * nd.NDC_MAX_ITERS + 31)):
        rc = lib.deconv_iterate_ex(3, I([4, 4, 4]), I([1, 1, 1]), None, None, None, iters, 0.0, 0.0, F32, 0, 0,
                                   trials, None, 0, None, None, None)
        assert rc == -1
    assert lib.deconv_iterate(3, I([4, 4, 4]), I([1, 1, 1]), None, None, None, big, 0.0, F32, 0, None, 0, None,
                              None, None) == -1


def test_deconv_binding_checks_caller_buffers():
    """The binding refuses stats / info / workspace tensors of the wrong
    dtype, layout or size before the library could write past them."""
    import torch
    from paper_1711_11224_amd import _check_out_buffer
    with pytest.raises(ValueError):
        _check_out_buffer(torch.zeros(8, dtype=torch.float32), "stats", torch.float64, 8)
    with pytest.raises(ValueError):
        _check_out_buffer(torch.zeros(7, dtype=torch.float64), "stats", torch.float64, 8)
    with pytest.raises(ValueError):
        _check_out_buffer(torch.zeros((4, 4), dtype=torch.float64).t(), "stats", torch.float64, 8)
    with pytest.raises(ValueError):
        _check_out_buffer(torch.zeros(2, dtype=torch.int64), "info", torch.int32, 2)
    with pytest.raises(ValueError):
        _check_out_buffer(torch.zeros(1, dtype=torch.int32), "info", torch.int32, 2)
    with pytest.raises(TypeError):
        _check_out_buffer(None, "info", torch.int32, 2)
    with pytest.raises(TypeError):  # right dtype and size, but host memory
        _check_out_buffer(torch.zeros(2, dtype=torch.int32), "info", torch.int32, 2)


def test_deconv_workspace_grows_with_the_laplacian_term():
    m, p = I([8, 9, 10]), I([1, 2, 3])
    base = lib.deconv_workspace_bytes(3, m, p, F32, 0)
    assert lib.deconv_workspace_bytes_ex(3, m, p, F32, 0, 0) == base
    # two (m+2)-extent arrays and one X-sized array at least
    assert lib.deconv_workspace_bytes_ex(3, m, p, F32, 0, 1) >= base + 4 * (2 * 10 * 11 * 12 + 8 * 9 * 10)


def test_tile_override_checks_and_table():
    """The kernel-form override: bad operator or form -> NDC_EINVAL, a form
    that cannot run the problem -> NDC_EUNSUPPORTED; installed choices are
    reported back by ndc_tile_choice and removed by NDC_FORM_AUTO / clear."""
    m, p = I([128, 512, 512]), I([31, 15, 15])
    out = (ctypes.c_int * 2)()
    assert lib.ndc_tile_override(3, m, p, F32, 0, 2, nd.NDC_FORM_MFMA4, 8) == nd.NDC_EINVAL
    assert lib.ndc_tile_override(3, m, p, F32, 0, 0, 9, 0) == nd.NDC_EINVAL
    assert lib.ndc_tile_override(3, m, p, F32, 0, 0, nd.NDC_FORM_SMALL, 0) == nd.NDC_EUNSUPPORTED  # 63x31x31 taps
    assert lib.ndc_tile_override(3, m, p, F32, 0, 0, nd.NDC_FORM_MFMA4, 12) == nd.NDC_EUNSUPPORTED
    assert lib.ndc_tile_override(3, m, p, F32, 0, 0, nd.NDC_FORM_MFMA32, 3) == nd.NDC_EUNSUPPORTED  # FP32 storage, native
    assert lib.ndc_tile_override(3, m, p, F32, nd.NDC_PREC_SPLIT_BF16, 1, nd.NDC_FORM_MFMA32, 4) == nd.NDC_EUNSUPPORTED
    assert lib.ndc_tile_choice(3, m, p, F32, 0, 0, out) == 0 and list(out) == [nd.NDC_FORM_MFMA4, 8]
    assert lib.ndc_tile_override(3, m, p, F32, 0, 0, nd.NDC_FORM_MFMA4, 16) == 0
    assert lib.ndc_tile_choice(3, m, p, F32, 0, 0, out) == 0 and list(out) == [nd.NDC_FORM_MFMA4, 16]
    assert lib.ndc_tile_choice(3, m, p, F32, 0, 1, out) == 0 and list(out) == [nd.NDC_FORM_MFMA4, 8]  # other operator
    assert lib.ndc_tile_override(3, m, p, F32, 0, 0, nd.NDC_FORM_AUTO, 0) == 0
    assert lib.ndc_tile_choice(3, m, p, F32, 0, 0, out) == 0 and list(out) == [nd.NDC_FORM_MFMA4, 8]
    assert lib.ndc_tile_override(3, m, p, F32, nd.NDC_PREC_BF16, 1, nd.NDC_FORM_MFMA32, 3) == 0
    assert lib.ndc_tile_choice(3, m, p, F32, nd.NDC_PREC_BF16, 1, out) == 0 and list(out) == [nd.NDC_FORM_MFMA32, 3]
    # the row-slot tiles: bf16 and FP32 native (not split-bf16, not FP64),
    # PSF planes <= 64, rows and taps <= 32
    assert lib.ndc_tile_override(3, m, p, nd.NDC_F64, 0, 0, nd.NDC_FORM_SLOT, 0) == nd.NDC_EUNSUPPORTED
    assert lib.ndc_tile_override(3, m, p, F32, nd.NDC_PREC_SPLIT_BF16, 0, nd.NDC_FORM_SLOT, 0) == nd.NDC_EUNSUPPORTED
    assert lib.ndc_tile_override(3, m, p, F32, 0, 0, nd.NDC_FORM_SLOT, 0) == 0
    assert lib.ndc_tile_choice(3, m, p, F32, 0, 0, out) == 0 and list(out) == [nd.NDC_FORM_SLOT, 0]
    assert lib.ndc_tile_override(3, m, p, F32, 0, 0, nd.NDC_FORM_AUTO, 0) == 0
    assert lib.ndc_tile_override(3, m, p, F32, nd.NDC_PREC_BF16, 0, nd.NDC_FORM_SLOT, 0) == 0
    assert lib.ndc_tile_choice(3, m, p, F32, nd.NDC_PREC_BF16, 0, out) == 0 and list(out) == [nd.NDC_FORM_SLOT, 0]
    assert lib.ndc_tile_override(3, m, nd.i64_array([32, 15, 15]), F32, nd.NDC_PREC_BF16, 0, nd.NDC_FORM_SLOT,
                                 0) == nd.NDC_EUNSUPPORTED  # 65 PSF planes
    assert lib.ndc_tile_override(3, m, p, F32, 0, 0, nd.NDC_FORM_SLOT + 1, 0) == nd.NDC_EINVAL
    lib.ndc_tile_override_clear()
    # the built-in rule: the row-slot tile for PSFs this large in bf16
    assert lib.ndc_tile_choice(3, m, p, F32, nd.NDC_PREC_BF16, 1, out) == 0 and list(out) == [nd.NDC_FORM_SLOT, 0]
    assert lib.ndc_tile_choice(3, m, p, F32, nd.NDC_PREC_SPLIT_BF16, 1, out) == 0 and list(out) == [nd.NDC_FORM_MFMA32, 2]
