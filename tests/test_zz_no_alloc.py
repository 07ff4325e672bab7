"""conv_dH_nd_noalloc (the PSF gradient with the library's own scratch
array, for callers that cannot allocate) against conv_dH_nd with a caller
workspace: the same kernels in the same order, so the results must agree
bit for bit, on two calls in a row (the second smaller, reusing the array)
in both storage types."""
import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1711_11224_amd as m
    return m


def _run(nd, x, g, psf, noalloc):
    lib = nd.lib
    p = [(e - 1) // 2 for e in psf]
    mm, pp = nd.i64_array(x.shape), nd.i64_array(p)
    dt = 1 if x.dtype == torch.float64 else 0
    dh = torch.full(psf, float("nan"), dtype=x.dtype, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if noalloc:
        rc = lib.conv_dH_nd_noalloc(x.dim(), mm, pp, x.data_ptr(), g.data_ptr(), dh.data_ptr(), dt, st)
    else:
        nb = lib.conv_dH_workspace_bytes(x.dim(), mm, pp, dt)
        ws = torch.empty(max(1, nb), dtype=torch.uint8, device="cuda")
        rc = lib.conv_dH_nd(x.dim(), mm, pp, x.data_ptr(), g.data_ptr(), dh.data_ptr(), dt, ws.data_ptr(), nb, st)
    assert rc == 0, nd.strerror(rc)
    torch.cuda.synchronize()
    return dh


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_dH_equals_workspace_dH(nd, dtype):
    rng = np.random.default_rng(71)
    # the differentiable workload's shape, then a smaller ragged one
    for m, psf in (((64, 256, 256), (41, 21, 21)), ((9, 37, 70), (5, 7, 9))):
        print("case noalloc dH m=%s psf=%s %s" % (m, psf, dtype), file=sys.stderr, flush=True)
        gshape = [a + b - 1 for a, b in zip(m, psf)]
        x = torch.from_numpy(rng.random(m)).to(dtype).cuda()
        g = torch.from_numpy(rng.standard_normal(gshape)).to(dtype).cuda()
        a = _run(nd, x, g, psf, noalloc=False)
        b = _run(nd, x, g, psf, noalloc=True)
        assert not torch.isnan(b).any()
        assert torch.equal(a, b)


def test_noalloc_dH_rejects_oversized_partials(nd):
    """A problem whose split-K partials exceed the array is refused before
    anything is enqueued; the output stays untouched."""
    m, psf = (160, 512, 512), (63, 31, 31)
    p = [(e - 1) // 2 for e in psf]
    need = nd.lib.conv_dH_workspace_bytes(3, nd.i64_array(m), nd.i64_array(p), 0)
    assert need > nd._native.NDC_DH_SCRATCH_BYTES
    x = torch.zeros(m, device="cuda")
    g = torch.zeros([a + b - 1 for a, b in zip(m, psf)], device="cuda")
    dh = torch.full(psf, 7.0, device="cuda")
    rc = nd.lib.conv_dH_nd_noalloc(3, nd.i64_array(m), nd.i64_array(p), x.data_ptr(), g.data_ptr(), dh.data_ptr(),
                                   0, None)
    assert rc == nd._native.NDC_EWORKSPACE
    torch.cuda.synchronize()
    assert bool((dh == 7.0).all())
