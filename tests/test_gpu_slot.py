"""The row-slot tiles (NDC_FORM_SLOT, installed per problem through the
override table), bf16 and FP32: oracle parity (bf16 on bf16-rounded
operands, where only the FP32 summation order differs from the FP64
oracle) on shapes that reach every split of the PSF planes between the
waves (1..16 planes per wave), both tap-chunk counts, 31 of 32 row slots in
use, columns shared between work-groups, ragged x and z tails, 1-D and 2-D
problems; run-to-run determinism; the deconvolution's and Richardson-Lucy's
epilogues on the form; and the metric workload on sampled outputs."""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def at():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1711_11224_amd as nd  # noqa: F401
    from paper_1711_11224_amd import autotune
    yield autotune
    nd.lib.ndc_tile_override_clear()


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def bf16(a):
    """Round to bfloat16 (nearest even) and back, as the kernels do."""
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(torch.bfloat16).to(torch.float32).numpy()


def install(at, m, k, prec="bf16", form="slot"):
    for op in at.OPS:
        at.set_form(m, k, op, form, 0, prec)
        assert at.current_form(m, k, op, prec) == (form, 0)


def clear(at, m, k, prec="bf16"):
    for op in at.OPS:
        at.set_form(m, k, op, "auto", 0, prec)


PRECS = ["bf16", "fp32"]


# (m, PSF extents): PSF planes per wave / passes / tap chunks noted
CASES = [((20, 40, 45), (63, 3, 5)),     # 8 per wave in two passes of 4 (edge tiles 1..7), 1 chunk
         ((30, 33, 70), (35, 31, 21)),   # 5 per wave: two passes of 3; ky = 31; 2 chunks
         ((40, 60, 33), (41, 9, 11)),    # 6 per wave: two passes of 3; ragged x tile
         ((7, 100, 40), (13, 31, 31)),   # many columns split between work-groups; 31 x 31 rows
         ((11, 23, 97), (27, 15, 31)),   # 4 per wave, one pass; z tail of 5 planes
         ((3, 64, 64), (5, 7, 17)),      # fewer planes than one tile; 17 taps = 2 chunks
         ((200, 300), (31, 31)),         # 2-D: one PSF plane, one output plane of eight
         ((1000,), (31,)),               # 1-D
         ((9, 17, 31), (1, 1, 1))]       # one tap


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("m,k", CASES)
def test_slot_matches_oracle_on_rounded_operands(at, m, k, prec):
    import paper_1711_11224_amd as nd
    say("case slot m=%s k=%s %s" % (m, k, prec))
    rng = np.random.default_rng(synth.stable_seed(m, k))
    x = rng.random(m).astype(np.float32)
    h = rng.standard_normal(k).astype(np.float32)
    r = rng.standard_normal([a + b - 1 for a, b in zip(m, k)]).astype(np.float32)
    # operands as the kernel multiplies them
    xb, hb, rb = (bf16(x), bf16(h), bf16(r)) if prec == "bf16" else (x, h, r)
    install(at, m, k, prec)
    try:
        xt, ht, rt = (torch.from_numpy(v).cuda() for v in (x, h, r))
        y = nd.conv_full_nd(xt, ht, precision=prec)
        g = nd.conv_adjoint_nd(rt, ht, precision=prec)
        y2 = nd.conv_full_nd(xt, ht, precision=prec)
        g2 = nd.conv_adjoint_nd(rt, ht, precision=prec)
        torch.cuda.synchronize()
    finally:
        clear(at, m, k, prec)
    assert torch.equal(y, y2) and torch.equal(g, g2)  # deterministic summation order
    y, g = y.cpu().numpy(), g.cpu().numpy()
    # exact up to FP32 accumulation against the operands as multiplied ...
    assert rel_l2(y, oracle.conv_full(xb, hb)) <= 1e-5
    assert rel_l2(g, oracle.conv_adjoint(rb, hb)) <= 1e-5
    # ... and within the precision's tolerance of the unrounded operator
    tol = 1e-2 if prec == "bf16" else 1e-5
    assert rel_l2(y, oracle.conv_full(x, h)) <= tol
    assert rel_l2(g, oracle.conv_adjoint(r, h)) <= tol


@pytest.mark.parametrize("prec", PRECS)
def test_slot_deconvolution_and_richardson_lucy(at, prec):
    """Five projected-gradient steps (residual, update, gradient and norm
    epilogues; Cauchy first trials) and five Richardson-Lucy steps
    (quotient and multiplicative epilogues) with the form installed, against
    the FP64 oracle at the bound the deconvolution tests use for the
    precision (5e-2 bf16, 1e-4 FP32)."""
    import paper_1711_11224_amd as nd
    say("case slot deconvolution %s" % prec)
    tol = 5e-2 if prec == "bf16" else 1e-4
    rng = np.random.default_rng(23)
    m, k = (10, 44, 70), (9, 11, 21)
    h = rng.random(k).astype(np.float32) + 0.1
    h /= h.sum()
    xt = rng.random(m)
    y = (oracle.conv_full(xt, h) + 0.01 * rng.standard_normal([a + b - 1 for a, b in zip(m, k)])).astype(np.float32)
    x0 = np.full(m, float(xt.mean()), dtype=np.float32)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    install(at, m, k, prec)
    try:
        xg, st, info = nd.deconv_iterate(dev(y), dev(h), dev(x0), 5, lam=0.01, precision=prec, rule="cauchy")
        xr = dev(x0)
        _, rs, rinfo = nd.rl_iterate(dev(np.maximum(y, 0)), dev(h), xr, 5, precision=prec)
        torch.cuda.synchronize()
    finally:
        clear(at, m, k, prec)
    xo, so, done, status = oracle.deconv(y.astype(np.float64), h.astype(np.float64), x0.astype(np.float64), 5,
                                         lam=0.01, rule="cauchy")
    assert info.cpu().tolist() == [5, 0] and (done, status) == (5, 0)
    f = st.cpu().numpy()[:, 0]
    assert np.all(np.diff(f) < 0)
    assert np.all(np.abs(f - so[:, 0]) <= tol * np.abs(so[:, 0]))
    assert rel_l2(xg.cpu().numpy(), xo) <= tol
    xro, dro = oracle.richardson_lucy(np.maximum(y, 0).astype(np.float64), h.astype(np.float64),
                                      x0.astype(np.float64), 5)
    assert rinfo.cpu().tolist()[1] == 0
    assert rel_l2(xr.cpu().numpy(), xro) <= tol
    assert np.all(np.abs(rs.cpu().numpy() - dro) <= tol * np.abs(dro))


@pytest.mark.parametrize("prec", PRECS)
def test_slot_metric_workload_sampled(at, prec):
    """X 128x512x512, PSF 63x31x31 with the form installed: 2048 sampled
    outputs of each operator against the oracle (bf16: on bf16-rounded
    operands)."""
    import paper_1711_11224_amd as nd
    cfg = synth.CONFIGS["c3_metric"]
    m, k = tuple(cfg.shape), tuple(cfg.psf_shape)
    say("case slot metric %s" % prec)
    rnd = bf16 if prec == "bf16" else (lambda a: a)
    x = synth.make_objects(cfg).astype(np.float32)
    h = synth.psf_for(cfg).astype(np.float32)
    rng = np.random.default_rng(7)
    r = rng.standard_normal([a + b - 1 for a, b in zip(m, k)]).astype(np.float32)
    iy = rng.choice(r.size, 2048, replace=False)
    ix = rng.choice(x.size, 2048, replace=False)
    install(at, m, k, prec)
    try:
        y = nd.conv_full_nd(torch.from_numpy(x).cuda(), torch.from_numpy(h).cuda(), precision=prec)
        ys = y.view(-1)[torch.from_numpy(iy).cuda()].cpu().numpy()
        del y
        g = nd.conv_adjoint_nd(torch.from_numpy(r).cuda(), torch.from_numpy(h).cuda(), precision=prec)
        gs = g.view(-1)[torch.from_numpy(ix).cuda()].cpu().numpy()
        del g
    finally:
        clear(at, m, k, prec)
    assert rel_l2(ys, oracle.conv_full_at(rnd(x), rnd(h), iy)) <= 1e-5
    assert rel_l2(gs, oracle.conv_adjoint_at(rnd(r), rnd(h), ix)) <= 1e-5
