"""GPU parity: every entry point of the C ABI against the FP64 oracle on the
same seeded inputs.  Tolerances are relative L2 errors: 1e-5 for FP32,
1e-12 for FP64, 1e-2 for bf16 and 1e-4 for split-bf16 operands; shapes and
crop extents must match exactly."""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "fp64": 1e-12, "bf16": 1e-2, "split_bf16": 1e-4}


@pytest.fixture(scope="module")
def nd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1711_11224_amd as m
    return m


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (den if den > 0 else 1.0)


def gpu(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


# Shapes spanning several tiles, ragged tails, 2p >= m, unit extents, n = 1..3.
CASES = [
    ((5, 37, 70), (2, 3, 4)),
    ((3, 16, 64), (1, 0, 2)),
    ((2, 3, 130), (3, 5, 1)),
    ((1, 1, 1), (0, 0, 0)),
    ((4, 20, 9), (0, 2, 7)),
    ((70,), (5,)),
    ((33, 47), (4, 6)),
    ((7, 19, 150), (3, 9, 15)),
    # every axis <= 7 taps (the streaming small-PSF kernel): several 16 x 64
    # tiles and 32-plane z blocks with ragged tails, 2p >= m, kz = 1, 2-D
    ((40, 37, 150), (3, 3, 3)),
    ((9, 70, 65), (1, 2, 1)),
    ((3, 5, 200), (2, 1, 3)),
    ((70, 20, 20), (0, 3, 1)),
    ((100, 130), (3, 2)),
]


@pytest.mark.parametrize("dtype", ["fp32", "fp64"])
@pytest.mark.parametrize("m,p", CASES)
def test_conv_full_and_adjoint(nd, m, p, dtype):
    say("case conv m=%s p=%s %s" % (m, p, dtype))
    rng = np.random.default_rng(synth.stable_seed(m, p))
    npdt = np.float32 if dtype == "fp32" else np.float64
    h = rng.standard_normal([2 * q + 1 for q in p]).astype(npdt)  # asymmetric, signed
    x = rng.random(m).astype(npdt)
    y = nd.conv_full_nd(gpu(x, npdt), gpu(h, npdt)).cpu().numpy()
    yo = oracle.conv_full(x, h)
    assert y.shape == yo.shape
    assert rel_l2(y, yo) <= TOL[dtype]
    r = rng.standard_normal(yo.shape).astype(npdt)
    g = nd.conv_adjoint_nd(gpu(r, npdt), gpu(h, npdt)).cpu().numpy()
    go = oracle.conv_adjoint(r, h)
    assert g.shape == tuple(m)
    assert rel_l2(g, go) <= TOL[dtype]


# the last two exceed the matrix-core tiles (ky = 37, kx = 41): general kernel
@pytest.mark.parametrize("prec", ["bf16", "split_bf16"])
@pytest.mark.parametrize("m,p", [((5, 37, 70), (2, 3, 4)), ((6, 40, 100), (3, 7, 15)), ((33, 47), (4, 6)),
                                 ((3, 80, 60), (1, 18, 4)), ((3, 20, 100), (1, 2, 20))])
def test_reduced_precision(nd, m, p, prec):
    say("case prec m=%s p=%s %s" % (m, p, prec))
    rng = np.random.default_rng(11)
    h = rng.random([2 * q + 1 for q in p]).astype(np.float32)
    h /= h.sum()
    x = rng.random(m).astype(np.float32)
    y = nd.conv_full_nd(gpu(x, np.float32), gpu(h, np.float32), precision=prec).cpu().numpy()
    assert rel_l2(y, oracle.conv_full(x, h)) <= TOL[prec]
    r = rng.standard_normal(y.shape).astype(np.float32)
    g = nd.conv_adjoint_nd(gpu(r, np.float32), gpu(h, np.float32), precision=prec).cpu().numpy()
    assert rel_l2(g, oracle.conv_adjoint(r, h)) <= TOL[prec]


# PSF rows of 11..33 taps take the 32x32x16 form in bf16 and split-bf16:
# 3 and 4 Toeplitz chunks per row (kx 11, 17 / 19, 31, 33), 2, 3 and 4 x blocks
# per wave with ragged x tails, several 64-row tiles, ky = 33, 2p >= m, z groups
# with ragged tails, a 2-D problem (three of the four planes of a group idle),
# a 256^3 volume with >= 512 work-groups (the widest tiles), and 1-D.
WIDE_CASES = [((9, 70, 130), (2, 16, 15)), ((5, 100, 64), (1, 5, 5)), ((3, 40, 250), (4, 3, 8)),
              ((4, 30, 90), (2, 4, 9)), ((80, 150), (12, 16)), ((2, 10, 20), (1, 8, 12)),
              ((6, 20, 256), (2, 2, 10)), ((256, 256, 256), (0, 1, 5)), ((300,), (12,))]


@pytest.mark.parametrize("form", ["1", "0"], ids=["mfma32x32", "mfma4x4"])
@pytest.mark.parametrize("prec", ["bf16", "split_bf16"])
@pytest.mark.parametrize("m,p", WIDE_CASES)
def test_reduced_precision_wide_rows(nd, m, p, prec, form, monkeypatch):
    """Both matrix-core forms of the bf16 operators on every case (the
    library picks one by volume; NDC_MFMA32 forces it here)."""
    monkeypatch.setenv("NDC_MFMA32", form)
    say("case wide m=%s p=%s %s form %s" % (m, p, prec, form))
    rng = np.random.default_rng(synth.stable_seed(m, p))
    h = rng.standard_normal([2 * q + 1 for q in p]).astype(np.float32)  # asymmetric, signed
    x = rng.random(m).astype(np.float32)
    y = nd.conv_full_nd(gpu(x, np.float32), gpu(h, np.float32), precision=prec).cpu().numpy()
    yo = oracle.conv_full(x, h)
    assert y.shape == yo.shape
    assert rel_l2(y, yo) <= TOL[prec]
    r = rng.standard_normal(yo.shape).astype(np.float32)
    g = nd.conv_adjoint_nd(gpu(r, np.float32), gpu(h, np.float32), precision=prec).cpu().numpy()
    assert g.shape == tuple(m)
    assert rel_l2(g, oracle.conv_adjoint(r, h)) <= TOL[prec]


@pytest.mark.parametrize("rule,mu", [("fixed", 0.0), ("cauchy", 0.0), ("bb", 0.0), ("fixed", 0.05)])
@pytest.mark.parametrize("prec,tol", [("bf16", 5e-2), ("split_bf16", 5e-4)])
def test_deconv_reduced_precision_wide_rows(nd, prec, tol, rule, mu, monkeypatch):
    """Five projected-gradient steps with the 32x32x16 operators against the
    FP64 oracle, for each first-trial rule and with the Laplacian term: the
    residual, update, gradient and norm epilogues all run on this tile.
    Each step moves X by delta*G with G from both operators, so the iterate
    and f carry a few times the operators' relative error e; the bound is 5e
    for each precision, as for f(X^0) at the metric size."""
    monkeypatch.setenv("NDC_MFMA32", "1")
    say("case deconv wide %s %s mu=%g" % (prec, rule, mu))
    rng = np.random.default_rng(21)
    m, p = (6, 40, 70), (2, 6, 12)
    h = rng.random([2 * q + 1 for q in p]).astype(np.float32) + 0.1
    h /= h.sum()
    xt = rng.random(m)
    y = (oracle.conv_full(xt, h) + 0.01 * rng.standard_normal([a + 2 * b for a, b in zip(m, p)])).astype(np.float32)
    x0 = np.full(m, float(xt.mean()), dtype=np.float32)
    xg, st, info = nd.deconv_iterate(gpu(y, np.float32), gpu(h, np.float32), gpu(x0, np.float32), 5, lam=0.01,
                                     precision=prec, rule=rule, mu=mu)
    torch.cuda.synchronize()
    xo, so, done, status = oracle.deconv(y.astype(np.float64), h.astype(np.float64), x0.astype(np.float64), 5,
                                         lam=0.01, rule=rule, mu=mu)
    assert info.cpu().tolist() == [5, 0] and (done, status) == (5, 0)
    f = st.cpu().numpy()[:, 0]
    assert np.all(np.diff(f) < 0)
    assert np.all(np.abs(f - so[:, 0]) <= tol * np.abs(so[:, 0]))
    assert float(xg.min()) >= 0.0
    assert rel_l2(xg.cpu().numpy(), xo) <= tol


# dH cases: one and several 128-column / 16-row tiles with ragged tails, PSF
# rows or columns spanning several 24-wide blocks, 1x1x1 PSF, 1-D and 2-D,
# and the broadcast form
DH_CASES = [((6, 9, 11), (1, 2, 3)), ((16, 40, 40), (3, 2, 4)), ((20, 33), (2, 5)),
            ((4, 50, 300), (1, 13, 2)), ((3, 70, 140), (2, 3, 14)), ((2, 20, 130), (0, 0, 0)),
            ((300,), (7,)), ((5, 37, 29), (2, 10, 10)),
            # broadcast form (21- and 25-row PSF planes): scalar and 16-byte
            # staging, fewer X planes than PSF planes, ragged x tiles
            ((9, 37, 70), (4, 10, 10)), ((12, 40, 64), (15, 10, 10)), ((7, 150, 136), (3, 12, 12)),
            ((5, 33, 257), (2, 10, 11)), ((6, 30, 68), (2, 10, 11))]  # last: 16-byte X, scalar G


@pytest.mark.parametrize("dtype", ["fp32", "fp64"])
@pytest.mark.parametrize("m,p", DH_CASES)
def test_conv_dH(nd, m, p, dtype):
    say("case dH m=%s p=%s %s" % (m, p, dtype))
    rng = np.random.default_rng(5)
    npdt = np.float32 if dtype == "fp32" else np.float64
    x = rng.random(m).astype(npdt)
    gr = rng.standard_normal([a + 2 * b for a, b in zip(m, p)]).astype(npdt)
    ps = [2 * q + 1 for q in p]
    dh = nd.conv_dH_nd(gpu(x, npdt), gpu(gr, npdt), ps).cpu().numpy()
    assert rel_l2(dh, oracle.conv_dH(x, gr, ps)) <= TOL[dtype]


def test_deterministic(nd):
    rng = np.random.default_rng(3)
    x = gpu(rng.random((9, 50, 80)), np.float32)
    h = gpu(rng.random((7, 5, 9)), np.float32)
    a = nd.conv_full_nd(x, h)
    b = nd.conv_full_nd(x, h)
    assert torch.equal(a, b)
    c = nd.conv_adjoint_nd(a, h)
    d = nd.conv_adjoint_nd(b, h)
    assert torch.equal(c, d)


def test_errors_on_device(nd):
    x = torch.zeros((4, 4), device="cuda")
    h = torch.zeros((3, 3), device="cuda")
    with pytest.raises(TypeError):
        nd.conv_full_nd(x.cpu(), h)
    import ctypes
    lib = nd.lib
    host = np.zeros(36, dtype=np.float32)
    rc = lib.conv_full_nd(2, nd.i64_array([4, 4]), nd.i64_array([1, 1]), ctypes.c_void_p(x.data_ptr()),
                          ctypes.c_void_p(h.data_ptr()), ctypes.c_void_p(host.ctypes.data), 0, 0, None)
    assert rc == -1  # host output pointer rejected before any launch
    y = torch.zeros((6, 6), device="cuda")
    rc = lib.conv_full_nd(2, nd.i64_array([4, 4]), nd.i64_array([1, 1]), ctypes.c_void_p(y.data_ptr()),
                          ctypes.c_void_p(h.data_ptr()), ctypes.c_void_p(y.data_ptr() + 8), 0, 0, None)
    assert rc == -3


# ---------------------------------------------------------------- deconvolution
def _check_deconv(nd, y, h, x0, iters, lam, npdt, tol_x, tol_f, prec="native", rule="fixed", tol_d=1e-14,
                  mu=0.0):
    xg, st, info = nd.deconv_iterate(gpu(y, npdt), gpu(h, npdt), gpu(x0, npdt), iters, lam=lam, precision=prec,
                                     rule=rule, mu=mu)
    torch.cuda.synchronize()
    xo, so, done, status = oracle.deconv(y.astype(np.float64), h.astype(np.float64), x0.astype(np.float64),
                                         iters, lam=lam, rule=rule, mu=mu)
    inf = info.cpu().numpy()
    stg = st.cpu().numpy()
    assert int(inf[0]) == done and int(inf[1]) == status
    # the accept/reject decisions must agree exactly; delta_0 = 1/||H||_1^2 is a
    # double sum taken in a different order on each side, so allow rounding
    np.testing.assert_array_equal(stg[1:done + 1, 2], so[1:done + 1, 2])
    np.testing.assert_allclose(stg[1:done + 1, 1], so[1:done + 1, 1], rtol=tol_d, atol=0)
    assert rel_l2(xg.cpu().numpy(), xo) <= tol_x
    f_g, f_o = stg[:done + 1, 0], so[:done + 1, 0]
    assert np.all(np.abs(f_g - f_o) <= tol_f * np.abs(f_o))
    assert np.all(np.diff(f_g) < 0)
    assert np.all(xg.cpu().numpy() >= 0)
    return xg, stg, inf


def test_deconv_c1_fp64_full(nd):
    """2-D, FP64, 64x64 X, 9x9 PSF, Poisson at peak 1000, 50 iterations."""
    cfg = synth.CONFIGS["c1_2d_f64"]
    say("case deconv c1")
    x_true = synth.make_objects(cfg)
    h = synth.psf_for(cfg)
    y = synth.add_noise(oracle.conv_full(x_true, h), cfg)
    x0 = synth.flat_start(y, h, cfg.shape)
    _check_deconv(nd, y, h, x0, cfg.iters, 0.0, np.float64, 1e-10, 1e-12)


@pytest.mark.parametrize("lam", [0.0, 0.3])
def test_deconv_fp32_small(nd, lam):
    say("case deconv fp32 small lam=%g" % lam)
    rng = np.random.default_rng(21)
    m, p = (6, 24, 70), (2, 3, 5)
    h = synth.gaussian_psf([2 * q + 1 for q in p], (1.0, 1.5, 2.0)).astype(np.float32)
    x_true = rng.random(m)
    y = (oracle.conv_full(x_true, h) + 0.05 * rng.standard_normal([a + 2 * b for a, b in zip(m, p)]))
    y = y.astype(np.float32)
    x0 = np.full(m, 0.4, dtype=np.float32)
    _check_deconv(nd, y, h, x0, 20, lam, np.float32, 1e-5, 1e-5)


@pytest.mark.parametrize("rule", ["cauchy", "bb"])
def test_deconv_step_rules_fp64(nd, rule):
    """Cauchy / Barzilai-Borwein first trials against the oracle, 2-D FP64
    (64x64 X, 9x9 PSF, Poisson noise): same decisions, deltas to 1e-9."""
    cfg = synth.CONFIGS["c1_2d_f64"]
    say("case deconv rule %s fp64" % rule)
    x_true = synth.make_objects(cfg)
    h = synth.psf_for(cfg)
    y = synth.add_noise(oracle.conv_full(x_true, h), cfg)
    x0 = synth.flat_start(y, h, cfg.shape)
    _check_deconv(nd, y, h, x0, 30, 0.0, np.float64, 1e-8, 1e-11, rule=rule, tol_d=1e-9)


def _rule_problem_fp32():
    rng = np.random.default_rng(31)
    m, p = (6, 24, 70), (2, 3, 5)
    h = synth.gaussian_psf([2 * q + 1 for q in p], (1.0, 1.5, 2.0)).astype(np.float32)
    y = (oracle.conv_full(rng.random(m), h) + 0.05 * rng.standard_normal([a + 2 * b for a, b in zip(m, p)]))
    return y.astype(np.float32), h, np.full(m, 0.4, dtype=np.float32)


def _check_rule_fp32(nd, y, h, x0, iters, lam, mu, rule, tol_d, max_flips=0, tol_fr=1e-6):
    """An FP32 run with a Cauchy / BB first trial against the FP64 oracle.

    * accept / halve decisions: identical, except at most `max_flips` of
      them (reported); iters_done identical when none may differ;
    * accepted deltas up to the first differing decision: relative `tol_d`.
      The Cauchy delta is a ratio of norms of the current gradient; the BB
      delta is a Rayleigh quotient of the previous step, i.e. of the
      difference of two iterates, so the FP32 trajectory's rounding reaches
      it amplified;
    * once the deltas differ the trajectories do too, so X and f are
      compared under delta-replay (the oracle repeats the GPU's accepted
      deltas in FP64): X within 1e-5 (1e-4 with the Laplacian term, whose
      high-frequency modes are stretched by steps longer than 2/L) and f
      within `tol_fr` at every step;
    * the final X also within 1e-4 of the oracle's own search."""
    xg, st, info = nd.deconv_iterate(gpu(y, np.float32), gpu(h, np.float32), gpu(x0, np.float32), iters, lam=lam,
                                     rule=rule, mu=mu)
    torch.cuda.synchronize()
    done, status = [int(v) for v in info.cpu().tolist()]
    stg, xg = st.cpu().numpy(), xg.cpu().numpy()
    yd, hd, x0d = y.astype(np.float64), h.astype(np.float64), x0.astype(np.float64)
    xo, so, done_o, status_o = oracle.deconv(yd, hd, x0d, iters, lam=lam, rule=rule, mu=mu)
    n = min(done, done_o)
    flips = np.flatnonzero(stg[1:n + 1, 2] != so[1:n + 1, 2])
    first = int(flips[0]) + 1 if len(flips) else n + 1
    assert len(flips) <= max_flips
    if max_flips == 0:
        assert (done, status) == (done_o, status_o)
    else:
        assert status == 0 and done == iters
    np.testing.assert_allclose(stg[1:first, 1], so[1:first, 1], rtol=tol_d, atol=0)
    assert np.all(np.diff(stg[:done + 1, 0]) < 0) and xg.min() >= 0
    xr, sr, _, _ = oracle.deconv(yd, hd, x0d, done, lam=lam, mu=mu, deltas=stg[1:done + 1, 1])
    assert rel_l2(xg, xr) <= (1e-4 if mu else 1e-5)
    assert np.all(np.abs(stg[:done + 1, 0] - sr[:done + 1, 0]) <= tol_fr * np.abs(sr[:done + 1, 0]))
    assert rel_l2(xg, xo) <= 1e-4
    dd = np.abs(stg[1:first, 1] - so[1:first, 1]) / so[1:first, 1]
    say("  %s lam=%g mu=%g: %d steps, %d of %d decisions differ; delta %.1e; X vs replay %.1e, vs oracle %.1e"
        % (rule, lam, mu, done, len(flips), n, dd.max() if len(dd) else 0.0, rel_l2(xg, xr), rel_l2(xg, xo)))


@pytest.mark.parametrize("rule", ["cauchy", "bb"])
@pytest.mark.parametrize("lam", [0.0, 0.01])
def test_deconv_step_rules_fp32(nd, rule, lam):
    """FP32 3-D, 30 iterations with identical accept / halve decisions (BB
    halves in several of them).  With these weights f stays well above the
    FP32 resolution for all 30 steps (the oracle's f is still 1e-5 or more
    above its limit), so every decision is a real one."""
    say("case deconv rule %s fp32 lam=%g" % (rule, lam))
    y, h, x0 = _rule_problem_fp32()
    _check_rule_fp32(nd, y, h, x0, 30, lam, 0.0, rule, 1e-4 if rule == "cauchy" else 2e-2)


@pytest.mark.parametrize("rule", ["cauchy", "bb"])
def test_deconv_step_rules_fp32_long(nd, rule):
    """60 FP32 iterations: strict decrease, X >= 0, and a lower objective
    than the fixed first trial reaches in the same number of iterations."""
    say("case deconv rule %s fp32 long" % rule)
    y, h, x0 = _rule_problem_fp32()
    res = {}
    for r in ("fixed", rule):
        xg, st, info = nd.deconv_iterate(gpu(y, np.float32), gpu(h, np.float32), gpu(x0, np.float32), 60, rule=r)
        torch.cuda.synchronize()
        inf, stg = info.cpu().tolist(), st.cpu().numpy()
        assert inf == [60, 0]
        assert np.all(np.diff(stg[:, 0]) < 0)
        assert xg.min().item() >= 0
        res[r] = stg[-1, 0]
    assert res[rule] < res["fixed"]


@pytest.mark.parametrize("rule", ["cauchy", "bb"])
def test_deconv_step_rules_fp32_at_rounding_level(nd, rule):
    """lambda = 0.3 makes the problem well conditioned: the oracle's f comes
    within 1e-9 of its minimum in about 9 BB (13 Cauchy) steps and the FP64
    oracle itself stops for want of descent at step 20 (29).  An FP32 run
    cannot resolve decreases that small, so its decisions must match only
    while f is above that level; later ones may legitimately differ.  Checked
    instead: the first 6 steps' decisions match exactly, every accepted step
    decreases f, X >= 0, the run converges to the oracle's unique minimiser,
    and replaying the GPU's accepted deltas in the oracle (delta-replay)
    reproduces its X.  The number of differing decisions is reported."""
    say("case deconv rule %s fp32 rounding level" % rule)
    y, h, x0 = _rule_problem_fp32()
    lam, iters = 0.3, 30
    xg, st, info = nd.deconv_iterate(gpu(y, np.float32), gpu(h, np.float32), gpu(x0, np.float32), iters, lam=lam,
                                     rule=rule)
    torch.cuda.synchronize()
    done, status = [int(v) for v in info.cpu().tolist()]
    stg, xg = st.cpu().numpy(), xg.cpu().numpy()
    yd, hd, x0d = y.astype(np.float64), h.astype(np.float64), x0.astype(np.float64)
    xo, so, done_o, _ = oracle.deconv(yd, hd, x0d, 60, lam=lam, rule=rule)
    assert done >= 6 and status in (0, 1)
    np.testing.assert_array_equal(stg[1:7, 2], so[1:7, 2])
    assert np.all(np.diff(stg[:done + 1, 0]) < 0) and xg.min() >= 0
    f_min = so[done_o, 0]
    assert abs(stg[done, 0] - f_min) <= 1e-6 * f_min
    assert rel_l2(xg, xo) <= 1e-3
    xr, sr, _, _ = oracle.deconv(yd, hd, x0d, done, lam=lam, deltas=stg[1:done + 1, 1])
    assert rel_l2(xg, xr) <= 1e-4
    n = min(done, done_o)
    diff = int(np.sum(stg[1:n + 1, 2] != so[1:n + 1, 2]))
    say("  %s: %d GPU steps (status %d), %d oracle steps; %d of %d decisions differ; "
        "X vs delta-replay %.2e, vs minimiser %.2e" % (rule, done, status, done_o, diff, n, rel_l2(xg, xr),
                                                       rel_l2(xg, xo)))


@pytest.mark.parametrize("rule", ["fixed", "cauchy", "bb"])
def test_deconv_laplacian_fp64(nd, rule):
    """Tikhonov-Miller term mu/2 ||L X||^2 (2-D 5-point stencil) against the
    oracle: 2-D FP64, 64x64 X, 9x9 PSF, 30 iterations."""
    cfg = synth.CONFIGS["c1_2d_f64"]
    say("case deconv laplacian %s fp64" % rule)
    x_true = synth.make_objects(cfg)
    h = synth.psf_for(cfg)
    y = synth.add_noise(oracle.conv_full(x_true, h), cfg)
    x0 = synth.flat_start(y, h, cfg.shape)
    _check_deconv(nd, y, h, x0, 30, 0.0, np.float64, 1e-8, 1e-11, rule=rule, tol_d=1e-9, mu=0.05)


def test_deconv_laplacian_fp64_1d(nd):
    """1-D (3-tap stencil) with lambda and mu together."""
    say("case deconv laplacian 1-D")
    rng = np.random.default_rng(33)
    h = synth.gaussian_psf([11], (2.0,))
    y = oracle.conv_full(10.0 * rng.random(300), h) + 0.1 * rng.standard_normal(310)
    _check_deconv(nd, y, h, np.full(300, 5.0), 25, 0.2, np.float64, 1e-8, 1e-11, tol_d=1e-9, mu=0.3)


def test_deconv_laplacian_fp32(nd):
    """3-D 7-point stencil through the small-PSF kernels, FP32, fixed first
    trial: 30 iterations with identical decisions and deltas."""
    say("case deconv laplacian fixed fp32")
    y, h, x0 = _rule_problem_fp32()
    _check_deconv(nd, y, h, x0, 30, 0.0, np.float32, 1e-4, 1e-5, tol_d=1e-6, mu=0.05)


@pytest.mark.parametrize("rule", ["cauchy", "bb"])
def test_deconv_laplacian_fp32_step_rules(nd, rule):
    """The Laplacian term with the Cauchy and BB first trials, FP32, 30
    iterations.  Cauchy: identical decisions.  BB: its deltas follow the
    FP32 trajectory (see _check_rule_fp32) and one late trial near the
    acceptance boundary may be decided differently; X and f then follow
    under delta-replay."""
    say("case deconv laplacian %s fp32" % rule)
    y, h, x0 = _rule_problem_fp32()
    if rule == "cauchy":
        _check_rule_fp32(nd, y, h, x0, 30, 0.0, 0.05, rule, 1e-3)
    else:
        # the stencil's top modes (eigenvalues up to mu (4n)^2 = 7.2 here) are
        # stretched by BB steps longer than 2/L, so the FP32 rounding that
        # enters the Rayleigh quotient grows faster than without the term:
        # deltas measured within 6.2e-2 before the flip
        _check_rule_fp32(nd, y, h, x0, 30, 0.0, 0.05, rule, 1e-1, max_flips=1, tol_fr=3e-5)


# ------------------------------------------- schedule, no host wait, graphs
def test_deconv_trial_budget_and_resume(nd):
    """A budget of trial slots smaller than the steps asked for stops with
    NDC_STOP_TRIALS after exactly that many accepted steps (no rejections
    here); a second call from the returned X continues the fixed-rule run
    bitwise."""
    say("case deconv trial budget")
    rng = np.random.default_rng(8)
    m = (5, 30, 40)
    h = synth.gaussian_psf([3, 7, 7], (1.0, 1.2, 1.2)).astype(np.float32)
    y = gpu(oracle.conv_full(rng.random(m), h) + 0.01, np.float32)
    hg = gpu(h, np.float32)
    xa, _, ia = nd.deconv_iterate(y, hg, torch.full(m, 0.3, device="cuda"), 7)
    xb, sb, ib = nd.deconv_iterate(y, hg, torch.full(m, 0.3, device="cuda"), 7, max_trials=4)
    assert ib.cpu().tolist() == [4, 2]
    assert not torch.isnan(sb[4]).any() and torch.isnan(sb[5]).all()
    xb, _, ib = nd.deconv_iterate(y, hg, xb, 3)
    assert ia.cpu().tolist() == [7, 0] and ib.cpu().tolist() == [3, 0]
    assert torch.equal(xa, xb)


def test_deconv_returns_without_waiting(nd):
    """The call only enqueues work: with a long-running kernel queued in
    front of it on the same stream it returns before the stream is idle, and
    the result after synchronising equals a plain run."""
    say("case deconv no host wait")
    rng = np.random.default_rng(5)
    m = (6, 40, 64)
    h = synth.gaussian_psf([5, 9, 9], (1.0, 1.5, 1.5)).astype(np.float32)
    y = gpu(oracle.conv_full(rng.random(m), h) + 0.01, np.float32)
    hg = gpu(h, np.float32)
    xa, _, _ = nd.deconv_iterate(y, hg, torch.full(m, 0.3, device="cuda"), 5)
    torch.cuda.synchronize()
    big = torch.randn(4096, 4096, device="cuda")
    x = torch.full(m, 0.3, device="cuda")
    for _ in range(20):  # ~ tens of ms of queued work
        big = big @ big
        big = big / big.norm()
    xb, _, info = nd.deconv_iterate(y, hg, x, 5)
    pending = not torch.cuda.current_stream().query()
    torch.cuda.synchronize()
    assert pending
    assert info.cpu().tolist() == [5, 0] and torch.equal(xa, xb)


@pytest.mark.parametrize("rule,mu", [("fixed", 0.0), ("bb", 0.0), ("cauchy", 0.05)])
def test_deconv_graph_capture_replays_equal_eager(nd, rule, mu):
    """deconv_iterate captured into a graph: each replay, started from the
    same X^0 (restored by eager work between replays), equals an eager call
    bitwise in X, stats and info."""
    say("case deconv graph capture %s mu=%g" % (rule, mu))
    y, h, x0 = _rule_problem_fp32()
    yg, hg, x0g = gpu(y, np.float32), gpu(h, np.float32), gpu(x0, np.float32)
    iters = 6
    xe, se, ie = nd.deconv_iterate(yg, hg, x0g.clone(), iters, rule=rule, mu=mu)
    torch.cuda.synchronize()
    need = nd.deconv_workspace_bytes_ex(list(x0.shape), list(h.shape), regularised=1 if mu > 0 else 0)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    stats = torch.full((iters + 1, 4), float("nan"), dtype=torch.float64, device="cuda")
    info = torch.zeros(2, dtype=torch.int32, device="cuda")
    x = x0g.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            nd.deconv_iterate(yg, hg, x, iters, ws=ws, stats=stats, info=info, rule=rule, mu=mu)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        x.copy_(x0g)
        stats.fill_(float("nan"))
        info.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert info.cpu().tolist() == ie.cpu().tolist(), rep
        assert torch.equal(x, xe), rep
        assert bool(torch.all((stats == se) | (torch.isnan(stats) & torch.isnan(se)))), rep


def test_deconv_stops_without_descent(nd):
    """Y = A X^0 exactly (integers, exact in FP32): f(X^0) = 0, no step can
    decrease it, the loop stops with status 1 after 30 halvings."""
    rng = np.random.default_rng(2)
    h = rng.integers(1, 4, (3, 3, 3)).astype(np.float32)
    x0 = rng.integers(0, 3, (4, 5, 6)).astype(np.float32)
    y = oracle.conv_full(x0, h).astype(np.float32)
    xg, st, info = nd.deconv_iterate(gpu(y, np.float32), gpu(h, np.float32), gpu(x0, np.float32), 3)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0, 1]
    np.testing.assert_array_equal(xg.cpu().numpy(), x0)


def test_deconv_nonfinite(nd):
    h = np.full((3, 3), 1 / 9, dtype=np.float32)
    y = np.ones((6, 6), dtype=np.float32)
    y[2, 2] = np.nan
    xg, st, info = nd.deconv_iterate(gpu(y, np.float32), gpu(h, np.float32), gpu(np.zeros((4, 4)), np.float32), 3)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [0, -4]


def test_deconv_resume_is_exact(nd):
    """The adopted step rule is stateless: 6 steps equal 3 + 3 bitwise."""
    rng = np.random.default_rng(8)
    m, p = (5, 30, 40), (1, 3, 3)
    h = synth.gaussian_psf([3, 7, 7], (1.0, 1.2, 1.2)).astype(np.float32)
    y = gpu(oracle.conv_full(rng.random(m), h) + 0.01, np.float32)
    hg = gpu(h, np.float32)
    xa, _, _ = nd.deconv_iterate(y, hg, torch.full(m, 0.3, device="cuda"), 6)
    xb, _, _ = nd.deconv_iterate(y, hg, torch.full(m, 0.3, device="cuda"), 3)
    xb, _, _ = nd.deconv_iterate(y, hg, xb, 3)
    assert torch.equal(xa, xb)


def _random_wide_cases(n, seed=31):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        nd_ = int(rng.integers(1, 4))
        px = int(rng.integers(5, 17))  # kx 11..33
        p = [int(rng.integers(0, 6)) for _ in range(nd_ - 1)] + [px]
        if nd_ >= 2:
            p[-2] = int(rng.integers(0, 17))  # ky up to 33
        m = [int(rng.integers(1, 12)) for _ in range(nd_ - 2)] + ([int(rng.integers(1, 90))] if nd_ >= 2 else []) + \
            [int(rng.integers(1, 200))]
        out.append((tuple(m), tuple(p)))
    return out


@pytest.mark.parametrize("prec", ["bf16", "split_bf16"])
@pytest.mark.parametrize("m,p", _random_wide_cases(12))
def test_reduced_precision_wide_rows_random(nd, m, p, prec, monkeypatch):
    """Seeded random shapes (1-D to 3-D, 2p >= m included) on the forced
    32x32x16 form against the oracle."""
    monkeypatch.setenv("NDC_MFMA32", "1")
    say("case wide random m=%s p=%s %s" % (m, p, prec))
    rng = np.random.default_rng(synth.stable_seed(m, p))
    h = rng.standard_normal([2 * q + 1 for q in p]).astype(np.float32)
    x = rng.random(m).astype(np.float32)
    y = nd.conv_full_nd(gpu(x, np.float32), gpu(h, np.float32), precision=prec).cpu().numpy()
    yo = oracle.conv_full(x, h)
    assert y.shape == yo.shape
    assert rel_l2(y, yo) <= TOL[prec]
    r = rng.standard_normal(yo.shape).astype(np.float32)
    g = nd.conv_adjoint_nd(gpu(r, np.float32), gpu(h, np.float32), precision=prec).cpu().numpy()
    assert g.shape == tuple(m)
    assert rel_l2(g, oracle.conv_adjoint(r, h)) <= TOL[prec]


def _random_cases(n, seed=57):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        nd_ = int(rng.integers(1, 4))
        # half axis widths from 0 to 20: small-PSF kernel, matrix-core tile and, past 16, the general kernel
        p = tuple(int(rng.integers(0, 4)) if rng.random() < 0.4 else int(rng.integers(0, 21)) for _ in range(nd_))
        m = tuple(int(rng.integers(1, 9 if i < nd_ - 2 else 70)) for i in range(nd_))
        out.append((m, p))
    return out


@pytest.mark.parametrize("dtype", ["fp32", "fp64"])
@pytest.mark.parametrize("m,p", _random_cases(12))
def test_conv_random_shapes(nd, m, p, dtype):
    """Seeded random shapes across all kernels (1-D to 3-D, 2p >= m included)."""
    say("case random m=%s p=%s %s" % (m, p, dtype))
    rng = np.random.default_rng(synth.stable_seed(m, p, dtype))
    npdt = np.float32 if dtype == "fp32" else np.float64
    h = rng.standard_normal([2 * q + 1 for q in p]).astype(npdt)
    x = rng.random(m).astype(npdt)
    y = nd.conv_full_nd(gpu(x, npdt), gpu(h, npdt)).cpu().numpy()
    yo = oracle.conv_full(x, h)
    assert y.shape == yo.shape
    assert rel_l2(y, yo) <= TOL[dtype]
    r = rng.standard_normal(yo.shape).astype(npdt)
    g = nd.conv_adjoint_nd(gpu(r, npdt), gpu(h, npdt)).cpu().numpy()
    assert g.shape == tuple(m)
    assert rel_l2(g, oracle.conv_adjoint(r, h)) <= TOL[dtype]


@pytest.mark.parametrize("dtype", ["fp32", "fp64"])
@pytest.mark.parametrize("m,p", _random_cases(10, seed=91))
def test_conv_dH_random_shapes(nd, m, p, dtype):
    """PSF gradient on seeded random shapes (1-D to 3-D)."""
    say("case dH random m=%s p=%s %s" % (m, p, dtype))
    rng = np.random.default_rng(synth.stable_seed(m, p, dtype, 1))
    npdt = np.float32 if dtype == "fp32" else np.float64
    x = rng.random(m).astype(npdt)
    gr = rng.standard_normal([a + 2 * b for a, b in zip(m, p)]).astype(npdt)
    ps = [2 * q + 1 for q in p]
    dh = nd.conv_dH_nd(gpu(x, npdt), gpu(gr, npdt), ps).cpu().numpy()
    assert dh.shape == tuple(ps)
    assert rel_l2(dh, oracle.conv_dH(x, gr, ps)) <= TOL[dtype]


def _random_deconv_cases(n, seed=123):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        nd_ = int(rng.integers(1, 4))
        m = tuple(int(rng.integers(2, 8 if j < nd_ - 2 else 40)) for j in range(nd_))
        p = tuple(int(rng.integers(0, 6)) for _ in range(nd_))
        rule = ("fixed", "cauchy", "bb")[i % 3]
        lam = float(rng.choice([0.0, 0.05]))
        mu = float(rng.choice([0.0, 0.02]))
        out.append((m, p, rule, lam, mu))
    return out


@pytest.mark.parametrize("m,p,rule,lam,mu", _random_deconv_cases(9))
def test_deconv_random_fp64(nd, m, p, rule, lam, mu):
    """FP64 deconvolution on seeded random problems (1-D to 3-D, every first
    trial, with and without the Tikhonov and Laplacian terms): the same
    decisions as the oracle, X, f and delta to rounding."""
    say("case deconv random m=%s p=%s %s lam=%g mu=%g" % (m, p, rule, lam, mu))
    rng = np.random.default_rng(synth.stable_seed(m, p, rule))
    h = rng.random([2 * q + 1 for q in p]) + 0.05
    h /= h.sum()
    y = oracle.conv_full(rng.random(m) + 0.1, h) + 0.01 * rng.standard_normal([a + 2 * b for a, b in zip(m, p)])
    x0 = np.full(m, float(np.mean(y)))
    _check_deconv(nd, y, h, x0, 10, lam, np.float64, 1e-9, 1e-11, rule=rule, tol_d=1e-9, mu=mu)
