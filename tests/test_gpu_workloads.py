"""Parity at the workload sizes, in the launch configuration the benchmark
times: the 3-D FP32 workload (X 64x128x128, PSF 31x15x15) in full, the
metric workload (X 128x512x512, PSF 63x31x31) on sampled outputs the oracle
computes one by one, for every precision, and the deconvolution trajectory
against the oracle's stored one."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import synth
from tests.conftest import ROOT

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16": 1e-2, "split_bf16": 1e-4}


@pytest.fixture(scope="module")
def nd():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1711_11224_amd as m
    return m


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.fixture(scope="module")
def c2(nd):
    cfg = synth.CONFIGS["c2_3d_f32"]
    x = synth.make_objects(cfg).astype(np.float32)
    h = synth.psf_for(cfg).astype(np.float32)
    yo = oracle.conv_full(x, h)
    r = np.random.default_rng(1).standard_normal(yo.shape).astype(np.float32)
    go = oracle.conv_adjoint(r, h)
    return cfg, x, h, yo, r, go


@pytest.mark.parametrize("prec", ["fp32", "bf16", "split_bf16"])
def test_c2_full_outputs(nd, c2, prec):
    cfg, x, h, yo, r, go = c2
    say("case c2 full %s" % prec)
    dev = lambda a: torch.from_numpy(a).cuda()
    y = nd.conv_full_nd(dev(x), dev(h), precision=prec).cpu().numpy()
    assert y.shape == yo.shape == (94, 142, 142)
    assert rel_l2(y, yo) <= TOL[prec]
    g = nd.conv_adjoint_nd(dev(r), dev(h), precision=prec).cpu().numpy()
    assert g.shape == cfg.shape
    assert rel_l2(g, go) <= TOL[prec]


@pytest.fixture(scope="module")
def c3(nd):
    cfg = synth.CONFIGS["c3_metric"]
    x = synth.make_objects(cfg).astype(np.float32)
    h = synth.psf_for(cfg).astype(np.float32)
    rng = np.random.default_rng(2)
    r = rng.standard_normal([a + b - 1 for a, b in zip(cfg.shape, cfg.psf_shape)]).astype(np.float32)
    iy = rng.choice(r.size, 2048, replace=False)
    ix = rng.choice(x.size, 2048, replace=False)
    yo = oracle.conv_full_at(x, h, iy)
    go = oracle.conv_adjoint_at(r, h, ix)
    return cfg, x, h, r, iy, ix, yo, go


@pytest.mark.parametrize("prec", ["fp32", "bf16", "split_bf16"])
def test_c3_sampled_outputs(nd, c3, prec):
    cfg, x, h, r, iy, ix, yo, go = c3
    say("case c3 sampled %s" % prec)
    xt, ht, rt = torch.from_numpy(x).cuda(), torch.from_numpy(h).cuda(), torch.from_numpy(r).cuda()
    y = nd.conv_full_nd(xt, ht, precision=prec)
    assert tuple(y.shape) == (190, 542, 542)
    assert rel_l2(y.view(-1)[torch.from_numpy(iy).cuda()].cpu().numpy(), yo) <= TOL[prec]
    del y
    g = nd.conv_adjoint_nd(rt, ht, precision=prec)
    assert tuple(g.shape) == (128, 512, 512)
    assert rel_l2(g.view(-1)[torch.from_numpy(ix).cuda()].cpu().numpy(), go) <= TOL[prec]


def test_c3_forward_edges_exact_subvolume(nd, c3):
    """A corner sub-volume of the metric forward (every clipped boundary
    tile type) against the oracle evaluated at each of its voxels."""
    cfg, x, h, r, *_ = c3
    say("case c3 corner")
    y = nd.conv_full_nd(torch.from_numpy(x).cuda(), torch.from_numpy(h).cuda()).cpu().numpy()
    zz, yy, xx = np.meshgrid(np.r_[0:3, 188:190], np.r_[0:3, 539:542], np.r_[0:5, 537:542], indexing="ij")
    idx = np.ravel_multi_index((zz.ravel(), yy.ravel(), xx.ravel()), y.shape)
    assert rel_l2(y.ravel()[idx], oracle.conv_full_at(x, h, idx)) <= 1e-5


def test_c3_transpose_edges_exact_subvolume(nd, c3):
    """A corner sub-volume of the metric transpose (the first and last
    planes, rows and columns of X, where the PSF reaches past Y's zero
    padding) against the oracle evaluated at each of its voxels."""
    cfg, x, h, r, *_ = c3
    say("case c3 transpose corner")
    g = nd.conv_adjoint_nd(torch.from_numpy(r).cuda(), torch.from_numpy(h).cuda()).cpu().numpy()
    zz, yy, xx = np.meshgrid(np.r_[0:3, 125:128], np.r_[0:3, 509:512], np.r_[0:5, 507:512], indexing="ij")
    idx = np.ravel_multi_index((zz.ravel(), yy.ravel(), xx.ravel()), g.shape)
    assert rel_l2(g.ravel()[idx], oracle.conv_adjoint_at(r, h, idx)) <= 1e-5


def _c2_inputs():
    sys.path.insert(0, os.path.join(ROOT, "tests", "golden"))
    import make_c2_trajectory as mk
    return mk.inputs(), mk.sha


def test_c2_deconv_100_iterations_vs_oracle_trajectory(nd):
    """100 projected-gradient steps on the 3-D FP32 workload against the FP64
    oracle's stored trajectory: same number of accepted steps and the same
    step sizes; f_k within 1e-5 relative; X on 4096 sampled voxels within
    1e-4 relative L2 (FP32 rounding accumulated over 100 steps)."""
    path = os.path.join(ROOT, "tests", "golden", "c2_deconv_trajectory.json")
    if not os.path.exists(path):
        pytest.skip("trajectory not generated")
    gold = json.load(open(path))
    say("case c2 deconv 100")
    (cfg, y, h, x0), sha = _c2_inputs()
    assert sha(y) == gold["y_sha256"] and sha(x0) == gold["x0_sha256"] and sha(h) == gold["h_sha256"]
    xg, st, info = nd.deconv_iterate(torch.from_numpy(y).cuda(), torch.from_numpy(h).cuda(),
                                     torch.from_numpy(x0).cuda(), cfg.iters)
    torch.cuda.synchronize()
    done, status = info.cpu().tolist()
    assert done == gold["done"] and status == gold["status"]
    st = st.cpu().numpy()
    np.testing.assert_array_equal(st[1:done + 1, 2], np.array(gold["rejections"]))
    np.testing.assert_allclose(st[1:done + 1, 1], np.array(gold["delta"]), rtol=1e-14)
    f = np.array(gold["f"])
    assert np.max(np.abs(st[:done + 1, 0] - f) / np.abs(f)) <= 1e-5
    xs = xg.cpu().numpy().ravel()[np.array(gold["sample_idx"])]
    assert rel_l2(xs, np.array(gold["x_samples"])) <= 1e-4
    assert np.all(np.diff(st[:done + 1, 0]) < 0)


# Tolerance on f(X^0) = 1/2||A X^0 - Y||^2 for the flat start: the operator's
# relative error e enters R = A X^0 - Y amplified by ||A X^0|| / ||R|| (about
# 2.5 for these inputs) and f doubles it, so 5e for each precision.
F0_TOL = {"fp32": 5e-5, "bf16": 5e-2, "split_bf16": 5e-4}


@pytest.fixture(scope="module")
def c3_deconv_inputs(nd):
    cfg = synth.CONFIGS["c3_metric"]
    rng = np.random.default_rng(5)
    factors = synth.gaussian_factors(cfg.psf_shape, cfg.sigmas)
    h = synth.psf_for(cfg).astype(np.float32)
    y = rng.poisson(50.0, size=[a + b - 1 for a, b in zip(cfg.shape, cfg.psf_shape)]).astype(np.float32)
    x0 = synth.flat_start(y, h, cfg.shape).astype(np.float32)
    ax0 = oracle.conv_full_separable(np.full(cfg.shape, float(x0.ravel()[0])), factors)
    f0 = 0.5 * float(np.sum((ax0 - y.astype(np.float64)) ** 2))
    return cfg, h, y, x0, f0, ax0


@pytest.mark.parametrize("prec", ["fp32", "bf16", "split_bf16"])
def test_c3_deconv_steps_properties(nd, c3_deconv_inputs, prec):
    """Metric workload, a few steps in each precision: every step accepted,
    f strictly decreasing, X >= 0, and f(X^0) against the oracle (flat X^0
    with the separable Gaussian PSF, one 1-D full convolution per axis)."""
    cfg, h, y, x0, f0, _ = c3_deconv_inputs
    say("case c3 deconv %s" % prec)
    xg, st, info = nd.deconv_iterate(torch.from_numpy(y).cuda(), torch.from_numpy(h).cuda(),
                                     torch.from_numpy(x0).cuda(), 3, precision=prec)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [3, 0]
    f = st.cpu().numpy()[:, 0]
    assert np.all(np.diff(f) < 0)
    assert float(xg.min()) >= 0.0
    assert abs(f[0] - f0) <= F0_TOL[prec] * f0


@pytest.mark.parametrize("prec", ["fp32", "bf16", "split_bf16"])
def test_c3_first_step_sampled_x_vs_oracle(nd, c3_deconv_inputs, prec):
    """Metric workload, one projected-gradient step (Step 2) from the flat
    start in each precision, against the oracle on 2048 sampled voxels:
    the first trial is the fixed rule's delta_0 = 1 / ||H||_1^2 and is
    accepted (f decreases for any delta <= 1/L); X_1 = max(X_0 - delta_0
    A^T (A X_0 - Y), 0) with the oracle's residual of the flat start (one
    1-D full convolution per axis) and its transpose evaluated at each
    sampled voxel.  Tolerance: the operator's relative error e reaches the
    gradient through R (amplified by ||A X_0|| / ||R||) and directly, and
    X_1 through delta_0 ||g|| / ||X_1|| (both measured on the oracle's
    side), so amp * (ratio + 1) * e, with e = 1e-5 / 1e-2 / 1e-4."""
    cfg, h, y, x0, f0, ax0 = c3_deconv_inputs
    say("case c3 first step sampled X %s" % prec)
    xg, st, info = nd.deconv_iterate(torch.from_numpy(y).cuda(), torch.from_numpy(h).cuda(),
                                     torch.from_numpy(x0).cuda(), 1, precision=prec)
    torch.cuda.synchronize()
    assert info.cpu().tolist() == [1, 0]
    st = st.cpu().numpy()
    h64 = h.astype(np.float64)
    d0 = oracle.initial_delta(h64)
    assert st[1, 2] == 0 and abs(st[1, 1] - d0) <= 1e-12 * d0
    r = ax0 - y.astype(np.float64)
    idx = np.random.default_rng(17).choice(x0.size, 2048, replace=False)
    g = oracle.conv_adjoint_at(r, h64, idx)
    x1 = np.maximum(x0.astype(np.float64).ravel()[idx] - d0 * g, 0.0)
    amp = d0 * np.linalg.norm(g) / np.linalg.norm(x1)
    ratio = float(np.linalg.norm(ax0) / np.linalg.norm(r))
    e = {"fp32": 1e-5, "bf16": 1e-2, "split_bf16": 1e-4}[prec]
    got = xg.view(-1)[torch.from_numpy(idx).cuda()].cpu().numpy()
    err = rel_l2(got, x1)
    say("  rel L2 %.2e (tolerance %.2e; amp %.2f, ratio %.2f)" % (err, amp * (ratio + 1) * e, amp, ratio))
    assert err <= amp * (ratio + 1) * e


# ---- the paper's two 2-D experiment shapes (synthetic stand-ins) ----------

def snr_db(est, ref):
    """SNR = 10 log10(||ref||^2 / ||est - ref||^2) over X's extent."""
    ref = np.asarray(ref, np.float64)
    return 10.0 * np.log10(np.sum(ref * ref) / np.sum((np.asarray(est, np.float64) - ref) ** 2))


PAPER_CASES = [(name, std) for name, w in synth.PAPER_2D.items() for std in w["noise"]]


@pytest.mark.parametrize("name,std", PAPER_CASES)
def test_paper_2d_deconv_vs_oracle(nd, name, std):
    """100 FP32 iterations from the blurred start X0 = max(crop(Y), 0) against
    the FP64 oracle: same decisions, objective to 1e-5, X to 1e-4, SNR to
    0.01 dB."""
    say("case paper 2-D %s std %g" % (name, std))
    w = synth.PAPER_2D[name]
    x = w["object"]()
    h = synth.gaussian_psf(w["psf"], w["sigma"])
    y = synth.gaussian_noise(oracle.conv_full(x, h), std, seed=11)
    p = [(e - 1) // 2 for e in w["psf"]]
    x0 = np.maximum(y[p[0]:p[0] + x.shape[0], p[1]:p[1] + x.shape[1]], 0.0)
    yg = torch.from_numpy(y.astype(np.float32)).cuda()
    hg = torch.from_numpy(h.astype(np.float32)).cuda()
    xg = torch.from_numpy(x0.astype(np.float32)).cuda()
    xg, st, info = nd.deconv_iterate(yg, hg, xg, 100)
    torch.cuda.synchronize()
    xo, so, done, status = oracle.deconv(y.astype(np.float32).astype(np.float64), h.astype(np.float32),
                                         x0.astype(np.float32).astype(np.float64), 100)
    stg = st.cpu().numpy()
    assert info.cpu().tolist() == [done, status] == [100, 0]
    np.testing.assert_array_equal(stg[1:, 2], so[1:, 2])
    assert np.all(np.abs(stg[:, 0] - so[:, 0]) <= 1e-5 * np.abs(so[:, 0]))
    xe = xg.cpu().numpy()
    assert rel_l2(xe, xo) <= 1e-4
    assert abs(snr_db(xe, x) - snr_db(xo, x)) <= 0.01
