"""Richardson-Lucy with the library's operators (rl_iterate) against the
oracle's richardson_lucy: iterates and I-divergences element by element on
the same seeded inputs."""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


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
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).cuda()


def _problem(seed, m, k, sig, counts=200.0):
    """A non-negative object blurred by a Gaussian PSF, Poisson counts."""
    rng = np.random.default_rng(seed)
    h = synth.gaussian_psf(k, sig)
    x = rng.random(m) ** 4  # mostly dim, a few bright voxels
    y = rng.poisson(counts * oracle.conv_full(x, h)).astype(np.float64) / counts
    x0 = synth.flat_start(y, h, m)
    return y, h, x0


def _check(nd, y, h, x0, iters, npdt, tol_x, tol_d, precision="native"):
    xg, st, info = nd.rl_iterate(gpu(y, npdt), gpu(h, npdt), gpu(x0, npdt), iters, precision=precision)
    torch.cuda.synchronize()
    yd, hd = y.astype(npdt).astype(np.float64), h.astype(npdt).astype(np.float64)
    xo, do = oracle.richardson_lucy(yd, hd, x0.astype(npdt).astype(np.float64), iters)
    assert info.cpu().tolist() == [iters, 0]
    e_x = rel_l2(xg.cpu().numpy(), xo)
    dg = st.cpu().numpy()
    e_d = float(np.max(np.abs(dg - do) / np.abs(do)))
    say("  X %.2e, divergence %.2e" % (e_x, e_d))
    assert e_x <= tol_x
    assert e_d <= tol_d
    assert xg.min().item() >= 0
    return xg, dg


@pytest.mark.parametrize("m,k", [((7, 37, 70), (5, 7, 9)), ((3, 20, 150), (3, 5, 15)), ((45, 50), (9, 9)),
                                 ((200,), (11,))])
def test_rl_fp64(nd, m, k):
    """FP64, 20 iterations: several tiles, ragged tails, 1-D to 3-D."""
    say("case rl fp64 m=%s k=%s" % (m, k))
    y, h, x0 = _problem(synth.stable_seed(m, k), m, k, tuple(0.25 * e for e in k))
    _check(nd, y, h, x0, 20, np.float64, 1e-12, 1e-12)


@pytest.mark.parametrize("m,k", [((10, 40, 64), (7, 9, 9)), ((6, 24, 70), (5, 7, 11))])
def test_rl_fp32(nd, m, k):
    """FP32, 50 iterations.  Each iteration applies two operators with a
    relative error of about 1e-6 (blocked FP32 sums) to a multiplicative
    update, so errors add up to about 50 x 2e-6."""
    say("case rl fp32 m=%s k=%s" % (m, k))
    y, h, x0 = _problem(synth.stable_seed(m, k, "f32"), m, k, tuple(0.3 * e for e in k))
    xg, dg = _check(nd, y, h, x0, 50, np.float32, 1e-4, 1e-5)
    assert np.all(np.diff(dg) <= 1e-6 * abs(dg[0]))  # the EM iteration never increases D


def test_rl_fp32_3d_workload(nd):
    """The 3-D FP32 workload (X 64x128x128, PSF 31x15x15, Poisson plus read
    noise; Y clipped at 0 since the method needs Y >= 0), 3 iterations."""
    cfg = synth.CONFIGS["c2_3d_f32"]
    say("case rl c2")
    x = synth.make_objects(cfg)
    h = synth.psf_for(cfg)
    y = np.maximum(synth.add_noise(oracle.conv_full_separable(x, synth.gaussian_factors(cfg.psf_shape, cfg.sigmas)),
                                   cfg), 0.0)
    _check(nd, y, h, synth.flat_start(y, h, cfg.shape), 3, np.float32, 1e-5, 1e-5)


def test_rl_paper_2d_shape(nd):
    """The paper's 225x225 image shape with a 5x5 PSF and noise std 5
    (Y clipped at 0), FP32, 100 iterations from the flat start."""
    w = synth.PAPER_2D["image225"]
    say("case rl 2-D 225")
    x = w["object"]()
    h = synth.gaussian_psf(w["psf"], w["sigma"])
    y = np.maximum(synth.gaussian_noise(oracle.conv_full(x, h), 5.0, seed=11), 0.0)
    _check(nd, y, h, synth.flat_start(y, h, x.shape), 100, np.float32, 1e-4, 1e-5)


def test_rl_reduced_precision(nd):
    """bf16 operands: one iteration within twice the operator tolerance
    (two operators, 2 x 1e-2); split-bf16: 10 iterations within
    2 x 10 x 1e-4 (each iteration's two operators, errors adding)."""
    m, k = (8, 40, 80), (5, 11, 13)
    say("case rl bf16 / split")
    y, h, x0 = _problem(71, m, k, (1.2, 2.5, 3.0))
    _check(nd, y, h, x0, 1, np.float32, 2e-2, 2e-2, precision="bf16")
    _check(nd, y, h, x0, 10, np.float32, 2e-3, 2e-3, precision="split_bf16")


def test_rl_graph_capture_replays_equal_eager(nd):
    say("case rl graph capture")
    y, h, x0 = _problem(72, (9, 33, 47), (5, 7, 7), (1.0, 1.5, 1.5))
    yg, hg, x0g = gpu(y, np.float32), gpu(h, np.float32), gpu(x0, np.float32)
    xe, se, ie = nd.rl_iterate(yg, hg, x0g.clone(), 7)
    torch.cuda.synchronize()
    need = nd.lib.rl_workspace_bytes(3, nd.i64_array(x0.shape), nd.i64_array([2, 3, 3]), 0, 0)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    stats = torch.zeros(8, dtype=torch.float64, device="cuda")
    info = torch.zeros(2, dtype=torch.int32, device="cuda")
    x = x0g.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            nd.rl_iterate(yg, hg, x, 7, ws=ws, stats=stats, info=info)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        x.copy_(x0g)
        stats.zero_()
        info.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(x, xe) and torch.equal(stats, se) and torch.equal(info, ie), rep


def test_rl_status_words(nd):
    """A PSF summing to 0 stops before the first update (X untouched,
    NDC_EINVAL in info); a NaN in Y stops on the first divergence."""
    say("case rl status")
    x0 = torch.full((4, 6, 8), 0.5, device="cuda")
    y = torch.ones((6, 8, 10), device="cuda")
    x, _, info = nd.rl_iterate(y, torch.zeros((3, 3, 3), device="cuda"), x0.clone(), 3)
    assert info.cpu().tolist() == [0, -1] and torch.equal(x, x0)
    y[2, 3, 4] = float("nan")
    x, st, info = nd.rl_iterate(y, torch.full((3, 3, 3), 1 / 27, device="cuda"), x0.clone(), 3)
    assert info.cpu().tolist() == [0, -4] and torch.equal(x, x0) and torch.isnan(st[0])
