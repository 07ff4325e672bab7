"""Differentiable form: ConvFull's hand-written backward against central
finite differences and the FP64 oracle's gradients, and sigma refinement of
a Gaussian PSF driven by it."""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ad():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1711_11224_amd.autograd as m
    return m


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def test_fd_fp64_8cube(ad):
    """Loss 1/2||X (x) H - Y||^2 is quadratic in X and in H, so central
    differences (eps 1e-3) are exact up to rounding."""
    say("case fd fp64 8^3")
    rng = np.random.default_rng(0)
    x = rng.random((8, 8, 8))
    h = rng.random((5, 3, 7))
    y = rng.random((12, 10, 14))
    xt = torch.tensor(x, device="cuda", requires_grad=True)
    ht = torch.tensor(h, device="cuda", requires_grad=True)
    loss = 0.5 * ((ad.conv_full_ad(xt, ht) - torch.tensor(y, device="cuda")) ** 2).sum()
    loss.backward()
    gx, gh = xt.grad.cpu().numpy(), ht.grad.cpu().numpy()
    L = lambda xx, hh: 0.5 * np.sum((oracle.conv_full(xx, hh) - y) ** 2)
    eps = 1e-3
    for idx in [(0, 0, 0), (3, 4, 5), (7, 7, 7), (2, 6, 1)]:
        xp, xm = x.copy(), x.copy()
        xp[idx] += eps
        xm[idx] -= eps
        assert abs((L(xp, h) - L(xm, h)) / (2 * eps) - gx[idx]) <= 1e-7 * max(1, abs(gx[idx]))
    for idx in [(0, 0, 0), (2, 1, 3), (4, 2, 6), (1, 0, 5)]:
        hp, hm = h.copy(), h.copy()
        hp[idx] += eps
        hm[idx] -= eps
        assert abs((L(x, hp) - L(x, hm)) / (2 * eps) - gh[idx]) <= 1e-7 * max(1, abs(gh[idx]))
    r = oracle.conv_full(x, h) - y
    assert rel_l2(gx, oracle.conv_adjoint(r, h)) <= 1e-12
    assert rel_l2(gh, oracle.conv_dH(x, r, h.shape)) <= 1e-12


def test_fp32_gradients_vs_oracle_and_fd(ad):
    """FP32 kernels: within 1e-5 of the FP64 oracle's gradient and 1e-4 of
    FP64 central differences on an 8^3 crop."""
    say("case fd fp32 8^3")
    rng = np.random.default_rng(1)
    x = rng.random((8, 8, 8)).astype(np.float32)
    h = synth.gaussian_psf((7, 5, 5), (1.5, 1.0, 1.2)).astype(np.float32)
    y = (oracle.conv_full(x, h) + 0.1 * rng.standard_normal((14, 12, 12))).astype(np.float32)
    xt = torch.tensor(x, device="cuda", requires_grad=True)
    ht = torch.tensor(h, device="cuda", requires_grad=True)
    loss = 0.5 * ((ad.conv_full_ad(xt, ht) - torch.tensor(y, device="cuda")) ** 2).sum()
    loss.backward()
    r = oracle.conv_full(x, h) - y
    gx_o, gh_o = oracle.conv_adjoint(r, h), oracle.conv_dH(x, r, h.shape)
    assert rel_l2(xt.grad.cpu().numpy(), gx_o) <= 1e-5
    assert rel_l2(ht.grad.cpu().numpy(), gh_o) <= 1e-5
    xd, hd = x.astype(np.float64), h.astype(np.float64)
    L = lambda xx, hh: 0.5 * np.sum((oracle.conv_full(xx, hh) - y) ** 2)
    eps = 1e-3
    fd = []
    for idx in [(0, 0, 0), (3, 4, 5), (7, 2, 7)]:
        xp, xm = xd.copy(), xd.copy()
        xp[idx] += eps
        xm[idx] -= eps
        fd.append(((L(xp, hd) - L(xm, hd)) / (2 * eps), float(xt.grad[idx])))
    for idx in [(3, 2, 2), (0, 1, 4), (6, 4, 0)]:
        hp, hm = hd.copy(), hd.copy()
        hp[idx] += eps
        hm[idx] -= eps
        fd.append(((L(xd, hp) - L(xd, hm)) / (2 * eps), float(ht.grad[idx])))
    for want, got in fd:
        assert abs(got - want) <= 1e-4 * max(1.0, abs(want))


def test_c5_gradients_sampled(ad):
    """Differentiable workload size: 256x256x64 X, 21x21x41 PSF.  dX on
    sampled voxels and dH on sampled taps against the oracle."""
    cfg = synth.CONFIGS["c5_diff"]
    say("case c5 gradients")
    rng = np.random.default_rng(4)
    x = synth.make_objects(cfg).astype(np.float32)
    h = synth.psf_for(cfg).astype(np.float32)
    gup = rng.standard_normal([a + b - 1 for a, b in zip(cfg.shape, cfg.psf_shape)]).astype(np.float32)
    xt = torch.tensor(x, device="cuda", requires_grad=True)
    ht = torch.tensor(h, device="cuda", requires_grad=True)
    yt = ad.conv_full_ad(xt, ht)
    yt.backward(torch.tensor(gup, device="cuda"))
    iy = rng.choice(yt.numel(), 512, replace=False)
    assert rel_l2(yt.detach().cpu().numpy().ravel()[iy], oracle.conv_full_at(x, h, iy)) <= 1e-5
    ix = rng.choice(x.size, 512, replace=False)
    assert rel_l2(xt.grad.cpu().numpy().ravel()[ix], oracle.conv_adjoint_at(gup, h, ix)) <= 1e-5
    ih = rng.choice(h.size, 48, replace=False)
    assert rel_l2(ht.grad.cpu().numpy().ravel()[ih], oracle.conv_dH_at(x, gup, h.shape, ih)) <= 1e-5


def test_sigma_refinement(ad):
    """Blind refinement: with X known, Adam on log-sigma through ConvFull's
    dH backward moves the PSF widths from the guess toward the truth."""
    say("case sigma refinement")
    rng = np.random.default_rng(9)
    shape, psf = (24, 48, 48), (21, 15, 15)
    true_s, guess_s = (4.0, 2.5, 2.5), (3.0, 1.8, 2.0)
    x = rng.random(shape).astype(np.float32)
    h_true = synth.gaussian_psf(psf, true_s).astype(np.float32)
    y = torch.tensor(oracle.conv_full(x, h_true).astype(np.float32), device="cuda")
    xt = torch.tensor(x, device="cuda")
    model = ad.GaussianPSF(psf, guess_s)
    opt = torch.optim.Adam(model.parameters(), lr=0.05)
    err0 = np.abs(np.array(guess_s) - np.array(true_s)).max()
    losses = []
    for _ in range(60):
        opt.zero_grad()
        loss = 0.5 * ((ad.conv_full_ad(xt, model()) - y) ** 2).sum()
        loss.backward()
        opt.step()
        losses.append(float(loss.detach()))
    s = model.sigmas().detach().cpu().numpy()
    err = np.abs(s - np.array(true_s)).max()
    say("sigmas", s, "loss", losses[0], "->", losses[-1])
    assert losses[-1] < 0.05 * losses[0]
    assert err < 0.2 * err0


def _c5_data():
    """The differentiable workload: X 64x256x256, true PSF 41x21x21 with
    sigma (6, 2.5, 2.5) (z, y, x), Y = X (x) H plus Poisson and read noise.
    Y is in photon units (its noise-free part peaks at 500), so the object
    is returned in the same units: X scaled by the factor the noise model
    applied to the blurred image."""
    cfg = synth.CONFIGS["c5_diff"]
    x = synth.make_objects(cfg)
    h = synth.psf_for(cfg)
    b = oracle.conv_full_separable(x, synth.gaussian_factors(cfg.psf_shape, cfg.sigmas))
    y = synth.add_noise(b, cfg)
    x = x * (cfg.peak_photons / b.max())
    return cfg, x.astype(np.float32), h.astype(np.float32), y.astype(np.float32)


def test_c5_joint_refinement(ad):
    """Joint X and sigma refinement at the differentiable workload's size
    from the flat start and the guess sigma (5, 2, 2): 30 joint steps, each
    one forward with the hand-written dX / dH backward.  The loss falls by
    over 10x and every X stays non-negative; the sigmas it reaches are
    reported (the loss alone does not identify them from below, see
    JointRefiner)."""
    say("case c5 joint refinement")
    cfg, x, h, y = _c5_data()
    guess = tuple(cfg.extra["guess_sigmas"])
    yt = torch.tensor(y, device="cuda")
    x0 = torch.tensor(synth.flat_start(y, h, cfg.shape), dtype=torch.float32, device="cuda")
    model = ad.GaussianPSF(cfg.psf_shape, guess)
    ref = ad.JointRefiner(yt, x0, model, lr=0.02)
    losses = []
    for _ in range(30):
        losses.append(float(ref.step()))
        assert float(ref.x.min()) >= 0
    torch.cuda.synchronize()
    s = model.sigmas().detach().cpu().numpy()
    say("  joint: loss %.4e -> %.4e, sigmas %s (true %s)" % (losses[0], losses[-1], np.round(s, 3), cfg.sigmas))
    assert losses[-1] < 0.1 * losses[0]
    assert np.all(np.isfinite(s)) and np.all(s > 0)


def test_c5_sigma_refinement_known_object(ad):
    """At the same size, with X known (where sigma is identifiable), Adam on
    log sigma through ConvFull's dH backward cuts the sigma error by 5x or
    more from the guess (5, 2, 2) toward (6, 2.5, 2.5)."""
    say("case c5 sigma refinement, X known")
    cfg, x, h, y = _c5_data()
    guess = np.array(cfg.extra["guess_sigmas"])
    true = np.array(cfg.sigmas)
    yt, xt = torch.tensor(y, device="cuda"), torch.tensor(x, device="cuda")
    model = ad.GaussianPSF(cfg.psf_shape, tuple(guess))
    opt = torch.optim.Adam(model.parameters(), lr=0.03)
    losses = []
    for _ in range(60):
        opt.zero_grad()
        loss = 0.5 * ((ad.conv_full_ad(xt, model()) - yt) ** 2).sum()
        loss.backward()
        opt.step()
        losses.append(float(loss.detach()))
    s = model.sigmas().detach().cpu().numpy()
    err0, err = np.abs(guess - true).max(), np.abs(s - true).max()
    say("  known X: sigmas %s, error %.3f -> %.3f, loss %.4e -> %.4e" % (np.round(s, 3), err0, err, losses[0],
                                                                       losses[-1]))
    assert losses[-1] < losses[0]
    assert err <= 0.2 * err0
