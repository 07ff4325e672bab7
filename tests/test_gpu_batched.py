"""Batched form: persistent launches over many volumes with their own
extents and PSFs, per-volume line searches, hipGraph replay, autotuner."""
import os
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
    import paper_1711_11224_amd.batched  # noqa: F401
    return m


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def same(a, b):
    """Bitwise equality that treats NaN as equal to NaN (row 0 of the stats
    holds NaN for the undefined step size and step length)."""
    return a.shape == b.shape and bool(torch.all((a == b) | (torch.isnan(a) & torch.isnan(b))))


def rel_l2(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


SMALL = [((6, 20, 70), (3, 5, 9)), ((9, 17, 33), (5, 3, 3)), ((4, 40, 64), (1, 7, 31)),
         ((12, 12, 12), (9, 9, 15)), ((3, 5, 130), (3, 3, 7)), ((7, 33, 20), (7, 33, 33))]


def small_batch(rng):
    xs, hs, ys = [], [], []
    for m, k in SMALL:
        xs.append(rng.random(m).astype(np.float32))
        hs.append(rng.standard_normal(k).astype(np.float32))
    return xs, hs


@pytest.mark.parametrize("tuning", [(4, 2, 0, 1), (2, 1, 1, 1), (4, 1, 2, 0)])
def test_batch_conv_vs_oracle(nd, tuning):
    say("case batch conv", tuning)
    rng = np.random.default_rng(10)
    xs, hs = small_batch(rng)
    plan = nd.batched.BatchPlan([m for m, _ in SMALL], [k for _, k in SMALL], tuning=tuning)
    gx = [torch.from_numpy(x).cuda() for x in xs]
    gh = [torch.from_numpy(h).cuda() for h in hs]
    ys = plan.conv_full(gx, gh)
    rs = [np.random.default_rng(i).standard_normal(tuple(y.shape)).astype(np.float32) for i, y in enumerate(ys)]
    gs = plan.conv_adjoint([torch.from_numpy(r).cuda() for r in rs], gh)
    for v, (x, h) in enumerate(zip(xs, hs)):
        assert rel_l2(ys[v].cpu().numpy(), oracle.conv_full(x, h)) <= 1e-5
        assert rel_l2(gs[v].cpu().numpy(), oracle.conv_adjoint(rs[v], h)) <= 1e-5
    plan.close()


def mfma_path(psf):
    """The single-volume call takes the matrix-core tile (same sums, same
    order as the batched tile) unless every PSF axis is <= 7, where the
    streaming small-PSF kernel sums in another order."""
    return max(psf) > 7


def test_batch_conv_equals_single_volume_bitwise(nd):
    """The batched operators run each volume's single-volume kernel (on the
    plan's side streams), so every output, small-PSF volumes included, is
    bitwise equal to a single-volume call on the caller's stream; the
    tuning (which shapes only the deconvolution's persistent launches) does
    not change that."""
    say("case batch == single")
    rng = np.random.default_rng(11)
    xs, hs = small_batch(rng)
    gx = [torch.from_numpy(x).cuda() for x in xs]
    gh = [torch.from_numpy(h).cuda() for h in hs]
    assert any(not mfma_path(k) for _, k in SMALL) and any(mfma_path(k) for _, k in SMALL)
    for tuning in ((4, 2, 1, 1), (2, 1, 0, 0)):
        plan = nd.batched.BatchPlan([m for m, _ in SMALL], [k for _, k in SMALL], tuning=tuning)
        ys = plan.conv_full(gx, gh)
        gs = plan.conv_adjoint(ys, gh)
        for v in range(len(SMALL)):
            assert torch.equal(ys[v], nd.conv_full_nd(gx[v], gh[v])), (tuning, v)
            assert torch.equal(gs[v], nd.conv_adjoint_nd(ys[v], gh[v])), (tuning, v)
        plan.close()


def _deconv_inputs(rng, specs):
    ys, hs, x0s = [], [], []
    for m, k in specs:
        h = synth.gaussian_psf(k, tuple(0.3 * e for e in k)).astype(np.float32)
        xt = rng.random(m)
        y = (oracle.conv_full(xt, h) + 0.02 * rng.standard_normal([a + b - 1 for a, b in zip(m, k)]))
        ys.append(y.astype(np.float32))
        hs.append(h)
        x0s.append(np.full(m, 0.4, dtype=np.float32))
    return ys, hs, x0s


# the persistent tile, and each volume's own kernels on the plan's streams
STEP_FORMS = [(4, 2, 0), (0, 1, 0)]


@pytest.mark.parametrize("form", STEP_FORMS)
def test_batch_deconv_vs_oracle_and_single(nd, form):
    say("case batch deconv", form)
    rng = np.random.default_rng(12)
    specs = SMALL[:4]
    ys, hs, x0s = _deconv_inputs(rng, specs)
    plan = nd.batched.BatchPlan([m for m, _ in specs], [k for _, k in specs], tuning=form + (1,))
    gy = [torch.from_numpy(a).cuda() for a in ys]
    gh = [torch.from_numpy(a).cuda() for a in hs]
    gx = [torch.from_numpy(a).cuda() for a in x0s]
    xs, stats, info = plan.deconv(gy, gh, gx, 8, lam=0.1)
    info = info.cpu().numpy()
    for v in range(len(specs)):
        xo, so, done, status = oracle.deconv(ys[v], hs[v], x0s[v], 8, lam=0.1)
        assert info[v].tolist() == [done, status]
        st = stats[v].cpu().numpy()
        np.testing.assert_array_equal(st[1:done + 1, 2], so[1:done + 1, 2])
        assert rel_l2(xs[v].cpu().numpy(), xo) <= 1e-5
        assert np.all(np.abs(st[:done + 1, 0] - so[:done + 1, 0]) <= 1e-5 * np.abs(so[:done + 1, 0]))
        # X bitwise equal to the single-volume path (every output is the same sum
        # in the same order); f is summed over that path's own tile partition
        x1, st1, inf1 = nd.deconv_iterate(gy[v], gh[v], torch.from_numpy(x0s[v]).cuda(), 8, lam=0.1)
        if mfma_path(specs[v][1]) or form[0] == 0:
            assert torch.equal(x1, xs[v])
            np.testing.assert_allclose(st1.cpu().numpy(), stats[v].cpu().numpy(), rtol=1e-12, equal_nan=True)
        else:
            assert rel_l2(x1.cpu().numpy(), xs[v].cpu().numpy()) <= 1e-6
    plan.close()


@pytest.mark.parametrize("form", STEP_FORMS)
def test_batch_graph_replays_equal_eager(nd, form):
    """The hipGraph-captured step replayed many times, with eager work and
    synchronisations between calls, gives bitwise the same result as the
    same kernels launched one by one."""
    say("case batch graph vs eager", form)
    rng = np.random.default_rng(13)
    specs = SMALL[:3]
    for trial in range(2):
        ys, hs, x0s = _deconv_inputs(rng, specs)
        out = {}
        for graph in (1, 0):
            plan = nd.batched.BatchPlan([m for m, _ in specs], [k for _, k in specs], tuning=form + (graph,))
            gx = [torch.from_numpy(a).cuda() for a in x0s]
            xs, stats, info = plan.deconv([torch.from_numpy(a).cuda() for a in ys],
                                          [torch.from_numpy(a).cuda() for a in hs], gx, 6)
            torch.cuda.synchronize()
            _ = (torch.ones(1000, device="cuda") * 2).sum().item()  # unrelated eager work between replays
            out[graph] = ([x.clone() for x in xs], [s.clone() for s in stats], info.clone())
            plan.close()
        for a, b in zip(out[1][0], out[0][0]):
            assert torch.equal(a, b)
        for a, b in zip(out[1][1], out[0][1]):
            assert same(a, b)
        assert torch.equal(out[1][2], out[0][2])


@pytest.mark.parametrize("form", STEP_FORMS)
def test_batch_calls_capture_into_a_graph(nd, form):
    """ndc_batch_deconv and the batched operators enqueue work only, so a
    caller can capture them; replays from the same X^0 (restored eagerly in
    between) equal eager calls bitwise."""
    say("case batch capture", form)
    rng = np.random.default_rng(14)
    specs = SMALL[:3]
    ys, hs, x0s = _deconv_inputs(rng, specs)
    plan = nd.batched.BatchPlan([m for m, _ in specs], [k for _, k in specs], tuning=form + (1,))
    gy = [torch.from_numpy(a).cuda() for a in ys]
    gh = [torch.from_numpy(a).cuda() for a in hs]
    x0 = [torch.from_numpy(a).cuda() for a in x0s]
    xe, se, ie = plan.deconv(gy, gh, [a.clone() for a in x0], 5)
    ye = plan.conv_full(xe, gh)
    torch.cuda.synchronize()
    xe, se, ie, ye = [a.clone() for a in xe], [a.clone() for a in se], ie.clone(), [a.clone() for a in ye]
    xs = [a.clone() for a in x0]
    yo = [torch.empty_like(a) for a in ye]
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            _, stats, info = plan.deconv(gy, gh, xs, 5)
            plan.conv_full(xs, gh, ys=yo)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        for a, b in zip(xs, x0):
            a.copy_(b)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(info, ie), rep
        for a, b in zip(xs, xe):
            assert torch.equal(a, b), rep
        for a, b in zip(stats, se):
            assert same(a, b), rep
        for a, b in zip(yo, ye):
            assert torch.equal(a, b), rep
    del g
    torch.cuda.synchronize()
    plan.close()


def test_batch_step_graph_follows_new_arrays(nd):
    """With the volumes' own kernels the step graph carries the call's
    addresses and lambda: one plan called on two sets of arrays and two
    lambdas, alternately, matches a plan without the graph on every call."""
    say("case batch graph recapture")
    rng = np.random.default_rng(15)
    specs = SMALL[:3]
    shapes, psfs = [m for m, _ in specs], [k for _, k in specs]
    sets = []
    for _ in range(2):
        ys, hs, x0s = _deconv_inputs(rng, specs)
        sets.append(([torch.from_numpy(a).cuda() for a in ys], [torch.from_numpy(a).cuda() for a in hs], x0s))
    plan = nd.batched.BatchPlan(shapes, psfs, tuning=(0, 1, 0, 1))
    ref = nd.batched.BatchPlan(shapes, psfs, tuning=(0, 1, 0, 0))
    for call, (si, lam) in enumerate([(0, 0.0), (1, 0.0), (0, 0.0), (0, 0.05), (1, 0.05)]):
        gy, gh, x0s = sets[si]
        xa, sa, ia = plan.deconv(gy, gh, [torch.from_numpy(a).cuda() for a in x0s], 4, lam=lam)
        xb, sb, ib = ref.deconv(gy, gh, [torch.from_numpy(a).cuda() for a in x0s], 4, lam=lam)
        torch.cuda.synchronize()
        assert torch.equal(ia, ib), call
        for a, b in zip(xa, xb):
            assert torch.equal(a, b), call
        for a, b in zip(sa, sb):
            assert same(a, b), call
    plan.close()
    ref.close()


@pytest.mark.parametrize("form", STEP_FORMS)
def test_batched_workload_64_volumes(nd, form):
    """The batched workload: 64 volumes of 32^3 .. 96x160x160 with their own
    Gaussian PSFs (odd extents 9..31 per axis), 50 steps in one plan with
    the hipGraph, in both step forms (the bench's tuning takes the volumes'
    own kernels).  Every volume runs all steps with f strictly decreasing
    and X >= 0; three volumes are rerun alone and must match bitwise."""
    cfgs = synth.batched_configs(64)
    say("case c4 batched 64", form)
    ys, hs, x0s = [], [], []
    for c in cfgs:
        x = synth.make_objects(c)
        fac = synth.gaussian_factors(c.psf_shape, c.sigmas)
        h = synth.gaussian_psf(c.psf_shape, c.sigmas).astype(np.float32)
        y = synth.add_noise(oracle.conv_full_separable(x, fac), c).astype(np.float32)
        ys.append(torch.from_numpy(y).cuda())
        hs.append(torch.from_numpy(h).cuda())
        x0s.append(synth.flat_start(y, h, c.shape).astype(np.float32))
    plan = nd.batched.BatchPlan([c.shape for c in cfgs], [c.psf_shape for c in cfgs],
                                tuning=(4, 2, 2, 1) if form[0] else (0, 1, 0, 1))
    xs = [torch.from_numpy(a).cuda() for a in x0s]
    xs, stats, info = plan.deconv(ys, hs, xs, 50)
    info = info.cpu().numpy()
    assert np.all(info[:, 0] == 50) and np.all(info[:, 1] == 0)
    for v in range(64):
        f = stats[v].cpu().numpy()[:, 0]
        assert np.all(np.diff(f) < 0)
        assert float(xs[v].min()) >= 0
    for v in (0, 17, 63):
        x1, st1, _ = nd.deconv_iterate(ys[v], hs[v], torch.from_numpy(x0s[v]).cuda(), 50)
        assert torch.equal(x1, xs[v])
    plan.close()


def test_batched_workload_64_volumes_operators_sampled(nd):
    """The batched workload's operators (64 volumes, 32^3 .. 96x160x160,
    PSFs 9..31 per axis, the tuning the bench uses) against the oracle on
    256 sampled outputs of each operator in every volume, plus each
    volume's eight corner outputs (where the fewest taps are in range)."""
    cfgs = synth.batched_configs(64)
    say("case c4 batched 64 operators sampled")
    rng = np.random.default_rng(64)
    xs = [rng.random(c.shape).astype(np.float32) for c in cfgs]
    hs = [synth.gaussian_psf(c.psf_shape, c.sigmas).astype(np.float32) for c in cfgs]
    rs = [rng.standard_normal([a + b - 1 for a, b in zip(c.shape, c.psf_shape)]).astype(np.float32) for c in cfgs]
    plan = nd.batched.BatchPlan([c.shape for c in cfgs], [c.psf_shape for c in cfgs], tuning=(4, 2, 2, 1))
    gh = [torch.from_numpy(h).cuda() for h in hs]
    ys = plan.conv_full([torch.from_numpy(x).cuda() for x in xs], gh)
    gs = plan.conv_adjoint([torch.from_numpy(r).cuda() for r in rs], gh)
    torch.cuda.synchronize()
    for v, c in enumerate(cfgs):
        y, g = ys[v].cpu().numpy(), gs[v].cpu().numpy()
        for out, shape, fn, src in ((y, y.shape, oracle.conv_full_at, xs[v]), (g, g.shape, oracle.conv_adjoint_at, rs[v])):
            corners = np.ravel_multi_index(np.array(np.meshgrid(*[[0, e - 1] for e in shape], indexing="ij")).reshape(3, -1),
                                           shape)
            idx = np.concatenate([rng.choice(out.size, 256, replace=False), corners])
            assert rel_l2(out.ravel()[idx], fn(src, hs[v].astype(np.float64), idx)) <= 1e-5, (v, c.shape, c.psf_shape)
    plan.close()


def test_autotuner_table(nd, tmp_path):
    """The batch tuner stores the batch's tuning and each volume's kernel
    forms; plan_for installs those forms, and the batched operators then
    run them (bitwise equal to single-volume calls with the same forms)."""
    from paper_1711_11224_amd import autotune
    say("case autotune")
    specs = SMALL[:3]
    shapes, psfs = [m for m, _ in specs], [k for _, k in specs]
    table = str(tmp_path / "table.json")
    try:
        best, times = autotune.tune(shapes, psfs, candidates=[(4, 2, 0, 1), (2, 2, 1, 1), (4, 1, 2, 1), (0, 1, 0, 1)],
                                    table=table)
        assert best in times and times[best] == min(times.values())
        assert autotune.best_tuning(shapes, psfs, table=table) == best
        entries = autotune.load_table(table)
        stored = {}
        for m, k in specs:
            e = entries[autotune.conv_signature(m, k, "fp32", torch.float32)]
            stored[(m, k)] = tuple(tuple(e[op]["form"]) for op in autotune.OPS)
        nd.lib.ndc_tile_override_clear()
        plan = nd.batched.plan_for(shapes, psfs, table=table)
        assert plan.tuning == best
        for m, k in specs:
            assert tuple(autotune.current_form(m, k, op) for op in autotune.OPS) == stored[(m, k)]
        rng = np.random.default_rng(16)
        gx = [torch.from_numpy(rng.random(m).astype(np.float32)).cuda() for m, _ in specs]
        gh = [torch.from_numpy(rng.standard_normal(k).astype(np.float32)).cuda() for _, k in specs]
        ys = plan.conv_full(gx, gh)
        for v in range(len(specs)):
            assert torch.equal(ys[v], nd.conv_full_nd(gx[v], gh[v]))
        plan.close()
    finally:
        nd.lib.ndc_tile_override_clear()  # leave no forms installed for later tests


@pytest.mark.parametrize("tuning", [(4, 2, 2, 1), (2, 1, 0, 0)])
def test_batch_conv_random_volumes_vs_oracle(nd, tuning):
    """A seeded batch of 10 random volumes (extents 1..40 per axis, 2p >= m
    included) with their own PSFs (kx 3..33, ky <= 33) against the oracle."""
    say("case batch random", tuning)
    rng = np.random.default_rng(77)
    shapes, psfs = [], []
    for _ in range(10):
        shapes.append(tuple(int(rng.integers(1, 41)) for _ in range(3)))
        psfs.append((2 * int(rng.integers(0, 9)) + 1, 2 * int(rng.integers(0, 17)) + 1,
                     2 * int(rng.integers(1, 17)) + 1))
    xs = [rng.random(m).astype(np.float32) for m in shapes]
    hs = [rng.standard_normal(k).astype(np.float32) for k in psfs]
    plan = nd.batched.BatchPlan(shapes, psfs, tuning=tuning)
    gh = [torch.from_numpy(h).cuda() for h in hs]
    ys = plan.conv_full([torch.from_numpy(x).cuda() for x in xs], gh)
    rs = [np.random.default_rng(i).standard_normal(tuple(y.shape)).astype(np.float32) for i, y in enumerate(ys)]
    gs = plan.conv_adjoint([torch.from_numpy(r).cuda() for r in rs], gh)
    for v, (x, h) in enumerate(zip(xs, hs)):
        assert rel_l2(ys[v].cpu().numpy(), oracle.conv_full(x, h)) <= 1e-5
        assert rel_l2(gs[v].cpu().numpy(), oracle.conv_adjoint(rs[v], h)) <= 1e-5
    plan.close()
