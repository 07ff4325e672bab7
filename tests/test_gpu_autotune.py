"""Kernel forms and the autotuner: every form the library can run a problem
with computes the same operator (oracle parity at the precision's
tolerance; the 4x4 tile's two x-block widths and the 32x32 tile's widths
bitwise alike), and the tuner installs and records its choice."""
import sys

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fp32": 1e-5, "bf16": 1e-2, "split_bf16": 1e-4}


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


CASES = [((6, 40, 70), (3, 5, 7), "fp32"),      # small-PSF kernel, both tiles, general kernel
         ((5, 37, 130), (3, 9, 21), "fp32"),    # both tile widths, ragged tails
         ((6, 70, 150), (5, 13, 31), "bf16"),   # 4x4 and 32x32 bf16 tiles, every width
         ((6, 70, 150), (5, 13, 31), "split_bf16")]


@pytest.mark.parametrize("m,k,prec", CASES)
def test_every_form_matches_the_oracle(at, m, k, prec):
    import paper_1711_11224_amd as nd
    say("case forms m=%s k=%s %s" % (m, k, prec))
    rng = np.random.default_rng(synth.stable_seed(m, k, prec))
    x = rng.random(m).astype(np.float32)
    h = rng.standard_normal(k).astype(np.float32)
    r = rng.standard_normal([a + b - 1 for a, b in zip(m, k)]).astype(np.float32)
    yo, go = oracle.conv_full(x, h), oracle.conv_adjoint(r, h)
    xt, ht, rt = (torch.from_numpy(v).cuda() for v in (x, h, r))
    taps = int(np.prod(k))
    seen = {}
    for form, param in at.conv_candidates(prec, taps):
        for op in at.OPS:
            try:
                at.set_form(m, k, op, form, param, prec)
            except nd.NdcError:
                continue
            assert at.current_form(m, k, op, prec) == (form, param)
            if op == "forward":
                out = nd.conv_full_nd(xt, ht, precision=prec).cpu().numpy()
                assert rel_l2(out, yo) <= TOL[prec], (form, param)
            else:
                out = nd.conv_adjoint_nd(rt, ht, precision=prec).cpu().numpy()
                assert rel_l2(out, go) <= TOL[prec], (form, param)
            seen.setdefault((op, form), []).append(out)
            at.set_form(m, k, op, "auto", 0, prec)
    # widths of one tile form differ only in how outputs are grouped
    for (op, form), outs in seen.items():
        if form in ("mfma4", "mfma32"):
            for o in outs[1:]:
                np.testing.assert_array_equal(o, outs[0])
    assert len(seen) >= 4


def test_override_reaches_the_deconvolution(at):
    """An installed form is used inside deconv_iterate too: 16x64 tiles give
    the same iterates bitwise as the default 32x32 tiles."""
    import paper_1711_11224_amd as nd
    say("case forms in deconvolution")
    rng = np.random.default_rng(5)
    m, k = (6, 40, 64), (5, 9, 9)
    h = synth.gaussian_psf(k, (1.0, 1.5, 1.5)).astype(np.float32)
    y = torch.from_numpy((oracle.conv_full(rng.random(m), h) + 0.01).astype(np.float32)).cuda()
    ht = torch.from_numpy(h).cuda()
    xa, sa, _ = nd.deconv_iterate(y, ht, torch.full(m, 0.3, device="cuda"), 5)
    for op in at.OPS:
        at.set_form(m, k, op, "mfma4", 16)
    xb, sb, _ = nd.deconv_iterate(y, ht, torch.full(m, 0.3, device="cuda"), 5)
    for op in at.OPS:
        at.set_form(m, k, op, "auto")
    assert torch.equal(xa, xb)


def test_tune_conv_installs_and_records(at, tmp_path):
    import paper_1711_11224_amd as nd
    say("case tune_conv")
    table = str(tmp_path / "t.json")
    m, k = (8, 64, 96), (5, 11, 11)
    res = at.tune_conv(m, k, "fp32", reps=2, table=table)
    for op in at.OPS:
        best, times = res[op]
        assert best == min(((f, int(p)) for f, p in (key.split("/") for key in times)),
                           key=lambda c: times["%s/%d" % c])
        assert at.current_form(m, k, op) == tuple(best)
    nd.lib.ndc_tile_override_clear()
    assert at.apply_table(table) == 2
    for op in at.OPS:
        assert at.current_form(m, k, op) == tuple(res[op][0])
    nd.lib.ndc_tile_override_clear()
