"""Pins of the FP64 oracle against facts fixed by the paper and by
mathematics, never against the oracle itself.  CPU only.

Each test names the passage or identity it checks.  Integer-valued inputs
make the sums exact in double precision, so those comparisons are exact."""
import numpy as np
import pytest

import oracle
from tests.conftest import read_golden

RNG = np.random.default_rng(12345)


def _int_array(shape, lo=-4, hi=5, rng=RNG):
    return rng.integers(lo, hi, size=shape).astype(np.float64)


TINY_SHAPES = [
    # (m, p): n = 1..4, p_i = 0, m_i = 1 and 2p_i >= m_i all occur.
    ((5,), (2,)),
    ((1,), (3,)),
    ((3, 4), (1, 2)),
    ((2, 3), (3, 1)),
    ((4, 1), (0, 2)),
    ((3, 4, 5), (1, 2, 1)),
    ((2, 2, 3), (0, 1, 2)),
    ((1, 3, 2), (2, 0, 1)),
    ((2, 1, 3, 2), (1, 0, 2, 1)),
]


# ---------------------------------------------------------------- Property 1
def test_eq1_golden_2d(golden):
    """Eq. 1 written out by hand (block Toeplitz of (S1) bands) equals both
    the recursive builder and the convolution applied to unit vectors."""
    g = golden("eq1_block_toeplitz_2d.txt")
    A_ref = np.array([[float(v) for v in r.split()] for r in g["main"]])
    H = np.array([[2, 3, 5], [7, 11, 13], [17, 19, 23]], dtype=np.float64)
    A = oracle.explicit_A((2, 2), H)
    assert A.shape == (16, 4)
    np.testing.assert_array_equal(A, A_ref)
    for c in range(4):
        e = np.zeros(4)
        e[c] = 1.0
        np.testing.assert_array_equal(oracle.conv_full(e.reshape(2, 2), H).ravel(), A_ref[:, c])


def test_s1_s8_golden_1d(golden):
    """(S1) and its transpose (S8) for n = 1."""
    g = golden("s1_s8_banded_1d.txt")
    S1 = np.array([[float(v) for v in r.split()] for r in g["S1"]])
    S8 = np.array([[float(v) for v in r.split()] for r in g["S8"]])
    h = np.array([2.0, 3.0, 5.0])
    np.testing.assert_array_equal(oracle.explicit_A((4,), h), S1)
    np.testing.assert_array_equal(S1.T, S8)
    y = np.array([1.0, -2.0, 3.0, 4.0, -5.0, 6.0])
    np.testing.assert_array_equal(oracle.conv_adjoint(y, h), S8 @ y)


@pytest.mark.parametrize("m,p", TINY_SHAPES)
def test_O1_full_conv_equals_explicit_A(m, p):
    """Y^v = A_n^h X^v (Eq. 1) with A from the block recursion, exact."""
    h = _int_array([2 * q + 1 for q in p])
    x = _int_array(m)
    y = oracle.conv_full(x, h)
    assert y.shape == tuple(a + 2 * b for a, b in zip(m, p))
    A = oracle.explicit_A(m, h)
    np.testing.assert_array_equal(A @ x.ravel(), y.ravel())


@pytest.mark.parametrize("m,p", TINY_SHAPES)
def test_O2_adjoint_is_transpose(m, p):
    """(A_n^h)^T applied to Y (Property 2's left side), exact on integers,
    plus <Ax, y> = <x, A^T y> on random reals.  H is asymmetric so a
    missing flip cannot pass."""
    h = _int_array([2 * q + 1 for q in p])
    r = _int_array([a + 2 * b for a, b in zip(m, p)])
    A = oracle.explicit_A(m, h)
    g = oracle.conv_adjoint(r, h)
    assert g.shape == tuple(m)
    np.testing.assert_array_equal(A.T @ r.ravel(), g.ravel())
    xr = RNG.standard_normal(m)
    yr = RNG.standard_normal(r.shape)
    hr = RNG.standard_normal(h.shape)
    lhs = float(np.sum(oracle.conv_full(xr, hr) * yr))
    rhs = float(np.sum(xr * oracle.conv_adjoint(yr, hr)))
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))


@pytest.mark.parametrize("m,p", TINY_SHAPES)
def test_O3_property2_literal_crop(m, p):
    """Eq. 2 literally (convolve with H~, extent m+4p, crop at 2p) equals the
    transpose; the uncropped result equals the extended transpose (S9),
    i.e. the full-convolution matrix of H~ applied to Y."""
    h = _int_array([2 * q + 1 for q in p])
    r = _int_array([a + 2 * b for a, b in zip(m, p)])
    g_lit, ext = oracle.conv_adjoint_literal(r, h, return_extended=True)
    assert ext.shape == tuple(a + 4 * b for a, b in zip(m, p))
    np.testing.assert_array_equal(g_lit, oracle.conv_adjoint(r, h))
    hf = h[tuple(slice(None, None, -1) for _ in h.shape)]
    A_ext = oracle.explicit_A(r.shape, hf)
    np.testing.assert_array_equal(A_ext @ r.ravel(), ext.ravel())


# ---------------------------------------------------------------- library special cases
@pytest.mark.parametrize("m,p", [((7, 9), (2, 3)), ((5, 6, 4), (1, 2, 1)), ((3, 3, 3), (2, 2, 2))])
def test_O4_scipy_direct(m, p):
    from scipy import signal
    h = RNG.standard_normal([2 * q + 1 for q in p])
    x = RNG.standard_normal(m)
    y = oracle.conv_full(x, h)
    np.testing.assert_allclose(y, signal.convolve(x, h, mode="full", method="direct"), rtol=0, atol=1e-12)
    r = RNG.standard_normal(y.shape)
    np.testing.assert_allclose(oracle.conv_adjoint(r, h), signal.correlate(r, h, mode="valid", method="direct"),
                               rtol=0, atol=1e-12)


def test_O12_fft_crosscheck_medium():
    """A larger 3-D case against an FFT (test-only), ~1e-12."""
    m, p = (12, 20, 24), (3, 4, 5)
    h = RNG.standard_normal([2 * q + 1 for q in p])
    x = RNG.standard_normal(m)
    y = oracle.conv_full(x, h)
    shp = y.shape
    ax = (0, 1, 2)
    yf = np.fft.irfftn(np.fft.rfftn(x, shp, axes=ax) * np.fft.rfftn(h, shp, axes=ax), shp, axes=ax)
    assert np.max(np.abs(y - yf)) <= 1e-11 * np.max(np.abs(y))
    r = RNG.standard_normal(shp)
    # correlation: G[k] = sum_j h[j] r[k+j] = (r conv flip(h))[k+2p]
    hf = h[::-1, ::-1, ::-1]
    big = [a + 2 * b for a, b in zip(shp, h.shape)]
    full = np.fft.irfftn(np.fft.rfftn(r, big, axes=ax) * np.fft.rfftn(hf, big, axes=ax), big, axes=ax)
    sl = tuple(slice(2 * q, 2 * q + a) for q, a in zip(p, m))
    g = oracle.conv_adjoint(r, h)
    assert np.max(np.abs(g - full[sl])) <= 1e-11 * np.max(np.abs(g))


# ---------------------------------------------------------------- closed forms
def test_O5_delta_psf():
    x = _int_array((4, 5, 6))
    p = (1, 2, 3)
    h = np.zeros([2 * q + 1 for q in p])
    h[p] = 1.0  # delta at the centre
    y = oracle.conv_full(x, h)
    np.testing.assert_array_equal(y, np.pad(x, [(q, q) for q in p]))
    r = _int_array(y.shape)
    np.testing.assert_array_equal(oracle.conv_adjoint(r, h), r[1:5, 2:7, 3:9])
    h0 = np.zeros_like(h)
    h0[0, 0, 0] = 1.0  # delta at index 0: Y[:m] = X, rest zero
    y0 = oracle.conv_full(x, h0)
    np.testing.assert_array_equal(y0[:4, :5, :6], x)
    assert np.count_nonzero(y0) == np.count_nonzero(x)


def test_O6_binomial_rows(golden):
    rows = golden("binomial_rows.txt")["rows"]
    for line in rows:
        _, xa, hb, want = [s.split() for s in line.split("|")]
        x = np.array([float(v) for v in xa])
        h = np.array([float(v) for v in hb])
        w = np.array([float(v) for v in want])
        np.testing.assert_array_equal(oracle.conv_full(x, h), w)
    # separable n-D products of binomials stay products of binomials
    c2, c4 = np.array([1.0, 2, 1]), np.array([1.0, 4, 6, 4, 1])
    c6 = np.array([1.0, 6, 15, 20, 15, 6, 1])
    x = np.einsum("i,j,k->ijk", c4, c2, c4)
    h = np.einsum("i,j,k->ijk", c2, c4, c2)
    np.testing.assert_array_equal(oracle.conv_full(x, h), np.einsum("i,j,k->ijk", c6, c6, c6))


def test_O7_mass_and_moments_add():
    x = RNG.random((6, 7, 8))
    h = RNG.random((3, 5, 7))
    y = oracle.conv_full(x, h)
    assert abs(y.sum() - x.sum() * h.sum()) <= 1e-12 * y.sum()
    for ax in range(3):
        def mom(a):
            other = tuple(i for i in range(3) if i != ax)
            w = a.sum(axis=other)
            t = np.arange(w.size, dtype=np.float64)
            mu = (w * t).sum() / w.sum()
            return mu, (w * (t - mu) ** 2).sum() / w.sum()
        mx, vx = mom(x)
        mh, vh = mom(h)
        my, vy = mom(y)
        assert abs(my - (mx + mh)) <= 1e-12 * my
        assert abs(vy - (vx + vh)) <= 1e-11 * vy


def test_O8_separable_equals_nd():
    fz, fy, fx = RNG.random(5), RNG.random(3), RNG.random(7)
    h = np.einsum("i,j,k->ijk", fz, fy, fx)
    x = RNG.standard_normal((6, 5, 9))
    a = oracle.conv_full(x, h)
    b = oracle.conv_full_separable(x, [fz, fy, fx])
    assert np.max(np.abs(a - b)) <= 1e-13 * np.max(np.abs(a))


# ---------------------------------------------------------------- sampled evaluation
def test_at_functions_match_dense():
    x = RNG.standard_normal((5, 6, 7))
    h = RNG.standard_normal((3, 5, 3))
    y = oracle.conv_full(x, h)
    idx = RNG.choice(y.size, 50, replace=False)
    np.testing.assert_array_equal(oracle.conv_full_at(x, h, idx), y.ravel()[idx])
    g = oracle.conv_adjoint(y, h)
    idx = RNG.choice(g.size, 40, replace=False)
    np.testing.assert_array_equal(oracle.conv_adjoint_at(y, h, idx), g.ravel()[idx])
    dh = oracle.conv_dH(x, y, h.shape)
    idx = RNG.choice(dh.size, 20, replace=False)
    np.testing.assert_array_equal(oracle.conv_dH_at(x, y, h.shape, idx), dh.ravel()[idx])


# ---------------------------------------------------------------- gradient in H
def test_O13_dH_is_transpose_of_conv_in_H():
    """Convolution commutes: Y = A_X vec(H), so the H-gradient is A_X^T R.
    X has odd extents so it can serve as the template of explicit_A."""
    x = _int_array((3, 5))
    h = _int_array((5, 3))
    r = _int_array((3 + 4, 5 + 2))
    dh = oracle.conv_dH(x, r, h.shape)
    A_x = oracle.explicit_A(h.shape, x)  # acts on vec(H)
    np.testing.assert_array_equal(A_x @ h.ravel(), oracle.conv_full(x, h).ravel())
    np.testing.assert_array_equal(A_x.T @ r.ravel(), dh.ravel())


def test_O13_dH_central_differences():
    """The loss is quadratic in H, so a central difference is exact up to
    rounding."""
    x = RNG.random((4, 5, 6))
    h = RNG.random((3, 3, 5))
    y = RNG.random((6, 7, 10))
    r = oracle.conv_full(x, h) - y
    dh = oracle.conv_dH(x, r, h.shape)
    eps = 1e-3
    for j in [(0, 0, 0), (1, 2, 3), (2, 1, 4), (0, 2, 2)]:
        hp, hm = h.copy(), h.copy()
        hp[j] += eps
        hm[j] -= eps
        lp = 0.5 * np.sum((oracle.conv_full(x, hp) - y) ** 2)
        lm = 0.5 * np.sum((oracle.conv_full(x, hm) - y) ** 2)
        assert abs((lp - lm) / (2 * eps) - dh[j]) <= 1e-8 * max(1.0, abs(dh[j]))


# ---------------------------------------------------------------- the iteration
def test_O9_eq6_literal_equals_fused():
    x_true = RNG.random((6, 7))
    h = RNG.random((3, 5))
    y = oracle.conv_full(x_true, h) + 0.01 * RNG.standard_normal((8, 11))
    x0 = np.full(x_true.shape, 0.5)
    xa, sa, da, _ = oracle.deconv(y, h, x0, 20)
    xb, sb, db, _ = oracle.deconv(y, h, x0, 20, literal_eq6=True)
    assert da == db == 20
    np.testing.assert_allclose(xa, xb, rtol=0, atol=1e-12)
    np.testing.assert_allclose(sa[:, 0], sb[:, 0], rtol=1e-12)


def test_O10_converges_to_nnls_and_kkt():
    from scipy.optimize import nnls
    m, hs = (4, 5), (3, 3)
    h = RNG.random(hs) + 0.1
    x_true = np.maximum(RNG.standard_normal(m), 0)
    y = oracle.conv_full(x_true, h) + 0.05 * RNG.standard_normal((6, 7))
    x, stats, done, status = oracle.deconv(y, h, np.zeros(m), 4000)
    assert status in (0, 1)
    assert np.all(x >= 0)
    f = stats[:, 0]
    assert np.all(np.diff(f[: done + 1]) < 0)  # strict decrease on every accepted step
    A = oracle.explicit_A(m, h)
    x_ref, _ = nnls(A, y.ravel())
    assert np.linalg.norm(x.ravel() - x_ref) <= 1e-6 * max(1.0, np.linalg.norm(x_ref))
    g = A.T @ (A @ x.ravel() - y.ravel())
    act = x.ravel() <= 1e-12
    assert np.all(g[act] >= -1e-6)
    assert np.all(np.abs(g[~act]) <= 1e-6)


@pytest.mark.parametrize("lam", [0.0, 0.5])
def test_O11_delta_psf_one_step(lam):
    """Delta PSF: A^T A = I, delta_0 = 1/(1+lam), X^0 = 0, so one step gives
    max(crop_p(Y)/(1+lam), 0) exactly."""
    p = (1, 2)
    h = np.zeros((3, 5))
    h[p] = 1.0
    y = _int_array((5, 8))
    x, stats, done, _ = oracle.deconv(y, h, np.zeros((3, 4)), 1, lam=lam)
    assert done == 1
    np.testing.assert_array_equal(x, np.maximum(y[1:4, 2:6] / (1.0 + lam), 0))
    assert stats[1, 1] == 1.0 / (1.0 + lam)


def test_deconv_stops_at_stationary_point():
    """Y = A X^0 exactly gives f(X^0) = 0: no strict decrease is possible."""
    h = _int_array((3, 3), 1, 4)
    x0 = _int_array((4, 4), 0, 3)
    y = oracle.conv_full(x0, h)
    x, stats, done, status = oracle.deconv(y, h, x0, 5)
    assert done == 0 and status == 1
    np.testing.assert_array_equal(x, x0)


def test_deconv_nonfinite_stops():
    h = np.ones((3, 3)) / 9
    y = np.ones((6, 6))
    y[2, 2] = np.nan
    _, _, done, status = oracle.deconv(y, h, np.zeros((4, 4)), 3)
    assert done == 0 and status == 2


def test_deconv_replay_matches_search():
    x_true = RNG.random((5, 6))
    h = RNG.random((3, 3))
    y = oracle.conv_full(x_true, h)
    x0 = np.full((5, 6), 0.3)
    xa, sa, da, _ = oracle.deconv(y, h, x0, 10)
    xb, sb, db, _ = oracle.deconv(y, h, x0, 10, deltas=sa[1:, 1])
    np.testing.assert_array_equal(xa, xb)


# ---- step-size rules (first trial of an iteration; halving as before) ----

def _grad(x, y, h, lam):
    return oracle.conv_adjoint(oracle.conv_full(x, h) - y, h) + lam * x


@pytest.mark.parametrize("lam,mu", [(0.0, 0.0), (0.3, 0.0), (0.0, 0.4), (0.3, 0.05)])
def test_cauchy_trial_minimises_along_the_gradient(lam, mu):
    """Away from the bound the Cauchy trial is the exact minimiser of
    f(X - t g) over t: the directional derivative vanishes there and nearby
    t give larger f.  With mu > 0 the objective and gradient carry the
    Laplacian term, so the minimiser needs its mu ||L g||^2 in the
    denominator."""
    rng = np.random.default_rng(21)
    h = rng.random((3, 5, 3))
    y = oracle.conv_full(50.0 + rng.random((4, 9, 7)), h)
    x = 50.0 + rng.random((4, 9, 7))          # far above 0: no clipping
    g = oracle.gradient(x, y, h, lam, mu)
    d = oracle.first_trial("cauchy", g, h, lam, oracle.initial_delta(h, lam, mu), mu=mu)
    xt = x - d * g
    assert xt.min() > 0
    slope = float(np.sum(g * oracle.gradient(xt, y, h, lam, mu)))
    assert abs(slope) <= 1e-10 * float(np.sum(g * g))
    f = oracle.objective(xt, y, h, lam, mu)
    for t in (0.5, 0.9, 0.99, 1.01, 1.1, 2.0):
        assert oracle.objective(x - t * d * g, y, h, lam, mu) > f


@pytest.mark.parametrize("lam,mu", [(0.0, 0.0), (0.2, 0.0), (0.0, 0.3), (0.2, 0.3)])
def test_cauchy_trial_is_the_dense_rayleigh_quotient(lam, mu):
    """The Cauchy trial equals <g,g> / g^T (A^T A + lam I + mu L^T L) g with
    A and L built as dense matrices by the block recursion of Property 1
    (explicit_A), so no convolution routine enters the reference value."""
    rng = np.random.default_rng(25)
    m = (3, 4, 5)
    h = rng.random((3, 3, 5))
    g = rng.standard_normal(m)
    A = oracle.explicit_A(m, h)
    L = oracle.explicit_A(m, oracle.laplacian(3))
    gv = g.ravel()
    hess = A.T @ A + lam * np.eye(gv.size) + mu * L.T @ L
    ref = float(gv @ gv) / float(gv @ hess @ gv)
    d = oracle.first_trial("cauchy", g, h, lam, oracle.initial_delta(h, lam, mu), mu=mu)
    assert abs(d - ref) <= 1e-12 * ref


@pytest.mark.parametrize("lam", [0.0, 0.3])
def test_bb_trial_is_the_secant_quotient(lam):
    """f is quadratic, so g(X1) - g(X0) = (A^T A + lam) (X1 - X0) for any two
    points: the BB quotient from gradient differences equals
    <s,s> / (||A s||^2 + lam ||s||^2) from a direct forward of s."""
    rng = np.random.default_rng(22)
    h = rng.random((1, 3, 5))
    y = oracle.conv_full(rng.random((3, 6, 8)), h)
    x0, x1 = rng.random((3, 6, 8)), rng.random((3, 6, 8))
    g0, g1 = _grad(x0, y, h, lam), _grad(x1, y, h, lam)
    s = x1 - x0
    d = oracle.first_trial("bb", g1, h, lam, oracle.initial_delta(h, lam), s, g0)
    a_s = oracle.conv_full(s, h)
    ref = float(np.sum(s * s)) / (float(np.sum(a_s * a_s)) + lam * float(np.sum(s * s)))
    assert abs(d - ref) <= 1e-12 * ref


def test_bb_second_trial_is_first_cauchy_step():
    """With an unclipped first step s = -delta0 g0, the BB quotient of the
    second iteration reduces to the Cauchy trial at X^0."""
    rng = np.random.default_rng(23)
    h = rng.random((3, 3, 3))
    y = oracle.conv_full(50.0 + rng.random((4, 8, 8)), h)
    x0 = 50.0 + rng.random((4, 8, 8))
    _, sb, done, _ = oracle.deconv(y, h, x0, 2, rule="bb")
    _, sc, _, _ = oracle.deconv(y, h, x0, 1, rule="cauchy")
    assert done == 2 and sb[1, 2] == 0 and sb[2, 2] == 0
    assert sb[1, 1] == oracle.initial_delta(h)
    assert abs(sb[2, 1] - sc[1, 1]) <= 1e-12 * sc[1, 1]


@pytest.mark.parametrize("rule", ["cauchy", "bb"])
def test_step_rules_decrease_and_stay_nonnegative(rule):
    rng = np.random.default_rng(24)
    h = rng.random((3, 5, 5))
    y = oracle.conv_full(rng.random((4, 12, 12)), h) + 0.01
    x, st, done, status = oracle.deconv(y, h, np.full((4, 12, 12), 0.5), 12, rule=rule)
    assert done == 12 and status == 0
    assert np.all(np.diff(st[:, 0]) < 0)
    assert x.min() >= 0
    # faster than the fixed first trial on this problem
    _, sf, _, _ = oracle.deconv(y, h, np.full((4, 12, 12), 0.5), 12)
    assert st[-1, 0] < sf[-1, 0]


def test_bb_falls_back_without_curvature():
    h = np.ones((3, 3))
    g = np.ones((4, 4))
    d0 = oracle.initial_delta(h)
    assert oracle.first_trial("bb", g, h, 0.0, d0, np.zeros((4, 4)), g) == d0   # <s,y> = 0
    assert oracle.first_trial("bb", g, h, 0.0, d0, None, None) == d0            # first iteration
    assert oracle.first_trial("cauchy", np.zeros((4, 4)), h, 0.0, d0) == d0     # g = 0


# ---- Tikhonov-Miller (Laplacian) term mu/2 ||L X||^2 ----

def test_laplacian_stencil_is_the_second_difference():
    """In 1-D, (L x)[i] over the full extent is x[i-2] - 2 x[i-1] + x[i]
    (zero outside), i.e. the second difference centred at i-1."""
    x = RNG.random(9)
    lx = oracle.conv_full(x, oracle.laplacian(1))
    xp = np.concatenate([[0.0, 0.0], x, [0.0, 0.0]])
    ref = np.array([xp[i] - 2 * xp[i + 1] + xp[i + 2] for i in range(11)])
    np.testing.assert_allclose(lx, ref, rtol=0, atol=1e-15)
    l3 = oracle.laplacian(3)
    assert l3.sum() == 0 and np.array_equal(l3, l3[::-1, ::-1, ::-1]) and np.abs(l3).sum() == 12


@pytest.mark.parametrize("lam,mu", [(0.0, 0.2), (0.3, 0.05)])
def test_gradient_matches_finite_differences_with_laplacian(lam, mu):
    rng = np.random.default_rng(41)
    h = rng.random((3, 3, 5))
    x = rng.random((4, 5, 6))
    y = oracle.conv_full(rng.random((4, 5, 6)), h)
    g = oracle.gradient(x, y, h, lam, mu)
    v = rng.standard_normal(x.shape)
    eps = 1e-4
    fd = (oracle.objective(x + eps * v, y, h, lam, mu) - oracle.objective(x - eps * v, y, h, lam, mu)) / (2 * eps)
    assert abs(fd - float(np.sum(g * v))) <= 1e-7 * abs(fd)


def test_laplacian_regularised_solution_closed_form():
    """With the identity PSF the regularised objective is minimised by
    X* = (I + mu L^T L)^{-1} Y; L is built as the dense matrix of the full
    convolution (explicit_A, not conv_full) and Y is large enough that the
    bound X >= 0 stays inactive."""
    mu, m = 0.1, (5, 6)
    y = 10.0 + RNG.random(m)
    h = np.ones((1, 1))
    L = oracle.explicit_A(m, oracle.laplacian(2))
    xs = np.linalg.solve(np.eye(30) + mu * L.T @ L, y.ravel()).reshape(m)
    # the loop runs until f stops decreasing in FP64 (status 1): ||X - X*||
    # shrinks by (1 - delta_0) per step, about 1e-7 relative when it stops
    x, st, done, status = oracle.deconv(y, h, np.full(m, 5.0), 300, mu=mu)
    assert done >= 100 and status in (0, 1) and xs.min() > 0
    np.testing.assert_allclose(x, xs, rtol=1e-6, atol=0)


def test_initial_delta_bounds_the_curvature_with_laplacian():
    """delta_0 <= 1 / lambda_max(A^T A + lam I + mu L^T L) (dense check)."""
    rng = np.random.default_rng(42)
    m, lam, mu = (4, 5), 0.2, 0.3
    h = rng.random((3, 3))
    A = oracle.explicit_A(m, h)
    L = oracle.explicit_A(m, oracle.laplacian(2))
    top = np.linalg.eigvalsh(A.T @ A + lam * np.eye(20) + mu * L.T @ L).max()
    assert oracle.initial_delta(h, lam, mu) <= 1.0 / top


# ---- Richardson-Lucy with the same operators (the paper's comparison method) ----

def _rl_problem(rng, m=(4, 7, 9), k=(3, 3, 5), clean=False):
    h = rng.random(k) + 0.05
    x_true = rng.random(m) + 0.1
    y = oracle.conv_full(x_true, h)
    if not clean:
        y = rng.poisson(20.0 * y).astype(np.float64) / 20.0
    return y, h, x_true


def test_rl_normaliser_is_psf_sum():
    """A^T 1 = sum H at every voxel: every tap of the transpose lands inside
    Y's extent (Property 2), so the normaliser is a constant (exact on
    integers)."""
    h = RNG.integers(0, 5, (3, 5, 3)).astype(np.float64)
    n = oracle.conv_adjoint(np.ones((6 + 2, 7 + 4, 5 + 2)), h)
    assert n.shape == (6, 7, 5) and np.all(n == h.sum())


def test_rl_delta_psf_one_step():
    """With the delta PSF at its centre A X is X zero-padded by p, so one
    step from any positive X^0 gives the crop of Y."""
    rng = np.random.default_rng(61)
    h = np.zeros((3, 5, 3))
    h[1, 2, 1] = 1.0
    y = rng.random((6, 9, 7))
    x1, d = oracle.richardson_lucy(y, h, rng.random((4, 5, 5)) + 0.5, 1)
    np.testing.assert_allclose(x1, y[1:5, 2:7, 1:6], rtol=1e-15, atol=0)
    assert d[1] <= d[0]


def test_rl_conserves_flux():
    """sum X^{k+1} * sum H = sum of Y over the outputs A X^k reaches: the
    update redistributes exactly the observed counts."""
    rng = np.random.default_rng(62)
    y, h, _ = _rl_problem(rng)
    x0 = rng.random((4, 7, 9)) + 0.2
    for iters in (1, 2, 5):
        x, _ = oracle.richardson_lucy(y, h, x0, iters)
        assert abs(x.sum() * h.sum() - y.sum()) <= 1e-12 * y.sum()


def test_rl_true_object_is_a_fixed_point():
    """Noise-free data: Y / (A X*) = 1 on the support, A^T 1 / sum H = 1, so
    X* is returned unchanged."""
    rng = np.random.default_rng(63)
    y, h, x_true = _rl_problem(rng, clean=True)
    x1, d = oracle.richardson_lucy(y, h, x_true, 3)
    np.testing.assert_allclose(x1, x_true, rtol=1e-13, atol=0)
    assert abs(d[0]) <= 1e-12 * y.sum()


def test_rl_divergence_decreases_and_x_stays_nonnegative():
    """RL is an EM iteration for the Poisson likelihood: the I-divergence
    never increases and X stays non-negative."""
    rng = np.random.default_rng(64)
    y, h, _ = _rl_problem(rng, m=(5, 12, 12), k=(3, 5, 5))
    x, d = oracle.richardson_lucy(y, h, np.full((5, 12, 12), y.sum() / (h.sum() * 720)), 25)
    assert np.all(np.diff(d) <= 1e-12 * abs(d[0])) and d[-1] < d[0]
    assert x.min() >= 0


def test_rl_step_with_dense_operator():
    """One step against A built densely by the block recursion of Property 1
    (explicit_A, no convolution routine): X * A^T (Y / A X) / A^T 1."""
    rng = np.random.default_rng(65)
    m, k = (3, 4, 5), (3, 3, 3)
    y, h, _ = _rl_problem(rng, m=m, k=k)
    x0 = rng.random(m) + 0.3
    A = oracle.explicit_A(m, h)
    ax = A @ x0.ravel()
    ref = x0.ravel() * (A.T @ (y.ravel() / ax)) / (A.T @ np.ones(A.shape[0]))
    x1, d = oracle.richardson_lucy(y, h, x0, 1)
    np.testing.assert_allclose(x1.ravel(), ref, rtol=1e-13, atol=0)
    yv = y.ravel()
    pos = yv > 0
    dref = float(np.sum(yv[pos] * np.log(yv[pos] / ax[pos])) - yv.sum() + ax.sum())
    assert abs(d[0] - dref) <= 1e-12 * abs(dref)


def test_i_divergence_special_values():
    """0 log 0 = 0; a positive count where the model is 0 is infinite; equal
    arrays give 0."""
    assert oracle.i_divergence(np.array([0.0, 2.0]), np.array([1.0, 2.0])) == 1.0
    assert oracle.i_divergence(np.array([1.0]), np.array([0.0])) == np.inf
    assert oracle.i_divergence(np.array([3.0, 0.5]), np.array([3.0, 0.5])) == 0.0
