"""FP64 CPU oracle for the paper's n-D full convolution, its transpose and the
projected-gradient deconvolution built from them.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code
with the HIP library and never imports it.

Source: "Properties on n-dimensional convolution for image deconvolution"
(arXiv 1711.11224).  Conventions: X has extent m_i, the PSF H has extent
2p_i+1 and Y = X (x) H has extent m_i+2p_i (Eq. 4); arrays are C order
(the row partitioning of {.}^v under Eq. 1).

Functions and the passage each follows:
  conv_full            Property 1 / (S2): y(s) = sum_k x(k) h(s-k)
  conv_adjoint         (A^h)^T y from the transposed banded matrix (S8)
  conv_adjoint_literal Property 2, Eq. 2: crop M_{2p} of Y (x) H~
  conv_dH              gradient of 1/2||X(x)H - Y||^2 in H (Property 1 with the
                       roles of X and H swapped)
  *_at                 the same sums at listed output indices only
  explicit_A           the matrix A_n^h of Eq. 1 built by the block recursion
                       of Property 1 (S1, S5, S10), independent of conv_full
  objective            f = 1/2||A X - Y||^2 (+ lam/2 ||X||^2), section
                       "Application to 2-dimensional deconvolution"
  deconv               Steps 1-3 with the step-size acceptance rule
                       f(X^{k+1}) < f(X^k), gradient by Eq. 6
  richardson_lucy      the maximum-likelihood (Richardson-Lucy) iteration
                       the paper compares against (Introduction; Fig. 2f),
                       built from the same two operators
  i_divergence         the Poisson negative log-likelihood it decreases

Readings where the paper is silent (initial step, shrink factor, the
regularisation weight) are stated in each docstring.
"""
import ctypes
import os

import numpy as np

from .build import LIB, build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            _build()
        lib = ctypes.CDLL(LIB)
        i64p = ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.POINTER(ctypes.c_double)
        for name in ("ora_conv_full", "ora_conv_adjoint", "ora_conv_dH"):
            f = getattr(lib, name)
            f.argtypes = [ctypes.c_int, i64p, i64p, dp, dp, dp]
            f.restype = ctypes.c_int
        lib.ora_conv_adjoint_literal.argtypes = [ctypes.c_int, i64p, i64p, dp, dp, dp, dp]
        lib.ora_conv_adjoint_literal.restype = ctypes.c_int
        for name in ("ora_conv_full_at", "ora_conv_adjoint_at", "ora_conv_dH_at"):
            f = getattr(lib, name)
            f.argtypes = [ctypes.c_int, i64p, i64p, dp, dp, i64p, ctypes.c_int64, dp]
            f.restype = ctypes.c_int
        lib.ora_threads.argtypes = []
        lib.ora_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t=ctypes.c_double):
    return a.ctypes.data_as(ctypes.POINTER(t))


def _mp(m, p):
    m = np.ascontiguousarray(m, dtype=np.int64)
    p = np.ascontiguousarray(p, dtype=np.int64)
    return m, p


def _psf_half(h):
    for e in h.shape:
        if e % 2 != 1:
            raise ValueError("PSF extents must be odd (2p_i+1), got %s" % (h.shape,))
    return [(e - 1) // 2 for e in h.shape]


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return _load().ora_threads()


def conv_full(x, h):
    """Y = X (x) H, the 'full' discrete convolution (Property 1, (S2), Eq. 4).

    x: extent m_i; h: extent 2p_i+1; returns extent m_i+2p_i, float64.
    Values outside X's box are zero (the banded matrix (S1) has no wrap)."""
    x, h = _d(x), _d(h)
    if x.ndim != h.ndim:
        raise ValueError("x and h must have the same number of axes")
    p = _psf_half(h)
    m, pp = _mp(x.shape, p)
    y = np.empty([a + 2 * b for a, b in zip(x.shape, p)], dtype=np.float64)
    rc = _load().ora_conv_full(x.ndim, _ptr(m, ctypes.c_int64), _ptr(pp, ctypes.c_int64),
                               _ptr(x), _ptr(h), _ptr(y))
    if rc:
        raise ValueError("ora_conv_full failed (%d)" % rc)
    return y


def conv_adjoint(r, h):
    """(A^h)^T r: G[k] = sum_{j in [0,2p]} H[j] R[k+j] (rows of (S8)).

    r: extent m_i+2p_i; returns extent m_i."""
    r, h = _d(r), _d(h)
    p = _psf_half(h)
    mm = [a - 2 * b for a, b in zip(r.shape, p)]
    if min(mm) < 1:
        raise ValueError("r must be at least as large as h on every axis")
    m, pp = _mp(mm, p)
    g = np.empty(mm, dtype=np.float64)
    rc = _load().ora_conv_adjoint(r.ndim, _ptr(m, ctypes.c_int64), _ptr(pp, ctypes.c_int64),
                                  _ptr(r), _ptr(h), _ptr(g))
    if rc:
        raise ValueError("ora_conv_adjoint failed (%d)" % rc)
    return g


def conv_adjoint_literal(r, h, return_extended=False):
    """Property 2 (Eq. 2) literally: convolve r with the flipped PSF
    H~(s) = H(2p-s) into the extended result of extent m_i+4p_i, then keep
    the window M_{2p}.  The paper's 1-based window 2p+1 .. m+2p+1 is read as
    0-based offset 2p_i and length m_i."""
    r, h = _d(r), _d(h)
    p = _psf_half(h)
    mm = [a - 2 * b for a, b in zip(r.shape, p)]
    if min(mm) < 1:
        raise ValueError("r must be at least as large as h on every axis")
    m, pp = _mp(mm, p)
    g = np.empty(mm, dtype=np.float64)
    ext = np.empty([a + 4 * b for a, b in zip(mm, p)], dtype=np.float64)
    rc = _load().ora_conv_adjoint_literal(r.ndim, _ptr(m, ctypes.c_int64), _ptr(pp, ctypes.c_int64),
                                          _ptr(r), _ptr(h), _ptr(g), _ptr(ext))
    if rc:
        raise ValueError("ora_conv_adjoint_literal failed (%d)" % rc)
    return (g, ext) if return_extended else g


def conv_dH(x, r, psf_shape):
    """dH[j] = sum_k X[k] R[k+j]: the gradient of 1/2||X (x) H - Y||^2 with
    respect to H when R = X (x) H - Y.  Convolution commutes, so this is
    A_X^T R (Property 1 with X as the template)."""
    x, r = _d(x), _d(r)
    p = [(e - 1) // 2 for e in psf_shape]
    for e in psf_shape:
        if e % 2 != 1:
            raise ValueError("PSF extents must be odd")
    if list(r.shape) != [a + 2 * b for a, b in zip(x.shape, p)]:
        raise ValueError("r must have extent m_i+2p_i")
    m, pp = _mp(x.shape, p)
    dh = np.empty(list(psf_shape), dtype=np.float64)
    rc = _load().ora_conv_dH(x.ndim, _ptr(m, ctypes.c_int64), _ptr(pp, ctypes.c_int64),
                             _ptr(x), _ptr(r), _ptr(dh))
    if rc:
        raise ValueError("ora_conv_dH failed (%d)" % rc)
    return dh


def conv_full_at(x, h, flat_idx):
    """Full convolution evaluated only at the given flat output indices."""
    x, h = _d(x), _d(h)
    p = _psf_half(h)
    m, pp = _mp(x.shape, p)
    idx = np.ascontiguousarray(flat_idx, dtype=np.int64)
    out = np.empty(idx.size, dtype=np.float64)
    rc = _load().ora_conv_full_at(x.ndim, _ptr(m, ctypes.c_int64), _ptr(pp, ctypes.c_int64),
                                  _ptr(x), _ptr(h), _ptr(idx, ctypes.c_int64), idx.size, _ptr(out))
    if rc:
        raise ValueError("ora_conv_full_at failed (%d)" % rc)
    return out


def conv_adjoint_at(r, h, flat_idx):
    """Transpose evaluated only at the given flat X-shaped indices."""
    r, h = _d(r), _d(h)
    p = _psf_half(h)
    mm = [a - 2 * b for a, b in zip(r.shape, p)]
    m, pp = _mp(mm, p)
    idx = np.ascontiguousarray(flat_idx, dtype=np.int64)
    out = np.empty(idx.size, dtype=np.float64)
    rc = _load().ora_conv_adjoint_at(r.ndim, _ptr(m, ctypes.c_int64), _ptr(pp, ctypes.c_int64),
                                     _ptr(r), _ptr(h), _ptr(idx, ctypes.c_int64), idx.size, _ptr(out))
    if rc:
        raise ValueError("ora_conv_adjoint_at failed (%d)" % rc)
    return out


def conv_dH_at(x, r, psf_shape, flat_idx):
    """conv_dH evaluated only at the given flat PSF-shaped indices."""
    x, r = _d(x), _d(r)
    p = [(e - 1) // 2 for e in psf_shape]
    m, pp = _mp(x.shape, p)
    idx = np.ascontiguousarray(flat_idx, dtype=np.int64)
    out = np.empty(idx.size, dtype=np.float64)
    rc = _load().ora_conv_dH_at(x.ndim, _ptr(m, ctypes.c_int64), _ptr(pp, ctypes.c_int64),
                                _ptr(x), _ptr(r), _ptr(idx, ctypes.c_int64), idx.size, _ptr(out))
    if rc:
        raise ValueError("ora_conv_dH_at failed (%d)" % rc)
    return out


def conv_full_separable(x, factors):
    """Full convolution with a separable PSF H = f_0 (outer) f_1 ... given as
    1-D factors: one full convolution per axis, each with a PSF that is 1 wide
    on every other axis.  Equal to conv_full(x, outer(factors)) up to rounding
    (pinned by test); used to make large test inputs in O(N sum K_i)."""
    y = _d(x)
    n = y.ndim
    if len(factors) != n:
        raise ValueError("one factor per axis")
    for ax, f in enumerate(factors):
        f = _d(f).reshape(-1)
        shape = [1] * n
        shape[ax] = f.size
        y = conv_full(y, f.reshape(shape))
    return y


def explicit_A(m, h):
    """The dense matrix A_n^h of Eq. 1 (shape prod(m+2p) x prod(m)), built by
    the block recursion of Property 1 and its proof:

      n = 1 : the banded Toeplitz matrix of (S1), column j holding h(0..2p)
              in rows j..j+2p;
      n > 1 : block (s_1, k_1) of A_n equals A_{n-1} built from the slice
              H[s_1-k_1, ...] when 0 <= s_1-k_1 <= 2p_1, else zero (Eq. 1,
              (S5), (S10)).  Written as sum_j S_j kron A_{n-1}(H[j,...]) where
              S_j is the (m_1+2p_1) x m_1 shift matrix with ones at (r+j, r).

    It never calls conv_full: it is the independent check of the indexing."""
    h = _d(h)
    m = list(m)
    if h.ndim != len(m):
        raise ValueError("h and m must agree on the number of axes")
    p = _psf_half(h)
    m1, p1 = m[0], p[0]
    if h.ndim == 1:
        A = np.zeros((m1 + 2 * p1, m1))
        for col in range(m1):
            for t in range(2 * p1 + 1):
                A[col + t, col] = h[t]
        return A
    blocks = []
    for j in range(2 * p1 + 1):
        S = np.zeros((m1 + 2 * p1, m1))
        for r in range(m1):
            S[r + j, r] = 1.0
        blocks.append(np.kron(S, explicit_A(m[1:], h[j])))
    return sum(blocks)


def laplacian(ndim):
    """The discrete Laplacian as a 3x..x3 stencil over `ndim` axes: -2*ndim at
    the centre, +1 at the two neighbours along each axis, 0 elsewhere.  As a
    PSF under the full convolution it is the operator L of the Tikhonov-Miller
    term (zero outside X's box, no wrap), the regularised family the paper's
    introduction names."""
    l = np.zeros((3,) * ndim)
    c = (1,) * ndim
    l[c] = -2.0 * ndim
    for ax in range(ndim):
        for d in (0, 2):
            idx = list(c)
            idx[ax] = d
            l[tuple(idx)] = 1.0
    return l


def objective(x, y, h, lam=0.0, mu=0.0):
    """f(X) = 1/2 ||A X - Y||_2^2 + lam/2 ||X||_2^2 + mu/2 ||L X||_2^2.
    lam = mu = 0 is the paper's objective; lam is the identity (Tikhonov)
    weight and mu the Laplacian (Tikhonov-Miller) weight this library adds."""
    r = conv_full(x, h) - _d(y)
    x = _d(x)
    f = 0.5 * float(np.sum(r * r)) + 0.5 * lam * float(np.sum(x * x))
    if mu:
        lx = conv_full(x, laplacian(x.ndim))
        f += 0.5 * mu * float(np.sum(lx * lx))
    return f


def initial_delta(h, lam=0.0, mu=0.0):
    """delta_0 = 1/(||h||_1^2 + lam + mu ||l||_1^2).  The paper fixes no
    initial step; since ||A||_2 <= ||h||_1 (Young's inequality) this is at
    most 1/L for the gradient's Lipschitz constant L, so a first trial fails
    the decrease test only at a stationary point.  ||l||_1 = 4n for the
    Laplacian over n axes."""
    h = _d(h)
    l1 = 4.0 * h.ndim if mu else 0.0
    return 1.0 / (float(np.sum(np.abs(h))) ** 2 + lam + mu * l1 * l1)


def gradient(x, y, h, lam=0.0, mu=0.0):
    """grad f = A^T (A X - Y) + lam X + mu L^T L X (the fused form of Eq. 6)."""
    x = _d(x)
    g = conv_adjoint(conv_full(x, h) - _d(y), h) + lam * x
    if mu:
        l = laplacian(x.ndim)
        g = g + mu * conv_adjoint(conv_full(x, l), l)
    return g


STEP_RULES = ("fixed", "cauchy", "bb")


def first_trial(rule, g, h, lam, d0, s_prev=None, g_prev=None, mu=0.0):
    """First trial step of one iteration.  The paper's rule only demands that
    the accepted delta_k decreases f; the first trial is free:

      fixed:  delta_0 = 1/(||h||_1^2 + lam) every iteration;
      cauchy: the exact line minimiser along -g of the unprojected objective,
              <g,g> / (||A g||^2 + lam ||g||^2 + mu ||L g||^2);
      bb:     Barzilai-Borwein, <s,s> / <s,y> with s = X^k - X^{k-1} and
              y = g^k - g^{k-1} (delta_0 on the first iteration).

    A non-positive or non-finite quotient falls back to delta_0."""
    if rule == "fixed":
        return d0
    if rule == "cauchy":
        ag = conv_full(g, h)
        num = float(np.sum(g * g))
        den = float(np.sum(ag * ag)) + lam * num
        if mu:
            lg = conv_full(g, laplacian(g.ndim))
            den += mu * float(np.sum(lg * lg))
    elif rule == "bb":
        if s_prev is None:
            return d0
        num = float(np.sum(s_prev * s_prev))
        den = float(np.sum(s_prev * (g - g_prev)))
    else:
        raise ValueError("unknown step rule %r" % (rule,))
    q = num / den if den > 0 else np.inf
    return q if np.isfinite(q) and q > 0 else d0


def deconv(y, h, x0, iters, lam=0.0, jmax=30, literal_eq6=False, deltas=None, rule="fixed", mu=0.0):
    """Non-negative projected gradient of the section "Application to
    2-dimensional deconvolution", applied to any n:

      Step 1: X^0 is given (x0).
      Step 2: X^{k+1} = max{X^k - delta_k (A^T A X^k - A^T Y), 0}, with the
              gradient from Eq. 6 (fused as A^T (A X^k - Y) + lam X^k, or
              with literal_eq6=True as M(H~ (x) (H (x) X)) - M(H~ (x) Y)).
      Step 3: repeat for `iters` accepted steps.

    delta_k is "confirmed by" f(X^{k+1}) < f(X^k): start at initial_delta()
    and halve on failure, at most jmax trials; equality counts as failure.
    If no trial decreases f, or f becomes non-finite, the loop stops early.
    With deltas given (one per step) the steps are replayed with those values
    and no test.  `rule` picks the first trial of each iteration (see
    first_trial); the halving that follows is the same for every rule.  mu
    adds the Laplacian term mu/2 ||L X||^2 to f (and mu L^T L X to g).

    Returns (X, stats, iters_done, status): stats rows (f_k, delta_k,
    rejections_k, ||X^{k+1}-X^k||_2), row 0 holding f(X^0); status 0 for a
    full run, 1 for no descent, 2 for a non-finite objective."""
    y, h = _d(y), _d(h)
    x = _d(x0).copy()
    f_k = objective(x, y, h, lam, mu)
    stats = [(f_k, np.nan, 0.0, np.nan)]
    d0 = initial_delta(h, lam, mu)
    done, status = 0, 0
    s_prev = g_prev = None
    if not np.isfinite(f_k):
        return x, np.array(stats), 0, 2
    for k in range(iters):
        if literal_eq6:
            g = conv_adjoint_literal(conv_full(x, h), h) - conv_adjoint_literal(y, h)
        else:
            g = conv_adjoint(conv_full(x, h) - y, h)
        g = g + lam * x
        if mu:
            lap = laplacian(x.ndim)
            g = g + mu * conv_adjoint(conv_full(x, lap), lap)
        if deltas is not None:
            d = float(deltas[k])
            xt = np.maximum(x - d * g, 0.0)
            f_t = objective(xt, y, h, lam, mu)
            stats.append((f_t, d, 0.0, float(np.linalg.norm(xt - x))))
            x, f_k, done = xt, f_t, done + 1
            continue
        d, rej, accepted = first_trial(rule, g, h, lam, d0, s_prev, g_prev, mu), 0, False
        for _ in range(jmax):
            xt = np.maximum(x - d * g, 0.0)
            f_t = objective(xt, y, h, lam, mu)
            if not np.isfinite(f_t):
                status = 2
                break
            if f_t < f_k:
                accepted = True
                break
            d *= 0.5
            rej += 1
        if not accepted:
            status = status or 1
            break
        stats.append((f_t, d, float(rej), float(np.linalg.norm(xt - x))))
        s_prev, g_prev = xt - x, g
        x, f_k, done = xt, f_t, done + 1
    return x, np.array(stats), done, status


def i_divergence(y, ax):
    """I-divergence D(y || Ax) = sum_s y_s log(y_s / (Ax)_s) - y_s + (Ax)_s,
    the Poisson negative log-likelihood up to a constant, with 0 log 0 = 0 and
    +inf where (Ax)_s = 0 < y_s.  Meant for y >= 0."""
    y, ax = _d(y), _d(ax)
    pos = y > 0
    with np.errstate(divide="ignore", invalid="ignore"):
        t = np.where(pos, y * np.log(np.where(pos, y, 1.0) / ax), 0.0)
    t = np.where(pos & (ax <= 0), np.inf, t)
    return float(np.sum(t - y + ax))


def richardson_lucy(y, h, x0, iters):
    """The Richardson-Lucy (maximum-likelihood) iteration with the paper's
    operators:

      X^{k+1} = X^k * A^T(Y / (A X^k)) / A^T 1

    with A the full convolution (Property 1) and A^T its transpose (Property
    2), 1 the all-ones array of Y's extent, and the ratio taken as 0 where
    A X^k = 0 (such outputs receive nothing from X^k).  Preconditions: Y,
    H, X^0 >= 0 and sum H > 0.

    Returns (X^iters, divergences) with divergences[k] = D(Y || A X^k) for
    k = 0..iters (i_divergence)."""
    y, h = _d(y), _d(h)
    x = _d(x0).copy()
    norm = conv_adjoint(np.ones(y.shape), h)  # A^T 1
    divs = []
    for k in range(iters + 1):
        ax = conv_full(x, h)
        divs.append(i_divergence(y, ax))
        if k == iters:
            break
        with np.errstate(divide="ignore", invalid="ignore"):
            q = np.where(ax > 0, y / np.where(ax > 0, ax, 1.0), 0.0)
        x = x * conv_adjoint(q, h) / norm
    return x, np.array(divs)
