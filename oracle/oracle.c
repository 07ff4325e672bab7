/*
 * FP64 CPU oracle for the n-dimensional full convolution and its transpose.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file: only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header or table with the HIP
 * library.
 *
 * Every routine is a plain loop over the definitions of the paper
 * "Properties on n-dimensional convolution for image deconvolution"
 * (arXiv 1711.11224):
 *   - ora_conv_full            : the discrete convolution of Property 1 and of
 *                                the supplementary equation (S2), X of extent
 *                                m_i, H of extent 2p_i+1, Y of extent m_i+2p_i
 *                                (the size convention of Eq. 4).
 *   - ora_conv_adjoint         : (A_n^h)^T applied to Y, written as the sum
 *                                over the nonzero entries of the transposed
 *                                banded matrix (S8): G[k] = sum_j H[j] R[k+j].
 *   - ora_conv_adjoint_literal : Property 2 word for word, Eq. 2: convolve
 *                                with the flipped PSF H~(s) = H(2p-s) into the
 *                                extended result of extent m_i+4p_i, then keep
 *                                the window M_{2p} (0-based offset 2p_i,
 *                                length m_i).
 *   - ora_conv_dH              : derivative of 1/2||X (x) H - Y||^2 with
 *                                respect to H.  Convolution commutes, so by
 *                                Property 1 with the roles of X and H swapped
 *                                the derivative is A_X^T R, i.e.
 *                                dH[j] = sum_k X[k] R[k+j].
 *   - ora_conv_full_at / ora_conv_adjoint_at : the same two sums evaluated
 *                                only at a list of flat output indices.
 *
 * Arrays are C order (axis 0 slowest): the row-by-row stacking that the
 * vectorisation {.}^v under Eq. 1 uses.  Sums run in the natural lexicographic
 * tap order; there is no blocking, fusion or reordering.  OpenMP splits the
 * output elements statically; each element is summed by one thread in the
 * same order, so results do not depend on the thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_MAXN 8

static int64_t ora_prod(int n, const int64_t *e) {
  int64_t r = 1;
  for (int i = 0; i < n; ++i) r *= e[i];
  return r;
}

static int ora_check(int n, const int64_t *m, const int64_t *p) {
  if (n < 1 || n > ORA_MAXN || !m || !p) return -1;
  for (int i = 0; i < n; ++i)
    if (m[i] < 1 || p[i] < 0) return -1;
  return 0;
}

/* Flat C-order offset of multi-index v inside a box of extents e. */
static int64_t ora_flat(int n, const int64_t *v, const int64_t *e) {
  int64_t f = 0;
  for (int i = 0; i < n; ++i) f = f * e[i] + v[i];
  return f;
}

/* y(s) = sum_k x(k) h(s-k), summed over the taps j = s-k that keep both
 * k inside [0,m) and j inside [0,2p] (zero extension outside).  Taps are
 * visited in lexicographic order; the last axis is the inner loop. */
static double ora_full_one(int n, const int64_t *m, const int64_t *p,
                           const double *X, const double *H, const int64_t *s) {
  int64_t lo[ORA_MAXN], hi[ORA_MAXN], j[ORA_MAXN], eh[ORA_MAXN], k[ORA_MAXN];
  for (int i = 0; i < n; ++i) {
    eh[i] = 2 * p[i] + 1;
    lo[i] = s[i] - (m[i] - 1) > 0 ? s[i] - (m[i] - 1) : 0;
    hi[i] = s[i] < 2 * p[i] ? s[i] : 2 * p[i];
    if (lo[i] > hi[i]) return 0.0;
    j[i] = lo[i];
  }
  const int L = n - 1;
  double acc = 0.0;
  for (;;) {
    /* row of H at j[0..L-1], column 0; row of X at k[0..L-1] = s - j, column 0 */
    j[L] = 0;
    for (int i = 0; i < L; ++i) k[i] = s[i] - j[i];
    k[L] = 0;
    const double *hrow = H + ora_flat(n, j, eh);
    const double *xrow = X + ora_flat(n, k, m);
    for (int64_t t = lo[L]; t <= hi[L]; ++t) acc += hrow[t] * xrow[s[L] - t];
    int i = L - 1;
    while (i >= 0) {
      if (++j[i] <= hi[i]) break;
      j[i] = lo[i];
      --i;
    }
    if (i < 0) break;
  }
  return acc;
}

/* (A^T r)(k) = sum_{j in [0,2p]} h(j) r(k+j): every tap is in range.  Taps
 * in lexicographic order; the last axis is the inner loop. */
static double ora_adj_one(int n, const int64_t *m, const int64_t *p,
                          const double *R, const double *H, const int64_t *k) {
  int64_t j[ORA_MAXN], eh[ORA_MAXN], er[ORA_MAXN], t[ORA_MAXN];
  for (int i = 0; i < n; ++i) {
    eh[i] = 2 * p[i] + 1;
    er[i] = m[i] + 2 * p[i];
    j[i] = 0;
  }
  const int L = n - 1;
  double acc = 0.0;
  for (;;) {
    for (int i = 0; i < L; ++i) t[i] = k[i] + j[i];
    t[L] = k[L];
    j[L] = 0;
    const double *hrow = H + ora_flat(n, j, eh);
    const double *rrow = R + ora_flat(n, t, er);
    for (int64_t c = 0; c <= 2 * p[L]; ++c) acc += hrow[c] * rrow[c];
    int i = L - 1;
    while (i >= 0) {
      if (++j[i] <= 2 * p[i]) break;
      j[i] = 0;
      --i;
    }
    if (i < 0) break;
  }
  return acc;
}

static void ora_unflat(int n, int64_t f, const int64_t *e, int64_t *v) {
  for (int i = n - 1; i >= 0; --i) {
    v[i] = f % e[i];
    f /= e[i];
  }
}

int ora_conv_full(int n, const int64_t *m, const int64_t *p, const double *X,
                  const double *H, double *Y) {
  if (ora_check(n, m, p) || !X || !H || !Y) return -1;
  int64_t ey[ORA_MAXN];
  for (int i = 0; i < n; ++i) ey[i] = m[i] + 2 * p[i];
  int64_t ny = ora_prod(n, ey);
#pragma omp parallel for schedule(static)
  for (int64_t f = 0; f < ny; ++f) {
    int64_t s[ORA_MAXN];
    ora_unflat(n, f, ey, s);
    Y[f] = ora_full_one(n, m, p, X, H, s);
  }
  return 0;
}

int ora_conv_adjoint(int n, const int64_t *m, const int64_t *p, const double *R,
                     const double *H, double *G) {
  if (ora_check(n, m, p) || !R || !H || !G) return -1;
  int64_t nx = ora_prod(n, m);
#pragma omp parallel for schedule(static)
  for (int64_t f = 0; f < nx; ++f) {
    int64_t k[ORA_MAXN];
    ora_unflat(n, f, m, k);
    G[f] = ora_adj_one(n, m, p, R, H, k);
  }
  return 0;
}

/* Property 2 literally: Yhat = R (x) H~ with R of extent m+2p, so Yhat has
 * extent (m+2p)+2p = m+4p; the result is Yhat cropped to offset 2p, length m. */
int ora_conv_adjoint_literal(int n, const int64_t *m, const int64_t *p,
                             const double *R, const double *H, double *G,
                             double *Yhat_out /* nullable, extent m+4p */) {
  if (ora_check(n, m, p) || !R || !H || !G) return -1;
  int64_t er[ORA_MAXN], eh[ORA_MAXN], ehat[ORA_MAXN];
  for (int i = 0; i < n; ++i) {
    er[i] = m[i] + 2 * p[i];
    eh[i] = 2 * p[i] + 1;
    ehat[i] = m[i] + 4 * p[i];
  }
  int64_t nh = ora_prod(n, eh), nhat = ora_prod(n, ehat), nx = ora_prod(n, m);
  double *Hf = (double *)malloc(sizeof(double) * (size_t)nh);
  double *Yhat = (double *)malloc(sizeof(double) * (size_t)nhat);
  if (!Hf || !Yhat) { free(Hf); free(Yhat); return -2; }
  /* H~(s) = H(2p - s) on every axis. */
  for (int64_t f = 0; f < nh; ++f) {
    int64_t s[ORA_MAXN], t[ORA_MAXN];
    ora_unflat(n, f, eh, s);
    for (int i = 0; i < n; ++i) t[i] = 2 * p[i] - s[i];
    Hf[f] = H[ora_flat(n, t, eh)];
  }
  int rc = ora_conv_full(n, er, p, R, Hf, Yhat);
  if (rc == 0) {
    for (int64_t f = 0; f < nx; ++f) {
      int64_t k[ORA_MAXN];
      ora_unflat(n, f, m, k);
      for (int i = 0; i < n; ++i) k[i] += 2 * p[i];
      G[f] = Yhat[ora_flat(n, k, ehat)];
    }
    if (Yhat_out) memcpy(Yhat_out, Yhat, sizeof(double) * (size_t)nhat);
  }
  free(Hf);
  free(Yhat);
  return rc;
}

/* dH[j] = sum_{k in [0,m)} X[k] R[k+j], j in [0,2p]. */
int ora_conv_dH(int n, const int64_t *m, const int64_t *p, const double *X,
                const double *R, double *dH) {
  if (ora_check(n, m, p) || !X || !R || !dH) return -1;
  int64_t eh[ORA_MAXN], er[ORA_MAXN];
  for (int i = 0; i < n; ++i) {
    eh[i] = 2 * p[i] + 1;
    er[i] = m[i] + 2 * p[i];
  }
  int64_t nh = ora_prod(n, eh);
#pragma omp parallel for schedule(static)
  for (int64_t f = 0; f < nh; ++f) {
    int64_t j[ORA_MAXN], k[ORA_MAXN], t[ORA_MAXN];
    ora_unflat(n, f, eh, j);
    for (int i = 0; i < n; ++i) k[i] = 0;
    double acc = 0.0;
    for (;;) {
      for (int i = 0; i < n; ++i) t[i] = k[i] + j[i];
      acc += X[ora_flat(n, k, m)] * R[ora_flat(n, t, er)];
      int i = n - 1;
      while (i >= 0) {
        if (++k[i] < m[i]) break;
        k[i] = 0;
        --i;
      }
      if (i < 0) break;
    }
    dH[f] = acc;
  }
  return 0;
}

/* Full convolution evaluated only at the flat output indices idx[0..cnt). */
int ora_conv_full_at(int n, const int64_t *m, const int64_t *p, const double *X,
                     const double *H, const int64_t *idx, int64_t cnt, double *out) {
  if (ora_check(n, m, p) || !X || !H || (cnt > 0 && (!idx || !out))) return -1;
  int64_t ey[ORA_MAXN];
  for (int i = 0; i < n; ++i) ey[i] = m[i] + 2 * p[i];
  int64_t ny = ora_prod(n, ey);
  for (int64_t q = 0; q < cnt; ++q)
    if (idx[q] < 0 || idx[q] >= ny) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < cnt; ++q) {
    int64_t s[ORA_MAXN];
    ora_unflat(n, idx[q], ey, s);
    out[q] = ora_full_one(n, m, p, X, H, s);
  }
  return 0;
}

/* Transpose evaluated only at the flat X-shaped indices idx[0..cnt). */
int ora_conv_adjoint_at(int n, const int64_t *m, const int64_t *p, const double *R,
                        const double *H, const int64_t *idx, int64_t cnt, double *out) {
  if (ora_check(n, m, p) || !R || !H || (cnt > 0 && (!idx || !out))) return -1;
  int64_t nx = ora_prod(n, m);
  for (int64_t q = 0; q < cnt; ++q)
    if (idx[q] < 0 || idx[q] >= nx) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < cnt; ++q) {
    int64_t k[ORA_MAXN];
    ora_unflat(n, idx[q], m, k);
    out[q] = ora_adj_one(n, m, p, R, H, k);
  }
  return 0;
}

/* Threads an OpenMP parallel region of this library will use. */
int ora_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* dH evaluated only at the flat PSF-shaped indices idx[0..cnt). */
int ora_conv_dH_at(int n, const int64_t *m, const int64_t *p, const double *X, const double *R,
                   const int64_t *idx, int64_t cnt, double *out) {
  if (ora_check(n, m, p) || !X || !R || (cnt > 0 && (!idx || !out))) return -1;
  int64_t eh[ORA_MAXN], er[ORA_MAXN];
  for (int i = 0; i < n; ++i) {
    eh[i] = 2 * p[i] + 1;
    er[i] = m[i] + 2 * p[i];
  }
  int64_t nh = ora_prod(n, eh);
  for (int64_t q = 0; q < cnt; ++q)
    if (idx[q] < 0 || idx[q] >= nh) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t q = 0; q < cnt; ++q) {
    int64_t j[ORA_MAXN], k[ORA_MAXN], t[ORA_MAXN];
    ora_unflat(n, idx[q], eh, j);
    for (int i = 0; i < n; ++i) k[i] = 0;
    double acc = 0.0;
    for (;;) {
      for (int i = 0; i < n; ++i) t[i] = k[i] + j[i];
      acc += X[ora_flat(n, k, m)] * R[ora_flat(n, t, er)];
      int i = n - 1;
      while (i >= 0) {
        if (++k[i] < m[i]) break;
        k[i] = 0;
        --i;
      }
      if (i < 0) break;
    }
    out[q] = acc;
  }
  return 0;
}
