// Projected-gradient deconvolution (Steps 1-3 of the paper's algorithm) with
// the step-size acceptance rule f(X^{k+1}) < f(X^k) decided on the device.
//
// One trial slot is a fixed launch sequence whose kernels read the phase word
// in device memory and return at once when they have nothing to do:
//   1. transpose of R with the UPDATE epilogue   (phase NEW):   G, X_t, partials
//   2. elementwise update with the halved delta  (phase RETRY): X_t, partials
//   3. forward of X_t with the RESID epilogue    (NEW|RETRY):   R_t, partials
//   4. decide (one work-group): f(X_t) < f(X^k) ? accept : halve delta
//   5. commit (only right after an acceptance): X <- X_t, R <- R_t
// A call enqueues a fixed number of slots (the accepted steps plus room for
// rejected trials) and never waits on the host: slots after the last step
// find the phase DONE and return at once, and a closing kernel reports a run
// that used every slot before reaching `iters` steps.  The whole call can
// therefore be captured into a graph.
//
// With a Cauchy or Barzilai-Borwein first trial the gradient comes first and
// the trial is computed from it on the device:
//   1. transpose of R with the GRAD epilogue     (phase NEW):   G, <g,g>
//   1b. forward of G with the NORM epilogue      (NEW, Cauchy): ||A g||^2
//   1c. step (one work-group): delta from the rule, phase -> RETRY
// and steps 2-5 follow as for a halved retry.  With BB the update also stores
// the step D = X_t - X and the trial forward is taken of D: the RINC epilogue
// forms R_t = R + A D and ||A D||^2, so the BB denominator
// <s, g^k - g^{k-1}> = ||A s||^2 + lambda ||s||^2 + mu ||L s||^2 (f is
// quadratic) is summed from products of the step itself instead of from the
// difference of two rounded gradients, which cancels as steps shrink.
//
// With the Tikhonov-Miller term mu/2 ||L X||^2 (L: full convolution by the
// 3^n Laplacian stencil, through the same operators) the step also runs
//   0. transpose of P = L X^k by the stencil      (NEW):  Q = L^T L X^k
//      (the gradient epilogues add mu*Q)
//   3b. forward of X_t (BB: of D) by the stencil  (NEW|RETRY): P_t, ||P_t||^2
// and commit also moves P <- P_t; f and the decision include mu/2 ||P||^2.
#include <math.h>

#include "ndc_device.h"
#include "ndc_internal.h"

namespace ndc {
namespace {

constexpr int ET = 256;          // elementwise work-group size
constexpr int EW_MAX_BLOCKS = 1024;

inline int64_t ew_blocks(int64_t n) {
  int64_t b = (n + ET * 4 - 1) / (ET * 4);
  return b < 1 ? 1 : (b > EW_MAX_BLOCKS ? EW_MAX_BLOCKS : b);
}

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// Deterministic one-work-group sum of part[stride*i + comp], i < cnt.
__device__ double wg_sum(const double *part, int64_t cnt, int comp, double (*red)[2]) {
  double s = 0.0, dummy = 0.0;
  for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) s += part[2 * i + comp];
  block_sum2(s, dummy, red);
  __syncthreads();
  return s;  // valid in thread 0
}

template <typename T>
__global__ __launch_bounds__(ET) void init_kernel(const T *__restrict__ H, int64_t nh, double lambda, int iters,
                                                  int jmax, int rule, double mu, int ndim, DState *st) {
  __shared__ double red[ET / 64][2];
  double s = 0.0, dummy = 0.0;
  for (int64_t i = threadIdx.x; i < nh; i += ET) s += fabs((double)H[i]);
  block_sum2(s, dummy, red);
  if (threadIdx.x == 0) {
    const double l1 = 4.0 * ndim;  // ||Laplacian stencil||_1
    st->delta0 = 1.0 / (s * s + lambda + mu * l1 * l1);
    st->delta = st->delta0;
    st->lambda = lambda;
    st->f_cur = 0.0;
    st->phase = PH_NEW;
    st->k = 0;
    st->rej = 0;
    st->status = 0;
    st->iters = iters;
    st->jmax = jmax;
    st->accepted = 0;
    st->rule = rule;
    st->ss = 0.0;
    st->sy = 0.0;
    st->mu = mu;
  }
}

// The 3^n Laplacian stencil over the problem's n axes, embedded in the folded
// 3-D extent (k3 = 2 p3 + 1 with p3 = 1 on those axes, 0 on the leading ones):
// -2n at the centre, +1 at the two neighbours along each axis.
template <typename T>
__global__ void laplacian_kernel(T *__restrict__ l, int kz, int ky, int kx, int ndim) {
  const int e = threadIdx.x;
  if (e >= kz * ky * kx) return;
  const int a = e / (ky * kx), b = (e / kx) % ky, c = e % kx;
  const int da = a - kz / 2, db = b - ky / 2, dc = c - kx / 2;
  const int off = (da != 0) + (db != 0) + (dc != 0);
  l[e] = off == 0 ? (T)(-2 * ndim) : (off == 1 ? (T)1 : (T)0);
}

// First trial of a Cauchy / BB iteration.  Cauchy: <g,g> from the GRAD
// epilogue's partials and ||A g||^2 (and ||L g||^2) from NORM forwards of g.
// BB: <s,s> and <s,y> that decide_kernel kept from the last accepted step.
__global__ __launch_bounds__(ET) void step_kernel(DState *st, const double *part_grad, int64_t ng,
                                                  const double *part_ag, int64_t na, const double *part_lg,
                                                  int64_t nl) {
  if (st->phase != PH_NEW) return;
  __shared__ double red[ET / 64][2];
  const bool cauchy = st->rule == NDC_STEP_CAUCHY;  // uniform
  const double gg = cauchy ? wg_sum(part_grad, ng, 0, red) : 0.0;
  const double ag = cauchy ? wg_sum(part_ag, na, 0, red) : 0.0;
  const double lg = (cauchy && nl) ? wg_sum(part_lg, nl, 0, red) : 0.0;
  if (threadIdx.x != 0) return;
  double num = 0.0, den = 0.0;
  if (cauchy) {
    num = gg;
    den = ag + st->lambda * gg + st->mu * lg;
  } else if (st->k > 0) {  // BB; delta_0 on the first iteration of a call
    num = st->ss;
    den = st->sy;
  }
  const double q = den > 0.0 ? num / den : 0.0;
  st->delta = (isfinite(q) && q > 0.0) ? q : st->delta0;
  st->phase = PH_RETRY;
}

template <typename T>
__global__ __launch_bounds__(ET) void sumsq_kernel(const T *__restrict__ x, int64_t n, double *part) {
  __shared__ double red[ET / 64][2];
  double s0 = 0.0, s1 = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)ET + threadIdx.x; i < n; i += (int64_t)gridDim.x * ET) {
    const double v = (double)x[i];
    s0 += v * v;
  }
  block_sum2(s0, s1, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s0;
    part[2 * blockIdx.x + 1] = 0.0;
  }
}

__global__ __launch_bounds__(ET) void f0_kernel(DState *st, const double *part_fwd, int64_t nf,
                                                const double *part_x, int64_t nx, const double *part_reg,
                                                int64_t nreg, double *stats, int *info) {
  __shared__ double red[ET / 64][2];
  const double r2 = wg_sum(part_fwd, nf, 0, red);
  const double x2 = wg_sum(part_x, nx, 0, red);
  const double l2 = nreg ? wg_sum(part_reg, nreg, 0, red) : 0.0;
  if (threadIdx.x == 0) {
    const double f0 = 0.5 * r2 + 0.5 * st->lambda * x2 + 0.5 * st->mu * l2;
    st->f_cur = f0;
    if (!isfinite(f0)) {
      st->status = NDC_ENONFINITE;
      st->phase = PH_DONE;
    } else {
      st->phase = st->iters > 0 ? PH_NEW : PH_DONE;
    }
    if (stats) {
      stats[0] = f0;
      stats[1] = NAN;
      stats[2] = 0.0;
      stats[3] = NAN;
    }
    if (info) {
      info[0] = 0;
      info[1] = st->status;
    }
  }
}

// X_t = max(X - delta G, 0) for a retry (and every BB trial), with the
// partials of ||X_t||^2 and ||X_t - X||^2; D (nullable) receives X_t - X.
template <typename T>
__global__ __launch_bounds__(ET) void update_kernel(const T *__restrict__ X, const T *__restrict__ G,
                                                    T *__restrict__ Xt, T *__restrict__ D, int64_t n,
                                                    const DState *st, double *part) {
  if (st->phase != PH_RETRY) return;
  __shared__ double red[ET / 64][2];
  const T d = (T)st->delta;
  double s0 = 0.0, s1 = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)ET + threadIdx.x; i < n; i += (int64_t)gridDim.x * ET) {
    const T x = X[i];
    const T xt = proj_nonneg<T>(x - d * G[i]);
    Xt[i] = xt;
    if (D) D[i] = xt - x;
    s0 += (double)xt * (double)xt;
    const double dd = (double)xt - (double)x;
    s1 += dd * dd;
  }
  block_sum2(s0, s1, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s0;
    part[2 * blockIdx.x + 1] = s1;
  }
}

__global__ __launch_bounds__(ET) void decide_kernel(DState *st, const double *part_fwd, int64_t nf,
                                                    const double *part_upd, int64_t n_adj, int64_t n_ew,
                                                    const double *part_reg, int64_t nreg, double *stats,
                                                    int *info) {
  const int phase = st->phase;  // uniform
  if (phase == PH_DONE) {
    if (threadIdx.x == 0) st->accepted = 0;
    return;
  }
  __shared__ double red[ET / 64][2];
  const int64_t nu = phase == PH_NEW ? n_adj : n_ew;
  const double r2 = wg_sum(part_fwd, nf, 0, red);
  const double x2 = wg_sum(part_upd, nu, 0, red);
  const double dx2 = wg_sum(part_upd, nu, 1, red);
  const double l2 = nreg ? wg_sum(part_reg, nreg, 0, red) : 0.0;
  // BB trials come from a forward of the step D (RINC): ||A D||^2, ||L D||^2
  const bool bb = st->rule == NDC_STEP_BB;  // uniform
  const double ad2 = bb ? wg_sum(part_fwd, nf, 1, red) : 0.0;
  const double ld2 = (bb && nreg) ? wg_sum(part_reg, nreg, 1, red) : 0.0;
  if (threadIdx.x != 0) return;
  const double ft = 0.5 * r2 + 0.5 * st->lambda * x2 + 0.5 * st->mu * l2;
  if (!isfinite(ft)) {
    st->status = NDC_ENONFINITE;
    st->phase = PH_DONE;
    st->accepted = 0;
  } else if (ft < st->f_cur) {
    const int k = st->k + 1;
    if (stats) {
      stats[4 * k + 0] = ft;
      stats[4 * k + 1] = st->delta;
      stats[4 * k + 2] = (double)st->rej;
      stats[4 * k + 3] = sqrt(dx2);
    }
    st->k = k;
    st->f_cur = ft;
    st->ss = dx2;
    st->sy = ad2 + st->lambda * dx2 + st->mu * ld2;
    st->rej = 0;
    st->delta = st->delta0;
    st->accepted = 1;
    st->phase = k >= st->iters ? PH_DONE : PH_NEW;
  } else {
    st->accepted = 0;
    st->rej += 1;
    st->delta *= 0.5;
    if (st->rej >= st->jmax) {
      st->status = 1;
      st->phase = PH_DONE;
    } else {
      st->phase = PH_RETRY;
    }
  }
  if (info) {
    info[0] = st->k;
    info[1] = st->status;
  }
}

// Closes a call: a run still going after its last trial slot stops with
// status NDC_STOP_TRIALS (the accepted steps so far stand).
__global__ void finish_kernel(DState *st, int *info) {
  if (threadIdx.x != 0 || st->phase == PH_DONE) return;
  st->status = NDC_STOP_TRIALS;
  st->phase = PH_DONE;
  if (info) {
    info[0] = st->k;
    info[1] = st->status;
  }
}

template <typename T>
__global__ __launch_bounds__(ET) void commit_kernel(const DState *st, T *__restrict__ X, const T *__restrict__ Xt,
                                                    int64_t n, T *__restrict__ R, const T *__restrict__ Rt,
                                                    int64_t ny, T *__restrict__ P, const T *__restrict__ Pt,
                                                    int64_t np) {
  if (!st->accepted) return;
  int64_t m = n > ny ? n : ny;
  if (P && np > m) m = np;
  for (int64_t i = blockIdx.x * (int64_t)ET + threadIdx.x; i < m; i += (int64_t)gridDim.x * ET) {
    if (i < n) X[i] = Xt[i];
    if (i < ny) R[i] = Rt[i];
    if (P && i < np) P[i] = Pt[i];
  }
}

struct WsLayout {
  size_t state, part_fwd, part_upd, xt, g, r, rt, sbuf;
  size_t lap, part_reg, p, pt, q;  // Tikhonov-Miller term (when regularised)
  size_t total;
};

// Tikhonov-Miller geometry: the 3^n Laplacian over the problem's last n of
// the 3 folded axes (ndim = 0: no regularisation buffers).
struct RegSizes {
  int ndim;
  int64_t pl3[3], NP, NL;
  Geom gl, gla;
  ConvPlan pl, pla;
};

RegSizes reg_sizes(const int64_t m3[3], int ndim, int dtype, int precision) {
  RegSizes r{};
  r.ndim = ndim;
  if (!ndim) return r;
  r.NP = 1;
  r.NL = 1;
  for (int i = 0; i < 3; ++i) {
    r.pl3[i] = i >= 3 - ndim ? 1 : 0;
    r.NP *= m3[i] + 2 * r.pl3[i];
    r.NL *= 2 * r.pl3[i] + 1;
  }
  r.gl = forward_geom(m3, r.pl3);
  r.gla = adjoint_geom(m3, r.pl3);
  r.pl = plan_conv(r.gl, dtype, precision);
  r.pla = plan_conv(r.gla, dtype, precision);
  return r;
}

WsLayout layout(int64_t N, int64_t NY, size_t esz, int64_t nf, int64_t nu, const RegSizes &R) {
  WsLayout L;
  size_t o = 0;
  L.state = o;
  o += align256(sizeof(DState));
  L.part_fwd = o;
  o += align256((size_t)nf * 2 * sizeof(double));
  L.part_upd = o;
  o += align256((size_t)nu * 2 * sizeof(double));
  L.xt = o;
  o += align256((size_t)N * esz);
  L.g = o;
  o += align256((size_t)N * esz);
  L.r = o;
  o += align256((size_t)NY * esz);
  L.rt = o;
  o += align256((size_t)NY * esz);
  L.sbuf = o;  // trial step D = X_t - X (Barzilai-Borwein rule)
  o += align256((size_t)N * esz);
  L.lap = L.part_reg = L.p = L.pt = L.q = 0;
  if (R.ndim) {
    L.lap = o;
    o += align256((size_t)R.NL * esz);
    L.part_reg = o;
    o += align256((size_t)R.pl.nblocks * 2 * sizeof(double));
    L.p = o;  // L X^k
    o += align256((size_t)R.NP * esz);
    L.pt = o;  // L X_t
    o += align256((size_t)R.NP * esz);
    L.q = o;  // L^T L X^k
    o += align256((size_t)N * esz);
  }
  L.total = o;
  return L;
}

struct Sizes {
  int64_t N, NY, NH;
  Geom gf, ga;
  ConvPlan pf, pa;
  int64_t n_ew;
};

Sizes sizes_for(const int64_t m3[3], const int64_t p3[3], int dtype, int precision) {
  Sizes s;
  s.N = m3[0] * m3[1] * m3[2];
  s.NY = (m3[0] + 2 * p3[0]) * (m3[1] + 2 * p3[1]) * (m3[2] + 2 * p3[2]);
  s.NH = (2 * p3[0] + 1) * (2 * p3[1] + 1) * (2 * p3[2] + 1);
  s.gf = forward_geom(m3, p3);
  s.ga = adjoint_geom(m3, p3);
  s.pf = plan_conv(s.gf, dtype, precision);
  s.pa = plan_conv(s.ga, dtype, precision);
  s.n_ew = ew_blocks(s.N);
  return s;
}

template <typename T>
int deconv_t(const int64_t m3[3], const int64_t p3[3], const void *Y, const void *H, void *Xv, int iters,
             double lambda, double mu, int ndim, int dtype, int precision, void *ws, double *stats, int *info,
             int rule, int slots, hipStream_t s) {
  const Sizes S = sizes_for(m3, p3, dtype, precision);
  const RegSizes RS = reg_sizes(m3, mu > 0.0 ? ndim : 0, dtype, precision);
  const int64_t nu = S.pa.nblocks > S.n_ew ? S.pa.nblocks : S.n_ew;
  const WsLayout L = layout(S.N, S.NY, sizeof(T), S.pf.nblocks, nu, RS);
  char *w = (char *)ws;
  DState *st = (DState *)(w + L.state);
  double *part_fwd = (double *)(w + L.part_fwd);
  double *part_upd = (double *)(w + L.part_upd);
  T *X = (T *)Xv, *Xt = (T *)(w + L.xt), *G = (T *)(w + L.g), *R = (T *)(w + L.r), *Rt = (T *)(w + L.rt);
  T *D = rule == NDC_STEP_BB ? (T *)(w + L.sbuf) : nullptr;
  const bool reg = RS.ndim > 0;
  T *lap = reg ? (T *)(w + L.lap) : nullptr, *P = reg ? (T *)(w + L.p) : nullptr;
  T *Pt = reg ? (T *)(w + L.pt) : nullptr, *Q = reg ? (T *)(w + L.q) : nullptr;
  double *part_reg = reg ? (double *)(w + L.part_reg) : nullptr;
  const int64_t nreg = reg ? RS.pl.nblocks : 0;

  hipLaunchKernelGGL(init_kernel<T>, dim3(1), dim3(ET), 0, s, (const T *)H, S.NH, lambda, iters, 30, rule,
                     reg ? mu : 0.0, ndim, st);
  hipLaunchKernelGGL(sumsq_kernel<T>, dim3((unsigned)S.n_ew), dim3(ET), 0, s, (const T *)X, S.N, part_upd);
  Epi ef{};
  ef.mode = EPI_RESID;
  ef.Y = Y;
  ef.part = part_fwd;
  ef.phase = nullptr;
  if (launch_conv(S.pf, S.gf, dtype, precision, X, H, R, ef, s) != hipSuccess) return NDC_EDEVICE;
  Epi el{};  // P = L X with ||P||^2 (initial point, then every trial)
  el.mode = EPI_SQR;
  el.part = part_reg;
  if (reg) {
    hipLaunchKernelGGL(laplacian_kernel<T>, dim3(1), dim3(64), 0, s, lap, (int)RS.gl.kz, (int)RS.gl.ky,
                       (int)RS.gl.kx, ndim);
    if (launch_conv(RS.pl, RS.gl, dtype, NDC_PREC_NATIVE, X, lap, P, el, s) != hipSuccess) return NDC_EDEVICE;
  }
  hipLaunchKernelGGL(f0_kernel, dim3(1), dim3(ET), 0, s, st, (const double *)part_fwd, S.pf.nblocks,
                     (const double *)part_upd, S.n_ew, (const double *)part_reg, nreg, stats, info);
  if (hipGetLastError() != hipSuccess) return NDC_EDEVICE;

  Epi ea{};
  ea.mode = EPI_UPDATE;
  ea.X = X;
  ea.G = G;
  ea.lambda = lambda;
  ea.delta = &st->delta;
  ea.part = part_upd;
  ea.phase = &st->phase;
  ea.phase_mask = 1 << PH_NEW;
  ea.Q = Q;
  ea.mu = mu;
  Epi eg{};  // Cauchy / BB: gradient first
  eg.mode = EPI_GRAD;
  eg.X = X;
  eg.lambda = lambda;
  eg.part = part_upd;
  eg.phase = &st->phase;
  eg.phase_mask = 1 << PH_NEW;
  eg.Q = Q;
  eg.mu = mu;
  Epi en{};  // Cauchy: ||A g||^2
  en.mode = EPI_NORM;
  en.part = part_fwd;
  en.phase = &st->phase;
  en.phase_mask = 1 << PH_NEW;
  Epi enl = en;  // Cauchy with the Laplacian: ||L g||^2
  enl.part = part_reg;
  Epi eq{};  // Q = L^T P at the start of a step
  eq.mode = EPI_STORE;
  eq.phase = &st->phase;
  eq.phase_mask = 1 << PH_NEW;
  Epi et{};  // trial residual R_t = A X_t - Y
  et.mode = EPI_RESID;
  et.Y = Y;
  et.part = part_fwd;
  et.phase = &st->phase;
  et.phase_mask = (1 << PH_NEW) | (1 << PH_RETRY);
  Epi elt = el;  // P_t = L X_t for every trial
  elt.phase = &st->phase;
  elt.phase_mask = (1 << PH_NEW) | (1 << PH_RETRY);
  Epi ed = et;  // BB: R_t = R + A D and ||A D||^2
  ed.mode = EPI_RINC;
  ed.B = R;
  Epi eld = elt;  // BB: P_t = P + L D and ||L D||^2
  eld.mode = EPI_RINC;
  eld.B = P;
  int64_t ncm = S.NY > S.N ? S.NY : S.N;
  if (reg && RS.NP > ncm) ncm = RS.NP;
  const int64_t ncommit = ew_blocks(ncm);

  // A fixed schedule of trial slots, nothing read back on the host.
  for (int slot = 0; slot < slots; ++slot) {
    if (reg && launch_conv(RS.pla, RS.gla, dtype, NDC_PREC_NATIVE, P, lap, Q, eq, s) != hipSuccess)
      return NDC_EDEVICE;
    if (rule == NDC_STEP_FIXED) {
      if (launch_conv(S.pa, S.ga, dtype, precision, R, H, Xt, ea, s) != hipSuccess) return NDC_EDEVICE;
    } else {
      if (launch_conv(S.pa, S.ga, dtype, precision, R, H, G, eg, s) != hipSuccess) return NDC_EDEVICE;
      // (NORM stores nothing; R_t / P_t are passed as valid, unused outputs)
      if (rule == NDC_STEP_CAUCHY && launch_conv(S.pf, S.gf, dtype, precision, G, H, Rt, en, s) != hipSuccess)
        return NDC_EDEVICE;
      if (rule == NDC_STEP_CAUCHY && reg &&
          launch_conv(RS.pl, RS.gl, dtype, NDC_PREC_NATIVE, G, lap, Pt, enl, s) != hipSuccess)
        return NDC_EDEVICE;
      hipLaunchKernelGGL(step_kernel, dim3(1), dim3(ET), 0, s, st, (const double *)part_upd, S.pa.nblocks,
                         (const double *)part_fwd, S.pf.nblocks, (const double *)part_reg, nreg);
    }
    hipLaunchKernelGGL(update_kernel<T>, dim3((unsigned)S.n_ew), dim3(ET), 0, s, (const T *)X, (const T *)G, Xt, D,
                       S.N, (const DState *)st, part_upd);
    if (D) {
      if (launch_conv(S.pf, S.gf, dtype, precision, D, H, Rt, ed, s) != hipSuccess) return NDC_EDEVICE;
      if (reg && launch_conv(RS.pl, RS.gl, dtype, NDC_PREC_NATIVE, D, lap, Pt, eld, s) != hipSuccess)
        return NDC_EDEVICE;
    } else {
      if (launch_conv(S.pf, S.gf, dtype, precision, Xt, H, Rt, et, s) != hipSuccess) return NDC_EDEVICE;
      if (reg && launch_conv(RS.pl, RS.gl, dtype, NDC_PREC_NATIVE, Xt, lap, Pt, elt, s) != hipSuccess)
        return NDC_EDEVICE;
    }
    hipLaunchKernelGGL(decide_kernel, dim3(1), dim3(ET), 0, s, st, (const double *)part_fwd, S.pf.nblocks,
                       (const double *)part_upd, S.pa.nblocks, S.n_ew, (const double *)part_reg, nreg, stats,
                       info);
    hipLaunchKernelGGL(commit_kernel<T>, dim3((unsigned)ncommit), dim3(ET), 0, s, (const DState *)st, X,
                       (const T *)Xt, S.N, R, (const T *)Rt, S.NY, P, (const T *)Pt, reg ? RS.NP : 0);
    if (hipGetLastError() != hipSuccess) return NDC_EDEVICE;
  }
  hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(64), 0, s, st, info);
  return hipGetLastError() == hipSuccess ? NDC_OK : NDC_EDEVICE;
}

}  // namespace

size_t deconv_ws_bytes(const int64_t m3[3], const int64_t p3[3], int dtype, int precision, int reg_ndim) {
  const Sizes S = sizes_for(m3, p3, dtype, precision);
  const RegSizes RS = reg_sizes(m3, reg_ndim, dtype, precision);
  const int64_t nu = S.pa.nblocks > S.n_ew ? S.pa.nblocks : S.n_ew;
  const size_t esz = dtype == NDC_F64 ? sizeof(double) : sizeof(float);
  return layout(S.N, S.NY, esz, S.pf.nblocks, nu, RS).total;
}

int deconv_run(const int64_t m3[3], const int64_t p3[3], const void *Y, const void *H, void *X, int iters,
               double lambda, double mu, int ndim, int dtype, int precision, void *ws, double *stats, int *info,
               int rule, int slots, hipStream_t s) {
  if (dtype == NDC_F64)
    return deconv_t<double>(m3, p3, Y, H, X, iters, lambda, mu, ndim, dtype, precision, ws, stats, info, rule,
                            slots, s);
  return deconv_t<float>(m3, p3, Y, H, X, iters, lambda, mu, ndim, dtype, precision, ws, stats, info, rule, slots,
                         s);
}

}  // namespace ndc
