// Richardson-Lucy (maximum-likelihood) deconvolution, the iteration the paper
// compares its method against, built from the same two operators:
//   X^{k+1} = X^k * A^T(Y / (A X^k)) / A^T 1,   A^T 1 = sum H everywhere
// (every tap of the transpose lands inside Y's extent).  One iteration is
//   1. forward of X^k with the RLQ epilogue: Q = Y / (A X^k) (0 where
//      A X^k = 0) and the partials of D(Y || A X^k);
//   2. record (one work-group): D_k into stats, stop on a NaN divergence;
//   3. transpose of Q with the RLX epilogue: X <- X * (A^T Q) / sum H, in
//      place (each output element is read and written by one thread).
// A call enqueues iters + 1 forwards (the last one only evaluates D of the
// result) and returns without waiting on the host.
#include <math.h>

#include "ndc_device.h"
#include "ndc_internal.h"

namespace ndc {
namespace {

constexpr int RT = 256;

inline size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

// 1/sum H, or a stop with NDC_EINVAL when sum H is not positive and finite
template <typename T>
__global__ __launch_bounds__(RT) void rl_init_kernel(const T *__restrict__ H, int64_t nh, int iters, DState *st,
                                                     int *info) {
  __shared__ double red[RT / 64][2];
  double s = 0.0, dummy = 0.0;
  for (int64_t i = threadIdx.x; i < nh; i += RT) s += (double)H[i];
  block_sum2(s, dummy, red);
  if (threadIdx.x != 0) return;
  const bool ok = s > 0.0 && isfinite(s);
  st->delta = ok ? 1.0 / s : 0.0;
  st->k = 0;
  st->iters = iters;
  st->status = ok ? 0 : NDC_EINVAL;
  st->phase = ok ? PH_NEW : PH_DONE;
  if (info) {
    info[0] = 0;
    info[1] = st->status;
  }
}

// D(Y || A X^k) from the forward's partials; the transpose that follows runs
// only while k < iters.
__global__ __launch_bounds__(RT) void rl_record_kernel(DState *st, const double *part, int64_t np, double *stats,
                                                       int *info) {
  if (st->phase == PH_DONE) return;
  __shared__ double red[RT / 64][2];
  double s = 0.0, dummy = 0.0;
  for (int64_t i = threadIdx.x; i < np; i += RT) s += part[2 * i];
  block_sum2(s, dummy, red);
  if (threadIdx.x != 0) return;
  const int k = st->k;
  if (stats) stats[k] = s;
  if (isnan(s)) {
    st->status = NDC_ENONFINITE;
    st->phase = PH_DONE;
  } else if (k >= st->iters) {
    st->phase = PH_DONE;
  }
  st->k = k + 1;
  if (info) {
    info[0] = k;
    info[1] = st->status;
  }
}

struct RlLayout {
  size_t state, part, q, total;
};

RlLayout rl_layout(int64_t NY, size_t esz, int64_t nf) {
  RlLayout L;
  size_t o = 0;
  L.state = o;
  o += al256(sizeof(DState));
  L.part = o;
  o += al256((size_t)nf * 2 * sizeof(double));
  L.q = o;
  o += al256((size_t)NY * esz);
  L.total = o;
  return L;
}

}  // namespace

// Partial-sum slots: both launches write one pair per work-group.
int64_t rl_slots(const ConvPlan &pf, const ConvPlan &pa) { return pf.nblocks > pa.nblocks ? pf.nblocks : pa.nblocks; }

size_t rl_ws_bytes(const int64_t m3[3], const int64_t p3[3], int dtype, int precision) {
  const Geom gf = forward_geom(m3, p3), ga = adjoint_geom(m3, p3);
  const ConvPlan pf = plan_conv(gf, dtype, precision), pa = plan_conv(ga, dtype, precision);
  const int64_t NY = (int64_t)gf.oz * gf.oy * gf.ox;
  return rl_layout(NY, dtype == NDC_F64 ? sizeof(double) : sizeof(float), rl_slots(pf, pa)).total;
}

int rl_run(const int64_t m3[3], const int64_t p3[3], const void *Y, const void *H, void *X, int iters, int dtype,
           int precision, void *ws, double *stats, int *info, hipStream_t s) {
  const Geom gf = forward_geom(m3, p3), ga = adjoint_geom(m3, p3);
  const ConvPlan pf = plan_conv(gf, dtype, precision), pa = plan_conv(ga, dtype, precision);
  const int64_t NY = (int64_t)gf.oz * gf.oy * gf.ox;
  const int64_t NH = (int64_t)gf.kz * gf.ky * gf.kx;
  const RlLayout L = rl_layout(NY, dtype == NDC_F64 ? sizeof(double) : sizeof(float), rl_slots(pf, pa));
  char *w = (char *)ws;
  DState *st = (DState *)(w + L.state);
  double *part = (double *)(w + L.part);
  void *Q = w + L.q;
  if (dtype == NDC_F64)
    hipLaunchKernelGGL(rl_init_kernel<double>, dim3(1), dim3(RT), 0, s, (const double *)H, NH, iters, st, info);
  else
    hipLaunchKernelGGL(rl_init_kernel<float>, dim3(1), dim3(RT), 0, s, (const float *)H, NH, iters, st, info);
  Epi eq{};
  eq.mode = EPI_RLQ;
  eq.Y = Y;
  eq.part = part;
  eq.phase = &st->phase;
  eq.phase_mask = 1 << PH_NEW;
  Epi ex{};
  ex.mode = EPI_RLX;
  ex.delta = &st->delta;
  ex.part = part;  // RLX leaves zero partials; the forward's were read already
  ex.phase = &st->phase;
  ex.phase_mask = 1 << PH_NEW;
  for (int k = 0; k <= iters; ++k) {
    if (launch_conv(pf, gf, dtype, precision, X, H, Q, eq, s) != hipSuccess) return NDC_EDEVICE;
    hipLaunchKernelGGL(rl_record_kernel, dim3(1), dim3(RT), 0, s, st, (const double *)part, pf.nblocks, stats,
                       info);
    if (k < iters && launch_conv(pa, ga, dtype, precision, Q, H, X, ex, s) != hipSuccess) return NDC_EDEVICE;
  }
  return hipGetLastError() == hipSuccess ? NDC_OK : NDC_EDEVICE;
}

}  // namespace ndc
