// Batched form: many independent volumes, each with its own extents, PSF,
// step size and line search, through persistent launches (conv_batch.hip).
// One deconvolution trial slot for the whole batch is a fixed sequence
//   transpose+update (persistent) -> retry update -> forward+residual
//   (persistent) -> per-volume decide -> per-volume commit
// captured once into a hipGraph and replayed for a fixed number of slots.
// Every kernel reads the per-volume phase word and skips volumes with
// nothing to do.
//
// The kernels find each volume's arrays in a device table.  A call writes
// its pointers into that table with a small kernel that receives them as
// launch arguments (copied when the launch is enqueued), so no host buffer
// has to outlive the call and nothing waits on the host.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "ndc_device.h"
#include "ndc_internal.h"

using namespace ndc;

namespace {

constexpr int BT = 256;  // threads of the per-volume kernels
constexpr int EB = 64;   // work-groups per volume in elementwise kernels

inline size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

__device__ double bwg_sum(const double *part, int lo, int hi, int comp, double (*red)[2]) {
  double s = 0.0, dummy = 0.0;
  for (int i = lo + (int)threadIdx.x; i < hi; i += BT) s += part[2 * (int64_t)i + comp];
  block_sum2(s, dummy, red);
  __syncthreads();
  return s;
}

// grid = count: delta_0 and the state of each volume
__global__ __launch_bounds__(BT) void b_init_kernel(const BVol *vols, double lambda, int iters, int jmax) {
  __shared__ double red[BT / 64][2];
  const BVol &v = vols[blockIdx.x];
  const int64_t nh = (int64_t)(2 * v.p[0] + 1) * (2 * v.p[1] + 1) * (2 * v.p[2] + 1);
  double s = 0.0, dummy = 0.0;
  for (int64_t i = threadIdx.x; i < nh; i += BT) s += fabs((double)v.H[i]);
  block_sum2(s, dummy, red);
  if (threadIdx.x == 0) {
    DState *st = v.st;
    st->delta0 = 1.0 / (s * s + lambda);
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
    st->rule = NDC_STEP_FIXED;
    st->ss = 0.0;
    st->sy = 0.0;
    st->mu = 0.0;
  }
}

// grid = count * EB: ||X||^2 partials of each volume
__global__ __launch_bounds__(BT) void b_sumsq_kernel(const BVol *vols, double *part_ew) {
  __shared__ double red[BT / 64][2];
  const int vi = blockIdx.x / EB, bi = blockIdx.x % EB;
  const BVol &v = vols[vi];
  double s0 = 0.0, s1 = 0.0;
  for (int64_t i = bi * (int64_t)BT + threadIdx.x; i < v.n; i += (int64_t)EB * BT) {
    const double x = (double)v.X[i];
    s0 += x * x;
  }
  block_sum2(s0, s1, red);
  if (threadIdx.x == 0) {
    part_ew[2 * (int64_t)blockIdx.x] = s0;
    part_ew[2 * (int64_t)blockIdx.x + 1] = 0.0;
  }
}

// grid = count: f(X^0)
__global__ __launch_bounds__(BT) void b_f0_kernel(const BVol *vols, const double *part_fwd, const double *part_ew) {
  __shared__ double red[BT / 64][2];
  const int vi = blockIdx.x;
  const BVol &v = vols[vi];
  const double r2 = bwg_sum(part_fwd, v.fwd_lo, v.fwd_hi, 0, red);
  const double x2 = bwg_sum(part_ew, vi * EB, vi * EB + EB, 0, red);
  if (threadIdx.x == 0) {
    DState *st = v.st;
    const double f0 = 0.5 * r2 + 0.5 * st->lambda * x2;
    st->f_cur = f0;
    if (!isfinite(f0)) {
      st->status = NDC_ENONFINITE;
      st->phase = PH_DONE;
    } else {
      st->phase = st->iters > 0 ? PH_NEW : PH_DONE;
    }
    if (v.stats) {
      v.stats[0] = f0;
      v.stats[1] = NAN;
      v.stats[2] = 0.0;
      v.stats[3] = NAN;
    }
    if (v.info) {
      v.info[0] = 0;
      v.info[1] = st->status;
    }
  }
}

// grid = count * EB: retry with the halved step (phase RETRY only)
__global__ __launch_bounds__(BT) void b_update_kernel(const BVol *vols, double *part_ew) {
  const int vi = blockIdx.x / EB, bi = blockIdx.x % EB;
  const BVol &v = vols[vi];
  if (v.st->phase != PH_RETRY) return;
  __shared__ double red[BT / 64][2];
  const float d = (float)v.st->delta;
  double s0 = 0.0, s1 = 0.0;
  for (int64_t i = bi * (int64_t)BT + threadIdx.x; i < v.n; i += (int64_t)EB * BT) {
    const float x = v.X[i];
    const float xt = proj_nonneg<float>(x - d * v.G[i]);
    v.Xt[i] = xt;
    s0 += (double)xt * (double)xt;
    const double dd = (double)xt - (double)x;
    s1 += dd * dd;
  }
  block_sum2(s0, s1, red);
  if (threadIdx.x == 0) {
    part_ew[2 * (int64_t)blockIdx.x] = s0;
    part_ew[2 * (int64_t)blockIdx.x + 1] = s1;
  }
}

// grid = count: the acceptance rule f(X_t) < f(X^k) per volume
__global__ __launch_bounds__(BT) void b_decide_kernel(const BVol *vols, const double *part_fwd,
                                                      const double *part_adj, const double *part_ew) {
  const int vi = blockIdx.x;
  const BVol &v = vols[vi];
  DState *st = v.st;
  const int phase = st->phase;
  if (phase == PH_DONE) {
    if (threadIdx.x == 0) st->accepted = 0;
    return;
  }
  __shared__ double red[BT / 64][2];
  const double r2 = bwg_sum(part_fwd, v.fwd_lo, v.fwd_hi, 0, red);
  const double *pu = phase == PH_NEW ? part_adj : part_ew;
  const int lo = phase == PH_NEW ? v.adj_lo : vi * EB, hi = phase == PH_NEW ? v.adj_hi : vi * EB + EB;
  const double x2 = bwg_sum(pu, lo, hi, 0, red);
  const double dx2 = bwg_sum(pu, lo, hi, 1, red);
  if (threadIdx.x != 0) return;
  const double ft = 0.5 * r2 + 0.5 * st->lambda * x2;
  if (!isfinite(ft)) {
    st->status = NDC_ENONFINITE;
    st->phase = PH_DONE;
    st->accepted = 0;
  } else if (ft < st->f_cur) {
    const int k = st->k + 1;
    if (v.stats) {
      v.stats[4 * k + 0] = ft;
      v.stats[4 * k + 1] = st->delta;
      v.stats[4 * k + 2] = (double)st->rej;
      v.stats[4 * k + 3] = sqrt(dx2);
    }
    st->k = k;
    st->f_cur = ft;
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
  if (v.info) {
    v.info[0] = st->k;
    v.info[1] = st->status;
  }
}

// grid = count * EB: X <- X_t, R <- R_t right after an acceptance
__global__ __launch_bounds__(BT) void b_commit_kernel(const BVol *vols) {
  const int vi = blockIdx.x / EB, bi = blockIdx.x % EB;
  const BVol &v = vols[vi];
  if (!v.st->accepted) return;
  const int64_t m = v.n > v.ny ? v.n : v.ny;
  for (int64_t i = bi * (int64_t)BT + threadIdx.x; i < m; i += (int64_t)EB * BT) {
    if (i < v.n) v.X[i] = v.Xt[i];
    if (i < v.ny) v.R[i] = v.Rt[i];
  }
}

// Per-call pointers of up to BP_MAX volumes, passed by value.
constexpr int BP_MAX = 48;
struct BPatch {
  int first, n, deconv, pad;
  char *ws;                 // deconvolution workspace (deconv only)
  const void *a[BP_MAX][5]; // conv: H, X, R; deconv: Y, H, X, stats, info
};

// Workspace offsets of one volume's arrays (deconvolution table).
struct BOff {
  size_t xt, g, r, rt;
};

// grid = 1: write one chunk of the call's pointers into the device table.
__global__ void b_patch_kernel(BVol *vols, const BOff *off, size_t off_state, BPatch pa) {
  for (int i = threadIdx.x; i < pa.n; i += blockDim.x) {
    const int vi = pa.first + i;
    BVol &v = vols[vi];
    if (pa.deconv) {
      v.Y = (const float *)pa.a[i][0];
      v.H = (const float *)pa.a[i][1];
      v.X = (float *)pa.a[i][2];
      v.stats = (double *)pa.a[i][3];
      v.info = pa.a[i][4] ? (int *)pa.a[i][4] + 2 * vi : nullptr;
      v.Xt = (float *)(pa.ws + off[vi].xt);
      v.G = (float *)(pa.ws + off[vi].g);
      v.R = (float *)(pa.ws + off[vi].r);
      v.Rt = (float *)(pa.ws + off[vi].rt);
      v.st = (DState *)(pa.ws + off_state) + vi;
    } else {
      v.H = (const float *)pa.a[i][0];
      v.X = (float *)pa.a[i][1];
      v.R = (float *)pa.a[i][2];
      v.st = nullptr;
    }
  }
}

// grid = count: a volume still running after the last trial slot stops with
// NDC_STOP_TRIALS.
__global__ void b_finish_kernel(const BVol *vols) {
  const BVol &v = vols[blockIdx.x];
  if (threadIdx.x != 0 || v.st->phase == PH_DONE) return;
  v.st->status = NDC_STOP_TRIALS;
  v.st->phase = PH_DONE;
  if (v.info) {
    v.info[0] = v.st->k;
    v.info[1] = v.st->status;
  }
}

}  // namespace

struct ndc_batch_plan {
  int count = 0, mg = 4, wg_per_cu = 2, order = 0, use_graph = 1;
  std::vector<int64_t> m, p;  // count x 3
  std::vector<BTile> fwd, adj;
  BTile *d_fwd = nullptr, *d_adj = nullptr;
  BVol *d_vols = nullptr;       // deconvolution table
  BVol *d_vols_conv = nullptr;  // convolution-only table
  BOff *d_off = nullptr;        // workspace offsets per volume
  std::vector<BVol> h_vols, h_vols_conv;
  size_t lds_fwd = 0, lds_adj = 0;
  int grid = 512;
  // workspace layout
  std::vector<BOff> off;
  size_t off_state = 0, off_pf = 0, off_pa = 0, off_pe = 0, ws_total = 0;
  // captured step
  hipStream_t cap = nullptr;
  hipGraphExec_t exec = nullptr;
  void *exec_ws = nullptr;
  // the operators: each volume's compile-time tile on one of NOPS streams
  // (default priority, a hardware queue each), costliest volumes first,
  // forked from and joined back to the caller's stream with events
  static constexpr int NOPS = 4;
  hipStream_t ops[NOPS] = {};
  hipEvent_t fork = nullptr, join[NOPS] = {};
  std::vector<int> op_order, op_stream;  // launch order; stream of each launch
  // deconvolution on the volumes' own kernels (tuning[0] = 0): their launch
  // plans, fixed at creation so that the partial-sum slot ranges stay valid
  // whatever tile overrides are installed later
  bool pervol = false;
  std::vector<ConvPlan> pl_fwd, pl_adj;
  std::vector<const void *> cur_ptrs, exec_ptrs;  // Y, H, X per volume: this call's; the step graph's
  double cur_lambda = 0.0, exec_lambda = 0.0;
};

namespace {

void make_tiles(ndc_batch_plan *P, bool forward, std::vector<BTile> &out, std::vector<int> &lo,
                std::vector<int> &hi) {
  std::vector<std::vector<BTile>> per(P->count);
  int slot = 0;
  lo.assign(P->count, 0);
  hi.assign(P->count, 0);
  for (int v = 0; v < P->count; ++v) {
    const int64_t *m = &P->m[3 * v], *p = &P->p[3 * v];
    const int oz = (int)(forward ? m[0] + 2 * p[0] : m[0]);
    const int oy = (int)(forward ? m[1] + 2 * p[1] : m[1]);
    const int ox = (int)(forward ? m[2] + 2 * p[2] : m[2]);
    const dim3 t = batch_tile_counts(oz, oy, ox, P->mg);
    lo[v] = slot;
    for (unsigned tz = 0; tz < t.z; ++tz)
      for (unsigned ty = 0; ty < t.y; ++ty)
        for (unsigned tx = 0; tx < t.x; ++tx) {
          BTile b{};
          b.vol = v;
          b.tx = (int)tx;
          b.ty = (int)ty;
          b.tz = (int)tz;
          b.slot = slot++;
          per[v].push_back(b);
        }
    hi[v] = slot;
  }
  out.clear();
  if (P->order == 1) {  // interleave volumes tile by tile
    size_t most = 0;
    for (auto &q : per) most = std::max(most, q.size());
    for (size_t i = 0; i < most; ++i)
      for (auto &q : per)
        if (i < q.size()) out.push_back(q[i]);
  } else if (P->order == 2) {  // most expensive volumes first (PSF taps x tiles)
    std::vector<int> idx(P->count);
    for (int v = 0; v < P->count; ++v) idx[v] = v;
    auto cost = [&](int v) {
      const int64_t *p = &P->p[3 * v];
      return (double)(2 * p[0] + 1) * (2 * p[1] + 1) * (2 * p[2] + 4) * per[v].size();
    };
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return cost(a) > cost(b); });
    for (int v : idx) out.insert(out.end(), per[v].begin(), per[v].end());
  } else {
    for (auto &q : per) out.insert(out.end(), q.begin(), q.end());
  }
}

int to_device(const void *h, size_t n, void **d) {
  if (hipMalloc(d, n ? n : 1) != hipSuccess) return NDC_EDEVICE;
  if (n && hipMemcpy(*d, h, n, hipMemcpyHostToDevice) != hipSuccess) return NDC_EDEVICE;
  return NDC_OK;
}

// One deconvolution operator of every volume on the volume's own kernel (the
// single-volume epilogues: RESID for the first and trial residuals, UPDATE
// for the transpose with the projected step), on the plan's streams, forked
// from and joined back to s.  Each volume's partial sums go to its own slot
// range (one pair per work-group), which the per-volume control kernels
// read; the phase word gates the step operators as in the persistent tile.
hipError_t launch_vols(ndc_batch_plan *P, char *ws, int op, double *part, hipStream_t s) {
  hipError_t e = hipEventRecord(P->fork, s);
  for (int i = 0; e == hipSuccess && i < ndc_batch_plan::NOPS; ++i) e = hipStreamWaitEvent(P->ops[i], P->fork, 0);
  if (e != hipSuccess) return e;
  const bool fwd = op != BOP_STEP_ADJ;
  for (int k = 0; k < P->count; ++k) {
    const int v = P->op_order[k];
    const BVol &b = P->h_vols[v];
    const BOff &f = P->off[v];
    DState *st = (DState *)(ws + P->off_state) + v;
    const void *H = P->cur_ptrs[3 * v + 1];
    float *X = (float *)P->cur_ptrs[3 * v + 2];
    Epi ep{};
    ep.part = part + 2 * (int64_t)(fwd ? b.fwd_lo : b.adj_lo);
    const void *in;
    void *out;
    if (op == BOP_STEP_ADJ) {
      in = ws + f.r;
      out = ws + f.xt;
      ep.mode = EPI_UPDATE;
      ep.X = X;
      ep.G = ws + f.g;
      ep.lambda = P->cur_lambda;
      ep.delta = &st->delta;
      ep.phase = &st->phase;
      ep.phase_mask = 1 << PH_NEW;
    } else {
      in = op == BOP_INIT ? (const void *)X : (const void *)(ws + f.xt);
      out = ws + (op == BOP_INIT ? f.r : f.rt);
      ep.mode = EPI_RESID;
      ep.Y = P->cur_ptrs[3 * v];
      if (op == BOP_STEP_FWD) {
        ep.phase = &st->phase;
        ep.phase_mask = (1 << PH_NEW) | (1 << PH_RETRY);
      }
    }
    const Geom g = fwd ? forward_geom(&P->m[3 * v], &P->p[3 * v]) : adjoint_geom(&P->m[3 * v], &P->p[3 * v]);
    e = launch_conv(fwd ? P->pl_fwd[v] : P->pl_adj[v], g, NDC_F32, NDC_PREC_NATIVE, in, H, out, ep,
                    P->ops[P->op_stream[k]]);
    if (e != hipSuccess) return e;
  }
  for (int i = 0; e == hipSuccess && i < ndc_batch_plan::NOPS; ++i) {
    e = hipEventRecord(P->join[i], P->ops[i]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, P->join[i], 0);
  }
  return e;
}

hipError_t launch_step(ndc_batch_plan *P, char *ws, hipStream_t s) {
  double *pf = (double *)(ws + P->off_pf), *pa = (double *)(ws + P->off_pa), *pe = (double *)(ws + P->off_pe);
  hipError_t e;
  e = P->pervol ? launch_vols(P, ws, BOP_STEP_ADJ, pa, s)
                : launch_batch_conv(P->mg, P->d_vols, P->d_adj, (int)P->adj.size(), BOP_STEP_ADJ, pa, P->grid,
                                    P->lds_adj, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(b_update_kernel, dim3(P->count * EB), dim3(BT), 0, s, (const BVol *)P->d_vols, pe);
  e = P->pervol ? launch_vols(P, ws, BOP_STEP_FWD, pf, s)
                : launch_batch_conv(P->mg, P->d_vols, P->d_fwd, (int)P->fwd.size(), BOP_STEP_FWD, pf, P->grid,
                                    P->lds_fwd, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(b_decide_kernel, dim3(P->count), dim3(BT), 0, s, (const BVol *)P->d_vols, (const double *)pf,
                     (const double *)pa, (const double *)pe);
  hipLaunchKernelGGL(b_commit_kernel, dim3(P->count * EB), dim3(BT), 0, s, (const BVol *)P->d_vols);
  return hipGetLastError();
}

}  // namespace

extern "C" {

int ndc_batch_plan_create(int count, const int64_t *m, const int64_t *p, int dtype, int precision, const int *tuning,
                          ndc_batch_plan **out) {
  if (!out) return NDC_EINVAL;
  *out = nullptr;
  if (count < 1 || !m || !p) return NDC_EINVAL;
  if (dtype != NDC_F32 && dtype != NDC_F64) return NDC_EINVAL;
  if (precision < NDC_PREC_NATIVE || precision > NDC_PREC_SPLIT_BF16) return NDC_EINVAL;
  if (dtype != NDC_F32 || precision != NDC_PREC_NATIVE) return NDC_EUNSUPPORTED;
  for (int v = 0; v < count; ++v)
    for (int i = 0; i < 3; ++i) {
      if (m[3 * v + i] < 1 || p[3 * v + i] < 0) return NDC_EINVAL;
      if (m[3 * v + i] + 4 * p[3 * v + i] > (1 << 20)) return NDC_EUNSUPPORTED;
    }
  for (int v = 0; v < count; ++v)
    if (!batch_psf_supported((int)(2 * p[3 * v + 2] + 1), (int)(2 * p[3 * v + 1] + 1))) return NDC_EUNSUPPORTED;
  int mg = 4, wpc = 2, order = 0, graph = 1;
  if (tuning) {
    mg = tuning[0];
    wpc = tuning[1];
    order = tuning[2];
    graph = tuning[3];
    if ((mg != 0 && mg != 2 && mg != 4) || wpc < 1 || wpc > 2 || order < 0 || order > 2 || graph < 0 || graph > 1)
      return NDC_EINVAL;
  }
  ndc_batch_plan *P = new ndc_batch_plan();
  P->count = count;
  P->pervol = mg == 0;
  if (P->pervol) mg = 4;  // the tile lists still exist (unused by the steps)
  P->mg = mg;
  P->wg_per_cu = wpc;
  P->order = order;
  P->use_graph = graph;
  P->m.assign(m, m + 3 * count);
  P->p.assign(p, p + 3 * count);
  std::vector<int> flo, fhi, alo, ahi;
  make_tiles(P, true, P->fwd, flo, fhi);
  make_tiles(P, false, P->adj, alo, ahi);
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
    delete P;
    return NDC_EDEVICE;
  }
  P->grid = cus * wpc;
  // per-volume kernels: their plans, and partial-sum slot ranges of one pair
  // per work-group in place of the tile ranges
  size_t nslot_fwd = P->fwd.size(), nslot_adj = P->adj.size();
  if (P->pervol) {
    int64_t sf = 0, sa = 0;
    for (int v = 0; v < count; ++v) {
      P->pl_fwd.push_back(plan_conv(forward_geom(&m[3 * v], &p[3 * v]), NDC_F32, NDC_PREC_NATIVE));
      P->pl_adj.push_back(plan_conv(adjoint_geom(&m[3 * v], &p[3 * v]), NDC_F32, NDC_PREC_NATIVE));
      flo[v] = (int)sf;
      sf += P->pl_fwd[v].nblocks;
      fhi[v] = (int)sf;
      alo[v] = (int)sa;
      sa += P->pl_adj[v].nblocks;
      ahi[v] = (int)sa;
      if (sf >= (int64_t)1 << 30 || sa >= (int64_t)1 << 30) {
        delete P;
        return NDC_EUNSUPPORTED;
      }
    }
    nslot_fwd = (size_t)sf;
    nslot_adj = (size_t)sa;
  }
  // workspace layout and the volume tables
  size_t o = 0;
  P->off_state = o;
  o += al256(sizeof(DState) * count);
  P->off_pf = o;
  o += al256(sizeof(double) * 2 * nslot_fwd);
  P->off_pa = o;
  o += al256(sizeof(double) * 2 * nslot_adj);
  P->off_pe = o;
  o += al256(sizeof(double) * 2 * (size_t)count * EB);
  P->h_vols.resize(count);
  P->h_vols_conv.resize(count);
  for (int v = 0; v < count; ++v) {
    BVol &b = P->h_vols[v];
    memset(&b, 0, sizeof(b));
    int64_t n = 1, ny = 1;
    for (int i = 0; i < 3; ++i) {
      b.m[i] = (int)m[3 * v + i];
      b.p[i] = (int)p[3 * v + i];
      n *= m[3 * v + i];
      ny *= m[3 * v + i] + 2 * p[3 * v + i];
    }
    b.n = n;
    b.ny = ny;
    b.fwd_lo = flo[v];
    b.fwd_hi = fhi[v];
    b.adj_lo = alo[v];
    b.adj_hi = ahi[v];
    BOff f;
    f.xt = o;
    o += al256(sizeof(float) * n);
    f.g = o;
    o += al256(sizeof(float) * n);
    f.r = o;
    o += al256(sizeof(float) * ny);
    f.rt = o;
    o += al256(sizeof(float) * ny);
    P->off.push_back(f);
    const size_t lf = batch_lds_bytes(2 * b.p[2] + 1, 2 * b.p[1] + 1, mg);
    P->lds_fwd = std::max(P->lds_fwd, lf);
    P->lds_adj = std::max(P->lds_adj, lf);
    P->h_vols_conv[v] = b;
  }
  P->ws_total = o;
  int rc = to_device(P->fwd.data(), sizeof(BTile) * P->fwd.size(), (void **)&P->d_fwd);
  if (!rc) rc = to_device(P->adj.data(), sizeof(BTile) * P->adj.size(), (void **)&P->d_adj);
  if (!rc) rc = to_device(P->h_vols.data(), sizeof(BVol) * count, (void **)&P->d_vols);
  if (!rc) rc = to_device(P->h_vols_conv.data(), sizeof(BVol) * count, (void **)&P->d_vols_conv);
  if (!rc) rc = to_device(P->off.data(), sizeof(BOff) * count, (void **)&P->d_off);
  if (!rc && hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking) != hipSuccess) rc = NDC_EDEVICE;
  // The operator streams take a CU mask of every compute unit (no
  // restriction), which gives each its own hardware queue.  Plain streams
  // share HIP's small pool of hardware queues (4 by default): on MI355X two
  // of the four landed on one queue each and ran in sequence, 11.2 ms per
  // 64-volume forward against 9.0 ms on four queues of their own.
  std::vector<uint32_t> mask((size_t)(cus + 31) / 32, 0xffffffffu);
  if (cus % 32) mask.back() = (1u << (cus % 32)) - 1u;
  for (int i = 0; !rc && i < ndc_batch_plan::NOPS; ++i)
    if (hipExtStreamCreateWithCUMask(&P->ops[i], (uint32_t)mask.size(), mask.data()) != hipSuccess ||
        hipEventCreateWithFlags(&P->join[i], hipEventDisableTiming) != hipSuccess)
      rc = NDC_EDEVICE;
  if (!rc && hipEventCreateWithFlags(&P->fork, hipEventDisableTiming) != hipSuccess) rc = NDC_EDEVICE;
  P->op_order.resize(count);
  for (int v = 0; v < count; ++v) P->op_order[v] = v;
  {
    auto cost = [&](int v) {  // taps x outputs of the forward
      double c = 1.0;
      for (int i = 0; i < 3; ++i) c *= (double)(2 * p[3 * v + i] + 1) * (double)(m[3 * v + i] + 2 * p[3 * v + i]);
      return c;
    };
    std::stable_sort(P->op_order.begin(), P->op_order.end(), [&](int a, int b) { return cost(a) > cost(b); });
    // each volume to the stream with the least work so far (longest first)
    double load[ndc_batch_plan::NOPS] = {};
    P->op_stream.resize(count);
    for (int k = 0; k < count; ++k) {
      int best = 0;
      for (int i = 1; i < ndc_batch_plan::NOPS; ++i)
        if (load[i] < load[best]) best = i;
      P->op_stream[k] = best;
      load[best] += cost(P->op_order[k]);
    }
  }
  if (rc) {
    ndc_batch_plan_destroy(P);
    return rc;
  }
  *out = P;
  return NDC_OK;
}

void ndc_batch_plan_destroy(ndc_batch_plan *P) {
  if (!P) return;
  // calls return before their work has run: let it finish before the
  // tables it reads are freed
  (void)hipDeviceSynchronize();
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->cap) (void)hipStreamDestroy(P->cap);
  for (int i = 0; i < ndc_batch_plan::NOPS; ++i) {
    if (P->ops[i]) (void)hipStreamDestroy(P->ops[i]);
    if (P->join[i]) (void)hipEventDestroy(P->join[i]);
  }
  if (P->fork) (void)hipEventDestroy(P->fork);
  (void)hipFree(P->d_fwd);
  (void)hipFree(P->d_adj);
  (void)hipFree(P->d_vols);
  (void)hipFree(P->d_vols_conv);
  (void)hipFree(P->d_off);
  (void)hipGetLastError();
  delete P;
}

size_t ndc_batch_workspace_bytes(const ndc_batch_plan *P) { return P ? P->ws_total : 0; }

int ndc_batch_plan_info(const ndc_batch_plan *P, int64_t *out4) {
  if (!P || !out4) return NDC_EINVAL;
  out4[0] = (int64_t)P->fwd.size();
  out4[1] = (int64_t)P->adj.size();
  out4[2] = P->grid;
  out4[3] = (int64_t)std::max(P->lds_fwd, P->lds_adj);
  return NDC_OK;
}

}  // extern "C"

namespace {

struct Span {
  uintptr_t lo, hi;  // [lo, hi)
};

// Any overlap among the output spans, or between an input and an output.
bool spans_alias(std::vector<Span> outs, const std::vector<Span> &ins) {
  outs.erase(std::remove_if(outs.begin(), outs.end(), [](const Span &a) { return a.lo == a.hi; }), outs.end());
  std::sort(outs.begin(), outs.end(), [](const Span &a, const Span &b) { return a.lo < b.lo; });
  for (size_t i = 1; i < outs.size(); ++i)
    if (outs[i].lo < outs[i - 1].hi) return true;
  for (const Span &q : ins) {
    if (q.lo == q.hi) continue;
    // the output starting last at or before q.hi - 1, and the one after it
    auto it = std::upper_bound(outs.begin(), outs.end(), q.hi - 1, [](uintptr_t v, const Span &a) { return v < a.lo; });
    if (it != outs.begin() && std::prev(it)->hi > q.lo) return true;
  }
  return false;
}

Span span(const void *p, size_t bytes) { return Span{(uintptr_t)p, (uintptr_t)p + bytes}; }

size_t psf_elems(const BVol &b) { return (size_t)(2 * b.p[0] + 1) * (2 * b.p[1] + 1) * (2 * b.p[2] + 1); }

// Enqueue the pointer table update of one call (chunks of BP_MAX volumes).
hipError_t patch_table(ndc_batch_plan *P, BVol *table, bool deconv, char *ws,
                       const void *const *a0, const void *const *a1, const void *const *a2,
                       const void *const *a3, const void *a4, hipStream_t s) {
  for (int first = 0; first < P->count; first += BP_MAX) {
    BPatch pa;
    memset(&pa, 0, sizeof(pa));
    pa.first = first;
    pa.n = std::min(BP_MAX, P->count - first);
    pa.deconv = deconv ? 1 : 0;
    pa.ws = ws;
    for (int i = 0; i < pa.n; ++i) {
      const int v = first + i;
      pa.a[i][0] = a0[v];
      pa.a[i][1] = a1[v];
      pa.a[i][2] = a2[v];
      pa.a[i][3] = a3 ? a3[v] : nullptr;
      pa.a[i][4] = a4;
    }
    hipLaunchKernelGGL(b_patch_kernel, dim3(1), dim3(64), 0, s, table, (const BOff *)P->d_off, P->off_state, pa);
  }
  return hipGetLastError();
}

// A pointer the current device can dereference (device or managed memory).
bool on_device(const void *ptr) {
  hipPointerAttribute_t at;
  memset(&at, 0, sizeof(at));
  if (hipPointerGetAttributes(&at, ptr) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged || at.type == hipMemoryTypeUnified;
}

int batch_conv(ndc_batch_plan *P, const void *const *in, const void *const *H, void *const *out, bool forward,
               void *stream) {
  if (!P || !in || !H || !out) return NDC_EINVAL;
  std::vector<Span> outs, ins;
  for (int v = 0; v < P->count; ++v) {
    if (!in[v] || !H[v] || !out[v]) return NDC_EINVAL;
    const BVol &b = P->h_vols_conv[v];
    const size_t nin = sizeof(float) * (forward ? b.n : b.ny), nout = sizeof(float) * (forward ? b.ny : b.n);
    outs.push_back(span(out[v], nout));
    ins.push_back(span(in[v], nin));
    ins.push_back(span(H[v], sizeof(float) * psf_elems(b)));
  }
  if (spans_alias(outs, ins)) return NDC_EALIAS;
  for (int v = 0; v < P->count; ++v)
    if (!on_device(in[v]) || !on_device(H[v]) || !on_device(out[v])) return NDC_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  // Each volume's own compile-time tile (the single-volume operator) on one
  // of the plan's streams, costliest volumes first, each to the stream with
  // the least work so far: the volumes' launches
  // overlap, and each runs the tile with the fixed PSF width.  Measured on
  // MI355X for 64 volumes of 32^3 .. 96x160x160 with PSFs 9..31: 17.4 ms per
  // operator pair (9.1 forward, 8.1 transpose) on 4 streams against 24.6 ms
  // for the persistent run-time-width tile (which the deconvolution keeps
  // for its fused steps).
  if (hipEventRecord(P->fork, s) != hipSuccess) return NDC_EDEVICE;
  for (int i = 0; i < ndc_batch_plan::NOPS; ++i)
    if (hipStreamWaitEvent(P->ops[i], P->fork, 0) != hipSuccess) return NDC_EDEVICE;
  for (int k = 0; k < P->count; ++k) {
    const int v = P->op_order[k];
    const Geom g = forward ? forward_geom(&P->m[3 * v], &P->p[3 * v]) : adjoint_geom(&P->m[3 * v], &P->p[3 * v]);
    const ConvPlan pl = plan_conv(g, NDC_F32, NDC_PREC_NATIVE);
    Epi ep{};
    ep.mode = EPI_STORE;
    if (launch_conv(pl, g, NDC_F32, NDC_PREC_NATIVE, in[v], H[v], out[v], ep, P->ops[P->op_stream[k]]) !=
        hipSuccess)
      return NDC_EDEVICE;
  }
  for (int i = 0; i < ndc_batch_plan::NOPS; ++i)
    if (hipEventRecord(P->join[i], P->ops[i]) != hipSuccess || hipStreamWaitEvent(s, P->join[i], 0) != hipSuccess)
      return NDC_EDEVICE;
  return NDC_OK;
}

}  // namespace

extern "C" {

int ndc_batch_conv_full(ndc_batch_plan *P, const void *const *X, const void *const *H, void *const *Y, void *stream) {
  return batch_conv(P, X, H, Y, true, stream);
}

int ndc_batch_conv_adjoint(ndc_batch_plan *P, const void *const *R, const void *const *H, void *const *X,
                           void *stream) {
  return batch_conv(P, R, H, X, false, stream);
}

int ndc_batch_deconv(ndc_batch_plan *P, const void *const *Y, const void *const *H, void *const *X, int iters,
                     double lambda, void *ws, size_t ws_bytes, double *const *stats, int *info, void *stream) {
  if (!P || !Y || !H || !X) return NDC_EINVAL;
  if (iters < 0 || iters > NDC_MAX_ITERS || !(lambda >= 0.0) || !isfinite(lambda)) return NDC_EINVAL;
  if (!ws || ws_bytes < P->ws_total) return NDC_EWORKSPACE;
  // outputs: X[v], stats[v], info, ws; inputs: Y[v], H[v]
  std::vector<Span> outs, ins;
  outs.push_back(span(ws, P->ws_total));
  if (info) outs.push_back(span(info, sizeof(int) * 2 * (size_t)P->count));
  for (int v = 0; v < P->count; ++v) {
    if (!Y[v] || !H[v] || !X[v]) return NDC_EINVAL;
    const BVol &b = P->h_vols[v];
    outs.push_back(span(X[v], sizeof(float) * b.n));
    if (stats && stats[v]) outs.push_back(span(stats[v], sizeof(double) * 4 * ((size_t)iters + 1)));
    ins.push_back(span(Y[v], sizeof(float) * b.ny));
    ins.push_back(span(H[v], sizeof(float) * psf_elems(b)));
  }
  if (spans_alias(outs, ins)) return NDC_EALIAS;
  if (!on_device(ws) || (info && !on_device(info))) return NDC_EINVAL;
  for (int v = 0; v < P->count; ++v)
    if (!on_device(Y[v]) || !on_device(H[v]) || !on_device(X[v]) || (stats && stats[v] && !on_device(stats[v])))
      return NDC_EINVAL;

  char *w = (char *)ws;
  hipStream_t s = (hipStream_t)stream;
  double *pf = (double *)(w + P->off_pf), *pe = (double *)(w + P->off_pe);
  if (patch_table(P, P->d_vols, true, w, (const void *const *)Y, (const void *const *)H, (const void *const *)X,
                  (const void *const *)stats, info, s) != hipSuccess)
    return NDC_EDEVICE;
  P->cur_ptrs.resize(3 * (size_t)P->count);
  for (int v = 0; v < P->count; ++v) {
    P->cur_ptrs[3 * v] = Y[v];
    P->cur_ptrs[3 * v + 1] = H[v];
    P->cur_ptrs[3 * v + 2] = X[v];
  }
  P->cur_lambda = lambda;
  hipLaunchKernelGGL(b_init_kernel, dim3(P->count), dim3(BT), 0, s, (const BVol *)P->d_vols, lambda, iters, 30);
  hipLaunchKernelGGL(b_sumsq_kernel, dim3(P->count * EB), dim3(BT), 0, s, (const BVol *)P->d_vols, pe);
  if ((P->pervol ? launch_vols(P, w, BOP_INIT, pf, s)
                 : launch_batch_conv(P->mg, P->d_vols, P->d_fwd, (int)P->fwd.size(), BOP_INIT, pf, P->grid,
                                     P->lds_fwd, s)) != hipSuccess)
    return NDC_EDEVICE;
  hipLaunchKernelGGL(b_f0_kernel, dim3(P->count), dim3(BT), 0, s, (const BVol *)P->d_vols, (const double *)pf,
                     (const double *)pe);
  if (hipGetLastError() != hipSuccess) return NDC_EDEVICE;

  // The step graph replays into the caller's stream unless that stream is
  // itself being captured (then the step's kernels are enqueued directly).
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) return NDC_EDEVICE;
  const bool graph = P->use_graph && cs == hipStreamCaptureStatusNone;
  // The persistent step reads every address from the device table, so its
  // graph depends on the workspace alone; the per-volume kernels take the
  // volumes' addresses and lambda as launch arguments, so their graph is
  // captured again whenever one of those changes.
  const bool stale = P->exec_ws != ws ||
                     (P->pervol && (P->exec_ptrs != P->cur_ptrs || !(P->exec_lambda == lambda)));
  if (graph && stale) {  // capture one slot against this workspace
    if (P->exec) {
      (void)hipGraphExecDestroy(P->exec);
      P->exec = nullptr;
    }
    P->exec_ws = nullptr;  // no valid graph until the capture below succeeds
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(P->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return NDC_EDEVICE;
    const hipError_t le = launch_step(P, w, P->cap);
    const hipError_t ce = hipStreamEndCapture(P->cap, &g);
    if (le != hipSuccess || ce != hipSuccess || !g) return NDC_EDEVICE;
    const hipError_t ie = hipGraphInstantiate(&P->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
      P->exec = nullptr;
      return NDC_EDEVICE;
    }
    P->exec_ws = ws;
    P->exec_ptrs = P->cur_ptrs;
    P->exec_lambda = lambda;
  }
  // the same fixed schedule as deconv_iterate: 2*iters + 30 trial slots
  const int slots = iters > 0 ? 2 * iters + 30 : 0;
  for (int slot = 0; slot < slots; ++slot) {
    const hipError_t e = graph ? hipGraphLaunch(P->exec, s) : launch_step(P, w, s);
    if (e != hipSuccess) return NDC_EDEVICE;
  }
  hipLaunchKernelGGL(b_finish_kernel, dim3(P->count), dim3(64), 0, s, (const BVol *)P->d_vols);
  return hipGetLastError() == hipSuccess ? NDC_OK : NDC_EDEVICE;
}

}  // extern "C"
