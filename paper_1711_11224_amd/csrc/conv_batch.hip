// Persistent launch of the matrix-core correlation tile (mfma_tile.h) over
// a batch of volumes with their own extents and PSFs.
#include "mfma_tile.h"

namespace ndc {
namespace {
using namespace mfma;

__device__ inline Geom batch_geom(const BVol &v, bool forward) {
  Geom g;
  g.kz = 2 * v.p[0] + 1;
  g.ky = 2 * v.p[1] + 1;
  g.kx = 2 * v.p[2] + 1;
  if (forward) {
    g.oz = v.m[0] + 2 * v.p[0];
    g.oy = v.m[1] + 2 * v.p[1];
    g.ox = v.m[2] + 2 * v.p[2];
    g.iz = v.m[0];
    g.iy = v.m[1];
    g.ix = v.m[2];
    g.offz = 2 * v.p[0];
    g.offy = 2 * v.p[1];
    g.offx = 2 * v.p[2];
    g.flip = 1;
  } else {
    g.oz = v.m[0];
    g.oy = v.m[1];
    g.ox = v.m[2];
    g.iz = v.m[0] + 2 * v.p[0];
    g.iy = v.m[1] + 2 * v.p[1];
    g.ix = v.m[2] + 2 * v.p[2];
    g.offz = g.offy = g.offx = 0;
    g.flip = 0;
  }
  return g;
}

// Persistent launch over a tile list of many volumes with their own extents
// and PSFs: work-group w takes tiles w, w + grid, ... (a fixed assignment, so
// results do not depend on timing).  Volumes whose deconvolution phase has nothing
// to do skip their tiles.  The PSF width is a run-time value (mfma_tile_rt).
template <int MG>
__global__ __launch_bounds__(MT, 2) void batch_conv_kernel(const BVol *__restrict__ vols,
                                                           const BTile *__restrict__ tiles, int ntiles, int op,
                                                           double *__restrict__ part) {
  extern __shared__ __align__(16) float lds[];
  __shared__ double red[MT / 64][2];
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const BTile d = tiles[t];
    const BVol &v = vols[d.vol];
    const int ph = v.st ? v.st->phase : PH_NEW;
    if (op == BOP_STEP_ADJ && ph != PH_NEW) continue;
    if (op == BOP_STEP_FWD && ph == PH_DONE) continue;
    const bool fwd = (op == BOP_FWD || op == BOP_INIT || op == BOP_STEP_FWD);
    const Geom g = batch_geom(v, fwd);
    Epi ep{};
    ep.part = part;
    ep.phase = nullptr;
    const float *in;
    float *out;
    switch (op) {
      case BOP_FWD: in = v.X; out = v.R; ep.mode = EPI_STORE; break;
      case BOP_ADJ: in = v.R; out = v.X; ep.mode = EPI_STORE; break;
      case BOP_INIT: in = v.X; out = v.R; ep.mode = EPI_RESID; ep.Y = v.Y; break;
      case BOP_STEP_FWD: in = v.Xt; out = v.Rt; ep.mode = EPI_RESID; ep.Y = v.Y; break;
      default:
        in = v.R;
        out = v.Xt;
        ep.mode = EPI_UPDATE;
        ep.X = v.X;
        ep.G = v.G;
        ep.lambda = v.st->lambda;
        ep.delta = &v.st->delta;
        break;
    }
    mfma_tile_rt<MG>(in, v.H, out, g, ep, d.tx, d.ty, d.tz, d.slot, lds, red);
    __syncthreads();
  }
}


}  // namespace

bool batch_psf_supported(int kx, int ky) { return kx >= 3 && kx <= 33 && (kx & 1) && ky >= 1 && ky <= MAX_KY; }

dim3 batch_tile_counts(int oz, int oy, int ox, int mg) {
  return dim3((ox + MCOLS - 1) / MCOLS, (oy + MROWS - 1) / MROWS, (oz + mg - 1) / mg);
}

size_t batch_lds_bytes(int kx, int ky, int mg) {
  const RtShape S(kx);
  return sizeof(float) * (size_t)mfma_lds_floats(ky, S.stride, S.hs, mg);
}

hipError_t launch_batch_conv(int mg, const BVol *vols, const BTile *tiles, int ntiles, int op, double *part,
                             int grid, size_t lds_bytes, hipStream_t s) {
  // raise the dynamic-LDS limit once per process; call_once makes
  // concurrent first calls from several host threads safe
  static std::once_flag lds_once;
  std::call_once(lds_once, [] {
    const int cap = 160 * 1024 - 64;
    (void)hipFuncSetAttribute((const void *)batch_conv_kernel<2>, hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipFuncSetAttribute((const void *)batch_conv_kernel<4>, hipFuncAttributeMaxDynamicSharedMemorySize, cap);
    (void)hipGetLastError();
  });
  if (mg == 2)
    hipLaunchKernelGGL(batch_conv_kernel<2>, dim3(grid), dim3(MT), lds_bytes, s, vols, tiles, ntiles, op, part);
  else
    hipLaunchKernelGGL(batch_conv_kernel<4>, dim3(grid), dim3(MT), lds_bytes, s, vols, tiles, ntiles, op, part);
  return hipGetLastError();
}

}  // namespace ndc
