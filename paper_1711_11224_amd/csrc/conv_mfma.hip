// Single-volume launches of the matrix-core correlation tile (mfma_tile.h).
#include "mfma_tile.h"

namespace ndc {
namespace {
using namespace mfma;

template <int KX, int PREC, int XB>
__global__ __launch_bounds__(MT, 2) void conv_mfma_kernel(const float *__restrict__ in, const float *__restrict__ H,
                                                          float *__restrict__ out, Geom g, Epi ep, int nbx, int nby,
                                                          int nbz) {
  if (ep.phase && !((1 << *ep.phase) & ep.phase_mask)) return;  // uniform early exit
  extern __shared__ __align__(16) float lds[];
  __shared__ double red[MT / 64][2];
  // Tiles in x-fastest order.  (An XCD-grouped, z-fastest order that keeps
  // tiles sharing input planes on one L2 cuts HBM fetches but ends each XCD
  // on expensive mid-volume tiles; measured 5% slower for the forward.)
  const int id = blockIdx.x;
  (void)nbz;
  mfma_tile<KX, PREC, MG_DEFAULT, XB>(in, H, out, g, ep, id % nbx, (id / nbx) % nby, id / (nbx * nby), id, lds,
                                     red);
}

// x-blocks per instruction for a launch (see TileDims): 32-column tiles when
// they pad the output's x extent less than 64-column ones, and for the bf16
// forms (measured faster at every workload size); otherwise 64 columns.
int choose_xb(const Geom &g, int precision) {
  // the 32 x 32 tile (two row sets of operands in flight) unless the
  // 16-row x 64-column tile covers the output plane with less padding
  const int64_t a8 = (int64_t)((g.ox + 31) / 32) * ((g.oy + 31) / 32);
  const int64_t a16 = (int64_t)((g.ox + 63) / 64) * ((g.oy + 15) / 16);
  return (a8 <= a16 || precision != NDC_PREC_NATIVE) ? 8 : 16;
}

dim3 tile_counts(const Geom &g, int xb) {
  const int cols = 4 * xb, rows = 256 / xb;
  return dim3((g.ox + cols - 1) / cols, (g.oy + rows - 1) / rows, (g.oz + MG_DEFAULT - 1) / MG_DEFAULT);
}

template <int KX, int PREC, int XB>
hipError_t launch_kx_xb(const Geom &g, const void *in, const void *H, void *out, const Epi &ep, hipStream_t s) {
  using S = MfmaShape<KX, XB>;
  const size_t lds = sizeof(float) * (size_t)S::lds_floats(g.ky, MG_DEFAULT, PREC);
  // raise the dynamic-LDS limit once per process; call_once makes
  // concurrent first calls from several host threads safe
  static std::once_flag lds_once;
  std::call_once(lds_once, [] {
    (void)hipFuncSetAttribute((const void *)conv_mfma_kernel<KX, PREC, XB>,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)(sizeof(float) * S::lds_floats(MAX_KY, MG_DEFAULT, PREC)));
    (void)hipGetLastError();
  });
  const dim3 t = tile_counts(g, XB);
  const unsigned total = t.x * t.y * t.z;
  hipLaunchKernelGGL((conv_mfma_kernel<KX, PREC, XB>), dim3(total), dim3(MT), lds, s, (const float *)in,
                     (const float *)H, (float *)out, g, ep, (int)t.x, (int)t.y, (int)t.z);
  return hipGetLastError();
}

template <int KX, int PREC>
hipError_t launch_kx(int xb, const Geom &g, const void *in, const void *H, void *out, const Epi &ep,
                     hipStream_t s) {
  if constexpr (PREC != PREC_NATIVE_) {
    return launch_kx_xb<KX, PREC, 8>(g, in, H, out, ep, s);  // bf16 forms: 32 x 32 tile only
  } else {
    if (xb == 8) return launch_kx_xb<KX, PREC, 8>(g, in, H, out, ep, s);
    return launch_kx_xb<KX, PREC, 16>(g, in, H, out, ep, s);
  }
}

template <int PREC>
hipError_t launch_prec(int xb, const Geom &g, const void *in, const void *H, void *out, const Epi &ep,
                       hipStream_t s) {
  switch (g.kx) {
#define NDC_KX(K) \
  case K: return launch_kx<K, PREC>(xb, g, in, H, out, ep, s);
    NDC_KX(3) NDC_KX(5) NDC_KX(7) NDC_KX(9) NDC_KX(11) NDC_KX(13) NDC_KX(15) NDC_KX(17)
    NDC_KX(19) NDC_KX(21) NDC_KX(23) NDC_KX(25) NDC_KX(27) NDC_KX(29) NDC_KX(31) NDC_KX(33)
#undef NDC_KX
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool mfma_supported(const Geom &g, int dtype, int) {
  if (dtype != NDC_F32) return false;
  if (g.kx < 3 || g.kx > 33 || (g.kx & 1) == 0 || g.ky > MAX_KY) return false;
  if (getenv("NDC_FORCE_VALU")) return false;
  return true;
}

ConvPlan plan_conv_mfma(const Geom &g, int, int precision, int xb) {
  ConvPlan pl{};
  pl.variant = 1;
  pl.xb = precision != NDC_PREC_NATIVE ? 8 : (xb == 8 || xb == 16 ? xb : choose_xb(g, precision));
  const dim3 t = tile_counts(g, pl.xb);
  pl.grid = dim3(t.x * t.y * t.z);
  pl.block = dim3(MT);
  pl.lds_bytes = 0;
  pl.nblocks = (int64_t)t.x * t.y * t.z;
  return pl;
}

hipError_t launch_conv_mfma(const ConvPlan &pl, const Geom &g, int, int precision, const void *in, const void *H,
                            void *out, const Epi &ep, hipStream_t s) {
  switch (precision) {
    case NDC_PREC_BF16: return launch_prec<PREC_BF16_>(8, g, in, H, out, ep, s);
    case NDC_PREC_SPLIT_BF16: return launch_prec<PREC_SPLIT_>(8, g, in, H, out, ep, s);
    default: return launch_prec<PREC_NATIVE_>(pl.xb, g, in, H, out, ep, s);
  }
}

}  // namespace ndc
