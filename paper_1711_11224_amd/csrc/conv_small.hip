// Small-PSF streaming kernel: variant checks, launch shape and dispatch to
// the instantiations (conv_small.h; one translation unit per storage type
// and pair of z tap counts).
#include "conv_small.h"

namespace ndc {

hipError_t launch_small_f32_k13(const Geom &g, const void *in, const void *H, void *out, const Epi &ep, hipStream_t s);
int occupancy_small_f32_k13(const Geom &g);
hipError_t launch_small_f32_k5(const Geom &g, const void *in, const void *H, void *out, const Epi &ep, hipStream_t s);
int occupancy_small_f32_k5(const Geom &g);
hipError_t launch_small_f32_k7(const Geom &g, const void *in, const void *H, void *out, const Epi &ep, hipStream_t s);
int occupancy_small_f32_k7(const Geom &g);
hipError_t launch_small_f64_k13(const Geom &g, const void *in, const void *H, void *out, const Epi &ep, hipStream_t s);
int occupancy_small_f64_k13(const Geom &g);
hipError_t launch_small_f64_k5(const Geom &g, const void *in, const void *H, void *out, const Epi &ep, hipStream_t s);
int occupancy_small_f64_k5(const Geom &g);
hipError_t launch_small_f64_k7(const Geom &g, const void *in, const void *H, void *out, const Epi &ep, hipStream_t s);
int occupancy_small_f64_k7(const Geom &g);

// Output planes per work-group: about 16, with the number of work-groups
// snapped to a whole number of rounds of resident work-groups (a partial last
// round leaves most CUs idle while it runs), and no fewer than 2 (kz - 1),
// which bounds the restaged z halo to half the planes.
int small_zchunk(const Geom &g, int per_cu) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess || cus < 1) {
    (void)hipGetLastError();
    cus = 1;
  }
  const double columns = (double)((g.ox + STX - 1) / STX) * ((g.oy + STY - 1) / STY);
  const double per_round = (double)per_cu * cus / columns;  // z chunks per column in one round
  const double rounds = std::max(1.0, std::round(std::ceil(g.oz / 16.0) / per_round));
  const int64_t chunks = std::max<int64_t>(1, std::llround(rounds * per_round));
  const int zc = (int)((g.oz + chunks - 1) / chunks);
  return std::max(zc, std::min(g.oz, std::max(1, 2 * (g.kz - 1))));
}

namespace {

hipError_t launch_small_dt(const Geom &g, int dtype, const void *in, const void *H, void *out, const Epi &ep,
                           hipStream_t s) {
  if (dtype == NDC_F64) {
    if (g.kz <= 3) return launch_small_f64_k13(g, in, H, out, ep, s);
    return g.kz == 5 ? launch_small_f64_k5(g, in, H, out, ep, s) : launch_small_f64_k7(g, in, H, out, ep, s);
  }
  if (g.kz <= 3) return launch_small_f32_k13(g, in, H, out, ep, s);
  return g.kz == 5 ? launch_small_f32_k5(g, in, H, out, ep, s) : launch_small_f32_k7(g, in, H, out, ep, s);
}

int small_occupancy_dt(const Geom &g, int dtype) {
  if (dtype == NDC_F64) {
    if (g.kz <= 3) return occupancy_small_f64_k13(g);
    return g.kz == 5 ? occupancy_small_f64_k5(g) : occupancy_small_f64_k7(g);
  }
  if (g.kz <= 3) return occupancy_small_f32_k13(g);
  return g.kz == 5 ? occupancy_small_f32_k5(g) : occupancy_small_f32_k7(g);
}

}  // namespace

bool small_supported(const Geom &g, int dtype, int precision) {
  if (precision != NDC_PREC_NATIVE) return false;
  if (g.kx > SMAXK || g.ky > SMAXK || g.kz > SMAXK || !(g.kx & 1) || !(g.kz & 1)) return false;
  if (g.offz < 0) return false;
  if ((int64_t)g.iy * g.ix >= ((int64_t)1 << 31)) return false;  // 31-bit element offsets inside a plane
  const size_t bytes = dtype == NDC_F64 ? small_lds_bytes<double>(g.kz) : small_lds_bytes<float>(g.kz);
  return bytes <= 64 * 1024;
}

int64_t small_blocks(const Geom &g, int dtype) {
  const int zc = small_zchunk(g, small_occupancy_dt(g, dtype));
  return (int64_t)((g.ox + STX - 1) / STX) * ((g.oy + STY - 1) / STY) * ((g.oz + zc - 1) / zc);
}

hipError_t launch_conv_small(const Geom &g, int dtype, const void *in, const void *H, void *out, const Epi &ep,
                             hipStream_t s) {
  return launch_small_dt(g, dtype, in, H, out, ep, s);
}

}  // namespace ndc
