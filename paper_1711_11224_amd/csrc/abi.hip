// C ABI entry points (include/ndconv.h): argument checks, n-D folding,
// kernel-variant choice and launches.  Every check runs before anything is
// enqueued; nothing here throws, aborts or allocates device memory.
#include <limits.h>
#include <math.h>

#include <mutex>
#include <vector>
#include <stdlib.h>
#include <string.h>

#include "ndc_device.h"
#include "ndc_internal.h"

namespace ndc {

size_t deconv_ws_bytes(const int64_t m3[3], const int64_t p3[3], int dtype, int precision, int reg_ndim);
int deconv_run(const int64_t m3[3], const int64_t p3[3], const void *Y, const void *H, void *X, int iters,
               double lambda, double mu, int ndim, int dtype, int precision, void *ws, double *stats, int *info,
               int rule, int slots, hipStream_t s);
size_t rl_ws_bytes(const int64_t m3[3], const int64_t p3[3], int dtype, int precision);
int rl_run(const int64_t m3[3], const int64_t p3[3], const void *Y, const void *H, void *X, int iters, int dtype,
           int precision, void *ws, double *stats, int *info, hipStream_t s);
bool mfma_supported(const Geom &g, int dtype, int precision);
bool dh_supported(const int64_t m3[3], const int64_t p3[3], int dtype);
size_t dh_workspace_bytes(const int64_t m3[3], const int64_t p3[3], int dtype);
hipError_t launch_dh(const int64_t m3[3], const int64_t p3[3], int dtype, const void *X, const void *G, void *dH,
                     void *ws, hipStream_t s);
ConvPlan plan_conv_mfma(const Geom &g, int dtype, int precision, int xb);
bool mfma32_supported(const Geom &g, int dtype, int precision);
bool mfma32_fits(const Geom &g, int dtype, int precision);
bool mfma32_nt_ok(int nt, int precision);
ConvPlan plan_conv_mfma32(const Geom &g, int precision, int nt);
hipError_t launch_conv_mfma32(const ConvPlan &pl, const Geom &g, int precision, const void *in, const void *H,
                              void *out, const Epi &ep, hipStream_t s);
bool slot_fits(const Geom &g, int dtype, int precision);
bool slot_preferred(const Geom &g, int dtype, int precision);
ConvPlan plan_conv_slot(const Geom &g);
bool slot32_fits(const Geom &g, int dtype, int precision);
ConvPlan plan_conv_slot32(const Geom &g);
hipError_t launch_conv_slot32(const ConvPlan &pl, const Geom &g, const void *in, const void *H, void *out,
                              const Epi &ep, hipStream_t s);
hipError_t launch_conv_slot(const ConvPlan &pl, const Geom &g, const void *in, const void *H, void *out,
                            const Epi &ep, hipStream_t s);
bool small_supported(const Geom &g, int dtype, int precision);
int64_t small_blocks(const Geom &g, int dtype);
hipError_t launch_conv_small(const Geom &g, int dtype, const void *in, const void *H, void *out, const Epi &ep,
                             hipStream_t s);
hipError_t launch_conv_mfma(const ConvPlan &pl, const Geom &g, int dtype, int precision, const void *in,
                            const void *H, void *out, const Epi &ep, hipStream_t s);

bool fold3(int n, const int64_t *m, const int64_t *p, int64_t m3[3], int64_t p3[3]) {
  if (n < 1 || n > 3) return false;
  for (int i = 0; i < 3; ++i) {
    m3[i] = 1;
    p3[i] = 0;
  }
  for (int i = 0; i < n; ++i) {
    m3[3 - n + i] = m[i];
    p3[3 - n + i] = p[i];
  }
  return true;
}

Geom forward_geom(const int64_t m3[3], const int64_t p3[3]) {
  Geom g;
  g.oz = (int)(m3[0] + 2 * p3[0]);
  g.oy = (int)(m3[1] + 2 * p3[1]);
  g.ox = (int)(m3[2] + 2 * p3[2]);
  g.iz = (int)m3[0];
  g.iy = (int)m3[1];
  g.ix = (int)m3[2];
  g.kz = (int)(2 * p3[0] + 1);
  g.ky = (int)(2 * p3[1] + 1);
  g.kx = (int)(2 * p3[2] + 1);
  g.offz = (int)(2 * p3[0]);
  g.offy = (int)(2 * p3[1]);
  g.offx = (int)(2 * p3[2]);
  g.flip = 1;
  return g;
}

Geom adjoint_geom(const int64_t m3[3], const int64_t p3[3]) {
  Geom g;
  g.oz = (int)m3[0];
  g.oy = (int)m3[1];
  g.ox = (int)m3[2];
  g.iz = (int)(m3[0] + 2 * p3[0]);
  g.iy = (int)(m3[1] + 2 * p3[1]);
  g.ix = (int)(m3[2] + 2 * p3[2]);
  g.kz = (int)(2 * p3[0] + 1);
  g.ky = (int)(2 * p3[1] + 1);
  g.kx = (int)(2 * p3[2] + 1);
  g.offz = g.offy = g.offx = 0;
  g.flip = 0;
  return g;
}

static int64_t grid_blocks(dim3 g) { return (int64_t)g.x * g.y * g.z; }

// Variant choice: small PSFs (every axis <= 7 taps) are bound by HBM and
// stream through conv_small; large bf16 PSFs (57+ planes of 25+ x 25+ taps)
// take the row-slot tile; other wide ones go to the matrix cores when the x
// width fits the MFMA tile (the bf16 forms of rows 11..33 taps wide on the
// 32x32x16 instruction, the rest on the 4x4 forms); everything else takes
// the general VALU kernel.
static bool small_fits(const Geom &g, int dtype, int precision) {
  return g.kx <= 7 && g.ky <= 7 && g.kz <= 7 && small_supported(g, dtype, precision);
}

static bool use_small(const Geom &g, int dtype, int precision) {
  return small_fits(g, dtype, precision) && !getenv("NDC_FORCE_VALU");
}

static ConvPlan plan_small(const Geom &g, int dtype) {
  ConvPlan pl{};
  pl.variant = 2;
  pl.nblocks = small_blocks(g, dtype);
  pl.grid = dim3((unsigned)pl.nblocks);
  pl.block = dim3(256);
  return pl;
}

static ConvPlan plan_valu(const Geom &g) {
  ConvPlan pl{};
  pl.variant = 0;
  pl.grid = valu_grid(g, 1);
  pl.block = dim3(256);
  pl.nblocks = grid_blocks(pl.grid);
  return pl;
}

// Whether `form` (NDC_FORM_*) with `param` can run this problem.
static bool form_fits(const Geom &g, int dtype, int precision, int form, int param) {
  switch (form) {
    case NDC_FORM_VALU: return true;
    case NDC_FORM_SMALL: return small_fits(g, dtype, precision);
    case NDC_FORM_MFMA4:
      return mfma_supported(g, dtype, precision) &&
             (param == 8 || (param == 16 && precision == NDC_PREC_NATIVE));
    case NDC_FORM_MFMA32:
      return mfma32_fits(g, dtype, precision) && mfma_supported(g, dtype, precision) &&
             mfma32_nt_ok(param, precision);
    case NDC_FORM_SLOT: return slot_fits(g, dtype, precision) || slot32_fits(g, dtype, precision);
    default: return false;
  }
}

// Kernel-form overrides set by ndc_tile_override (the autotuner): exact
// problem geometry, storage type and precision -> form and its parameter.
struct TileOverride {
  Geom g;
  int dtype, precision, form, param;
};
static std::mutex override_mu;
static std::vector<TileOverride> overrides;

static bool same_geom(const Geom &a, const Geom &b) {
  return a.oz == b.oz && a.oy == b.oy && a.ox == b.ox && a.iz == b.iz && a.iy == b.iy && a.ix == b.ix &&
         a.kz == b.kz && a.ky == b.ky && a.kx == b.kx && a.offz == b.offz && a.offy == b.offy &&
         a.offx == b.offx && a.flip == b.flip;
}

static bool find_override(const Geom &g, int dtype, int precision, int &form, int &param) {
  std::lock_guard<std::mutex> lock(override_mu);
  for (const TileOverride &o : overrides)
    if (o.dtype == dtype && o.precision == precision && same_geom(o.g, g)) {
      form = o.form;
      param = o.param;
      return true;
    }
  return false;
}

ConvPlan plan_conv(const Geom &g, int dtype, int precision) {
  int form = 0, param = 0;
  if (find_override(g, dtype, precision, form, param) && form_fits(g, dtype, precision, form, param)) {
    switch (form) {
      case NDC_FORM_SMALL: return plan_small(g, dtype);
      case NDC_FORM_MFMA4: return plan_conv_mfma(g, dtype, precision, param);
      case NDC_FORM_MFMA32: return plan_conv_mfma32(g, precision, param);
      case NDC_FORM_SLOT: return precision == NDC_PREC_BF16 ? plan_conv_slot(g) : plan_conv_slot32(g);
      default: return plan_valu(g);
    }
  }
  if (use_small(g, dtype, precision)) return plan_small(g, dtype);
  if (slot_preferred(g, dtype, precision)) return plan_conv_slot(g);
  if (mfma32_supported(g, dtype, precision) && mfma_supported(g, dtype, precision))
    return plan_conv_mfma32(g, precision, 0);
  if (mfma_supported(g, dtype, precision)) return plan_conv_mfma(g, dtype, precision, 0);
  return plan_valu(g);
}

hipError_t launch_conv(const ConvPlan &pl, const Geom &g, int dtype, int precision, const void *in, const void *H,
                       void *out, const Epi &ep, hipStream_t s) {
  if (pl.variant == 1) return launch_conv_mfma(pl, g, dtype, precision, in, H, out, ep, s);
  if (pl.variant == 2) return launch_conv_small(g, dtype, in, H, out, ep, s);
  if (pl.variant == 3) return launch_conv_mfma32(pl, g, precision, in, H, out, ep, s);
  if (pl.variant == 4) return launch_conv_slot(pl, g, in, H, out, ep, s);
  if (pl.variant == 5) return launch_conv_slot32(pl, g, in, H, out, ep, s);
  return launch_conv_valu(g, dtype, precision, in, H, out, ep, 1, g.kz, s);
}

}  // namespace ndc

using namespace ndc;

namespace {

// Largest extent any axis may take (input, output or tap) so that every
// in-kernel index fits in int; the 3-D folding keeps products in int64.
constexpr int64_t kMaxAxis = (int64_t)1 << 24;
constexpr int64_t kMaxElems = (int64_t)1 << 36;
constexpr int kMaxGridYZ = 65535;

int check_problem(int n, const int64_t *m, const int64_t *p, int dtype, int precision, int64_t m3[3],
                  int64_t p3[3]) {
  if (n < 1 || !m || !p) return NDC_EINVAL;
  if (n > 3) return NDC_EUNSUPPORTED;
  for (int i = 0; i < n; ++i)
    if (m[i] < 1 || p[i] < 0) return NDC_EINVAL;
  if (dtype != NDC_F32 && dtype != NDC_F64) return NDC_EINVAL;
  if (precision != NDC_PREC_NATIVE && precision != NDC_PREC_BF16 && precision != NDC_PREC_SPLIT_BF16)
    return NDC_EINVAL;
  if (dtype == NDC_F64 && precision != NDC_PREC_NATIVE) return NDC_EUNSUPPORTED;
  fold3(n, m, p, m3, p3);
  int64_t ny = 1;
  for (int i = 0; i < 3; ++i) {
    if (m3[i] > kMaxAxis || p3[i] > kMaxAxis || m3[i] + 4 * p3[i] > kMaxAxis) return NDC_EUNSUPPORTED;
    ny *= m3[i] + 2 * p3[i];
    if (ny > kMaxElems) return NDC_EUNSUPPORTED;
  }
  // grid limits of the launches (y: 16-row tiles, z: output planes)
  if (m3[0] + 2 * p3[0] > kMaxGridYZ || (m3[1] + 2 * p3[1] + 15) / 16 > kMaxGridYZ) return NDC_EUNSUPPORTED;
  return NDC_OK;
}

size_t esize(int dtype) { return dtype == NDC_F64 ? sizeof(double) : sizeof(float); }

bool overlap(const void *a, size_t na, const void *b, size_t nb) {
  const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
  return na && nb && x < y + nb && y < x + na;
}

// A pointer the current device can dereference (device or managed memory).
bool device_ptr(const void *ptr) {
  hipPointerAttribute_t at;
  memset(&at, 0, sizeof(at));
  hipError_t e = hipPointerGetAttributes(&at, ptr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged || at.type == hipMemoryTypeUnified;
}

struct Extents {
  int64_t m3[3], p3[3];
  size_t nx, ny, nh;  // element counts
};

int prepare(int n, const int64_t *m, const int64_t *p, int dtype, int precision, Extents &E) {
  int rc = check_problem(n, m, p, dtype, precision, E.m3, E.p3);
  if (rc) return rc;
  E.nx = E.ny = E.nh = 1;
  for (int i = 0; i < 3; ++i) {
    E.nx *= (size_t)E.m3[i];
    E.ny *= (size_t)(E.m3[i] + 2 * E.p3[i]);
    E.nh *= (size_t)(2 * E.p3[i] + 1);
  }
  return NDC_OK;
}

}  // namespace

extern "C" {

const char *ndc_strerror(int status) {
  switch (status) {
    case NDC_OK: return "success";
    case NDC_EINVAL: return "invalid argument (rank, extent, half-width, count, pointer or scalar)";
    case NDC_EUNSUPPORTED:
      return "valid request the library does not support (rank > 3, sizes, bf16 with FP64, or a kernel form that "
             "cannot run the problem)";
    case NDC_EALIAS: return "an output buffer overlaps an input or another output";
    case NDC_ENONFINITE: return "non-finite objective";
    case NDC_EDEVICE: return "HIP runtime or kernel launch failure";
    case NDC_EWORKSPACE: return "workspace missing or too small";
    default: return "unknown status";
  }
}

int ndc_version(void) { return (1 << 16) | 0; }

int ndc_tile_override(int n, const int64_t *m, const int64_t *p, int dtype, int precision, int op, int form,
                      int param) {
  Extents E;
  int rc = prepare(n, m, p, dtype, precision, E);
  if (rc) return rc;
  if (op != 0 && op != 1) return NDC_EINVAL;
  if (form < NDC_FORM_AUTO || form > NDC_FORM_SLOT) return NDC_EINVAL;
  const Geom g = op == 0 ? forward_geom(E.m3, E.p3) : adjoint_geom(E.m3, E.p3);
  if (form != NDC_FORM_AUTO && !form_fits(g, dtype, precision, form, param)) return NDC_EUNSUPPORTED;
  std::lock_guard<std::mutex> lock(override_mu);
  for (size_t i = 0; i < overrides.size(); ++i)
    if (overrides[i].dtype == dtype && overrides[i].precision == precision && same_geom(overrides[i].g, g)) {
      overrides.erase(overrides.begin() + (long)i);
      break;
    }
  if (form != NDC_FORM_AUTO) {
    if (overrides.size() >= NDC_MAX_TILE_OVERRIDES) return NDC_EUNSUPPORTED;
    overrides.push_back(TileOverride{g, dtype, precision, form, form == NDC_FORM_MFMA4 || form == NDC_FORM_MFMA32 ? param : 0});
  }
  return NDC_OK;
}

void ndc_tile_override_clear(void) {
  std::lock_guard<std::mutex> lock(override_mu);
  overrides.clear();
}

int ndc_tile_choice(int n, const int64_t *m, const int64_t *p, int dtype, int precision, int op, int *out2) {
  Extents E;
  int rc = prepare(n, m, p, dtype, precision, E);
  if (rc) return rc;
  if ((op != 0 && op != 1) || !out2) return NDC_EINVAL;
  const Geom g = op == 0 ? forward_geom(E.m3, E.p3) : adjoint_geom(E.m3, E.p3);
  const ConvPlan pl = plan_conv(g, dtype, precision);
  static const int form_of[6] = {NDC_FORM_VALU, NDC_FORM_MFMA4, NDC_FORM_SMALL, NDC_FORM_MFMA32, NDC_FORM_SLOT,
                                 NDC_FORM_SLOT};
  out2[0] = form_of[pl.variant];
  out2[1] = pl.variant == 1 ? pl.xb : (pl.variant == 3 ? pl.nt : 0);
  return NDC_OK;
}

int conv_full_nd(int n, const int64_t *m, const int64_t *p, const void *X, const void *H, void *Y, int dtype,
                 int precision, void *stream) {
  Extents E;
  int rc = prepare(n, m, p, dtype, precision, E);
  if (rc) return rc;
  if (!X || !H || !Y) return NDC_EINVAL;
  const size_t es = esize(dtype);
  if (overlap(Y, E.ny * es, X, E.nx * es) || overlap(Y, E.ny * es, H, E.nh * es)) return NDC_EALIAS;
  if (!device_ptr(X) || !device_ptr(H) || !device_ptr(Y)) return NDC_EINVAL;
  const Geom g = forward_geom(E.m3, E.p3);
  const ConvPlan pl = plan_conv(g, dtype, precision);
  Epi ep{};
  ep.mode = EPI_STORE;
  return launch_conv(pl, g, dtype, precision, X, H, Y, ep, (hipStream_t)stream) == hipSuccess ? NDC_OK
                                                                                              : NDC_EDEVICE;
}

int conv_adjoint_nd(int n, const int64_t *m, const int64_t *p, const void *R, const void *H, void *X, int dtype,
                    int precision, void *stream) {
  Extents E;
  int rc = prepare(n, m, p, dtype, precision, E);
  if (rc) return rc;
  if (!R || !H || !X) return NDC_EINVAL;
  const size_t es = esize(dtype);
  if (overlap(X, E.nx * es, R, E.ny * es) || overlap(X, E.nx * es, H, E.nh * es)) return NDC_EALIAS;
  if (!device_ptr(R) || !device_ptr(H) || !device_ptr(X)) return NDC_EINVAL;
  const Geom g = adjoint_geom(E.m3, E.p3);
  const ConvPlan pl = plan_conv(g, dtype, precision);
  Epi ep{};
  ep.mode = EPI_STORE;
  return launch_conv(pl, g, dtype, precision, R, H, X, ep, (hipStream_t)stream) == hipSuccess ? NDC_OK
                                                                                              : NDC_EDEVICE;
}

// dH = valid correlation of G (extent m+2p) with X (extent m) as the taps:
// output extent 2p+1.  Split-K over X's z-planes keeps the chip busy; the
// per-split outputs go to the workspace and are summed in fixed order.
static void dH_split(const int64_t m3[3], const int64_t p3[3], Geom &g, int &ksplit, int &zchunk) {
  g.oz = (int)(2 * p3[0] + 1);
  g.oy = (int)(2 * p3[1] + 1);
  g.ox = (int)(2 * p3[2] + 1);
  g.iz = (int)(m3[0] + 2 * p3[0]);
  g.iy = (int)(m3[1] + 2 * p3[1]);
  g.ix = (int)(m3[2] + 2 * p3[2]);
  g.kz = (int)m3[0];
  g.ky = (int)m3[1];
  g.kx = (int)m3[2];
  g.offz = g.offy = g.offx = 0;
  g.flip = 0;
  const dim3 base = valu_grid(g, 1);
  const int64_t nb = grid_blocks(base);
  int64_t s = (2048 + nb - 1) / nb;
  if (s > g.kz) s = g.kz;
  if (s * g.oz > kMaxGridYZ) s = kMaxGridYZ / g.oz;
  if (s < 1) s = 1;
  zchunk = (int)((g.kz + s - 1) / s);
  ksplit = (g.kz + zchunk - 1) / zchunk;
}

size_t conv_dH_workspace_bytes(int n, const int64_t *m, const int64_t *p, int dtype) {
  Extents E;
  if (prepare(n, m, p, dtype, NDC_PREC_NATIVE, E)) return 0;
  if (dh_supported(E.m3, E.p3, dtype)) return dh_workspace_bytes(E.m3, E.p3, dtype);
  Geom g;
  int ks, zc;
  dH_split(E.m3, E.p3, g, ks, zc);
  return ks > 1 ? (size_t)ks * E.nh * esize(dtype) : 0;
}

}  // extern "C"

// conv_dH_nd's body.  With scratch_max > 0 the split-K partials go to the
// library's own scratch array (conv_dH_nd_noalloc): `ws` is then obtained
// only after every argument check, from get_scratch, and must fit in
// scratch_max bytes.
int ndc::dH_checked(int n, const int64_t *m, const int64_t *p, const void *X, const void *G, void *dH, int dtype,
                    void *ws, size_t ws_bytes, size_t scratch_max, void *(*get_scratch)(), void *stream) {
  Extents E;
  int rc = prepare(n, m, p, dtype, NDC_PREC_NATIVE, E);
  if (rc) return rc;
  if (!X || !G || !dH) return NDC_EINVAL;
  const size_t es = esize(dtype);
  Geom g;
  int ks, zc;
  dH_split(E.m3, E.p3, g, ks, zc);
  const bool dedicated = dh_supported(E.m3, E.p3, dtype);
  const size_t need = dedicated ? dh_workspace_bytes(E.m3, E.p3, dtype) : (ks > 1 ? (size_t)ks * E.nh * es : 0);
  if (scratch_max) {
    if (need > scratch_max) return NDC_EWORKSPACE;
  } else if (need && (!ws || ws_bytes < need)) {
    return NDC_EWORKSPACE;
  }
  if (overlap(dH, E.nh * es, X, E.nx * es) || overlap(dH, E.nh * es, G, E.ny * es)) return NDC_EALIAS;
  if (!scratch_max && need &&
      (overlap(ws, need, X, E.nx * es) || overlap(ws, need, G, E.ny * es) || overlap(ws, need, dH, E.nh * es)))
    return NDC_EALIAS;
  if (!device_ptr(X) || !device_ptr(G) || !device_ptr(dH) || (!scratch_max && need && !device_ptr(ws)))
    return NDC_EINVAL;
  if (scratch_max && need) {
    ws = get_scratch();
    if (!ws) return NDC_EDEVICE;
  }
  Epi ep{};
  ep.mode = EPI_STORE;
  hipStream_t s = (hipStream_t)stream;
  if (dedicated) return launch_dh(E.m3, E.p3, dtype, X, G, dH, ws, s) == hipSuccess ? NDC_OK : NDC_EDEVICE;
  if (ks == 1) {
    if (launch_conv_valu(g, dtype, NDC_PREC_NATIVE, G, X, dH, ep, 1, g.kz, s) != hipSuccess) return NDC_EDEVICE;
    return NDC_OK;
  }
  if (launch_conv_valu(g, dtype, NDC_PREC_NATIVE, G, X, ws, ep, ks, zc, s) != hipSuccess) return NDC_EDEVICE;
  if (launch_splitk_reduce(dtype, ws, dH, (int64_t)E.nh, ks, s) != hipSuccess) return NDC_EDEVICE;
  return NDC_OK;
}

extern "C" {

int conv_dH_nd(int n, const int64_t *m, const int64_t *p, const void *X, const void *G, void *dH, int dtype,
               void *ws, size_t ws_bytes, void *stream) {
  return dH_checked(n, m, p, X, G, dH, dtype, ws, ws_bytes, 0, nullptr, stream);
}

size_t deconv_workspace_bytes(int n, const int64_t *m, const int64_t *p, int dtype, int precision) {
  Extents E;
  if (prepare(n, m, p, dtype, precision, E)) return 0;
  return deconv_ws_bytes(E.m3, E.p3, dtype, precision, 0);
}

size_t deconv_workspace_bytes_ex(int n, const int64_t *m, const int64_t *p, int dtype, int precision,
                                 int regularised) {
  Extents E;
  if (prepare(n, m, p, dtype, precision, E)) return 0;
  return deconv_ws_bytes(E.m3, E.p3, dtype, precision, regularised ? n : 0);
}

// Trial slots enqueued by one call: `iters` accepted steps, one rejected
// trial per step on average, and one full halving sequence.
static int default_trials(int iters) { return iters > 0 ? 2 * iters + 30 : 0; }

static int deconv_checked(int n, const int64_t *m, const int64_t *p, const void *Y, const void *H, void *X,
                          int iters, double lambda, double mu, int dtype, int precision, int rule, int max_trials,
                          void *ws, size_t ws_bytes, double *stats, int *info, void *stream) {
  if (rule != NDC_STEP_FIXED && rule != NDC_STEP_CAUCHY && rule != NDC_STEP_BB) return NDC_EINVAL;
  if (!(mu >= 0.0) || !isfinite(mu)) return NDC_EINVAL;
  Extents E;
  int rc = prepare(n, m, p, dtype, precision, E);
  if (rc) return rc;
  if (!Y || !H || !X) return NDC_EINVAL;
  if (iters < 0 || iters > NDC_MAX_ITERS || !(lambda >= 0.0) || !isfinite(lambda)) return NDC_EINVAL;
  if (max_trials < 0 || max_trials > 2 * NDC_MAX_ITERS + 30) return NDC_EINVAL;
  const int slots = iters == 0 ? 0 : (max_trials > 0 ? max_trials : default_trials(iters));
  const size_t need = deconv_ws_bytes(E.m3, E.p3, dtype, precision, mu > 0.0 ? n : 0);
  if (!ws || ws_bytes < need) return NDC_EWORKSPACE;
  const size_t es = esize(dtype);
  const size_t ns = stats ? (size_t)4 * ((size_t)iters + 1) * sizeof(double) : 0;
  const size_t ni = info ? 2 * sizeof(int) : 0;
  // outputs: X, ws, stats, info; inputs: Y, H
  const void *outs[4] = {X, ws, stats, info};
  const size_t outn[4] = {E.nx * es, need, ns, ni};
  for (int i = 0; i < 4; ++i) {
    if (overlap(outs[i], outn[i], Y, E.ny * es) || overlap(outs[i], outn[i], H, E.nh * es)) return NDC_EALIAS;
    for (int j = i + 1; j < 4; ++j)
      if (overlap(outs[i], outn[i], outs[j], outn[j])) return NDC_EALIAS;
  }
  if (!device_ptr(Y) || !device_ptr(H) || !device_ptr(X) || !device_ptr(ws)) return NDC_EINVAL;
  if ((stats && !device_ptr(stats)) || (info && !device_ptr(info))) return NDC_EINVAL;
  return deconv_run(E.m3, E.p3, Y, H, X, iters, lambda, mu, n, dtype, precision, ws, stats, info, rule, slots,
                    (hipStream_t)stream);
}

int deconv_iterate(int n, const int64_t *m, const int64_t *p, const void *Y, const void *H, void *X, int iters,
                   double lambda, int dtype, int precision, void *ws, size_t ws_bytes, double *stats, int *info,
                   void *stream) {
  return deconv_checked(n, m, p, Y, H, X, iters, lambda, 0.0, dtype, precision, NDC_STEP_FIXED, 0, ws, ws_bytes,
                        stats, info, stream);
}

size_t rl_workspace_bytes(int n, const int64_t *m, const int64_t *p, int dtype, int precision) {
  Extents E;
  if (prepare(n, m, p, dtype, precision, E)) return 0;
  return rl_ws_bytes(E.m3, E.p3, dtype, precision);
}

int rl_iterate(int n, const int64_t *m, const int64_t *p, const void *Y, const void *H, void *X, int iters,
               int dtype, int precision, void *ws, size_t ws_bytes, double *stats, int *info, void *stream) {
  Extents E;
  int rc = prepare(n, m, p, dtype, precision, E);
  if (rc) return rc;
  if (!Y || !H || !X) return NDC_EINVAL;
  if (iters < 0 || iters > NDC_MAX_ITERS) return NDC_EINVAL;
  const size_t need = rl_ws_bytes(E.m3, E.p3, dtype, precision);
  if (!ws || ws_bytes < need) return NDC_EWORKSPACE;
  const size_t es = esize(dtype);
  const size_t ns = stats ? ((size_t)iters + 1) * sizeof(double) : 0;
  const size_t ni = info ? 2 * sizeof(int) : 0;
  const void *outs[4] = {X, ws, stats, info};
  const size_t outn[4] = {E.nx * es, need, ns, ni};
  for (int i = 0; i < 4; ++i) {
    if (overlap(outs[i], outn[i], Y, E.ny * es) || overlap(outs[i], outn[i], H, E.nh * es)) return NDC_EALIAS;
    for (int j = i + 1; j < 4; ++j)
      if (overlap(outs[i], outn[i], outs[j], outn[j])) return NDC_EALIAS;
  }
  if (!device_ptr(Y) || !device_ptr(H) || !device_ptr(X) || !device_ptr(ws)) return NDC_EINVAL;
  if ((stats && !device_ptr(stats)) || (info && !device_ptr(info))) return NDC_EINVAL;
  return rl_run(E.m3, E.p3, Y, H, X, iters, dtype, precision, ws, stats, info, (hipStream_t)stream);
}

int deconv_iterate_ex(int n, const int64_t *m, const int64_t *p, const void *Y, const void *H, void *X, int iters,
                      double lambda, double mu, int dtype, int precision, int rule, int max_trials, void *ws,
                      size_t ws_bytes, double *stats, int *info, void *stream) {
  return deconv_checked(n, m, p, Y, H, X, iters, lambda, mu, dtype, precision, rule, max_trials, ws, ws_bytes,
                        stats, info, stream);
}

}  // extern "C"
