// PSF gradient  dH[a,b,c] = sum_{z,y,x} X[z,y,x] G[z+a, y+b, x+c]
// (the transpose of Property 1 with X as the template; G = X (x) H - Y).
//
// The output is PSF-sized and the contraction runs over all of X, so the
// kernel splits the contraction (split-K over X's z-planes) and parallelises
// over PSF planes a:
//   work-group (a, split s): one PSF plane, X planes [s*zc, (s+1)*zc);
//   thread b + ky*cg: PSF row b, taps c = 8cg .. 8cg+7 of that row.
// X and G tiles of 8 rows x 128 columns are staged in LDS; every thread
// reads the same X values (LDS broadcast) and a sliding 12-wide window of its
// G row, 32 FMAs per 4 LDS reads.  Threads are numbered along b first.  Sums are blocked per staged tile, and the
// per-split planes are added in fixed order in double precision afterwards.
#include "ndc_device.h"
#include "ndc_internal.h"

namespace ndc {
namespace {

constexpr int DYC = 8;    // X rows per staged tile
constexpr int DXC = 128;  // X columns per staged tile
constexpr int DCT = 8;    // taps per thread along x

struct DhGeom {
  int mz, my, mx;     // X extent
  int kz, ky, kx;     // PSF extent
  int gy, gx;         // G extent in y, x (my+ky-1, mx+kx-1)
  int ncg;            // thread groups along c
  int zc, nsplit;     // X planes per split, number of splits
  int gstride;        // LDS row stride of the G tile
};

template <typename T>
__global__ void dh_kernel(const T *__restrict__ X, const T *__restrict__ G, T *__restrict__ part, DhGeom d) {
  extern __shared__ __align__(16) unsigned char dh_lds[];
  T *xs = (T *)dh_lds;             // DYC x DXC
  T *gs = xs + DYC * DXC;          // (DYC + ky - 1) x gstride
  const int a = blockIdx.x % d.kz, s = blockIdx.x / d.kz;
  // lanes run along b first: with the G row stride = 4 mod 32 floats, eight
  // consecutive lanes' 16-byte window reads land on distinct bank groups
  const int tid = threadIdx.x, cg = tid / d.ky, b = tid - cg * d.ky;
  const bool active = cg < d.ncg;
  const int c0 = DCT * cg;
  const int grow = DYC + d.ky - 1;

  double outer[DCT];
#pragma unroll
  for (int r = 0; r < DCT; ++r) outer[r] = 0.0;

  const int z_lo = s * d.zc, z_hi = min(d.mz, z_lo + d.zc);
  for (int z = z_lo; z < z_hi; ++z) {
    for (int y0 = 0; y0 < d.my; y0 += DYC) {
      for (int x0 = 0; x0 < d.mx; x0 += DXC) {
        __syncthreads();
        for (int e = tid; e < DYC * DXC; e += blockDim.x) {
          const int r = e / DXC, q = e - r * DXC;
          const int y = y0 + r, x = x0 + q;
          xs[e] = (y < d.my && x < d.mx) ? X[((int64_t)z * d.my + y) * d.mx + x] : (T)0;
        }
        for (int e = tid; e < grow * d.gstride; e += blockDim.x) {
          const int r = e / d.gstride, q = e - r * d.gstride;
          const int y = y0 + r, x = x0 + q;
          gs[e] = (y < d.gy && x < d.gx && q < DXC + d.kx - 1) ? G[((int64_t)(z + a) * d.gy + y) * d.gx + x] : (T)0;
        }
        __syncthreads();
        if (active) {
          T acc[DCT];
#pragma unroll
          for (int r = 0; r < DCT; ++r) acc[r] = (T)0;
          for (int y = 0; y < DYC; ++y) {
            const T *xrow = xs + y * DXC;
            const T *grow_p = gs + (y + b) * d.gstride + c0;
            for (int x = 0; x < DXC; x += 4) {
              T xv[4], w[DCT + 4];
#pragma unroll
              for (int u = 0; u < 4; ++u) xv[u] = xrow[x + u];
#pragma unroll
              for (int u = 0; u < DCT + 4; ++u) w[u] = grow_p[x + u];
#pragma unroll
              for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int r = 0; r < DCT; ++r) acc[r] += xv[u] * w[u + r];
            }
          }
#pragma unroll
          for (int r = 0; r < DCT; ++r) outer[r] += (double)acc[r];
        }
      }
    }
  }
  if (active) {
    T *dst = part + (int64_t)s * d.kz * d.ky * d.kx + ((int64_t)a * d.ky + b) * d.kx;
#pragma unroll
    for (int r = 0; r < DCT; ++r)
      if (c0 + r < d.kx) dst[c0 + r] = (T)outer[r];
  }
}

DhGeom dh_geom(const int64_t m3[3], const int64_t p3[3]) {
  DhGeom d;
  d.mz = (int)m3[0];
  d.my = (int)m3[1];
  d.mx = (int)m3[2];
  d.kz = (int)(2 * p3[0] + 1);
  d.ky = (int)(2 * p3[1] + 1);
  d.kx = (int)(2 * p3[2] + 1);
  d.gy = d.my + d.ky - 1;
  d.gx = d.mx + d.kx - 1;
  d.ncg = (d.kx + DCT - 1) / DCT;
  // enough work-groups to fill the chip, each a whole number of X planes
  int want = (4096 + d.kz - 1) / d.kz;
  if (want > d.mz) want = d.mz;
  if (want < 1) want = 1;
  d.zc = (d.mz + want - 1) / want;
  d.nsplit = (d.mz + d.zc - 1) / d.zc;
  d.gstride = ((DXC + DCT * d.ncg + 4 + 27) / 32) * 32 + 4;  // >= needed columns, = 4 mod 32
  return d;
}

size_t dh_lds_bytes(const DhGeom &d, size_t es) {
  return es * ((size_t)DYC * DXC + (size_t)(DYC + d.ky - 1) * d.gstride);
}

}  // namespace

bool dh_supported(const int64_t m3[3], const int64_t p3[3], int dtype) {
  const DhGeom d = dh_geom(m3, p3);
  const size_t es = dtype == NDC_F64 ? 8 : 4;
  return d.ky * d.ncg <= 256 && dh_lds_bytes(d, es) <= 96 * 1024;
}

size_t dh_workspace_bytes(const int64_t m3[3], const int64_t p3[3], int dtype) {
  const DhGeom d = dh_geom(m3, p3);
  const size_t es = dtype == NDC_F64 ? 8 : 4;
  return (size_t)d.nsplit * d.kz * d.ky * d.kx * es;
}

hipError_t launch_dh(const int64_t m3[3], const int64_t p3[3], int dtype, const void *X, const void *G, void *dH,
                     void *ws, hipStream_t s) {
  const DhGeom d = dh_geom(m3, p3);
  const size_t es = dtype == NDC_F64 ? 8 : 4;
  const int threads = ((d.ky * d.ncg + 63) / 64) * 64;
  const dim3 grid((unsigned)(d.kz * d.nsplit));
  const size_t lds = dh_lds_bytes(d, es);
  static bool attr_set = false;  // allow up to 96 KB of LDS (idempotent)
  if (!attr_set) {
    (void)hipFuncSetAttribute((const void *)dh_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    (void)hipFuncSetAttribute((const void *)dh_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    (void)hipGetLastError();
    attr_set = true;
  }
  if (dtype == NDC_F64)
    hipLaunchKernelGGL(dh_kernel<double>, grid, dim3(threads), lds, s, (const double *)X, (const double *)G,
                       (double *)ws, d);
  else
    hipLaunchKernelGGL(dh_kernel<float>, grid, dim3(threads), lds, s, (const float *)X, (const float *)G,
                       (float *)ws, d);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_splitk_reduce(dtype, ws, dH, (int64_t)d.kz * d.ky * d.kx, d.nsplit, s);
}

}  // namespace ndc
