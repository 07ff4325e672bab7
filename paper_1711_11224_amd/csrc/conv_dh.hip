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

#include <type_traits>

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

// ---------------------------------------------------------------------------
// FP32 matrix-core form (v_mfma_f32_4x4x1f32, 16 independent 4x4 blocks).
//
// Instruction block k takes the x position x0 + k of a 16-wide chunk; lane
// 4k+i holds A_k[i] = G[zg, yg, x + c0 + i], lane 4k+j holds
// B_k[j] = X[zg - a, yg - b0 - j, x], so register i of lane 4k+j gathers
//   dH[a, b0 + j, c0 + i] += G[zg, yg, x + c0 + i] * X[zg - a, yg - b0 - j, x]
// for one G row yg: a 4 (b) x 4 (c) tile of one PSF plane per instruction.
// A wave keeps up to 6 x 6 such tiles (a 24 x 24 block of the PSF plane) in
// registers, reading 6 G and 6 X values from LDS per 36 instructions.
//
// Work-group (a, PSF block, split s): PSF plane a, one block of rows/columns
// of it, X plane z and a range of G rows (the split).  G and X tiles of
// 16 or 32 G rows x 128 columns (with the X halo of the block's rows) are
// staged in LDS; wave w takes a quarter of the rows of each tile.  At the end the 16 x
// blocks and the 4 waves are summed in fixed order and the split's partial
// PSF block is written; the splits are added in double precision afterwards.
constexpr int HQX = 128;             // X columns per staged tile
constexpr int HMT = 6;               // max 4-wide tiles per block along b and c
constexpr int HXS = HQX + 16;        // X tile row stride (= 16 mod 64: 4 rows x 16 lanes, no bank conflict)
constexpr int HGS = HQX + 4 * HMT + 4;                  // G tile row stride (>= 128 + 23 + 1)
constexpr int HTHREADS = 256;
__host__ __device__ constexpr int dh_tile_rows(int t) { return t >= 6 ? 32 : 16; }
static_assert(HTHREADS == 2 * HQX, "staging: two rows of 128 columns per pass");

struct DhmGeom {
  int mz, my, mx, kz, ky, kx, gy, gx;
  int tb, tc, nbb, nbc;   // tiles per block along b / c, blocks along b / c
  int nys, ysplit;        // G-row splits per X plane, G rows per split (multiple of the tile height)
  int nsplit;             // mz * nys
};

DhmGeom dhm_geom(const int64_t m3[3], const int64_t p3[3]) {
  int HQY;
  DhmGeom d;
  d.mz = (int)m3[0];
  d.my = (int)m3[1];
  d.mx = (int)m3[2];
  d.kz = (int)(2 * p3[0] + 1);
  d.ky = (int)(2 * p3[1] + 1);
  d.kx = (int)(2 * p3[2] + 1);
  d.gy = d.my + d.ky - 1;
  d.gx = d.mx + d.kx - 1;
  const int ntb = (d.ky + 3) / 4, ntc = (d.kx + 3) / 4;
  d.nbb = (ntb + HMT - 1) / HMT;
  d.nbc = (ntc + HMT - 1) / HMT;
  d.tb = (ntb + d.nbb - 1) / d.nbb;
  d.tc = (ntc + d.nbc - 1) / d.nbc;
  HQY = dh_tile_rows(d.tb > d.tc ? d.tb : d.tc);
  // G-row splits per X plane: the count whose work-groups fill whole rounds
  // of the resident slots (256 CUs x 2) best, costing each split's rounds
  // by its tiles plus a quarter tile of per-work-group overhead (X halo,
  // reduction); fewer splits on ties
  const int64_t base = (int64_t)d.kz * d.nbb * d.nbc * d.mz;
  const int ytiles = (d.gy + HQY - 1) / HQY;
  constexpr int64_t slots = 512;
  int per = ytiles;
  double best = -1.0;
  for (int n = 1; n <= ytiles && n <= 32; ++n) {
    const int pn = (ytiles + n - 1) / n;
    const int nys = (ytiles + pn - 1) / pn;
    const int64_t rounds = (base * nys + slots - 1) / slots;
    const double cost = (double)rounds * (pn + 0.25);
    if (best < 0.0 || cost < best * 0.999) {
      best = cost;
      per = pn;
    }
  }
  d.ysplit = per * HQY;
  d.nys = (d.gy + d.ysplit - 1) / d.ysplit;
  d.nsplit = d.mz * d.nys;
  return d;
}

typedef float dh_v4f __attribute__((ext_vector_type(4)));

template <int B, int E, typename F>
__device__ __forceinline__ void dh_sfor(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    dh_sfor<B + 1, E>(f);
  }
}

// T x T tiles per wave (T = the larger of the block's tile counts; tiles past
// the block are computed and dropped).
template <int T>
__global__ __launch_bounds__(HTHREADS, 2) void dh_mfma_kernel(const float *__restrict__ X, const float *__restrict__ G,
                                                              float *__restrict__ part, DhmGeom d) {
  constexpr int HQY = dh_tile_rows(T);             // G rows per staged tile (HQY / 4 per wave)
  constexpr int HXR = HQY + 4 * T - 1;             // X tile rows
  __shared__ __align__(16) float lds[HXR * HXS + HQY * HGS];
  __shared__ float red[4][4 * HMT * HMT][4];  // [wave][tile*4 + j][i]
  float *xt = lds;                 // HXR x HXS
  float *gt = lds + HXR * HXS;     // HQY x HGS
  int id = blockIdx.x;
  const int a = id % d.kz;
  id /= d.kz;
  const int bc = id % d.nbc;
  id /= d.nbc;
  const int bb = id % d.nbb;
  const int split = id / d.nbb;
  const int z = split / d.nys, ys = split - z * d.nys;
  const int b0 = bb * 4 * d.tb, c0 = bc * 4 * d.tc;
  constexpr int xrows = HQY + 4 * T - 1;                // X rows staged per tile
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int k = lane >> 2, q4 = lane & 3;               // block (x offset), i or j
  const int cx = tid & (HQX - 1), rp = tid / HQX;       // staging column and row parity
  const float *Xp = X + (int64_t)z * d.my * d.mx;
  const float *Gp = G + (int64_t)(z + a) * d.gy * d.gx;

  dh_v4f acc[T][T];
#pragma unroll
  for (int u = 0; u < T; ++u)
#pragma unroll
    for (int v = 0; v < T; ++v) acc[u][v] = (dh_v4f){0.f, 0.f, 0.f, 0.f};

  const int y_lo = ys * d.ysplit, y_hi = min(d.gy, y_lo + d.ysplit);
  for (int yt = y_lo; yt < y_hi; yt += HQY) {
    for (int xt0 = 0; xt0 < d.mx; xt0 += HQX) {
      // Staging: every load of the tile is issued first, unconditionally, at
      // offsets clamped into the plane, and the LDS writes zero what lies
      // outside; the loads are then in flight together instead of one
      // memory latency each.  Thread columns: cx (and cx + 128 .. for G's
      // last HGS - 128 columns), rows of the same parity rp.
      constexpr int NXU = (xrows + 1) / 2;                          // X rows per thread
      constexpr int NGU = HQY / 2;                                  // G rows per thread, first 128 columns
      constexpr int GEX = HGS - HQX;                                // G columns past 128
      constexpr int NGE = (HQY * GEX + HTHREADS - 1) / HTHREADS;    // those per thread
      // X rows yt - b0 - 4T + 1 .. yt + HQY - 1 - b0, columns xt0 .. xt0 + 127
      const int xr0 = yt - b0 - 4 * T + 1;
      const int xx = xt0 + cx, xxc = min(xx, d.mx - 1);
      const int xg = xt0 + c0 + cx, xgc = min(xg, d.gx - 1);
      float xv[NXU], gv[NGU], ge[NGE];
#pragma unroll
      for (int u = 0; u < NXU; ++u) {
        const int yc = min(max(xr0 + 2 * u + rp, 0), d.my - 1);
        xv[u] = Xp[(unsigned)(yc * d.mx + xxc)];
      }
#pragma unroll
      for (int u = 0; u < NGU; ++u) {
        const int yc = min(yt + 2 * u + rp, d.gy - 1);
        gv[u] = Gp[(unsigned)(yc * d.gx + xgc)];
      }
#pragma unroll
      for (int v = 0; v < NGE; ++v) {
        const int e = tid + HTHREADS * v, r = min(e / GEX, HQY - 1), c = HQX + e % GEX;
        const int yc = min(yt + r, d.gy - 1), xc = min(xt0 + c0 + c, d.gx - 1);
        ge[v] = Gp[(unsigned)(yc * d.gx + xc)];
      }
      __syncthreads();  // previous tile no longer read
#pragma unroll
      for (int u = 0; u < NXU; ++u) {
        const int r = 2 * u + rp, yx = xr0 + r;
        if (r < xrows) xt[r * HXS + cx] = (yx >= 0 && yx < d.my && xx < d.mx) ? xv[u] : 0.f;
      }
#pragma unroll
      for (int u = 0; u < NGU; ++u) {
        const int r = 2 * u + rp;
        gt[r * HGS + cx] = (yt + r < y_hi && xg < d.gx) ? gv[u] : 0.f;
      }
#pragma unroll
      for (int v = 0; v < NGE; ++v) {
        const int e = tid + HTHREADS * v, r = e / GEX, c = HQX + e % GEX;
        if (r < HQY) gt[r * HGS + c] = (yt + r < y_hi && xt0 + c0 + c < d.gx) ? ge[v] : 0.f;
      }
      __syncthreads();
      const int nch = min(HQX, d.mx - xt0 + 15) / 16;  // 16-wide chunks with any X column
#pragma unroll 1
      for (int r = 0; r < HQY / 4; ++r) {
        const int row = (HQY / 4) * w + r;  // G row inside the tile
        if (yt + row >= y_hi) break;
#pragma unroll 1
        for (int ch = 0; ch < nch; ++ch) {
          float av[T], bv[T];
#pragma unroll
          for (int v = 0; v < T; ++v) av[v] = gt[row * HGS + 16 * ch + k + 4 * v + q4];
#pragma unroll
          for (int u = 0; u < T; ++u)  // X row for b = b0 + 4u + j: tile row row + 4T - 1 - 4u - j (>= 0)
            bv[u] = xt[(row + 4 * T - 1 - 4 * u - q4) * HXS + 16 * ch + k];
          dh_sfor<0, T>([&](auto uc) {
            constexpr int u = decltype(uc)::value;
            dh_sfor<0, T>([&](auto vc) {
              constexpr int v = decltype(vc)::value;
              acc[u][v] = __builtin_amdgcn_mfma_f32_4x4x1f32(av[v], bv[u], acc[u][v], 0, 0, 0);
            });
          });
        }
      }
    }
  }

  // sum the 16 x blocks (lanes 4k + j, k = 0..15) in fixed order
#pragma unroll
  for (int u = 0; u < T; ++u) {
#pragma unroll
    for (int v = 0; v < T; ++v)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float t = acc[u][v][i];
        t += __shfl_xor(t, 4);
        t += __shfl_xor(t, 8);
        t += __shfl_xor(t, 16);
        t += __shfl_xor(t, 32);
        acc[u][v][i] = t;
      }
    __builtin_amdgcn_sched_barrier(0);  // one tile row at a time: bounded temporaries
  }
  if (lane < 4) {
#pragma unroll
    for (int u = 0; u < T; ++u)
#pragma unroll
      for (int v = 0; v < T; ++v)
#pragma unroll
        for (int i = 0; i < 4; ++i) red[w][(u * T + v) * 4 + lane][i] = acc[u][v][i];
  }
  __syncthreads();
  // the 4 waves in fixed order; entry (u, v, j, i) is dH[a, b0+4u+j, c0+4v+i]
  for (int e = tid; e < T * T * 16; e += HTHREADS) {
    const int i = e & 3, j = (e >> 2) & 3, uv = e >> 4, u = uv / T, v = uv - u * T;
    const int b = b0 + 4 * u + j, c = c0 + 4 * v + i;
    if (b < d.ky && c < d.kx && b < b0 + 4 * d.tb && c < c0 + 4 * d.tc) {
      const float sum = ((red[0][uv * 4 + j][i] + red[1][uv * 4 + j][i]) + red[2][uv * 4 + j][i]) + red[3][uv * 4 + j][i];
      part[(int64_t)split * d.kz * d.ky * d.kx + ((int64_t)a * d.ky + b) * d.kx + c] = sum;
    }
  }
}

}  // namespace

bool dh_supported(const int64_t m3[3], const int64_t p3[3], int dtype) {
  if (dtype == NDC_F32)  // matrix-core form: any PSF (blocks of 24 x 24); 32-bit offsets inside a plane
    return m3[1] * m3[2] < ((int64_t)1 << 31) && (m3[1] + 2 * p3[1]) * (m3[2] + 2 * p3[2]) < ((int64_t)1 << 31);
  const DhGeom d = dh_geom(m3, p3);
  return d.ky * d.ncg <= 256 && dh_lds_bytes(d, 8) <= 96 * 1024;
}

size_t dh_workspace_bytes(const int64_t m3[3], const int64_t p3[3], int dtype) {
  if (dtype == NDC_F32) {
    const DhmGeom d = dhm_geom(m3, p3);
    return (size_t)d.nsplit * d.kz * d.ky * d.kx * sizeof(float);
  }
  const DhGeom d = dh_geom(m3, p3);
  return (size_t)d.nsplit * d.kz * d.ky * d.kx * sizeof(double);
}

hipError_t launch_dh(const int64_t m3[3], const int64_t p3[3], int dtype, const void *X, const void *G, void *dH,
                     void *ws, hipStream_t s) {
  if (dtype == NDC_F32) {
    const DhmGeom d = dhm_geom(m3, p3);
    const int64_t blocks = (int64_t)d.kz * d.nbb * d.nbc * d.nsplit;
    const dim3 grid((unsigned)blocks), block(HTHREADS);
    switch (max(d.tb, d.tc)) {
#define NDC_DHM(T)                                                                                            \
  case T:                                                                                                      \
    hipLaunchKernelGGL(dh_mfma_kernel<T>, grid, block, 0, s, (const float *)X, (const float *)G, (float *)ws, d); \
    break;
      NDC_DHM(1) NDC_DHM(2) NDC_DHM(3) NDC_DHM(4) NDC_DHM(5) NDC_DHM(6)
#undef NDC_DHM
      default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_splitk_reduce(dtype, ws, dH, (int64_t)d.kz * d.ky * d.kx, d.nsplit, s);
  }
  const DhGeom d = dh_geom(m3, p3);
  const size_t es = dtype == NDC_F64 ? 8 : 4;
  const int threads = ((d.ky * d.ncg + 63) / 64) * 64;
  const dim3 grid((unsigned)(d.kz * d.nsplit));
  const size_t lds = dh_lds_bytes(d, es);
  // raise the dynamic-LDS limit once per process; call_once makes
  // concurrent first calls from several host threads safe
  static std::once_flag lds_once;
  std::call_once(lds_once, [] {
    (void)hipFuncSetAttribute((const void *)dh_kernel<double>, hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    (void)hipFuncSetAttribute((const void *)dh_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize, 96 * 1024);
    (void)hipGetLastError();
  });
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
