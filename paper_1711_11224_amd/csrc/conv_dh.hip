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

#include <algorithm>
#include <cstdint>
#include <mutex>
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
template <int T, bool XV>
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
      // XV: 16-byte X loads (X's rows a multiple of 4 floats, X aligned):
      // thread columns c4, c4 + 1 .. c4 + 3, rows of the same residue mod 8
      constexpr int NX4 = (xrows + 7) / 8;
      const int c4 = (tid & 31) * 4, r8 = tid >> 5;
      const int x4 = xt0 + c4, x4c = min(x4, d.mx - 4);
      float xv[XV ? 1 : NXU], gv[NGU], ge[NGE];
      float4 xv4[XV ? NX4 : 1];
      if constexpr (XV) {
#pragma unroll
        for (int u = 0; u < NX4; ++u) {
          const int yc = min(max(xr0 + 8 * u + r8, 0), d.my - 1);
          xv4[u] = *(const float4 *)(Xp + (unsigned)(yc * d.mx + x4c));
        }
      } else {
#pragma unroll
        for (int u = 0; u < NXU; ++u) {
          const int yc = min(max(xr0 + 2 * u + rp, 0), d.my - 1);
          xv[u] = Xp[(unsigned)(yc * d.mx + xxc)];
        }
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
      if constexpr (XV) {
#pragma unroll
        for (int u = 0; u < NX4; ++u) {
          const int r = 8 * u + r8, yx = xr0 + r;
          if (r < xrows)
            *(float4 *)(xt + r * HXS + c4) = (yx >= 0 && yx < d.my && x4 < d.mx) ? xv4[u] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
      } else {
#pragma unroll
        for (int u = 0; u < NXU; ++u) {
          const int r = 2 * u + rp, yx = xr0 + r;
          if (r < xrows) xt[r * HXS + cx] = (yx >= 0 && yx < d.my && xx < d.mx) ? xv[u] : 0.f;
        }
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

// ---------------------------------------------------------------------------
// FP32 matrix-core form with a broadcast G operand (where whole PSF planes of
// rows fill the instruction's 64 lanes).
//
// v_mfma_f32_4x4x1f32 with CBSZ = 4, ABID = m: every block takes its A
// operand from block m, so the 16 blocks share one G segment and each lane
// brings its own X value.  For G plane zg, G row yg and the x position
// x = xc + m of a 16-wide chunk:
//   A[i] = G[zg, yg, x + c0 + 4t + i]    (lane 4m + i of the A register of c tile t)
//   B[r] = X[zg - a_r, yg - b_r, x]      (lane r = 4k + j: one (a, b) pair per lane)
// so register i of lane r of tile t gathers dH[a_r, b_r, c0 + 4t + i].  The
// 16 instructions of a chunk accumulate into the same registers (a dependent
// chain, which the matrix unit issues back to back) and no lanes are summed
// afterwards.  Lane r < na * ky takes PSF plane a0 + r / ky and row r % ky:
// na whole planes per group, whose X planes zg - a are staged in LDS.
//
// Work-group (G plane zg, group g of zg's PSF planes, c block, G-row split
// ys): zg pairs with the planes a in [max(0, zg - mz + 1), min(kz - 1, zg)]
// (X plane zx = zg - a inside X); group g takes na of them.  Its sums over
// the split's G rows go to slot zx * nys + ys of the split sum, so every
// (zx, a) pair of the contraction lands in exactly one slot.
constexpr int BQX = 128;              // X columns per staged tile
constexpr int BXS = BQX + 1;          // X tile row stride (= 1 mod 64, see the plane stride)
constexpr int BTC = 8;                // c tiles (32 taps) per work-group
constexpr int BGS = BQX + 4 * BTC;    // G tile row stride (>= 16 * 7 + 15 + 4 * 7 + 3 + 1)
constexpr int BLDS_MAX = 80 * 1024;   // two work-groups per CU
constexpr int BBATCH = 32;            // staging loads in flight per thread

struct DhbGeom {
  int mz, my, mx, kz, ky, kx, gy, gx;
  int na;              // PSF planes per group (na * ky <= 64 lanes)
  int ngmax;           // groups per G plane, at most
  int tc, ncb;         // c tiles per work-group, c blocks
  int hqy, pr, ps;     // G rows per tile; X rows per plane (hqy + ky - 1); X plane stride in LDS
  int nys, ysplit;     // G-row splits, G rows per split
  int lds;             // dynamic LDS bytes
};

// X plane stride: = ky mod 64 floats, so with a row stride = 1 mod 64 the 64
// lanes' B operands (plane p, row base - b, the same column) sit at
// p * ky - b + const mod 64: distinct banks for the na * ky <= 64 pairs.
int dhb_plane_stride(int pr, int ky) { return pr * BXS + (((ky - pr * BXS) % 64) + 64) % 64; }

int dhb_lds_bytes(int hqy, int na, int ky, int tc) {
  const int pr = hqy + ky - 1;
  const int floats = hqy * BGS + BXS + na * dhb_plane_stride(pr, ky);
  return 4 * std::max(floats, 4 * tc * 4 * 64);  // the cross-wave sum reuses the area
}

// Geometry of the broadcast form; na = 0 where it does not apply (PSF rows
// wider than 64, too few lanes filled, or no tile height fits the LDS budget).
DhbGeom dhb_geom(const int64_t m3[3], const int64_t p3[3]) {
  DhbGeom d{};
  d.mz = (int)m3[0];
  d.my = (int)m3[1];
  d.mx = (int)m3[2];
  d.kz = (int)(2 * p3[0] + 1);
  d.ky = (int)(2 * p3[1] + 1);
  d.kx = (int)(2 * p3[2] + 1);
  d.gy = d.my + d.ky - 1;
  d.gx = d.mx + d.kx - 1;
  d.na = 0;
  if (d.ky > 64) return d;
  const int na = 64 / d.ky;
  const int fill = std::min(na, std::min(d.kz, d.mz)) * d.ky;  // lanes used by a full group
  if (fill < 40) return d;
  d.tc = std::min(BTC, (d.kx + 3) / 4);
  d.ncb = (d.kx + 4 * d.tc - 1) / (4 * d.tc);
  // Taken where it issues at least 10% fewer products per PSF plane than
  // the 4 x 4 tile form (whose T x T tiles pad both PSF axes to multiples of
  // 4) and the PSF rows are 17 taps or wider: measured on MI355X, it is
  // 1.06-1.31x faster there (41 x 21 x 21, 31 x 21 x 21, 31 x 25 x 25) and
  // level or slower elsewhere (9-tap rows, 15 x 15 and 31 x 31 planes).
  {
    const DhmGeom m = dhm_geom(m3, p3);
    const int t = std::max(m.tb, m.tc);
    const double tile_area = (double)m.nbb * m.nbc * 16.0 * t * t;
    const double bcast_area = 64.0 / na * 4.0 * d.tc * d.ncb;
    if (d.kx < 17 || tile_area < 1.1 * bcast_area) return d;
  }
  for (int hqy = 32; hqy >= 8; hqy /= 2) {
    if (dhb_lds_bytes(hqy, na, d.ky, d.tc) <= BLDS_MAX) {
      d.hqy = hqy;
      break;
    }
  }
  if (!d.hqy) return d;
  d.na = na;
  d.pr = d.hqy + d.ky - 1;
  d.ps = dhb_plane_stride(d.pr, d.ky);
  d.lds = dhb_lds_bytes(d.hqy, na, d.ky, d.tc);
  d.ngmax = (std::min(d.kz, d.mz) + na - 1) / na;
  // work-groups with planes, per split
  const int gz = d.mz + d.kz - 1;
  int64_t busy = 0;
  for (int zg = 0; zg < gz; ++zg) {
    const int l = std::min(d.kz - 1, zg) - std::max(0, zg - d.mz + 1) + 1;
    busy += (l + na - 1) / na;
  }
  busy *= d.ncb;
  // splits of the G rows: whole rounds of the resident slots (256 CUs x 2),
  // each split's rounds costed by its tiles plus a quarter tile
  const int ytiles = (d.gy + d.hqy - 1) / d.hqy;
  constexpr int64_t slots = 512;
  int per = ytiles;
  double best = -1.0;
  for (int n = 1; n <= ytiles && n <= 32; ++n) {
    const int pn = (ytiles + n - 1) / n;
    const int nys = (ytiles + pn - 1) / pn;
    const int64_t rounds = (busy * nys + slots - 1) / slots;
    const double cost = (double)rounds * (pn + 0.25);
    if (best < 0.0 || cost < best * 0.999) {
      best = cost;
      per = pn;
    }
  }
  d.ysplit = per * d.hqy;
  d.nys = (d.gy + d.ysplit - 1) / d.ysplit;
  return d;
}

template <int TC, int HQY>
__global__ __launch_bounds__(HTHREADS, 2) void dh_bcast_kernel(const float *__restrict__ X, const float *__restrict__ G,
                                                               float *__restrict__ part, DhbGeom d) {
  extern __shared__ __align__(16) float bl[];
  float *gt = bl;                  // HQY x BGS
  float *zr = gt + HQY * BGS;      // one row of zeros (BXS)
  float *xt = zr + BXS;            // na planes x ps
  int id = blockIdx.x;
  const int g = id % d.ngmax;
  id /= d.ngmax;
  const int cb = id % d.ncb;
  id /= d.ncb;
  const int ys = id % d.nys;
  const int zg = id / d.nys;
  const int alo = max(0, zg - d.mz + 1), ahi = min(d.kz - 1, zg);
  const int a0 = alo + g * d.na;
  if (a0 > ahi) return;  // no PSF plane in this group (uniform)
  const int nag = min(d.na, ahi - a0 + 1);
  const int c0 = cb * 4 * TC;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t K = (int64_t)d.kz * d.ky * d.kx;

  // this lane's (a, b) pair; lanes past the group read the zero row
  const int lp = lane / d.ky, lb = lane - lp * d.ky;
  const bool lv = lp < nag;
  const int xlane = lv ? (int)(xt - bl) + lp * d.ps + (d.ky - 1 - lb) * BXS : (int)(zr - bl);
  const int xstep = lv ? BXS : 0;  // per G row
  const int glane = (lane >> 2) + (lane & 3);  // A operand: column m + i

  for (int e = tid; e < BXS; e += HTHREADS) zr[e] = 0.f;

  dh_v4f acc[TC];
#pragma unroll
  for (int t = 0; t < TC; ++t) acc[t] = (dh_v4f){0.f, 0.f, 0.f, 0.f};

  const int y_lo = ys * d.ysplit, y_hi = min(d.gy, y_lo + d.ysplit);
  const float *Gp = G + (int64_t)zg * d.gy * d.gx;
  const int cx = tid & (BQX - 1), rp = tid / BQX;  // staging column and row parity
  const int nxr = nag * d.pr;                      // X rows staged per tile (all planes)
  const bool x_vec = (d.mx & 3) == 0 && ((uintptr_t)X & 15) == 0;  // 16-byte X loads
  const bool g_vec = (d.gx & 3) == 0 && ((uintptr_t)G & 15) == 0;  // 16-byte G loads
  for (int yt = y_lo; yt < y_hi; yt += HQY) {
    for (int xt0 = 0; xt0 < d.mx; xt0 += BQX) {
      __syncthreads();  // previous tile no longer read
      // G rows yt .. yt + HQY - 1, columns xt0 + c0 + [0, BGS): loads first
      // (unconditional, at clamped offsets), then the LDS writes with what
      // lies outside G zeroed; 16-byte loads where G's rows allow them
      if (g_vec) {
        constexpr int G4 = BGS / 4, NG4 = (HQY * G4 + HTHREADS - 1) / HTHREADS;
        float4 gv4[NG4];
#pragma unroll
        for (int v = 0; v < NG4; ++v) {
          const int e = tid + HTHREADS * v, r = min(e / G4, HQY - 1), c = (e % G4) * 4;
          gv4[v] = *(const float4 *)(Gp + (unsigned)(min(yt + r, d.gy - 1) * d.gx + min(xt0 + c0 + c, d.gx - 4)));
        }
#pragma unroll
        for (int v = 0; v < NG4; ++v) {
          const int e = tid + HTHREADS * v, r = e / G4, c = (e % G4) * 4;
          if (e < HQY * G4) {
            const bool ok = yt + r < y_hi && xt0 + c0 + c < d.gx;
            *(float4 *)(gt + r * BGS + c) = ok ? gv4[v] : make_float4(0.f, 0.f, 0.f, 0.f);
          }
        }
      } else {
        constexpr int NGU = HQY / 2, NGE = HQY * (BGS - BQX) / HTHREADS;
        float gv[NGU], ge[NGE];
        const int xg = xt0 + c0 + cx, xgc = min(xg, d.gx - 1);
#pragma unroll
        for (int u = 0; u < NGU; ++u) gv[u] = Gp[(unsigned)(min(yt + 2 * u + rp, d.gy - 1) * d.gx + xgc)];
#pragma unroll
        for (int v = 0; v < NGE; ++v) {
          const int e = tid + HTHREADS * v, r = e / (BGS - BQX), c = BQX + e % (BGS - BQX);
          ge[v] = Gp[(unsigned)(min(yt + r, d.gy - 1) * d.gx + min(xt0 + c0 + c, d.gx - 1))];
        }
#pragma unroll
        for (int u = 0; u < NGU; ++u) {
          const int r = 2 * u + rp;
          gt[r * BGS + cx] = (yt + r < y_hi && xg < d.gx) ? gv[u] : 0.f;
        }
#pragma unroll
        for (int v = 0; v < NGE; ++v) {
          const int e = tid + HTHREADS * v, r = e / (BGS - BQX), c = BQX + e % (BGS - BQX);
          gt[r * BGS + c] = (yt + r < y_hi && xt0 + c0 + c < d.gx) ? ge[v] : 0.f;
        }
      }
      // X planes zg - a0 - p (p < nag), rows yt - ky + 1 .. yt + HQY - 1,
      // columns xt0 .. xt0 + 127, in batches of loads in flight together:
      // 16-byte loads where X's rows allow them
      if (x_vec) {
        constexpr int B4 = 16;
        const int c4 = (tid & 31) * 4, rs = tid >> 5;
        const int xx = xt0 + c4, xxc = min(xx, d.mx - 4);
        const bool xok = xx < d.mx;
        int p = 0, rr = rs;
        for (int u0 = rs; u0 < nxr; u0 += 8 * B4) {
          float4 xv[B4];
          int pp = p, r2 = rr;
#pragma unroll
          for (int q = 0; q < B4; ++q) {
            const int zc = zg - a0 - min(pp, nag - 1);
            const int yc = min(max(yt - d.ky + 1 + r2, 0), d.my - 1);
            xv[q] = *(const float4 *)(X + (int64_t)zc * d.my * d.mx + (unsigned)(yc * d.mx + xxc));
            r2 += 8;
            if (r2 >= d.pr) {
              r2 -= d.pr;
              ++pp;
            }
          }
#pragma unroll
          for (int q = 0; q < B4; ++q) {
            const int y = yt - d.ky + 1 + rr;
            if (p < nag) {
              const bool ok = y >= 0 && y < d.my && xok;
              float *dst = xt + p * d.ps + rr * BXS + c4;
              dst[0] = ok ? xv[q].x : 0.f;
              dst[1] = ok ? xv[q].y : 0.f;
              dst[2] = ok ? xv[q].z : 0.f;
              dst[3] = ok ? xv[q].w : 0.f;
            }
            rr += 8;
            if (rr >= d.pr) {
              rr -= d.pr;
              ++p;
            }
          }
        }
      } else {
        const int xx = xt0 + cx, xxc = min(xx, d.mx - 1);
        int p = 0, rr = rp;  // plane and row of this thread's next X row
        for (int u0 = rp; u0 < nxr; u0 += 2 * BBATCH) {
          float xv[BBATCH];
          int pp = p, r2 = rr;
#pragma unroll
          for (int q = 0; q < BBATCH; ++q) {
            const int zc = zg - a0 - min(pp, nag - 1);
            const int yc = min(max(yt - d.ky + 1 + r2, 0), d.my - 1);
            xv[q] = X[(int64_t)zc * d.my * d.mx + (unsigned)(yc * d.mx + xxc)];
            r2 += 2;
            if (r2 >= d.pr) {
              r2 -= d.pr;
              ++pp;
            }
          }
#pragma unroll
          for (int q = 0; q < BBATCH; ++q) {
            const int y = yt - d.ky + 1 + rr;
            if (p < nag) xt[p * d.ps + rr * BXS + cx] = (y >= 0 && y < d.my && xx < d.mx) ? xv[q] : 0.f;
            rr += 2;
            if (rr >= d.pr) {
              rr -= d.pr;
              ++p;
            }
          }
        }
      }
      __syncthreads();
      // 16-wide chunks with any X column, rounded up to pairs: a chunk past
      // the last lies in the tile and its X columns, past the volume, are
      // staged as zeros, so its products add nothing
      const int nch = min(BQX, d.mx - xt0 + 15) / 16;
      const int nch2 = min(BQX / 16, (nch + 1) & ~1);
#pragma unroll 1
      for (int r = 0; r < HQY / 4; ++r) {
        const int row = (HQY / 4) * w + r;  // G row inside the tile
        if (yt + row >= y_hi) break;
        const float *gl = gt + row * BGS + glane;
        const float *xl = bl + xlane + row * xstep;
        auto rd = [&](float(&av)[TC], float(&bv)[16], int ch) __attribute__((always_inline)) {
#pragma unroll
          for (int t = 0; t < TC; ++t) av[t] = gl[16 * ch + 4 * t];
#pragma unroll
          for (int m = 0; m < 16; ++m) bv[m] = xl[16 * ch + m];
        };
        auto mm = [&](const float(&av)[TC], const float(&bv)[16]) __attribute__((always_inline)) {
          // x positions outer, c tiles inner: consecutive instructions
          // write different accumulators
          dh_sfor<0, 16>([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            dh_sfor<0, TC>([&](auto tc_) {
              constexpr int t = decltype(tc_)::value;
              acc[t] = __builtin_amdgcn_mfma_f32_4x4x1f32(av[t], bv[m], acc[t], 4, m, 0);
            });
          });
        };
        // two operand sets: the next chunk's are read while this chunk's
        // instructions run (after the last pair the last chunk is read again)
        float a0v[TC], b0v[16], a1v[TC], b1v[16];
        rd(a0v, b0v, 0);
#pragma unroll 1
        for (int ch = 0; ch < nch2; ch += 2) {
          rd(a1v, b1v, ch + 1);
          mm(a0v, b0v);
          rd(a0v, b0v, min(ch + 2, nch2 - 1));
          mm(a1v, b1v);
          // order: each set's reads (ds_read2: TC / 2 + 8) spread over the
          // first instructions of the other set's chunk
          constexpr int NR = (TC + 1) / 2 + 8;
          dh_sfor<0, 2>([&](auto) {
            dh_sfor<0, NR>([&](auto) {
              __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
              __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
            });
            __builtin_amdgcn_sched_group_barrier(0x008, 16 * TC - 4 * NR, 0);
          });
        }
      }
    }
  }

  // the 4 waves' sums in fixed order (the LDS tiles are reused)
  __syncthreads();
  float *red = bl;  // [w][t][i][lane]
#pragma unroll
  for (int t = 0; t < TC; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) red[((w * TC + t) * 4 + i) * 64 + lane] = acc[t][i];
  __syncthreads();
  for (int e = tid; e < TC * 4 * 64; e += HTHREADS) {
    const int l = e & 63, ti = e >> 6, i = ti & 3, t = ti >> 2;
    const int p = l / d.ky, b = l - p * d.ky, c = c0 + 4 * t + i;
    if (p < nag && c < d.kx) {
      const int a = a0 + p, zx = zg - a;
      const float sum = ((red[(0 * TC * 4 + ti) * 64 + l] + red[(1 * TC * 4 + ti) * 64 + l]) +
                         red[(2 * TC * 4 + ti) * 64 + l]) + red[(3 * TC * 4 + ti) * 64 + l];
      part[((int64_t)zx * d.nys + ys) * K + ((int64_t)a * d.ky + b) * d.kx + c] = sum;
    }
  }
}

template <int TC, int HQY>
hipError_t launch_dhb_t(const DhbGeom &d, const float *X, const float *G, float *ws, hipStream_t s) {
  static std::once_flag once;  // dynamic LDS above 64 KiB, once per instantiation
  std::call_once(once, [] {
    (void)hipFuncSetAttribute((const void *)dh_bcast_kernel<TC, HQY>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              BLDS_MAX);
    (void)hipGetLastError();
  });
  const int64_t blocks = (int64_t)(d.mz + d.kz - 1) * d.nys * d.ncb * d.ngmax;
  hipLaunchKernelGGL((dh_bcast_kernel<TC, HQY>), dim3((unsigned)blocks), dim3(HTHREADS), d.lds, s, X, G, ws, d);
  return hipGetLastError();
}

template <int TC>
hipError_t launch_dhb_tc(const DhbGeom &d, const float *X, const float *G, float *ws, hipStream_t s) {
  switch (d.hqy) {
    case 32: return launch_dhb_t<TC, 32>(d, X, G, ws, s);
    case 16: return launch_dhb_t<TC, 16>(d, X, G, ws, s);
    case 8: return launch_dhb_t<TC, 8>(d, X, G, ws, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_dhb(const DhbGeom &d, const float *X, const float *G, float *ws, hipStream_t s) {
  switch (d.tc) {
    case 1: return launch_dhb_tc<1>(d, X, G, ws, s);
    case 2: return launch_dhb_tc<2>(d, X, G, ws, s);
    case 3: return launch_dhb_tc<3>(d, X, G, ws, s);
    case 4: return launch_dhb_tc<4>(d, X, G, ws, s);
    case 5: return launch_dhb_tc<5>(d, X, G, ws, s);
    case 6: return launch_dhb_tc<6>(d, X, G, ws, s);
    case 7: return launch_dhb_tc<7>(d, X, G, ws, s);
    case 8: return launch_dhb_tc<8>(d, X, G, ws, s);
    default: return hipErrorInvalidValue;
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
    const DhbGeom b = dhb_geom(m3, p3);
    if (b.na) return (size_t)b.mz * b.nys * b.kz * b.ky * b.kx * sizeof(float);
    const DhmGeom d = dhm_geom(m3, p3);
    return (size_t)d.nsplit * d.kz * d.ky * d.kx * sizeof(float);
  }
  const DhGeom d = dh_geom(m3, p3);
  return (size_t)d.nsplit * d.kz * d.ky * d.kx * sizeof(double);
}

hipError_t launch_dh(const int64_t m3[3], const int64_t p3[3], int dtype, const void *X, const void *G, void *dH,
                     void *ws, hipStream_t s) {
  if (dtype == NDC_F32) {
    const DhbGeom b = dhb_geom(m3, p3);
    if (b.na) {
      const hipError_t e = launch_dhb(b, (const float *)X, (const float *)G, (float *)ws, s);
      if (e != hipSuccess) return e;
      return launch_splitk_reduce(dtype, ws, dH, (int64_t)b.kz * b.ky * b.kx, b.mz * b.nys, s);
    }
    const DhmGeom d = dhm_geom(m3, p3);
    const int64_t blocks = (int64_t)d.kz * d.nbb * d.nbc * d.nsplit;
    const dim3 grid((unsigned)blocks), block(HTHREADS);
    const bool xv = (d.mx & 3) == 0 && ((uintptr_t)X & 15) == 0;  // 16-byte X staging
    switch (max(d.tb, d.tc)) {
#define NDC_DHM(T)                                                                                            \
  case T:                                                                                                      \
    if (xv)                                                                                                    \
      hipLaunchKernelGGL((dh_mfma_kernel<T, true>), grid, block, 0, s, (const float *)X, (const float *)G,     \
                         (float *)ws, d);                                                                      \
    else                                                                                                       \
      hipLaunchKernelGGL((dh_mfma_kernel<T, false>), grid, block, 0, s, (const float *)X, (const float *)G,    \
                         (float *)ws, d);                                                                      \
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
