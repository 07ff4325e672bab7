// Direct correlation kernel on the vector ALUs: the general path for every
// shape, dtype and precision (small PSFs, FP64, and half-widths the MFMA
// kernel does not cover).
//
// out[s] = sum_t Hc[t] in[s + t - off] over a zero-extended input (see Geom).
// A work-group owns a 16 x 64 output tile of one output z-plane.  For each
// z-tap it stages a (16+15) x 96 window of the input plane and a 16 x 32
// block of taps in LDS, then every thread accumulates 4 consecutive x
// outputs with a 4-tap sliding window.  Tap ranges are clipped per tile so
// the zero padding of the forward operator costs no multiply-adds outside
// the tile edges.  Sums are blocked: per tap row (<= 32 taps), per z-plane,
// then across z-planes, which keeps FP32 rounding near 1e-6 relative even
// for 60k-tap PSFs.
#include "ndc_internal.h"
#include "ndc_device.h"

namespace ndc {
namespace {

constexpr int VT = 256;
constexpr int TXT = 16;
constexpr int RX = 4;
constexpr int TX = TXT * RX;  // 64 outputs along x
constexpr int TY = VT / TXT;  // 16 rows
constexpr int BC = 16;        // y-taps per staged chunk
constexpr int CC = 32;        // x-taps per staged chunk (multiple of 4)
constexpr int TROWS = TY + BC - 1;
constexpr int TSTRIDE = TX + CC;  // >= TX + CC - 1, multiple of 4

template <typename T, int PREC>
struct Acc { using type = float; };
template <>
struct Acc<double, PREC_NATIVE_> { using type = double; };
template <>
struct Acc<float, PREC_NATIVE_> { using type = float; };

// Operand planes held in LDS: one for native and bf16 (values already
// rounded), two (hi, lo) for split-bf16.
template <int PREC>
struct NPlanes { static constexpr int v = 1; };
template <>
struct NPlanes<PREC_SPLIT_> { static constexpr int v = 2; };

template <typename A, int PREC>
__device__ inline void put_operand(A *base, int plane_stride, int e, double v) {
  if constexpr (PREC == PREC_NATIVE_) {
    base[e] = (A)v;
  } else if constexpr (PREC == PREC_BF16_) {
    base[e] = bf16_round((float)v);
  } else {
    float f = (float)v;
    float hi = bf16_round(f);
    base[e] = hi;
    base[plane_stride + e] = bf16_round(f - hi);
  }
}

// acc += h * x for one tap, in the precision's arithmetic.
template <typename A, int PREC>
__device__ inline A mac(A acc, A hh, A hl, A xh, A xl) {
  if constexpr (PREC == PREC_SPLIT_) {
    acc = fmaf(hh, xh, acc);
    acc = fmaf(hh, xl, acc);
    return fmaf(hl, xh, acc);
  } else {
    (void)hl;
    (void)xl;
    return acc + hh * xh;
  }
}

template <typename T, int PREC>
__global__ __launch_bounds__(VT) void conv_valu_kernel(const T *__restrict__ in, const T *__restrict__ H,
                                                       T *__restrict__ out, Geom g, Epi ep, int ksplit,
                                                       int zchunk) {
  using A = typename Acc<T, PREC>::type;
  constexpr int NP = NPlanes<PREC>::v;
  if (ep.phase && !((1 << *ep.phase) & ep.phase_mask)) return;  // uniform early exit

  __shared__ A tile[NP * TROWS * TSTRIDE];
  __shared__ A hch[NP * BC * CC];
  __shared__ double red[VT / 64][2];

  const int tid = threadIdx.x, tx = tid % TXT, ty = tid / TXT;
  const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
  const int z = blockIdx.z / ksplit, sidx = blockIdx.z % ksplit;

  // Clip tap ranges to those that reach the input for some output of the tile.
  int a_lo = max(0, g.offz - z), a_hi = min(g.kz - 1, g.iz - 1 + g.offz - z);
  a_lo = max(a_lo, sidx * zchunk);
  a_hi = min(a_hi, sidx * zchunk + zchunk - 1);
  const int b_lo = max(0, g.offy - y0 - (TY - 1)), b_hi = min(g.ky - 1, g.iy - 1 + g.offy - y0);
  const int c_lo = max(0, g.offx - x0 - (TX - 1)), c_hi = min(g.kx - 1, g.ix - 1 + g.offx - x0);

  A outer[RX];
#pragma unroll
  for (int r = 0; r < RX; ++r) outer[r] = 0;

  for (int a = a_lo; a <= a_hi; ++a) {
    const int zin = z + a - g.offz;
    const int ha = g.flip ? g.kz - 1 - a : a;
    A mid[RX];
#pragma unroll
    for (int r = 0; r < RX; ++r) mid[r] = 0;
    for (int b0 = b_lo; b0 <= b_hi; b0 += BC) {
      const int nb = min(BC, b_hi - b0 + 1);
      for (int c0 = c_lo; c0 <= c_hi; c0 += CC) {
        const int nc = min(CC, c_hi - c0 + 1);
        __syncthreads();
        for (int e = tid; e < TROWS * TSTRIDE; e += VT) {
          const int r = e / TSTRIDE, q = e - r * TSTRIDE;
          const int yin = y0 + b0 + r - g.offy, xin = x0 + c0 + q - g.offx;
          double v = 0.0;
          if (r < TY + nb - 1 && q < TX + nc - 1 && yin >= 0 && yin < g.iy && xin >= 0 && xin < g.ix)
            v = (double)in[((int64_t)zin * g.iy + yin) * g.ix + xin];
          put_operand<A, PREC>(tile, TROWS * TSTRIDE, e, v);
        }
        for (int e = tid; e < BC * CC; e += VT) {
          const int b = e / CC, c = e - b * CC;
          double v = 0.0;
          if (b < nb && c < nc) {
            const int hb = g.flip ? g.ky - 1 - (b0 + b) : b0 + b;
            const int hc = g.flip ? g.kx - 1 - (c0 + c) : c0 + c;
            v = (double)H[((int64_t)ha * g.ky + hb) * g.kx + hc];
          }
          put_operand<A, PREC>(hch, BC * CC, e, v);
        }
        __syncthreads();
        const int nc4 = nc & ~3;
        for (int b = 0; b < nb; ++b) {
          A inner[RX];
#pragma unroll
          for (int r = 0; r < RX; ++r) inner[r] = 0;
          const int rowoff = (ty + b) * TSTRIDE + tx * RX;
          for (int c = 0; c < nc4; c += 4) {
            A wh[RX + 4], wl[RX + 4], hh[4], hl[4];
#pragma unroll
            for (int u = 0; u < RX + 4; ++u) {
              wh[u] = tile[rowoff + c + u];
              wl[u] = NP == 2 ? tile[TROWS * TSTRIDE + rowoff + c + u] : (A)0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              hh[u] = hch[b * CC + c + u];
              hl[u] = NP == 2 ? hch[BC * CC + b * CC + c + u] : (A)0;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
              for (int r = 0; r < RX; ++r) inner[r] = mac<A, PREC>(inner[r], hh[u], hl[u], wh[r + u], wl[r + u]);
          }
          for (int c = nc4; c < nc; ++c) {
            const A h1 = hch[b * CC + c];
            const A h2 = NP == 2 ? hch[BC * CC + b * CC + c] : (A)0;
#pragma unroll
            for (int r = 0; r < RX; ++r) {
              const A w1 = tile[rowoff + c + r];
              const A w2 = NP == 2 ? tile[TROWS * TSTRIDE + rowoff + c + r] : (A)0;
              inner[r] = mac<A, PREC>(inner[r], h1, h2, w1, w2);
            }
          }
#pragma unroll
          for (int r = 0; r < RX; ++r) mid[r] += inner[r];
        }
      }
    }
#pragma unroll
    for (int r = 0; r < RX; ++r) outer[r] += mid[r];
  }

  // Epilogue ------------------------------------------------------------------
  double s0 = 0.0, s1 = 0.0;
  const int y = y0 + ty;
  if (y < g.oy) {
    T *dst = out + (ksplit > 1 ? (int64_t)sidx * g.oz * g.oy * g.ox : 0);
#pragma unroll
    for (int r = 0; r < RX; ++r) {
      const int x = x0 + tx * RX + r;
      if (x < g.ox) {
        const int64_t idx = ((int64_t)z * g.oy + y) * g.ox + x;
        apply_epilogue<T>(dst, idx, (T)outer[r], ep, s0, s1);
      }
    }
  }
  if (ep.mode != EPI_STORE) {
    block_sum2(s0, s1, red);
    if (tid == 0) {
      const int64_t blk = blockIdx.x + (int64_t)gridDim.x * (blockIdx.y + (int64_t)gridDim.y * blockIdx.z);
      ep.part[2 * blk] = s0;
      ep.part[2 * blk + 1] = s1;
    }
  }
}

// Sum the ksplit partial outputs of a split-K launch in fixed order.
template <typename T>
__global__ void splitk_reduce_kernel(const T *__restrict__ parts, T *__restrict__ out, int64_t n, int ksplit) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int s = 0; s < ksplit; ++s) acc += (double)parts[(int64_t)s * n + i];
  out[i] = (T)acc;
}

template <typename T, int PREC>
hipError_t launch_valu_t(const Geom &g, const void *in, const void *H, void *out, const Epi &ep, int ksplit,
                         int zchunk, hipStream_t s) {
  dim3 grid((g.ox + TX - 1) / TX, (g.oy + TY - 1) / TY, g.oz * ksplit);
  hipLaunchKernelGGL((conv_valu_kernel<T, PREC>), grid, dim3(VT), 0, s, (const T *)in, (const T *)H, (T *)out, g,
                     ep, ksplit, zchunk);
  return hipGetLastError();
}

}  // namespace

dim3 valu_grid(const Geom &g, int ksplit) {
  return dim3((g.ox + TX - 1) / TX, (g.oy + TY - 1) / TY, g.oz * ksplit);
}

hipError_t launch_conv_valu(const Geom &g, int dtype, int precision, const void *in, const void *H, void *out,
                            const Epi &ep, int ksplit, int zchunk, hipStream_t s) {
  if (dtype == NDC_F64) return launch_valu_t<double, PREC_NATIVE_>(g, in, H, out, ep, ksplit, zchunk, s);
  switch (precision) {
    case NDC_PREC_BF16: return launch_valu_t<float, PREC_BF16_>(g, in, H, out, ep, ksplit, zchunk, s);
    case NDC_PREC_SPLIT_BF16: return launch_valu_t<float, PREC_SPLIT_>(g, in, H, out, ep, ksplit, zchunk, s);
    default: return launch_valu_t<float, PREC_NATIVE_>(g, in, H, out, ep, ksplit, zchunk, s);
  }
}

hipError_t launch_splitk_reduce(int dtype, const void *parts, void *out, int64_t n, int ksplit, hipStream_t s) {
  const int bt = 256;
  dim3 grid((unsigned)((n + bt - 1) / bt));
  if (dtype == NDC_F64)
    hipLaunchKernelGGL(splitk_reduce_kernel<double>, grid, dim3(bt), 0, s, (const double *)parts, (double *)out, n,
                       ksplit);
  else
    hipLaunchKernelGGL(splitk_reduce_kernel<float>, grid, dim3(bt), 0, s, (const float *)parts, (float *)out, n,
                       ksplit);
  return hipGetLastError();
}

}  // namespace ndc
