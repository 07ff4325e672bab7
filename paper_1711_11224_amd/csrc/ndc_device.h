// Device-side helpers shared by the library's kernels.
#pragma once
#include "ndc_internal.h"

namespace ndc {

enum { PREC_NATIVE_ = 0, PREC_BF16_ = 1, PREC_SPLIT_ = 2 };

// Round a float to the nearest bfloat16 (ties to even) and return it as a
// float.  Infinities pass through; NaNs stay NaN (quiet bit forced).
__device__ inline float bf16_round(float v) {
  uint32_t u = __float_as_uint(v);
  if ((u & 0x7f800000u) == 0x7f800000u) return __uint_as_float((u | ((u & 0x007fffffu) ? 0x00400000u : 0u)) & 0xffff0000u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

// max(v, 0) that keeps NaN (the projection of Step 2 must not hide NaN).
template <typename T>
__device__ inline T proj_nonneg(T v) {
  return v > (T)0 ? v : (v != v ? v : (T)0);
}

template <typename T>
__device__ inline void apply_epilogue(T *out, int64_t idx, T acc, const Epi &ep, double &s0, double &s1) {
  if (ep.mode == EPI_STORE) {
    out[idx] = acc;
  } else if (ep.mode == EPI_RESID) {
    const T r = acc - ((const T *)ep.Y)[idx];
    out[idx] = r;
    s0 += (double)r * (double)r;
  } else if (ep.mode == EPI_GRAD) {
    T g = acc + (T)ep.lambda * ((const T *)ep.X)[idx];
    if (ep.Q) g += (T)ep.mu * ((const T *)ep.Q)[idx];
    out[idx] = g;
    s0 += (double)g * (double)g;
  } else if (ep.mode == EPI_RINC) {
    const T r = ((const T *)ep.B)[idx] + acc;
    out[idx] = r;
    s0 += (double)r * (double)r;
    s1 += (double)acc * (double)acc;
  } else if (ep.mode == EPI_RLQ) {
    const T y = ((const T *)ep.Y)[idx];
    out[idx] = acc > (T)0 ? y / acc : (T)0;
    // y log(y/a) - y + a with 0 log 0 = 0 (+inf where a = 0 < y)
    const double yd = (double)y, ad = (double)acc;
    s0 += (yd > 0.0 ? (ad > 0.0 ? yd * log(yd / ad) : INFINITY) : 0.0) - yd + ad;
  } else if (ep.mode == EPI_RLX) {
    out[idx] = out[idx] * acc * (T)(*ep.delta);
  } else if (ep.mode == EPI_NORM) {
    s0 += (double)acc * (double)acc;
  } else if (ep.mode == EPI_SQR) {
    out[idx] = acc;
    s0 += (double)acc * (double)acc;
  } else {
    const T x = ((const T *)ep.X)[idx];
    T gr = acc + (T)ep.lambda * x;
    if (ep.Q) gr += (T)ep.mu * ((const T *)ep.Q)[idx];
    ((T *)ep.G)[idx] = gr;
    const T xt = proj_nonneg<T>(x - (T)(*ep.delta) * gr);
    out[idx] = xt;
    s0 += (double)xt * (double)xt;
    const double d = (double)xt - (double)x;
    s1 += d * d;
  }
}

// Deterministic work-group sum of two doubles: xor butterfly inside each
// 64-lane wave, then wave partials in index order.  The result is valid in
// thread 0.  `red` holds one pair per wave.
__device__ inline void block_sum2(double &s0, double &s1, double (*red)[2]) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    s0 += __shfl_xor(s0, off, 64);
    s1 += __shfl_xor(s1, off, 64);
  }
  const int w = threadIdx.x / 64, nw = blockDim.x / 64;
  if ((threadIdx.x & 63) == 0) {
    red[w][0] = s0;
    red[w][1] = s1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0, b = 0.0;
    for (int i = 0; i < nw; ++i) {
      a += red[i][0];
      b += red[i][1];
    }
    s0 = a;
    s1 = b;
  }
}

// Launchers defined in the kernel files.
dim3 valu_grid(const Geom &g, int ksplit);
hipError_t launch_conv_valu(const Geom &g, int dtype, int precision, const void *in, const void *H, void *out,
                            const Epi &ep, int ksplit, int zchunk, hipStream_t s);
hipError_t launch_splitk_reduce(int dtype, const void *parts, void *out, int64_t n, int ksplit, hipStream_t s);

}  // namespace ndc
