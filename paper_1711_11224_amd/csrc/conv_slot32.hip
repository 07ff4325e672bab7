// FP32 correlation on the 32x32x2 matrix instruction with the output rows of
// a column held in rotating accumulator slots (the FP32 counterpart of
// conv_slot.hip), for PSFs with kx <= 32, ky <= 32 and kz <= 64.
//
// out[s] = sum_t Hc[t] in[s + t - off]  (see Geom).
//
// v_mfma_f32_32x32x2_f32: D[32x32] += A[32x2] B[2x32].  Lane l holds
//   A[m = l % 32][k = l / 32] and B[k = l / 32][n = l % 32] (one float each),
//   and D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32] in accumulator register r.
// Mapping, for input row yi of input plane zi, PSF plane a and tap pair j:
//   m = output column x0 + m, k = PSF tap c = 2 j + k along x,
//   n = row slot (the output row y = n (mod 32) whose PSF row b = yi + offy
//   - y lies in [0, 32));
//   A[m][k] = in[zi][yi][x0 + m + c - offx],
//   B[k][n] = Hc[a][b(n)][c]   (zero for b(n) >= ky or c >= kx).
// As in the bf16 form a slot keeps its output row while the input rows
// advance and is written out and cleared when the row is complete, so the
// products are PSF taps but for the slots past ky and the taps past kx
// (94% at 31 x 31 PSF rows, against 91% for the 4x4x1 Toeplitz tile).  At
// the FP32 rate an input row carries eight times the bf16 form's matrix
// time, which buries the per-row staging, slot clearing and barrier.
//
// Work-group: 4 waves (one per SIMD) over one column of 8 output planes x 32
// output columns, walked down its rows; the PSF planes reaching the column
// are split between the waves (NB each).  A wave streams the staged input
// planes; input plane w NB + s feeds output plane zo through PSF plane
// aw0 + s - zo.  The A operand of a plane is one float per tap pair read
// from the staged FP32 row; the B operands (one float per lane per PSF
// plane and tap pair) are read from the PSF in global memory (L1/L2), a tap
// pair's NB planes at a time.  Partial rows of the waves are summed in LDS
// in wave order.  The launch is persistent: one
// work-group per CU takes a contiguous run of (column, output row) units of
// near-equal cost.

#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <type_traits>

#include "ndc_device.h"
#include "ndc_internal.h"

namespace ndc {

namespace {

typedef float v16f __attribute__((ext_vector_type(16)));

template <int B, int E, typename F>
__device__ __forceinline__ void floop(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    floop<B + 1, E>(f);
  }
}

constexpr int FT = 256;      // threads per work-group (4 waves, one per SIMD)
constexpr int FW = FT / 64;  // waves
constexpr int FZ = 8;        // output planes per column
constexpr int FMAX_KZ = 64;  // PSF planes: 4 waves x up to 16
constexpr int FMAX_KY = 32;  // row slots
constexpr int FMAX_KX = 32;  // 16 tap pairs

template <int NC>  // tap pairs (8: kx <= 16, 16: kx <= 32)
struct FShape {
  static constexpr int SC = 32 + 2 * NC;                          // staged floats per input plane row
  static constexpr int NST = ((FMAX_KZ + FZ - 1) * SC + FT - 1) / FT;  // staged floats per thread
};

// PSF planes per wave when na planes are split between the 4 waves.
__host__ __device__ inline int f32slot_nb(int na) {
  const int n = (na + FW - 1) / FW;
  return n <= 2 ? n : n <= 4 ? 4 : n <= 6 ? 6 : n <= 8 ? 8 : n <= 12 ? 12 : 16;
}

__host__ __device__ inline int f32slot_planes(int kz) { return FW * f32slot_nb(kz) + FZ - 1; }

template <int NC>
__host__ __device__ inline size_t f32slot_lds_bytes(int kz) {
  return 2 * (size_t)f32slot_planes(kz) * FShape<NC>::SC * 4 + 2 * (size_t)FW * FZ * 32 * 4;
}

__device__ __forceinline__ void f32slot_arange(const Geom &g, int zt, int &alo, int &ahi) {
  const int z0 = zt * FZ, zmax = min(z0 + FZ, g.oz) - 1;
  alo = max(0, g.offz - zmax);
  ahi = min(g.kz - 1, g.iz - 1 + g.offz - z0);
}

// Cost of one output row of a column in z-tile zt, in PSF planes per wave:
// the planes plus about two planes' worth for the staging, slot finishing,
// reduction and barrier of the row.
__device__ __forceinline__ int64_t f32slot_cost(const Geom &g, int zt) {
  int alo, ahi;
  f32slot_arange(g, zt, alo, ahi);
  return (int64_t)f32slot_nb(max(1, ahi - alo + 1)) + 2;
}

template <int NC, bool RLQ, int NB>
__device__ __forceinline__ void f32slot_segment(const float *__restrict__ in, const float *__restrict__ H,
                                                float *__restrict__ out, const Geom &g, const Epi &ep,
                                                float *stage0, float *stage1, float *part, int z0, int x0, int alo,
                                                int ahi, int ya, int yb, double &s0, double &s1) {
  using S = FShape<NC>;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int n = lane & 31, gg = lane >> 5;
  const int na = ahi - alo + 1;
  const int aw0 = alo + w * NB;
  const int cnt = min(NB, ahi + 1 - aw0);  // PSF planes of this wave (<= 0: none)
  const int nwv = (na + NB - 1) / NB;      // waves with PSF planes
  const int np = FW * NB + FZ - 1;         // staged planes
  const int zi0 = z0 + alo - g.offz;       // input plane of staged plane 0
  const int yi0 = max(0, ya - g.offy);
  const int yi1 = yb - 1 + g.ky - 1 - g.offy;

  // Staging of input row yi: float c of plane p is column x0 - offx + c.
  // Unconditional loads from clamped addresses, zeros applied at the LDS
  // write (see conv_slot.hip).
  float sv[S::NST];
  unsigned svok = 0;
  auto load_row = [&](int yi) {
    svok = 0;
#pragma unroll
    for (int u = 0; u < S::NST; ++u) {
      const int e = tid + u * FT;
      const int p = e / S::SC, c = e - p * S::SC;
      const int zi = zi0 + p, xin = x0 - g.offx + c;
      const bool ok = p < np && zi >= 0 && zi < g.iz && xin >= 0 && xin < g.ix;
      sv[u] = in[((int64_t)min(max(zi, 0), g.iz - 1) * g.iy + yi) * g.ix + min(max(xin, 0), g.ix - 1)];
      svok |= (ok ? 1u : 0u) << u;
    }
  };
  auto store_row = [&](float *st) {
#pragma unroll
    for (int u = 0; u < S::NST; ++u) {
      asm volatile("" : "+v"(sv[u]));  // keep the loads' uses here
      const int e = tid + u * FT;
      if (e < np * S::SC) st[e] = ((svok >> u) & 1u) ? sv[u] : 0.f;
    }
  };

  // B operands at input row yi: lane (n, gg) takes tap c = 2 j + gg of slot
  // n's PSF row of plane aw0 + al, zero for an idle slot, a tap past kx or a
  // plane past the wave's count.  Addresses are clamped into H.
  int hrow = 0, hcg = 0;
  bool rowok = false;
  auto prep_b = [&](int yi) {
    const int b = (yi + g.offy - n) & 31;
    rowok = b < g.ky;
    const int hb = g.flip ? g.ky - 1 - b : b;
    hrow = rowok ? hb * g.kx : 0;
    hcg = g.flip ? g.kx - 1 - gg : gg;
  };
  // All NB planes' operands of tap pair j (one register per plane).  Every
  // load is unconditional, at a 32-bit offset clamped into H (kz ky kx <=
  // 2^16), and zeroed with a bit mask: a select on the loaded value lets the
  // compiler sink the load into a branch and wait for it there.
  const int kyx = g.ky * g.kx;
  auto load_bj = [&](int j, float (&bo)[NB]) {
    const int c = 2 * j + gg;
    const int hc = min(max(g.flip ? hcg - 2 * j : hcg + 2 * j, 0), g.kx - 1);
    const unsigned keep = (rowok && c < g.kx) ? ~0u : 0u;
#pragma unroll
    for (int al = 0; al < NB; ++al) {
      const int a = aw0 + al;
      const int ha = min(max(g.flip ? g.kz - 1 - a : a, 0), g.kz - 1);
      const unsigned v = __float_as_uint(H[ha * kyx + hrow + hc]);
      bo[al] = __uint_as_float(v & (al < cnt ? keep : 0u));
    }
  };

  // A operand of staged plane p, tap pair j: lane (m = n, gg) reads column
  // m + 2 j + gg.
  const int aoff = n + gg;

  v16f acc[FZ];
#pragma unroll
  for (int zo = 0; zo < FZ; ++zo) acc[zo] = (v16f){};

  // Tap pairs outer, planes inner: the NB B operands of a tap pair sit in
  // registers (the next pair's load a whole pair ahead, which covers the
  // global-memory latency), the A operand of each (plane, pair) is one LDS
  // read issued a plane ahead.  Staged plane w NB + s feeds output plane zo
  // through PSF plane aw0 + s - zo.
  // Two-level summation: the row's products accumulate in fresh registers
  // (the first instruction of each output plane takes a zero C) and are added
  // to the slots once per row, so a slot sums ky row totals of 2 NB NC
  // products each rather than one chain of ky 2 NB NC products; on 63 x 31 x
  // 31 taps this keeps the FP32 rounding error at the 4x4 tile's level.
  auto compute = [&](const float *st) {
    const float *q = st + w * NB * S::SC + aoff;
    float b0[NB], b1[NB];
    v16f t[FZ];
    load_bj(0, b0);
    floop<0, NC>([&](auto jc) {
      constexpr int j = decltype(jc)::value;
      float(&bj)[NB] = (j & 1) ? b1 : b0;
      float(&bn)[NB] = (j & 1) ? b0 : b1;
      if constexpr (j + 1 < NC) load_bj(j + 1, bn);
      float a0 = q[2 * j], a1;
      floop<0, NB + FZ - 1>([&](auto sc) {
        constexpr int s = decltype(sc)::value;
        constexpr int zlo = s - NB + 1 > 0 ? s - NB + 1 : 0;
        constexpr int zhi = s < FZ - 1 ? s : FZ - 1;
        float &a = (s & 1) ? a1 : a0;
        float &an = (s & 1) ? a0 : a1;
        if constexpr (s + 1 < NB + FZ - 1) an = q[(s + 1) * S::SC + 2 * j];
        floop<zlo, zhi + 1>([&](auto zc) {
          constexpr int zo = zhi - (decltype(zc)::value - zlo);  // descending: the same slot's instructions further apart
          if constexpr (j == 0 && s == zo)  // output plane zo's first product of the row
            t[zo] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bj[s - zo], (v16f){}, 0, 0, 0);
          else
            t[zo] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, bj[s - zo], t[zo], 0, 0, 0);
        });
        __builtin_amdgcn_sched_barrier(0);
      });
    });
#pragma unroll
    for (int zo = 0; zo < FZ; ++zo) acc[zo] += t[zo];
  };

  // Finished row in slot nf: lanes nf, nf + 32 hold its 32 columns.
  auto finish_row = [&](int nf, bool keep, float *pb) {
    if (n == nf) {
      if (keep) {
#pragma unroll
        for (int zo = 0; zo < FZ; ++zo)
#pragma unroll
          for (int qd = 0; qd < 4; ++qd) {
            const float4 v = make_float4(acc[zo][4 * qd], acc[zo][4 * qd + 1], acc[zo][4 * qd + 2],
                                         acc[zo][4 * qd + 3]);
            *(float4 *)(pb + (w * FZ + zo) * 32 + 8 * qd + 4 * gg) = v;
          }
      }
#pragma unroll
      for (int zo = 0; zo < FZ; ++zo) acc[zo] = (v16f){};
    }
  };

  auto reduce_row = [&](int yf, const float *pb) {
    if (tid < FZ * 32) {
      const int zo = tid >> 5, x = tid & 31;
      const int z = z0 + zo, xo = x0 + x;
      if (z < g.oz && xo < g.ox) {
        float v = 0.f;
        for (int ww = 0; ww < nwv; ++ww) v += pb[(ww * FZ + zo) * 32 + x];
        if constexpr (!RLQ) {
          if (ep.mode == EPI_RLQ) __builtin_unreachable();
        }
        apply_epilogue<float>(out, ((int64_t)z * g.oy + yf) * g.ox + xo, v, ep, s0, s1);
      }
    }
  };

  constexpr int PB = FW * FZ * 32;
  load_row(min(yi0, g.iy - 1));
  store_row(stage0);
  __syncthreads();
  int pend = -1;
  int k = 0;
  for (int yi = yi0; yi <= yi1; ++yi, ++k) {
    const float *cur = (k & 1) ? stage1 : stage0;
    float *nxt = (k & 1) ? stage0 : stage1;
    float *pcur = part + (k & 1) * PB;
    const float *pprev = part + ((k & 1) ^ 1) * PB;
    if (pend >= 0) reduce_row(pend, pprev);
    load_row(min(yi + 1, g.iy - 1));
    if (cnt > 0) {
      if (yi < g.iy) {
        prep_b(yi);
        compute(cur);
      }
      const int yf = yi + g.offy - (g.ky - 1);
      finish_row(yf & 31, yf >= ya && yf < yb, pcur);
    }
    {
      const int yf = yi + g.offy - (g.ky - 1);
      pend = (yf >= ya && yf < yb) ? yf : -1;
    }
    store_row(nxt);
    __syncthreads();
  }
  if (pend >= 0) reduce_row(pend, part + ((k & 1) ^ 1) * PB);
  __syncthreads();
}

template <int NC, bool RLQ>
__device__ __forceinline__ void f32slot_run(const float *in, const float *H, float *out, const Geom &g,
                                            const Epi &ep, float *stage0, float *stage1, float *part, int z0,
                                            int x0, int alo, int ahi, int ya, int yb, double &s0, double &s1) {
  switch (f32slot_nb(ahi - alo + 1)) {
#define NDC_F32SLOT_NB(K)                                                                                    \
  case K:                                                                                                    \
    f32slot_segment<NC, RLQ, K>(in, H, out, g, ep, stage0, stage1, part, z0, x0, alo, ahi, ya, yb, s0, s1); \
    break;
    NDC_F32SLOT_NB(1)
    NDC_F32SLOT_NB(2)
    NDC_F32SLOT_NB(4)
    NDC_F32SLOT_NB(6)
    NDC_F32SLOT_NB(8)
    NDC_F32SLOT_NB(12)
    NDC_F32SLOT_NB(16)
#undef NDC_F32SLOT_NB
    default: break;
  }
}

template <int NC, bool RLQ>
__global__ __launch_bounds__(FT, 1) void conv_slot32_kernel(const float *__restrict__ in,
                                                            const float *__restrict__ H, float *__restrict__ out,
                                                            Geom g, Epi ep, int nxt, int nzt) {
  if (ep.phase && !((1 << *ep.phase) & ep.phase_mask)) return;  // uniform early exit
  using S = FShape<NC>;
  extern __shared__ __align__(16) float flds[];
  __shared__ double red[FW][2];
  const int tid = threadIdx.x;
  const int nps = f32slot_planes(g.kz);
  float *stage0 = flds;
  float *stage1 = stage0 + nps * S::SC;
  float *part = stage1 + nps * S::SC;

  // Persistent split as in conv_slot.hip.
  const int G = gridDim.x, bid = blockIdx.x;
  const int L = (G % 8 == 0) ? (bid % 8) * (G / 8) + bid / 8 : bid;
  const int64_t colrows = (int64_t)nxt * g.oy;
  int64_t T = 0;
  for (int zt = 0; zt < nzt; ++zt) T += f32slot_cost(g, zt) * colrows;
  auto locate = [&](int64_t u) -> int64_t {
    int64_t accu = 0, base = 0;
    for (int zt = 0; zt < nzt; ++zt) {
      const int64_t cz = f32slot_cost(g, zt);
      if (u <= accu + (colrows - 1) * cz) {
        const int64_t r = u - accu;
        return base + (r <= 0 ? 0 : (r + cz - 1) / cz);
      }
      accu += colrows * cz;
      base += colrows;
    }
    return base;
  };
  const int64_t u0 = locate(T * L / G), u1 = locate(T * (L + 1) / G);

  double s0 = 0.0, s1 = 0.0;
  for (int64_t u = u0; u < u1;) {
    const int64_t col = u / g.oy;
    const int ya = (int)(u - col * g.oy);
    const int64_t uend = min(u1, (col + 1) * g.oy);
    const int yb = ya + (int)(uend - u);
    const int zt = (int)(col / nxt), xt = (int)(col - (int64_t)zt * nxt);
    int alo, ahi;
    f32slot_arange(g, zt, alo, ahi);
    f32slot_run<NC, RLQ>(in, H, out, g, ep, stage0, stage1, part, zt * FZ, xt * 32, alo, ahi, ya, yb, s0, s1);
    u = uend;
  }
  if (ep.mode != EPI_STORE) {
    block_sum2(s0, s1, red);
    if (tid == 0) {
      ep.part[2 * (int64_t)bid] = s0;
      ep.part[2 * (int64_t)bid + 1] = s1;
    }
  }
}

template <int NC, bool RLQ>
hipError_t launch_f32slot(const ConvPlan &pl, const Geom &g, const void *in, const void *H, void *out,
                          const Epi &ep, hipStream_t s) {
  static std::once_flag lds_once;
  std::call_once(lds_once, [] {
    (void)hipFuncSetAttribute((const void *)conv_slot32_kernel<NC, RLQ>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)f32slot_lds_bytes<NC>(FMAX_KZ));
    (void)hipGetLastError();
  });
  const int nxt = (g.ox + 31) / 32, nzt = (g.oz + FZ - 1) / FZ;
  hipLaunchKernelGGL((conv_slot32_kernel<NC, RLQ>), pl.grid, dim3(FT), pl.lds_bytes, s, (const float *)in,
                     (const float *)H, (float *)out, g, ep, nxt, nzt);
  return hipGetLastError();
}

int f32slot_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) {
    (void)hipGetLastError();
    cus = 1;
  }
  return cus;
}

}  // namespace

// The FP32 row-slot tile can run this problem (FP32 storage, native
// precision, PSF extents).
bool slot32_fits(const Geom &g, int dtype, int precision) {
  return dtype == NDC_F32 && precision == NDC_PREC_NATIVE && g.kx <= FMAX_KX && g.ky <= FMAX_KY &&
         g.kz <= FMAX_KZ;
}

ConvPlan plan_conv_slot32(const Geom &g) {
  ConvPlan pl{};
  pl.variant = 5;
  const int64_t units = (int64_t)((g.ox + 31) / 32) * ((g.oz + FZ - 1) / FZ) * g.oy;
  const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(f32slot_cus(), units / 32));
  pl.grid = dim3((unsigned)grid);
  pl.block = dim3(FT);
  pl.lds_bytes = g.kx <= 16 ? f32slot_lds_bytes<8>(g.kz) : f32slot_lds_bytes<16>(g.kz);
  pl.nblocks = grid;
  return pl;
}

hipError_t launch_conv_slot32(const ConvPlan &pl, const Geom &g, const void *in, const void *H, void *out,
                              const Epi &ep, hipStream_t s) {
  const bool rlq = ep.mode == EPI_RLQ;
  if (g.kx <= 16)
    return rlq ? launch_f32slot<8, true>(pl, g, in, H, out, ep, s) : launch_f32slot<8, false>(pl, g, in, H, out, ep, s);
  return rlq ? launch_f32slot<16, true>(pl, g, in, H, out, ep, s) : launch_f32slot<16, false>(pl, g, in, H, out, ep, s);
}

}  // namespace ndc
