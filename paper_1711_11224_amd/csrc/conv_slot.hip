// bf16 correlation on the 32x32x16 matrix instruction with the output rows
// of a column held in rotating accumulator slots, for PSFs with kx <= 32,
// ky <= 32 and kz <= 64 (FP32 storage, FP32 accumulation).
//
// out[s] = sum_t Hc[t] in[s + t - off]  (see Geom).
//
// v_mfma_f32_32x32x16_bf16: D[32x32] += A[32x16] B[16x32].  Lane l holds
//   A[m = l % 32][k = 8 (l / 32) + e] and B[k = 8 (l / 32) + e][n = l % 32]
//   for e = 0..7, and D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32] in
//   accumulator register r.
// Mapping, for input row yi of input plane zi, PSF plane a and tap chunk j:
//   m = output column x0 + m, k = PSF tap c = 16 j + k along x,
//   n = row slot: slot n holds the output row y = n (mod 32) whose PSF row
//   b = yi + offy - y lies in [0, 32);
//   A[m][k] = in[zi][yi][x0 + m + c - offx]   (a window of the input row),
//   B[k][n] = Hc[a][b(n)][c]   (zero for b(n) >= ky or c >= kx).
// Walking yi upward, a slot keeps its output row while the row's PSF row b
// advances by one per input row; the row is complete at b = ky - 1, is
// written out, and its slot is cleared for the row 32 further down.  So
// every product is a PSF tap except for the slots past ky and the taps past
// kx (94% at 31 x 31 PSF rows, against 48% for the Toeplitz form of
// conv_mfma32.hip, whose x window is the contraction).
//
// Work-group: 8 waves over one column of 8 output planes x 32 output
// columns, walked down its rows.  The PSF planes that reach the column are
// split between the waves (up to 8 each).  A wave loads its B operands
// (its PSF planes at the current input row's slot rows) into registers once
// per input row and streams the staged input planes through them; each input
// plane feeds the 8 output planes it reaches.  The waves' partial rows are
// summed in LDS in wave order (deterministic).  The whole PSF sits in LDS for
// the work-group's lifetime as bf16, the 16-byte chunks of each row permuted
// so that eight lanes reading eight consecutive rows hit distinct banks; one
// input row of every input plane the column reaches is staged per step,
// double-buffered.  The launch is persistent: one work-group per CU takes a
// contiguous run of (column, output row) units of near-equal cost, so a
// column shared by two work-groups costs one refill of ky - 1 rows.

#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <type_traits>

#include "ndc_device.h"
#include "ndc_internal.h"

namespace ndc {

namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));

template <int B, int E, typename F>
__device__ __forceinline__ void sloop(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sloop<B + 1, E>(f);
  }
}

constexpr int ST = 256;      // threads per work-group (4 waves, one per SIMD)
constexpr int SW = ST / 64;  // waves
constexpr int SZ = 8;        // output planes per column
constexpr int SMAX_KZ = 64;  // PSF planes: 4 waves x up to 16
constexpr int SMAX_KY = 32;  // row slots
constexpr int SMAX_KX = 32;  // two chunks of 16 taps

template <int NJ>
struct SShape {
  static constexpr int ROWB = 32 * NJ;     // bytes of one PSF row in LDS (16 NJ taps)
  static constexpr int SCW = 16 + 8 * NJ;  // dwords of one staged input row (32 + 16 NJ columns)
  static constexpr int NPAIR = ((SMAX_KZ + SZ - 1) * SCW + ST - 1) / ST;  // staged dwords per thread
};

// PSF planes per wave when the column's na planes are split between the
// waves: ceil(na / 4) rounded up to an instantiated count.
__host__ __device__ inline int slot_nb(int na) {
  const int n = (na + SW - 1) / SW;
  return n <= 2 ? n : n <= 4 ? 4 : n <= 6 ? 6 : n <= 8 ? 8 : n <= 12 ? 12 : 16;
}

// Staged input planes at most: 4 waves x their planes + the 7 more the last
// wave's planes reach.
__host__ __device__ inline int slot_planes(int kz) { return SW * slot_nb(kz) + SZ - 1; }


// LDS bytes: the PSF (kz planes of ky rows) and a zero row, two staging
// buffers, two buffers of partial rows (4 waves x 8 planes x 32 columns).
template <int NJ>
__host__ __device__ inline size_t slot_lds_bytes(int kz, int ky) {
  using S = SShape<NJ>;
  return (size_t)kz * ky * S::ROWB + S::ROWB + 2 * (size_t)slot_planes(kz) * S::SCW * 4 +
         2 * (size_t)SW * SZ * 32 * 4;
}

// Position of 16-byte chunk c of PSF row b: permuted by the row's place
// among the rows sharing one 128-byte bank line.
template <int NJ>
__device__ __forceinline__ int chunk_pos(int c, int b) {
  return NJ == 2 ? c ^ ((b >> 1) & 3) : c ^ ((b >> 2) & 1);
}

__device__ __forceinline__ unsigned pack2_bf16(float a, float b) {
  const unsigned short ua = __builtin_bit_cast(unsigned short, (__bf16)a);
  const unsigned short ub = __builtin_bit_cast(unsigned short, (__bf16)b);
  return (unsigned)ua | ((unsigned)ub << 16);
}

// PSF planes a whose input planes reach z-tile zt (output planes
// [8 zt, 8 zt + 8) clipped to oz): zi = zo + a - offz in [0, iz).
__device__ __forceinline__ void slot_arange(const Geom &g, int zt, int &alo, int &ahi) {
  const int z0 = zt * SZ, zmax = min(z0 + SZ, g.oz) - 1;
  alo = max(0, g.offz - zmax);
  ahi = min(g.kz - 1, g.iz - 1 + g.offz - z0);
}

// Cost of one output row of a column in z-tile zt, in units of one PSF
// plane per wave: the planes plus the per-row staging, slot finishing,
// reduction and barrier, which cost about 20 planes' worth (measured on
// MI355X: about 4 us of fixed time per row against 0.2 us per plane).
__device__ __forceinline__ int64_t slot_cost(const Geom &g, int zt) {
  int alo, ahi;
  slot_arange(g, zt, alo, ahi);
  return (int64_t)slot_nb(max(1, ahi - alo + 1)) + 20;
}

// One column segment: output planes z0.., columns x0.., rows [ya, yb).
template <int NJ, bool RLQ, int NB>
__device__ __forceinline__ void slot_segment(const float *__restrict__ in, float *__restrict__ out,
                                             const Geom &g, const Epi &ep, const unsigned char *psf,
                                             unsigned *stage0, unsigned *stage1, float *part, int z0, int x0,
                                             int alo, int ahi, int ya, int yb, double &s0, double &s1) {
  using S = SShape<NJ>;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int n = lane & 31, gg = lane >> 5;
  const int pp = g.ky * S::ROWB;  // bytes per PSF plane
  const int zoff = g.kz * pp;  // the zero row after the PSF planes
  const int na = ahi - alo + 1;
  const int aw0 = alo + w * NB;
  const int cnt = min(NB, ahi + 1 - aw0);  // PSF planes of this wave (<= 0: none)
  const int nwv = (na + NB - 1) / NB;      // waves with PSF planes
  const int np = SW * NB + SZ - 1;         // staged planes (the reach of every wave)
  const int zi0 = z0 + alo - g.offz;        // input plane of staged plane 0
  const int yi0 = max(0, ya - g.offy);
  const int yi1 = yb - 1 + g.ky - 1 - g.offy;  // steps past the input only finish rows

  // Staging of input row yi: dword d of plane p holds columns 2d, 2d + 1 of
  // the window x0 - offx + [0, 32 + 16 NJ), zero outside the input.  The
  // loads are unconditional, from addresses clamped into the input, and the
  // zeros are applied when the row is written to LDS: a conditional load
  // lets the compiler pack its value right after it, which waits for it
  // there instead of after the row's matrix instructions.
  float sv[2 * S::NPAIR];
  unsigned svok = 0;  // bit 2u: first value inside the input, 2u + 1: second
  auto load_row = [&](int yi) {
    svok = 0;
#pragma unroll
    for (int u = 0; u < S::NPAIR; ++u) {
      const int e = tid + u * ST;
      const int p = e / S::SCW, d = e - p * S::SCW;
      const int zi = zi0 + p, xin = x0 - g.offx + 2 * d;
      const bool zok = p < np && zi >= 0 && zi < g.iz;
      const bool ok0 = zok && xin >= 0 && xin < g.ix;
      const bool ok1 = zok && xin + 1 >= 0 && xin + 1 < g.ix;
      const float *row = in + ((int64_t)min(max(zi, 0), g.iz - 1) * g.iy + yi) * g.ix;
      sv[2 * u] = row[min(max(xin, 0), g.ix - 1)];
      sv[2 * u + 1] = row[min(max(xin + 1, 0), g.ix - 1)];
      svok |= (ok0 ? 1u : 0u) << (2 * u);
      svok |= (ok1 ? 1u : 0u) << (2 * u + 1);
    }
  };
  auto store_row = [&](unsigned *st) {
#pragma unroll
    for (int u = 0; u < S::NPAIR; ++u) {
      asm volatile("" : "+v"(sv[2 * u]), "+v"(sv[2 * u + 1]));  // keep the loads' uses here
      const int e = tid + u * ST;
      const float v0 = ((svok >> (2 * u)) & 1u) ? sv[2 * u] : 0.f;
      const float v1 = ((svok >> (2 * u + 1)) & 1u) ? sv[2 * u + 1] : 0.f;
      if (e < np * S::SCW) st[e] = pack2_bf16(v0, v1);
    }
  };

  // B operands of this wave at input row yi: lane (n, gg) reads chunk
  // 2 j + gg of slot n's PSF row in plane aw0 + al (the zero row for an idle
  // slot or a plane past the wave's count).
  int bbase[NJ], bstride = 0;
  auto prep_b = [&](int yi) {
    const int b = (yi + g.offy - n) & 31;
    const bool rowok = b < g.ky;
    bstride = rowok ? pp : 0;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int c = 2 * j + gg;
      bbase[j] = rowok ? aw0 * pp + b * S::ROWB + 16 * chunk_pos<NJ>(c, b) : zoff + 16 * c;
    }
  };
  // Planes past the wave's count read the zero row; the choice is integer
  // masking (no branch: al is a constant, cnt uniform).
  auto load_b = [&](int al, v8bf (&bo)[NJ]) {
    const int keep = (al - cnt) >> 31;  // -1 when al < cnt, else 0
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int zc = zoff + 16 * (2 * j + gg);
      const unsigned off = (unsigned)(zc + ((bbase[j] + al * bstride - zc) & keep));
      bo[j] = __builtin_bit_cast(v8bf, *(const v4u *)(psf + off));
    }
  };

  // A operand of staged plane p: lane (m = n, gg) needs columns
  // m + 16 j + 8 gg .. +7, i.e. five dwords realigned by one column when m
  // is odd.
  const int sh = (n & 1) * 2;
  const int aoff = (n >> 1) + 4 * gg;
  auto load_a = [&](const unsigned *st, int p, v8bf (&a)[NJ]) {
    const unsigned *q = st + p * S::SCW + aoff;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const unsigned d0 = q[8 * j], d1 = q[8 * j + 1], d2 = q[8 * j + 2], d3 = q[8 * j + 3], d4 = q[8 * j + 4];
      v4u v;
      v[0] = __builtin_amdgcn_alignbyte(d1, d0, sh);
      v[1] = __builtin_amdgcn_alignbyte(d2, d1, sh);
      v[2] = __builtin_amdgcn_alignbyte(d3, d2, sh);
      v[3] = __builtin_amdgcn_alignbyte(d4, d3, sh);
      a[j] = __builtin_bit_cast(v8bf, v);
    }
  };

  v16f acc[SZ];
#pragma unroll
  for (int zo = 0; zo < SZ; ++zo) acc[zo] = (v16f){};

  // Staged plane w NB + s feeds output plane zo through PSF plane
  // aw0 + s - zo (s in [0, NB + 7)).  Plane s needs the B operands of the
  // wave's planes s - 7 .. s: a window of 9 register sets (plane al in set
  // al % 9) where the next plane's operands load while set (al - 8) % 9 is
  // dead, and the A operands one plane ahead.  The scheduling barrier keeps
  // the compiler from hoisting more reads (their registers would not fit
  // beside the accumulators).
  auto compute = [&](const unsigned *st) {
    const int p0 = w * NB;
    v8bf bw[9][NJ];
    v8bf a0[NJ], a1[NJ];
    load_b(0, bw[0]);
    load_a(st, p0, a0);
    sloop<0, NB + SZ - 1>([&](auto sc) {
      constexpr int s = decltype(sc)::value;
      constexpr int zlo = s - NB + 1 > 0 ? s - NB + 1 : 0;
      constexpr int zhi = s < SZ - 1 ? s : SZ - 1;
      v8bf(&a)[NJ] = (s & 1) ? a1 : a0;
      v8bf(&an)[NJ] = (s & 1) ? a0 : a1;
      if constexpr (s + 1 < NB) load_b(s + 1, bw[(s + 1) % 9]);
      if constexpr (s + 1 < NB + SZ - 1) load_a(st, p0 + s + 1, an);
      sloop<0, NJ>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        sloop<zlo, zhi + 1>([&](auto zc) {
          constexpr int zo = decltype(zc)::value;
          acc[zo] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[j], bw[(s - zo) % 9][j], acc[zo], 0, 0, 0);
        });
      });
      __builtin_amdgcn_sched_barrier(0);
    });
  };

  // The row in slot nf is complete: lanes nf and nf + 32 hold its 32
  // columns (register r: column 8 (r / 4) + 4 gg + r % 4); write them to the
  // wave's partial row when kept, then clear the slot.
  auto finish_row = [&](int nf, bool keep, float *pb) {
    if (n == nf) {
      if (keep) {
#pragma unroll
        for (int zo = 0; zo < SZ; ++zo)
#pragma unroll
          for (int qd = 0; qd < 4; ++qd) {
            const float4 v = make_float4(acc[zo][4 * qd], acc[zo][4 * qd + 1], acc[zo][4 * qd + 2],
                                         acc[zo][4 * qd + 3]);
            *(float4 *)(pb + (w * SZ + zo) * 32 + 8 * qd + 4 * gg) = v;
          }
      }
#pragma unroll
      for (int zo = 0; zo < SZ; ++zo) acc[zo] = (v16f){};
    }
  };

  // Sum of the waves' partial rows (wave order), epilogue and store.
  auto reduce_row = [&](int yf, const float *pb) {
    if (tid < SZ * 32) {
      const int zo = tid >> 5, x = tid & 31;
      const int z = z0 + zo, xo = x0 + x;
      if (z < g.oz && xo < g.ox) {
        float v = 0.f;
        for (int ww = 0; ww < nwv; ++ww) v += pb[(ww * SZ + zo) * 32 + x];
        if constexpr (!RLQ) {
          if (ep.mode == EPI_RLQ) __builtin_unreachable();
        }
        apply_epilogue<float>(out, ((int64_t)z * g.oy + yf) * g.ox + xo, v, ep, s0, s1);
      }
    }
  };

  constexpr int PB = SW * SZ * 32;  // floats of one partial-row buffer
  // Every row load is consumed by its store on the same path (rows past the
  // input are clamped to the last one and staged unused), so no load is left
  // in flight across a branch: the compiler's wait analysis then never has
  // to wait for the next row's loads inside the matrix instructions.
  load_row(min(yi0, g.iy - 1));
  store_row(stage0);
  __syncthreads();
  int pend = -1;  // row whose partials wait in the other buffer
  int k = 0;
  for (int yi = yi0; yi <= yi1; ++yi, ++k) {
    const unsigned *cur = (k & 1) ? stage1 : stage0;
    unsigned *nxt = (k & 1) ? stage0 : stage1;
    float *pcur = part + (k & 1) * PB;
    const float *pprev = part + ((k & 1) ^ 1) * PB;
    // the epilogue's own loads complete before the next row's staging loads
    // are issued: the staging loads then stay in flight through the matrix
    // instructions (a wait for a later load would wait for them too)
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
  __syncthreads();  // LDS is reused by the next segment
}

// PSF planes per wave NB = slot_nb(na): one instantiation per count.
template <int NJ, bool RLQ>
__device__ __forceinline__ void slot_run(const float *in, float *out, const Geom &g, const Epi &ep,
                                         const unsigned char *psf, unsigned *stage0, unsigned *stage1, float *part,
                                         int z0, int x0, int alo, int ahi, int ya, int yb, double &s0, double &s1) {
  switch (slot_nb(ahi - alo + 1)) {
#define NDC_SLOT_NB(K)                                                                                        \
  case K:                                                                                                     \
    slot_segment<NJ, RLQ, K>(in, out, g, ep, psf, stage0, stage1, part, z0, x0, alo, ahi, ya, yb, s0, s1); \
    break;
    NDC_SLOT_NB(1)
    NDC_SLOT_NB(2)
    NDC_SLOT_NB(4)
    NDC_SLOT_NB(6)
    NDC_SLOT_NB(8)
    NDC_SLOT_NB(12)
    NDC_SLOT_NB(16)
#undef NDC_SLOT_NB
    default: break;
  }
}

// RLQ: the instantiation that also serves the Richardson-Lucy quotient
// epilogue (its logarithm's constants would otherwise hold registers beside
// the accumulators in every instantiation).
template <int NJ, bool RLQ>
__global__ __launch_bounds__(ST, 1) void conv_slot_kernel(const float *__restrict__ in,
                                                          const float *__restrict__ H, float *__restrict__ out,
                                                          Geom g, Epi ep, int nxt, int nzt) {
  if (ep.phase && !((1 << *ep.phase) & ep.phase_mask)) return;  // uniform early exit
  using S = SShape<NJ>;
  extern __shared__ __align__(16) unsigned char slds[];
  __shared__ double red[SW][2];
  const int tid = threadIdx.x;
  const int pp = g.ky * S::ROWB;
  const int nps = slot_planes(g.kz);
  unsigned char *psf = slds;
  unsigned char *zrow = slds + g.kz * pp;
  unsigned *stage0 = (unsigned *)(zrow + S::ROWB);
  unsigned *stage1 = stage0 + nps * S::SCW;
  float *part = (float *)(stage1 + nps * S::SCW);

  // PSF planes of Hc as bf16: tap pair (2 d, 2 d + 1) of row b of plane a
  // at a pp + b ROWB + 16 chunk_pos(d / 4, b) + 4 (d % 4); taps past kx zero.
  {
    constexpr int DW = S::ROWB / 4;  // dwords per row
    const int words = g.kz * g.ky * DW;
    for (int e = tid; e < words; e += ST) {
      const int ab = e / DW, d = e - ab * DW;
      const int a = ab / g.ky, b = ab - a * g.ky;
      const int ha = g.flip ? g.kz - 1 - a : a;
      const int hb = g.flip ? g.ky - 1 - b : b;
      const float *hrow = H + ((int64_t)ha * g.ky + hb) * g.kx;
      const int c0 = 2 * d;
      const float v0 = c0 < g.kx ? hrow[g.flip ? g.kx - 1 - c0 : c0] : 0.f;
      const float v1 = c0 + 1 < g.kx ? hrow[g.flip ? g.kx - 2 - c0 : c0 + 1] : 0.f;
      *(unsigned *)(psf + a * pp + b * S::ROWB + 16 * chunk_pos<NJ>(d >> 2, b) + 4 * (d & 3)) = pack2_bf16(v0, v1);
    }
    for (int e = tid; e < S::ROWB / 4; e += ST) ((unsigned *)zrow)[e] = 0u;
  }
  // (the first segment's barrier orders these writes before any read)

  // Persistent split: work-group L takes the (column, output row) units
  // whose cost prefix falls in [T L / G, T (L + 1) / G); XCD x (= block
  // index mod 8) gets the contiguous range of logical indices x G/8 ..
  const int G = gridDim.x, bid = blockIdx.x;
  const int L = (G % 8 == 0) ? (bid % 8) * (G / 8) + bid / 8 : bid;
  const int64_t colrows = (int64_t)nxt * g.oy;  // units of one z-tile
  int64_t T = 0;
  for (int zt = 0; zt < nzt; ++zt) T += slot_cost(g, zt) * colrows;
  // first unit whose cost prefix is >= u (the end when none)
  auto locate = [&](int64_t u) -> int64_t {
    int64_t accu = 0, base = 0;
    for (int zt = 0; zt < nzt; ++zt) {
      const int64_t cz = slot_cost(g, zt);
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
    slot_arange(g, zt, alo, ahi);
    slot_run<NJ, RLQ>(in, out, g, ep, psf, stage0, stage1, part, zt * SZ, xt * 32, alo, ahi, ya, yb, s0, s1);
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

template <int NJ, bool RLQ>
hipError_t launch_slot(const ConvPlan &pl, const Geom &g, const void *in, const void *H, void *out, const Epi &ep,
                       hipStream_t s) {
  static std::once_flag lds_once;
  std::call_once(lds_once, [] {
    (void)hipFuncSetAttribute((const void *)conv_slot_kernel<NJ, RLQ>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024 - (int)(SW * 2 * sizeof(double)));
    (void)hipGetLastError();
  });
  const int nxt = (g.ox + 31) / 32, nzt = (g.oz + SZ - 1) / SZ;
  hipLaunchKernelGGL((conv_slot_kernel<NJ, RLQ>), pl.grid, dim3(ST), pl.lds_bytes, s, (const float *)in,
                     (const float *)H, (float *)out, g, ep, nxt, nzt);
  return hipGetLastError();
}

int cu_count() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) {
    (void)hipGetLastError();
    cus = 1;
  }
  return cus;
}

}  // namespace

// The row-slot tile can run this problem (bf16, PSF extents, LDS).
bool slot_fits(const Geom &g, int dtype, int precision) {
  if (dtype != NDC_F32 || precision != NDC_PREC_BF16) return false;
  if (g.kx > SMAX_KX || g.ky > SMAX_KY || g.kz > SMAX_KZ) return false;
  const size_t lds = g.kx <= 16 ? slot_lds_bytes<1>(g.kz, g.ky) : slot_lds_bytes<2>(g.kz, g.ky);
  return lds + SW * 2 * sizeof(double) <= 160 * 1024;
}

// The built-in choice: the form wins where each input row carries much
// matrix work (measured on MI355X, bf16: at 63 x 31 x 31 taps it takes the
// forward of a 128 x 512 x 512 volume from 6.5 to 5.1 ms and the transpose
// from 6.3 to 3.7 ms against the 32x32 Toeplitz tile; it ties at 31 x 15 x 15
// and loses at 15 PSF planes or fewer, and on 2-D problems, where its fixed
// cost per row dominates).  NDC_SLOT=1 / 0 forces it on / off where it fits.
bool slot_preferred(const Geom &g, int dtype, int precision) {
  if (!slot_fits(g, dtype, precision)) return false;
  if (const char *f = getenv("NDC_SLOT")) {
    if (f[0] == '1') return true;
    if (f[0] == '0') return false;
  }
  const int64_t cols = (int64_t)((g.ox + 31) / 32) * ((g.oz + SZ - 1) / SZ);
  return g.kz >= 57 && g.ky >= 25 && g.kx >= 25 && cols >= 128;
}

ConvPlan plan_conv_slot(const Geom &g) {
  ConvPlan pl{};
  pl.variant = 4;
  const int64_t units = (int64_t)((g.ox + 31) / 32) * ((g.oz + SZ - 1) / SZ) * g.oy;
  // one work-group per CU (the LDS holds one), at least 32 rows each
  const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(cu_count(), units / 32));
  pl.grid = dim3((unsigned)grid);
  pl.block = dim3(ST);
  pl.lds_bytes = g.kx <= 16 ? slot_lds_bytes<1>(g.kz, g.ky) : slot_lds_bytes<2>(g.kz, g.ky);
  pl.nblocks = grid;
  return pl;
}

hipError_t launch_conv_slot(const ConvPlan &pl, const Geom &g, const void *in, const void *H, void *out,
                            const Epi &ep, hipStream_t s) {
  const bool rlq = ep.mode == EPI_RLQ;
  if (g.kx <= 16) return rlq ? launch_slot<1, true>(pl, g, in, H, out, ep, s) : launch_slot<1, false>(pl, g, in, H, out, ep, s);
  return rlq ? launch_slot<2, true>(pl, g, in, H, out, ep, s) : launch_slot<2, false>(pl, g, in, H, out, ep, s);
}

}  // namespace ndc
