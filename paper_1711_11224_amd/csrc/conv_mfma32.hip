// bf16 and split-bf16 correlation on the 32x32x16 matrix instruction, for
// PSFs with 11 <= kx <= 33 and ky <= 33 (FP32 storage, FP32 accumulation).
//
// out[s] = sum_t Hc[t] in[s + t - off]  (see Geom).
//
// v_mfma_f32_32x32x16_bf16: D[32x32] += A[32x16] B[16x32].  Lane l holds
//   A[m = l % 32][k = 8 (l / 32) + e] and B[k = 8 (l / 32) + e][n = l % 32]
//   for e = 0..7, and D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32] in
//   accumulator register r.
// Mapping (a Toeplitz form of one PSF row along x):
//   m = output column x0 + m, n = output row, k = input column;
//   chunk j covers input columns x0 - offx + 16 j + k, and
//   A_j[m][k] = Hc_row[16 j + k - m] (zero outside [0, kx)),
//   B_j[k][n] = in_row(n + b)[x0 - offx + 16 j + k],
//   so sum_j sum_k A_j B_j = sum_c Hc_row[c] in_row[x0 + m + c - offx].
//   NJ = ceil((kx + 31) / 16) chunks per row: kx of every 16 NJ steps are
//   PSF taps, the rest Toeplitz zeros (48% of the steps are taps at kx = 31,
//   against 91% for the 4x4 form, at four times its peak rate).
// Split-bf16 adds the lo*hi and hi*lo products of v = hi + lo,
// lo = bf16(v - hi), for both operands.
//
// Work-group: 8 waves; output tile 4 z-planes x 64 rows x 32 NT columns.
// Wave w owns plane w & 3 and rows 32 (w >> 2) .. +31, as NT 32x32
// accumulator blocks side by side along x.  Input chunk s (16 columns) of a
// row serves block t with chunk j = s - 2 t, so a row of the wave reads
// 2 NT + NJ - 1 input chunks for NT NJ instructions.
// One input plane at a time is staged in LDS as bf16 (hi, and lo for the
// split form), rounded once; the next plane is loaded into registers while
// the current one is used.  The PSF planes of the 4 output planes sit in an
// LDS ring of 4 slots.  Each PSF row is stored twice (shifted by one element)
// with zero gaps between rows, so every lane reads its 8 Toeplitz taps with
// 4-byte aligned loads and no branches.

#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "ndc_device.h"
#include "ndc_internal.h"

namespace ndc {

namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));

template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(f);
  }
}

constexpr int WT = 512;       // threads per work-group (8 waves)
constexpr int WPLANES = 4;    // output z-planes per work-group
constexpr int WROWS = 64;     // output rows per work-group
constexpr int WMAX_KY = 33;
constexpr int WMIN_KX = 11;   // narrower PSF rows stay on the 4x4 form
constexpr int WMAX_KX = 33;
constexpr int WHP = 64;       // bf16 pitch of a PSF row in the ring (>= kx + 31, >= 16 NJ)
constexpr int WMAX_KXY = WMAX_KX * WMAX_KY;
constexpr int WNH = (WMAX_KXY + WT - 1) / WT;

template <int NT>
struct WShape {
  static constexpr int COLS = 32 * NT;                         // output columns per work-group
  static constexpr int TCOLS = COLS + 32;                      // staged input columns
  static constexpr int STRIDE = ((TCOLS + 15) / 16) * 16 + 8;  // bf16; odd multiple of 8: ds_read_b128
                                                               // of 16 rows hits 16 distinct bank quads
  static constexpr int NPAIR = ((WROWS + WMAX_KY - 1) * TCOLS / 2 + WT - 1) / WT;  // column pairs per thread
};

// bf16 elements of one copy of a PSF plane in the ring: a leading gap of 32,
// rows at 32 + 64 b, and a trailing gap; = 64 mod 128 so that the two copies
// of a row start 32 banks apart.
__host__ __device__ inline int ring_plane_elems(int ky) { return 128 * ((ky + 2) / 2) + 64; }

template <int NT>
__host__ __device__ inline size_t w_lds_bytes(int ky, int split) {
  using S = WShape<NT>;
  const size_t tile = (size_t)(WROWS + ky - 1) * S::STRIDE * (split ? 2 : 1);
  const size_t ring = (size_t)4 * (split ? 4 : 2) * ring_plane_elems(ky);
  return 2 * (tile + ring);
}

__device__ __forceinline__ unsigned pack_bf16(float a, float b) {
  const unsigned short ua = __builtin_bit_cast(unsigned short, (__bf16)a);
  const unsigned short ub = __builtin_bit_cast(unsigned short, (__bf16)b);
  return (unsigned)ua | ((unsigned)ub << 16);
}

__device__ __forceinline__ float bf16_hi(float v) { return (float)(__bf16)v; }

template <int NJ, int NT, int PREC>
__global__ __launch_bounds__(WT, 1) void conv_mfma32_kernel(const float *__restrict__ in,
                                                            const float *__restrict__ H, float *__restrict__ out,
                                                            Geom g, Epi ep, int nbx, int nby) {
  if (ep.phase && !((1 << *ep.phase) & ep.phase_mask)) return;  // uniform early exit
  constexpr bool SPLIT = PREC == PREC_SPLIT_;
  constexpr int NCOPY = SPLIT ? 4 : 2;  // ring copies per plane: hi even/odd (+ lo even/odd)
  constexpr int NS = 2 * (NT - 1) + NJ;  // input chunks per row of a wave
  using S = WShape<NT>;
  extern __shared__ __align__(16) unsigned short ldsb[];
  __shared__ double red[WT / 64][2];

  const int id = blockIdx.x;
  const int tx = id % nbx, ty = (id / nbx) % nby, tz = id / (nbx * nby);
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int q = w & 3, hh = w >> 2;      // output plane, row half
  const int n = lane & 31, gg = lane >> 5;
  const int x0 = tx * S::COLS, y0 = ty * WROWS, z0 = tz * WPLANES;
  const int rows = WROWS + g.ky - 1;
  const int tplane = rows * S::STRIDE;   // bf16 elements of one staged plane
  const int pe = ring_plane_elems(g.ky);
  unsigned short *tile = ldsb;
  unsigned short *ring = ldsb + (SPLIT ? 2 : 1) * tplane;

  // input planes that reach the tile, clipped to the input
  const int r_lo = max(0, z0 - g.offz);
  const int r_hi = min(g.iz - 1, z0 + WPLANES - 1 + g.kz - 1 - g.offz);

  // Staging: thread pair u covers tile row r, columns c, c+1 (c even).  x0,
  // offx and c are even, so a pair is inside the input, has only its first
  // column inside (odd ix) or none.  Offsets within a plane and a validity
  // mask are set once; loads read in-bounds addresses only and the values
  // outside the input are zeroed at staging, so no load is waited for early.
  constexpr int HALF = S::TCOLS / 2;
  unsigned goff[S::NPAIR];
  uint32_t gval = 0;  // bit 2u: first column valid, bit 2u + 1: second
#pragma unroll
  for (int u = 0; u < S::NPAIR; ++u) {
    const int e = tid + u * WT;
    const int r = e / HALF, c = 2 * (e - r * HALF);
    const int yin = y0 + r - g.offy, xin = x0 + c - g.offx;
    const bool v0 = r < rows && yin >= 0 && yin < g.iy && xin >= 0 && xin < g.ix;
    const bool v1 = v0 && xin + 1 < g.ix;
    goff[u] = v0 ? (unsigned)(yin * g.ix + xin) : 0u;
    gval |= (v0 ? 1u : 0u) << (2 * u);
    gval |= (v1 ? 1u : 0u) << (2 * u + 1);
  }
  float inreg[2 * S::NPAIR];
  auto load_plane = [&](int zin) {
    const float *plane = in + (int64_t)zin * g.iy * g.ix;
#pragma unroll
    for (int u = 0; u < S::NPAIR; ++u) {
      inreg[2 * u] = plane[goff[u]];
      inreg[2 * u + 1] = plane[goff[u] + ((gval >> (2 * u + 1)) & 1u)];
    }
  };
  auto store_plane = [&]() {
#pragma unroll
    for (int u = 0; u < S::NPAIR; ++u) {
      const int e = tid + u * WT;
      if (e < rows * HALF) {
        const int r = e / HALF, c = 2 * (e - r * HALF);
        const float v0 = ((gval >> (2 * u)) & 1u) ? inreg[2 * u] : 0.f;
        const float v1 = ((gval >> (2 * u + 1)) & 1u) ? inreg[2 * u + 1] : 0.f;
        *(unsigned *)(tile + r * S::STRIDE + c) = pack_bf16(v0, v1);
        if constexpr (SPLIT) *(unsigned *)(tile + tplane + r * S::STRIDE + c) = pack_bf16(v0 - bf16_hi(v0), v1 - bf16_hi(v1));
      }
    }
  };
  float hreg[WNH];
  auto load_h = [&](int a) {  // PSF plane a of Hc
#pragma unroll
    for (int u = 0; u < WNH; ++u) {
      const int e = tid + u * WT;
      const int b = e / g.kx, c = e - b * g.kx;
      float v = 0.f;
      if (b < g.ky) {
        const int ha = g.flip ? g.kz - 1 - a : a;
        const int hb = g.flip ? g.ky - 1 - b : b;
        const int hc = g.flip ? g.kx - 1 - c : c;
        v = H[((int64_t)ha * g.ky + hb) * g.kx + hc];
      }
      hreg[u] = v;
    }
  };
  auto store_h = [&](int a) {  // data positions only; the gaps stay zero
    unsigned short *slot = ring + (a & 3) * NCOPY * pe;
#pragma unroll
    for (int u = 0; u < WNH; ++u) {
      const int e = tid + u * WT;
      const int b = e / g.kx, c = e - b * g.kx;
      if (b < g.ky) {
        const float v = hreg[u];
        const __bf16 hi = (__bf16)v;
        const unsigned short uh = __builtin_bit_cast(unsigned short, hi);
        slot[32 + WHP * b + c] = uh;
        slot[pe + 33 + WHP * b + c] = uh;
        if constexpr (SPLIT) {
          const unsigned short ul = __builtin_bit_cast(unsigned short, (__bf16)(v - (float)hi));
          slot[2 * pe + 32 + WHP * b + c] = ul;
          slot[3 * pe + 33 + WHP * b + c] = ul;
        }
      }
    }
  };

  v16f acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = (v16f){};

  const bool wave_live = y0 + 32 * hh < g.oy && z0 + q < g.oz;
  // PSF rows whose input rows reach this wave's outputs
  const int b_lo = max(0, g.offy - y0 - 32 * hh - 31);
  const int b_hi = min(g.ky - 1, g.iy - 1 + g.offy - y0 - 32 * hh);
  // A operand: lane (m = n, gg) reads taps 16 j + 8 gg - m .. +7 of a row,
  // from the copy shifted by m & 1, so the read is 4-byte aligned
  const int a_off = (n & 1) * pe + 32 + (n & 1) + 8 * gg - n;
  // B operand: row n + b of the wave's rows, columns 16 s + 8 gg .. +7
  const int b_off = (32 * hh + n) * S::STRIDE + 8 * gg;

  if (r_lo <= r_hi) {
    // prologue: zero the ring, then stage the first plane and its PSF planes
    {
      unsigned *r32 = (unsigned *)ring;
      const int nwords = 4 * NCOPY * pe / 2;
      for (int e = tid; e < nwords; e += WT) r32[e] = 0u;
    }
    load_plane(r_lo);
    __syncthreads();
    store_plane();
    for (int a = max(0, r_lo - z0 - WPLANES + 1 + g.offz); a <= min(g.kz - 1, r_lo - z0 + g.offz); ++a) {
      load_h(a);
      store_h(a);
    }
    __syncthreads();

    for (int zin = r_lo; zin <= r_hi; ++zin) {
      const bool more = zin < r_hi;
      const int a_new = zin + 1 - z0 + g.offz;
      const bool new_h = more && a_new >= 0 && a_new < g.kz;
      if (more) load_plane(zin + 1);
      if (new_h) load_h(a_new);

      const int aq = zin - z0 - q + g.offz;
      if (wave_live && aq >= 0 && aq < g.kz) {
        const unsigned short *ha = ring + (aq & 3) * NCOPY * pe + a_off;
        const unsigned short *bs = tile + b_off;
        // operands of one PSF row: NJ Toeplitz chunks of the row, NS input
        // chunks (and their lo halves in the split form)
        constexpr int NJL = SPLIT ? NJ : 1, NSL = SPLIT ? NS : 1;
        struct Ops {
          v8bf ah[NJ], al[NJL], bh[NS], bl[NSL];
        };
        auto fetch = [&](int b, Ops &o) {
#pragma unroll
          for (int j = 0; j < NJ; ++j) {
            const unsigned *p = (const unsigned *)(ha + WHP * b + 16 * j);
            o.ah[j] = __builtin_bit_cast(v8bf, (v4u){p[0], p[1], p[2], p[3]});
            if constexpr (SPLIT) {
              const unsigned *pl = (const unsigned *)(ha + 2 * pe + WHP * b + 16 * j);
              o.al[j] = __builtin_bit_cast(v8bf, (v4u){pl[0], pl[1], pl[2], pl[3]});
            }
          }
          const unsigned short *brow = bs + b * S::STRIDE;
#pragma unroll
          for (int c = 0; c < NS; ++c) {
            o.bh[c] = __builtin_bit_cast(v8bf, *(const v4u *)(brow + 16 * c));
            if constexpr (SPLIT) o.bl[c] = __builtin_bit_cast(v8bf, *(const v4u *)(brow + tplane + 16 * c));
          }
        };
        // chunk-major order: consecutive instructions accumulate into
        // different blocks, so none waits for the one before it
        auto mm = [&](const Ops &o) {
          sfor<0, NJ>([&](auto jc) {
            constexpr int j = decltype(jc)::value;
            if constexpr (SPLIT) {
              sfor<0, NT>([&](auto tc) {
                constexpr int t = decltype(tc)::value;
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.al[j], o.bh[2 * t + j], acc[t], 0, 0, 0);
              });
              sfor<0, NT>([&](auto tc) {
                constexpr int t = decltype(tc)::value;
                acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.ah[j], o.bl[2 * t + j], acc[t], 0, 0, 0);
              });
            }
            sfor<0, NT>([&](auto tc) {
              constexpr int t = decltype(tc)::value;
              acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o.ah[j], o.bh[2 * t + j], acc[t], 0, 0, 0);
            });
          });
        };
        constexpr int NDS = (2 * NJ + NS) * (SPLIT ? 2 : 1);  // LDS read instructions per row
        constexpr int NMM = NJ * NT * (SPLIT ? 3 : 1);        // matrix instructions per row
        if constexpr (SPLIT) {
          // one register set: a row's reads are issued ahead of its
          // instructions (three products per pair of operands cover them)
          for (int b = b_lo; b <= b_hi; ++b) {
            Ops o;
            fetch(b, o);
            mm(o);
            __builtin_amdgcn_sched_group_barrier(0x100, NDS, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, NMM, 0);
          }
        } else if (b_lo <= b_hi) {
          // two register sets: the next row's reads are spread through this
          // row's instructions
          auto interleave = [&]() {
            sfor<0, NDS>([&](auto ic) {
              __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
              if constexpr (decltype(ic)::value < NMM) __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            });
            if constexpr (NMM > NDS) __builtin_amdgcn_sched_group_barrier(0x008, NMM - NDS, 0);
          };
          Ops o0, o1;
          fetch(b_lo, o0);
          for (int b = b_lo;; b += 2) {
            fetch(min(b + 1, b_hi), o1);  // past the end: row b_hi again, unused
            mm(o0);
            interleave();
            if (b + 1 > b_hi) break;
            fetch(min(b + 2, b_hi), o0);
            mm(o1);
            interleave();
            if (b + 2 > b_hi) break;
          }
        }
      }

      if (more) {
        __syncthreads();  // every wave is done with this plane and the oldest PSF slot
        store_plane();
        if (new_h) store_h(a_new);
        __syncthreads();
      }
    }
  }

  // Epilogue: register r of lane (n, gg) in block t holds
  // x = x0 + 32 t + 8 (r / 4) + 4 gg + r % 4, row y0 + 32 hh + n.
  double s0 = 0.0, s1 = 0.0;
  const int z = z0 + q, y = y0 + 32 * hh + n;
  if (z < g.oz && y < g.oy) {
    const int64_t rowbase = ((int64_t)z * g.oy + y) * g.ox;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int x = x0 + 32 * t + 8 * (r / 4) + 4 * gg + (r % 4);
        if (x < g.ox) apply_epilogue<float>(out, rowbase + x, acc[t][r], ep, s0, s1);
      }
  }
  if (ep.mode != EPI_STORE) {
    block_sum2(s0, s1, red);
    if (tid == 0) {
      ep.part[2 * (int64_t)id] = s0;
      ep.part[2 * (int64_t)id + 1] = s1;
    }
  }
}

dim3 w_tiles(const Geom &g, int nt) {
  return dim3((g.ox + 32 * nt - 1) / (32 * nt), (g.oy + WROWS - 1) / WROWS, (g.oz + WPLANES - 1) / WPLANES);
}

// x blocks per wave: the fewest padded output columns; on a tie the wider
// tile when it still makes two work-groups per CU or more (measured: the
// wider tile reads fewer operand bytes per instruction, but with fewer than
// two rounds of work-groups the narrower one balances the CUs better).  Up
// to 4 blocks for bf16 and 3 for split-bf16: beyond that the two operand
// register sets (bf16) or the hi and lo operands (split) no longer fit; at
// those widths the compiler spills 10-15 staging registers, which costs less
// than the narrower tile (checked by timing).
constexpr int max_nt(int precision) { return precision == NDC_PREC_SPLIT_BF16 ? 3 : 4; }

int choose_nt(const Geom &g, int precision) {
  int best = 0;
  int64_t best_cols = 0;
  for (int nt = 2; nt <= max_nt(precision); ++nt) {
    const int64_t cols = (int64_t)((g.ox + 32 * nt - 1) / (32 * nt)) * (32 * nt);
    const dim3 t = w_tiles(g, nt);
    const int64_t wgs = (int64_t)t.x * t.y * t.z;
    if (best == 0 || cols < best_cols || (cols == best_cols && wgs >= 512)) {
      best = nt;
      best_cols = cols;
    }
  }
  return best;
}


template <int NJ, int NT, int PREC>
hipError_t launch_w(const Geom &g, const void *in, const void *H, void *out, const Epi &ep, hipStream_t s) {
  const size_t lds = w_lds_bytes<NT>(g.ky, PREC == PREC_SPLIT_);
  // raise the dynamic-LDS limit once per process; call_once makes
  // concurrent first calls from several host threads safe
  static std::once_flag lds_once;
  std::call_once(lds_once, [] {
    (void)hipFuncSetAttribute((const void *)conv_mfma32_kernel<NJ, NT, PREC>,
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)w_lds_bytes<NT>(WMAX_KY, PREC == PREC_SPLIT_));
    (void)hipGetLastError();
  });
  const dim3 t = w_tiles(g, NT);
  hipLaunchKernelGGL((conv_mfma32_kernel<NJ, NT, PREC>), dim3(t.x * t.y * t.z), dim3(WT), lds, s,
                     (const float *)in, (const float *)H, (float *)out, g, ep, (int)t.x, (int)t.y);
  return hipGetLastError();
}

template <int NJ, int PREC>
hipError_t launch_nj(int nt, const Geom &g, const void *in, const void *H, void *out, const Epi &ep,
                     hipStream_t s) {
  switch (nt) {
    case 2: return launch_w<NJ, 2, PREC>(g, in, H, out, ep, s);
    case 3: return launch_w<NJ, 3, PREC>(g, in, H, out, ep, s);
    default:
      if constexpr (PREC == PREC_SPLIT_) return hipErrorInvalidValue;
      else return launch_w<NJ, 4, PREC>(g, in, H, out, ep, s);
  }
}

template <int PREC>
hipError_t launch_prec32(int nt, const Geom &g, const void *in, const void *H, void *out, const Epi &ep,
                         hipStream_t s) {
  if (g.kx + 31 <= 48) return launch_nj<3, PREC>(nt, g, in, H, out, ep, s);
  return launch_nj<4, PREC>(nt, g, in, H, out, ep, s);
}

}  // namespace

// The 32x32 tile can run this problem (PSF row width, plane size, LDS).
bool mfma32_fits(const Geom &g, int dtype, int precision) {
  if (dtype != NDC_F32 || precision == NDC_PREC_NATIVE) return false;
  if (g.kx < WMIN_KX || g.kx > WMAX_KX || g.ky > WMAX_KY) return false;
  if ((int64_t)g.iy * g.ix >= ((int64_t)1 << 31)) return false;  // 32-bit offsets within a plane
  return w_lds_bytes<3>(g.ky, 1) <= 160 * 1024 && w_lds_bytes<4>(g.ky, 0) <= 160 * 1024;
}

bool mfma32_nt_ok(int nt, int precision) { return nt >= 2 && nt <= max_nt(precision); }

bool mfma32_supported(const Geom &g, int dtype, int precision) {
  if (!mfma32_fits(g, dtype, precision)) return false;
  // NDC_MFMA32=1 / 0 forces this form on / off wherever it is supported
  // (tests and timing); otherwise the volume decides.
  if (const char *f = getenv("NDC_MFMA32")) {
    if (f[0] == '1') return true;
    if (f[0] == '0') return false;
  }
  // The 4 x 64 x 32 NT tile needs a volume that fills the chip: measured
  // on MI355X over 22 shapes, it beats the 4x4 form when (output plane area /
  // padded tile area) x min(1, work-groups / 256) >= 0.5, and loses or ties
  // below.
  const int nt = choose_nt(g, precision);
  const dim3 t = w_tiles(g, nt);
  const double pad = (double)g.ox * g.oy / ((double)t.x * 32 * nt * t.y * WROWS);
  const double fill = std::min(1.0, (double)t.x * t.y * t.z / 256.0);
  return pad * fill >= 0.5;
}

ConvPlan plan_conv_mfma32(const Geom &g, int precision, int nt) {
  ConvPlan pl{};
  pl.variant = 3;
  pl.nt = mfma32_nt_ok(nt, precision) ? nt : choose_nt(g, precision);
  const dim3 t = w_tiles(g, pl.nt);
  pl.grid = dim3(t.x * t.y * t.z);
  pl.block = dim3(WT);
  pl.lds_bytes = 0;
  pl.nblocks = (int64_t)t.x * t.y * t.z;
  return pl;
}

hipError_t launch_conv_mfma32(const ConvPlan &pl, const Geom &g, int precision, const void *in, const void *H,
                              void *out, const Epi &ep, hipStream_t s) {
  if (precision == NDC_PREC_SPLIT_BF16) return launch_prec32<PREC_SPLIT_>(pl.nt, g, in, H, out, ep, s);
  return launch_prec32<PREC_BF16_>(pl.nt, g, in, H, out, ep, s);
}

}  // namespace ndc
