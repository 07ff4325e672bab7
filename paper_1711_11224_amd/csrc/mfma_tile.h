#pragma once
// Matrix-core correlation kernels for PSFs wide enough along x that the
// contraction is dense (3 <= kx <= 33, ky <= 33, any kz).
//
// out[s] = sum_t Hc[t] in[s + t - off]  (see Geom), FP32 storage.
//
// FP32: v_mfma_f32_4x4x1f32 (16 independent 4x4 blocks, K = 1).
//   Block b, lanes 4b..4b+3.  D_b[i][j] += A_src[i] * B_b[j], D_b[i][j] in
//   accumulator register i of lane 4b+j.  With CBSZ = 4 the A operand of
//   every block is taken from block ABID, so one VGPR holds A for 16 steps.
// Mapping (a Toeplitz form of one PSF row):
//   lane 4b+j, register i  <->  output (row j, x = x0 + 4b + i)
//   step k in [0, kx+3):  A[i] = Hc_row[k - i] (zero outside [0,kx)),
//                         B[j] = in_row_j[x0 + 4b + k - offx]
//   so sum_k A[i] B[j] = sum_t Hc_row[t] in_row_j[x + t - offx].
//   Only 3 of every kx+3 steps multiply Toeplitz zeros.
// BF16 / split-BF16: v_mfma_f32_4x4x4bf16_1k, the same mapping with four
//   consecutive steps per instruction (A[i][k'] = Hc_row[4c + k' - i],
//   B[k'][j] = in_row_j[x0 + 4b + 4c + k' - offx]).  Operands are rounded to
//   bf16 (nearest even) in registers from the FP32 LDS tiles; split-BF16 adds
//   the hi*lo and lo*hi products of v = hi + lo, lo = bf16(v - hi).
// Work-group: 4 waves, output tile G=4 z-planes x 16 rows x 64 columns;
// wave w owns rows 4w..4w+3 of every plane.  Input planes stream through a
// double-buffered LDS tile; each staged plane feeds the G output planes it
// reaches through G different PSF planes, held in an LDS ring of G+1 planes.
// Partial sums are blocked into FP32 accumulators per input plane (all PSF
// rows of that plane), then added to the output accumulators.

#include <type_traits>

#include "ndc_device.h"
#include "ndc_internal.h"

namespace ndc {
namespace mfma {


typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v4bf __attribute__((ext_vector_type(4)));
typedef short v4s __attribute__((ext_vector_type(4)));

// Compile-time loop: f(integral_constant<int, I>) for I in [B, E).
template <int B, int E, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

constexpr int MT = 256;       // threads per work-group (4 waves)
constexpr int MG_DEFAULT = 4; // output z-planes per work-group (single-volume launches)
constexpr int MROWS = 16;     // output rows per work-group
constexpr int MCOLS = 64;     // output columns per work-group
constexpr int MAX_KY = 33;

// Tile shape: XB of the 16 instruction blocks lie along x (4 columns each),
// the other 16/XB stack along y, so a wave covers 4*16/XB rows x 4*XB columns
// and a work-group (4 waves) 16*16/XB rows x 4*XB columns.
template <int XB>
struct TileDims {
  static constexpr int RG = 16 / XB;      // row groups per instruction
  static constexpr int WR = 4 * RG;       // rows per wave
  static constexpr int ROWS = 4 * WR;     // rows per work-group
  static constexpr int COLS = 4 * XB;     // columns per work-group
};

template <int KX, int XB = 16>
struct MfmaShape {
  static constexpr int KS = KX + 3;               // unit steps per PSF row
  static constexpr int NC = (KS + 15) / 16;       // FP32: broadcast A registers per row
  static_assert(NC <= 4, "A operands of a row are held in one float4 per plane");
  static constexpr int NW = (KS + 3) / 4;         // float4 input windows per lane (= bf16 chunks)
  static constexpr int NCB = (NW + 15) / 16;      // bf16: broadcast A registers per row
  static constexpr int TCOLS = 4 * XB - 4 + 4 * NW;               // staged input columns
  static constexpr int STRIDE = ((TCOLS + 15) / 32) * 32 + 16;    // = 16 mod 32 floats
  static constexpr int HS = 16 * NC + 4;          // LDS PSF row stride (>= 4*NW + 3)
  // bf16 input tiles: row stride in bf16 elements, = 16 mod 64 so the 8-byte
  // window reads of 16 lanes (4 rows x 4 x-blocks) hit distinct bank pairs
  static constexpr int STRIDE_B = ((TCOLS + 47) / 64) * 64 + 16;
  static constexpr int NIN = ((TileDims<XB>::ROWS + MAX_KY - 1) * TCOLS + MT - 1) / MT;
  // floats of LDS one staged input plane takes (planes: 1 FP32, 1 bf16, 2 bf16 hi/lo)
  __host__ __device__ static constexpr int tile_floats(int rows, int prec) {
    return prec == 0 ? rows * STRIDE : ((prec == 2 ? 2 : 1) * rows * STRIDE_B / 2 + 3) / 4 * 4;
  }
  __host__ __device__ static constexpr int lds_floats(int ky, int mg, int prec) {
    return 2 * tile_floats(TileDims<XB>::ROWS + ky - 1, prec) + (mg + 1) * ky * HS + HS;  // + zero row
  }
  static constexpr int NH = (MAX_KY * HS + MT - 1) / MT;
};

__host__ __device__ constexpr int mfma_lds_floats(int ky, int stride, int hs, int mg, int rows = MROWS) {
  return 2 * (rows + ky - 1) * stride + (mg + 1) * ky * hs + hs;  // + zero row
}

__device__ __forceinline__ v4s to_bf16(v4f v) { return __builtin_bit_cast(v4s, __builtin_convertvector(v, v4bf)); }
__device__ __forceinline__ void split_bf16(v4f v, v4s &hi, v4s &lo) {
  const v4bf h = __builtin_convertvector(v, v4bf);
  hi = __builtin_bit_cast(v4s, h);
  lo = to_bf16(v - __builtin_convertvector(h, v4f));
}

// One output tile (G z-planes x 16 rows x 64 columns at tile coordinates
// tx, ty, tz) of the correlation; `slot` is the tile's partial-sum slot.
// All threads of the work-group call it; it leaves LDS free on return.
template <int KX, int PREC, int MG, int XB = 16>
__device__ __forceinline__ void mfma_tile(const float *__restrict__ in, const float *__restrict__ H,
                                          float *__restrict__ out, const Geom &g, const Epi &ep, int tx, int ty,
                                          int tz, int64_t slot, float *lds, double (*red)[2]) {
  using S = MfmaShape<KX, XB>;
  using T = TileDims<XB>;
  const int rows = T::ROWS + g.ky - 1;
  const int tfl = S::tile_floats(rows, PREC);
  float *tile0 = lds;
  float *tile1 = lds + tfl;
  float *ring = lds + 2 * tfl;
  float *zrow = ring + (MG + 1) * g.ky * S::HS;  // HS zeros: A operand of planes out of reach
  const int hplane = g.ky * S::HS;
  const int lo_off = rows * S::STRIDE_B;  // bf16 elements from hi plane to lo plane (split)

  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index, uniform
  const int bb = lane >> 2, jj = lane & 3;  // instruction block, row (B, D) or step offset (A)
  const int xb = bb % XB, rg = bb / XB;       // x-block and row group of this lane's outputs
  const int wrow = w * T::WR + rg * 4 + jj;   // output row within the tile
  const int x0 = tx * T::COLS, y0 = ty * T::ROWS, z0 = tz * MG;

  // input planes that reach this tile, clipped to the input
  const int r_lo = max(0, z0 - g.offz);
  const int r_hi = min(g.iz - 1, z0 + MG - 1 + g.kz - 1 - g.offz);

  // staging helpers ------------------------------------------------------------
  // The staging loads are unconditional, from offsets clamped into the
  // input (and the PSF), with a bit per element for what lies outside; the
  // zeros are applied at the LDS stores, and an empty asm keeps each loaded
  // value's first use there.  A conditional load lets the compiler merge its
  // value right after it, which waits for the load before the plane's
  // matrix instructions instead of after them.
  static_assert(S::NIN <= 32 && S::NH <= 32, "one mask bit per staged element");
  float inreg[S::NIN];
  float hreg[S::NH];
  unsigned inok = 0, hok = 0;
  auto load_plane = [&](int zin) {
    const float *plane = in + (int64_t)zin * g.iy * g.ix;
    inok = 0;
#pragma unroll
    for (int u = 0; u < S::NIN; ++u) {
      const int e = tid + u * MT;
      const int r = e / S::TCOLS, q = e - r * S::TCOLS;
      const int yin = y0 + r - g.offy, xin = x0 + q - g.offx;
      const bool ok = r < rows && yin >= 0 && yin < g.iy && xin >= 0 && xin < g.ix;
      const int yc = min(max(yin, 0), g.iy - 1), xc = min(max(xin, 0), g.ix - 1);
      inreg[u] = plane[(unsigned)(yc * g.ix + xc)];
      inok |= (ok ? 1u : 0u) << u;
    }
  };
  auto store_plane = [&](float *t) {
#pragma unroll
    for (int u = 0; u < S::NIN; ++u) {
      asm volatile("" : "+v"(inreg[u]));  // keep the load's use here
      const int e = tid + u * MT;
      const int r = e / S::TCOLS, q = e - r * S::TCOLS;
      const float v = ((inok >> u) & 1u) ? inreg[u] : 0.f;
      if (r < rows) {
        if constexpr (PREC == PREC_NATIVE_) {
          t[r * S::STRIDE + q] = v;
        } else {  // rounded once here instead of once per PSF row
          __bf16 *tb = (__bf16 *)t;
          const __bf16 hi = (__bf16)v;
          tb[r * S::STRIDE_B + q] = hi;
          if constexpr (PREC == PREC_SPLIT_) tb[lo_off + r * S::STRIDE_B + q] = (__bf16)(v - (float)hi);
        }
      }
    }
  };
  auto load_h = [&](int a) {  // PSF plane a of Hc, rows padded with 3 leading zeros
    const int ha = g.flip ? g.kz - 1 - a : a;
    hok = 0;
#pragma unroll
    for (int u = 0; u < S::NH; ++u) {
      const int e = tid + u * MT;
      const int b = e / S::HS, t = e - b * S::HS - 3;
      const bool ok = b < g.ky && t >= 0 && t < KX;
      const int bc = min(b, g.ky - 1), tcl = min(max(t, 0), KX - 1);
      const int hb = g.flip ? g.ky - 1 - bc : bc;
      const int hc = g.flip ? KX - 1 - tcl : tcl;
      hreg[u] = H[((int64_t)ha * g.ky + hb) * KX + hc];
      hok |= (ok ? 1u : 0u) << u;
    }
  };
  auto store_h = [&](int a) {
    float *dst = ring + (a % (MG + 1)) * hplane;
#pragma unroll
    for (int u = 0; u < S::NH; ++u) {
      asm volatile("" : "+v"(hreg[u]));  // keep the load's use here
      const int e = tid + u * MT;
      if (e < hplane) dst[e] = ((hok >> u) & 1u) ? hreg[u] : 0.f;
    }
  };

  v4f acc[MG];
#pragma unroll
  for (int q = 0; q < MG; ++q) acc[q] = (v4f){0.f, 0.f, 0.f, 0.f};

  if (r_lo <= r_hi) {
    // prologue: first input plane and the PSF planes its step needs
    load_plane(r_lo);
    store_plane(tile0);
    for (int a = max(0, r_lo - z0 - MG + 1 + g.offz); a <= min(g.kz - 1, r_lo - z0 + g.offz); ++a) {
      load_h(a);
      store_h(a);
    }
    for (int e = tid; e < S::HS; e += MT) zrow[e] = 0.f;
    __syncthreads();

    // rows of this wave's outputs that reach the input, as a tap range
    const int b_lo = max(0, g.offy - y0 - w * T::WR - (T::WR - 1));
    const int b_hi = min(g.ky - 1, g.iy - 1 + g.offy - y0 - w * T::WR);
    const bool wave_live = (y0 + w * T::WR < g.oy);

    for (int zin = r_lo; zin <= r_hi; ++zin) {
      const float *tile = ((zin - r_lo) & 1) ? tile1 : tile0;
      const bool more = zin < r_hi;
      const int a_new = zin + 1 - z0 + g.offz;
      const bool new_h = more && a_new >= 0 && a_new < g.kz;
      if (more) load_plane(zin + 1);
      if (new_h) load_h(a_new);

      if (wave_live) {
        int aq[MG];
        bool live[MG];
#pragma unroll
        for (int q = 0; q < MG; ++q) {
          aq[q] = zin - z0 - q + g.offz;
          live[q] = aq[q] >= 0 && aq[q] < g.kz && z0 + q < g.oz;
        }
        {
          if constexpr (PREC == PREC_NATIVE_) {
            // B operand: consecutive inputs of row (wrow + b), column 4*xb + k;
            // A operand: lane 4s+i holds Hc_row[16c + s - i], or 0 from the
            // zero row when output plane q is not reached (no branch).
            const float *hbase[MG];
            int hstep[MG];
#pragma unroll
            for (int q = 0; q < MG; ++q) {
              hbase[q] = (live[q] ? ring + ((aq[q] + MG + 1) % (MG + 1)) * hplane : zrow) + 3 + bb - jj;
              hstep[q] = live[q] ? S::HS : 0;
            }
            const float *src0 = tile + wrow * S::STRIDE + 4 * xb;
            // M: compile-time mask of the output planes whose products are
            // issued (all MG, or on the first and last planes of a tile's z
            // range only the planes the input plane reaches)
            auto fetch = [&](auto mc, int b, v4f(&win)[S::NW], v4f(&hv)[MG]) {
              constexpr unsigned M = decltype(mc)::value;
              static_for<0, MG>([&](auto qc) {
                constexpr int q = decltype(qc)::value;
                if constexpr ((M >> q) & 1u) {
#pragma unroll
                  for (int c = 0; c < S::NC; ++c) hv[q][c] = hbase[q][b * hstep[q] + 16 * c];
                }
              });
#pragma unroll
              for (int u = 0; u < S::KS / 4; ++u) win[u] = *(const v4f *)(src0 + b * S::STRIDE + 4 * u);
              // only the steps that exist: no load into registers left unused
              if constexpr (S::KS % 4 != 0) {
#pragma unroll
                for (int e = 0; e < S::KS % 4; ++e) win[S::NW - 1][e] = src0[b * S::STRIDE + 4 * (S::NW - 1) + e];
              }
            };
            // d: FP32 block sum of this input plane's contribution (all PSF
            // rows), added to the output accumulators once per plane
            v4f d[MG];
#pragma unroll
            for (int q = 0; q < MG; ++q) d[q] = (v4f){0.f, 0.f, 0.f, 0.f};
            auto mm = [&](auto mc, const v4f(&win)[S::NW], const v4f(&hv)[MG]) {
              constexpr unsigned M = decltype(mc)::value;
              static_for<0, S::KS>([&](auto kc) {
                constexpr int k = decltype(kc)::value;
                const float bk = win[k >> 2][k & 3];
                static_for<0, MG>([&](auto qc) {
                  constexpr int q = decltype(qc)::value;
                  if constexpr ((M >> q) & 1u)
                    d[q] = __builtin_amdgcn_mfma_f32_4x4x1f32(hv[q][k >> 4], bk, d[q], 4, k & 15, 0);
                });
              });
            };
            auto rows = [&](auto mc) {
              constexpr unsigned M = decltype(mc)::value;
              constexpr int NQ = __builtin_popcount(M);
              // The next row's LDS reads are spread through this row's matrix
              // instructions (two register sets, rows alternate between them).
              constexpr int NDS = S::NW + NQ * S::NC, NMM = S::KS * NQ;
              auto interleave = [&]() {
                static_for<0, NDS>([&](auto) {
                  __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                  __builtin_amdgcn_sched_group_barrier(0x008, NMM / NDS, 0);
                });
                __builtin_amdgcn_sched_group_barrier(0x008, NMM, 0);
              };
              if constexpr (XB != 8) {
                // one register set (the 16-block-wide tile has no registers
                // for two): the row's reads are issued ahead of its matrix
                // instructions
                for (int b = b_lo; b <= b_hi; ++b) {
                  v4f win[S::NW], hv[MG];
                  fetch(mc, b, win, hv);
                  mm(mc, win, hv);
                  __builtin_amdgcn_sched_group_barrier(0x100, NDS, 0);
                  __builtin_amdgcn_sched_group_barrier(0x008, NMM, 0);
                }
              } else if (b_lo <= b_hi) {
                v4f w0[S::NW], w1[S::NW];
                v4f h0[MG], h1[MG];  // A operands of one row: [q][c] (NC <= 4)
                fetch(mc, b_lo, w0, h0);
                for (int b = b_lo;; b += 2) {
                  fetch(mc, min(b + 1, b_hi), w1, h1);  // past the end: row b_hi again, unused
                  mm(mc, w0, h0);
                  interleave();
                  if (b + 1 > b_hi) break;
                  fetch(mc, min(b + 2, b_hi), w0, h0);
                  mm(mc, w1, h1);
                  interleave();
                  if (b + 2 > b_hi) break;
                }
              }
            };
            // The first and last MG - 1 input planes of a tile's z range reach
            // only some of its output planes: those (a contiguous run from the
            // first or to the last plane) issue only their own products.  Any
            // other mask runs every plane, the unreached ones against the zero
            // row.
            constexpr unsigned FULL = (1u << MG) - 1u;
            unsigned mask = 0;
#pragma unroll
            for (int q = 0; q < MG; ++q) mask |= (live[q] ? 1u : 0u) << q;
            if constexpr (XB == 8 && MG == 4) {
              switch (mask) {
                case 0x1: rows(std::integral_constant<unsigned, 0x1>{}); break;
                case 0x3: rows(std::integral_constant<unsigned, 0x3>{}); break;
                case 0x7: rows(std::integral_constant<unsigned, 0x7>{}); break;
                case 0x8: rows(std::integral_constant<unsigned, 0x8>{}); break;
                case 0xC: rows(std::integral_constant<unsigned, 0xC>{}); break;
                case 0xE: rows(std::integral_constant<unsigned, 0xE>{}); break;
                default: rows(std::integral_constant<unsigned, FULL>{}); break;
              }
            } else {
              rows(std::integral_constant<unsigned, FULL>{});
            }
#pragma unroll
            for (int q = 0; q < MG; ++q) acc[q] += d[q];
          } else {
            static_assert(S::NCB == 1, "bf16 A operands: one broadcast register per row");
            constexpr bool SPLIT = PREC == PREC_SPLIT_;
            constexpr int NL = SPLIT ? S::NW : 1;
            // A operand: lane 4s+i holds Hc_row[4s + k' - i], k' = 0..3 (chunk s;
            // chunks past the last are never broadcast, those lanes load the
            // last one); the zero row when output plane q is not reached
            const int ca = 4 * min(bb, S::NW - 1) + 3 - jj;
            const float *hb[MG];
            int hst[MG];
#pragma unroll
            for (int q = 0; q < MG; ++q) {
              hb[q] = (live[q] ? ring + ((aq[q] + MG + 1) % (MG + 1)) * hplane : zrow) + ca;
              hst[q] = live[q] ? S::HS : 0;
            }
            const short *srcb0 = (const short *)tile + wrow * S::STRIDE_B + 4 * xb;
            auto fetch = [&](int b, v4s(&bh)[S::NW], v4s(&bl)[NL], v4f(&av)[MG]) {
#pragma unroll
              for (int q = 0; q < MG; ++q) {
                const float *p4 = hb[q] + b * hst[q];
                av[q] = (v4f){p4[0], p4[1], p4[2], p4[3]};
              }
#pragma unroll
              for (int c = 0; c < S::NW; ++c) bh[c] = *(const v4s *)(srcb0 + b * S::STRIDE_B + 4 * c);
              if constexpr (SPLIT) {
#pragma unroll
                for (int c = 0; c < S::NW; ++c) bl[c] = *(const v4s *)(srcb0 + lo_off + b * S::STRIDE_B + 4 * c);
              }
            };
            // d: FP32 block sum of this input plane (all PSF rows)
            v4f d[MG];
#pragma unroll
            for (int q = 0; q < MG; ++q) d[q] = (v4f){0.f, 0.f, 0.f, 0.f};
            auto mm = [&](const v4s(&bh)[S::NW], const v4s(&bl)[NL], const v4f(&av)[MG]) {
              v4s ahi[MG], alo[MG];
#pragma unroll
              for (int q = 0; q < MG; ++q) {
                if constexpr (SPLIT)
                  split_bf16(av[q], ahi[q], alo[q]);
                else
                  ahi[q] = to_bf16(av[q]);
              }
              static_for<0, S::NW>([&](auto cc) {
                constexpr int c = decltype(cc)::value;
                static_for<0, MG>([&](auto qc) {
                  constexpr int q = decltype(qc)::value;
                  if constexpr (SPLIT) {
                    v4f t = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(alo[q], bh[c], d[q], 4, c, 0);
                    t = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(ahi[q], bl[c], t, 4, c, 0);
                    d[q] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(ahi[q], bh[c], t, 4, c, 0);
                  } else {
                    d[q] = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(ahi[q], bh[c], d[q], 4, c, 0);
                  }
                });
              });
            };
            constexpr int NDS = 4 * MG + S::NW * (SPLIT ? 2 : 1), NMM = S::NW * MG * (SPLIT ? 3 : 1);
            if constexpr (XB != 8 || SPLIT) {
              // one register set (split-bf16 has three times the instructions
              // per row to cover the reads): reads issued ahead of the row
              for (int b = b_lo; b <= b_hi; ++b) {
                v4s bh[S::NW], bl[NL];
                v4f av[MG];
                fetch(b, bh, bl, av);
                mm(bh, bl, av);
                __builtin_amdgcn_sched_group_barrier(0x100, NDS, 0);
                __builtin_amdgcn_sched_group_barrier(0x002, 8 * MG, 0);
                __builtin_amdgcn_sched_group_barrier(0x008, NMM, 0);
              }
            } else if (b_lo <= b_hi) {
              // the next row's LDS reads are spread through this row's
              // matrix instructions (two register sets)
              auto interleave = [&]() {
                __builtin_amdgcn_sched_group_barrier(0x002, 8 * MG, 0);
                static_for<0, NDS>([&](auto) {
                  __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
                  __builtin_amdgcn_sched_group_barrier(0x008, (NMM + NDS - 1) / NDS, 0);
                });
                __builtin_amdgcn_sched_group_barrier(0x008, NMM, 0);
              };
              v4s bh0[S::NW], bl0[NL], bh1[S::NW], bl1[NL];
              v4f av0[MG], av1[MG];
              fetch(b_lo, bh0, bl0, av0);
              for (int b = b_lo;; b += 2) {
                fetch(min(b + 1, b_hi), bh1, bl1, av1);  // past the end: row b_hi again, unused
                mm(bh0, bl0, av0);
                interleave();
                if (b + 1 > b_hi) break;
                fetch(min(b + 2, b_hi), bh0, bl0, av0);
                mm(bh1, bl1, av1);
                interleave();
                if (b + 2 > b_hi) break;
              }
            }
#pragma unroll
            for (int q = 0; q < MG; ++q) acc[q] += d[q];
          }
        }
      }

      // The next plane's stores stay after this plane's matrix instructions:
      // they target the other buffer, so the compiler may otherwise move them
      // up to the loads and wait for the loads there.
      asm volatile("" ::: "memory");
      if (more) store_plane(((zin + 1 - r_lo) & 1) ? tile1 : tile0);
      if (new_h) store_h(a_new);
      __syncthreads();
    }
  }

  // Epilogue: lane (bb, jj) holds x = x0 + 4xb + i, row y0 + wrow -------------
  double s0 = 0.0, s1 = 0.0;
  const int y = y0 + wrow;
  if (y < g.oy) {
#pragma unroll
    for (int q = 0; q < MG; ++q) {
      const int z = z0 + q;
      if (z < g.oz) {
        const int64_t rowbase = ((int64_t)z * g.oy + y) * g.ox;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int x = x0 + 4 * xb + i;
          if (x < g.ox) apply_epilogue<float>(out, rowbase + x, acc[q][i], ep, s0, s1);
        }
      }
    }
  }
  if (ep.mode != EPI_STORE) {
    block_sum2(s0, s1, red);
    if (tid == 0) {
      ep.part[2 * slot] = s0;
      ep.part[2 * slot + 1] = s1;
    }
  }
}


// Run-time PSF width variant of mfma_tile (FP32 only, 3 <= kx <= 33), for the
// batched launch where one kernel serves volumes with different PSFs.  Steps
// are processed in groups of 16 (one broadcast A register) made of four
// 4-step chunks (one float4 input window); the ABID of each instruction is
// 4*chunk + step, a compile-time constant, so only the group loop and the
// chunk count are run-time.  Padding costs at most 3 steps per PSF row.
constexpr int RT_MAX_KX = 33;
constexpr int RT_TCOLS_MAX = 60 + 4 * ((RT_MAX_KX + 3 + 3) / 4);
constexpr int RT_NIN = ((MROWS + MAX_KY - 1) * RT_TCOLS_MAX + MT - 1) / MT;
constexpr int RT_NH = (MAX_KY * (16 * ((RT_MAX_KX + 3 + 15) / 16) + 4) + MT - 1) / MT;

struct RtShape {
  int ks, nw, nc, tcols, stride, hs;
  __host__ __device__ explicit RtShape(int kx) {
    ks = kx + 3;
    nw = (ks + 3) / 4;
    nc = (ks + 15) / 16;
    tcols = 60 + 4 * nw;
    stride = ((tcols + 15) / 32) * 32 + 16;
    hs = 16 * nc + 4;
  }
};

template <int MG>
__device__ __forceinline__ void mfma_tile_rt(const float *__restrict__ in, const float *__restrict__ H,
                                             float *__restrict__ out, const Geom &g, const Epi &ep, int tx, int ty,
                                             int tz, int64_t slot, float *lds, double (*red)[2]) {
  const RtShape S(g.kx);
  const int rows = MROWS + g.ky - 1;
  float *tile0 = lds;
  float *tile1 = lds + rows * S.stride;
  float *ring = lds + 2 * rows * S.stride;
  float *zrow = ring + (MG + 1) * g.ky * S.hs;  // hs zeros: A operand of planes out of reach
  const int hplane = g.ky * S.hs;

  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int bb = lane >> 2, jj = lane & 3;
  const int x0 = tx * MCOLS, y0 = ty * MROWS, z0 = tz * MG;
  const int r_lo = max(0, z0 - g.offz);
  const int r_hi = min(g.iz - 1, z0 + MG - 1 + g.kz - 1 - g.offz);

  float inreg[RT_NIN];
  float hreg[RT_NH];
  // Unconditional staging loads with a mask, as in mfma_tile.
  static_assert(RT_NIN <= 32 && RT_NH <= 32, "one mask bit per staged element");
  unsigned inok = 0, hok = 0;
  auto load_plane = [&](int zin) {
    const float *plane = in + (int64_t)zin * g.iy * g.ix;
    inok = 0;
#pragma unroll
    for (int u = 0; u < RT_NIN; ++u) {
      const int e = tid + u * MT;
      const int r = e / S.tcols, q = e - r * S.tcols;
      const int yin = y0 + r - g.offy, xin = x0 + q - g.offx;
      const bool ok = r < rows && yin >= 0 && yin < g.iy && xin >= 0 && xin < g.ix;
      const int yc = min(max(yin, 0), g.iy - 1), xc = min(max(xin, 0), g.ix - 1);
      inreg[u] = plane[(unsigned)(yc * g.ix + xc)];
      inok |= (ok ? 1u : 0u) << u;
    }
  };
  auto store_plane = [&](float *t) {
#pragma unroll
    for (int u = 0; u < RT_NIN; ++u) {
      asm volatile("" : "+v"(inreg[u]));  // keep the load's use here
      const int e = tid + u * MT;
      const int r = e / S.tcols, q = e - r * S.tcols;
      if (r < rows) t[r * S.stride + q] = ((inok >> u) & 1u) ? inreg[u] : 0.f;
    }
  };
  auto load_h = [&](int a) {
    const int ha = g.flip ? g.kz - 1 - a : a;
    hok = 0;
#pragma unroll
    for (int u = 0; u < RT_NH; ++u) {
      const int e = tid + u * MT;
      const int b = e / S.hs, t = e - b * S.hs - 3;
      const bool ok = b < g.ky && t >= 0 && t < g.kx;
      const int bc = min(b, g.ky - 1), tcl = min(max(t, 0), g.kx - 1);
      const int hb = g.flip ? g.ky - 1 - bc : bc;
      const int hc = g.flip ? g.kx - 1 - tcl : tcl;
      hreg[u] = H[((int64_t)ha * g.ky + hb) * g.kx + hc];
      hok |= (ok ? 1u : 0u) << u;
    }
  };
  auto store_h = [&](int a) {
    float *dst = ring + (a % (MG + 1)) * hplane;
#pragma unroll
    for (int u = 0; u < RT_NH; ++u) {
      asm volatile("" : "+v"(hreg[u]));  // keep the load's use here
      const int e = tid + u * MT;
      if (e < hplane) dst[e] = ((hok >> u) & 1u) ? hreg[u] : 0.f;
    }
  };

  v4f acc[MG];
#pragma unroll
  for (int q = 0; q < MG; ++q) acc[q] = (v4f){0.f, 0.f, 0.f, 0.f};

  if (r_lo <= r_hi) {
    load_plane(r_lo);
    store_plane(tile0);
    for (int a = max(0, r_lo - z0 - MG + 1 + g.offz); a <= min(g.kz - 1, r_lo - z0 + g.offz); ++a) {
      load_h(a);
      store_h(a);
    }
    for (int e = tid; e < S.hs; e += MT) zrow[e] = 0.f;
    __syncthreads();
    const int b_lo = max(0, g.offy - y0 - 4 * w - 3);
    const int b_hi = min(g.ky - 1, g.iy - 1 + g.offy - y0 - 4 * w);
    const bool wave_live = (y0 + 4 * w < g.oy);

    for (int zin = r_lo; zin <= r_hi; ++zin) {
      const float *tile = ((zin - r_lo) & 1) ? tile1 : tile0;
      const bool more = zin < r_hi;
      const int a_new = zin + 1 - z0 + g.offz;
      const bool new_h = more && a_new >= 0 && a_new < g.kz;
      if (more) load_plane(zin + 1);
      if (new_h) load_h(a_new);

      if (wave_live) {
        // A operand rows of plane q, or the zero row when q is not reached
        const float *hbase[MG];
        int hstep[MG];
#pragma unroll
        for (int q = 0; q < MG; ++q) {
          const int aq = zin - z0 - q + g.offz;
          const bool live = aq >= 0 && aq < g.kz && z0 + q < g.oz;
          hbase[q] = (live ? ring + ((aq + MG + 1) % (MG + 1)) * hplane : zrow) + 3 + bb - jj;
          hstep[q] = live ? S.hs : 0;
        }
        // d: FP32 block sum of this input plane (all PSF rows)
        v4f d[MG];
#pragma unroll
        for (int q = 0; q < MG; ++q) d[q] = (v4f){0.f, 0.f, 0.f, 0.f};
        for (int b = b_lo; b <= b_hi; ++b) {
          const float *src = tile + (4 * w + jj + b) * S.stride + 4 * bb;
          for (int gi = 0; gi < S.nc; ++gi) {
            float hv[MG];
#pragma unroll
            for (int q = 0; q < MG; ++q) hv[q] = hbase[q][b * hstep[q] + 16 * gi];
            static_for<0, 4>([&](auto sc) {
              constexpr int sub = decltype(sc)::value;
              if (4 * gi + sub < S.nw) {
                const v4f win = *(const v4f *)(src + 16 * gi + 4 * sub);
                static_for<0, 4>([&](auto uc) {
                  constexpr int u = decltype(uc)::value;
                  static_for<0, MG>([&](auto qc) {
                    constexpr int q = decltype(qc)::value;
                    d[q] = __builtin_amdgcn_mfma_f32_4x4x1f32(hv[q], win[u], d[q], 4, 4 * sub + u, 0);
                  });
                });
              }
            });
          }
        }
#pragma unroll
        for (int q = 0; q < MG; ++q) acc[q] += d[q];
      }
      asm volatile("" ::: "memory");  // the stores stay after the matrix instructions
      if (more) store_plane(((zin + 1 - r_lo) & 1) ? tile1 : tile0);
      if (new_h) store_h(a_new);
      __syncthreads();
    }
  }

  double s0 = 0.0, s1 = 0.0;
  const int y = y0 + 4 * w + jj;
  if (y < g.oy) {
#pragma unroll
    for (int q = 0; q < MG; ++q) {
      const int z = z0 + q;
      if (z < g.oz) {
        const int64_t rowbase = ((int64_t)z * g.oy + y) * g.ox;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int x = x0 + 4 * bb + i;
          if (x < g.ox) apply_epilogue<float>(out, rowbase + x, acc[q][i], ep, s0, s1);
        }
      }
    }
  }
  if (ep.mode != EPI_STORE) {
    block_sum2(s0, s1, red);
    if (tid == 0) {
      ep.part[2 * slot] = s0;
      ep.part[2 * slot + 1] = s1;
    }
  }
}

}  // namespace mfma
}  // namespace ndc
