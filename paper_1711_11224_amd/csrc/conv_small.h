// Streaming correlation kernel for small PSFs (every axis <= 7 taps), where
// the operators are bound by HBM rather than by arithmetic.
//
// out[s] = sum_t Hc[t] in[s + t - off]  (see Geom), FP32 or FP64.
//
// A work-group owns a 16-row x 64-column column of the output and walks it
// along z, reading every input plane of its column from HBM once:
//   * the next input plane is in flight into registers while the current one
//     (double-buffered in LDS, one barrier per plane) is consumed;
//   * each thread keeps 4 consecutive x outputs of one row; for every tap row
//     b it loads a (4 + kx - 1)-wide window once and applies it to all kz
//     output planes the input plane reaches (kz x kx x 4 FMAs per window);
//   * the kz output planes in flight are register accumulators: the z walk
//     is unrolled kz times with its phase fixed so that output plane z always
//     lands in accumulator z mod kz, a compile-time index.  A plane is
//     finished (fused epilogue) when its last input plane has been added.
// Taps live in LDS (rows padded to 8) and are read as uniform float4.
#pragma once
#include <algorithm>
#include <atomic>
#include <cmath>

#include "ndc_device.h"
#include "ndc_internal.h"

#include <type_traits>

namespace ndc {

// Output planes per work-group (conv_small.hip).
int small_zchunk(const Geom &g, int per_cu);

namespace {

constexpr int ST = 256;          // threads
constexpr int SRX = 4;           // x outputs per thread
constexpr int STX = 16 * SRX;    // 64 output columns
constexpr int STY = ST / 16;     // 16 output rows
constexpr int SMAXK = 7;         // max taps per axis
constexpr int SCOLS = STX + SMAXK - 1;              // staged columns (70)
constexpr int SSTRIDE = (SCOLS + 3) / 4 * 4 + 4;    // 76
constexpr int SROWS = STY + SMAXK - 1;              // 22
constexpr int SPLANE = SROWS * SSTRIDE;
constexpr int SNIN = (SROWS * SCOLS + ST - 1) / ST; // staging registers per thread

template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(f);
  }
}

template <typename T>
__host__ __device__ constexpr size_t small_lds_bytes(int kz) {
  // two input planes, taps (kz*7 rows of 8)
  return sizeof(T) * ((size_t)2 * SPLANE + (size_t)kz * SMAXK * 8);
}

template <typename T, int KX, int KZ>
__global__ __launch_bounds__(ST) void conv_small_kernel(const T *__restrict__ in, const T *__restrict__ H,
                                                        T *__restrict__ out, Geom g, Epi ep, int nbx, int nby,
                                                        int zc) {
  if (ep.phase && !((1 << *ep.phase) & ep.phase_mask)) return;
  extern __shared__ __align__(16) unsigned char small_lds[];
  T *planes = (T *)small_lds;                  // 2 x SPLANE
  T *taps = planes + 2 * SPLANE;               // [a][b][8]
  __shared__ double red[ST / 64][2];

  const int id = blockIdx.x;
  const int tx = id % nbx, ty = (id / nbx) % nby, tz = id / (nbx * nby);
  const int x0 = tx * STX, y0 = ty * STY, zlo = tz * zc, zhi = min(g.oz, zlo + zc);
  const int tid = threadIdx.x, lx = tid % 16, ly = tid / 16;
  const int rows = STY + g.ky - 1, cols = STX + KX - 1;
  double s0 = 0.0, s1 = 0.0;

  // taps, flipped for the forward operator, rows padded with zeros to 8
  for (int e = tid; e < KZ * g.ky * 8; e += ST) {
    const int c = e % 8, ab = e / 8, b = ab % g.ky, a = ab / g.ky;
    T v = (T)0;
    if (c < KX) {
      const int ha = g.flip ? KZ - 1 - a : a, hb = g.flip ? g.ky - 1 - b : b, hc = g.flip ? KX - 1 - c : c;
      v = H[((int64_t)ha * g.ky + hb) * KX + hc];
    }
    taps[e] = v;
  }

  const int yo = y0 + ly, xo = x0 + lx * SRX;
  const int64_t ostride = (int64_t)g.oy * g.ox, orow = (int64_t)yo * g.ox + xo;
  auto emit = [&](int z, const T *acc) __attribute__((always_inline)) {  // finished output plane z
    if (yo < g.oy) {
      const int64_t base = z * ostride + orow;
#pragma unroll
      for (int r = 0; r < SRX; ++r)
        if (xo + r < g.ox) apply_epilogue<T>(out, base + r, acc[r], ep, s0, s1);
    }
  };
  // input planes of output plane z: [max(0, z-offz), min(iz-1, z-offz+kz-1)]
  auto last_in = [&](int z) __attribute__((always_inline)) { return min(g.iz - 1, z - g.offz + KZ - 1); };

  // output planes that no input plane reaches are zero
  for (int z = zlo; z < zhi; ++z)
    if (max(0, z - g.offz) > last_in(z)) {
      const T zero[SRX] = {};
      emit(z, zero);
    }

  const int r_lo = max(0, zlo - g.offz), r_hi = min(g.iz - 1, zhi - 1 + KZ - 1 - g.offz);
  // staging element u of this thread: offset inside an input plane (-1:
  // outside the input, staged as zero) and LDS offset inside a plane buffer
  // (-1: past the staged rows); both are the same for every plane
  // (the plane offset is clamped into the plane and a validity bit kept)
  unsigned goff[SNIN], gvalid = 0;
  int loff[SNIN];
#pragma unroll
  for (int u = 0; u < SNIN; ++u) {
    const int e = tid + u * ST;
    const int r = e / SCOLS, q = e - r * SCOLS;
    const int yin = y0 + r - g.offy, xin = x0 + q - g.offx;
    const bool ok = r < rows && q < cols && yin >= 0 && yin < g.iy && xin >= 0 && xin < g.ix;
    goff[u] = ok ? (unsigned)(yin * g.ix + xin) : 0u;
    gvalid |= ok ? 1u << u : 0u;
    loff[u] = r < SROWS ? r * SSTRIDE + q : -1;
  }
  const int64_t pstride = (int64_t)g.iy * g.ix;
  T inreg[SNIN];
  auto load_plane = [&](int zin) __attribute__((always_inline)) {
    // uniform plane base + 32-bit per-thread offsets (always inside the
    // plane); elements outside the input are zeroed when staged, so nothing
    // waits for these loads before the plane's compute
    const T *plane = in + zin * pstride;
#pragma unroll
    for (int u = 0; u < SNIN; ++u) inreg[u] = plane[goff[u]];
  };

  // acc[j]: output plane z with (z mod KZ) == j (z >= 0, offz >= 0)
  T acc[KZ][SRX];
#pragma unroll
  for (int j = 0; j < KZ; ++j)
#pragma unroll
    for (int r = 0; r < SRX; ++r) acc[j][r] = (T)0;

  T done[SRX];  // finished output plane pz (-1: none) not yet stored
  int pz = -1;
  auto stage = [&](int zin) __attribute__((always_inline)) {  // registers -> LDS buffer of plane zin
    T *pl = planes + ((zin - r_lo) & 1) * SPLANE;
#pragma unroll
    for (int v = 0; v < SNIN; ++v)
      if (loff[v] >= 0) pl[loff[v]] = (gvalid >> v) & 1u ? inreg[v] : (T)0;
  };
  // plane r_lo staged, plane r_lo + 1 in flight
  if (r_lo <= r_hi) {
    load_plane(r_lo);
    stage(r_lo);
    if (r_lo < r_hi) load_plane(r_lo + 1);
  }
  __syncthreads();
  // the walk starts at the input plane zs0 <= r_lo with (zs0 + offz) mod KZ
  // == 0, so input plane zs0 + u reaches output plane z = zs0 + u + offz - a
  // through tap plane a, and z mod KZ == (u - a) mod KZ
  const int zs0 = r_lo - (r_lo + g.offz) % KZ;
  for (int zs = zs0; zs <= r_hi; zs += KZ) {
    sfor<0, KZ>([&](auto uc) {
      constexpr int u = decltype(uc)::value;
      const int zin = zs + u;
      if (zin < r_lo || zin > r_hi) return;  // uniform
      const T *pl = planes + ((zin - r_lo) & 1) * SPLANE;
      // stores of the plane finished one input plane ago: in flight during
      // this plane's compute
      if (pz >= 0) {
        emit(pz, done);
        pz = -1;
      }

      bool live[KZ];
#pragma unroll
      for (int a = 0; a < KZ; ++a) {
        const int z = zin + g.offz - a;
        live[a] = z >= zlo && z < zhi;
      }
      for (int b = 0; b < g.ky; ++b) {
        const T *src = pl + (ly + b) * SSTRIDE + lx * SRX;
        T w[SRX + KX - 1];
#pragma unroll
        for (int e = 0; e < SRX + KX - 1; ++e) w[e] = src[e];
        sfor<0, KZ>([&](auto ac) {
          constexpr int a = decltype(ac)::value;
          constexpr int j = ((u - a) % KZ + KZ) % KZ;
          if (live[a]) {
            const T *hrow = taps + (a * g.ky + b) * 8;
#pragma unroll
            for (int c = 0; c < KX; ++c) {
              const T hv = hrow[c];
#pragma unroll
              for (int r = 0; r < SRX; ++r) acc[j][r] += hv * w[r + c];
            }
          }
        });
      }
      // output planes completed by this input plane
      sfor<0, KZ>([&](auto ac) {
        constexpr int a = decltype(ac)::value;
        constexpr int j = ((u - a) % KZ + KZ) % KZ;
        const int z = zin + g.offz - a;
        if (live[a] && zin == last_in(z)) {
          // below the last input plane at most one output plane finishes per
          // input plane: its values wait in `done` for the next staging step
          if (zin < g.iz - 1 && zin < r_hi) {
#pragma unroll
            for (int r = 0; r < SRX; ++r) done[r] = acc[j][r];
            pz = z;
          } else {
            emit(z, acc[j]);
          }
#pragma unroll
          for (int r = 0; r < SRX; ++r) acc[j][r] = (T)0;
        }
      });
      // Plane zin+1 (loaded during this plane) goes to the other buffer, whose
      // readers finished before the last barrier; then plane zin+2 is loaded.
      // One barrier per plane: after it plane zin+1 is staged and nobody
      // reads plane zin's buffer any more.
      if (zin < r_hi) {
        stage(zin + 1);
        if (zin + 1 < r_hi) load_plane(zin + 2);
      }
      __syncthreads();
    });
  }
  if (pz >= 0) emit(pz, done);

  if (ep.mode != EPI_STORE) {
    block_sum2(s0, s1, red);
    if (tid == 0) {
      ep.part[2 * (int64_t)id] = s0;
      ep.part[2 * (int64_t)id + 1] = s1;
    }
  }
}

// Work-groups of one instantiation that fit on a CU at once (registers and
// LDS), from the runtime's occupancy calculator, once per process.
template <typename T, int KX, int KZ>
int small_occupancy() {
  static std::atomic<int> n{0};
  int v = n.load(std::memory_order_relaxed);
  if (v == 0) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, conv_small_kernel<T, KX, KZ>, ST, small_lds_bytes<T>(KZ)) !=
            hipSuccess ||
        v < 1) {
      (void)hipGetLastError();
      v = 1;
    }
    n.store(v, std::memory_order_relaxed);
  }
  return v;
}

template <typename T, int KX, int KZ>
hipError_t launch_small_t(const Geom &g, const void *in, const void *H, void *out, const Epi &ep, hipStream_t s) {
  const int zc = small_zchunk(g, small_occupancy<T, KX, KZ>());
  const int nbx = (g.ox + STX - 1) / STX, nby = (g.oy + STY - 1) / STY, nbz = (g.oz + zc - 1) / zc;
  hipLaunchKernelGGL((conv_small_kernel<T, KX, KZ>), dim3(nbx * nby * nbz), dim3(ST), small_lds_bytes<T>(KZ), s,
                     (const T *)in, (const T *)H, (T *)out, g, ep, nbx, nby, zc);
  return hipGetLastError();
}

template <typename T, int KZ>
hipError_t launch_small_kz(const Geom &g, const void *in, const void *H, void *out, const Epi &ep, hipStream_t s) {
  switch (g.kx) {
    case 1: return launch_small_t<T, 1, KZ>(g, in, H, out, ep, s);
    case 3: return launch_small_t<T, 3, KZ>(g, in, H, out, ep, s);
    case 5: return launch_small_t<T, 5, KZ>(g, in, H, out, ep, s);
    case 7: return launch_small_t<T, 7, KZ>(g, in, H, out, ep, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int KZ>
int small_occupancy_kz(int kx) {
  switch (kx) {
    case 1: return small_occupancy<T, 1, KZ>();
    case 3: return small_occupancy<T, 3, KZ>();
    case 5: return small_occupancy<T, 5, KZ>();
    default: return small_occupancy<T, 7, KZ>();
  }
}

// One translation unit per storage type and pair of z tap counts keeps the
// (heavily unrolled) instantiations compiling in parallel.
template <typename T, int KZ0, int KZ1>
hipError_t launch_small_pair(const Geom &g, const void *in, const void *H, void *out, const Epi &ep, hipStream_t s) {
  if (g.kz == KZ0) return launch_small_kz<T, KZ0>(g, in, H, out, ep, s);
  if (g.kz == KZ1) return launch_small_kz<T, KZ1>(g, in, H, out, ep, s);
  return hipErrorInvalidValue;
}

template <typename T, int KZ0, int KZ1>
int small_occupancy_pair(const Geom &g) {
  return g.kz == KZ0 ? small_occupancy_kz<T, KZ0>(g.kx) : small_occupancy_kz<T, KZ1>(g.kx);
}

}  // namespace

#define NDC_SMALL_PART(NAME, T, KZ0, KZ1)                                                                      \
  hipError_t launch_small_##NAME(const Geom &g, const void *in, const void *H, void *out, const Epi &ep,       \
                                 hipStream_t s) {                                                              \
    return launch_small_pair<T, KZ0, KZ1>(g, in, H, out, ep, s);                                               \
  }                                                                                                            \
  int occupancy_small_##NAME(const Geom &g) { return small_occupancy_pair<T, KZ0, KZ1>(g); }

}  // namespace ndc
