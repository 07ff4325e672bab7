// Internal declarations of the gfx950 convolution library.  Not part of the
// C ABI (that is include/ndconv.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../../include/ndconv.h"

namespace ndc {

// Both operators are one correlation over a zero-extended input:
//   out[s] = sum_{t in [0,k)} Hc[t] * in[s + t - off]   (in = 0 outside [0,in_extent))
// Forward (Property 1): out extent m+2p, in = X (extent m), off = 2p and
//   Hc[t] = H[2p - t] (so the sum is sum_j H[j] X[s - j]).
// Transpose (Property 2): out extent m, in = R (extent m+2p), off = 0 and
//   Hc = H (every tap lands inside R).
struct Geom {
  int oz, oy, ox;        // output extent
  int iz, iy, ix;        // input extent
  int kz, ky, kx;        // tap extent (2p+1)
  int offz, offy, offx;  // input index = out + tap - off
  int flip;              // Hc[t] = H[k-1-t] on every axis
};

enum EpiMode {
  EPI_STORE = 0, EPI_RESID = 1, EPI_UPDATE = 2, EPI_GRAD = 3, EPI_NORM = 4, EPI_SQR = 5, EPI_RINC = 6,
  EPI_RLQ = 7, EPI_RLX = 8
};

// Deconvolution phases kept on the device (see deconv.hip).
enum Phase { PH_NEW = 0, PH_RETRY = 1, PH_DONE = 2 };

// Epilogue applied to each output value `acc` at flat index i:
//   STORE : out[i] = acc
//   RESID : r = acc - Y[i]; out[i] = r; part0 += r^2            (objective)
//   UPDATE: g = acc + lambda*X[i] (+ mu*Q[i] if Q); G[i] = g;
//           xt = max(X[i] - delta*g, 0); out[i] = xt;
//           part0 += xt^2, part1 += (xt - X[i])^2               (Step 2)
//   GRAD  : g = acc + lambda*X[i] (+ mu*Q[i] if Q); out[i] = g;
//           part0 += g^2                                        (first trials)
//   NORM  : nothing stored; part0 += acc^2                      (||A g||^2)
//   SQR   : out[i] = acc; part0 += acc^2                        (L X, ||L X||^2)
//   RINC  : out[i] = B[i] + acc; part0 += out[i]^2, part1 += acc^2
//           (acc = A d for a step d: the trial residual A(X+d) - Y from the
//           current one, and ||A d||^2 without cancellation)
//   RLQ   : q = Y[i]/acc where acc > 0, else 0; out[i] = q;
//           part0 += Y[i] log(Y[i]/acc) - Y[i] + acc             (I-divergence)
//   RLX   : out[i] = out[i] * acc * (*delta)  (in place: X <- X A^T q / sum H)
// Partial sums are double, one pair per work-group, written without atomics.
// If phase != nullptr the kernel runs only when (1 << *phase) & phase_mask.
struct Epi {
  int mode;
  const void *Y;
  const void *X;
  void *G;
  double lambda;
  const double *delta;
  double *part;
  const int *phase;
  int phase_mask;
  const void *Q;  // UPDATE / GRAD: L^T L X (Tikhonov-Miller term), or null
  double mu;      // its weight
  const void *B;  // RINC: the array the product is added to
};

struct DState {
  double f_cur;    // f(X^k)
  double delta;    // trial step of the current attempt
  double delta0;   // 1/(||H||_1^2 + lambda)
  double lambda;
  int phase;       // Phase
  int k;           // accepted steps
  int rej;         // rejected trials in the current step
  int status;      // 0, 1 (no descent) or NDC_ENONFINITE
  int iters;       // target accepted steps
  int jmax;        // trials per step
  int accepted;    // 1 right after an accepting decision (commit copies)
  int rule;        // first trial of each iteration: NDC_STEP_FIXED / CAUCHY / BB
  double ss;       // BB: <s,s> of the last accepted step s = X^k - X^{k-1}
  double mu;       // Tikhonov-Miller weight (0: off)
  double sy;       // BB: <s, g^k - g^{k-1}> = ||A s||^2 + lambda <s,s> + mu ||L s||^2
};

// Launch descriptors --------------------------------------------------------
struct ConvPlan {
  int variant;        // 0 = VALU direct, 1 = 4x4 matrix tile, 2 = small-PSF streaming, 3 = 32x32 bf16 tile,
                      // 4 = 32x32 bf16 row-slot tile, 5 = 32x32 FP32 row-slot tile
  dim3 grid, block;
  size_t lds_bytes;
  int64_t nblocks;    // number of work-groups (partial-sum slots)
  int xb;             // variant 1: x-blocks per instruction (8 or 16)
  int nt;             // variant 3: 32x32 blocks per wave along x (2..4)
};

// Batched form ---------------------------------------------------------------
// One volume of a batch (device table).  For the convolution-only batch
// calls X is the input and R the output of the forward (the reverse for the
// transpose); the deconvolution uses every field.
struct BVol {
  int m[3], p[3];
  const float *Y, *H;
  float *X, *Xt, *G, *R, *Rt;
  DState *st;
  double *stats;  // nullable, (iters+1) x 4
  int *info;      // nullable, 2 ints
  int64_t n, ny;  // element counts of X and Y
  int fwd_lo, fwd_hi, adj_lo, adj_hi;  // partial-sum slot ranges of its tiles
};

// One tile of the persistent launch: volume, tile coordinates, partial slot.
struct BTile {
  int vol, tx, ty, tz, slot, pad0, pad1, pad2;
};

enum BatchOp { BOP_FWD = 0, BOP_ADJ = 1, BOP_INIT = 2, BOP_STEP_FWD = 3, BOP_STEP_ADJ = 4 };

// conv_dH_nd and conv_dH_nd_noalloc (abi.hip): scratch_max = 0 takes the
// caller's workspace, otherwise get_scratch() supplies the partials' buffer.
int dH_checked(int n, const int64_t *m, const int64_t *p, const void *X, const void *G, void *dH, int dtype,
               void *ws, size_t ws_bytes, size_t scratch_max, void *(*get_scratch)(), void *stream);

// Fold an n-D problem (n <= 3) into 3-D extents.
bool fold3(int n, const int64_t *m, const int64_t *p, int64_t m3[3], int64_t p3[3]);
Geom forward_geom(const int64_t m3[3], const int64_t p3[3]);
Geom adjoint_geom(const int64_t m3[3], const int64_t p3[3]);

// Plans and launches (conv_*.hip).  Return hipSuccess or the launch error.
ConvPlan plan_conv(const Geom &g, int dtype, int precision);
hipError_t launch_conv(const ConvPlan &pl, const Geom &g, int dtype, int precision, const void *in,
                       const void *H, void *out, const Epi &ep, hipStream_t s);

// Batched persistent launch (conv_mfma.hip): walks tiles[0..ntiles) with a
// grid of `grid` work-groups; mg is 2 or 4 output planes per tile.
hipError_t launch_batch_conv(int mg, const BVol *vols, const BTile *tiles, int ntiles, int op, double *part,
                             int grid, size_t lds_bytes, hipStream_t s);
size_t batch_lds_bytes(int kx, int ky, int mg);
bool batch_psf_supported(int kx, int ky);
dim3 batch_tile_counts(int oz, int oy, int ox, int mg);

}  // namespace ndc
