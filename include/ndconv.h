/*
 * ndconv.h -- C ABI of the gfx950 (MI355X) library for the n-dimensional
 * full convolution, its transpose, and the projected-gradient deconvolution
 * built from them, following "Properties on n-dimensional convolution for
 * image deconvolution" (arXiv 1711.11224).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  n          number of axes, 1 <= n <= 3 (an n-D problem with n < 3 is run
 *             as 3-D with unit extents and zero half-widths in front).
 *  m[0..n)    extent of X on each axis, m_i >= 1 (the X size of Eq. 4).
 *  p[0..n)    PSF half-widths, p_i >= 0; H has extent 2p_i+1 (Property 1's
 *             template domain {0..2p_i}).  2p_i >= m_i is allowed.
 *  Y extent   m_i + 2p_i (Eq. 4).
 *  Layout     every array is dense C order, axis 0 slowest, matching the
 *             row partitioning of the vectorisation {.}^v under Eq. 1.
 *  Pointers   every array pointer is a DEVICE pointer on the current HIP
 *             device, owned by the caller; the library never keeps it after
 *             the call returns and never allocates memory the caller sees.
 *  dtype      NDC_F32 (float) or NDC_F64 (double): the storage type of X, H,
 *             Y and of any workspace arrays.
 *  precision  NDC_PREC_NATIVE computes the multiply-adds in the storage type.
 *             NDC_PREC_BF16 rounds both operands to bfloat16 (round to nearest
 *             even) and accumulates in float; NDC_PREC_SPLIT_BF16 writes each
 *             operand as hi + lo with hi = bf16(v), lo = bf16(v - hi) and sums
 *             hi*hi + hi*lo + lo*hi in float.  The bf16 forms need NDC_F32.
 *  stream     a hipStream_t passed as void*; NULL is the null stream.  All
 *             work is enqueued asynchronously on it.
 *
 * Errors: every argument check runs before anything is enqueued.  On a
 * negative status nothing was launched and no output was written.
 * NDC_EDEVICE reports a failed launch.  No entry point throws or aborts.
 * Calls on different streams that share an output buffer race.
 */
#ifndef NDCONV_H
#define NDCONV_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define NDC_API __attribute__((visibility("default")))
#else
#define NDC_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NDC_OK = 0,
  NDC_EINVAL = -1,       /* bad n, extent, half-width, count, pointer or scalar */
  NDC_EUNSUPPORTED = -2, /* valid request the library does not implement     */
  NDC_EALIAS = -3,       /* an output overlaps an input or another output     */
  NDC_ENONFINITE = -4,   /* reported in deconvolution status words only       */
  NDC_EDEVICE = -5,      /* a HIP runtime call or kernel launch failed         */
  NDC_EWORKSPACE = -6    /* workspace missing or smaller than required         */
} ndc_status;

typedef enum { NDC_F32 = 0, NDC_F64 = 1 } ndc_dtype;

typedef enum {
  NDC_PREC_NATIVE = 0,
  NDC_PREC_BF16 = 1,
  NDC_PREC_SPLIT_BF16 = 2
} ndc_precision;

/* Forward operator, Property 1 and Eq. 4: the full discrete convolution
 *   Y[s] = sum_{j in prod [0,2p_i]} H[j] X[s-j],  s in prod [0, m_i+2p_i),
 * with X taken as zero outside prod [0, m_i).  Y (prod(m_i+2p_i) elements)
 * is fully overwritten; X and H (prod(m_i), prod(2p_i+1) elements) are read. */
NDC_API int conv_full_nd(int n, const int64_t *m, const int64_t *p, const void *X, const void *H,
                 void *Y, int dtype, int precision, void *stream);

/* Transpose, Property 2 and Eq. 2: (A_n^h)^T applied to R equals the crop
 * M_{2p} of R convolved with the flipped PSF H~(s) = H(2p-s), i.e.
 *   X[k] = sum_{j in prod [0,2p_i]} H[j] R[k+j],  k in prod [0, m_i).
 * R has extent m_i+2p_i; X (prod(m_i) elements) is fully overwritten. */
NDC_API int conv_adjoint_nd(int n, const int64_t *m, const int64_t *p, const void *R, const void *H,
                    void *X, int dtype, int precision, void *stream);

/* Non-finite inputs (both operators): the matrix-core kernels also multiply
 * the zeros of their Toeplitz operands, so an Inf or NaN input element can
 * turn outputs near it into NaN even where no tap reaches it: up to 3
 * columns away in FP32 and in the narrow-row bf16 forms, up to 31 columns in
 * the bf16 forms for rows of 11-33 taps, and up to 3 planes away in FP32.
 * Finite inputs are unaffected (0 * x = 0). */

/* Gradient of 1/2 ||X (x) H - Y||^2 with respect to H, given the residual
 * G = X (x) H - Y (extent m_i+2p_i):  dH[j] = sum_k X[k] G[k+j],
 * j in prod [0,2p_i].  Convolution commutes, so this is Property 1's
 * transpose with X as the template.  dH (prod(2p_i+1)) is overwritten.
 * ws must hold conv_dH_workspace_bytes() bytes (may be 0 -> ws may be NULL). */
NDC_API size_t conv_dH_workspace_bytes(int n, const int64_t *m, const int64_t *p, int dtype);
NDC_API int conv_dH_nd(int n, const int64_t *m, const int64_t *p, const void *X, const void *G, void *dH,
               int dtype, void *ws, size_t ws_bytes, void *stream);

/* conv_dH_nd for callers that cannot allocate device memory (code under
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * kernels and result, bit for bit, with the split-K partials in a scratch
 * array of NDC_DH_SCRATCH_BYTES that the library holds in device memory on
 * each GPU it runs on, until the process ends.  The call allocates nothing.
 * NDC_EWORKSPACE (before anything is enqueued) when the partials would need
 * more than NDC_DH_SCRATCH_BYTES, i.e. when conv_dH_workspace_bytes() of
 * the problem exceeds it (32 MiB covers, e.g., a 128x512x512 X with a
 * 63x31x31 PSF); NDC_EDEVICE if the array's address cannot be obtained.
 * The array holds no state between calls (every partial is written before
 * it is read), but every call on one GPU uses the same array: calls that
 * overlap in time on one GPU (different streams, or host threads) race. */
#define NDC_DH_SCRATCH_BYTES ((size_t)1 << 25)
NDC_API int conv_dH_nd_noalloc(int n, const int64_t *m, const int64_t *p, const void *X, const void *G, void *dH,
                               int dtype, void *stream);

/* Projected-gradient deconvolution (Steps 1-3 of the paper's algorithm,
 * gradient by Eq. 6 in its fused form A^T(AX - Y) + lambda X):
 *   minimise f(X) = 1/2 ||A X - Y||^2 + lambda/2 ||X||^2  s.t. X >= 0,
 *   X^{k+1} = max(X^k - delta_k grad f(X^k), 0).
 * delta_k is accepted by the paper's rule f(X^{k+1}) < f(X^k): trials start
 * at delta_0 = 1/(||H||_1^2 + lambda) and halve, at most 30 per step; f is
 * evaluated in double precision.  lambda = 0 is the paper's objective.
 *
 *  Y      extent m_i+2p_i, read.   H extent 2p_i+1, read.
 *  X      in: X^0 (caller's initial solution); out: X^{iters_done}.
 *  iters  accepted steps to run (0 <= iters <= NDC_MAX_ITERS).
 *  ws     workspace of at least deconv_workspace_bytes() bytes, caller-owned,
 *         device memory; contents on entry are ignored.
 *  stats  nullable device array of 4*(iters+1) doubles: row k holds
 *         (f(X^k), delta used to reach X^k, rejected trials, ||X^k-X^{k-1}||);
 *         row 0 holds f(X^0).  Rows past iters_done are left untouched.
 *  info   nullable device array of 2 ints: (iters_done, status), status one
 *         of NDC_STOP_DONE, NDC_STOP_NO_DESCENT, NDC_STOP_TRIALS or
 *         NDC_ENONFINITE (stopped on a non-finite objective).
 *
 * Every trial (the first one of a step and each halved retry) costs one
 * forward convolution.  The call enqueues a fixed schedule of 2*iters + 30
 * trial slots (none for iters = 0) and returns without waiting: the accept,
 * halve and stop decisions are taken on the device, and slots after the run
 * has stopped return at once.  A run that has used every slot before
 * `iters` accepted steps stops with NDC_STOP_TRIALS; its accepted steps
 * stand, and since the fixed first trial keeps no state across steps a
 * second call from the returned X continues it exactly.  X, stats and info
 * are complete once the stream reaches the end of the call's work; the call
 * may be captured into a graph (each replay reruns the whole call). */
enum {
  NDC_STOP_DONE = 0,       /* iters accepted steps                              */
  NDC_STOP_NO_DESCENT = 1, /* no trial decreased f within 30 halvings          */
  NDC_STOP_TRIALS = 2      /* every enqueued trial slot used before iters steps */
};
#define NDC_MAX_ITERS (1 << 24)
NDC_API size_t deconv_workspace_bytes(int n, const int64_t *m, const int64_t *p, int dtype, int precision);
NDC_API int deconv_iterate(int n, const int64_t *m, const int64_t *p, const void *Y, const void *H, void *X,
                   int iters, double lambda, int dtype, int precision, void *ws, size_t ws_bytes,
                   double *stats, int *info, void *stream);

/* Extended deconvolution: the arguments of deconv_iterate plus
 *   rule: the first trial of each iteration (the halving on failure and the
 *         strict-decrease test that follow are those of deconv_iterate).
 *         The paper states only the acceptance rule f(X^{k+1}) < f(X^k) for
 *         delta_k (Step 2 of its deconvolution algorithm), so any first trial
 *         is admissible:
 *     NDC_STEP_FIXED  delta_0 (below), as deconv_iterate;
 *     NDC_STEP_CAUCHY <g,g> / (||A g||^2 + lambda ||g||^2 + mu ||L g||^2), the
 *                     line minimiser of the unprojected objective along -g;
 *                     one extra forward convolution per iteration;
 *     NDC_STEP_BB     Barzilai-Borwein <s,s>/<s,y>, s = X^k - X^{k-1},
 *                     y = g^k - g^{k-1}; delta_0 on the first iteration of a
 *                     call.  f is quadratic, so <s,y> is summed as
 *                     ||A s||^2 + lambda ||s||^2 + mu ||L s||^2 from a forward
 *                     of the step (no extra convolution: each BB trial's
 *                     forward is taken of X_t - X^k and added to the current
 *                     residual).  A non-positive or non-finite quotient falls
 *                     back to delta_0.
 *   mu:   weight of a Tikhonov-Miller term mu/2 ||L X||^2 (the regularised
 *         family the paper's introduction names; >= 0, 0 = off).  L is the
 *         full convolution by the discrete Laplacian over the problem's n
 *         axes (3^n stencil: -2n at the centre, +1 at the axis neighbours;
 *         zero outside X).  The gradient gains mu L^T L X and
 *         delta_0 = 1/(||H||_1^2 + lambda + mu (4n)^2).
 *   max_trials: trial slots to enqueue (0 = 2*iters + 30 as deconv_iterate,
 *         at most 2*NDC_MAX_ITERS + 30); a run that uses them all before
 *         `iters` steps stops with NDC_STOP_TRIALS.  Each unused slot costs
 *         a few launches that return at once, which is negligible next to a
 *         convolution except on tiny problems.
 * With mu > 0 the workspace is deconv_workspace_bytes_ex(..., 1) (larger by
 * two (m+2)-extent arrays, one X-sized array and the stencil); with mu = 0 it
 * is deconv_workspace_bytes.  NDC_EINVAL for an unknown rule, a negative or
 * non-finite mu or a max_trials out of range; otherwise errors and
 * asynchrony as deconv_iterate.  The BB rule keeps <s,s> and <s,y> of the
 * last accepted step on the device; a new call starts again from delta_0. */
enum { NDC_STEP_FIXED = 0, NDC_STEP_CAUCHY = 1, NDC_STEP_BB = 2 };
NDC_API size_t deconv_workspace_bytes_ex(int n, const int64_t *m, const int64_t *p, int dtype, int precision,
                                         int regularised);
NDC_API int deconv_iterate_ex(int n, const int64_t *m, const int64_t *p, const void *Y, const void *H, void *X,
                              int iters, double lambda, double mu, int dtype, int precision, int rule,
                              int max_trials, void *ws, size_t ws_bytes, double *stats, int *info, void *stream);

/* Richardson-Lucy (maximum-likelihood) deconvolution, the method the paper
 * compares its own against (Introduction; Fig. 2f), built from the same two
 * operators (Property 1 and Property 2):
 *   X^{k+1} = X^k * A^T(Y / (A X^k)) / A^T 1,   A^T 1 = sum H at every voxel,
 * the ratio taken as 0 where A X^k = 0.  It decreases the I-divergence
 * D(Y || A X) = sum Y log(Y / (A X)) - Y + A X (0 log 0 = 0), the Poisson
 * negative log-likelihood up to a constant.  Preconditions (not checked on
 * the host): Y >= 0, H >= 0 with sum H > 0, X^0 >= 0.
 *
 *  X      in: X^0; out: X^{iters}, updated in place.
 *  iters  iterations (0 <= iters <= NDC_MAX_ITERS); iters + 1 forward and
 *         iters transpose convolutions are enqueued, nothing waits on the host.
 *  ws     at least rl_workspace_bytes() bytes of device memory (one
 *         Y-sized array and small state), contents on entry ignored.
 *  stats  nullable device array of iters+1 doubles: D(Y || A X^k), k = 0..iters.
 *  info   nullable device array of 2 ints: (k of the last recorded
 *         divergence, status) with status NDC_STOP_DONE, NDC_ENONFINITE (a
 *         NaN divergence stopped the run; X holds the last iterate) or
 *         NDC_EINVAL (sum H not positive and finite: nothing ran).
 * Argument checks and aliasing rules as deconv_iterate; the call may be
 * captured into a graph. */
NDC_API size_t rl_workspace_bytes(int n, const int64_t *m, const int64_t *p, int dtype, int precision);
NDC_API int rl_iterate(int n, const int64_t *m, const int64_t *p, const void *Y, const void *H, void *X, int iters,
                       int dtype, int precision, void *ws, size_t ws_bytes, double *stats, int *info,
                       void *stream);

/* Batched form: many independent 3-D volumes, each with its own extents m,
 * half-widths p and PSF.  The deconvolution runs persistent launches that
 * walk one tile list for the whole batch, or (tuning[0] = 0) each volume's
 * own kernels on the plan's streams.  Every volume keeps its own step size
 * and acceptance decisions (the rule of deconv_iterate); one trial slot of
 * the whole batch is captured into a hipGraph (again when the workspace, or
 * for tuning[0] = 0 any volume's address or lambda, differs from the last
 * capture) and replayed per slot.  FP32 only; every
 * PSF needs 3 <= 2p_x+1 <= 33 and 2p_y+1 <= 33.
 *
 *  ndc_batch_plan_create: m and p are count x 3 host arrays (z, y, x);
 *    tuning is NULL or 4 ints {output planes per tile (2 or 4; 0: the
 *    deconvolution's operators run each volume's own single-volume kernel on
 *    the plan's streams instead of the persistent tile, and the next two
 *    values are unused), work-groups per CU (1 or 2), tile order (0 by
 *    volume, 1 interleaved, 2 costliest volume first), use the hipGraph (0
 *    or 1)}.  The plan owns small device tables; destroy it with
 *    ndc_batch_plan_destroy.
 *  ndc_batch_conv_full / ndc_batch_conv_adjoint: the two operators of every
 *    volume, each volume's single-volume kernel (as conv_full_nd /
 *    conv_adjoint_nd choose it) on one of the plan's 4 streams (each with a
 *    hardware queue of its own), costliest volumes first, forked from and
 *    joined back to `stream` with events; the pointer arguments are host
 *    arrays of count device pointers, read before the call returns.
 *  ndc_batch_deconv: `iters` accepted steps on every volume, X[v] updated in
 *    place; ws holds ndc_batch_workspace_bytes(); stats is NULL or a host
 *    array of count nullable device pointers (each 4*(iters+1) doubles, as in
 *    deconv_iterate); info is NULL or a device array of 2*count ints
 *    (iters_done, status) per volume.  The same fixed schedule of
 *    2*iters + 30 trial slots as deconv_iterate, with the same stop codes.
 *  All three are ordered on `stream` (the operators' side streams wait for
 *  it and it waits for them) and may be captured into a graph (inside a
 *  capture the step is enqueued kernel by kernel instead of as the plan's own
 *  graph).  Calls with one plan share its device tables, streams and events,
 *  so they must be ordered on one stream; overlapping calls with one plan on
 *  different streams race.  Every output is checked against every input and
 *  every other output (NDC_EALIAS) and every pointer must be device memory
 *  (NDC_EINVAL) before anything is enqueued.  ndc_batch_plan_destroy waits
 *  for the device to finish outstanding work first.
 *  ndc_batch_plan_info: (forward tiles, transpose tiles, persistent grid,
 *    LDS bytes per work-group). */
typedef struct ndc_batch_plan ndc_batch_plan;
NDC_API int ndc_batch_plan_create(int count, const int64_t *m, const int64_t *p, int dtype, int precision,
                                  const int *tuning, ndc_batch_plan **plan);
NDC_API void ndc_batch_plan_destroy(ndc_batch_plan *plan);
NDC_API size_t ndc_batch_workspace_bytes(const ndc_batch_plan *plan);
NDC_API int ndc_batch_plan_info(const ndc_batch_plan *plan, int64_t *out4);
NDC_API int ndc_batch_conv_full(ndc_batch_plan *plan, const void *const *X, const void *const *H, void *const *Y,
                                void *stream);
NDC_API int ndc_batch_conv_adjoint(ndc_batch_plan *plan, const void *const *R, const void *const *H,
                                   void *const *X, void *stream);
NDC_API int ndc_batch_deconv(ndc_batch_plan *plan, const void *const *Y, const void *const *H, void *const *X,
                             int iters, double lambda, void *ws, size_t ws_bytes, double *const *stats, int *info,
                             void *stream);

/* Kernel form per problem (the autotuner's hook).  Each operator of a
 * problem runs one of the library's kernel forms; by default a built-in rule
 * picks it from the PSF and volume size.  ndc_tile_override replaces that
 * choice for one exact problem (n, m, p, dtype, precision) and operator (op
 * 0 = forward conv_full_nd, 1 = transpose conv_adjoint_nd) wherever the
 * library runs that operator (the operators, deconv_iterate, rl_iterate):
 *   NDC_FORM_AUTO    remove the override (built-in rule);
 *   NDC_FORM_VALU    the general vector-ALU kernel (every problem);
 *   NDC_FORM_SMALL   the small-PSF streaming kernel (every axis <= 7 taps,
 *                    native precision);
 *   NDC_FORM_MFMA4   the 4x4x1 matrix-core tile, param = x-blocks per
 *                    instruction: 8 (32x32 outputs per wave group) or 16
 *                    (16x64, native precision only); 3 <= 2p_x+1 <= 33;
 *   NDC_FORM_MFMA32  the 32x32x16 bf16 tile (bf16 forms, 11 <= 2p_x+1 <= 33),
 *                    param = 32x32 blocks per wave along x, 2..4 (split-bf16:
 *                    2..3);
 *   NDC_FORM_SLOT    the row-slot tiles (2p_x+1 <= 32, 2p_y+1 <= 32,
 *                    2p_z+1 <= 64): output rows kept in rotating accumulator
 *                    slots, so the matrix products are PSF taps rather than
 *                    Toeplitz zeros; persistent, one work-group per CU.  bf16
 *                    on the 32x32x16 instruction (the PSF's bf16 copy within
 *                    the LDS budget, about 125 KiB at 63 x 31 x 31), FP32
 *                    storage in native precision on the 32x32x2 FP32
 *                    instruction.
 * NDC_EUNSUPPORTED if the form cannot run the problem (or the table, of
 * NDC_MAX_TILE_OVERRIDES entries, is full).  Every form computes the same
 * operator; results agree within the precision's rounding.  The table is
 * process-wide and guarded by a lock; a workspace sized before an override
 * changed a plan is checked again by each call.  ndc_tile_choice reports the
 * form and parameter the library would use now, as out2[0..1]. */
enum {
  NDC_FORM_AUTO = 0, NDC_FORM_VALU = 1, NDC_FORM_SMALL = 2, NDC_FORM_MFMA4 = 3, NDC_FORM_MFMA32 = 4,
  NDC_FORM_SLOT = 5
};
#define NDC_MAX_TILE_OVERRIDES 4096
NDC_API int ndc_tile_override(int n, const int64_t *m, const int64_t *p, int dtype, int precision, int op,
                              int form, int param);
NDC_API void ndc_tile_override_clear(void);
NDC_API int ndc_tile_choice(int n, const int64_t *m, const int64_t *p, int dtype, int precision, int op,
                            int *out2);

/* Static text for a status code (never NULL). */
NDC_API const char *ndc_strerror(int status);

/* Library ABI version: (major << 16) | minor. */
NDC_API int ndc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* NDCONV_H */
