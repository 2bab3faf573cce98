/*
 * histretinex.h -- C ABI of the MI355X (gfx950) HistRetinex library.
 *
 * HistRetinex (Zhao et al., arXiv 2510.21100) enhances a low-light image in
 * the histogram domain: it builds the histogram of the HSV value channel S
 * and of its gradient image (Sec. II, Eq. 3; Alg. 1 initialisation), fits
 * illumination and reflectance histograms to it by the alternating updates of
 * Eqs. (11)-(15) (Alg. 1), brightens the illumination locations and forms the
 * enhanced target histogram (Eqs. 17-20), and maps every pixel to that target
 * by histogram matching (end of Sec. III-C).
 *
 * Conventions shared by every call
 *  - Images are HWC interleaved RGB in device memory: 8-bit images are uint8
 *    (bits = 8, 256 levels), 10-bit images are uint16 holding values 0..1023
 *    (bits = 10, 1024 levels).  Rows are row_stride_bytes apart; a stride of
 *    exactly 3*width*element_size with a 16-byte aligned base takes the
 *    vectorised path, any other stride >= that takes a slower scalar path.
 *  - Widths up to 16384 (8-bit) / 8192 (10-bit) are supported.
 *  - bins must equal 2^bits.
 *  - All device pointers are caller-owned; the library never frees them.
 *  - Every compute call is asynchronous and ordered on `stream` (a
 *    hipStream_t passed as void*, NULL = the default stream).  Arguments are
 *    validated on the host before anything is enqueued: on any error the call
 *    returns a status, enqueues nothing and records a message readable through
 *    hr_last_error() (thread-local).
 *  - Data faults found on the device (a 10-bit value above 1023, histograms
 *    whose mass disagrees with npix) cannot be returned as a status: the value
 *    is clamped / the histogram mass is used, and a sticky bit is set in the
 *    workspace flags, read with hr_get_flags() after the stream is synchronised.
 *  - A workspace holds device scratch, counters and cached launch graphs.  Use
 *    one workspace per stream: two calls in flight on one workspace race.
 *
 * Histograms are in the paper's count units: hist_v[k] is the number of pixels
 * whose value channel equals k, illum/refl/target sum to the pixel count.
 */
#ifndef HISTRETINEX_H
#define HISTRETINEX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HR_ABI_VERSION 3

typedef enum {
  HR_OK = 0,
  HR_ERR_INVALID_ARG = 1, /* null pointer, bad size, bad parameter value      */
  HR_ERR_UNSUPPORTED = 2, /* valid but outside what the library implements   */
  HR_ERR_WORKSPACE = 3,   /* workspace too small for the request              */
  HR_ERR_DEVICE = 4       /* a HIP runtime call failed; see hr_last_error()   */
} hr_status;

/* sticky device flags (hr_get_flags) */
#define HR_FLAG_VALUE_CLAMPED 0x1u /* a 10-bit channel value > 1023 was read  */
#define HR_FLAG_HIST_MASS 0x2u     /* histogram mass != npix in hr_solve       */

/* One RGB image.  data: device pointer to the first pixel. */
typedef struct {
  const void* data;
  int32_t width;
  int32_t height;
  int64_t row_stride_bytes;
} hr_image;

/* Method parameters.
 *  bins    : number of levels l (256 or 1024; must be 2^bits)
 *  iters   : T >= 0, the maximum number of Alg. 1 update passes
 *  alpha   : weight of the illumination prior of Eq. (10), > 0
 *  beta    : weight of the reflectance prior of Eq. (10), > 0
 *  gamma   : illumination gamma of Eq. (17), > 0
 *  eps     : error threshold of Alg. 1's stopping rule, finite.  The rule is
 *            garbled in the paper; it is read as: stop after pass t when
 *            t = iters, or earlier when the squared Euclidean norms of the
 *            changes of both normalised histograms in that pass (L and R in
 *            probability units, each summing to 1) are at most eps.  eps <= 0
 *            runs exactly iters passes.  The changes are summed in FP32, so
 *            an image whose change in some pass lies within FP32 rounding of
 *            eps may stop one pass away from an FP64 evaluation.
 *  variant : 0, or HR_VARIANT_* bits selecting other readings of passages
 *            the paper leaves open (below); only the one-image calls take
 *            them: hr_solve the solver bits (the gradient bits belong to
 *            hr_build_hist_variant), the batched and differentiated calls
 *            none (HR_ERR_UNSUPPORTED) */
typedef struct {
  int32_t bins;
  int32_t iters;
  double alpha;
  double beta;
  double gamma;
  double eps;
  uint32_t variant;
  int32_t reserved; /* must be 0 */
} hr_params;

/* Variant readings (hr_params.variant, hr_build_hist_variant's variant).
 * The main path reads the paper as: forward-difference L1 gradient,
 * histogram rescaled so its largest occupied raw level lands on l-1,
 * Eqs. (12)-(13) multiplying by K (the stationarity conditions of Eq. 10),
 * L(0) = the image histogram.  The variants run through simple kernels (one
 * thread per pixel, a dense solver over all l levels), not the tuned path.
 *  HR_VARIANT_GRAD_L2      gradient sqrt(dx^2 + dy^2) of the forward
 *                          differences, rounded half up
 *  HR_VARIANT_GRAD_SOBEL   3x3 Sobel derivatives on the border-replicated
 *                          image, (|gx| + |gy|) / 4 rounded half up
 *                          (excludes HR_VARIANT_GRAD_L2)
 *  HR_VARIANT_GRAD_CLIP    raw gradient level j goes to min(j, l-1) instead
 *                          of being rescaled by the largest occupied level
 *  HR_VARIANT_UPDATE_DIV   Eqs. (12)-(13) as printed, dividing by K_ij;
 *                          cells with K = 0 (an empty level of L or R, an
 *                          empty class) contribute nothing
 *  HR_VARIANT_INIT_UNIFORM L(0) = 1/l on every level */
#define HR_VARIANT_GRAD_L2 0x1u
#define HR_VARIANT_GRAD_SOBEL 0x2u
#define HR_VARIANT_GRAD_CLIP 0x4u
#define HR_VARIANT_UPDATE_DIV 0x8u
#define HR_VARIANT_INIT_UNIFORM 0x10u

/* Launch schedule of the batched form (chosen by the autotuner).  A step is
 * one pass of the persistent workgroup over its pixels: 1024 threads x 8 px
 * (8-bit) or x 4 px (10-bit).
 *  tile_steps  : steps per histogram work item
 *  wg_per_cu   : persistent workgroups per compute unit (1..8; at launch
 *                capped at what one CU holds at once -- one, with the batched
 *                kernel's LDS and registers on gfx950)
 *  remap_steps : steps per remap work item
 *  Zero in a field selects the built-in default. */
typedef struct {
  int32_t tile_steps;
  int32_t wg_per_cu;
  int32_t remap_steps;
} hr_schedule;

typedef struct hr_workspace hr_workspace;

/* ---- workspace ------------------------------------------------------------ */

/* Create a workspace for up to max_images images per hr_enhance_batch call
 * at up to max_bins levels (256 or 1024) on the current HIP device.
 * Allocates device memory; returns HR_ERR_DEVICE if that fails. */
hr_status hr_workspace_create(int32_t max_images, int32_t max_bins, hr_workspace** ws);
/* Release a workspace (NULL is ignored).  Synchronises the device first. */
void hr_workspace_destroy(hr_workspace* ws);
/* Set the batched-form schedule used by later hr_enhance_batch calls. */
hr_status hr_workspace_set_schedule(hr_workspace* ws, const hr_schedule* sched);
/* Read (and clear, if clear != 0) the sticky device flags.  Synchronises the
 * device. */
hr_status hr_get_flags(hr_workspace* ws, uint32_t* flags, int32_t clear);

/* ---- the hot path, one image per call -------------------------------------- */

/* Histograms of one image (Eq. 3 and the gradient histogram of Alg. 1).
 *  hist_v        : device uint32[bins], out: H_C(S), the value-channel histogram
 *  hist_grad     : device uint32[bins], out: H_C(grad S), the gradient
 *                  histogram rescaled onto the l levels (sums to width*height)
 *  hist_grad_raw : device uint32[2*bins-1] or NULL, out: the gradient image's
 *                  histogram before rescaling (gradient values 0..2(l-1))
 * The gradient image is |S(x+1,y)-S(x,y)| + |S(x,y+1)-S(x,y)| with the last
 * column and row replicated; raw level j maps to round-half-up(j(l-1)/gmax),
 * gmax = largest occupied raw level (all to 0 when gmax = 0). */
hr_status hr_build_hist(const hr_image* img, int32_t bits, uint32_t* hist_v, uint32_t* hist_grad,
                        uint32_t* hist_grad_raw, hr_workspace* ws, void* stream);

/* hr_build_hist with another gradient operator or rescaling: variant holds
 * HR_VARIANT_GRAD_* bits only (any other bit: HR_ERR_INVALID_ARG); 0 is
 * hr_build_hist itself.  hist_v is the same value histogram; hist_grad and
 * hist_grad_raw follow the selected operator (raw levels 0..2(l-1)). */
hr_status hr_build_hist_variant(const hr_image* img, int32_t bits, uint32_t variant, uint32_t* hist_v,
                                uint32_t* hist_grad, uint32_t* hist_grad_raw, hr_workspace* ws, void* stream);

/* The histograms of hr_build_hist for n images of one bit depth, in one
 * launch (a grid of tiles per image; the last tile of an image rescales its
 * gradient histogram).
 *  in        : host array [n] of image descriptors
 *  hist_v    : device uint32[n][bins], out: H_C(S) of each image
 *  hist_grad : device uint32[n][bins], out: H_C(grad S) of each image
 * n must not exceed the workspace's max_images.  Uses the workspace's
 * per-image state and descriptor table: calls on one workspace are
 * stream-ordered (as with hr_enhance_batch). */
hr_status hr_build_hist_batch(const hr_image* in, int32_t n, int32_t bits, uint32_t* hist_v, uint32_t* hist_grad,
                              hr_workspace* ws, void* stream);

/* Alg. 1 followed by the reprocessing of Eqs. (17)-(20).
 *  hist_v, hist_grad : device uint32[bins] (as produced by hr_build_hist)
 *  npix              : number of pixels N (= sum of hist_v)
 *  illum             : device float[bins], out: final H~_C(L) of Eq. (14), counts
 *  refl              : device float[bins], out: final H~_C(R) of Eq. (15), counts
 *  target            : device float[bins], out: H_C(S~) of Eq. (20), counts
 *  passes            : device int32[1] or NULL, out: the passes run (p->iters,
 *                      or fewer when the stopping rule of p->eps fired)
 * The updates are Eq. (13) for R then Eq. (12) for L (with the weights K of
 * Eq. (11) multiplying, as in the stationarity conditions of Eq. (10)), then
 * the rescalings of Eqs. (15), (14), starting from R = H_C(grad S) and
 * L = H_C(S).  Runs in FP32 on one workgroup.  The histograms are checked on
 * the device: a mass of hist_v other than npix, or of hist_grad other than
 * that of hist_v, sets HR_FLAG_HIST_MASS (read with hr_get_flags) and the
 * histograms are used as given; histograms without any mass give zero
 * outputs.  With HR_VARIANT_UPDATE_DIV or HR_VARIANT_INIT_UNIFORM in
 * p->variant the dense variant solver runs instead (all l levels, FP32
 * state with FP64 sums; much slower). */
hr_status hr_solve(const uint32_t* hist_v, const uint32_t* hist_grad, int64_t npix,
                   const hr_params* p, float* illum, float* refl, float* target, int32_t* passes,
                   hr_workspace* ws, void* stream);

/* Histogram matching of the image to `target` (end of Sec. III-C) and the
 * pixel remap.
 *  in      : the image the histogram hist_v was built from
 *  hist_v  : device uint32[bins]
 *  target  : device float[bins], the target histogram (any positive scale)
 *  out     : device pointer, same element type and size as `in`, rows
 *            out_row_stride_bytes apart (may equal in->data)
 *  lut_out : device uint16[bins] or NULL, out: the level map
 * LUT[v] = min{k : F~(k) >= (F_S(v-1) + F_S(v))/2}, F~ the normalised running
 * sum of target and F_S the image CDF; each pixel keeps hue and saturation and
 * gets value LUT[V]: out_c = round-half-up(c * LUT[V] / V), black -> LUT[0]. */
hr_status hr_match(const hr_image* in, int32_t bits, const uint32_t* hist_v, const float* target,
                   void* out, int64_t out_row_stride_bytes, uint16_t* lut_out, hr_workspace* ws,
                   void* stream);

/* Classical histogram equalisation (Eq. 5), the comparator the paper
 * starts from, through the same remap as hr_match: level v goes to the
 * nearest level of (l-1) * F_S(v) (F_S the image CDF, ties upwards), i.e.
 * LUT[v] = floor((2 (l-1) c(v) + N) / (2N)) with c the running count of
 * hist_v and N its total, computed in integers (exact).
 *  in, bits, hist_v, out, out_row_stride_bytes, lut_out, ws, stream : as hr_match
 * A hist_v without mass maps every level to 0. */
hr_status hr_equalize(const hr_image* in, int32_t bits, const uint32_t* hist_v, void* out,
                      int64_t out_row_stride_bytes, uint16_t* lut_out, hr_workspace* ws, void* stream);

/* ---- the batched form --------------------------------------------------------- */

/* The whole pipeline (hr_build_hist, hr_solve, hr_match) over n images of
 * any sizes in one persistent launch, captured once in a HIP graph and
 * replayed.
 *  in   : host array [n] of image descriptors (device data pointers)
 *  out  : host array [n] of device output pointers (same element type/size)
 *  out_row_stride_bytes : host array [n]
 *  luts : device uint16[n][bins] or NULL: per-image level maps, out
 *  illum, refl, target : device float[n][bins] or NULL: per-image solver
 *         outputs, as hr_solve
 *  passes : device int32[n] or NULL: per-image passes run, as hr_solve
 * n must be in 1..max_images of the workspace. */
hr_status hr_enhance_batch(const hr_image* in, void* const* out, const int64_t* out_row_stride_bytes,
                           int32_t n, int32_t bits, const hr_params* p, uint16_t* luts,
                           float* illum, float* refl, float* target, int32_t* passes,
                           hr_workspace* ws, void* stream);

/* hr_enhance_batch for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Takes no workspace and allocates nothing (no hipMalloc, no
 * hipFree, no allocating library routine): the descriptor table travels as
 * a kernel argument, and the queue, counters and per-image states live in
 * one fixed device array of the library, about 0.5 MB on each GPU it runs
 * on, held until the process ends.  Every call on a GPU
 * shares that array: two calls that overlap on one GPU (different streams,
 * or threads without ordering) race; calls ordered on one stream do not.
 * Each call clears what must start at zero.  Results are those of
 * hr_enhance_batch with the default schedule (bit for bit).
 *  in, out, out_row_stride_bytes, bits, p, luts, illum, refl, target,
 *  passes : as hr_enhance_batch
 *  n      : 1..HR_NOALLOC_MAX_IMAGES; more is refused with HR_ERR_UNSUPPORTED
 *  flags  : device uint32[1] or NULL: the sticky device flags of the call are
 *           OR-ed into it (the caller clears it; NULL: not reported)
 *  stream : as everywhere; the call enqueues two kernels on it */
#define HR_NOALLOC_MAX_IMAGES 4
hr_status hr_enhance_batch_noalloc(const hr_image* in, void* const* out, const int64_t* out_row_stride_bytes,
                                   int32_t n, int32_t bits, const hr_params* p, uint16_t* luts,
                                   float* illum, float* refl, float* target, int32_t* passes,
                                   uint32_t* flags, void* stream);

/* ---- the differentiated form (256 levels; not part of the paper) ------------------
 *
 * Gradients of an enhancement loss with respect to the prior weights alpha,
 * beta of Eq. (10) and the target histogram h~ of Eq. (20).  The exact LUT is
 * piecewise constant in h~, so the loss uses a soft matching map m(v): the
 * piecewise-linear inverse of the normalised target CDF F~ through the knots
 * (k + 1/2, F~(k)) (and (-1/2, 0)), evaluated at the mid-rank image CDF u(v)
 * that the exact LUT uses, clamped to [0, l-1]; round(m(v)) = LUT[v].  The
 * loss of an image is the mean over its pixels and channels of
 * (c m(V) / (V (l-1)) - t_c)^2 (m(0) / (l-1) for black pixels) against a
 * target image t.  H_C(S), H_C(grad S) and the classes are constants.
 * Every call handles n images of one batch; arrays indexed [n] are per image.
 */

/* Alg. 1 for p->iters passes on each of n histogram pairs, keeping the
 * dense (L, R) of t = 0, ckpt_every, ..., iters (probability units).
 * Runs exactly p->iters passes: p->eps must be <= 0.
 *  hist_v, hist_grad : device uint32[n][256] (from hr_build_hist)
 *  ckpt_every        : 1..16, and p->iters must be a multiple of it
 *  ckpt              : device float[n][iters/ckpt_every + 1][2][256], out:
 *                      L at [..][0][level], R at [..][1][level]
 *  target            : device float[n][256], out: h~ of Eq. (20), counts */
hr_status hr_solve_ckpt(const uint32_t* hist_v, const uint32_t* hist_grad, int32_t n, const hr_params* p,
                        int32_t ckpt_every, float* ckpt, float* target, hr_workspace* ws, void* stream);

/* Soft-matching loss of n 8-bit images and its gradient with respect to h~.
 *  in         : host array [n] of image descriptors (8-bit)
 *  target_img : host array [n] of device pointers to float[H][W][3] (tight
 *               rows, 4-byte aligned): the target t of each image
 *  hist_v     : device uint32[n][256], H_C(S) of each image
 *  target     : device float[n][256], h~ (non-negative, positive sum)
 *  loss       : device double[n], out: the loss of each image
 *  dtarget    : device float[n][256], out: dLoss_i/dh~_i
 * Uses the workspace's scratch; calls on one workspace are stream-ordered. */
hr_status hr_softmatch_loss_grad(const hr_image* in, const float* const* target_img, int32_t n,
                                 const uint32_t* hist_v, const float* target, double* loss, float* dtarget,
                                 hr_workspace* ws, void* stream);

/* Reverse pass of hr_solve_ckpt: given dLoss/dh~ of each image, the
 * gradient with respect to alpha and beta through Eq. (20) and the K
 * passes of Eqs. (11)-(15), recomputing each checkpoint segment.
 *  hist_v, hist_grad, p, ckpt_every : as passed to hr_solve_ckpt
 *  ckpt     : device float, as written by hr_solve_ckpt
 *  dtarget  : device float[n][256], dLoss/dh~
 *  dalpha, dbeta : device double[n], out: per-image gradients */
hr_status hr_solve_vjp(const uint32_t* hist_v, const uint32_t* hist_grad, int32_t n, const hr_params* p,
                       int32_t ckpt_every, const float* ckpt, const float* dtarget, double* dalpha, double* dbeta,
                       hr_workspace* ws, void* stream);

/* ---- support ------------------------------------------------------------------ */

const char* hr_status_string(hr_status s);
const char* hr_last_error(void);
int32_t hr_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HISTRETINEX_H */
