// Declarations shared by the kernels and the C-ABI host layer: the batched
// form's device-side tables and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hr {

// One image as the kernels see it.  Pixel p (flat, row-major) is at
// in + (p / W) * in_stride + 3 * (p % W) * sizeof(pix_t).
struct ImgDesc {
  const uint8_t* in;
  uint8_t* out;
  int64_t in_stride;
  int64_t out_stride;
  int64_t npix;
  int32_t W;
  int32_t H;
  int32_t in_vec;   // rows are tight and the base is 16-byte aligned
  int32_t out_vec;
  int32_t ntiles;   // batched form: histogram items of this image
  int32_t tile0;    // batched form: first histogram item of this image
  int32_t rtiles;   // batched form: remap items of this image
  int32_t slot;     // batched form: index of this image in the caller's arrays
};

// Solver parameters as the kernels take them.
struct SolveParams {
  int32_t iters;       // the maximum number of passes T
  float alpha;
  float beta;
  int32_t ckpt_every;  // differentiated form: checkpoint interval (0: none)
  double inv_gamma;
  float eps;           // stopping threshold of Alg. 1 (<= 0: exactly iters passes)
  uint32_t variant;    // VARIANT_* bits of the solver (0: the main path's readings)
};

// Variant readings (the bits of hr_params.variant): the gradient operator and
// the rescaling of its histogram (histogram calls), the form of Eqs. (12)-(13)
// and the initial illumination histogram (solver calls).
constexpr uint32_t VARIANT_GRAD_L2 = 0x1u;
constexpr uint32_t VARIANT_GRAD_SOBEL = 0x2u;
constexpr uint32_t VARIANT_GRAD_CLIP = 0x4u;
constexpr uint32_t VARIANT_UPDATE_DIV = 0x8u;
constexpr uint32_t VARIANT_INIT_UNIFORM = 0x10u;
constexpr uint32_t VARIANT_GRAD_BITS = VARIANT_GRAD_L2 | VARIANT_GRAD_SOBEL | VARIANT_GRAD_CLIP;
constexpr uint32_t VARIANT_SOLVE_BITS = VARIANT_UPDATE_DIV | VARIANT_INIT_UNIFORM;

// Optional per-image outputs of the batched form, indexed by the caller's slot.
struct BatchOut {
  uint16_t* luts;
  float* illum;
  float* refl;
  float* target;
  int32_t* passes;
};

// Header of the batched descriptor table (device copy written per call, so a
// captured launch graph serves every call; the cursors arrive as zeros).
struct BatchHeader {
  uint32_t next;         // histogram-item cursor
  uint32_t rhead;        // ready-list position being remapped
  int32_t n;             // images in this call
  int32_t total_tiles;   // histogram items over all images
  uint32_t nready;       // images in the ready list
  uint32_t exited;       // workgroups that have left the kernel (the last resets the cursors)
  int64_t tile_px;       // pixels per histogram item (multiple of the pixel step)
  int64_t rtile_px;      // pixels per remap item (multiple of the pixel step)
  SolveParams params;
  BatchOut out;
};

// Per-image counters of the batched form.  They sit in the descriptor table
// after the ImgDesc array and are uploaded as zeros with it on every call.
struct ImgCounters {
  uint32_t done;   // histogram items merged so far
  uint32_t fifo;   // ready list: entry at this position = published image + 1 (0: not yet)
  uint32_t rnext;  // remap tiles of this image claimed so far
  uint32_t pad;
};

// Per-image device state of the batched form, `words(bins)` 32-bit words.
// The partial slots are zero between calls: the workgroup that adds them up
// clears them again.
// Histogram items merge into one of NSLOT partial histograms (item mod
// NSLOT), which spreads their atomics; the workgroup that merges the image's
// last item adds the slots up in slot order.
struct ImageState {
  static constexpr int NSLOT = 8;
  uint32_t done;   // hr_build_hist_batch: histogram tiles merged so far
  uint32_t pad[3];
  static constexpr int64_t words(int bins) { return 4 + 5 * (int64_t)bins + bins / 2 + NSLOT * 3LL * bins; }
  __host__ __device__ uint32_t* base() { return reinterpret_cast<uint32_t*>(this); }
  __host__ __device__ uint32_t* hs() { return base() + 4; }
  __host__ __device__ uint32_t* graw(int bins) { return base() + 4 + bins; }
  __host__ __device__ uint32_t* hg(int bins) { return base() + 4 + 3 * bins; }
  __host__ __device__ float* target(int bins) { return reinterpret_cast<float*>(base() + 4 + 4 * bins); }
  __host__ __device__ uint16_t* lut(int bins) { return reinterpret_cast<uint16_t*>(base() + 4 + 5 * bins); }
  // partial histogram k: value histogram [bins] then raw gradient histogram [2 bins]
  __host__ __device__ uint32_t* slot(int bins, int k) { return base() + 4 + 5 * bins + bins / 2 + k * 3 * bins; }
};

// Allocation-free form of the batched call: the descriptor table travels as a
// kernel argument and every buffer the kernels need lives in one fixed device
// array of the library (per GPU), so at most NOALLOC_MAX_IMAGES images per call.
constexpr int NOALLOC_MAX_IMAGES = 4;
struct NoallocTable {
  BatchHeader hdr;
  ImgDesc desc[NOALLOC_MAX_IMAGES];
};

namespace launch {
hipError_t fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);
hipError_t hist(int bits, const ImgDesc& d, int64_t tile_px, uint32_t* hs, uint32_t* graw, uint32_t* hg,
                uint32_t* ticket, uint32_t* flags, hipStream_t s);
hipError_t hist_batch(int bits, int n, const ImgDesc* desc, int64_t max_tiles, int64_t tile_px, uint32_t* hs,
                      uint32_t* hg, ImageState* st, uint32_t* flags, hipStream_t s);
hipError_t solve(int bins, const uint32_t* hS, const uint32_t* hG, int64_t npix, const SolveParams& p,
                 float* illum, float* refl, float* target, int32_t* passes, uint32_t* flags, hipStream_t s);
hipError_t equalize_lut(int bins, const uint32_t* hS, uint16_t* lut, uint16_t* lut_user, hipStream_t s);
hipError_t lut(int bins, const uint32_t* hS, const float* target, uint16_t* lut, uint16_t* lut_user,
               hipStream_t s);
hipError_t remap(int bits, const ImgDesc& d, int64_t tile_px, const uint16_t* lut, hipStream_t s);
hipError_t batch(int bits, int grid, BatchHeader* hdr, const ImgDesc* desc, ImgCounters* ctr, ImageState* st,
                 uint32_t* flags, hipStream_t s);
// persistent workgroups of the batched kernel one CU can hold (its LDS and
// registers allow), 0 on a query failure
int batch_max_wg_per_cu(int bits);
int step_px(int bits);
int batch_step_px(int bits);
int max_width(int bits);
// differentiated form (256 levels)
hipError_t solve_ckpt(int n, const uint32_t* hv, const uint32_t* hg, const SolveParams& p, int ncp, float* ckpt,
                      float* target, uint32_t* flags, hipStream_t s);
hipError_t softmatch(int n, const ImgDesc* desc, int64_t max_npix, const uint32_t* hv, const float* target,
                     float* m_tab, unsigned long long* acc, double* loss, float* dtarget, hipStream_t s);
hipError_t solve_vjp(int n, const uint32_t* hv, const uint32_t* hg, const SolveParams& p, int ncp, const float* ckpt,
                     const float* dtarget, double* dalpha, double* dbeta, uint32_t* flags, hipStream_t s);
int diff_seg_max();
// variant readings (hr_variant.hip)
hipError_t hist_variant(int bits, const ImgDesc& d, int64_t tile_px, uint32_t variant, uint32_t* hs, uint32_t* graw,
                        uint32_t* hg, uint32_t* ticket, uint32_t* flags, hipStream_t s);
hipError_t solve_variant(int bins, const uint32_t* hS, const uint32_t* hG, int64_t npix, const SolveParams& p,
                         float* illum, float* refl, float* target, int32_t* passes, uint32_t* flags, hipStream_t s);
// The batched kernel on the library's own fixed scratch (no allocation): t
// holds the header and the n descriptors in queue order; flags_user (device,
// may be NULL) receives the sticky flags.  Calls on one GPU share the scratch.
hipError_t batch_noalloc(int bits, int grid_per_cu, const NoallocTable& t, uint32_t* flags_user, hipStream_t s);
int64_t noalloc_scratch_bytes();
}  // namespace launch

}  // namespace hr
