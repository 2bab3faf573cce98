// C ABI of the HistRetinex library: argument validation, the workspace,
// kernel launches and the captured launch graph of the batched form.
// Validation happens before anything is enqueued; HIP errors become
// HR_ERR_DEVICE with the runtime's text in hr_last_error().
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/histretinex.h"
#include "hr_launch.hpp"

namespace {

thread_local std::string g_err;

hr_status fail(hr_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HR_HIP(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess) return fail(HR_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr int kPlainTileSteps = 16;  // upper bound; small images take fewer
constexpr int kPlainWgPerCu = 4;     // one-image kernels aim for this many tiles per CU
constexpr int kDefaultTileSteps = 32;
constexpr int kDefaultWgPerCu = 1;
constexpr int kDefaultRemapSteps = 8;
constexpr int kStaging = 2;

// pixels per workgroup of the one-image kernels: at most kPlainTileSteps
// steps, fewer when that leaves less than kPlainWgPerCu tiles per CU, but at
// least min_steps (a histogram tile pays for clearing and merging its
// private histograms)
int64_t plain_tile_px(int bits, int64_t npix, int cu_count, int64_t min_steps) {
  const int64_t step = hr::launch::step_px(bits);
  const int64_t want = (int64_t)kPlainWgPerCu * std::max(cu_count, 1);
  const int64_t steps = std::max<int64_t>(min_steps, std::min<int64_t>(kPlainTileSteps, npix / (want * step)));
  return steps * step;
}

// differentiated form scratch: the soft map (256 floats) and the pixel-pass
// sums (257 u64) per image
constexpr int kDiffBins = 256;
size_t diff_map_bytes(int n) { return sizeof(float) * kDiffBins * (size_t)n; }
size_t diff_bytes(int max_images) {
  return diff_map_bytes(max_images) + sizeof(unsigned long long) * (kDiffBins + 1) * (size_t)max_images;
}

// descriptor table: BatchHeader, ImgDesc[max_images], ImgCounters[max_images]
size_t table_bytes(int max_images) {
  return sizeof(hr::BatchHeader) + (size_t)max_images * (sizeof(hr::ImgDesc) + sizeof(hr::ImgCounters));
}
size_t counters_offset(int max_images) { return sizeof(hr::BatchHeader) + (size_t)max_images * sizeof(hr::ImgDesc); }

struct GraphEntry {
  bool valid = false;
  int bits = 0;
  int grid = 0;
  hipGraphExec_t exec = nullptr;
};

}  // namespace

struct hr_workspace {
  int device = 0;
  int max_images = 0;
  int max_bins = 0;
  int cu_count = 0;
  int max_wg[2] = {1, 1};  // batched workgroups one CU holds, 8-bit / 10-bit kernel
  hr_schedule sched{kDefaultTileSteps, kDefaultWgPerCu, kDefaultRemapSteps};
  uint32_t* d_flags = nullptr;   // [0] sticky flags, [1] plain-hist ticket
  uint32_t* d_graw = nullptr;    // plain: raw gradient histogram scratch [2*max_bins]
  uint16_t* d_lut = nullptr;     // plain: LUT scratch [max_bins]
  uint8_t* d_table = nullptr;    // BatchHeader + ImgDesc[max_images] + ImgCounters[max_images]
  uint32_t* d_state = nullptr;   // ImageState per image
  // d_state's partial slots are zero in the layout of this bit depth (0: all
  // of d_state is zero, -1: unknown)
  int state_clean_bits = 0;
  uint8_t* d_diff = nullptr;     // differentiated form: soft map [max_images][256] float, sums [max_images][257] u64
  uint8_t* h_stage[kStaging] = {nullptr, nullptr};
  hipEvent_t ev[kStaging] = {nullptr, nullptr};
  bool ev_used[kStaging] = {false, false};
  int slot = 0;
  hipStream_t capture = nullptr;
  GraphEntry graphs[kStaging][2];
  // the descriptor table on the device as the last batched launch left it
  // (its kernel resets the cursors and counters on the way out), with the
  // bit depth, grid and stream of that launch; empty when unknown
  std::vector<uint8_t> last_table;
  int last_bits = 0, last_grid = 0;
  hipStream_t last_stream = nullptr;
};

namespace {

int elem_size(int bits) { return bits == 8 ? 1 : 2; }

hr_status check_bits(int32_t bits) {
  if (bits != 8 && bits != 10) return fail(HR_ERR_UNSUPPORTED, "bits must be 8 or 10");
  return HR_OK;
}

hr_status check_ws(hr_workspace* ws, int bins) {
  if (!ws) return fail(HR_ERR_INVALID_ARG, "workspace is NULL");
  if (bins > ws->max_bins) return fail(HR_ERR_WORKSPACE, "workspace was created for fewer bins");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != ws->device)
    return fail(HR_ERR_INVALID_ARG, "current HIP device differs from the workspace's device");
  return HR_OK;
}

// Validates one image and fills the kernel descriptor (in part).
hr_status make_desc(const hr_image* img, int bits, const char* what, hr::ImgDesc* d) {
  if (!img) return fail(HR_ERR_INVALID_ARG, std::string(what) + ": image descriptor is NULL");
  if (!img->data) return fail(HR_ERR_INVALID_ARG, std::string(what) + ": image data is NULL");
  if (img->width <= 0 || img->height <= 0)
    return fail(HR_ERR_INVALID_ARG, std::string(what) + ": width and height must be positive");
  if (img->width > hr::launch::max_width(bits))
    return fail(HR_ERR_UNSUPPORTED, std::string(what) + ": image wider than " +
                                        std::to_string(hr::launch::max_width(bits)) + " pixels");
  const int es = elem_size(bits);
  const int64_t row = 3LL * img->width * es;
  if (img->row_stride_bytes < row)
    return fail(HR_ERR_INVALID_ARG, std::string(what) + ": row stride smaller than 3 * width * element size");
  const uintptr_t addr = reinterpret_cast<uintptr_t>(img->data);
  if (es == 2 && ((addr & 1u) || (img->row_stride_bytes & 1)))
    return fail(HR_ERR_INVALID_ARG, std::string(what) + ": 16-bit image data and stride must be even");
  const int64_t npix = (int64_t)img->width * img->height;
  if (npix >= (1LL << 32) - 1) return fail(HR_ERR_UNSUPPORTED, std::string(what) + ": image has 2^32 or more pixels");
  std::memset(d, 0, sizeof(*d));
  d->in = static_cast<const uint8_t*>(img->data);
  d->in_stride = img->row_stride_bytes;
  d->npix = npix;
  d->W = img->width;
  d->H = img->height;
  d->in_vec = (img->row_stride_bytes == row) && ((addr & 15u) == 0);
  return HR_OK;
}

hr_status set_out(hr::ImgDesc* d, void* out, int64_t stride, int bits, const char* what) {
  if (!out) return fail(HR_ERR_INVALID_ARG, std::string(what) + ": output pointer is NULL");
  const int64_t row = 3LL * d->W * elem_size(bits);
  if (stride < row) return fail(HR_ERR_INVALID_ARG, std::string(what) + ": output row stride too small");
  const uintptr_t addr = reinterpret_cast<uintptr_t>(out);
  if (elem_size(bits) == 2 && ((addr & 1u) || (stride & 1)))
    return fail(HR_ERR_INVALID_ARG, std::string(what) + ": 16-bit output data and stride must be even");
  d->out = static_cast<uint8_t*>(out);
  d->out_stride = stride;
  d->out_vec = (stride == row) && ((addr & 15u) == 0);
  return HR_OK;
}

hr_status check_params(const hr_params* p, int bits) {
  if (!p) return fail(HR_ERR_INVALID_ARG, "params is NULL");
  if (p->bins != 256 && p->bins != 1024) return fail(HR_ERR_UNSUPPORTED, "bins must be 256 or 1024");
  if (bits && p->bins != (1 << bits)) return fail(HR_ERR_INVALID_ARG, "bins must equal 2^bits");
  if (p->iters < 0 || p->iters > 100000) return fail(HR_ERR_INVALID_ARG, "iters must be in 0..100000");
  if (!(std::isfinite(p->alpha) && p->alpha > 0)) return fail(HR_ERR_INVALID_ARG, "alpha must be finite and > 0");
  if (!(std::isfinite(p->beta) && p->beta > 0)) return fail(HR_ERR_INVALID_ARG, "beta must be finite and > 0");
  if (!(std::isfinite(p->gamma) && p->gamma > 0)) return fail(HR_ERR_INVALID_ARG, "gamma must be finite and > 0");
  if (!std::isfinite(p->eps)) return fail(HR_ERR_INVALID_ARG, "eps must be finite");
  if (p->variant & ~(hr::VARIANT_GRAD_BITS | hr::VARIANT_SOLVE_BITS))
    return fail(HR_ERR_UNSUPPORTED, "unknown variant bits");
  if ((p->variant & hr::VARIANT_GRAD_L2) && (p->variant & hr::VARIANT_GRAD_SOBEL))
    return fail(HR_ERR_INVALID_ARG, "HR_VARIANT_GRAD_L2 and HR_VARIANT_GRAD_SOBEL exclude each other");
  if (p->reserved != 0) return fail(HR_ERR_INVALID_ARG, "reserved field must be 0");
  return HR_OK;
}

// The batched and differentiated calls run the main path's readings only.
hr_status check_no_variant(const hr_params* p, const char* what) {
  if (p->variant != 0)
    return fail(HR_ERR_UNSUPPORTED, std::string(what) + ": variant readings run through the one-image calls "
                                                        "(hr_build_hist_variant, hr_solve)");
  return HR_OK;
}

hr::SolveParams solve_params(const hr_params* p) {
  hr::SolveParams sp{};
  sp.iters = p->iters;
  sp.alpha = (float)p->alpha;
  sp.beta = (float)p->beta;
  sp.inv_gamma = 1.0 / p->gamma;
  sp.eps = p->eps > 0 ? (float)p->eps : 0.f;
  sp.variant = p->variant & hr::VARIANT_SOLVE_BITS;
  return sp;
}

void release(hr_workspace* ws) {
  if (!ws) return;
  for (int s = 0; s < kStaging; ++s) {
    for (int b = 0; b < 2; ++b)
      if (ws->graphs[s][b].exec) (void)hipGraphExecDestroy(ws->graphs[s][b].exec);
    if (ws->ev[s]) (void)hipEventDestroy(ws->ev[s]);
    if (ws->h_stage[s]) (void)hipHostFree(ws->h_stage[s]);
  }
  if (ws->capture) (void)hipStreamDestroy(ws->capture);
  (void)hipFree(ws->d_flags);
  (void)hipFree(ws->d_graw);
  (void)hipFree(ws->d_lut);
  (void)hipFree(ws->d_table);
  (void)hipFree(ws->d_state);
  (void)hipFree(ws->d_diff);
  delete ws;
}

}  // namespace

extern "C" {

int32_t hr_abi_version(void) { return HR_ABI_VERSION; }

const char* hr_last_error(void) { return g_err.c_str(); }

const char* hr_status_string(hr_status s) {
  switch (s) {
    case HR_OK: return "ok";
    case HR_ERR_INVALID_ARG: return "invalid argument";
    case HR_ERR_UNSUPPORTED: return "unsupported";
    case HR_ERR_WORKSPACE: return "workspace too small";
    case HR_ERR_DEVICE: return "device error";
  }
  return "unknown status";
}

hr_status hr_workspace_create(int32_t max_images, int32_t max_bins, hr_workspace** out) {
  if (!out) return fail(HR_ERR_INVALID_ARG, "output pointer is NULL");
  *out = nullptr;
  if (max_images < 1 || max_images > 65536) return fail(HR_ERR_INVALID_ARG, "max_images must be in 1..65536");
  if (max_bins != 256 && max_bins != 1024) return fail(HR_ERR_UNSUPPORTED, "max_bins must be 256 or 1024");
  hr_workspace* ws = new (std::nothrow) hr_workspace();
  if (!ws) return fail(HR_ERR_DEVICE, "host allocation failed");
  ws->max_images = max_images;
  ws->max_bins = max_bins;
#define HR_HIP_WS(call)                                                                           \
  do {                                                                                            \
    hipError_t e_ = (call);                                                                       \
    if (e_ != hipSuccess) {                                                                       \
      release(ws);                                                                                \
      return fail(HR_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));              \
    }                                                                                             \
  } while (0)
  HR_HIP_WS(hipGetDevice(&ws->device));
  HR_HIP_WS(hipDeviceGetAttribute(&ws->cu_count, hipDeviceAttributeMultiprocessorCount, ws->device));
  for (int b = 0; b < 2; ++b) ws->max_wg[b] = std::max(1, hr::launch::batch_max_wg_per_cu(b == 0 ? 8 : 10));
  HR_HIP_WS(hipMalloc(&ws->d_flags, 64));
  HR_HIP_WS(hipMalloc(&ws->d_graw, sizeof(uint32_t) * 2 * max_bins));
  HR_HIP_WS(hipMalloc(&ws->d_lut, sizeof(uint16_t) * max_bins));
  HR_HIP_WS(hipMalloc(&ws->d_table, table_bytes(max_images)));
  HR_HIP_WS(hipMalloc(&ws->d_state, sizeof(uint32_t) * hr::ImageState::words(max_bins) * max_images));
  HR_HIP_WS(hipMalloc(&ws->d_diff, diff_bytes(max_images)));
  for (int s = 0; s < kStaging; ++s) {
    HR_HIP_WS(hipHostMalloc(&ws->h_stage[s], table_bytes(max_images), hipHostMallocDefault));
    std::memset(ws->h_stage[s], 0, table_bytes(max_images));
    HR_HIP_WS(hipEventCreateWithFlags(&ws->ev[s], hipEventDisableTiming));
  }
  HR_HIP_WS(hipStreamCreateWithFlags(&ws->capture, hipStreamNonBlocking));
  HR_HIP_WS(hipMemset(ws->d_flags, 0, 64));
  HR_HIP_WS(hipMemset(ws->d_state, 0, sizeof(uint32_t) * hr::ImageState::words(max_bins) * max_images));
  HR_HIP_WS(hipDeviceSynchronize());
#undef HR_HIP_WS
  *out = ws;
  return HR_OK;
}

void hr_workspace_destroy(hr_workspace* ws) {
  if (!ws) return;
  (void)hipDeviceSynchronize();
  release(ws);
}

hr_status hr_workspace_set_schedule(hr_workspace* ws, const hr_schedule* sched) {
  if (!ws || !sched) return fail(HR_ERR_INVALID_ARG, "NULL argument");
  if (sched->tile_steps < 0 || sched->tile_steps > 4096) return fail(HR_ERR_INVALID_ARG, "tile_steps out of range");
  if (sched->wg_per_cu < 0 || sched->wg_per_cu > 8) return fail(HR_ERR_INVALID_ARG, "wg_per_cu out of range");
  if (sched->remap_steps < 0 || sched->remap_steps > 4096) return fail(HR_ERR_INVALID_ARG, "remap_steps out of range");
  ws->sched.tile_steps = sched->tile_steps ? sched->tile_steps : kDefaultTileSteps;
  ws->sched.wg_per_cu = sched->wg_per_cu ? sched->wg_per_cu : kDefaultWgPerCu;
  ws->sched.remap_steps = sched->remap_steps ? sched->remap_steps : kDefaultRemapSteps;
  return HR_OK;
}

hr_status hr_get_flags(hr_workspace* ws, uint32_t* flags, int32_t clear) {
  if (!ws || !flags) return fail(HR_ERR_INVALID_ARG, "NULL argument");
  HR_HIP(hipDeviceSynchronize());
  HR_HIP(hipMemcpy(flags, ws->d_flags, sizeof(uint32_t), hipMemcpyDeviceToHost));
  if (clear) HR_HIP(hipMemset(ws->d_flags, 0, sizeof(uint32_t)));
  return HR_OK;
}

hr_status hr_build_hist(const hr_image* img, int32_t bits, uint32_t* hist_v, uint32_t* hist_grad,
                        uint32_t* hist_grad_raw, hr_workspace* ws, void* stream) {
  hr_status st = check_bits(bits);
  if (st) return st;
  const int bins = 1 << bits;
  hr::ImgDesc d;
  if ((st = make_desc(img, bits, "hr_build_hist", &d))) return st;
  if (!hist_v || !hist_grad) return fail(HR_ERR_INVALID_ARG, "hr_build_hist: histogram pointer is NULL");
  if ((st = check_ws(ws, bins))) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint32_t* graw = hist_grad_raw ? hist_grad_raw : ws->d_graw;
  HR_HIP(hr::launch::fill_u32(hist_v, bins, 0, s));
  HR_HIP(hr::launch::fill_u32(graw, 2 * bins - 1, 0, s));
  const int64_t tile_px = plain_tile_px(bits, d.npix, ws->cu_count, 8);
  HR_HIP(hr::launch::hist(bits, d, tile_px, hist_v, graw, hist_grad, ws->d_flags + 1, ws->d_flags, s));
  return HR_OK;
}

hr_status hr_build_hist_variant(const hr_image* img, int32_t bits, uint32_t variant, uint32_t* hist_v,
                                uint32_t* hist_grad, uint32_t* hist_grad_raw, hr_workspace* ws, void* stream) {
  if (variant & ~hr::VARIANT_GRAD_BITS)
    return fail(HR_ERR_INVALID_ARG, "hr_build_hist_variant: only gradient variant bits belong here");
  if ((variant & hr::VARIANT_GRAD_L2) && (variant & hr::VARIANT_GRAD_SOBEL))
    return fail(HR_ERR_INVALID_ARG, "HR_VARIANT_GRAD_L2 and HR_VARIANT_GRAD_SOBEL exclude each other");
  if (variant == 0) return hr_build_hist(img, bits, hist_v, hist_grad, hist_grad_raw, ws, stream);
  hr_status st = check_bits(bits);
  if (st) return st;
  const int bins = 1 << bits;
  hr::ImgDesc d;
  if ((st = make_desc(img, bits, "hr_build_hist_variant", &d))) return st;
  if (!hist_v || !hist_grad) return fail(HR_ERR_INVALID_ARG, "hr_build_hist_variant: histogram pointer is NULL");
  if ((st = check_ws(ws, bins))) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint32_t* graw = hist_grad_raw ? hist_grad_raw : ws->d_graw;
  HR_HIP(hr::launch::fill_u32(hist_v, bins, 0, s));
  HR_HIP(hr::launch::fill_u32(graw, 2 * bins - 1, 0, s));
  constexpr int64_t kVariantTilePx = 256 * 16;
  HR_HIP(hr::launch::hist_variant(bits, d, kVariantTilePx, variant, hist_v, graw, hist_grad, ws->d_flags + 1,
                                  ws->d_flags, s));
  return HR_OK;
}

hr_status hr_build_hist_batch(const hr_image* in, int32_t n, int32_t bits, uint32_t* hist_v, uint32_t* hist_grad,
                              hr_workspace* ws, void* stream) {
  hr_status st = check_bits(bits);
  if (st) return st;
  const int bins = 1 << bits;
  if (!in || !hist_v || !hist_grad) return fail(HR_ERR_INVALID_ARG, "hr_build_hist_batch: NULL pointer");
  if (n < 1) return fail(HR_ERR_INVALID_ARG, "hr_build_hist_batch: n must be >= 1");
  std::vector<hr::ImgDesc> descs((size_t)n);
  int64_t max_npix = 0, total = 0;
  for (int i = 0; i < n; ++i) {
    if ((st = make_desc(&in[i], bits, "hr_build_hist_batch", &descs[i]))) return st;
    max_npix = std::max(max_npix, descs[i].npix);
    total += descs[i].npix;
  }
  if ((st = check_ws(ws, bins))) return st;
  if (n > ws->max_images) return fail(HR_ERR_WORKSPACE, "hr_build_hist_batch: n exceeds the workspace's max_images");
  // tiles sized on the whole batch: a few per compute unit
  const int64_t tile_px = plain_tile_px(bits, total, ws->cu_count, 8);
  const int64_t max_tiles = (max_npix + tile_px - 1) / tile_px;
  if (max_tiles > (1LL << 31) - 1 || n > 65535) return fail(HR_ERR_UNSUPPORTED, "hr_build_hist_batch: grid too large");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int slot = ws->slot;
  if (ws->ev_used[slot]) HR_HIP(hipEventSynchronize(ws->ev[slot]));
  uint8_t* stage = ws->h_stage[slot];
  std::memcpy(stage, descs.data(), sizeof(hr::ImgDesc) * (size_t)n);
  auto* desc_d = reinterpret_cast<hr::ImgDesc*>(ws->d_table + sizeof(hr::BatchHeader));
  ws->last_table.clear();  // the batched form's table is overwritten
  HR_HIP(hipMemcpyAsync(desc_d, stage, sizeof(hr::ImgDesc) * (size_t)n, hipMemcpyHostToDevice, s));
  auto* st_d = reinterpret_cast<hr::ImageState*>(ws->d_state);
  HR_HIP(hr::launch::fill_u32(hist_v, (int64_t)n * bins, 0, s));
  HR_HIP(hr::launch::fill_u32(ws->d_state, (int64_t)n * hr::ImageState::words(bins), 0, s));
  HR_HIP(hr::launch::hist_batch(bits, n, desc_d, max_tiles, tile_px, hist_v, hist_grad, st_d, ws->d_flags, s));
  // images < n: slots zero in this layout; the rest as before
  ws->state_clean_bits = (ws->state_clean_bits == 0 || ws->state_clean_bits == bits) ? bits : -1;
  HR_HIP(hipEventRecord(ws->ev[slot], s));
  ws->ev_used[slot] = true;
  ws->slot = (slot + 1) % kStaging;
  return HR_OK;
}

hr_status hr_solve(const uint32_t* hist_v, const uint32_t* hist_grad, int64_t npix, const hr_params* p,
                   float* illum, float* refl, float* target, int32_t* passes, hr_workspace* ws, void* stream) {
  hr_status st = check_params(p, 0);
  if (st) return st;
  if (!hist_v || !hist_grad) return fail(HR_ERR_INVALID_ARG, "hr_solve: histogram pointer is NULL");
  if (!illum || !refl || !target) return fail(HR_ERR_INVALID_ARG, "hr_solve: output pointer is NULL");
  if (npix <= 0 || npix >= (1LL << 32) - 1) return fail(HR_ERR_INVALID_ARG, "hr_solve: npix out of range");
  if (p->variant & hr::VARIANT_GRAD_BITS)
    return fail(HR_ERR_INVALID_ARG, "hr_solve: gradient variant bits belong to hr_build_hist_variant");
  if ((st = check_ws(ws, p->bins))) return st;
  const hr::SolveParams sp = solve_params(p);
  if (sp.variant) {
    HR_HIP(hr::launch::solve_variant(p->bins, hist_v, hist_grad, npix, sp, illum, refl, target, passes, ws->d_flags,
                                     static_cast<hipStream_t>(stream)));
    return HR_OK;
  }
  HR_HIP(hr::launch::solve(p->bins, hist_v, hist_grad, npix, sp, illum, refl, target, passes,
                           ws->d_flags, static_cast<hipStream_t>(stream)));
  return HR_OK;
}

hr_status hr_match(const hr_image* in, int32_t bits, const uint32_t* hist_v, const float* target, void* out,
                   int64_t out_row_stride_bytes, uint16_t* lut_out, hr_workspace* ws, void* stream) {
  hr_status st = check_bits(bits);
  if (st) return st;
  const int bins = 1 << bits;
  hr::ImgDesc d;
  if ((st = make_desc(in, bits, "hr_match", &d))) return st;
  if ((st = set_out(&d, out, out_row_stride_bytes, bits, "hr_match"))) return st;
  if (!hist_v || !target) return fail(HR_ERR_INVALID_ARG, "hr_match: histogram pointer is NULL");
  if ((st = check_ws(ws, bins))) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  HR_HIP(hr::launch::lut(bins, hist_v, target, ws->d_lut, lut_out, s));
  const int64_t tile_px = plain_tile_px(bits, d.npix, ws->cu_count, 1);
  HR_HIP(hr::launch::remap(bits, d, tile_px, ws->d_lut, s));
  return HR_OK;
}

hr_status hr_equalize(const hr_image* in, int32_t bits, const uint32_t* hist_v, void* out,
                      int64_t out_row_stride_bytes, uint16_t* lut_out, hr_workspace* ws, void* stream) {
  hr_status st = check_bits(bits);
  if (st) return st;
  const int bins = 1 << bits;
  hr::ImgDesc d;
  if ((st = make_desc(in, bits, "hr_equalize", &d))) return st;
  if ((st = set_out(&d, out, out_row_stride_bytes, bits, "hr_equalize"))) return st;
  if (!hist_v) return fail(HR_ERR_INVALID_ARG, "hr_equalize: histogram pointer is NULL");
  if ((st = check_ws(ws, bins))) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  HR_HIP(hr::launch::equalize_lut(bins, hist_v, ws->d_lut, lut_out, s));
  const int64_t tile_px = plain_tile_px(bits, d.npix, ws->cu_count, 1);
  HR_HIP(hr::launch::remap(bits, d, tile_px, ws->d_lut, s));
  return HR_OK;
}

hr_status hr_enhance_batch(const hr_image* in, void* const* out, const int64_t* out_row_stride_bytes, int32_t n,
                           int32_t bits, const hr_params* p, uint16_t* luts, float* illum, float* refl,
                           float* target, int32_t* passes, hr_workspace* ws, void* stream) {
  hr_status st = check_bits(bits);
  if (st) return st;
  if ((st = check_params(p, bits))) return st;
  if ((st = check_no_variant(p, "hr_enhance_batch"))) return st;
  const int bins = 1 << bits;
  if (!in || !out || !out_row_stride_bytes) return fail(HR_ERR_INVALID_ARG, "hr_enhance_batch: NULL array");
  if (n < 1) return fail(HR_ERR_INVALID_ARG, "hr_enhance_batch: n must be >= 1");
  std::vector<hr::ImgDesc> descs((size_t)n);
  for (int i = 0; i < n; ++i) {
    if ((st = make_desc(&in[i], bits, "hr_enhance_batch", &descs[i]))) return st;
    if ((st = set_out(&descs[i], out[i], out_row_stride_bytes[i], bits, "hr_enhance_batch"))) return st;
    descs[i].slot = i;
  }
  if ((st = check_ws(ws, bins))) return st;
  if (n > ws->max_images) return fail(HR_ERR_WORKSPACE, "hr_enhance_batch: n exceeds the workspace's max_images");
  // largest image first, so the last solves to start belong to small images
  std::vector<int> order((size_t)n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return descs[a].npix > descs[b].npix; });
  const int64_t tile_px = (int64_t)ws->sched.tile_steps * hr::launch::batch_step_px(bits);
  const int64_t rtile_px = (int64_t)ws->sched.remap_steps * hr::launch::batch_step_px(bits);
  int64_t tiles = 0, rtiles = 0;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int slot = ws->slot;
  if (ws->ev_used[slot]) HR_HIP(hipEventSynchronize(ws->ev[slot]));
  uint8_t* stage = ws->h_stage[slot];
  hr::ImgDesc* sd = reinterpret_cast<hr::ImgDesc*>(stage + sizeof(hr::BatchHeader));
  for (int k = 0; k < n; ++k) {
    hr::ImgDesc d = descs[order[k]];
    d.ntiles = (int32_t)((d.npix + tile_px - 1) / tile_px);
    d.tile0 = (int32_t)tiles;
    d.rtiles = (int32_t)((d.npix + rtile_px - 1) / rtile_px);
    tiles += d.ntiles;
    rtiles += d.rtiles;
    if (tiles + rtiles > (1LL << 30)) return fail(HR_ERR_UNSUPPORTED, "hr_enhance_batch: too many tiles");
    sd[k] = d;
  }
  // per-image counters start at zero on every call (uploaded with the table)
  std::memset(stage + counters_offset(ws->max_images), 0, sizeof(hr::ImgCounters) * (size_t)n);
  hr::BatchHeader hdr{};
  hdr.n = n;
  hdr.total_tiles = (int32_t)tiles;
  hdr.tile_px = tile_px;
  hdr.rtile_px = rtile_px;
  hdr.params = solve_params(p);
  hdr.out = hr::BatchOut{luts, illum, refl, target, passes};
  std::memcpy(stage, &hdr, sizeof(hdr));

  // more persistent workgroups than the CUs can hold at once would only queue
  // behind the resident ones
  const int grid = std::max(1, ws->cu_count * std::min(ws->sched.wg_per_cu, ws->max_wg[bits == 8 ? 0 : 1]));
  auto* hdr_d = reinterpret_cast<hr::BatchHeader*>(ws->d_table);
  auto* desc_d = reinterpret_cast<hr::ImgDesc*>(ws->d_table + sizeof(hr::BatchHeader));
  auto* ctr_d = reinterpret_cast<hr::ImgCounters*>(ws->d_table + counters_offset(ws->max_images));
  auto* st_d = reinterpret_cast<hr::ImageState*>(ws->d_state);
  const size_t tbytes = table_bytes(ws->max_images);
  if (ws->last_bits == bits && ws->last_grid == grid && ws->last_stream == s && ws->last_table.size() == tbytes &&
      std::memcmp(ws->last_table.data(), stage, tbytes) == 0 && ws->state_clean_bits == bits) {
    // the same table as the last launch on this stream, which reset its
    // cursors and counters when it ended: the kernel alone, no upload
    HR_HIP(hr::launch::batch(bits, grid, hdr_d, desc_d, ctr_d, st_d, ws->d_flags, s));
    return HR_OK;
  }
  ws->last_table.clear();
  GraphEntry& g = ws->graphs[slot][bits == 8 ? 0 : 1];
  if (!g.valid || g.grid != grid) {
    if (g.exec) {
      (void)hipGraphExecDestroy(g.exec);
      g.exec = nullptr;
      g.valid = false;
    }
    hipGraph_t graph = nullptr;
    HR_HIP(hipStreamBeginCapture(ws->capture, hipStreamCaptureModeThreadLocal));
    hipError_t e1 = hipMemcpyAsync(ws->d_table, stage, table_bytes(ws->max_images), hipMemcpyHostToDevice, ws->capture);
    hipError_t e3 = e1 == hipSuccess ? hr::launch::batch(bits, grid, hdr_d, desc_d, ctr_d, st_d, ws->d_flags,
                                                        ws->capture)
                                     : e1;
    hipError_t e4 = hipStreamEndCapture(ws->capture, &graph);
    if (e3 != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return fail(HR_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e3));
    }
    if (e4 != hipSuccess) return fail(HR_ERR_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e4));
    hipError_t e5 = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e5 != hipSuccess) return fail(HR_ERR_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e5));
    g.valid = true;
    g.bits = bits;
    g.grid = grid;
  }
  if (ws->state_clean_bits != 0 && ws->state_clean_bits != bits) {
    // another layout left data where this one's partial slots are
    HR_HIP(hr::launch::fill_u32(ws->d_state, hr::ImageState::words(ws->max_bins) * ws->max_images, 0, s));
  }
  ws->state_clean_bits = bits;
  HR_HIP(hipGraphLaunch(g.exec, s));
  HR_HIP(hipEventRecord(ws->ev[slot], s));
  ws->ev_used[slot] = true;
  ws->slot = (slot + 1) % kStaging;
  ws->last_table.assign(stage, stage + tbytes);
  ws->last_bits = bits;
  ws->last_grid = grid;
  ws->last_stream = s;
  return HR_OK;
}

hr_status hr_enhance_batch_noalloc(const hr_image* in, void* const* out, const int64_t* out_row_stride_bytes,
                                   int32_t n, int32_t bits, const hr_params* p, uint16_t* luts, float* illum,
                                   float* refl, float* target, int32_t* passes, uint32_t* flags, void* stream) {
  static_assert(HR_NOALLOC_MAX_IMAGES == hr::NOALLOC_MAX_IMAGES, "header and library agree on the limit");
  hr_status st = check_bits(bits);
  if (st) return st;
  if ((st = check_params(p, bits))) return st;
  if ((st = check_no_variant(p, "hr_enhance_batch_noalloc"))) return st;
  if (!in || !out || !out_row_stride_bytes) return fail(HR_ERR_INVALID_ARG, "hr_enhance_batch_noalloc: NULL array");
  if (n < 1) return fail(HR_ERR_INVALID_ARG, "hr_enhance_batch_noalloc: n must be >= 1");
  if (n > hr::NOALLOC_MAX_IMAGES)
    return fail(HR_ERR_UNSUPPORTED, "hr_enhance_batch_noalloc: n exceeds HR_NOALLOC_MAX_IMAGES (" +
                                        std::to_string(hr::NOALLOC_MAX_IMAGES) + ")");
  hr::ImgDesc descs[hr::NOALLOC_MAX_IMAGES];
  for (int i = 0; i < n; ++i) {
    if ((st = make_desc(&in[i], bits, "hr_enhance_batch_noalloc", &descs[i]))) return st;
    if ((st = set_out(&descs[i], out[i], out_row_stride_bytes[i], bits, "hr_enhance_batch_noalloc"))) return st;
    descs[i].slot = i;
  }
  // the queue order and item sizes of hr_enhance_batch with the default schedule
  int order[hr::NOALLOC_MAX_IMAGES];
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order, order + n, [&](int a, int b) { return descs[a].npix > descs[b].npix; });
  const int64_t tile_px = (int64_t)kDefaultTileSteps * hr::launch::batch_step_px(bits);
  const int64_t rtile_px = (int64_t)kDefaultRemapSteps * hr::launch::batch_step_px(bits);
  hr::NoallocTable t{};
  int64_t tiles = 0;
  for (int k = 0; k < n; ++k) {
    hr::ImgDesc d = descs[order[k]];
    d.ntiles = (int32_t)((d.npix + tile_px - 1) / tile_px);
    d.tile0 = (int32_t)tiles;
    d.rtiles = (int32_t)((d.npix + rtile_px - 1) / rtile_px);
    tiles += d.ntiles;
    t.desc[k] = d;
  }
  t.hdr.n = n;
  t.hdr.total_tiles = (int32_t)tiles;
  t.hdr.tile_px = tile_px;
  t.hdr.rtile_px = rtile_px;
  t.hdr.params = solve_params(p);
  t.hdr.out = hr::BatchOut{luts, illum, refl, target, passes};
  HR_HIP(hr::launch::batch_noalloc(bits, kDefaultWgPerCu, t, flags, static_cast<hipStream_t>(stream)));
  return HR_OK;
}

// ---- differentiated form -------------------------------------------------------

static hr_status check_diff(const hr_params* p, int32_t n, int32_t ckpt_every, const char* what) {
  hr_status st = check_params(p, 8);
  if (st) return st;
  if ((st = check_no_variant(p, what))) return st;
  if (p->eps > 0)
    return fail(HR_ERR_UNSUPPORTED, std::string(what) + ": the differentiated form runs exactly iters passes (eps <= 0)");
  if (n < 1) return fail(HR_ERR_INVALID_ARG, std::string(what) + ": n must be >= 1");
  if (ckpt_every < 1 || ckpt_every > hr::launch::diff_seg_max())
    return fail(HR_ERR_INVALID_ARG, std::string(what) + ": ckpt_every must be in 1.." +
                                        std::to_string(hr::launch::diff_seg_max()));
  if (p->iters % ckpt_every != 0)
    return fail(HR_ERR_INVALID_ARG, std::string(what) + ": iters must be a multiple of ckpt_every");
  return HR_OK;
}

hr_status hr_solve_ckpt(const uint32_t* hist_v, const uint32_t* hist_grad, int32_t n, const hr_params* p,
                        int32_t ckpt_every, float* ckpt, float* target, hr_workspace* ws, void* stream) {
  hr_status st = check_diff(p, n, ckpt_every, "hr_solve_ckpt");
  if (st) return st;
  if (!hist_v || !hist_grad || !ckpt || !target) return fail(HR_ERR_INVALID_ARG, "hr_solve_ckpt: NULL pointer");
  if ((st = check_ws(ws, 256))) return st;
  if (n > ws->max_images) return fail(HR_ERR_WORKSPACE, "hr_solve_ckpt: n exceeds the workspace's max_images");
  hr::SolveParams sp = solve_params(p);
  sp.ckpt_every = ckpt_every;
  HR_HIP(hr::launch::solve_ckpt(n, hist_v, hist_grad, sp, p->iters / ckpt_every + 1, ckpt, target, ws->d_flags,
                                static_cast<hipStream_t>(stream)));
  return HR_OK;
}

hr_status hr_softmatch_loss_grad(const hr_image* in, const float* const* target_img, int32_t n,
                                 const uint32_t* hist_v, const float* target, double* loss, float* dtarget,
                                 hr_workspace* ws, void* stream) {
  if (n < 1) return fail(HR_ERR_INVALID_ARG, "hr_softmatch_loss_grad: n must be >= 1");
  if (!in || !target_img || !hist_v || !target || !loss || !dtarget)
    return fail(HR_ERR_INVALID_ARG, "hr_softmatch_loss_grad: NULL pointer");
  std::vector<hr::ImgDesc> descs((size_t)n);
  int64_t max_npix = 0;
  hr_status st;
  for (int i = 0; i < n; ++i) {
    if ((st = make_desc(&in[i], 8, "hr_softmatch_loss_grad", &descs[i]))) return st;
    const uintptr_t a = reinterpret_cast<uintptr_t>(target_img[i]);
    if (!a || (a & 3u)) return fail(HR_ERR_INVALID_ARG, "hr_softmatch_loss_grad: target image NULL or misaligned");
    descs[i].out = reinterpret_cast<uint8_t*>(const_cast<float*>(target_img[i]));
    descs[i].out_stride = 12LL * descs[i].W;
    descs[i].slot = i;
    max_npix = std::max(max_npix, descs[i].npix);
  }
  if ((st = check_ws(ws, 256))) return st;
  if (n > ws->max_images) return fail(HR_ERR_WORKSPACE, "hr_softmatch_loss_grad: n exceeds the workspace's max_images");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int slot = ws->slot;
  if (ws->ev_used[slot]) HR_HIP(hipEventSynchronize(ws->ev[slot]));
  uint8_t* stage = ws->h_stage[slot];
  std::memcpy(stage, descs.data(), sizeof(hr::ImgDesc) * (size_t)n);
  auto* desc_d = reinterpret_cast<hr::ImgDesc*>(ws->d_table + sizeof(hr::BatchHeader));
  ws->last_table.clear();  // the batched form's table is overwritten
  HR_HIP(hipMemcpyAsync(desc_d, stage, sizeof(hr::ImgDesc) * (size_t)n, hipMemcpyHostToDevice, s));
  auto* m_tab = reinterpret_cast<float*>(ws->d_diff);
  auto* acc = reinterpret_cast<unsigned long long*>(ws->d_diff + diff_map_bytes(ws->max_images));
  HR_HIP(hr::launch::softmatch(n, desc_d, max_npix, hist_v, target, m_tab, acc, loss, dtarget, s));
  HR_HIP(hipEventRecord(ws->ev[slot], s));
  ws->ev_used[slot] = true;
  ws->slot = (slot + 1) % kStaging;
  return HR_OK;
}

hr_status hr_solve_vjp(const uint32_t* hist_v, const uint32_t* hist_grad, int32_t n, const hr_params* p,
                       int32_t ckpt_every, const float* ckpt, const float* dtarget, double* dalpha, double* dbeta,
                       hr_workspace* ws, void* stream) {
  hr_status st = check_diff(p, n, ckpt_every, "hr_solve_vjp");
  if (st) return st;
  if (!hist_v || !hist_grad || !ckpt || !dtarget || !dalpha || !dbeta)
    return fail(HR_ERR_INVALID_ARG, "hr_solve_vjp: NULL pointer");
  if ((st = check_ws(ws, 256))) return st;
  if (n > ws->max_images) return fail(HR_ERR_WORKSPACE, "hr_solve_vjp: n exceeds the workspace's max_images");
  hr::SolveParams sp = solve_params(p);
  sp.ckpt_every = ckpt_every;
  HR_HIP(hr::launch::solve_vjp(n, hist_v, hist_grad, sp, p->iters / ckpt_every + 1, ckpt, dtarget, dalpha, dbeta,
                               ws->d_flags, static_cast<hipStream_t>(stream)));
  return HR_OK;
}

}  // extern "C"
