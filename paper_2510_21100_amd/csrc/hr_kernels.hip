// Kernels of the HistRetinex pipeline for gfx950 and their launchers.
//
// One-image form: fill -> hist (last workgroup rescales the gradient
// histogram) -> solve (one workgroup) -> lut (one workgroup) -> remap.
// Batched form: one persistent kernel over a shared work queue holding every
// histogram tile of every image (largest image first) followed by every remap
// tile; the workgroup that finishes the last histogram tile of an image runs
// that image's solve and LUT and publishes it; remap tiles wait for it.
#include "hr_device.hpp"
#include "hr_launch.hpp"

#include <algorithm>

namespace hr {

// ---------------------------------------------------------------------------
// one-image kernels
// ---------------------------------------------------------------------------

__global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

template <int BITS>
__global__ __launch_bounds__(NT_PIX) void k_hist(ImgDesc d, int64_t tile_px, uint32_t* hs, uint32_t* graw,
                                                 uint32_t* hg, uint32_t* ticket, uint32_t* flags) {
  constexpr int BINS = Cfg<BITS>::BINS;
  __shared__ HistSmem<BITS> sm;
  __shared__ uint32_t red[NT_PIX / 64];
  __shared__ uint32_t last;
  const int64_t P0 = (int64_t)blockIdx.x * tile_px;
  const int64_t P1 = min(P0 + tile_px, d.npix);
  hist_tile<BITS, NT_PIX>(d, P0, P1, sm, hs, graw);
  if (threadIdx.x == 0) {
    if (sm.clamped) atomicOr(flags, FLAG_VALUE_CLAMPED);
    __threadfence();
    last = (atomicAdd(ticket, 1u) == gridDim.x - 1) ? 1u : 0u;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  rebin_gradient<BINS, NT_PIX>(graw, hg, sm.hs, red);
  if (threadIdx.x == 0) *ticket = 0;  // ready for the next call
}

template <int BINS, int NT>
__global__ __launch_bounds__(NT) void k_solve(const uint32_t* hS, const uint32_t* hG, int64_t npix, SolveParams p,
                                              uint32_t* lists, float* illum, float* refl, float* target,
                                              uint32_t* flags) {
  __shared__ SolveSmem<BINS, NT> sm;
  solve_image<BINS, NT>(hS, hG, npix, p, sm, lists, illum, refl, target, nullptr, flags);
}

template <int BINS, int NT>
__global__ __launch_bounds__(NT) void k_lut(const uint32_t* hS, const float* target, uint16_t* lut,
                                            uint16_t* lut_user) {
  __shared__ LutSmem<BINS, NT> sm;
  build_lut<BINS, NT>(hS, target, sm, lut);
  if (lut_user) {
    __syncthreads();
    for (int k = threadIdx.x; k < BINS; k += NT) lut_user[k] = lut[k];
  }
}

template <int BITS>
__global__ __launch_bounds__(NT_PIX) void k_remap(ImgDesc d, int64_t tile_px, const uint16_t* lut) {
  constexpr int BINS = Cfg<BITS>::BINS;
  __shared__ uint2 tab[BINS];
  load_remap_table<BINS, NT_PIX>(lut, tab);
  __syncthreads();
  const int64_t P0 = (int64_t)blockIdx.x * tile_px;
  const int64_t P1 = min(P0 + tile_px, d.npix);
  remap_tile<BITS, NT_PIX>(d, P0, P1, tab);
}

// ---------------------------------------------------------------------------
// batched persistent kernel
// ---------------------------------------------------------------------------

template <int BITS>
union BatchSmem {
  HistSmem<BITS> hist;
  SolveSmem<Cfg<BITS>::BINS, NT_PIX> solve;
  LutSmem<Cfg<BITS>::BINS, NT_PIX> lut;
  uint2 tab[Cfg<BITS>::BINS];
};

__global__ void k_batch_reset(BatchHeader* hdr, ImageState* st, int bins) {
  const int n = hdr->n;
  const int64_t words = (int64_t)n * ImageState::words(bins);
  uint32_t* base = reinterpret_cast<uint32_t*>(st);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x)
    base[i] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) hdr->next = 0;
}

// image owning batch tile `tile` (tile0 ascending over the descriptor table)
__device__ inline int image_of_tile(const ImgDesc* desc, int n, int tile) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int BITS>
__global__ __launch_bounds__(NT_PIX) void k_batch(BatchHeader* hdr, const ImgDesc* desc, ImageState* st,
                                                  uint32_t* lists_base, int64_t lists_stride, uint32_t* flags) {
  constexpr int BINS = Cfg<BITS>::BINS;
  __shared__ BatchSmem<BITS> sm;
  __shared__ uint32_t red[NT_PIX / 64];
  __shared__ int item_s;
  __shared__ uint32_t last_s;
  const int n = hdr->n;
  const int ht = hdr->total_tiles;
  const int64_t tile_px = hdr->tile_px;
  const SolveParams p = hdr->params;
  const BatchOut out = hdr->out;
  const int64_t st_words = ImageState::words(BINS);
  for (;;) {
    if (threadIdx.x == 0) item_s = (int)atomicAdd(&hdr->next, 1u);
    __syncthreads();
    const int item = item_s;
    __syncthreads();
    if (item >= 2 * ht) break;
    const bool is_hist = item < ht;
    const int tile = is_hist ? item : item - ht;
    const int i = image_of_tile(desc, n, tile);
    const ImgDesc d = desc[i];
    ImageState* s = reinterpret_cast<ImageState*>(reinterpret_cast<uint32_t*>(st) + i * st_words);
    uint32_t* hs = s->hs();
    uint32_t* graw = s->graw(BINS);
    const int64_t P0 = (int64_t)(tile - d.tile0) * tile_px;
    const int64_t P1 = min(P0 + tile_px, d.npix);
    if (is_hist) {
      hist_tile<BITS, NT_PIX>(d, P0, P1, sm.hist, hs, graw);
      if (threadIdx.x == 0) {
        if (sm.hist.clamped) atomicOr(flags, FLAG_VALUE_CLAMPED);
        __threadfence();
        last_s = (atomicAdd(&s->done, 1u) == (uint32_t)d.ntiles - 1) ? 1u : 0u;
      }
      __syncthreads();
      if (last_s) {
        __threadfence();
        uint32_t* hg = s->hg(BINS);
        rebin_gradient<BINS, NT_PIX>(graw, hg, reinterpret_cast<uint32_t*>(&sm), red);
        __threadfence();
        __syncthreads();
        __threadfence();
        float* tgt = s->target(BINS);
        solve_image<BINS, NT_PIX>(hs, hg, d.npix, p, sm.solve, lists_base + (int64_t)i * lists_stride,
                                  out.illum ? out.illum + (int64_t)d.slot * BINS : nullptr,
                                  out.refl ? out.refl + (int64_t)d.slot * BINS : nullptr, tgt, nullptr,
                                  flags);
        __threadfence();
        __syncthreads();
        __threadfence();
        uint16_t* lut = s->lut(BINS);
        build_lut<BINS, NT_PIX>(hs, tgt, sm.lut, lut);
        __syncthreads();
        if (out.target || out.luts) {
          for (int k = threadIdx.x; k < BINS; k += NT_PIX) {
            if (out.target) out.target[(int64_t)d.slot * BINS + k] = tgt[k];
            if (out.luts) out.luts[(int64_t)d.slot * BINS + k] = lut[k];
          }
        }
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0) __hip_atomic_store(&s->ready, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      }
    } else {
      if (threadIdx.x == 0) {
        while (__hip_atomic_load(&s->ready, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0u)
          __builtin_amdgcn_s_sleep(2);
      }
      __syncthreads();
      __threadfence();
      const uint16_t* lut = s->lut(BINS);
      for (int v = threadIdx.x; v < BINS; v += NT_PIX) {
        const uint32_t L = __hip_atomic_load(reinterpret_cast<const uint32_t*>(lut) + (v >> 1), __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t lv = (v & 1) ? (L >> 16) : (L & 0xffffu);
        const uint32_t m = v ? (uint32_t)((0xffffffffull + 2ull * v) / (2ull * v)) : 0u;
        sm.tab[v] = make_uint2(m, lv);
      }
      __syncthreads();
      remap_tile<BITS, NT_PIX>(d, P0, P1, sm.tab);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

namespace launch {

hipError_t fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int blocks = (int)std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_fill_u32, dim3(blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t hist(int bits, const ImgDesc& d, int64_t tile_px, uint32_t* hs, uint32_t* graw, uint32_t* hg,
                uint32_t* ticket, uint32_t* flags, hipStream_t s) {
  const int64_t tiles = (d.npix + tile_px - 1) / tile_px;
  if (bits == 8)
    hipLaunchKernelGGL(k_hist<8>, dim3((unsigned)tiles), dim3(NT_PIX), 0, s, d, tile_px, hs, graw, hg, ticket,
                       flags);
  else
    hipLaunchKernelGGL(k_hist<10>, dim3((unsigned)tiles), dim3(NT_PIX), 0, s, d, tile_px, hs, graw, hg, ticket,
                       flags);
  return hipGetLastError();
}

hipError_t solve(int bins, const uint32_t* hS, const uint32_t* hG, int64_t npix, const SolveParams& p,
                 uint32_t* lists, float* illum, float* refl, float* target, uint32_t* flags, hipStream_t s) {
  // same workgroup shape as the batched kernel's solver: identical results
  if (bins == 256)
    hipLaunchKernelGGL((k_solve<256, NT_PIX>), dim3(1), dim3(NT_PIX), 0, s, hS, hG, npix, p, lists, illum, refl,
                       target, flags);
  else
    hipLaunchKernelGGL((k_solve<1024, NT_PIX>), dim3(1), dim3(NT_PIX), 0, s, hS, hG, npix, p, lists, illum, refl,
                       target, flags);
  return hipGetLastError();
}

hipError_t lut(int bins, const uint32_t* hS, const float* target, uint16_t* lut, uint16_t* lut_user,
               hipStream_t s) {
  if (bins == 256)
    hipLaunchKernelGGL((k_lut<256, 256>), dim3(1), dim3(256), 0, s, hS, target, lut, lut_user);
  else
    hipLaunchKernelGGL((k_lut<1024, 256>), dim3(1), dim3(256), 0, s, hS, target, lut, lut_user);
  return hipGetLastError();
}

hipError_t remap(int bits, const ImgDesc& d, int64_t tile_px, const uint16_t* lut, hipStream_t s) {
  const int64_t tiles = (d.npix + tile_px - 1) / tile_px;
  if (bits == 8)
    hipLaunchKernelGGL(k_remap<8>, dim3((unsigned)tiles), dim3(NT_PIX), 0, s, d, tile_px, lut);
  else
    hipLaunchKernelGGL(k_remap<10>, dim3((unsigned)tiles), dim3(NT_PIX), 0, s, d, tile_px, lut);
  return hipGetLastError();
}

hipError_t batch_reset(BatchHeader* hdr, ImageState* st, int bins, hipStream_t s) {
  // fixed grid: the image count is read on the device, so a captured launch
  // serves any batch
  hipLaunchKernelGGL(k_batch_reset, dim3(512), dim3(256), 0, s, hdr, st, bins);
  return hipGetLastError();
}

hipError_t batch(int bits, int grid, BatchHeader* hdr, const ImgDesc* desc, ImageState* st, uint32_t* lists,
                 int64_t lists_stride, uint32_t* flags, hipStream_t s) {
  if (bits == 8)
    hipLaunchKernelGGL(k_batch<8>, dim3(grid), dim3(NT_PIX), 0, s, hdr, desc, st, lists, lists_stride, flags);
  else
    hipLaunchKernelGGL(k_batch<10>, dim3(grid), dim3(NT_PIX), 0, s, hdr, desc, st, lists, lists_stride, flags);
  return hipGetLastError();
}

int step_px(int bits) { return NT_PIX * (bits == 8 ? Cfg<8>::PX : Cfg<10>::PX); }
int max_width(int bits) {
  return bits == 8 ? Cfg<8>::RING - 2 * NT_PIX * Cfg<8>::PX : Cfg<10>::RING - 2 * NT_PIX * Cfg<10>::PX;
}

}  // namespace launch
}  // namespace hr
