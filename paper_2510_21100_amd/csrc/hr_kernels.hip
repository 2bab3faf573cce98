// Kernels of the HistRetinex pipeline for gfx950 and their launchers.
//
// One-image form: fill -> hist (last workgroup rescales the gradient
// histogram) -> solve (one workgroup) -> lut (one workgroup) -> remap.
// Batched form: one persistent kernel; workgroups take the histogram tiles of
// every image from one queue (largest image first); the workgroup that
// finishes the last histogram tile of an image runs that image's solve and
// LUT and appends the image to a ready list; remap tiles are then taken image
// by image in the order of that list.
#include "hr_device.hpp"
#include "hr_launch.hpp"

#include <algorithm>
#include <mutex>

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
  __shared__ HistSmem<BITS, NT_PIX> sm;
  __shared__ uint32_t red[NT_PIX / 64];
  __shared__ uint32_t last;
  const int64_t P0 = (int64_t)blockIdx.x * tile_px;
  const int64_t P1 = min(P0 + tile_px, d.npix);
  hist_tile<BITS, NT_PIX>(d, P0, P1, sm, hs, graw);
  if (threadIdx.x == 0) {
    if (sm.clamped) atomicOr(flags, FLAG_VALUE_CLAMPED);
    fence_release_agent();
    last = (atomicAdd(ticket, 1u) == gridDim.x - 1) ? 1u : 0u;
    if (last) fence_acquire_agent();
  }
  __syncthreads();
  if (!last) return;
  rebin_gradient<BINS, NT_PIX>(graw, hg, sm.hs, red);
  if (threadIdx.x == 0) *ticket = 0;  // ready for the next call
}

constexpr int NT_BATCH = NT_SOLVE;
// One 1024-thread batched workgroup per CU (its pixel loops and solver take
// most of the CU's registers), so its solver can take most of the CU's LDS.
template <int BITS> struct BatchBudget {
  static constexpr int value = 150 * 1024;
};

template <int BINS, int NT>
__global__ __launch_bounds__(NT) void k_solve(const uint32_t* hS, const uint32_t* hG, int64_t npix, SolveParams p,
                                              float* illum, float* refl, float* target,
                                              int32_t* passes, uint32_t* flags) {
  __shared__ SolveSmem<BINS, NT, SOLVE_BUDGET_PLAIN> sm;
  solve_image<BINS, NT, SOLVE_BUDGET_PLAIN>(
      hS, hG, npix, p, sm, illum, refl, target, flags,
      nullptr, passes);
}

// Classical histogram equalisation (Eq. 5): level v goes to the nearest
// level of (l-1) c(v) / N, ties upwards, c the running count: in integers
// floor((2 (l-1) c(v) + N) / (2N)).  One workgroup; the running count is an
// exact integer scan.
template <int BINS, int NT>
__global__ __launch_bounds__(NT) void k_he_lut(const uint32_t* hS, uint16_t* lut, uint16_t* lut_user) {
  __shared__ uint64_t c[BINS];
  __shared__ uint64_t red[NT / 64];
  for (int k = threadIdx.x; k < BINS; k += NT) c[k] = hS[k];
  __syncthreads();
  const uint64_t N = block_scan<NT, uint64_t, true>(c, BINS, red);
  for (int k = threadIdx.x; k < BINS; k += NT) {
    const uint16_t v = N ? (uint16_t)((2ull * (BINS - 1) * c[k] + N) / (2ull * N)) : (uint16_t)0;
    lut[k] = v;
    if (lut_user) lut_user[k] = v;
  }
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
  __shared__ float2 tab[BINS];
  __shared__ uint32_t stage[NT_PIX * 12];
  load_remap_table<BINS, NT_PIX>(lut, tab);
  __syncthreads();
  const int64_t P0 = (int64_t)blockIdx.x * tile_px;
  const int64_t P1 = min(P0 + tile_px, d.npix);
  remap_tile<BITS, NT_PIX>(d, P0, P1, tab, stage);
}

// ---------------------------------------------------------------------------
// batched persistent kernel
// ---------------------------------------------------------------------------

template <int BITS>
union BatchSmem {
  HistSmem<BITS, NT_BATCH> hist;
  SolveSmem<Cfg<BITS>::BINS, NT_BATCH, BatchBudget<BITS>::value> solve;
  LutSmem<Cfg<BITS>::BINS, NT_BATCH> lut;
  struct {
    float2 tab[Cfg<BITS>::BINS];                     // remap table of the current image
    uint32_t stage[NT_BATCH * 12];      // staged stores of the remap (48-byte chunks)
  } rm;
};



__device__ inline ImageState* state_of(ImageState* st, int64_t st_words, int i) {
  return reinterpret_cast<ImageState*>(reinterpret_cast<uint32_t*>(st) + i * st_words);
}

// Histograms of n images in one launch: grid (tiles of the largest image, n);
// the per-image state holds the raw gradient histogram and the tile ticket.
template <int BITS>
__global__ __launch_bounds__(NT_PIX) void k_hist_batch(const ImgDesc* __restrict__ desc, int64_t tile_px,
                                                       uint32_t* hs, uint32_t* hg, ImageState* st,
                                                       uint32_t* flags) {
  constexpr int BINS = Cfg<BITS>::BINS;
  __shared__ HistSmem<BITS, NT_PIX> sm;
  __shared__ uint32_t red[NT_PIX / 64];
  __shared__ uint32_t last;
  const int i = blockIdx.y;
  const ImgDesc d = desc[i];
  const int64_t P0 = (int64_t)blockIdx.x * tile_px;
  if (P0 >= d.npix) return;  // uniform: this image has fewer tiles
  const int64_t P1 = min(P0 + tile_px, d.npix);
  ImageState* s = state_of(st, ImageState::words(BINS), i);
  uint32_t* graw = s->graw(BINS);
  hist_tile<BITS, NT_PIX>(d, P0, P1, sm, hs + (size_t)i * BINS, graw);
  if (threadIdx.x == 0) {
    if (sm.clamped) atomicOr(flags, FLAG_VALUE_CLAMPED);
    fence_release_agent();
    const uint32_t ntiles = (uint32_t)((d.npix + tile_px - 1) / tile_px);
    last = (atomicAdd(&s->done, 1u) == ntiles - 1) ? 1u : 0u;
    if (last) fence_acquire_agent();
  }
  __syncthreads();
  if (!last) return;
  rebin_gradient<BINS, NT_PIX>(graw, hg + (size_t)i * BINS, sm.hs, red);
}

// Completes image i once all its histogram items are merged: adds up the
// partial histograms, rebins the gradient histogram, runs the solver and the
// LUT, then publishes the LUT.  Everything it needs is re-read from the
// tables, so nothing of the item loop stays live across the solver.
template <int BITS>
__device__ void finish_image(BatchHeader* hdr, const ImgDesc* desc, ImgCounters* ctr, ImageState* st,
                             int64_t st_words, int i, uint32_t* flags,
                             BatchSmem<BITS>& sm, uint32_t* red) {
  constexpr int BINS = Cfg<BITS>::BINS;
  ImageState* s = state_of(st, st_words, i);
  uint32_t* hs = s->hs();
  // The summed histograms are handed to the rebin and the solver's setup in
  // LDS (the solver's spare area, unused until its class list), so no wait
  // for global stores sits on the image's critical path; the value histogram
  // also goes to the state for the LUT.
  uint32_t* lhs = reinterpret_cast<uint32_t*>(sm.solve.spare);  // [BINS]
  uint32_t* lgraw = lhs + BINS;                                  // [2 BINS - 1]
  uint32_t* lhg = lhs + 3 * BINS;                                // [BINS]
  static_assert(sizeof(sm.solve.spare) >= 4 * BINS * sizeof(uint32_t), "spare holds the histograms");
  uint32_t gm = 0;
  for (int k = threadIdx.x; k < 3 * BINS; k += NT_BATCH) {
    uint32_t v = 0;
#pragma unroll
    for (int q = 0; q < ImageState::NSLOT; ++q)
      v += __hip_atomic_load(to_global(s->slot(BINS, q)) + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (k < BINS) {
      lhs[k] = v;
      hs[k] = v;
      lhg[k] = 0;
    } else if (k < 3 * BINS - 1) {
      lgraw[k - BINS] = v;
      if (v) gm = max(gm, (uint32_t)(k - BINS));
    }
  }
  // rebin of the gradient histogram (as rebin_gradient), in LDS
  const uint32_t gmax = block_max<NT_BATCH>(gm, red);
  for (int j = threadIdx.x; j <= (int)gmax; j += NT_BATCH) {
    const uint32_t c = lgraw[j];
    if (c) atomicAdd(&lhg[gmax ? (uint32_t)((2ull * (BINS - 1) * j + gmax) / (2ull * gmax)) : 0u], c);
  }
  __syncthreads();
  const int64_t npix = desc[i].npix;
  const int slot = desc[i].slot;
  const BatchOut out = hdr->out;
  float* tgt = s->target(BINS);
  solve_image<BINS, NT_BATCH, BatchBudget<BITS>::value, false>(
      lhs, lhg, npix, hdr->params, sm.solve, out.illum ? out.illum + (int64_t)slot * BINS : nullptr, out.refl ? out.refl + (int64_t)slot * BINS : nullptr,
      tgt, flags, nullptr, out.passes ? out.passes + slot : nullptr);
  drain_memory();
  __syncthreads();
  uint16_t* lut = s->lut(BINS);
  build_lut<BINS, NT_BATCH>(hs, tgt, sm.lut, lut);
  __syncthreads();
  if (out.target || out.luts) {
    for (int k = threadIdx.x; k < BINS; k += NT_BATCH) {
      if (out.target) out.target[(int64_t)slot * BINS + k] = tgt[k];
      if (out.luts) out.luts[(int64_t)slot * BINS + k] = lut[k];
    }
  }
  drain_memory();
  __syncthreads();
  if (threadIdx.x == 0) {
    // append to the ready list: position by arrival, entry = image + 1
    const uint32_t pos = atomicAdd(&hdr->nready, 1u);
    fence_release_agent();  // the LUT is in memory before the entry can be seen
    __hip_atomic_store(to_global(&ctr[pos].fifo), (uint32_t)i + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // zero the partial slots for the next call (no other workgroup touches them
  // now; their loads above have returned), after the image is published: the
  // stores are written back to memory with a release like the publication's,
  // where the next call's histogram atomics will find them
  for (int k = threadIdx.x; k < 3 * BINS; k += NT_BATCH) {
#pragma unroll
    for (int q = 0; q < ImageState::NSLOT; ++q) s->slot(BINS, q)[k] = 0u;
  }
  drain_memory();
  __syncthreads();
  if (threadIdx.x == 0) fence_release_agent();
}

// image owning histogram item `it` (tile0 ascending over the descriptor table)
__device__ inline int image_of_item(const ImgDesc* desc, int n, int it) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (desc[mid].tile0 <= it) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Claims a remap item (thread 0) from the image at the head of the ready
// list, advancing the head past images whose tiles are all claimed and
// waiting while the head's position is not yet written.  img = -1 once every
// image is claimed out.  Every image has at least one histogram item, so every
// position of the list is written in the end.
__device__ inline void claim_remap(BatchHeader* hdr, const ImgDesc* desc, ImgCounters* ctr, int n, int& img,
                                   int& tl) {
  for (;;) {
    const uint32_t pos = __hip_atomic_load(to_global(&hdr->rhead), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (pos >= (uint32_t)n) {
      img = -1;
      tl = -1;
      return;
    }
    const uint32_t v = __hip_atomic_load(to_global(&ctr[pos].fifo), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (v == 0u) {  // published position not written yet
      __builtin_amdgcn_s_sleep(2);
      continue;
    }
    const int c = (int)v - 1;
    const uint32_t t = atomicAdd(&ctr[c].rnext, 1u);
    if (t < (uint32_t)desc[c].rtiles) {
      img = c;
      tl = (int)t;
      return;
    }
    uint32_t expect = pos;
    __hip_atomic_compare_exchange_strong(to_global(&hdr->rhead), &expect, pos + 1u, __ATOMIC_RELAXED,
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

template <int BITS>
__global__ __launch_bounds__(NT_BATCH) void k_batch(BatchHeader* hdr, const ImgDesc* __restrict__ desc,
                                                    ImgCounters* ctr, ImageState* st, uint32_t* flags) {
  constexpr int BINS = Cfg<BITS>::BINS;
  __shared__ BatchSmem<BITS> sm;
  __shared__ uint32_t red[NT_BATCH / 64];
  __shared__ int item_s;
  __shared__ uint32_t last_s;
  const int64_t st_words = ImageState::words(BINS);
  // fixed for the launch (the queue cursors change on the device)
  const int ht = hdr->total_tiles, nimg = hdr->n;
  const int64_t tile_px = hdr->tile_px, rtile_px = hdr->rtile_px;
  int tab_img = -1;  // image whose remap table is in LDS
  // Histogram items, in queue order.  The workgroup that merges an image's
  // last item runs its solver and publishes it in the ready list.
  for (;;) {
    if (threadIdx.x == 0) item_s = (int)atomicAdd(&hdr->next, 1u);
    __syncthreads();
    const int item = __builtin_amdgcn_readfirstlane(item_s);
    __syncthreads();
    if (item >= ht) break;
    const int i = image_of_item(desc, nimg, item);
    ImageState* s = state_of(st, st_words, i);
    const ImgDesc d = desc[i];
    const int local = item - d.tile0;
    const int64_t P0 = (int64_t)local * tile_px;
    const int64_t P1 = min(P0 + tile_px, d.npix);
    uint32_t* part = s->slot(BINS, local % ImageState::NSLOT);
    hist_tile<BITS, NT_BATCH>(d, P0, P1, sm.hist, part, part + BINS);
    if (threadIdx.x == 0) {
      if (sm.hist.clamped) atomicOr(flags, FLAG_VALUE_CLAMPED);
      fence_release_agent();
      const bool last = atomicAdd(&ctr[i].done, 1u) == (uint32_t)d.ntiles - 1;
      if (last) fence_acquire_agent();
      last_s = last ? 1u : 0u;
    }
    __syncthreads();
    if (last_s) finish_image<BITS>(hdr, desc, ctr, st, st_words, i, flags, sm, red);
    __syncthreads();
  }
  // Remap items, images in the order their LUTs were published, so that no
  // workgroup waits on a solve while a published image has items left.
  // Thread 0 claims the next tile of the same image while this one runs; the
  // barriers here order LDS only (lds_wait + s_barrier), so the claim's
  // atomic stays in flight until the next item starts.
  int cur = -1;
  uint32_t ahead = 0xffffffffu;  // thread 0: tile claimed ahead on image cur
  for (;;) {
    if (threadIdx.x == 0) {
      int img = -1, tl = -1;
      if (cur >= 0 && ahead < (uint32_t)desc[cur].rtiles) {
        img = cur;
        tl = (int)ahead;
      } else {
        claim_remap(hdr, desc, ctr, nimg, img, tl);
      }
      item_s = img;
      last_s = (uint32_t)tl;
      cur = img;
      ahead = img >= 0 ? atomicAdd(&ctr[img].rnext, 1u) : 0xffffffffu;
    }
    lds_wait();
    bare_barrier();
    const int i = __builtin_amdgcn_readfirstlane(item_s);
    const int tile = __builtin_amdgcn_readfirstlane((int)last_s);
    if (i < 0) break;
    const ImgDesc d = desc[i];
    if (tab_img != i) {
      if (threadIdx.x == 0) fence_acquire_agent();  // pairs with the ready list's release
      __syncthreads();
      const uint16_t* lut = state_of(st, st_words, i)->lut(BINS);
      for (int v = threadIdx.x; v < BINS; v += NT_BATCH) {
        const uint32_t L = __hip_atomic_load(to_global(reinterpret_cast<const uint32_t*>(lut)) + (v >> 1),
                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t lv = (v & 1) ? (L >> 16) : (L & 0xffffu);
        sm.rm.tab[v] = remap_entry((uint32_t)v, lv);
      }
      lds_wait();
      bare_barrier();
      tab_img = i;
    }
    const int64_t P0 = (int64_t)tile * rtile_px;
    const int64_t P1 = min(P0 + rtile_px, d.npix);
    remap_tile<BITS, NT_BATCH>(d, P0, P1, sm.rm.tab, sm.rm.stage);
    lds_wait();  // every wave is done with item_s and the table before they change
    bare_barrier();
  }
  // The last workgroup to leave puts the cursors and the per-image counters
  // back to zero (every other workgroup has made its last access to them
  // before its count): the next launch with the same descriptor table finds
  // them as an upload would leave them.
  if (threadIdx.x == 0 && atomicAdd(&hdr->exited, 1u) == gridDim.x - 1) {
    for (int k = 0; k < nimg; ++k) ctr[k] = ImgCounters{0u, 0u, 0u, 0u};
    hdr->next = 0u;
    hdr->rhead = 0u;
    hdr->nready = 0u;
    hdr->exited = 0u;
  }
}

// ---------------------------------------------------------------------------
// allocation-free batched form: fixed scratch in the library's own device array
// ---------------------------------------------------------------------------

// Layout of the scratch array (bytes): the flags word the kernels write when
// the caller passes none, the descriptor table (header, descriptors, counters),
// the per-image states (room for NOALLOC_MAX_IMAGES states of the larger,
// 1024-level layout; a call strides them by the layout of its own level
// count, as the batched kernel does).
constexpr int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }
struct NoallocLayout {
  static constexpr int64_t FLAGS = 0;
  static constexpr int64_t TABLE = 256;
  static constexpr int64_t TABLE_BYTES =
      sizeof(BatchHeader) + NOALLOC_MAX_IMAGES * (sizeof(ImgDesc) + sizeof(ImgCounters));
  static constexpr int64_t STATE = align256(TABLE + TABLE_BYTES);
  static constexpr int64_t STATE_WORDS = ImageState::words(1024);  // per image
  static constexpr int64_t BYTES = align256(STATE + 4 * STATE_WORDS * NOALLOC_MAX_IMAGES);
};

// The scratch itself, about 0.5 MB on every GPU the library runs on, held
// until the process ends.  Host code never passes this name to a kernel: it
// is a host-side stand-in; the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) uint8_t scratch[NoallocLayout::BYTES];

// Writes the call's descriptor table into the scratch (header, descriptors,
// zero counters) and zeroes the partial histogram slots of its images in the
// layout of this bit depth (a previous call may have left another layout, or
// have been cut short).  Grid-stride over every block.
template <int BITS>
__global__ __launch_bounds__(256) void k_noalloc_setup(NoallocTable t, uint8_t* base) {
  constexpr int BINS = Cfg<BITS>::BINS;
  auto* hdr = reinterpret_cast<BatchHeader*>(base + NoallocLayout::TABLE);
  auto* desc = reinterpret_cast<ImgDesc*>(base + NoallocLayout::TABLE + sizeof(BatchHeader));
  auto* ctr = reinterpret_cast<ImgCounters*>(base + NoallocLayout::TABLE + sizeof(BatchHeader) +
                                             NOALLOC_MAX_IMAGES * sizeof(ImgDesc));
  const int n = t.hdr.n;
  const int64_t tid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  if (tid == 0) *hdr = t.hdr;
  if (tid < n) {
    desc[tid] = t.desc[tid];
    ctr[tid] = ImgCounters{0u, 0u, 0u, 0u};
  }
  constexpr int64_t SLOT_WORDS = (int64_t)ImageState::NSLOT * 3 * BINS;
  for (int64_t q = tid; q < (int64_t)n * SLOT_WORDS; q += nthreads) {
    const int i = (int)(q / SLOT_WORDS);
    // the batched kernel's state stride: words(BINS) of this bit depth
    auto* st = reinterpret_cast<ImageState*>(base + NoallocLayout::STATE + 4 * ImageState::words(BINS) * i);
    st->slot(BINS, 0)[q - i * SLOT_WORDS] = 0u;
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

hipError_t hist_batch(int bits, int n, const ImgDesc* desc, int64_t max_tiles, int64_t tile_px, uint32_t* hs,
                      uint32_t* hg, ImageState* st, uint32_t* flags, hipStream_t s) {
  const dim3 grid((unsigned)max_tiles, (unsigned)n);
  if (bits == 8)
    hipLaunchKernelGGL(k_hist_batch<8>, grid, dim3(NT_PIX), 0, s, desc, tile_px, hs, hg, st, flags);
  else
    hipLaunchKernelGGL(k_hist_batch<10>, grid, dim3(NT_PIX), 0, s, desc, tile_px, hs, hg, st, flags);
  return hipGetLastError();
}

hipError_t solve(int bins, const uint32_t* hS, const uint32_t* hG, int64_t npix, const SolveParams& p,
                 float* illum, float* refl, float* target, int32_t* passes, uint32_t* flags, hipStream_t s) {
  // same workgroup shape as the batched kernel's solver: identical results
  if (bins == 256)
    hipLaunchKernelGGL((k_solve<256, NT_SOLVE>), dim3(1), dim3(NT_SOLVE), 0, s, hS, hG, npix, p, illum, refl,
                       target, passes, flags);
  else
    hipLaunchKernelGGL((k_solve<1024, NT_SOLVE>), dim3(1), dim3(NT_SOLVE), 0, s, hS, hG, npix, p, illum, refl,
                       target, passes, flags);
  return hipGetLastError();
}

hipError_t equalize_lut(int bins, const uint32_t* hS, uint16_t* lut, uint16_t* lut_user, hipStream_t s) {
  if (bins == 256)
    hipLaunchKernelGGL((k_he_lut<256, 256>), dim3(1), dim3(256), 0, s, hS, lut, lut_user);
  else
    hipLaunchKernelGGL((k_he_lut<1024, 256>), dim3(1), dim3(256), 0, s, hS, lut, lut_user);
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


hipError_t batch(int bits, int grid, BatchHeader* hdr, const ImgDesc* desc, ImgCounters* ctr, ImageState* st,
                 uint32_t* flags, hipStream_t s) {
  if (bits == 8)
    hipLaunchKernelGGL(k_batch<8>, dim3(grid), dim3(NT_BATCH), 0, s, hdr, desc, ctr, st, flags);
  else
    hipLaunchKernelGGL(k_batch<10>, dim3(grid), dim3(NT_BATCH), 0, s, hdr, desc, ctr, st, flags);
  return hipGetLastError();
}

int batch_max_wg_per_cu(int bits) {
  int n = 0;
  const hipError_t e = bits == 8 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch<8>, NT_BATCH, 0)
                                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_batch<10>, NT_BATCH, 0);
  return e == hipSuccess ? n : 0;
}

int step_px(int bits) { return bits == 8 ? Pix<8, NT_PIX>::STEP : Pix<10, NT_PIX>::STEP; }
int batch_step_px(int bits) { return bits == 8 ? Pix<8, NT_BATCH>::STEP : Pix<10, NT_BATCH>::STEP; }
int max_width(int bits) { return bits == 8 ? MaxWidth<8>::value : MaxWidth<10>::value; }

int64_t noalloc_scratch_bytes() { return NoallocLayout::BYTES; }

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t* g_scratch[kMaxDevices] = {};  // device address of `scratch` on each GPU
int g_cus[kMaxDevices] = {};

// The scratch array's device address and the CU count of the current GPU,
// looked up once per device (with that device current) and kept.
hipError_t scratch_of_current_device(uint8_t** ptr, int* cus) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    int n = 0;
    e = hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    g_cus[dev] = n;
    g_scratch[dev] = static_cast<uint8_t*>(p);
  }
  *ptr = g_scratch[dev];
  *cus = g_cus[dev];
  return hipSuccess;
}
}  // namespace

hipError_t batch_noalloc(int bits, int grid_per_cu, const NoallocTable& t, uint32_t* flags_user, hipStream_t s) {
  uint8_t* base = nullptr;
  int cus = 0;
  hipError_t e = scratch_of_current_device(&base, &cus);
  if (e != hipSuccess) return e;
  auto* hdr = reinterpret_cast<BatchHeader*>(base + NoallocLayout::TABLE);
  auto* desc = reinterpret_cast<ImgDesc*>(base + NoallocLayout::TABLE + sizeof(BatchHeader));
  auto* ctr = reinterpret_cast<ImgCounters*>(base + NoallocLayout::TABLE + sizeof(BatchHeader) +
                                             NOALLOC_MAX_IMAGES * sizeof(ImgDesc));
  auto* st = reinterpret_cast<ImageState*>(base + NoallocLayout::STATE);
  uint32_t* flags = flags_user ? flags_user : reinterpret_cast<uint32_t*>(base + NoallocLayout::FLAGS);
  // the kernels stride the states by words(bins) of the call's level count
  static_assert(NoallocLayout::STATE_WORDS >= ImageState::words(256), "state layout");
  const int grid = std::max(1, cus * std::max(1, grid_per_cu));
  if (bits == 8) {
    hipLaunchKernelGGL(k_noalloc_setup<8>, dim3(16), dim3(256), 0, s, t, base);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch<8>, dim3(grid), dim3(NT_BATCH), 0, s, hdr, desc, ctr, st, flags);
  } else {
    hipLaunchKernelGGL(k_noalloc_setup<10>, dim3(16), dim3(256), 0, s, t, base);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_batch<10>, dim3(grid), dim3(NT_BATCH), 0, s, hdr, desc, ctr, st, flags);
  }
  return hipGetLastError();
}

}  // namespace launch
}  // namespace hr
