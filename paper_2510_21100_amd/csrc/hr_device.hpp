// Device building blocks of the HistRetinex pipeline for gfx950 (CDNA4).
//
// Three groups, each used both by the one-image kernels and by the persistent
// batched kernel:
//   * pixel tiles: value channel V = max(R,G,B) (Sec. II), the V histogram
//     (Eq. 3) and the gradient-image histogram (Alg. 1 initialisation), and the
//     remap of pixels through the matching LUT (end of Sec. III-C);
//   * the solver: the alternating histogram updates of Eqs. (11)-(15) (Alg. 1)
//     and the enhanced target histogram of Eqs. (17)-(20), all on one
//     workgroup with its state in LDS;
//   * the matching LUT: scans of the image and target histograms and an
//     inverse-CDF search per level.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hr_launch.hpp"

namespace hr {

constexpr int NT_PIX = 256;  // threads of a pixel-streaming workgroup

using v4u = uint32_t __attribute__((ext_vector_type(4)));
using v2u = uint32_t __attribute__((ext_vector_type(2)));

// Global-address-space view of a pointer known to point into device memory.
// Accesses through a generic pointer become flat instructions, which hold the
// LDS counter as well as the memory counter: every wait for an LDS result
// would then also wait for the pixel loads in flight.
template <typename T> using gptr = __attribute__((address_space(1))) T*;
template <typename T> __device__ inline gptr<T> to_global(T* p) { return (gptr<T>)p; }
constexpr uint32_t FLAG_VALUE_CLAMPED = 1u;
constexpr uint32_t FLAG_HIST_MASS = 2u;

// Per bit depth: element type and levels.
template <int BITS> struct Cfg;
template <> struct Cfg<8> {
  using pix_t = uint8_t;
  static constexpr int BINS = 256;
};
template <> struct Cfg<10> {
  using pix_t = uint16_t;
  static constexpr int BINS = 1024;
};


// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__device__ inline uint32_t umax3(uint32_t a, uint32_t b, uint32_t c) {
  return max(max(a, b), c);
}

// Cross-workgroup hand-off.  The release and acquire fences at agent scope
// write back / invalidate the whole L2 of the XCD, so one wave issues them on
// behalf of its workgroup: every wave first drains its own memory operations
// (non-returning atomics included) and meets the others at a barrier, then a
// single thread fences and signals; on the receiving side a single thread
// observes the signal and fences before the barrier that releases the rest.
__device__ inline void drain_memory() { __builtin_amdgcn_s_waitcnt(0); }
// Release at agent scope before a signal: the fence writes this XCD's L2 back
// to memory, and the wait makes that write-back complete before the signal's
// store or atomic is issued (the compiler does not always place a wait between
// the write-back and a later store, and a reader on another XCD could then see
// the signal before the data).
__device__ inline void fence_release_agent() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __builtin_amdgcn_s_waitcnt(0);
}
__device__ inline void fence_acquire_agent() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// Workgroup barrier for the pixel loops.  __syncthreads() waits for every
// outstanding LDS operation of the wave, the histogram atomics included; the
// ring hand-off only needs the ring stores, so the loops wait for those
// explicitly (lds_wait: LDS counter to zero, memory loads left in flight) and
// then meet at a bare s_barrier while the atomics drain.  The asm's memory
// clobber keeps the compiler from moving LDS accesses across it.
__device__ inline void lds_wait() { __builtin_amdgcn_s_waitcnt(0xC07F); }  // lgkmcnt(0) only
__device__ inline void bare_barrier() { asm volatile("s_barrier" ::: "memory"); }


// element k of a little-endian packed array of 8- or 16-bit lanes
template <typename T, int N>
__device__ inline uint32_t lane_of(const uint32_t (&w)[N], int k) {
  if constexpr (sizeof(T) == 1) {
    return (w[k >> 2] >> ((k & 3) * 8)) & 0xffu;
  } else {
    return (w[k >> 1] >> ((k & 1) * 16)) & 0xffffu;
  }
}

template <typename T, int N>
__device__ inline void set_lane(uint32_t (&w)[N], int k, uint32_t v) {
  if constexpr (sizeof(T) == 1) {
    const int s = (k & 3) * 8;
    w[k >> 2] = (w[k >> 2] & ~(0xffu << s)) | (v << s);
  } else {
    const int s = (k & 1) * 16;
    w[k >> 1] = (w[k >> 1] & ~(0xffffu << s)) | (v << s);
  }
}

// Cross-lane moves through DPP (a VALU operand modifier, no LDS round trip).
// Controls in the gfx9 encoding: row_shr:n shifts within rows of 16 lanes,
// row_bcast:15 / row_bcast:31 pass lane 15 of each row (lane 31) to the rows
// that the row mask enables.  Lanes without a source read zero.
namespace dpp {
constexpr int ROW_SHR = 0x110;  // + n, n = 1..15
constexpr int WAVE_SHL1 = 0x130;  // lane i takes lane i + 1 (lane 63: zero)
constexpr int BCAST15 = 0x142;
constexpr int BCAST31 = 0x143;
}  // namespace dpp

template <int CTRL, int ROWS>
__device__ inline uint32_t dpp32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, CTRL, ROWS, 0xf, true);
}

template <int CTRL, int ROWS, typename T>
__device__ inline T dpp_get(T x) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32- or 64-bit lanes");
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, dpp32<CTRL, ROWS>(__builtin_bit_cast(uint32_t, x)));
  } else {
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const uint64_t lo = dpp32<CTRL, ROWS>((uint32_t)u), hi = dpp32<CTRL, ROWS>((uint32_t)(u >> 32));
    return __builtin_bit_cast(T, lo | (hi << 32));
  }
}

template <typename T>
__device__ inline T read_lane(T x, int lane) {
  if constexpr (sizeof(T) == 4) {
    return __builtin_bit_cast(T, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x), lane));
  } else {
    const uint64_t u = __builtin_bit_cast(uint64_t, x);
    const uint64_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
    const uint64_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
    return __builtin_bit_cast(T, lo | (hi << 32));
  }
}

// Inclusive prefix sum over the 64 lanes of the wave (all lanes active).
template <typename T>
__device__ inline T wave_scan(T x) {
  x += dpp_get<dpp::ROW_SHR + 1, 0xf>(x);
  x += dpp_get<dpp::ROW_SHR + 2, 0xf>(x);
  x += dpp_get<dpp::ROW_SHR + 4, 0xf>(x);
  x += dpp_get<dpp::ROW_SHR + 8, 0xf>(x);
  x += dpp_get<dpp::BCAST15, 0xa>(x);
  x += dpp_get<dpp::BCAST31, 0xc>(x);
  return x;
}

// Sums over aligned groups of G lanes (G a power of two, 1..64), complete in
// the last lane of each group (other lanes hold partial sums).
template <typename T>
__device__ inline T group_sum_last(T x, int G) {
  const int p = threadIdx.x & 63, r = p & (G - 1);
  T y;
  y = dpp_get<dpp::ROW_SHR + 1, 0xf>(x);
  if (r >= 1) x += y;
  y = dpp_get<dpp::ROW_SHR + 2, 0xf>(x);
  if (r >= 2) x += y;
  y = dpp_get<dpp::ROW_SHR + 4, 0xf>(x);
  if (r >= 4) x += y;
  y = dpp_get<dpp::ROW_SHR + 8, 0xf>(x);
  if (r >= 8) x += y;
  if (G >= 32) x += dpp_get<dpp::BCAST15, 0xa>(x);
  if (G >= 64) x += dpp_get<dpp::BCAST31, 0xc>(x);
  return x;
}

template <typename T>
__device__ inline T wave_sum(T x) {
  return read_lane(wave_scan(x), 63);
}

template <typename T>
__device__ inline T wave_max(T x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x = max(x, __shfl_xor(x, o, 64));
  return x;
}

// Deterministic block reductions: every thread returns the same value,
// combined in a fixed order.  `red` holds NT/64 entries of T.
template <int NT, typename T>
__device__ inline T block_sum(T x, T* red) {
  x = wave_sum(x);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = x;
  __syncthreads();
  T s = red[0];
#pragma unroll
  for (int i = 1; i < NT / 64; ++i) s += red[i];
  return s;
}

template <int NT, typename T>
__device__ inline T block_max(T x, T* red) {
  x = wave_max(x);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = x;
  __syncthreads();
  T s = red[0];
#pragma unroll
  for (int i = 1; i < NT / 64; ++i) s = max(s, red[i]);
  return s;
}

// In-place exclusive (or inclusive) prefix sum of arr[0..n) in LDS, fixed
// association order.  Returns the total.  `red` holds NT/64 entries of T.
template <int NT, typename T, bool INCLUSIVE = false>
__device__ inline T block_scan(T* arr, int n, T* red) {
  const int t = threadIdx.x;
  const int per = (n + NT - 1) / NT;
  const int b0 = min(t * per, n), b1 = min(b0 + per, n);
  T local = T(0);
  for (int i = b0; i < b1; ++i) local += arr[i];
  // inclusive scan of the per-thread totals over the wave
  const int lane = t & 63;
  const T inc = wave_scan(local);
  __syncthreads();
  if (lane == 63) red[t >> 6] = inc;
  __syncthreads();
  T base = T(0);
  for (int i = 0; i < (t >> 6); ++i) base += red[i];
  T total = T(0);
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) total += red[i];
  T run = base + inc - local;  // exclusive prefix of this thread's first element
  for (int i = b0; i < b1; ++i) {
    const T v = arr[i];
    if (INCLUSIVE) {
      run += v;
      arr[i] = run;
    } else {
      arr[i] = run;
      run += v;
    }
  }
  __syncthreads();
  return total;
}

// ---------------------------------------------------------------------------
// pixel loads
// ---------------------------------------------------------------------------

// Pixels per thread per step: 48 bytes of RGB per thread for 256-thread
// workgroups, 24 bytes for 1024-thread workgroups (fewer registers).
template <int BITS, int NT>
struct Pix {
  static constexpr int ESZ = BITS == 8 ? 1 : 2;
  static constexpr int PX = (NT >= 1024 ? 24 : 48) / (3 * ESZ);
  static constexpr int NW = 3 * PX * ESZ / 4;  // dwords of RGB per chunk
  static constexpr int NV = PX * ESZ / 4;      // dwords of V per chunk
  static constexpr int STEP = NT * PX;
};

// NW dwords from a pointer aligned to NW*4/3 bytes, as three vector loads.
template <int NW>
__device__ inline void load_words(const uint8_t* ptr, uint32_t (&w)[NW]) {
  if constexpr (NW == 12) {
    const gptr<const v4u> s = to_global(reinterpret_cast<const v4u*>(ptr));
    const v4u a = s[0], b = s[1], c = s[2];
    w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w;
    w[4] = b.x; w[5] = b.y; w[6] = b.z; w[7] = b.w;
    w[8] = c.x; w[9] = c.y; w[10] = c.z; w[11] = c.w;
  } else {
    static_assert(NW == 6, "chunk of 24 or 48 bytes");
    const gptr<const v2u> s = to_global(reinterpret_cast<const v2u*>(ptr));
    const v2u a = s[0], b = s[1], c = s[2];
    w[0] = a.x; w[1] = a.y; w[2] = b.x; w[3] = b.y; w[4] = c.x; w[5] = c.y;
  }
}

template <int NW>
__device__ inline void store_words_nt(uint8_t* ptr, const uint32_t (&w)[NW]) {
  if constexpr (NW == 12) {
    const gptr<v4u> d = to_global(reinterpret_cast<v4u*>(ptr));
    __builtin_nontemporal_store(v4u{w[0], w[1], w[2], w[3]}, d);
    __builtin_nontemporal_store(v4u{w[4], w[5], w[6], w[7]}, d + 1);
    __builtin_nontemporal_store(v4u{w[8], w[9], w[10], w[11]}, d + 2);
  } else {
    const gptr<v2u> d = to_global(reinterpret_cast<v2u*>(ptr));
    __builtin_nontemporal_store(v2u{w[0], w[1]}, d);
    __builtin_nontemporal_store(v2u{w[2], w[3]}, d + 1);
    __builtin_nontemporal_store(v2u{w[4], w[5]}, d + 2);
  }
}

// Value channel of PX consecutive pixels p .. p+PX-1 (n of them valid).
template <int BITS, int NT>
__device__ inline void load_values(const ImgDesc& d, int64_t p, int n, uint32_t (&v)[Pix<BITS, NT>::PX],
                                   uint32_t& clamped) {
  using pix_t = typename Cfg<BITS>::pix_t;
  constexpr int PX = Pix<BITS, NT>::PX, NW = Pix<BITS, NT>::NW;
  constexpr uint32_t TOP = (1u << BITS) - 1;
  if (d.in_vec && n == PX) {
    uint32_t w[NW];
    load_words<NW>(d.in + p * 3 * (int64_t)sizeof(pix_t), w);
#pragma unroll
    for (int i = 0; i < PX; ++i) {
      uint32_t x = umax3(lane_of<pix_t>(w, 3 * i), lane_of<pix_t>(w, 3 * i + 1),
                         lane_of<pix_t>(w, 3 * i + 2));
      if (BITS > 8 && x > TOP) {
        clamped = 1;
        x = TOP;
      }
      v[i] = x;
    }
  } else {
    int64_t y = p / d.W;
    int x = (int)(p - y * d.W);
#pragma unroll
    for (int i = 0; i < PX; ++i) {
      uint32_t val = 0;
      if (i < n) {
        const gptr<const pix_t> px = to_global(reinterpret_cast<const pix_t*>(d.in + y * d.in_stride)) + 3 * x;
        val = umax3(px[0], px[1], px[2]);
        if (BITS > 8 && val > TOP) {
          clamped = 1;
          val = TOP;
        }
        if (++x == d.W) {
          x = 0;
          ++y;
        }
      }
      v[i] = val;
    }
  }
}

// ---------------------------------------------------------------------------
// histogram tile: V histogram of pixels [P0, P1) and gradient histogram of the
// same pixels.  The gradient needs V one pixel to the right and one row below,
// so V is computed for [P0, min(P1 + W, N)) into an LDS ring and the gradient
// trails the loads by one row.
// ---------------------------------------------------------------------------

// Widest supported image and the V-ring (entries, a power of two) for a
// workgroup of NT threads: the ring must hold one image row plus two steps.
template <int BITS> struct MaxWidth { static constexpr int value = BITS == 8 ? 16384 : 8192; };
constexpr int pow2_at_least(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// LDS of a histogram tile.  Each histogram has REP copies (thread t counts
// into copy t mod REP, at word level * REP + t mod REP) so that lanes of a
// wave hitting the same level mostly hit different words.  Low-light images
// put most pixels in a few levels, so the workgroups that own a whole CU take
// 16 copies.
template <int BITS, int NT>
struct HistSmem {
  static constexpr int BINS = Cfg<BITS>::BINS;
  static constexpr int REP = BITS == 8 ? (NT >= 512 ? 16 : 4) : (NT >= 512 ? 4 : 1);
  static constexpr int STRIDE = REP;
  // the value histogram of 8-bit pixels in the split kernel: 32 copies (a
  // dark image puts most lanes of a wave on a few levels)
  static constexpr int REPS = (BITS == 8 && NT >= 1024) ? 32 : REP;
  static constexpr int STRIDES = REPS;
  // 1024-thread workgroups split into a loading and a gradient half (see
  // HistTileSplit), whose steps are STEPH pixels and lie up to
  // 1 + ceil((W+1)/STEPH) steps apart; smaller ones alternate the two phases
  static constexpr int STEPH = Pix<BITS, (NT >= 1024 ? NT / 2 : NT)>::STEP;
  static constexpr int RING =
      NT >= 1024 ? pow2_at_least(STEPH * (2 + (MaxWidth<BITS>::value + STEPH) / STEPH))
                 : pow2_at_least(MaxWidth<BITS>::value + 2 * Pix<BITS, NT>::STEP);
  using pix_t = typename Cfg<BITS>::pix_t;
  static constexpr int RING_BYTES = RING * (int)sizeof(pix_t);
  // Small gradients (raw level < GSMALL) take most pixels of smooth images and
  // lanes of one wave tend to hit the same level.  With 10-bit pixels the
  // split kernel has only 4 copies, and these levels count into one copy per
  // lane, hgs[level * 64 + lane] (measured faster there; slower with the 16
  // copies of 8-bit pixels, where the address select costs more than it saves).
  static constexpr int GSMALL = (NT >= 1024 && BITS == 10) ? 32 : 0;
  uint32_t hs[BINS * STRIDES];
  uint32_t hg[(2 * BINS - 1) * STRIDE];
  uint32_t hgs[GSMALL > 0 ? GSMALL * 64 : 4];
  alignas(16) uint32_t ring[RING_BYTES / 4 + 16];  // + 64-byte mirror of the start: no wrap on reads
  uint32_t clamped;
};

// NV dwords starting at an arbitrary byte offset of the ring.
template <int NV>
__device__ inline void ring_read(const uint32_t* ring, uint32_t byteoff, uint32_t (&out)[NV]) {
  const uint32_t b = byteoff >> 2, sh = byteoff & 3;
  uint32_t dw[NV + 1];
#pragma unroll
  for (int k = 0; k <= NV; ++k) dw[k] = ring[b + k];
#pragma unroll
  for (int k = 0; k < NV; ++k) out[k] = __builtin_amdgcn_alignbyte(dw[k + 1], dw[k], sh);
}

template <int NV>
__device__ inline void ring_write(uint32_t* ring, uint32_t byteoff, const uint32_t (&w)[NV]) {
  if constexpr (NV == 4) {
    *reinterpret_cast<v4u*>(reinterpret_cast<uint8_t*>(ring) + byteoff) = v4u{w[0], w[1], w[2], w[3]};
  } else {
    *reinterpret_cast<v2u*>(reinterpret_cast<uint8_t*>(ring) + byteoff) = v2u{w[0], w[1]};
  }
}

// element k (run-time index) of a packed lane array of 2 or 4 dwords,
// through 64-bit shifts (no indexed register access)
template <typename T, int N>
__device__ inline uint32_t lane_dyn(const uint32_t (&w)[N], int k) {
  static_assert(N == 2 || N == 4, "2 or 4 dwords");
  constexpr int PER64 = 8 / (int)sizeof(T);
  uint64_t sel = ((uint64_t)w[1] << 32) | w[0];
  if constexpr (N == 4) {
    const uint64_t hi = ((uint64_t)w[3] << 32) | w[2];
    sel = k >= PER64 ? hi : sel;
  }
  const uint32_t x = (uint32_t)(sel >> ((k & (PER64 - 1)) * 8 * (int)sizeof(T)));
  return sizeof(T) == 1 ? (x & 0xffu) : (x & 0xffffu);
}

// |a - b| + |c - b| for values below 2^16
__device__ inline uint32_t grad_l1(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_sad_u16(a, b, __builtin_amdgcn_sad_u16(c, b, 0u));
}

using u16x2 = unsigned short __attribute__((ext_vector_type(2)));

// max of two pairs of 16-bit lanes (one packed instruction)
__device__ inline uint32_t max_u16x2(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, a),
                                                                 __builtin_bit_cast(u16x2, b)));
}

// V of 16 interleaved 8-bit RGB pixels (12 dwords): byte permutes gather R, G
// and B of two pixels into 16-bit lane pairs, two packed maxima give their V.
// v[i] gets V of pixel i; packed[q] the V of pixels 4q..4q+3 as bytes.
__device__ inline void values_packed_8(const uint32_t (&w)[12], uint32_t (&v)[16], uint32_t (&packed)[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t d0 = w[3 * q], d1 = w[3 * q + 1], d2 = w[3 * q + 2];
    // selector bytes: 0-3 pick bytes of the second operand, 4-7 of the first, 0x0c a zero
    const uint32_t r01 = __builtin_amdgcn_perm(d1, d0, 0x0c030c00u), g01 = __builtin_amdgcn_perm(d1, d0, 0x0c040c01u),
                   b01 = __builtin_amdgcn_perm(d1, d0, 0x0c050c02u);
    const uint32_t r23 = __builtin_amdgcn_perm(d2, d1, 0x0c050c02u), g23 = __builtin_amdgcn_perm(d2, d1, 0x0c060c03u),
                   b23 = __builtin_amdgcn_perm(d2, d1, 0x0c070c04u);
    const uint32_t v01 = max_u16x2(max_u16x2(r01, g01), b01), v23 = max_u16x2(max_u16x2(r23, g23), b23);
    packed[q] = __builtin_amdgcn_perm(v23, v01, 0x06040200u);
    v[4 * q] = v01 & 0xffffu;
    v[4 * q + 1] = v01 >> 16;
    v[4 * q + 2] = v23 & 0xffffu;
    v[4 * q + 3] = v23 >> 16;
  }
}

// Chunks (PX pixels of one thread, NW dwords) kept in flight per thread by
// the pixel loops: enough bytes per CU to cover the HBM latency.
//
// The loops overlap these loads with compute only if the compiler can count
// them: a load skipped on some path leaves the count unknown and it then
// waits for every outstanding load.  So the main loops run over steps in
// which every thread has a full chunk (a condition uniform over the
// workgroup) and issue their prefetches unconditionally, a prefetch that
// would leave the range re-reading chunk 0 of the image instead (in bounds:
// the vector paths require at least one full chunk).  Partial steps go to a
// tail with the same arithmetic.
constexpr int PREFETCH = 4;

// V of the PX pixels of a chunk from its NW words
template <int BITS, int PX, int NW>
__device__ inline void values_of_words(const uint32_t (&w)[NW], uint32_t (&v)[PX], uint32_t& clamped) {
  using pix_t = typename Cfg<BITS>::pix_t;
  constexpr uint32_t TOP = (1u << BITS) - 1;
#pragma unroll
  for (int i = 0; i < PX; ++i) {
    uint32_t m = umax3(lane_of<pix_t>(w, 3 * i), lane_of<pix_t>(w, 3 * i + 1), lane_of<pix_t>(w, 3 * i + 2));
    if (BITS > 8) {
      clamped |= m > TOP ? 1u : 0u;
      m = min(m, TOP);
    }
    v[i] = m;
  }
}

template <int BITS, int NT>
struct HistTile {
  using pix_t = typename Cfg<BITS>::pix_t;
  using SM = HistSmem<BITS, NT>;
  static constexpr int BINS = Cfg<BITS>::BINS, REP = SM::REP, SD = SM::STRIDE;
  static constexpr int PX = Pix<BITS, NT>::PX, NW = Pix<BITS, NT>::NW, NV = Pix<BITS, NT>::NV;
  static constexpr int STEP = Pix<BITS, NT>::STEP;
  static constexpr int RING = SM::RING, RING_BYTES = SM::RING_BYTES;
  static constexpr int ESZ = (int)sizeof(pix_t);
  static constexpr int64_t CB = 3 * ESZ;

  const ImgDesc& d;
  SM& sm;
  const int64_t P0, P1, N, E;  // V is needed for [P0, E)
  const int W, t, step_mod_w;
  uint32_t* hs;  // this thread's copy: level k at hs[k * SD]
  uint32_t* hg;
  int x;  // column of this thread's gradient chunk
  uint32_t clamped = 0;
  int64_t loaded, done;

  __device__ HistTile(const ImgDesc& d_, int64_t p0, int64_t p1, SM& sm_)
      : d(d_), sm(sm_), P0(p0), P1(p1), N(d_.npix), E(min(p1 + (int64_t)d_.W, d_.npix)), W(d_.W),
        t(threadIdx.x), step_mod_w(STEP % d_.W), hs(sm_.hs + (threadIdx.x & (REP - 1))),
        hg(sm_.hg + (threadIdx.x & (REP - 1))), loaded(p0), done(p0) {
    x = (int)((P0 + (int64_t)t * PX) % W);
  }

  // this thread's chunk of the load step starting at `at`, or chunk 0 when
  // that one is not full
  __device__ const uint8_t* chunk_or_first(int64_t at) const {
    const int64_t p = at + (int64_t)t * PX;
    return d.in + (p + PX <= E ? p : 0) * CB;
  }

  // V of the load step at `loaded` into the ring, V histogram of its pixels
  // below P1.  `have`: the chunk's words are in w (else n < PX or strided).
  __device__ void load_step(const uint32_t (&w)[NW], bool have) {
    const int64_t p = loaded + (int64_t)t * PX;
    const int n = (int)max((int64_t)0, min((int64_t)PX, E - p));
    if (n > 0) {
      uint32_t v[PX];
      if (have) values_of_words<BITS, PX, NW>(w, v, clamped);
      else load_values<BITS, NT>(d, p, n, v, clamped);
      uint32_t packed[NV];
#pragma unroll
      for (int q = 0; q < NV; ++q) packed[q] = 0;
#pragma unroll
      for (int i = 0; i < PX; ++i) set_lane<pix_t>(packed, i, v[i]);
      const uint32_t boff = (uint32_t)(((p - P0) & (RING - 1)) * ESZ);
      ring_write<NV>(sm.ring, boff, packed);
      if (boff < 64) ring_write<NV>(sm.ring, RING_BYTES + boff, packed);
      lds_wait();  // the ring stores are done before this wave's barrier
      const int64_t nh = P1 - p;  // pixels of the chunk inside the tile
      if (nh >= PX) {
#pragma unroll
        for (int i = 0; i < PX; ++i) atomicAdd(&hs[v[i] * SD], 1u);
      } else {
#pragma unroll
        for (int i = 0; i < PX; ++i)
          if (i < nh) atomicAdd(&hs[v[i] * SD], 1u);
      }
    }
  }

  // gradient of pixels [done, dend) once the row below them is in the ring:
  // right neighbour from the same chunk (or the next one), lower neighbour
  // one row further on
  __device__ void grad_step() {
    const int64_t dend = min(done + STEP, P1);
    if (min(dend - 1 + W, N - 1) + 1 > loaded) return;  // uniform
    const int64_t q = done + (int64_t)t * PX;
    const int n = (int)max((int64_t)0, min((int64_t)PX, dend - q));
    if (n > 0) {
      const uint32_t boff = (uint32_t)(((q - P0) & (RING - 1)) * ESZ);
      uint32_t own[NV];
      ring_read<NV>(sm.ring, boff, own);  // aligned: the shift is 0
      const uint32_t rboff = boff + PX * ESZ;  // <= RING_BYTES: mirror covers it
      const uint32_t right_last = ESZ == 1 ? (uint32_t)reinterpret_cast<const uint8_t*>(sm.ring)[rboff]
                                           : (uint32_t)reinterpret_cast<const uint16_t*>(sm.ring)[rboff >> 1];
      const uint32_t dboff = (uint32_t)(((q + W - P0) & (RING - 1)) * ESZ);
      uint32_t dn[NV];
      ring_read<NV>(sm.ring, dboff, dn);
      if (n == PX && N - W - q >= PX && W > PX) {
        // every pixel has a row below and at most one ends its row: count all
        // with their right neighbour, then move the row-end pixel to its
        // level without the horizontal term
#pragma unroll
        for (int i = 0; i < PX; ++i) {
          const uint32_t vv = lane_of<pix_t>(own, i);
          const uint32_t vr = (i + 1 < PX) ? lane_of<pix_t>(own, i + 1) : right_last;
          atomicAdd(&hg[grad_l1(vr, vv, lane_of<pix_t>(dn, i)) * SD], 1u);
        }
        const int e = W - 1 - x;
        if (e < PX) {
          const uint32_t ve = lane_dyn<pix_t>(own, e);
          const uint32_t vre = (e + 1 < PX) ? lane_dyn<pix_t>(own, e + 1) : right_last;
          const uint32_t vde = lane_dyn<pix_t>(dn, e);
          atomicSub(&hg[grad_l1(vre, ve, vde) * SD], 1u);
          atomicAdd(&hg[grad_l1(ve, ve, vde) * SD], 1u);
        }
      } else {
        int xx = x;
#pragma unroll
        for (int i = 0; i < PX; ++i) {
          if (i < n) {
            const uint32_t vv = lane_of<pix_t>(own, i);
            const uint32_t vr = (xx + 1 < W) ? ((i + 1 < PX) ? lane_of<pix_t>(own, i + 1) : right_last) : vv;
            const uint32_t vd = (q + i + W < N) ? lane_of<pix_t>(dn, i) : vv;
            atomicAdd(&hg[grad_l1(vr, vv, vd) * SD], 1u);
            if (++xx == W) xx = 0;
          }
        }
      }
    }
    x += step_mod_w;
    if (x >= W) x -= W;
    done = dend;
  }

  // one load step, then the gradient step if its rows are loaded; the
  // barriers separate ring stores from ring reads and reads from the next
  // step's stores
  __device__ void step(const uint32_t (&w)[NW], bool have) {
    load_step(w, have);
    loaded += STEP;
    bare_barrier();
    grad_step();
    bare_barrier();  // ring reads of this step have returned (their values are consumed)
  }

  __device__ void run() {
    if (d.in_vec && N >= PX) {
      uint32_t buf[PREFETCH][NW];
#pragma unroll
      for (int j = 0; j < PREFETCH; ++j) load_words<NW>(chunk_or_first(P0 + (int64_t)j * STEP), buf[j]);
      // steps whose chunks are all full, PREFETCH at a time
      while (loaded + (int64_t)PREFETCH * STEP <= E) {
#pragma unroll
        for (int k = 0; k < PREFETCH; ++k) {
          step(buf[k], true);  // buf[k] is refilled once its words are consumed
          load_words<NW>(chunk_or_first(loaded - STEP + (int64_t)PREFETCH * STEP), buf[k]);
        }
      }
      // the rest: possibly partial or empty load steps
      while (done < P1) {
#pragma unroll
        for (int k = 0; k < PREFETCH; ++k) {
          if (done < P1) {
            const int64_t p = loaded + (int64_t)t * PX;
            step(buf[k], p + PX <= E);
            load_words<NW>(chunk_or_first(loaded - STEP + (int64_t)PREFETCH * STEP), buf[k]);
          }
        }
      }
    } else {
      uint32_t none[NW];
#pragma unroll
      for (int q = 0; q < NW; ++q) none[q] = 0;
      while (done < P1) step(none, false);
    }
  }
};

// Histogram tile for 1024-thread workgroups: the first half of the waves
// (producers) stream the load steps into the ring and count V, the second
// half (consumers) form the gradient of the step `lag` steps behind, so the
// memory-bound and the LDS-bound halves of the work overlap; one barrier per
// step.  Each half works like a 512-thread workgroup (Pix<BITS, NT/2>).  The
// consumer's rows (its step, one row below it and one pixel further) were
// written in earlier steps, and the producer's current step overwrites only
// ring slots older than the consumer's step (the ring holds lag + 1 steps).
template <int BITS, int NT>
struct HistTileSplit {
  static constexpr int NH = NT / 2;
  using pix_t = typename Cfg<BITS>::pix_t;
  using SM = HistSmem<BITS, NT>;
  static constexpr int BINS = Cfg<BITS>::BINS, REP = SM::REP, SD = SM::STRIDE;
  static constexpr int PX = Pix<BITS, NH>::PX, NW = Pix<BITS, NH>::NW, NV = Pix<BITS, NH>::NV;
  static constexpr int STEP = Pix<BITS, NH>::STEP;
  static constexpr int RING = SM::RING, RING_BYTES = SM::RING_BYTES;
  static constexpr int ESZ = (int)sizeof(pix_t);
  static constexpr int64_t CB = 3 * ESZ;
  static_assert(RING >= STEP * (2 + (MaxWidth<BITS>::value + STEP) / STEP), "ring too small for the lag");

  const ImgDesc& d;
  SM& sm;
  const int64_t P0, P1, N, E;
  const int W, tt, step_mod_w;
  const bool producer;
  uint32_t* hs;
  uint32_t* hg;
  uint32_t* hgl;  // this lane's copy of the small gradient levels
  int x;
  uint32_t clamped = 0;
  static constexpr uint32_t GSMALL = SM::GSMALL;

  // `producer` is read from lane 0 as a scalar: NH is a multiple of 64, so the
  // halves are whole waves, and a scalar branch keeps the two loops (and
  // their registers) apart
  __device__ HistTileSplit(const ImgDesc& d_, int64_t p0, int64_t p1, SM& sm_)
      : d(d_), sm(sm_), P0(p0), P1(p1), N(d_.npix), E(min(p1 + (int64_t)d_.W, d_.npix)), W(d_.W),
        tt(threadIdx.x & (NH - 1)), step_mod_w(STEP % d_.W), producer(__builtin_amdgcn_readfirstlane((int)threadIdx.x) < NH),
        hs(sm_.hs + (threadIdx.x & (SM::REPS - 1))), hg(sm_.hg + (threadIdx.x & (REP - 1))),
        hgl(sm_.hgs + (threadIdx.x & 63)) {
    x = (int)((P0 + (int64_t)tt * PX) % W);
  }

  // counter of raw gradient level g for this lane
  __device__ uint32_t* gslot(uint32_t g) const { return g < GSMALL ? hgl + g * 64 : hg + g * SD; }

  __device__ const uint8_t* chunk_or_first(int64_t at) const {
    const int64_t p = at + (int64_t)tt * PX;
    return d.in + (p + PX <= E ? p : 0) * CB;
  }

  // producer: load step starting at `at` into the ring, V histogram below P1
  __device__ void load_step(int64_t at, const uint32_t (&w)[NW], bool have) {
    const int64_t p = at + (int64_t)tt * PX;
    const int n = (int)max((int64_t)0, min((int64_t)PX, E - p));
    if (n <= 0) return;
    uint32_t v[PX];
    uint32_t packed[NV];
    bool done_v = false;
    if constexpr (BITS == 8 && PX == 16 && NW == 12 && NV == 4) {
      if (have) {
        values_packed_8(w, v, packed);
        done_v = true;
      }
    }
    if (!done_v) {
      if (have) values_of_words<BITS, PX, NW>(w, v, clamped);
      else load_values<BITS, NH>(d, p, n, v, clamped);
#pragma unroll
      for (int q = 0; q < NV; ++q) packed[q] = 0;
#pragma unroll
      for (int i = 0; i < PX; ++i) set_lane<pix_t>(packed, i, v[i]);
    }
    const uint32_t boff = (uint32_t)(((p - P0) & (RING - 1)) * ESZ);
    ring_write<NV>(sm.ring, boff, packed);
    if (boff < 64) ring_write<NV>(sm.ring, RING_BYTES + boff, packed);
    lds_wait();  // the ring stores are done before this wave's barrier
    const int64_t nh = P1 - p;
    if (nh >= PX) {
#pragma unroll
      for (int i = 0; i < PX; ++i) atomicAdd(&hs[v[i] * SM::STRIDES], 1u);
    } else {
#pragma unroll
      for (int i = 0; i < PX; ++i)
        if (i < nh) atomicAdd(&hs[v[i] * SM::STRIDES], 1u);
    }
  }

  // consumer: gradient of the pixels [at, min(at + STEP, P1))
  __device__ void grad_step(int64_t at) {
    static_assert(NV == 4 && PX * ESZ == 16, "one 16-byte ring chunk per thread");
    const uint8_t* ringb = reinterpret_cast<const uint8_t*>(sm.ring);
    const int64_t dend = min(at + STEP, P1);
    const int64_t q = at + (int64_t)tt * PX;
    const int n = (int)max((int64_t)0, min((int64_t)PX, dend - q));
    // Own chunk: q - P0 is a multiple of PX, so the chunk is one aligned
    // 16-byte read (consecutive lanes, consecutive chunks: no bank
    // conflicts).  Its right neighbour is the next lane's first pixel (the
    // last lane of the wave reads it from the ring).  All lanes take part.
    const uint32_t boff = (uint32_t)(((q - P0) & (RING - 1)) * ESZ);
    const v4u ov = *reinterpret_cast<const v4u*>(ringb + boff);
    const uint32_t own[NV] = {ov.x, ov.y, ov.z, ov.w};
    uint32_t right_last = dpp_get<dpp::WAVE_SHL1, 0xf>(own[0]);
    if ((threadIdx.x & 63) == 63) right_last = reinterpret_cast<const uint32_t*>(ringb + boff + 16)[0];
    right_last &= ESZ == 1 ? 0xffu : 0xffffu;
    if (n > 0) {
      // Chunk one row down: it starts W pixels on, at the same byte offset
      // mod 16 in every lane (W ESZ mod 16), so two aligned 16-byte reads
      // and a shift by that wave-uniform offset.
      const uint32_t dboff = (uint32_t)(((q + W - P0) & (RING - 1)) * ESZ);
      const uint32_t dbase = dboff & ~15u, sh = dboff & 3u;
      const int dsel = __builtin_amdgcn_readfirstlane((int)((dboff >> 2) & 3u));
      const v4u d0 = *reinterpret_cast<const v4u*>(ringb + dbase);
      const v4u d1 = *reinterpret_cast<const v4u*>(ringb + dbase + 16);
      const uint32_t w8[8] = {d0.x, d0.y, d0.z, d0.w, d1.x, d1.y, d1.z, d1.w};
      uint32_t dn[NV];
      switch (dsel) {
        case 0:
#pragma unroll
          for (int k = 0; k < NV; ++k) dn[k] = __builtin_amdgcn_alignbyte(w8[k + 1], w8[k], sh);
          break;
        case 1:
#pragma unroll
          for (int k = 0; k < NV; ++k) dn[k] = __builtin_amdgcn_alignbyte(w8[k + 2], w8[k + 1], sh);
          break;
        case 2:
#pragma unroll
          for (int k = 0; k < NV; ++k) dn[k] = __builtin_amdgcn_alignbyte(w8[k + 3], w8[k + 2], sh);
          break;
        default:
#pragma unroll
          for (int k = 0; k < NV; ++k) dn[k] = __builtin_amdgcn_alignbyte(w8[k + 4], w8[k + 3], sh);
          break;
      }
      if (n == PX && N - W - q >= PX && W > PX) {
        if constexpr (BITS == 8) {
          // |right - own| + |down - own| of four pixels per dword: one byte
          // permute packs (right, down) as 16-bit lanes, one packs (own,
          // own), and one SAD adds both differences
#pragma unroll
          for (int wd = 0; wd < 4; ++wd) {
            const uint32_t o = own[wd], dw = dn[wd], nx = wd + 1 < 4 ? own[wd + 1] : right_last;
#pragma unroll
            for (int pp = 0; pp < 4; ++pp) {
              const uint32_t a = pp < 3 ? __builtin_amdgcn_perm(dw, o, 0x0c000c00u | (uint32_t)(pp + 1) | (uint32_t)(4 + pp) << 16)
                                        : __builtin_amdgcn_perm(dw, nx, 0x0c070c00u);
              const uint32_t b = __builtin_amdgcn_perm(o, o, 0x0c000c00u | (uint32_t)pp | (uint32_t)pp << 16);
              atomicAdd(gslot(__builtin_amdgcn_sad_u16(a, b, 0u)), 1u);
            }
          }
        } else {
#pragma unroll
          for (int i = 0; i < PX; ++i) {
            const uint32_t vv = lane_of<pix_t>(own, i);
            const uint32_t vr = (i + 1 < PX) ? lane_of<pix_t>(own, i + 1) : right_last;
            atomicAdd(gslot(grad_l1(vr, vv, lane_of<pix_t>(dn, i))), 1u);
          }
        }
        const int e = W - 1 - x;
        if (e < PX) {
          const uint32_t ve = lane_dyn<pix_t>(own, e);
          const uint32_t vre = (e + 1 < PX) ? lane_dyn<pix_t>(own, e + 1) : right_last;
          const uint32_t vde = lane_dyn<pix_t>(dn, e);
          __hip_atomic_fetch_sub(gslot(grad_l1(vre, ve, vde)), 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
          atomicAdd(gslot(grad_l1(ve, ve, vde)), 1u);
        }
      } else {
        int xx = x;
#pragma unroll
        for (int i = 0; i < PX; ++i) {
          if (i < n) {
            const uint32_t vv = lane_of<pix_t>(own, i);
            const uint32_t vr = (xx + 1 < W) ? ((i + 1 < PX) ? lane_of<pix_t>(own, i + 1) : right_last) : vv;
            const uint32_t vd = (q + i + W < N) ? lane_of<pix_t>(dn, i) : vv;
            atomicAdd(gslot(grad_l1(vr, vv, vd)), 1u);
            if (++xx == W) xx = 0;
          }
        }
      }
    }
    x += step_mod_w;
    if (x >= W) x -= W;
  }

  __device__ void run() {
    const int64_t nload = (E - P0 + STEP - 1) / STEP;   // load steps with pixels
    const int64_t ngrad = (P1 - P0 + STEP - 1) / STEP;  // gradient steps
    const int64_t lag = 1 + (W + STEP) / STEP;          // 1 + ceil((W + 1) / STEP)
    const int64_t K = lag + ngrad;                      // iterations (covers nload)
    int64_t k = 0;
    if (d.in_vec && N >= PX) {
      // The halves run loops of their own, one barrier per iteration each
      // (K in both), so the producer's loads sit outside any branch and the
      // compiler waits only for the oldest step in flight.  `producer` is
      // uniform per wave (NH is a multiple of 64).
      if (producer) {
        const int64_t nfull = (E - P0) / STEP;  // load steps whose chunks are all full
        uint32_t buf[PREFETCH][NW];
#pragma unroll
        for (int j = 0; j < PREFETCH; ++j) load_words<NW>(chunk_or_first(P0 + (int64_t)j * STEP), buf[j]);
        while (k + PREFETCH <= nfull) {
#pragma unroll
          for (int kk = 0; kk < PREFETCH; ++kk) {
            load_step(P0 + k * STEP, buf[kk], true);
            load_words<NW>(chunk_or_first(P0 + (k + PREFETCH) * STEP), buf[kk]);
            bare_barrier();
            ++k;
          }
        }
        while (k < K) {
#pragma unroll
          for (int kk = 0; kk < PREFETCH; ++kk) {
            if (k < K) {  // uniform
              if (k < nload) {
                const int64_t p = P0 + k * STEP + (int64_t)tt * PX;
                load_step(P0 + k * STEP, buf[kk], p + PX <= E);
              }
              load_words<NW>(chunk_or_first(P0 + (k + PREFETCH) * STEP), buf[kk]);
              bare_barrier();
              ++k;
            }
          }
        }
      } else {
        for (; k < K; ++k) {
          if (k >= lag) grad_step(P0 + (k - lag) * STEP);
          bare_barrier();
        }
      }
    } else {
      uint32_t none[NW];
#pragma unroll
      for (int q = 0; q < NW; ++q) none[q] = 0;
      for (; k < K; ++k) {
        if (producer) {
          if (k < nload) load_step(P0 + k * STEP, none, false);
        } else if (k >= lag) {
          grad_step(P0 + (k - lag) * STEP);
        }
        bare_barrier();
      }
    }
  }
};

template <int BITS, int NT>
__device__ void hist_tile(const ImgDesc& d, int64_t P0, int64_t P1, HistSmem<BITS, NT>& sm,
                          uint32_t* __restrict__ g_hs, uint32_t* __restrict__ g_graw) {
  using SM = HistSmem<BITS, NT>;
  constexpr int BINS = Cfg<BITS>::BINS, REP = SM::REP, SD = SM::STRIDE;
  const int t = threadIdx.x;
  for (int i = t; i < BINS * SM::STRIDES; i += NT) sm.hs[i] = 0;
  for (int i = t; i < (2 * BINS - 1) * SD; i += NT) sm.hg[i] = 0;
  for (int i = t; i < SM::GSMALL * 64; i += NT) sm.hgs[i] = 0;
  if (t == 0) sm.clamped = 0;
  __syncthreads();
  uint32_t clamped;
  if constexpr (NT >= 1024) {
    HistTileSplit<BITS, NT> ht(d, P0, P1, sm);
    ht.run();
    clamped = ht.clamped;
  } else {
    HistTile<BITS, NT> ht(d, P0, P1, sm);
    ht.run();
    clamped = ht.clamped;
  }
  if (clamped) atomicOr(&sm.clamped, 1u);
  __syncthreads();
  for (int k = t; k < BINS; k += NT) {
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < SM::REPS; ++r) s += sm.hs[k * SM::STRIDES + r];
    if (s) __hip_atomic_fetch_add(to_global(g_hs) + k, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  for (int k = t; k < 2 * BINS - 1; k += NT) {
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < REP; ++r) s += sm.hg[k * SD + r];
    if (k < SM::GSMALL)
      for (int l = 0; l < 64; ++l) s += sm.hgs[k * 64 + l];  // counts wrap mod 2^32: a copy may hold a -1
    if (s) __hip_atomic_fetch_add(to_global(g_graw) + k, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  // every wave's merge atomics are performed before any thread of the
  // workgroup signals completion of the tile
  drain_memory();
  __syncthreads();
}

// Gradient histogram onto the l levels: raw level j -> round-half-up(j(l-1)/gmax).
// Reads raw counts with device-coherent loads (they were produced by atomics
// of other workgroups).  `tmp` is BINS words of LDS, `red` NT/64 words.
template <int BINS, int NT>
__device__ void rebin_gradient(const uint32_t* g_graw, uint32_t* g_hg, uint32_t* tmp, uint32_t* red) {
  const int t = threadIdx.x;
  uint32_t gm = 0;
  for (int j = t; j < 2 * BINS - 1; j += NT) {
    const uint32_t c = __hip_atomic_load(to_global(g_graw) + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (c) gm = max(gm, (uint32_t)j);
  }
  for (int k = t; k < BINS; k += NT) tmp[k] = 0;
  const uint32_t gmax = block_max<NT>(gm, red);
  for (int j = t; j <= (int)gmax; j += NT) {
    const uint32_t c = __hip_atomic_load(to_global(g_graw) + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (c) {
      const uint32_t q = gmax ? (uint32_t)((2ull * (BINS - 1) * j + gmax) / (2ull * gmax)) : 0u;
      atomicAdd(&tmp[q], c);
    }
  }
  __syncthreads();
  for (int k = t; k < BINS; k += NT) g_hg[k] = tmp[k];
}

// ---------------------------------------------------------------------------
// remap tile: out_c = round-half-up(c * LUT[V] / V) = floor(t) with
// t = (2 c LUT[V] + V) / (2V), black -> LUT[0].  Evaluated as
// trunc(fma(c, ratio[V], bias[V])) from a table in LDS: for V >= 1 ratio is
// LUT[V] / V rounded up to FP32 and bias = 1/2, so c * ratio + 1/2 exceeds t
// by less than 1023 * 2^-23; t is a multiple of 1/(2V) >= 1/2046, hence the
// rounded FMA stays in [floor(t), floor(t) + 1) and truncation is exact.  For
// V = 0 every channel is 0, ratio = 0 and bias = LUT[0] + 1/2.
// ---------------------------------------------------------------------------

__device__ inline float2 remap_entry(uint32_t v, uint32_t L) {
  if (v == 0) return make_float2(0.f, (float)L + 0.5f);
  float r = (float)((double)L / (double)v);
  if ((double)r * (double)v < (double)L) r = __uint_as_float(__float_as_uint(r) + 1u);
  return make_float2(r, 0.5f);
}

template <int BITS, int PX, int NW>
__device__ inline void remap_words(const uint32_t (&w)[NW], uint32_t (&o)[NW], const float2* tab) {
  using pix_t = typename Cfg<BITS>::pix_t;
  constexpr float TOPF = (float)((1u << BITS) - 1);
#pragma unroll
  for (int k = 0; k < NW; ++k) o[k] = 0;
#pragma unroll
  for (int i = 0; i < PX; ++i) {
    float r = (float)lane_of<pix_t>(w, 3 * i), g = (float)lane_of<pix_t>(w, 3 * i + 1),
          b = (float)lane_of<pix_t>(w, 3 * i + 2);
    if (BITS > 8) {
      r = fminf(r, TOPF);
      g = fminf(g, TOPF);
      b = fminf(b, TOPF);
    }
    const float2 e = tab[(uint32_t)fmaxf(fmaxf(r, g), b)];
    set_lane<pix_t>(o, 3 * i, (uint32_t)fmaf(r, e.x, e.y));
    set_lane<pix_t>(o, 3 * i + 1, (uint32_t)fmaf(g, e.x, e.y));
    set_lane<pix_t>(o, 3 * i + 2, (uint32_t)fmaf(b, e.x, e.y));
  }
}

// n (< PX for a partial chunk) pixels from p, one at a time (any row stride)
template <int BITS>
__device__ void remap_pixels(const ImgDesc& d, int64_t p, int n, const float2* tab) {
  using pix_t = typename Cfg<BITS>::pix_t;
  constexpr uint32_t TOP = (1u << BITS) - 1;
  int64_t y = p / d.W;
  int x = (int)(p - y * d.W);
  for (int i = 0; i < n; ++i) {
    const gptr<const pix_t> s = to_global(reinterpret_cast<const pix_t*>(d.in + y * d.in_stride)) + 3 * x;
    const gptr<pix_t> o = to_global(reinterpret_cast<pix_t*>(d.out + y * d.out_stride)) + 3 * x;
    const uint32_t r = min((uint32_t)s[0], TOP), g = min((uint32_t)s[1], TOP), bl = min((uint32_t)s[2], TOP);
    const float2 e = tab[umax3(r, g, bl)];
    o[0] = (pix_t)(uint32_t)fmaf((float)r, e.x, e.y);
    o[1] = (pix_t)(uint32_t)fmaf((float)g, e.x, e.y);
    o[2] = (pix_t)(uint32_t)fmaf((float)bl, e.x, e.y);
    if (++x == d.W) {
      x = 0;
      ++y;
    }
  }
}

// Writes a wave's 48-byte chunks (lane l holds the 12 dwords of pixels
// pw + l PX .., consecutive in memory from out_wave) through the wave's LDS
// stage `sw` (64 x 12 dwords): the chunks go to the stage in lane order and
// come back 16 bytes at a time, so that each store instruction writes one
// contiguous 1 KB stretch instead of 16 bytes every 48.  LDS accesses of one
// wave complete in order, so the wave barriers (which keep the compiler from
// reordering them) are the only waits.
__device__ inline void store_wave_staged(uint8_t* out_wave, const uint32_t (&o)[12], uint32_t* sw) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int q = 0; q < 3; ++q)
    *reinterpret_cast<v4u*>(sw + lane * 12 + 4 * q) = v4u{o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]};
  __builtin_amdgcn_wave_barrier();
  const gptr<v4u> dst = to_global(reinterpret_cast<v4u*>(out_wave));
#pragma unroll
  for (int q = 0; q < 3; ++q)
    __builtin_nontemporal_store(*reinterpret_cast<const v4u*>(sw + 4 * (lane + 64 * q)), dst + lane + 64 * q);
  __builtin_amdgcn_wave_barrier();
}

// Remaps pixels [P0, P1) of d through tab.  stage: NT * 12 dwords of LDS for
// the staged stores of waves whose chunks are all full.
template <int BITS, int NT>
__device__ void remap_tile(const ImgDesc& d, int64_t P0, int64_t P1, const float2* tab, uint32_t* stage) {
  using pix_t = typename Cfg<BITS>::pix_t;
  // 48-byte chunks (16 or 8 pixels, three 16-byte loads) at every workgroup
  // size; the 1024-thread workgroup keeps two in flight per thread, the same
  // bytes as four 24-byte chunks and measured 0.5% faster in the batched
  // launches (three in flight: 1% slower on the 8-bit batch)
  constexpr int PX = 48 / (3 * (int)sizeof(pix_t)), NW = 12, STEP = NT * PX;
  constexpr int PF = NT >= 1024 ? 2 : PREFETCH;
  constexpr int64_t CB = 3 * (int64_t)sizeof(pix_t);
  const bool vec = d.in_vec && d.out_vec;
  // The input is re-read with ordinary loads and the output written with
  // nontemporal stores: measured against nontemporal loads, the ordinary ones
  // take 1.5-2% off the batched launches; ordinary stores add 5-7%.  The
  // staged stores take another 1% off.
  uint32_t* sw = stage + (threadIdx.x >> 6) * (64 * NW);  // this wave's stage
  const int lane = threadIdx.x & 63;
  // chunk j of this thread (pixels p0 + j STEP ..) lives in buf[j mod PF]
  const int64_t p0 = P0 + (int64_t)threadIdx.x * PX;
  uint32_t buf[PF][NW];
#pragma unroll
  for (int j = 0; j < PF; ++j) {
    const int64_t p = p0 + (int64_t)j * STEP;
    if (vec && p + PX <= P1) load_words<NW>(d.in + p * CB, buf[j]);
  }
  for (int64_t p = p0; p < P1;) {
#pragma unroll
    for (int k = 0; k < PF; ++k) {
      if (p < P1) {
        const int n = (int)min((int64_t)PX, P1 - p);
        if (vec && n == PX) {
          uint32_t o[NW];
          remap_words<BITS, PX, NW>(buf[k], o, tab);
          const int64_t pf = p + (int64_t)PF * STEP;
          if (pf + PX <= P1) load_words<NW>(d.in + pf * CB, buf[k]);
          const int64_t pw = p - (int64_t)lane * PX;  // the wave's first pixel
          if (pw + 64 * PX <= P1)  // every chunk of the wave is full
            store_wave_staged(d.out + pw * CB, o, sw);
          else
            store_words_nt<NW>(d.out + p * CB, o);
        } else {
          remap_pixels<BITS>(d, p, n, tab);
        }
        p += STEP;
      }
    }
  }
}

// Remap table from a LUT in global memory.
template <int BINS, int NT>
__device__ inline void load_remap_table(const uint16_t* lut, float2* tab) {
  for (int v = threadIdx.x; v < BINS; v += NT) tab[v] = remap_entry((uint32_t)v, (uint32_t)lut[v]);
}

// ---------------------------------------------------------------------------
// matching LUT: LUT[v] = min{k : F~(k) >= u(v)}, u(v) = (cS(v-1) + cS(v)) / 2N,
// F~(k) = C(k) / C(l-1), C the running sum of the target histogram (FP64).
// ---------------------------------------------------------------------------

template <int BINS, int NT>
struct LutSmem {
  double F[BINS];
  uint64_t cs[BINS];
  double redd[NT / 64];
  uint64_t redu[NT / 64];
};

template <int BINS, int NT>
__device__ void build_lut(const uint32_t* hS, const float* target, LutSmem<BINS, NT>& sm, uint16_t* lut_out) {
  const int t = threadIdx.x;
  for (int k = t; k < BINS; k += NT) {
    sm.F[k] = (double)target[k];
    sm.cs[k] = hS[k];
  }
  __syncthreads();
  const double Ctot = block_scan<NT, double, true>(sm.F, BINS, sm.redd);
  const uint64_t N = block_scan<NT, uint64_t, true>(sm.cs, BINS, sm.redu);
  // running maximum: the scan's association can dip by an ulp across thread
  // blocks; the first index reaching u is the same for C and its running max
  {
    const int per = (BINS + NT - 1) / NT;
    const int b0 = min(t * per, BINS), b1 = min(b0 + per, BINS);
    double m = -1.0;
    for (int i = b0; i < b1; ++i) m = max(m, sm.F[i]);
    // inclusive max-scan of thread maxima
    double inc = m;
    const int lane = t & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      double y = __shfl_up(inc, o, 64);
      if (lane >= o) inc = max(inc, y);
    }
    __syncthreads();
    if (lane == 63) sm.redd[t >> 6] = inc;
    __syncthreads();
    double run = -1.0;
    for (int i = 0; i < (t >> 6); ++i) run = max(run, sm.redd[i]);
    double ex = __shfl_up(inc, 1, 64);
    if (lane > 0) run = max(run, ex);
    for (int i = b0; i < b1; ++i) {
      run = max(run, sm.F[i]);
      sm.F[i] = run;
    }
    __syncthreads();
  }
  for (int k = t; k < BINS; k += NT) sm.F[k] = sm.F[k] / Ctot;
  __syncthreads();
  const double twoN = 2.0 * (double)N;
  for (int v = t; v < BINS; v += NT) {
    const uint64_t c = sm.cs[v];
    const uint64_t h = hS[v];
    const double u = (double)(2 * c - h) / twoN;
    int lo = 0, hi = BINS - 1;  // F[BINS-1] = 1 >= u
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (sm.F[mid] >= u)
        hi = mid;
      else
        lo = mid + 1;
    }
    lut_out[v] = (uint16_t)lo;
  }
}

// ---------------------------------------------------------------------------
// solver
//
// Histograms are kept compacted over their occupied levels: A = supp H_C(S)
// (illumination levels a), B = supp H_C(grad S) (reflectance levels b).  The
// updates keep L and R zero outside A and B, and every cell outside A x B
// contributes an exact zero, so the sweeps run over A x B only:
//   class sweep  d_m = sum_{index(a,b)=m} L_a R_b       (Eq. 8 with Eq. 6)
//   column sweep u_b = sum_a L_a^2 rho_index(a,b)        (Eq. 13, K = L R / d)
//   row sweep    v_a = sum_b R'_b R_b rho_index(a,b)     (Eq. 12)
// with rho_m = s_m / d_m, so that K_ab s_index(a,b) = L_a R_b rho_index(a,b).
//
// The loops are shaped for issue rate: every lane of a wave runs the same
// trip count (chunks and slices are padded with cells that point at a zero),
// the class of a cell comes from a table built once per image, and partial
// sums are combined inside a wave (butterflies, segmented scans).  Every sum
// has a fixed association, so results do not depend on timing.
// ---------------------------------------------------------------------------

template <int BINS> struct CellT;
template <> struct CellT<256> {
  using type = uint16_t;
  static constexpr int SHIFT = 8;
};
template <> struct CellT<1024> {
  using type = uint32_t;
  static constexpr int SHIFT = 10;
};

template <int BINS, int NT>
struct SolveCore {
  static constexpr int RMAX = BINS == 256 ? 2 : 1;  // rounds of chunks per lane
  static constexpr int PAD = BINS + 256;            // zero padding of the sweep inputs (G * L <= 2n + 256)
  float sc[BINS], gc[BINS];                         // s, g on A, B
  float lc[BINS + 4], rc[BINS + 4];                 // current L on A, R on B; [n] = 0
  alignas(16) float l2c[BINS + PAD];                // L^2 on A (zero padded), later L'
  alignas(16) float wc[BINS + PAD];                 // R' R on B (zero padded)
  alignas(16) float af[BINS + PAD];                 // levels a of A as floats (zero padded)
  alignas(16) float bq[BINS + PAD];                 // levels b of B over (l-1), FP32 (zero padded)
  float lraw[BINS + 4];                             // L' of Eq. (12) on A, before Eq. (15); [n] = 0
  float rn[BINS + 4];                               // R' of Eq. (13) on B, before Eq. (14); [n] = 0
  // running sums of R by level (class totals without a list).  At 1024 levels
  // the entries past l repeat the total, up to the largest run bound a class
  // group reaches (E(4) on row a = 1: floor(7 (l-1) / 2) + 1 = 3581), so the
  // bounds need no clamp to l.
  static constexpr int RCUM = BINS == 1024 ? 7 * (BINS - 1) / 2 + 2 : BINS + 1;
  double rcum[RCUM];
  float sd[BINS];                                   // s by level (dense)
  float inv2a[BINS];                                // 1 / (2a) for the rows of A
  alignas(8) float rho[BINS + 4];                   // s_m / d_m by class
  uint16_t A[BINS], B[BINS];
  int32_t off[BINS + 1];                            // first chunk of class m
  int32_t csz[BINS];                                // cells of class m
  int32_t PA[BINS + 1], PB[BINS + 1];               // occupied levels below a / b
  int32_t lane_cells[NT];                           // list build: cells of each lane's rows, then their rank
  int16_t chunk_cls[RMAX * NT];                     // class of chunk u (-1: padding)
  float redf[5][NT / 64];  // wave partials: sum L^2, sum R'', sum L', change of L, change of R
  uint64_t redu[NT / 64];
  double redd[NT / 64];
  int32_t redi[NT / 64];
  int32_t nA, nB, nc, C, CS, R, nAp, nBp;           // CS: cell stride of a chunk
  int32_t tab_lds, use_list;
};

// The class list and the class tables take the LDS left in `budget` bytes.
template <int BINS, int NT, int BUDGET>
struct SolveSmem : SolveCore<BINS, NT> {
  static constexpr int FREE = BUDGET - (int)sizeof(SolveCore<BINS, NT>) > 64
                                  ? BUDGET - (int)sizeof(SolveCore<BINS, NT>)
                                  : 64;
  alignas(16) uint32_t spare[FREE / 4];
  // the target sums (BINS x u64) and the gamma table (BINS doubles) reuse spare
  static_assert(FREE >= 16 * BINS, "LDS budget too small for the solver");
};

// index(a, b) of Eq. (10): nearest level of a*b/(l-1)^2 on the grid k/(l-1),
// i.e. round(a*b/(l-1)); l-1 is odd so there are no ties.
template <int BINS>
__device__ inline int class_of(int a, int b) {
  constexpr uint32_t D = BINS - 1;
  return (int)((2u * (uint32_t)a * (uint32_t)b + D) / (2u * D));
}

// Reflectance levels b of class m in illumination row a = A[i], for a >= m
// (the only rows that reach class m): the b with
// (2m-1)(l-1) < 2ab < (2m+1)(l-1), as a compacted index range [jlo, jhi) of
// B (jlo = jhi: empty).  Both bounds (2m +- 1)(l-1) / 2a are odd multiples of
// l-1 over an even number, so they lie at least 1/2a from an integer, and
// below 1.5 (l-1); the FP32 product with the rounded reciprocal 1/2a is within
// 2^-23 relative, under 2e-4, so truncation gives the exact floors.  The lower
// bound's + 1 goes into the same FMA (one more rounding of at most 2^-13 below
// 2^11): still exact (checked for every a and m <= a at l = 256 and 1024).
template <int BINS, typename SM>
__device__ inline void class_run_upper(const SM& sm, int i, int m, int& jlo, int& jhi) {
  constexpr uint32_t D = BINS - 1;
  const int a = sm.A[i];
  if (a == 0) {  // m = 0: the whole row
    jlo = 0;
    jhi = sm.nB;
    return;
  }
  const float inv = sm.inv2a[i];
  const uint32_t blo = m == 0 ? 0u : (uint32_t)fmaf((float)((2u * m - 1u) * D), inv, 1.f);
  const uint32_t bhi = min((uint32_t)((float)((2u * m + 1u) * D) * inv), (uint32_t)(BINS - 1));
  jlo = sm.PB[blo];
  jhi = sm.PB[max(bhi + 1u, blo)];  // blo > bhi: empty
}

template <int NT>
__device__ inline void wave_partial(float x, float* red) {
  x = wave_scan(x);
  if ((threadIdx.x & 63) == 63) red[threadIdx.x >> 6] = x;
}

// Block sums of the wave partials in ra and rb (NT / 64 <= 16 entries each),
// in every lane: one LDS read per wave (row 0 of the wave takes ra, row 1
// takes rb), a scan inside the rows, then lanes 15 and 31.  Every wave adds
// in the same order, so all lanes get the same bits.
template <int NT>
__device__ inline float2 block_read2(const float* ra, const float* rb) {
  constexpr int NW = NT / 64;
  static_assert(NW <= 16, "one row of lanes per array");
  const int lane = threadIdx.x & 63;
  float x = 0.f;
  if (lane < NW)
    x = ra[lane];
  else if (lane >= 16 && lane < 16 + NW)
    x = rb[lane - 16];
  x += dpp_get<dpp::ROW_SHR + 1, 0xf>(x);
  x += dpp_get<dpp::ROW_SHR + 2, 0xf>(x);
  x += dpp_get<dpp::ROW_SHR + 4, 0xf>(x);
  x += dpp_get<dpp::ROW_SHR + 8, 0xf>(x);
  return make_float2(read_lane(x, 15), read_lane(x, 31));
}

template <int NT>
__device__ inline float block_read(const float* red) {
  constexpr int NW = NT / 64;
  static_assert(NW <= 16, "one row of lanes");
  const int lane = threadIdx.x & 63;
  float x = lane < NW ? red[lane] : 0.f;
  x += dpp_get<dpp::ROW_SHR + 1, 0xf>(x);
  x += dpp_get<dpp::ROW_SHR + 2, 0xf>(x);
  x += dpp_get<dpp::ROW_SHR + 4, 0xf>(x);
  x += dpp_get<dpp::ROW_SHR + 8, 0xf>(x);
  return read_lane(x, 15);
}

// largest power of two <= x (x >= 1), capped at 64
__device__ inline int pow2_floor64(int x) {
  int p = 1;
  while (p * 2 <= x && p < 64) p *= 2;
  return p;
}

template <int BINS, int NT, int BUDGET>
__device__ inline typename CellT<BINS>::type* cell_store(SolveSmem<BINS, NT, BUDGET>& sm) {
  return reinterpret_cast<typename CellT<BINS>::type*>(sm.spare);
}

// Class tables (256 levels only), after the class list in LDS: tab[i*nBp + j]
// = index(A[i], B[j]) for the row sweep and tabT[j*nAp + i] for the column
// sweep, one byte per cell.
template <int BINS, int NT, int BUDGET>
__device__ inline uint8_t* class_table(SolveSmem<BINS, NT, BUDGET>& sm) {
  using cell_t = typename CellT<BINS>::type;
  return reinterpret_cast<uint8_t*>(sm.spare) + (((size_t)sm.R * NT * sm.CS * sizeof(cell_t) + 15) & ~(size_t)15);
}

// Lanes of the class sweep without a list.  Class q (level A[q]) collects
// the rows q..nA-1 (a >= A[q]; lower rows never reach class A[q]), so the
// classes carry nA, nA-1, ..., 1 rows.  With at most c rows per lane, class q
// gets ceil((nA - q) / c) consecutive lanes; c is the smallest value for
// which all classes fit in NT lanes (c = 1 when nA (nA + 1) / 2 <= NT).
struct ClassLanes {
  int q, k, g, c;  // class index (-1: idle lane), lane within the class, lanes of the class, rows per lane
};

// sum_{w=1..n} ceil(w / c)
__device__ inline int lanes_upto(int n, int c) {
  const int k = n / c, r = n - k * c;
  return c * (k * (k + 1) / 2) + r * (k + 1);
}

template <int NT>
__device__ inline ClassLanes class_lanes(int nA, int t) {
  ClassLanes r{-1, 0, 1, 1};
  if (nA <= 0) return r;
  int lo = 1, hi = nA;  // lanes_upto(nA, nA) = nA <= NT
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (lanes_upto(nA, mid) <= NT)
      hi = mid;
    else
      lo = mid + 1;
  }
  const int c = lo, total = lanes_upto(nA, c);
  r.c = c;
  if (t >= total) return r;
  // first lane of class q: total - lanes_upto(nA - q, c), increasing in q
  int a = 0, b = nA - 1;
  while (a < b) {
    const int mid = (a + b + 1) >> 1;
    if (total - lanes_upto(nA - mid, c) <= t)
      a = mid;
    else
      b = mid - 1;
  }
  r.q = a;
  r.k = t - (total - lanes_upto(nA - a, c));
  r.g = (nA - a + c - 1) / c;
  return r;
}

// Lanes of the class sweep without a list: the levels in groups of CK
// consecutive classes (group p: classes CK p .. CK p + CK - 1, up to the
// largest level of A), reached by the rows a >= CK p.  With at most c rows
// per lane, group p gets ceil(rows_p / c) consecutive lanes; c is the
// smallest value for which all groups fit in NT lanes.  first: LDS scratch
// of P + 1 ints.  Every thread of the block calls it.
template <int BINS, int NT, int CK>
__device__ ClassLanes group_lanes(SolveCore<BINS, NT>& sm, int* first) {
  const int t = threadIdx.x, nA = sm.nA;
  const int P = sm.A[nA - 1] / CK + 1;  // <= BINS / CK <= NT
  if (t < 64) {
    int lo = 1, hi = nA;  // c = nA: one lane per group
    while (lo < hi) {
      const int c = (lo + hi) >> 1;
      int n = 0;
      for (int q = t; q < P; q += 64) n += (nA - sm.PA[CK * q] + c - 1) / c;
      if (wave_sum(n) <= NT)
        hi = c;
      else
        lo = c + 1;
    }
    if (t == 0) sm.redi[0] = lo;
  }
  __syncthreads();
  const int c = sm.redi[0];
  for (int q = t; q <= P; q += NT) first[q] = q < P ? (nA - sm.PA[CK * q] + c - 1) / c : 0;
  __syncthreads();
  block_scan<NT, int32_t>(first, P + 1, sm.redi);
  ClassLanes r{-1, 0, 1, c};
  if (t < first[P]) {
    int a = 0, b = P - 1;  // last group whose first lane is <= t
    while (a < b) {
      const int mid = (a + b + 1) >> 1;
      if (first[mid] <= t)
        a = mid;
      else
        b = mid - 1;
    }
    r.q = a;
    r.k = t - first[a];
    r.g = first[a + 1] - first[a];
  }
  __syncthreads();
  return r;
}

// Cell words of a class-list chunk, four at a time.
template <typename cell_t>
__device__ __forceinline__ void cells_of(const cell_t* q, uint32_t* e) {
  if constexpr (sizeof(cell_t) == 2) {
    const v2u w = *reinterpret_cast<const v2u*>(q);
    e[0] = w.x & 0xffffu;
    e[1] = w.x >> 16;
    e[2] = w.y & 0xffffu;
    e[3] = w.y >> 16;
  } else {
    const v4u w = *reinterpret_cast<const v4u*>(q);
    e[0] = w.x;
    e[1] = w.y;
    e[2] = w.z;
    e[3] = w.w;
  }
}

// sum over s in [s0, s1) of x[s] rho[class], classes one byte each from the
// table row (4 per word, zero past np); s0 and s1 - s0 multiples of 4, x
// zero-padded.  Four partial sums (s mod 4) in fixed order; eight cells at a
// time with all gathers issued before the first product.
__device__ __forceinline__ float table_dot(const float* x, const uint32_t* trow, const float* rho, int s0, int s1,
                                           int np) {
  float a4[4] = {0.f, 0.f, 0.f, 0.f};
  int s = s0;
  for (; s + 8 <= s1; s += 8) {
    const v4u x0 = *reinterpret_cast<const v4u*>(x + s);
    const v4u x1 = *reinterpret_cast<const v4u*>(x + s + 4);
    const uint32_t c0 = s < np ? trow[s >> 2] : 0u;
    const uint32_t c1 = s + 4 < np ? trow[(s >> 2) + 1] : 0u;
    float r[8];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      r[q] = rho[(c0 >> (8 * q)) & 0xffu];
      r[4 + q] = rho[(c1 >> (8 * q)) & 0xffu];
    }
    __builtin_amdgcn_sched_barrier(0);
    a4[0] = fmaf(__uint_as_float(x0.x), r[0], a4[0]);
    a4[1] = fmaf(__uint_as_float(x0.y), r[1], a4[1]);
    a4[2] = fmaf(__uint_as_float(x0.z), r[2], a4[2]);
    a4[3] = fmaf(__uint_as_float(x0.w), r[3], a4[3]);
    a4[0] = fmaf(__uint_as_float(x1.x), r[4], a4[0]);
    a4[1] = fmaf(__uint_as_float(x1.y), r[5], a4[1]);
    a4[2] = fmaf(__uint_as_float(x1.z), r[6], a4[2]);
    a4[3] = fmaf(__uint_as_float(x1.w), r[7], a4[3]);
  }
  if (s < s1) {
    const v4u x0 = *reinterpret_cast<const v4u*>(x + s);
    const uint32_t c0 = s < np ? trow[s >> 2] : 0u;
    float r[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) r[q] = rho[(c0 >> (8 * q)) & 0xffu];
    __builtin_amdgcn_sched_barrier(0);
    a4[0] = fmaf(__uint_as_float(x0.x), r[0], a4[0]);
    a4[1] = fmaf(__uint_as_float(x0.y), r[1], a4[1]);
    a4[2] = fmaf(__uint_as_float(x0.z), r[2], a4[2]);
    a4[3] = fmaf(__uint_as_float(x0.w), r[3], a4[3]);
  }
  return (a4[0] + a4[1]) + (a4[2] + a4[3]);
}

// Class of a level pair from a (as a float) and b / (l-1) (FP32), in either
// order: the product rounded to the nearest integer by one fused add of 2^23
// (the low mantissa bits of the sum are then the integer).  Exact for every
// a, b < l at l = 256 and 1024: the product of the two floats is within
// 1.3e-4 of a b / (l-1), which lies at least 1/(2(l-1)) from a half-integer.
__device__ __forceinline__ uint32_t class_of(float u, float v) {
  return __float_as_uint(fmaf(u, v, 8388608.f)) - 0x4B000000u;
}

// sum over s in [s0, s1) of x[s] rho[index(a, b)] with the class from
// class_of (u[s] and v are a and b / (l-1), in either order).  s0 and
// s1 - s0 multiples of 4; x and u zero-padded.  Same shape as table_dot.
__device__ __forceinline__ float class_dot(const float* x, const float* u, float v, const float* rho, int s0,
                                           int s1) {
  float a4[4] = {0.f, 0.f, 0.f, 0.f};
  int s = s0;
  for (; s + 8 <= s1; s += 8) {
    const v4u x0 = *reinterpret_cast<const v4u*>(x + s);
    const v4u x1 = *reinterpret_cast<const v4u*>(x + s + 4);
    const v4u u0 = *reinterpret_cast<const v4u*>(u + s);
    const v4u u1 = *reinterpret_cast<const v4u*>(u + s + 4);
    const uint32_t uu[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
    float r[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) r[q] = rho[class_of(__uint_as_float(uu[q]), v)];
    __builtin_amdgcn_sched_barrier(0);
    a4[0] = fmaf(__uint_as_float(x0.x), r[0], a4[0]);
    a4[1] = fmaf(__uint_as_float(x0.y), r[1], a4[1]);
    a4[2] = fmaf(__uint_as_float(x0.z), r[2], a4[2]);
    a4[3] = fmaf(__uint_as_float(x0.w), r[3], a4[3]);
    a4[0] = fmaf(__uint_as_float(x1.x), r[4], a4[0]);
    a4[1] = fmaf(__uint_as_float(x1.y), r[5], a4[1]);
    a4[2] = fmaf(__uint_as_float(x1.z), r[6], a4[2]);
    a4[3] = fmaf(__uint_as_float(x1.w), r[7], a4[3]);
  }
  if (s < s1) {
    const v4u x0 = *reinterpret_cast<const v4u*>(x + s);
    const v4u u0 = *reinterpret_cast<const v4u*>(u + s);
    const uint32_t uu[4] = {u0.x, u0.y, u0.z, u0.w};
    float r[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) r[q] = rho[class_of(__uint_as_float(uu[q]), v)];
    __builtin_amdgcn_sched_barrier(0);
    a4[0] = fmaf(__uint_as_float(x0.x), r[0], a4[0]);
    a4[1] = fmaf(__uint_as_float(x0.y), r[1], a4[1]);
    a4[2] = fmaf(__uint_as_float(x0.z), r[2], a4[2]);
    a4[3] = fmaf(__uint_as_float(x0.w), r[3], a4[3]);
  }
  return (a4[0] + a4[1]) + (a4[2] + a4[3]);
}

// For w = 0..3: out[w] = sum over s in [s0, s1) of x[s] rho[index(a, b)]
// with the class from class_of (u[s] and v[w] are a and b / (l-1), in either
// order).  The four sums share each read of x and u.  s0 and s1 - s0
// multiples of 4; x and u zero-padded.
__device__ __forceinline__ void class_dot4(const float* x, const float* u, const float (&v)[4], const float* rho,
                                           int s0, int s1, float (&out)[4]) {
  float a[4][2] = {{0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}, {0.f, 0.f}};
  for (int s = s0; s < s1; s += 4) {
    const v4u x0 = *reinterpret_cast<const v4u*>(x + s);
    const v4u u0 = *reinterpret_cast<const v4u*>(u + s);
    const float xx[4] = {__uint_as_float(x0.x), __uint_as_float(x0.y), __uint_as_float(x0.z), __uint_as_float(x0.w)};
    const float uu[4] = {__uint_as_float(u0.x), __uint_as_float(u0.y), __uint_as_float(u0.z), __uint_as_float(u0.w)};
    float r[4][4];
#pragma unroll
    for (int w = 0; w < 4; ++w)
#pragma unroll
      for (int q = 0; q < 4; ++q) r[w][q] = rho[class_of(uu[q], v[w])];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int w = 0; w < 4; ++w)
#pragma unroll
      for (int q = 0; q < 4; ++q) a[w][q & 1] = fmaf(xx[q], r[w][q], a[w][q & 1]);
  }
#pragma unroll
  for (int w = 0; w < 4; ++w) out[w] = a[w][0] + a[w][1];
}

// Dense sweep without a class list, first pass: out[o] = sum over the nin
// inputs s of x[s] rho[index] (u[s], vout[o] as in class_dot4).  The inputs
// are cut into G slices; lane j of slice k takes the outputs j, j + S,
// j + 2S, j + 3S (S = ceil(nout / 4)), so the lanes of a wave read the same
// x and u and gather rho at neighbouring classes.  part[k * 4S + o] gets
// slice k's sum for output o; sweep_total adds the slices up.
template <int NT>
__device__ inline void sweep_part(int nout, int nin, const float* x, const float* u, const float* vout,
                                  const float* rho, float* part) {
  const int t = threadIdx.x;
  const int S = (nout + 3) >> 2, ninp = (nin + 3) & ~3;
  const int G = min(min(NT / S, 32), ninp >> 2);
  const int L = ((ninp + G - 1) / G + 3) & ~3;
  const int k = t / S, j = t - k * S;
  if (k < G) {
    const int s0 = k * L, s1 = min(s0 + L, ninp);
    const float v[4] = {vout[j], vout[j + S], vout[j + 2 * S], vout[j + 3 * S]};
    float acc[4];
    class_dot4(x, u, v, rho, s0, max(s0, s1), acc);
#pragma unroll
    for (int w = 0; w < 4; ++w) part[k * 4 * S + w * S + j] = acc[w];
  }
}

// Second pass: the total of output o, slices in order.
template <int NT>
__device__ inline float sweep_total(int o, int nout, int nin, const float* part) {
  const int S = (nout + 3) >> 2, ninp = (nin + 3) & ~3;
  const int G = min(min(NT / S, 32), ninp >> 2);
  float acc = part[o];
  for (int k = 1; k < G; ++k) acc += part[k * 4 * S + o];
  return acc;
}

// Largest nA nB for which the class list is used at 256 levels: measured on
// one CU, the list form's passes cost about 2 us + 0.25 us per thousand
// cells (the list gathers two values per cell) and the running-sum form's
// about 5 us + 0.09 us per thousand; with the list's build included the two
// totals cross between 36k cells (list 462 us, running sums 482 us) and 44k
// (655 us against 534 us).
constexpr int64_t LIST_MAX_CELLS = 40000;

// Class-major list of the cells (i, j) of A x B whose class has s_m > 0
// (other classes have rho = 0 and their totals are never used), cut into
// chunks of exactly C cells (C a multiple of 4; the last chunk of a class
// padded with a cell pointing at zeros).  Chunks are laid out over R rounds of
// NT lanes; the chunks of a class are consecutive and never cross a 64-chunk
// boundary, so a class is summed inside one wave of one round.  Within a
// class the cells are ordered by row and column.  Chunk u holds its cells
// contiguously from u * CS.  256 levels only.  The list is built, and used,
// only when the occupied cells nA nB are at most LIST_MAX_CELLS and the list
// fits in LDS; larger images take the running-sum form of the class totals.
template <int BINS, int NT, int BUDGET>
__device__ __forceinline__ void build_class_list(SolveSmem<BINS, NT, BUDGET>& sm) {
  using cell_t = typename CellT<BINS>::type;
  constexpr int SH = CellT<BINS>::SHIFT;
  constexpr int MAXCH = 32;  // chunks per class
  constexpr int RMAX = SolveCore<BINS, NT>::RMAX;
  static_assert(BINS <= NT * RMAX / 2, "every class must get a chunk");
  const int t = threadIdx.x;
  const int nA = sm.nA, nB = sm.nB;
  if ((int64_t)nA * nB > LIST_MAX_CELLS) {  // the same in every thread
    if (t == 0) {
      sm.use_list = 0;
      sm.tab_lds = 0;
      sm.C = 0;
      sm.CS = 0;
      sm.R = 0;
      sm.nAp = (nA + 3) & ~3;
      sm.nBp = (nB + 3) & ~3;
    }
    __syncthreads();
    return;
  }
  // The (class, row) pairs over balanced lanes (class q = A[q] has the rows
  // q..nA-1), each lane a contiguous range of its class's rows: the lane's
  // cells, then its rank in the class's row-major order from the lanes before
  const ClassLanes cl = class_lanes<NT>(nA, t);
  int mcls = -1, i0 = 0, i1 = 0, mine = 0;
  if (cl.q >= 0) {
    mcls = sm.A[cl.q];
    i0 = cl.q + cl.k * cl.c;
    i1 = min(i0 + cl.c, nA);
    for (int i = i0; i < i1; ++i) {
      int jlo, jhi;
      class_run_upper<BINS>(sm, i, mcls, jlo, jhi);
      mine += jhi - jlo;
    }
  }
  sm.lane_cells[t] = mine;
  for (int u = t; u < RMAX * NT; u += NT) sm.chunk_cls[u] = -1;
  for (int m = t; m < BINS; m += NT) sm.csz[m] = 0;
  // the levels as the class tables take them: a, and b / (l-1) in FP32
  // (zero padded)
  for (int q = t; q < BINS + SolveCore<BINS, NT>::PAD; q += NT) {
    sm.af[q] = q < nA ? (float)sm.A[q] : 0.f;
    sm.bq[q] = q < nB ? (float)sm.B[q] / (float)(BINS - 1) : 0.f;
  }
  __syncthreads();
  // the lanes of a class are consecutive: the cells of the class's lanes
  // before this one are a difference of two block prefix sums
  block_scan<NT, int32_t>(sm.lane_cells, NT, sm.redi);
  int before = 0;
  if (cl.q >= 0) {
    before = sm.lane_cells[t] - sm.lane_cells[t - cl.k];
    if (cl.k == cl.g - 1) sm.csz[mcls] = before + mine;
  }
  __syncthreads();
  sm.lane_cells[t] = before;  // rank of the lane's first cell in its class (read after the layout's barrier)
  int mx = 0, tot = 0;
  for (int m = t; m < BINS; m += NT) {
    const int c = sm.csz[m];
    mx = max(mx, c);
    tot += c;
  }
  // largest class and total cells in one block reduction
  mx = wave_max(mx);
  tot = wave_sum(tot);
  if ((t & 63) == 0) {
    sm.redi[t >> 6] = mx;
    sm.redu[t >> 6] = (uint64_t)tot;
  }
  __syncthreads();
  int nc = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
    mx = max(mx, sm.redi[i]);
    nc += (int)sm.redu[i];
  }
  if (t < 64) {
    // one wave lays the chunks out, classes in order, each class's chunks
    // inside one 64-chunk group: a class that would straddle a group
    // boundary starts the next group.  Per block of 64 classes (one per
    // lane) the positions are a prefix sum of the chunk counts; the first
    // straddling class is moved to the next boundary and the scan repeated
    // until none straddles, which is the sequential greedy result.  The
    // chunk size starts at about one round of chunks and grows until the
    // layout fits RMAX rounds; it fits at the latest when every class has one
    // chunk (C >= mx): at most BINS chunks and no padding.
    constexpr int Q = (BINS + 63) / 64;
    const int lane = t;
    int cs[Q], offs[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      cs[q] = sm.csz[q * 64 + lane];
      offs[q] = 0;
    }
    int C = max(4, max((mx + MAXCH - 1) / MAXCH, (nc + NT - 1) / NT));
    C = (C + 3) & ~3;
    int pos = 0;
    for (;;) {
      pos = 0;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const int nv = (cs[q] + C - 1) / C;
        int pad = 0;
        for (int guard = 0; guard <= 64; ++guard) {
          const int w = nv + pad;
          const int incl = wave_scan(w);
          offs[q] = pos + incl - nv;  // start of this class after its padding
          const bool straddle = nv > 0 && (offs[q] & 63) + nv > 64;
          const uint64_t mask = __ballot(straddle);
          if (!mask) {
            pos += read_lane(incl, 63);
            break;
          }
          if (lane == (int)__builtin_ctzll(mask)) pad += 64 - (offs[q] & 63);
        }
      }
      if (pos <= RMAX * NT || C >= mx) break;
      C = min((mx + 3) & ~3, (C + C / 2 + 3) & ~3);
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) sm.off[q * 64 + lane] = offs[q];
    if (lane == 0) {
      sm.off[BINS] = pos;
      sm.nc = nc;
      sm.C = C;
      sm.CS = (C & 7) == 4 ? C : C + 4;  // C = 4 mod 8: conflict-free 8-byte reads
      sm.R = max(1, (pos + NT - 1) / NT);
      const int64_t ncells = (int64_t)sm.R * NT * sm.CS;
      const int64_t cell_bytes = ncells * sizeof(cell_t);
      sm.use_list = cell_bytes <= (int64_t)sizeof(sm.spare) ? 1 : 0;
      sm.nAp = (nA + 3) & ~3;
      sm.nBp = (nB + 3) & ~3;
      const int64_t tab_bytes = (int64_t)nA * sm.nBp + (int64_t)nB * sm.nAp + 16;
      sm.tab_lds = (sm.use_list && ((cell_bytes + 15) & ~15) + tab_bytes <= (int64_t)sizeof(sm.spare)) ? 1 : 0;
    }
  }
  __syncthreads();
  if (!sm.use_list) return;  // the solver sums the classes without a list
  const int C = sm.C, CS = sm.CS, R = sm.R;
  cell_t* cells = cell_store(sm);
  const cell_t zero_cell = (cell_t)(nA | (nB << SH));  // lc[nA] = rc[nB] = 0
  for (int m = t; m < BINS; m += NT) {
    const int c = sm.csz[m];
    for (int u = 0; u * C < c; ++u) sm.chunk_cls[sm.off[m] + u] = (int16_t)m;
  }
  __syncthreads();
  // zero cells: padding chunks, and the slots of a class's last chunk past
  // its cells (chunk u of class m holds the class's cells (u - off[m]) C ..)
  for (int u = t; u < R * NT; u += NT) {
    const int m = sm.chunk_cls[u];
    const int s0 = m >= 0 ? max(0, min(C, sm.csz[m] - (u - sm.off[m]) * C)) : 0;
    for (int s = s0; s < C; ++s) cells[(size_t)u * CS + s] = zero_cell;
  }
  // the cells, one lane per chunk (C cells each): the chunk's first cell has
  // rank (u - off[m]) C in its class; the class's lanes of the count above
  // (consecutive, c rows each from row q) hold the ranks of their first
  // cells, so a binary search names the lane and at most c rows are skipped
  // from its first row before the chunk's cells follow the rows' runs
  {
    const int c = cl.c;
    const int total = lanes_upto(nA, c);
    for (int r = 0; r < R; ++r) {
      const int u = r * NT + t;
      const int m = sm.chunk_cls[u];
      if (m < 0) continue;
      const int q = sm.PA[m];  // m is a level of A: its class index
      const int f = total - lanes_upto(nA - q, c), g = (nA - q + c - 1) / c;
      const int rank0 = (u - sm.off[m]) * C;
      int lo = 0, hi = g - 1;  // last lane whose first rank is <= rank0
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (sm.lane_cells[f + mid] <= rank0)
          lo = mid;
        else
          hi = mid - 1;
      }
      int skip = rank0 - sm.lane_cells[f + lo];
      int i = q + lo * c, jlo = 0, jhi = 0;
      for (;; ++i) {  // the row holding rank rank0 (it exists: rank0 < csz[m])
        class_run_upper<BINS>(sm, i, m, jlo, jhi);
        if (skip < jhi - jlo) break;
        skip -= jhi - jlo;
      }
      int j = jlo + skip;
      const int n = min(C, sm.csz[m] - rank0);
      for (int k = 0; k < n; ++k) {
        while (j == jhi) {  // next row with cells of class m
          ++i;
          class_run_upper<BINS>(sm, i, m, jlo, jhi);
          j = jlo;
        }
        cells[(size_t)u * CS + k] = (cell_t)(i | (j << SH));
        ++j;
      }
    }
  }
  if (sm.tab_lds) {
    // four classes per word; rows padded to nBp (nAp) bytes with class 0
    // (the zero padding of af and bq gives class 0).  A row has at most 64
    // words (nB, nA <= 256), so a wave covers 64 / words whole rows at a
    // time and each lane keeps one word position: no index division in the
    // loops, one FMA per class (class_of on a and b / (l-1), exact).
    uint32_t* tab = reinterpret_cast<uint32_t*>(class_table(sm));
    uint32_t* tabT = tab + (nA * sm.nBp >> 2);
    const int wave = t >> 6, lane = t & 63;
    {
      const int wr = sm.nBp >> 2, rpw = 64 / wr, sub = lane / wr, w = lane - sub * wr;
      if (sub < rpw) {
        const float4 v = *reinterpret_cast<const float4*>(&sm.bq[4 * w]);
        for (int i = wave * rpw + sub; i < nA; i += (NT / 64) * rpw) {
          const float a = sm.af[i];
          tab[i * wr + w] = class_of(a, v.x) | class_of(a, v.y) << 8 | class_of(a, v.z) << 16 | class_of(a, v.w) << 24;
        }
      }
    }
    {
      const int wc = sm.nAp >> 2, rpw = 64 / wc, sub = lane / wc, w = lane - sub * wc;
      if (sub < rpw) {
        const float4 u = *reinterpret_cast<const float4*>(&sm.af[4 * w]);
        for (int j = wave * rpw + sub; j < nB; j += (NT / 64) * rpw) {
          const float v = sm.bq[j];
          tabT[j * wc + w] = class_of(u.x, v) | class_of(u.y, v) << 8 | class_of(u.z, v) << 16 | class_of(u.w, v) << 24;
        }
      }
    }
  }
  __syncthreads();
}

// Reciprocal for the per-pass scalars of the solver (the rescalings of Eqs.
// (14)-(15), the denominators of Eqs. (12)-(13), rho = s / d): the hardware
// v_rcp_f32, within one ulp, one instruction instead of the ten of an IEEE
// division that every wave would otherwise repeat in every pass.
__device__ inline float rcp_approx(float x) { return __builtin_amdgcn_rcpf(x); }

// Dense (L, R) of a checkpoint into state[0..2 BINS): L' / sum L' and
// R' / sum R' (Eqs. 14, 15), the values the next pass works with (invL, invR:
// the reciprocal sums); level k of L at [k], of R at [BINS + k], 0 at
// unoccupied levels.
template <int BINS, int NT>
__device__ inline void write_state(const SolveCore<BINS, NT>& sm, float* state, float invL, float invR) {
  for (int k = threadIdx.x; k < BINS; k += NT) {
    state[k] = sm.sd[k] > 0.f ? sm.lraw[sm.PA[k]] * invL : 0.f;
    state[BINS + k] = sm.PB[k + 1] > sm.PB[k] ? sm.rn[sm.PB[k]] * invR : 0.f;
  }
}

// The Alg. 1 loop; returns the number of passes run.  LIST: class totals
// from the class list and sweeps over power-of-two lane groups per output
// (else class totals from running sums over row runs, four classes per lane,
// and sweeps with four outputs per lane over input slices); TAB: the class
// tables are in LDS (else the sweeps compute the classes).
//
// Stopping rule (Alg. 1): at most p.iters passes; with p.eps > 0 the loop
// also ends after a pass whose changes of the normalised L and R both have a
// squared norm of at most eps.  The normalisation of a pass is folded into
// the next pass's class sweep, which is where the new L and R meet the old
// ones: the changes of pass t are summed there, in pass t + 1, and the
// decision (the same bits in every lane) is taken after its barrier.
// Index of the running sums for the lower run bound x = (2m-1)(l-1)/2a + 1
// computed in FP32: truncated, and clamped to l where the sums are not padded
// past it (256 levels).
template <int BINS>
__device__ __forceinline__ uint32_t run_bound(float x) {
  if constexpr (BINS == 1024)
    return (uint32_t)x;
  else
    return min((uint32_t)x, (uint32_t)BINS);
}

template <int BINS, int NT, int BUDGET, bool LIST, bool TAB>
__device__ __forceinline__ int iterate(SolveSmem<BINS, NT, BUDGET>& sm, const SolveParams& p, float* ckpt) {
  using cell_t = typename CellT<BINS>::type;
  constexpr int SH = CellT<BINS>::SHIFT;
  constexpr uint32_t MASK = (1u << SH) - 1;
  constexpr int PAD = SolveCore<BINS, NT>::PAD;
  static_assert(BINS <= NT, "one lane per class at least");
  static_assert(SolveSmem<BINS, NT, BUDGET>::FREE >= 8 * NT, "lane partials of the class sweep");
  const int t = threadIdx.x, lane = t & 63;
  const int nA = sm.nA, nB = sm.nB, C = sm.C, CS = sm.CS, R = sm.R;
  const cell_t* cells = cell_store(sm);
  const uint8_t* tab = class_table(sm);
  const uint8_t* tabT = tab + nA * sm.nBp;
  const int nAp = sm.nAp, nBp = sm.nBp;
  // dense sweeps with a class list: output o split over G lanes (a power of
  // two); slice k covers L inputs (a multiple of 4), zero-padded past the end
  // lanes the two dense sweeps spread their outputs over; waves past them
  // skip the sweep and contribute zero partial sums
  constexpr int SWEEP_LANES = NT;
  const int Gc = nB <= SWEEP_LANES ? pow2_floor64(SWEEP_LANES / nB) : 1;
  const int Gr = nA <= SWEEP_LANES ? pow2_floor64(SWEEP_LANES / nA) : 1;
  // the first thread of this wave, as a scalar: the wave-level tests below
  // compile to scalar branches
  const int wave0 = __builtin_amdgcn_readfirstlane(t & ~63);
  const bool col_wave = wave0 < nB * Gc, row_wave = wave0 < nA * Gr;
  const int Lc = ((nA + Gc - 1) / Gc + 3) & ~3, Lr = ((nB + Gr - 1) / Gr + 3) & ~3;
  // without a class list the slice sums of sweep_part go to spare (4 NT floats)
  float* sweep_buf = reinterpret_cast<float*>(sm.spare);
  static_assert(LIST || sizeof(sm.spare) >= 4 * NT * sizeof(float), "spare holds the sweep slice sums");
  for (int q = t; q < BINS + PAD; q += NT) {
    if (q >= nA) sm.l2c[q] = 0.f;
    if (q >= nB) sm.wc[q] = 0.f;
    if (!TAB) {
      sm.af[q] = q < nA ? (float)sm.A[q] : 0.f;
      sm.bq[q] = q < nB ? (float)sm.B[q] / (float)(BINS - 1) : 0.f;
    }
  }
  for (int m = t; m < BINS + 4; m += NT) sm.rho[m] = 0.f;
  // the passes start from L' = L(0), R' = R(0) with unit sums (Eqs. 14, 15
  // are folded into the next pass's class sweep)
  for (int i = t; i <= nA; i += NT) sm.lraw[i] = i < nA ? sm.lc[i] : 0.f;
  for (int j = t; j <= nB; j += NT) sm.rn[j] = j < nB ? sm.rc[j] : 0.f;
  for (int w = t; w < NT / 64; w += NT) {
    sm.redf[1][w] = w == 0 ? 1.f : 0.f;
    sm.redf[2][w] = w == 0 ? 1.f : 0.f;
  }
  if (t == 0) {
    sm.lc[nA] = 0.f;
    sm.rc[nB] = 0.f;
  }
  // without a list: classes in groups of CK (see group_lanes)
  constexpr int CK = 4;
  ClassLanes cl{-1, 0, 1, 1};
  if constexpr (!LIST) cl = group_lanes<BINS, NT, CK>(sm, reinterpret_cast<int*>(sm.spare));
  // class list: per round, the first lane of this lane's class in the wave
  // (64: padding chunk) and the class this lane completes (-1: none)
  constexpr int RMAX = SolveCore<BINS, NT>::RMAX;
  int seg0r[RMAX], donecls[RMAX];
  const int nchunks = LIST ? sm.off[BINS] : 0;
#pragma unroll
  for (int r = 0; r < RMAX; ++r) {
    seg0r[r] = 64;
    donecls[r] = -1;
    if (LIST && r < R) {
      const int u = r * NT + t;
      const int cls = sm.chunk_cls[u];
      if (cls >= 0) {
        seg0r[r] = sm.off[cls] & 63;
        if ((u - sm.off[cls] + 1) * C >= sm.csz[cls]) donecls[r] = cls;
      }
    }
  }
  __syncthreads();

  const bool track = p.eps > 0.f;
  int passes = p.iters;
  for (int it = 0; it < p.iters; ++it) {
    // sums of the previous pass's L', R' (Eqs. 14, 15)
    const float2 sums = block_read2<NT>(sm.redf[2], sm.redf[1]);
    const float sumL = sums.x, sumR = sums.y, invL = rcp_approx(sumL), invR = rcp_approx(sumR);
    if (ckpt && p.ckpt_every > 0 && it % p.ckpt_every == 0)
      write_state<BINS, NT>(sm, ckpt + (size_t)(it / p.ckpt_every) * 2 * BINS, invL, invR);
    // Eqs. (6), (8), (11): class totals d_m and rho_m = s_m / d_m, from the
    // unnormalised L', R': d_m = (sum of L' R' over the class) / (sumL sumR)
    {
      const float sLR = sumL * sumR;
      if constexpr (LIST) {
        // one chunk per lane and round; a class is summed inside its wave
#pragma unroll
        for (int r = 0; r < RMAX; ++r) {
          if (r >= R || r * NT + wave0 >= nchunks) break;  // whole wave of padding
          const int u = r * NT + t;
          const cell_t* cp = cells + (size_t)u * CS;
          // four partial sums (cell position mod 4), fixed order; eight cells
          // at a time, all sixteen gathers issued before the first product
          float a4[4] = {0.f, 0.f, 0.f, 0.f};
          int k = 0;
          for (; k + 8 <= C; k += 8) {
            uint32_t e[8];
            cells_of<cell_t>(cp + k, e);
            cells_of<cell_t>(cp + k + 4, e + 4);
            float lv[8], rv[8];
#pragma unroll
            for (int x = 0; x < 8; ++x) {
              lv[x] = sm.lraw[e[x] & MASK];
              rv[x] = sm.rn[e[x] >> SH];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int x = 0; x < 8; ++x) a4[x & 3] = fmaf(lv[x], rv[x], a4[x & 3]);
          }
          if (k < C) {  // C is a multiple of 4
            uint32_t e[4];
            cells_of<cell_t>(cp + k, e);
            float lv[4], rv[4];
#pragma unroll
            for (int x = 0; x < 4; ++x) {
              lv[x] = sm.lraw[e[x] & MASK];
              rv[x] = sm.rn[e[x] >> SH];
            }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int x = 0; x < 4; ++x) a4[x] = fmaf(lv[x], rv[x], a4[x]);
          }
          float acc = (a4[0] + a4[1]) + (a4[2] + a4[3]);
          const int seg0 = seg0r[r];  // lane of the class's first chunk
          {  // inclusive segmented scan over the class's lanes
            float y;
            y = dpp_get<dpp::ROW_SHR + 1, 0xf>(acc);
            if (lane - 1 >= seg0) acc += y;
            y = dpp_get<dpp::ROW_SHR + 2, 0xf>(acc);
            if (lane - 2 >= seg0) acc += y;
            y = dpp_get<dpp::ROW_SHR + 4, 0xf>(acc);
            if (lane - 4 >= seg0) acc += y;
            y = dpp_get<dpp::ROW_SHR + 8, 0xf>(acc);
            if (lane - 8 >= seg0) acc += y;
            y = dpp_get<dpp::BCAST15, 0xa>(acc);  // rows 1, 3 from lanes 15, 47
            if ((lane & ~15) - 1 >= seg0) acc += y;
            y = dpp_get<dpp::BCAST31, 0xc>(acc);  // rows 2, 3 from lane 31
            if (31 >= seg0) acc += y;
          }
          if (donecls[r] >= 0) sm.rho[donecls[r]] = acc > 0.f ? sm.sd[donecls[r]] * sLR * rcp_approx(acc) : 0.f;
        }
      } else {
        // rows of A, each contributing a run of B, summed as a difference of
        // FP64 running sums of R (O(1) per run); only the classes of occupied
        // levels (s_m > 0, i.e. m in A) are needed.  Lanes as in cl: the
        // rows of a class are dealt round-robin over its lanes.  The running
        // sums are indexed by level (rcum[b] = sum of R over the levels of B
        // below b), so a run's level bounds address them directly.
        for (int b = t; b <= BINS; b += NT) {
          double v = 0.0;
          if (b < BINS) {
            const int j = sm.PB[b];
            if (sm.PB[b + 1] > j) v = (double)sm.rn[j];
          }
          sm.rcum[b] = v;
        }
        __syncthreads();
        block_scan<NT, double>(sm.rcum, BINS + 1, sm.redd);
        if constexpr (BINS == 1024) {
          constexpr int RCUM = SolveCore<BINS, NT>::RCUM;
          for (int b = BINS + 1 + t; b < RCUM; b += NT) sm.rcum[b] = sm.rcum[BINS];
          __syncthreads();
        }
        // A lane takes CK consecutive classes m0 .. m0 + CK - 1 on its rows:
        // on row a the runs of the classes are [E(m), E(m + 1)) with
        // E(m) = floor((2m - 1)(l-1) / 2a) + 1 (capped at l, E(0) = 0), the
        // lower bound of class_run_upper (one FMA and a truncation), so CK + 1
        // bounds and running-sum
        // reads give the CK runs.  Classes above a get E = l on both ends, an
        // exact zero.  Two rows per step, each stage's LDS reads issued
        // together.
        double acc[CK];
#pragma unroll
        for (int w = 0; w < CK; ++w) acc[w] = 0.0;
        if (cl.q >= 0) {
          constexpr uint32_t D = BINS - 1;
          const int m0 = CK * cl.q, g = cl.g;
          float num[CK + 1];  // (2m - 1)(l-1), exact in FP32
#pragma unroll
          for (int w = 0; w <= CK; ++w) num[w] = (float)((2 * (m0 + w) - 1) * (int)D);
          int i = sm.PA[m0] + cl.k;
          if (i < nA && sm.A[i] == 0) {  // a = 0 (group 0): the whole row is class 0
            acc[0] = (double)sm.lraw[i] * (sm.rcum[BINS] - sm.rcum[0]);
            i += g;
          }
          for (; i + g < nA; i += 2 * g) {
            float inv[2], lv[2];
#pragma unroll
            for (int x = 0; x < 2; ++x) {
              inv[x] = sm.inv2a[i + x * g];
              lv[x] = sm.lraw[i + x * g];
            }
            __builtin_amdgcn_sched_barrier(0);
            double r[2][CK + 1];
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
              for (int w = 0; w <= CK; ++w) {
                const uint32_t e = (m0 + w) ? run_bound<BINS>(fmaf(num[w], inv[x], 1.f)) : 0u;
                r[x][w] = sm.rcum[e];
              }
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int x = 0; x < 2; ++x) {
              const double l = (double)lv[x];
#pragma unroll
              for (int w = 0; w < CK; ++w) acc[w] = fma(l, r[x][w + 1] - r[x][w], acc[w]);
            }
          }
          if (i < nA) {
            const float inv = sm.inv2a[i];
            const double l = (double)sm.lraw[i];
            double r[CK + 1];
#pragma unroll
            for (int w = 0; w <= CK; ++w) {
              const uint32_t e = (m0 + w) ? run_bound<BINS>(fmaf(num[w], inv, 1.f)) : 0u;
              r[w] = sm.rcum[e];
            }
#pragma unroll
            for (int w = 0; w < CK; ++w) acc[w] = fma(l, r[w + 1] - r[w], acc[w]);
          }
        }
        // The group's lanes [f, f + g) add up: a segmented scan inside each
        // wave the group spans gives one piece per wave, kept at index
        // q + (wave of the lane) (unique: groups are consecutive); the
        // group's first lane adds its pieces in wave order.
        double* piece = reinterpret_cast<double*>(sm.spare);  // [P + NT / 64][CK]
        static_assert(LIST || sizeof(sm.spare) >= (BINS / CK + NT / 64) * CK * sizeof(double),
                      "spare holds the class pieces");
        {
          const int f = t - cl.k, wv = t >> 6;
          const int seg0 = cl.q >= 0 ? max(f - (t & ~63), 0) : lane;
#pragma unroll
          for (int w = 0; w < CK; ++w) {
            double x = acc[w], y;
            y = dpp_get<dpp::ROW_SHR + 1, 0xf>(x);
            if (lane - 1 >= seg0) x += y;
            y = dpp_get<dpp::ROW_SHR + 2, 0xf>(x);
            if (lane - 2 >= seg0) x += y;
            y = dpp_get<dpp::ROW_SHR + 4, 0xf>(x);
            if (lane - 4 >= seg0) x += y;
            y = dpp_get<dpp::ROW_SHR + 8, 0xf>(x);
            if (lane - 8 >= seg0) x += y;
            y = dpp_get<dpp::BCAST15, 0xa>(x);
            if ((lane & ~15) - 1 >= seg0) x += y;
            y = dpp_get<dpp::BCAST31, 0xc>(x);
            if (31 >= seg0) x += y;
            acc[w] = x;
          }
          if (cl.q >= 0 && (lane == 63 || cl.k == cl.g - 1)) {
#pragma unroll
            for (int w = 0; w < CK; ++w) piece[(cl.q + wv) * CK + w] = acc[w];
          }
          __syncthreads();
          if (cl.q >= 0 && cl.k == 0) {
            const int w0 = f >> 6, w1 = (f + cl.g - 1) >> 6;
            double d[CK];
#pragma unroll
            for (int w = 0; w < CK; ++w) d[w] = piece[(cl.q + w0) * CK + w];
            for (int v = w0 + 1; v <= w1; ++v)
#pragma unroll
              for (int w = 0; w < CK; ++w) d[w] += piece[(cl.q + v) * CK + w];
#pragma unroll
            for (int w = 0; w < CK; ++w) {
              const int m = CK * cl.q + w;
              if (m >= BINS || sm.PA[m + 1] == sm.PA[m]) continue;  // only the classes of A
              sm.rho[m] = d[w] > 0.0 ? sm.sd[m] * sLR * rcp_approx((float)d[w]) : 0.f;
            }
          }
        }
      }
      float ql = 0.f, dl = 0.f, dr = 0.f;
      for (int i = t; i < nA; i += NT) {
        const float l = sm.lraw[i] * invL;  // Eq. (15)
        const float e = l - sm.lc[i];       // change of L in the previous pass
        dl = fmaf(e, e, dl);
        sm.lc[i] = l;
        sm.l2c[i] = l * l;
        ql += l * l;
      }
      for (int j = t; j < nB; j += NT) {
        const float r = sm.rn[j] * invR;  // Eq. (14)
        const float e = r - sm.rc[j];
        dr = fmaf(e, e, dr);
        sm.rc[j] = r;
      }
      wave_partial<NT>(ql, sm.redf[0]);
      if (track) {
        wave_partial<NT>(dl, sm.redf[3]);
        wave_partial<NT>(dr, sm.redf[4]);
      }
    }
    __syncthreads();
    if (track && it > 0) {
      // stopping rule for the pass just completed (uniform over the block)
      const float2 ch = block_read2<NT>(sm.redf[3], sm.redf[4]);
      if (ch.x <= p.eps && ch.y <= p.eps) {
        passes = it;
        break;
      }
    }
    // Eq. (13): R'_b = (R_b sum_a L_a^2 rho_index(a,b) + beta G_b) / (sum L^2 + beta).
    // The sweeps keep R'' = (sum L^2 + beta) R' instead: the rescaling of
    // Eq. (15) removes the common factor, and Eq. (12) below takes it into
    // its prior term.
    {
      float sr = 0.f;
      if constexpr (!LIST) {
        sweep_part<NT>(nB, nA, sm.l2c, sm.af, sm.bq, sm.rho, sweep_buf);
        __syncthreads();
        for (int o = t; o < nB; o += NT) {
          const float r = sm.rc[o];
          const float rn = fmaf(r, sweep_total<NT>(o, nB, nA, sweep_buf), p.beta * sm.gc[o]);
          sm.rn[o] = rn;
          sm.wc[o] = rn * r;
          sr += rn;
        }
      } else {
        for (int base = 0; base < nB * Gc; base += NT) {
          if (base + wave0 >= nB * Gc) break;  // whole wave past the outputs
          const int q = base + t;
          const int o = min(q / Gc, nB - 1), k = q & (Gc - 1);
          const int s0 = k * Lc;  // a multiple of 4
          const float r = sm.rc[o], bg = p.beta * sm.gc[o];
          float acc = 0.f;
          if constexpr (TAB) {
            const uint32_t* trow = reinterpret_cast<const uint32_t*>(tabT + o * nAp);
            acc = table_dot(sm.l2c, trow, sm.rho, s0, s0 + Lc, nAp);
          } else {
            acc = class_dot(sm.l2c, sm.af, sm.bq[o], sm.rho, s0, s0 + Lc);
          }
          acc = group_sum_last(acc, Gc);
          if (k == Gc - 1 && q / Gc < nB) {
            const float rn = fmaf(r, acc, bg);
            sm.rn[o] = rn;
            sm.wc[o] = rn * r;
            sr += rn;
          }
        }
      }
      if (!LIST || col_wave)
        wave_partial<NT>(sr, sm.redf[1]);
      else if (lane == 63)
        sm.redf[1][t >> 6] = 0.f;
    }
    __syncthreads();
    // Eq. (12): L'_a = (L_a sum_b R'_b R_b rho_index(a,b) + alpha S_a) / (sum R'^2 + alpha).
    // With R' = R'' / Dr (Dr = sum L^2 + beta), L' is proportional to
    // L_a sum_b R''_b R_b rho + alpha Dr S_a with a factor common to every
    // level, which the rescaling of Eq. (14) removes: that is what is kept.
    {
      const float aD = p.alpha * (block_read<NT>(sm.redf[0]) + p.beta);
      float sl = 0.f;
      if constexpr (!LIST) {
        sweep_part<NT>(nA, nB, sm.wc, sm.bq, sm.af, sm.rho, sweep_buf);
        __syncthreads();
        for (int o = t; o < nA; o += NT) {
          const float ln = fmaf(sm.lc[o], sweep_total<NT>(o, nA, nB, sweep_buf), aD * sm.sc[o]);
          sm.lraw[o] = ln;
          sl += ln;
        }
      } else {
        for (int base = 0; base < nA * Gr; base += NT) {
          if (base + wave0 >= nA * Gr) break;  // whole wave past the outputs
          const int q = base + t;
          const int o = min(q / Gr, nA - 1), k = q & (Gr - 1);
          const int s0 = k * Lr;
          const float lo = sm.lc[o], as = aD * sm.sc[o];
          float acc = 0.f;
          if constexpr (TAB) {
            const uint32_t* trow = reinterpret_cast<const uint32_t*>(tab + o * nBp);
            acc = table_dot(sm.wc, trow, sm.rho, s0, s0 + Lr, nBp);
          } else {
            acc = class_dot(sm.wc, sm.bq, sm.af[o], sm.rho, s0, s0 + Lr);
          }
          acc = group_sum_last(acc, Gr);
          if (k == Gr - 1 && q / Gr < nA) {
            const float ln = fmaf(lo, acc, as);
            sm.lraw[o] = ln;
            sl += ln;
          }
        }
      }
      if (!LIST || row_wave)
        wave_partial<NT>(sl, sm.redf[2]);
      else if (lane == 63)
        sm.redf[2][t >> 6] = 0.f;
    }
    __syncthreads();
  }
  // Eqs. (15), (14) of the last pass
  {
    const float2 sums = block_read2<NT>(sm.redf[2], sm.redf[1]);
    const float invL = 1.f / sums.x, invR = 1.f / sums.y;
    if (ckpt && p.ckpt_every > 0 && p.iters % p.ckpt_every == 0)
      write_state<BINS, NT>(sm, ckpt + (size_t)(p.iters / p.ckpt_every) * 2 * BINS, invL, invR);
    for (int i = t; i < nA; i += NT) sm.lc[i] = sm.lraw[i] * invL;
    for (int j = t; j < nB; j += NT) sm.rc[j] = sm.rn[j] * invR;
  }
  __syncthreads();
  return passes;
}

// LDS budget of the one-image solver: most of a CU's 160 KB.
constexpr int SOLVE_BUDGET_PLAIN = 150 * 1024;
// solver scratch per image in global memory (32-bit words), as allocated by
// the workspace: 3 * l^2
constexpr int NT_SOLVE = 1024;  // solver workgroup (one-image and batched kernels alike)

// Setup of the solve (Alg. 1 initialisation): masses, the occupied levels A
// of s and B of g (compacted, with their prefix counts PA, PB), s and g in
// probability units, L = s and R = g.  Returns N = sum of hS.  npix < 0 skips
// the check of the mass against npix (the gradient histogram is still
// checked against hS).
template <int BINS, int NT>
__device__ uint64_t solve_setup(const uint32_t* hS, const uint32_t* hG, int64_t npix, SolveCore<BINS, NT>& sm,
                                uint32_t* flags) {
  const int t = threadIdx.x;
  uint64_t ms = 0, mg = 0;
  for (int k = t; k < BINS; k += NT) {
    ms += hS[k];
    mg += hG[k];
  }
  const uint64_t Ns = block_sum<NT>(ms, sm.redu);
  const uint64_t Ng = block_sum<NT>(mg, sm.redu);
  if (t == 0 && ((npix >= 0 && Ns != (uint64_t)npix) || Ng != Ns)) atomicOr(flags, FLAG_HIST_MASS);
  for (int k = t; k < BINS + 1; k += NT) sm.PA[k] = (k < BINS && hS[k]) ? 1 : 0;
  __syncthreads();
  const int nA = block_scan<NT, int32_t>(sm.PA, BINS + 1, sm.redi);
  const double invS = 1.0 / (double)Ns, invG = 1.0 / (double)Ng;
  for (int k = t; k < BINS; k += NT) {
    const float sv = (float)((double)hS[k] * invS);
    sm.sd[k] = sv;
    if (hS[k]) {
      const int i = sm.PA[k];
      sm.A[i] = (uint16_t)k;
      sm.sc[i] = sv;
    }
  }
  for (int k = t; k < BINS + 1; k += NT) sm.PB[k] = (k < BINS && hG[k]) ? 1 : 0;
  __syncthreads();
  const int nB = block_scan<NT, int32_t>(sm.PB, BINS + 1, sm.redi);
  for (int k = t; k < BINS; k += NT) {
    if (hG[k]) {
      const int j = sm.PB[k];
      sm.B[j] = (uint16_t)k;
      sm.gc[j] = (float)((double)hG[k] * invG);
    }
  }
  if (t == 0) {
    sm.nA = nA;
    sm.nB = nB;
  }
  __syncthreads();
  for (int i = t; i < nA; i += NT) {
    sm.inv2a[i] = sm.A[i] ? 1.f / (float)(2 * sm.A[i]) : 0.f;
    sm.lc[i] = sm.sc[i];  // L(0) = H_C(S)
  }
  for (int j = t; j < nB; j += NT) sm.rc[j] = sm.gc[j];  // R(0) = H_C(grad S)
  __syncthreads();
  return Ns;
}

// Alg. 1 (Eqs. 11-15) for at most p.iters passes and the target histogram of
// Eqs. (17)-(20).  hS/hG: image and gradient histograms (global).  Writes
// illum/refl/target (counts, dense over the l levels) and the
// number of passes run when non-null, and with ckpt non-null and
// p.ckpt_every > 0 the dense (L, R) of t = 0, every, 2 every, ... (2 l floats
// each, see write_state).
template <int BINS, int NT, int BUDGET, bool MAY_BE_EMPTY = true>
__device__ __forceinline__ void solve_image(const uint32_t* hS, const uint32_t* hG, int64_t npix, SolveParams p,
                            SolveSmem<BINS, NT, BUDGET>& sm, float* illum, float* refl, float* target, uint32_t* flags, float* ckpt = nullptr,
                            int32_t* passes_out = nullptr) {
  const int t = threadIdx.x;
  const uint64_t Ns = solve_setup<BINS, NT>(hS, hG, npix, sm, flags);
  const int nA = sm.nA, nB = sm.nB;
  // no mass at all (flagged by the setup; histograms of an image always have
  // mass, MAY_BE_EMPTY = false): zero outputs
  if (MAY_BE_EMPTY && (nA == 0 || nB == 0)) {
    for (int k = t; k < BINS; k += NT) {
      if (target) target[k] = 0.f;
      if (illum) illum[k] = 0.f;
      if (refl) refl[k] = 0.f;
    }
    if (ckpt && p.ckpt_every > 0)
      for (int64_t k = t; k < (int64_t)(p.iters / p.ckpt_every + 1) * 2 * BINS; k += NT) ckpt[k] = 0.f;
    if (passes_out && t == 0) *passes_out = 0;
    return;
  }
  int passes;
  if constexpr (BINS == 256) {
    build_class_list<BINS, NT, BUDGET>(sm);
    if (!sm.use_list)
      passes = iterate<BINS, NT, BUDGET, false, false>(sm, p, ckpt);
    else if (sm.tab_lds)
      passes = iterate<BINS, NT, BUDGET, true, true>(sm, p, ckpt);
    else
      passes = iterate<BINS, NT, BUDGET, true, false>(sm, p, ckpt);
  } else {
    if (t == 0) {
      sm.C = 0;
      sm.CS = 0;
      sm.R = 0;
      sm.nAp = (nA + 3) & ~3;
      sm.nBp = (nB + 3) & ~3;
    }
    __syncthreads();
    passes = iterate<BINS, NT, BUDGET, false, false>(sm, p, ckpt);
  }
  if (passes_out && t == 0) *passes_out = passes;

  // Eqs. (17)-(20): target_k = N * sum over cells with round(theta_a * b) = k
  // of L_a R_b.  Products of two floats are exact in FP64; they are summed in
  // 2^-62 fixed point, so the result does not depend on the order.
  unsigned long long* tacc = reinterpret_cast<unsigned long long*>(sm.spare);  // BINS x u64
  double* theta = reinterpret_cast<double*>(sm.spare) + BINS;                 // BINS doubles
  for (int k = t; k < BINS; k += NT) tacc[k] = 0ull;
  for (int i = t; i < nA; i += NT) {
    const int a = sm.A[i];
    theta[i] = a ? pow((double)a / (double)(BINS - 1), p.inv_gamma) : 0.0;  // Eq. (17)
  }
  __syncthreads();
  constexpr int JC = 8;  // columns per work item
  const int nJC = (nB + JC - 1) / JC;
  for (int q = t; q < nA * nJC; q += NT) {
    const int i = q / nJC, j0 = (q - (q / nJC) * nJC) * JC, j1 = min(j0 + JC, nB);
    const double th = theta[i];
    const double la = (double)sm.lc[i];
    int cur = -1;
    unsigned long long run = 0;
    for (int j = j0; j < j1; ++j) {
      const int k = (int)floor(th * (double)sm.B[j] + 0.5);  // Eq. (19)
      const unsigned long long qv = __double2ull_rn(la * (double)sm.rc[j] * 0x1p62);
      if (k != cur) {
        if (cur >= 0 && run) atomicAdd(&tacc[cur], run);
        cur = k;
        run = 0;
      }
      run += qv;
    }
    if (cur >= 0 && run) atomicAdd(&tacc[cur], run);
  }
  __syncthreads();
  const double Nd = (double)Ns;
  for (int k = t; k < BINS; k += NT) {
    if (target) target[k] = (float)(Nd * ((double)tacc[k] * 0x1p-62));
    if (illum) illum[k] = 0.f;
    if (refl) refl[k] = 0.f;
  }
  __syncthreads();
  for (int i = t; i < nA; i += NT)
    if (illum) illum[sm.A[i]] = (float)(Nd * (double)sm.lc[i]);
  for (int j = t; j < nB; j += NT)
    if (refl) refl[sm.B[j]] = (float)(Nd * (double)sm.rc[j]);
  __syncthreads();
}

}  // namespace hr
