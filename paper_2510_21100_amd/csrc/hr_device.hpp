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
constexpr uint32_t FLAG_VALUE_CLAMPED = 1u;
constexpr uint32_t FLAG_HIST_MASS = 2u;

// Per bit depth: element type, levels, pixels per thread per step, V-ring
// entries (power of two) and copies of each LDS histogram (spreads
// same-level atomics over banks).
template <int BITS> struct Cfg;
template <> struct Cfg<8> {
  using pix_t = uint8_t;
  static constexpr int BINS = 256, PX = 16, RING = 32768, REP = 4;
};
template <> struct Cfg<10> {
  using pix_t = uint16_t;
  static constexpr int BINS = 1024, PX = 8, RING = 16384, REP = 1;
};

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------

__device__ inline uint32_t umax3(uint32_t a, uint32_t b, uint32_t c) {
  return max(max(a, b), c);
}

__device__ inline uint32_t absdiff(uint32_t a, uint32_t b) { return a > b ? a - b : b - a; }

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

template <typename T>
__device__ inline T wave_sum(T x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
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
  T inc = local;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    T y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
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

// Value channel of PX consecutive pixels p .. p+PX-1 (n of them valid).
// Vectorised: three 16-byte loads cover the 48 bytes of the chunk.
template <int BITS>
__device__ inline void load_values(const ImgDesc& d, int64_t p, int n, uint32_t (&v)[Cfg<BITS>::PX],
                                   uint32_t& clamped) {
  using pix_t = typename Cfg<BITS>::pix_t;
  constexpr int PX = Cfg<BITS>::PX;
  constexpr uint32_t TOP = (1u << BITS) - 1;
  if (d.in_vec && n == PX) {
    const uint4* src = reinterpret_cast<const uint4*>(d.in + p * 3 * (int64_t)sizeof(pix_t));
    const uint4 a = src[0], b = src[1], c = src[2];
    const uint32_t w[12] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w};
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
        const pix_t* px = reinterpret_cast<const pix_t*>(d.in + y * d.in_stride) + 3 * x;
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

template <int BITS>
struct HistSmem {
  static constexpr int BINS = Cfg<BITS>::BINS, REP = Cfg<BITS>::REP, RING = Cfg<BITS>::RING;
  using pix_t = typename Cfg<BITS>::pix_t;
  static constexpr int RING_BYTES = RING * (int)sizeof(pix_t);
  uint32_t hs[BINS * REP];
  uint32_t hg[(2 * BINS - 1) * REP];
  uint32_t ring[RING_BYTES / 4 + 16];  // + 64-byte mirror of the start: no wrap on reads
  uint32_t clamped;
};

// 16 bytes starting at an arbitrary byte offset of the ring.
__device__ inline uint4 ring_read16(const uint32_t* ring, uint32_t byteoff) {
  const uint32_t b = byteoff >> 2, sh = byteoff & 3;
  const uint32_t d0 = ring[b], d1 = ring[b + 1], d2 = ring[b + 2], d3 = ring[b + 3], d4 = ring[b + 4];
  uint4 r;
  r.x = __builtin_amdgcn_alignbyte(d1, d0, sh);
  r.y = __builtin_amdgcn_alignbyte(d2, d1, sh);
  r.z = __builtin_amdgcn_alignbyte(d3, d2, sh);
  r.w = __builtin_amdgcn_alignbyte(d4, d3, sh);
  return r;
}

template <int BITS, int NT>
__device__ void hist_tile(const ImgDesc& d, int64_t P0, int64_t P1, HistSmem<BITS>& sm,
                          uint32_t* __restrict__ g_hs, uint32_t* __restrict__ g_graw) {
  using pix_t = typename Cfg<BITS>::pix_t;
  constexpr int BINS = Cfg<BITS>::BINS, PX = Cfg<BITS>::PX, REP = Cfg<BITS>::REP;
  constexpr int RING = Cfg<BITS>::RING;
  constexpr int RING_BYTES = HistSmem<BITS>::RING_BYTES;
  constexpr int STEP = NT * PX;
  constexpr int ESZ = (int)sizeof(pix_t);
  const int t = threadIdx.x;
  const int rep = t & (REP - 1);
  const int64_t N = d.npix;
  const int W = d.W;
  const int64_t E = min(P1 + (int64_t)W, N);

  for (int i = t; i < BINS * REP; i += NT) sm.hs[i] = 0;
  for (int i = t; i < (2 * BINS - 1) * REP; i += NT) sm.hg[i] = 0;
  if (t == 0) sm.clamped = 0;
  __syncthreads();

  uint32_t clamped = 0;
  int64_t loaded = P0, done = P0;
  while (done < P1) {
    const int64_t dend = min(done + STEP, P1);
    const int64_t need = min(dend - 1 + W, N - 1) + 1;
    while (loaded < need) {
      const int64_t p = loaded + (int64_t)t * PX;
      const int n = (int)max((int64_t)0, min((int64_t)PX, E - p));
      if (n > 0) {
        uint32_t v[PX];
        load_values<BITS>(d, p, n, v, clamped);
        uint32_t packed[4] = {0, 0, 0, 0};
#pragma unroll
        for (int i = 0; i < PX; ++i) set_lane<pix_t>(packed, i, v[i]);
        const uint32_t boff = (uint32_t)(((p - P0) & (RING - 1)) * ESZ);
        uint4* dst = reinterpret_cast<uint4*>(reinterpret_cast<uint8_t*>(sm.ring) + boff);
        *dst = make_uint4(packed[0], packed[1], packed[2], packed[3]);
        if (boff < 64) {
          uint4* mir = reinterpret_cast<uint4*>(reinterpret_cast<uint8_t*>(sm.ring) + RING_BYTES + boff);
          *mir = make_uint4(packed[0], packed[1], packed[2], packed[3]);
        }
        const int nh = (int)max((int64_t)0, min((int64_t)n, P1 - p));
#pragma unroll
        for (int i = 0; i < PX; ++i)
          if (i < nh) atomicAdd(&sm.hs[v[i] * REP + rep], 1u);
      }
      loaded += STEP;
      __syncthreads();
    }
    // gradient of pixels [done, dend)
    const int64_t q = done + (int64_t)t * PX;
    const int n = (int)max((int64_t)0, min((int64_t)PX, dend - q));
    if (n > 0) {
      const uint32_t boff = (uint32_t)(((q - P0) & (RING - 1)) * ESZ);
      const uint4 own4 = *reinterpret_cast<const uint4*>(reinterpret_cast<const uint8_t*>(sm.ring) + boff);
      const uint32_t own[4] = {own4.x, own4.y, own4.z, own4.w};
      const uint32_t rboff = boff + PX * ESZ;  // <= RING_BYTES: mirror covers it
      const uint32_t right_last =
          ESZ == 1 ? (uint32_t)reinterpret_cast<const uint8_t*>(sm.ring)[rboff]
                   : (uint32_t)reinterpret_cast<const uint16_t*>(sm.ring)[rboff >> 1];
      const uint32_t dboff = (uint32_t)(((q + W - P0) & (RING - 1)) * ESZ);
      const uint4 dn4 = ring_read16(sm.ring, dboff);
      const uint32_t dn[4] = {dn4.x, dn4.y, dn4.z, dn4.w};
      int x = (int)(q % W);
#pragma unroll
      for (int i = 0; i < PX; ++i) {
        if (i < n) {
          const uint32_t v = lane_of<pix_t>(own, i);
          const uint32_t vr = (i + 1 < PX) ? lane_of<pix_t>(own, i + 1) : right_last;
          const uint32_t vd = lane_of<pix_t>(dn, i);
          uint32_t g = 0;
          if (x + 1 < W) g += absdiff(vr, v);
          if (q + i + W < N) g += absdiff(vd, v);
          atomicAdd(&sm.hg[g * REP + rep], 1u);
          if (++x == W) x = 0;
        }
      }
    }
    done = dend;
    __syncthreads();
  }
  if (clamped) atomicOr(&sm.clamped, 1u);
  __syncthreads();
  for (int k = t; k < BINS; k += NT) {
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < REP; ++r) s += sm.hs[k * REP + r];
    if (s) atomicAdd(&g_hs[k], s);
  }
  for (int k = t; k < 2 * BINS - 1; k += NT) {
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < REP; ++r) s += sm.hg[k * REP + r];
    if (s) atomicAdd(&g_graw[k], s);
  }
}

// Gradient histogram onto the l levels: raw level j -> round-half-up(j(l-1)/gmax).
// Reads raw counts with device-coherent loads (they were produced by atomics
// of other workgroups).  `tmp` is BINS words of LDS, `red` NT/64 words.
template <int BINS, int NT>
__device__ void rebin_gradient(const uint32_t* g_graw, uint32_t* g_hg, uint32_t* tmp, uint32_t* red) {
  const int t = threadIdx.x;
  uint32_t gm = 0;
  for (int j = t; j < 2 * BINS - 1; j += NT) {
    const uint32_t c = __hip_atomic_load(g_graw + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (c) gm = max(gm, (uint32_t)j);
  }
  for (int k = t; k < BINS; k += NT) tmp[k] = 0;
  const uint32_t gmax = block_max<NT>(gm, red);
  for (int j = t; j <= (int)gmax; j += NT) {
    const uint32_t c = __hip_atomic_load(g_graw + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (c) {
      const uint32_t q = gmax ? (uint32_t)((2ull * (BINS - 1) * j + gmax) / (2ull * gmax)) : 0u;
      atomicAdd(&tmp[q], c);
    }
  }
  __syncthreads();
  for (int k = t; k < BINS; k += NT) g_hg[k] = tmp[k];
}

// ---------------------------------------------------------------------------
// remap tile: out_c = round-half-up(c * LUT[V] / V), black -> LUT[0].
// The division by 2V is a multiply-high by M[V] = ceil(2^32 / (2V)), exact for
// every numerator 2cL + V < 2^32 / (2V - 1) (all 10-bit cases included).
// `tab[v]` = {M[v], LUT[v]} in LDS.
// ---------------------------------------------------------------------------

template <int BITS>
__device__ inline uint32_t remap_channel(uint32_t c, uint32_t v, uint2 e) {
  const uint32_t q = __umulhi(2u * c * e.y + v, e.x);
  return v ? q : e.y;
}

template <int BITS, int NT>
__device__ void remap_tile(const ImgDesc& d, int64_t P0, int64_t P1, const uint2* tab) {
  using pix_t = typename Cfg<BITS>::pix_t;
  constexpr int PX = Cfg<BITS>::PX;
  constexpr int STEP = NT * PX;
  constexpr uint32_t TOP = (1u << BITS) - 1;
  for (int64_t p = P0 + (int64_t)threadIdx.x * PX; p < P1; p += STEP) {
    const int n = (int)min((int64_t)PX, P1 - p);
    if (d.in_vec && d.out_vec && n == PX) {
      const v4u* src = reinterpret_cast<const v4u*>(d.in + p * 3 * (int64_t)sizeof(pix_t));
      const v4u a = __builtin_nontemporal_load(src), b = __builtin_nontemporal_load(src + 1),
                c = __builtin_nontemporal_load(src + 2);
      uint32_t w[12] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w, c.x, c.y, c.z, c.w};
#pragma unroll
      for (int i = 0; i < PX; ++i) {
        uint32_t r = lane_of<pix_t>(w, 3 * i), g = lane_of<pix_t>(w, 3 * i + 1),
                 bl = lane_of<pix_t>(w, 3 * i + 2);
        if (BITS > 8) {
          r = min(r, TOP);
          g = min(g, TOP);
          bl = min(bl, TOP);
        }
        const uint32_t v = umax3(r, g, bl);
        const uint2 e = tab[v];
        set_lane<pix_t>(w, 3 * i, remap_channel<BITS>(r, v, e));
        set_lane<pix_t>(w, 3 * i + 1, remap_channel<BITS>(g, v, e));
        set_lane<pix_t>(w, 3 * i + 2, remap_channel<BITS>(bl, v, e));
      }
      v4u* dst = reinterpret_cast<v4u*>(d.out + p * 3 * (int64_t)sizeof(pix_t));
      __builtin_nontemporal_store(v4u{w[0], w[1], w[2], w[3]}, dst);
      __builtin_nontemporal_store(v4u{w[4], w[5], w[6], w[7]}, dst + 1);
      __builtin_nontemporal_store(v4u{w[8], w[9], w[10], w[11]}, dst + 2);
    } else {
      int64_t y = p / d.W;
      int x = (int)(p - y * d.W);
      for (int i = 0; i < n; ++i) {
        const pix_t* s = reinterpret_cast<const pix_t*>(d.in + y * d.in_stride) + 3 * x;
        pix_t* o = reinterpret_cast<pix_t*>(d.out + y * d.out_stride) + 3 * x;
        uint32_t r = s[0], g = s[1], bl = s[2];
        if (BITS > 8) {
          r = min(r, TOP);
          g = min(g, TOP);
          bl = min(bl, TOP);
        }
        const uint32_t v = umax3(r, g, bl);
        const uint2 e = tab[v];
        o[0] = (pix_t)remap_channel<BITS>(r, v, e);
        o[1] = (pix_t)remap_channel<BITS>(g, v, e);
        o[2] = (pix_t)remap_channel<BITS>(bl, v, e);
        if (++x == d.W) {
          x = 0;
          ++y;
        }
      }
    }
  }
}

// Remap table {M[v], LUT[v]} from a LUT in global memory.
template <int BINS, int NT>
__device__ inline void load_remap_table(const uint16_t* lut, uint2* tab) {
  for (int v = threadIdx.x; v < BINS; v += NT) {
    const uint32_t m = v ? (uint32_t)((0xffffffffull + 2ull * v) / (2ull * v)) : 0u;  // ceil(2^32 / 2v)
    tab[v] = make_uint2(m, (uint32_t)lut[v]);
  }
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
// ---------------------------------------------------------------------------

template <int BINS, int NT>
struct SolveSmem {
  float s[BINS], g[BINS];     // image / gradient histograms, probability units
  float lv[BINS], rv[BINS];   // current illumination / reflectance histograms
  float rho[BINS];            // s_m / d_m per class
  float acc[BINS];            // output of a segmented sweep
  float rn[BINS];             // R' of Eq. (13) before rescaling
  union {
    struct {
      float l2[BINS];  // L_a^2, later L' of Eq. (12) before rescaling
      float w[BINS];   // R'_b R_b
    } it;
    unsigned long long tacc[BINS];  // fixed-point class sums of Eq. (20)
  } u;
  int32_t off[3][BINS + 1];   // segment offsets: rows, columns, classes
  uint16_t A[BINS], B[BINS];  // occupied levels of s and g, ascending
  float first_sum[NT], last_sum[NT];
  float redf[NT / 64];
  uint64_t redu[NT / 64];
  int32_t redi[NT / 64];
  int32_t nA, nB, nc;
  int32_t C[3];
};

// index(a, b) of Eq. (10): nearest level of a*b/(l-1)^2 on the grid k/(l-1),
// i.e. round(a*b/(l-1)); l-1 is odd so there are no ties.
template <int BINS>
__device__ inline int class_of(int a, int b) {
  constexpr int D = BINS - 1;
  return (2 * a * b + D) / (2 * D);
}

__device__ inline uint32_t pack_cell(int key, int x, int y) {
  return ((uint32_t)key << 20) | ((uint32_t)x << 10) | (uint32_t)y;
}

// position of the i-th entry of a list stored chunk-interleaved for
// coalesced reads: chunk t (entries [tC, tC+C)) is column t
template <int NT>
__device__ inline int list_pos(int i, int C) {
  return (i % C) * NT + i / C;
}

// out[k] = sum over list entries with key k of X[x] * Y[y], for every key
// (0 for empty segments).  Each thread sums one chunk of C consecutive
// entries; segments crossing chunk borders are completed from the chunk
// partials in chunk order.  Fixed association -> deterministic.
template <int BINS, int NT>
__device__ void seg_sweep(const uint32_t* __restrict__ list, int nc, int C, const int32_t* off,
                          const float* X, const float* Y, float* out, float* first_sum, float* last_sum) {
  const int t = threadIdx.x;
  const int i0 = t * C, i1 = min(i0 + C, nc);
  if (i0 < i1) {
    uint32_t e = list[(0) * NT + t];
    int cur = (int)(e >> 20);
    float acc = 0.f;
    bool first = true;
    for (int i = i0, s = 0;;) {
      acc = fmaf(X[(e >> 10) & 1023u], Y[e & 1023u], acc);
      ++i;
      ++s;
      int k = -1;
      if (i < i1) {
        e = list[s * NT + t];
        k = (int)(e >> 20);
      }
      if (k != cur) {
        const int o1 = off[cur], o2 = off[cur + 1];
        if (o1 >= i0 && o2 <= i1) {
          out[cur] = acc;
        } else {
          if (first) first_sum[t] = acc;
          if (k < 0) last_sum[t] = acc;
        }
        if (k < 0) break;
        cur = k;
        acc = 0.f;
        first = false;
      }
    }
  }
  __syncthreads();
  for (int k = t; k < BINS; k += NT) {
    const int o1 = off[k], o2 = off[k + 1];
    if (o1 == o2) {
      out[k] = 0.f;
      continue;
    }
    const int t1 = o1 / C, t2 = (o2 - 1) / C;
    if (t1 == t2) continue;
    float s = last_sum[t1];
    for (int u = t1 + 1; u < t2; ++u) s += first_sum[u];
    s += first_sum[t2];
    out[k] = s;
  }
  __syncthreads();
}

// Builds the three segment lists of the active cells (a in supp s, b in
// supp g, s[index(a,b)] > 0): by row a, by column b and by class m.
// Cells outside these sets contribute exact zeros to every sweep.
template <int BINS, int NT>
__device__ void build_lists(SolveSmem<BINS, NT>& sm, uint32_t* lists) {
  const int t = threadIdx.x;
  constexpr int MAXCH = 32;  // at most this many chunks per segment
  const int nA = sm.nA, nB = sm.nB;
  for (int k = t; k < 3 * (BINS + 1); k += NT) (&sm.off[0][0])[k] = 0;
  __syncthreads();
  for (int q = t; q < nA * nB; q += NT) {
    const int i = q / nB, j = q - (q / nB) * nB;
    const int a = sm.A[i], b = sm.B[j];
    const int m = class_of<BINS>(a, b);
    if (sm.s[m] > 0.f) {
      atomicAdd(&sm.off[0][a], 1);
      atomicAdd(&sm.off[1][b], 1);
      atomicAdd(&sm.off[2][m], 1);
    }
  }
  __syncthreads();
  int32_t mx[3];
  for (int r = 0; r < 3; ++r) {
    int m = 0;
    for (int k = t; k < BINS; k += NT) m = max(m, sm.off[r][k]);
    mx[r] = block_max<NT>(m, sm.redi);
  }
  int nc = 0;
  for (int r = 0; r < 3; ++r) nc = block_scan<NT, int32_t>(sm.off[r], BINS + 1, sm.redi);
  if (t == 0) {
    sm.nc = nc;
    for (int r = 0; r < 3; ++r) sm.C[r] = max(1, max((nc + NT - 1) / NT, (mx[r] + MAXCH - 1) / MAXCH));
  }
  __syncthreads();
  const int Cr = sm.C[0], Cc = sm.C[1], Cm = sm.C[2];
  uint32_t* Lr = lists;
  uint32_t* Lc = lists + BINS * BINS;
  uint32_t* Lm = lists + 2 * BINS * BINS;
  for (int i = t; i < nA; i += NT) {  // rows, b ascending
    const int a = sm.A[i];
    int pos = sm.off[0][a];
    for (int j = 0; j < nB; ++j) {
      const int b = sm.B[j];
      const int m = class_of<BINS>(a, b);
      if (sm.s[m] > 0.f) Lr[list_pos<NT>(pos++, Cr)] = pack_cell(a, b, m);
    }
  }
  for (int j = t; j < nB; j += NT) {  // columns, a ascending
    const int b = sm.B[j];
    int pos = sm.off[1][b];
    for (int i = 0; i < nA; ++i) {
      const int a = sm.A[i];
      const int m = class_of<BINS>(a, b);
      if (sm.s[m] > 0.f) Lc[list_pos<NT>(pos++, Cc)] = pack_cell(b, a, m);
    }
  }
  for (int m = t; m < BINS; m += NT) {  // classes, (a, b) ascending
    int pos = sm.off[2][m];
    if (sm.off[2][m + 1] == pos) continue;
    for (int i = 0; i < nA; ++i) {
      const int a = sm.A[i];
      if (a < m) continue;  // index(a, b) <= a
      // class is non-decreasing in b: find the run of class m in row a
      int lo = 0, hi = nB;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (class_of<BINS>(a, sm.B[mid]) >= m) hi = mid; else lo = mid + 1;
      }
      int j = lo;
      for (; j < nB && class_of<BINS>(a, sm.B[j]) == m; ++j) Lm[list_pos<NT>(pos++, Cm)] = pack_cell(m, a, sm.B[j]);
    }
  }
  __syncthreads();
}

// Alg. 1 (Eqs. 11-15) for p.iters passes and the target histogram of
// Eqs. (17)-(20).  hS/hG: image and gradient histograms (global); lists:
// 3*BINS*BINS words of global scratch.  Writes illum/refl/target (counts)
// if the pointers are non-null, and the target into `target_lds` (counts).
template <int BINS, int NT>
__device__ void solve_image(const uint32_t* hS, const uint32_t* hG, int64_t npix, SolveParams p,
                            SolveSmem<BINS, NT>& sm, uint32_t* lists, float* illum, float* refl,
                            float* target, float* target_lds, uint32_t* flags) {
  const int t = threadIdx.x;
  // histograms -> probability units; occupied levels
  uint64_t ms = 0, mg = 0;
  for (int k = t; k < BINS; k += NT) {
    ms += hS[k];
    mg += hG[k];
  }
  const uint64_t Ns = block_sum<NT>(ms, sm.redu);
  const uint64_t Ng = block_sum<NT>(mg, sm.redu);
  if (t == 0 && (Ns != (uint64_t)npix || Ng != Ns)) atomicOr(flags, FLAG_HIST_MASS);
  const double invS = 1.0 / (double)Ns, invG = 1.0 / (double)Ng;
  for (int k = t; k < BINS; k += NT) {
    const float sv = (float)((double)hS[k] * invS);
    const float gv = (float)((double)hG[k] * invG);
    sm.s[k] = sv;
    sm.g[k] = gv;
    sm.lv[k] = sv;  // L(0) = H_C(S)
    sm.rv[k] = gv;  // R(0) = H_C(grad S)
    sm.off[0][k] = sv > 0.f ? 1 : 0;
    sm.off[1][k] = gv > 0.f ? 1 : 0;
  }
  __syncthreads();
  const int nA = block_scan<NT, int32_t>(sm.off[0], BINS, sm.redi);
  const int nB = block_scan<NT, int32_t>(sm.off[1], BINS, sm.redi);
  for (int k = t; k < BINS; k += NT) {
    if (sm.s[k] > 0.f) sm.A[sm.off[0][k]] = (uint16_t)k;
    if (sm.g[k] > 0.f) sm.B[sm.off[1][k]] = (uint16_t)k;
  }
  if (t == 0) {
    sm.nA = nA;
    sm.nB = nB;
  }
  __syncthreads();
  build_lists<BINS, NT>(sm, lists);
  const int nc = sm.nc;
  const uint32_t* Lr = lists;
  const uint32_t* Lc = lists + BINS * BINS;
  const uint32_t* Lm = lists + 2 * BINS * BINS;

  for (int it = 0; it < p.iters; ++it) {
    // Eqs. (8), (11): class totals d_m and rho_m = s_m / d_m (K_ab s_index = L_a R_b rho)
    seg_sweep<BINS, NT>(Lm, nc, sm.C[2], sm.off[2], sm.lv, sm.rv, sm.acc, sm.first_sum, sm.last_sum);
    float ql = 0.f;
    for (int k = t; k < BINS; k += NT) {
      const float d = sm.acc[k];
      sm.rho[k] = (d > 0.f && sm.s[k] > 0.f) ? sm.s[k] / d : 0.f;
      const float l = sm.lv[k];
      sm.u.it.l2[k] = l * l;
      ql += l * l;
    }
    const float sumL2 = block_sum<NT>(ql, sm.redf);  // includes the barrier
    // Eq. (13): R'_b = (R_b sum_a L_a^2 rho_index(a,b) + beta G_b) / (sum L^2 + beta)
    seg_sweep<BINS, NT>(Lc, nc, sm.C[1], sm.off[1], sm.u.it.l2, sm.rho, sm.acc, sm.first_sum, sm.last_sum);
    const float denR = sumL2 + p.beta;
    float qr = 0.f;
    for (int k = t; k < BINS; k += NT) {
      const float r = sm.rv[k];
      const float rn = (r * sm.acc[k] + p.beta * sm.g[k]) / denR;
      sm.rn[k] = rn;
      sm.u.it.w[k] = rn * r;
      qr += rn * rn;
    }
    const float sumR2 = block_sum<NT>(qr, sm.redf);
    // Eq. (12): L'_a = (L_a sum_b R'_b R_b rho_index(a,b) + alpha S_a) / (sum R'^2 + alpha)
    seg_sweep<BINS, NT>(Lr, nc, sm.C[0], sm.off[0], sm.u.it.w, sm.rho, sm.acc, sm.first_sum, sm.last_sum);
    const float denL = sumR2 + p.alpha;
    float sl = 0.f, sr = 0.f;
    for (int k = t; k < BINS; k += NT) {
      const float ln = (sm.lv[k] * sm.acc[k] + p.alpha * sm.s[k]) / denL;
      sm.u.it.l2[k] = ln;
      sl += ln;
      sr += sm.rn[k];
    }
    const float sumL = block_sum<NT>(sl, sm.redf);
    const float sumR = block_sum<NT>(sr, sm.redf);
    // Eqs. (15), (14): rescale to unit mass
    for (int k = t; k < BINS; k += NT) {
      sm.lv[k] = sm.u.it.l2[k] / sumL;
      sm.rv[k] = sm.rn[k] / sumR;
    }
    __syncthreads();
  }

  // Eqs. (17)-(20): target_k = N * sum over cells with round(theta_a * b) = k
  // of L_a R_b.  Products of two floats are exact in FP64; they are summed in
  // 2^-62 fixed point, so the result does not depend on the order.
  for (int k = t; k < BINS; k += NT) sm.u.tacc[k] = 0ull;
  __syncthreads();
  for (int i = t; i < nA; i += NT) {
    const int a = sm.A[i];
    const double theta = a ? pow((double)a / (double)(BINS - 1), p.inv_gamma) : 0.0;
    const double la = (double)sm.lv[a];
    int cur = -1;
    unsigned long long run = 0;
    for (int j = 0; j < nB; ++j) {
      const int b = sm.B[j];
      const int k = (int)floor(theta * (double)b + 0.5);
      const unsigned long long q = __double2ull_rn(la * (double)sm.rv[b] * 0x1p62);
      if (k != cur) {
        if (cur >= 0 && run) atomicAdd(&sm.u.tacc[cur], run);
        cur = k;
        run = 0;
      }
      run += q;
    }
    if (cur >= 0 && run) atomicAdd(&sm.u.tacc[cur], run);
  }
  __syncthreads();
  const double Nd = (double)Ns;
  for (int k = t; k < BINS; k += NT) {
    const float tv = (float)(Nd * ((double)sm.u.tacc[k] * 0x1p-62));
    if (target_lds) target_lds[k] = tv;
    if (target) target[k] = tv;
    if (illum) illum[k] = (float)(Nd * (double)sm.lv[k]);
    if (refl) refl[k] = (float)(Nd * (double)sm.rv[k]);
  }
  __syncthreads();
}

}  // namespace hr
