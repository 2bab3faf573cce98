// Variant readings of passages the paper leaves open, behind the same C ABI
// as the main path.  These kernels are written for clarity over speed (the
// benchmarked path uses the readings the pipeline is built on):
//
//  * k_hist_variant: the value histogram (Eq. 3) and the gradient histogram
//    (Alg. 1 initialisation) with another gradient operator -- forward
//    differences with the rounded Euclidean magnitude, or the 3x3 Sobel
//    derivatives (|gx| + |gy|) / 4 rounded -- and the raw levels either
//    rescaled by their largest occupied level or clipped at l-1.  One thread
//    per pixel reads the neighbours' values straight from memory.
//  * k_solve_variant: Alg. 1 over all l levels (no compaction) with Eqs.
//    (12)-(13) either multiplying by K (the reading of the main path) or
//    dividing by K as printed, cells with K = 0 left out, and L(0) either the
//    image histogram or uniform.  One workgroup; every sum has a fixed order.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hr_device.hpp"
#include "hr_launch.hpp"

namespace hr {

// V at (x, y) with the coordinates clamped to the image (replicated border);
// 10-bit values above 1023 are clamped and flagged like on the main path.
template <int BITS>
__device__ inline int value_at(const ImgDesc& d, int x, int y, uint32_t& clamped) {
  using pix_t = typename Cfg<BITS>::pix_t;
  constexpr uint32_t TOP = (1u << BITS) - 1;
  x = min(max(x, 0), d.W - 1);
  y = min(max(y, 0), d.H - 1);
  const pix_t* p = reinterpret_cast<const pix_t*>(d.in + (int64_t)y * d.in_stride) + 3 * (int64_t)x;
  uint32_t m = umax3(p[0], p[1], p[2]);
  if (BITS > 8) {
    clamped |= m > TOP ? 1u : 0u;
    m = min(m, TOP);
  }
  return (int)m;
}

// round-half-up(sqrt(q)) for 0 <= q < 2^22, exactly: r = floor(sqrt(q))
// (the FP32 root corrected by one either way), plus one when q - r^2 > r.
__device__ inline int round_sqrt(int q) {
  int r = (int)sqrtf((float)q);
  if (r * r > q) --r;
  if ((r + 1) * (r + 1) <= q) ++r;
  return r + (q - r * r > r ? 1 : 0);
}

template <int BITS>
__device__ inline int gradient_at(const ImgDesc& d, int x, int y, uint32_t variant, uint32_t& clamped) {
  const int v = value_at<BITS>(d, x, y, clamped);
  if (variant & VARIANT_GRAD_SOBEL) {
    int n[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) n[i][j] = (i == 1 && j == 1) ? v : value_at<BITS>(d, x + j - 1, y + i - 1, clamped);
    const int gx = (n[0][2] + 2 * n[1][2] + n[2][2]) - (n[0][0] + 2 * n[1][0] + n[2][0]);
    const int gy = (n[2][0] + 2 * n[2][1] + n[2][2]) - (n[0][0] + 2 * n[0][1] + n[0][2]);
    return (abs(gx) + abs(gy) + 2) >> 2;
  }
  const int dx = x + 1 < d.W ? value_at<BITS>(d, x + 1, y, clamped) - v : 0;
  const int dy = y + 1 < d.H ? value_at<BITS>(d, x, y + 1, clamped) - v : 0;
  if (variant & VARIANT_GRAD_L2) return round_sqrt(dx * dx + dy * dy);
  return abs(dx) + abs(dy);
}

// Histograms of one image with a variant gradient: LDS histograms per
// workgroup merged with global atomics; the workgroup that merges last puts
// the raw levels onto the l levels (largest occupied level onto l-1, or
// clipped at l-1).
template <int BITS>
__global__ __launch_bounds__(256) void k_hist_variant(ImgDesc d, int64_t tile_px, uint32_t variant, uint32_t* hs,
                                                      uint32_t* graw, uint32_t* hg, uint32_t* ticket,
                                                      uint32_t* flags) {
  constexpr int BINS = Cfg<BITS>::BINS;
  __shared__ uint32_t lhs[BINS];
  __shared__ uint32_t lg[2 * BINS - 1];
  __shared__ uint32_t red[256 / 64];
  __shared__ uint32_t last;
  __shared__ uint32_t clamped_any;
  for (int k = threadIdx.x; k < 2 * BINS - 1; k += 256) {
    if (k < BINS) lhs[k] = 0;
    lg[k] = 0;
  }
  if (threadIdx.x == 0) clamped_any = 0;
  __syncthreads();
  uint32_t clamped = 0;
  const int64_t P0 = (int64_t)blockIdx.x * tile_px, P1 = min(P0 + tile_px, d.npix);
  for (int64_t p = P0 + threadIdx.x; p < P1; p += 256) {
    const int y = (int)(p / d.W), x = (int)(p - (int64_t)y * d.W);
    atomicAdd(&lhs[value_at<BITS>(d, x, y, clamped)], 1u);
    atomicAdd(&lg[gradient_at<BITS>(d, x, y, variant, clamped)], 1u);
  }
  if (clamped) atomicOr(&clamped_any, 1u);
  __syncthreads();
  for (int k = threadIdx.x; k < 2 * BINS - 1; k += 256) {
    if (k < BINS && lhs[k]) atomicAdd(&hs[k], lhs[k]);
    if (lg[k]) atomicAdd(&graw[k], lg[k]);
  }
  // every wave's merge atomics are performed before thread 0 releases
  drain_memory();
  __syncthreads();
  if (threadIdx.x == 0) {
    if (clamped_any) atomicOr(flags, FLAG_VALUE_CLAMPED);
    fence_release_agent();
    last = (atomicAdd(ticket, 1u) == gridDim.x - 1) ? 1u : 0u;
    if (last) fence_acquire_agent();
  }
  __syncthreads();
  if (!last) return;
  if (variant & VARIANT_GRAD_CLIP) {
    for (int k = threadIdx.x; k < BINS; k += 256) lhs[k] = 0;
    __syncthreads();
    for (int j = threadIdx.x; j < 2 * BINS - 1; j += 256) {
      const uint32_t c = __hip_atomic_load(to_global(graw) + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (c) atomicAdd(&lhs[min(j, BINS - 1)], c);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < BINS; k += 256) hg[k] = lhs[k];
  } else {
    rebin_gradient<BINS, 256>(graw, hg, lhs, red);
  }
  if (threadIdx.x == 0) *ticket = 0;  // ready for the next call
}

// LDS of the variant solver: dense vectors over all l levels.
template <int BINS, int NT>
struct VariantSmem {
  float s[BINS], g[BINS], l[BINS], r[BINS];
  float lraw[BINS], rraw[BINS];  // L', R' before the rescaling of Eqs. (14), (15)
  float x[BINS], rho[BINS];      // the column-sweep input, the class weights
  double rc[BINS + 1];           // running sums of R by level
  unsigned long long tacc[BINS];  // Eq. (20) sums in 2^-62 fixed point
  double theta[BINS];
  double redd[NT / 64];
  uint64_t redu[NT / 64];
  int32_t redi[NT / 64];
};

// Alg. 1 and Eqs. (17)-(20) with the variant bits of SolveParams::variant.
// Every lane owns at most one level (BINS <= NT); every sum runs over the
// levels in order, in FP64.
template <int BINS, int NT>
__global__ __launch_bounds__(NT) void k_solve_variant(const uint32_t* hS, const uint32_t* hG, int64_t npix,
                                                      SolveParams p, float* illum, float* refl, float* target,
                                                      int32_t* passes_out, uint32_t* flags) {
  static_assert(BINS <= NT, "one lane per level");
  constexpr uint32_t D = BINS - 1;
  __shared__ VariantSmem<BINS, NT> sm;
  const int t = threadIdx.x;
  const bool div = (p.variant & VARIANT_UPDATE_DIV) != 0;
  uint64_t ms = 0, mg = 0;
  if (t < BINS) {
    ms = hS[t];
    mg = hG[t];
  }
  const uint64_t Ns = block_sum<NT>(ms, sm.redu);
  const uint64_t Ng = block_sum<NT>(mg, sm.redu);
  if (t == 0 && ((npix >= 0 && Ns != (uint64_t)npix) || Ng != Ns)) atomicOr(flags, FLAG_HIST_MASS);
  if (Ns == 0 || Ng == 0) {
    if (t < BINS) {
      illum[t] = 0.f;
      refl[t] = 0.f;
      target[t] = 0.f;
    }
    if (passes_out && t == 0) *passes_out = 0;
    return;
  }
  if (t < BINS) {
    const float sv = (float)((double)hS[t] / (double)Ns), gv = (float)((double)hG[t] / (double)Ng);
    sm.s[t] = sv;
    sm.g[t] = gv;
    sm.l[t] = (p.variant & VARIANT_INIT_UNIFORM) ? 1.f / (float)BINS : sv;  // L(0)
    sm.r[t] = gv;                                                            // R(0)
  }
  __syncthreads();
  int passes = p.iters;
  for (int it = 0; it < p.iters; ++it) {
    // Eqs. (6), (8): class totals d_m = sum over a of L_a (sum of R over the
    // levels b of row a in class m); the run of class m on row a >= 1 is
    // (2m-1)(l-1) < 2ab < (2m+1)(l-1), exact integer bounds
    if (t <= BINS) sm.rc[t] = t < BINS ? (double)sm.r[t] : 0.0;
    __syncthreads();
    block_scan<NT, double>(sm.rc, BINS + 1, sm.redd);
    double dm = 0.0;
    if (t < BINS) {
      const uint32_t m = (uint32_t)t;
      if (m == 0) dm = (double)sm.l[0] * sm.rc[BINS];
      for (uint32_t a = 1; a < BINS; ++a) {
        const float la = sm.l[a];
        if (la == 0.f) continue;
        const uint32_t lo = m == 0 ? 0u : min((2u * m - 1u) * D / (2u * a) + 1u, (uint32_t)BINS);
        const uint32_t hi = min((2u * m + 1u) * D / (2u * a) + 1u, (uint32_t)BINS);
        if (hi > lo) dm = fma((double)la, sm.rc[hi] - sm.rc[lo], dm);
      }
      // Eq. (11): K_ab = L_a R_b / d_m; the sweeps take rho_m = s_m / d_m
      // (multiplying by K) or sigma_m = s_m d_m (dividing by K)
      sm.rho[t] = dm > 0.0 ? (float)(div ? (double)sm.s[t] * dm : (double)sm.s[t] / dm) : 0.f;
      const float la = sm.l[t];
      sm.x[t] = div ? (la > 0.f ? 1.f : 0.f) : la * la;
    }
    __syncthreads();
    // Eq. (13) for R, level b = t
    double qL = 0.0;
    for (int a = 0; a < BINS; ++a) qL = fma((double)sm.l[a], (double)sm.l[a], qL);
    if (t < BINS) {
      const uint32_t b = (uint32_t)t;
      double u = 0.0;
      for (uint32_t a = 0; a < BINS; ++a) {
        const float xa = sm.x[a];
        if (xa != 0.f) u = fma((double)xa, (double)sm.rho[(2u * a * b + D) / (2u * D)], u);
      }
      const float rb = sm.r[b];
      const double lead = div ? (rb > 0.f ? u / (double)rb : 0.0) : (double)rb * u;
      sm.rraw[b] = (float)((lead + (double)p.beta * (double)sm.g[b]) / (qL + (double)p.beta));
    }
    __syncthreads();
    // Eq. (12) for L, level a = t, with the new unnormalised R
    double qR = 0.0;
    for (int b = 0; b < BINS; ++b) qR = fma((double)sm.rraw[b], (double)sm.rraw[b], qR);
    if (t < BINS) {
      const uint32_t a = (uint32_t)t;
      double v = 0.0;
      for (uint32_t b = 0; b < BINS; ++b) {
        const float rb = sm.r[b];
        if (rb == 0.f) continue;
        const double y = div ? (double)sm.rraw[b] / (double)rb : (double)sm.rraw[b] * (double)rb;
        v = fma(y, (double)sm.rho[(2u * a * b + D) / (2u * D)], v);
      }
      const float la = sm.l[a];
      const double lead = div ? (la > 0.f ? v / (double)la : 0.0) : (double)la * v;
      sm.lraw[a] = (float)((lead + (double)p.alpha * (double)sm.s[a]) / (qR + (double)p.alpha));
    }
    __syncthreads();
    // Eqs. (15), (14) and the stopping rule of Alg. 1
    double sL = 0.0, sR = 0.0;
    for (int k = 0; k < BINS; ++k) {
      sL += (double)sm.lraw[k];
      sR += (double)sm.rraw[k];
    }
    float dl = 0.f, dr = 0.f;
    if (t < BINS) {
      const float ln = (float)((double)sm.lraw[t] / sL), rn = (float)((double)sm.rraw[t] / sR);
      dl = (ln - sm.l[t]) * (ln - sm.l[t]);
      dr = (rn - sm.r[t]) * (rn - sm.r[t]);
    }
    const float chL = block_sum<NT>(dl, reinterpret_cast<float*>(sm.redi));
    const float chR = block_sum<NT>(dr, reinterpret_cast<float*>(sm.redi));
    if (t < BINS) {
      sm.l[t] = (float)((double)sm.lraw[t] / sL);
      sm.r[t] = (float)((double)sm.rraw[t] / sR);
    }
    __syncthreads();
    if (p.eps > 0.f && it + 1 < p.iters && chL <= p.eps && chR <= p.eps) {
      passes = it + 1;
      break;
    }
  }
  if (passes_out && t == 0) *passes_out = passes;
  // Eqs. (17)-(20): target_k = N * sum over cells with round(theta_a b) = k
  // of L_a R_b, exact FP64 products summed in 2^-62 fixed point
  if (t < BINS) {
    sm.tacc[t] = 0ull;
    sm.theta[t] = t ? pow((double)t / (double)D, p.inv_gamma) : 0.0;
  }
  __syncthreads();
  if (t < BINS) {
    const double la = (double)sm.l[t], th = sm.theta[t];
    if (la > 0.0)
      for (int b = 0; b < BINS; ++b) {
        const float rb = sm.r[b];
        if (rb == 0.f) continue;
        const int k = (int)floor(th * (double)b + 0.5);
        atomicAdd(&sm.tacc[k], __double2ull_rn(la * (double)rb * 0x1p62));
      }
  }
  __syncthreads();
  if (t < BINS) {
    const double Nd = (double)Ns;
    target[t] = (float)(Nd * ((double)sm.tacc[t] * 0x1p-62));
    illum[t] = (float)(Nd * (double)sm.l[t]);
    refl[t] = (float)(Nd * (double)sm.r[t]);
  }
}

namespace launch {

hipError_t hist_variant(int bits, const ImgDesc& d, int64_t tile_px, uint32_t variant, uint32_t* hs, uint32_t* graw,
                        uint32_t* hg, uint32_t* ticket, uint32_t* flags, hipStream_t s) {
  const int64_t tiles = (d.npix + tile_px - 1) / tile_px;
  if (bits == 8)
    hipLaunchKernelGGL(k_hist_variant<8>, dim3((unsigned)tiles), dim3(256), 0, s, d, tile_px, variant, hs, graw, hg,
                       ticket, flags);
  else
    hipLaunchKernelGGL(k_hist_variant<10>, dim3((unsigned)tiles), dim3(256), 0, s, d, tile_px, variant, hs, graw, hg,
                       ticket, flags);
  return hipGetLastError();
}

hipError_t solve_variant(int bins, const uint32_t* hS, const uint32_t* hG, int64_t npix, const SolveParams& p,
                         float* illum, float* refl, float* target, int32_t* passes, uint32_t* flags, hipStream_t s) {
  if (bins == 256)
    hipLaunchKernelGGL((k_solve_variant<256, 256>), dim3(1), dim3(256), 0, s, hS, hG, npix, p, illum, refl, target,
                       passes, flags);
  else
    hipLaunchKernelGGL((k_solve_variant<1024, 1024>), dim3(1), dim3(1024), 0, s, hS, hG, npix, p, illum, refl,
                       target, passes, flags);
  return hipGetLastError();
}

}  // namespace launch
}  // namespace hr
