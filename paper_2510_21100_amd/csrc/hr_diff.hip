// Differentiated form of the HistRetinex solve and matching (8-bit, 256
// levels).  Not part of the paper: the exact LUT is piecewise constant in the
// target histogram, so the gradient runs through a soft matching map m(v),
// the piecewise-linear inverse of the normalised target CDF through the knots
// (k + 1/2, F~(k)), evaluated at the mid-rank source CDF u(v); round(m(v)) is
// the exact LUT value.  The loss of an image is the mean over pixels and
// channels of (c m(V) / (V (l-1)) - t_c)^2 against a target image t.
//
//   k_solve_ckpt  Alg. 1 forward with the dense (L, R) every few passes
//   k_softmap     m(v) from H_C(S) and the target h~
//   k_softloss    one pixel pass: loss and G[v] = sum over pixels at level v
//                 of sum_c (out_c - t_c) * (c, or 1 for black pixels)
//   k_softgrad    dLoss/dm(v), then dLoss/dh~ through the inverse-CDF map
//   k_solve_vjp   dLoss/dh~ -> Eq. (20) adjoint -> reverse through the
//                 passes of Eqs. (11)-(15), recomputing each checkpoint
//                 segment -> dLoss/dalpha, dLoss/dbeta
//
// Fixed-point (2^-24 and 2^-32) integer atomics keep the pixel-pass sums
// independent of the order in which workgroups arrive.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "hr_device.hpp"
#include "hr_launch.hpp"

namespace hr {

constexpr int DIFF_BINS = 256;
constexpr int NT_VJP = 1024;  // reverse pass: outputs split over lane groups, classes over balanced lanes
constexpr int SEG_MAX = 16;   // largest checkpoint interval
constexpr double G_SCALE = 16777216.0;       // 2^24: fixed point of G[v]
constexpr double LOSS_SCALE = 4294967296.0;  // 2^32: fixed point of the squared errors

// Two block sums for the barriers of one: each value is summed exactly as
// block_sum sums it (wave sum, then the waves in order).
template <int NT, typename T, typename U>
__device__ inline void block_sum2(T& x, U& y, T* redx, U* redy) {
  x = wave_sum(x);
  y = wave_sum(y);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    redx[w] = x;
    redy[w] = y;
  }
  __syncthreads();
  T sx = redx[0];
  U sy = redy[0];
#pragma unroll
  for (int i = 1; i < NT / 64; ++i) {
    sx += redx[i];
    sy += redy[i];
  }
  x = sx;
  y = sy;
}

// ---------------------------------------------------------------------------
// forward with checkpoints: one workgroup per image
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(NT_SOLVE) void k_solve_ckpt(const uint32_t* hv, const uint32_t* hg, SolveParams p,
                                                          int ncp, float* ckpt, float* target, uint32_t* flags) {
  constexpr int BINS = DIFF_BINS;
  __shared__ SolveSmem<BINS, NT_SOLVE, SOLVE_BUDGET_PLAIN> sm;
  const int i = blockIdx.x;
  solve_image<BINS, NT_SOLVE, SOLVE_BUDGET_PLAIN>(
      hv + (size_t)i * BINS, hg + (size_t)i * BINS, -1, p, sm, nullptr, nullptr, target + (size_t)i * BINS, flags,
      ckpt + (size_t)i * ncp * 2 * BINS);
}

// ---------------------------------------------------------------------------
// soft matching map
// ---------------------------------------------------------------------------

struct SoftSmem {
  double F[DIFF_BINS];    // normalised target CDF
  double u[DIFF_BINS];    // mid-rank source CDF
  uint64_t cs[DIFF_BINS];
  double redd[DIFF_BINS / 64];
  uint64_t redu[DIFF_BINS / 64];
  double gF[DIFF_BINS];
  double dm[DIFF_BINS];
  double t1[DIFF_BINS], t2[DIFF_BINS];  // a level's terms of dLoss/dF~ at k - 1 and at k
  int kv[DIFF_BINS];                    // its branch k (-1: no terms)
  double suf[DIFF_BINS];                // suffix sums of dLoss/dF~
  double dot;                           // sum of dLoss/dF~(k) F~(k)
};

// CDFs of one image: F~(k) = C(k) / C(l-1) with C the running sum of the
// target, u(v) = (cS(v-1) + cS(v)) / (2N).  NT = DIFF_BINS threads.
__device__ double soft_cdfs(const uint32_t* hS, const float* target, SoftSmem& sm, uint64_t& N) {
  constexpr int BINS = DIFF_BINS;
  const int t = threadIdx.x;
  sm.F[t] = (double)target[t];
  sm.cs[t] = hS[t];
  __syncthreads();
  const double S = block_scan<BINS, double, true>(sm.F, BINS, sm.redd);
  N = block_scan<BINS, uint64_t, true>(sm.cs, BINS, sm.redu);
  sm.F[t] = t == BINS - 1 ? 1.0 : sm.F[t] / S;
  sm.u[t] = (double)(2 * sm.cs[t] - hS[t]) / (2.0 * (double)N);
  __syncthreads();
  return S;
}

// k = min{k : F~(k) >= u}; lo = F~(k-1) (0 for k = 0), hi = F~(k)
__device__ inline int soft_branch(const SoftSmem& sm, double u, double& lo, double& hi) {
  int a = 0, b = DIFF_BINS - 1;
  while (a < b) {
    const int mid = (a + b) >> 1;
    if (sm.F[mid] >= u) b = mid; else a = mid + 1;
  }
  lo = a > 0 ? sm.F[a - 1] : 0.0;
  hi = sm.F[a];
  return a;
}

__global__ __launch_bounds__(DIFF_BINS) void k_softmap(const uint32_t* hv, const float* target, float* m_out) {
  constexpr int BINS = DIFF_BINS;
  __shared__ SoftSmem sm;
  const int i = blockIdx.x, t = threadIdx.x;
  uint64_t N;
  soft_cdfs(hv + (size_t)i * BINS, target + (size_t)i * BINS, sm, N);
  double lo, hi;
  const int k = soft_branch(sm, sm.u[t], lo, hi);
  const double m = (double)k - 0.5 + (sm.u[t] - lo) / (hi - lo);
  m_out[(size_t)i * BINS + t] = (float)fmin(fmax(m, 0.0), (double)(BINS - 1));
}

// ---------------------------------------------------------------------------
// pixel pass: loss and the weighted level histogram G
// ---------------------------------------------------------------------------

// One pixel of the loss pass: its squared errors into sq (channels in order)
// and its G term, in 2^-24 units, into the lane's run of equal levels; a run
// goes to the level's LDS counter when the level changes (integer sums, so
// the totals do not depend on how the pixels are grouped).
template <typename TP>
__device__ __forceinline__ void soft_pixel(uint32_t c0, uint32_t c1, uint32_t c2, TP tp, const float* scale,
                                           float black, float& sq, int& cur, long long& run,
                                           unsigned long long* g_lds) {
  const uint32_t V = umax3(c0, c1, c2);
  const float s = scale[V];
  float gsum = 0.f;
  const uint32_t cc[3] = {c0, c1, c2};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float o = V ? (float)cc[c] * s : black;
    const float e = o - tp[c];
    sq = fmaf(e, e, sq);
    gsum = fmaf(e, V ? (float)cc[c] : 1.f, gsum);
  }
  const long long gq = __double2ll_rn((double)gsum * G_SCALE);
  if ((int)V != cur) {
    if (cur >= 0 && run) atomicAdd(&g_lds[cur], (unsigned long long)run);
    cur = (int)V;
    run = 0;
  }
  run += gq;
}

// One workgroup per (tile, image); desc[i].in is the image, desc[i].out the
// FP32 HWC target image (tight rows), acc[i] holds BINS int64 sums of G in
// 2^-24 units followed by the squared-error sum in 2^-32 units.  A lane takes
// PX consecutive pixels per step; on tight, 16-byte aligned images their 48
// bytes of RGB and 192 bytes of target come in as 16-byte loads, otherwise
// pixel by pixel through the row stride.
__global__ __launch_bounds__(NT_PIX) void k_softloss(const ImgDesc* desc, const float* m_tab, int64_t tile_px,
                                                     unsigned long long* acc) {
  constexpr int BINS = DIFF_BINS;
  constexpr int PX = 16;
  __shared__ float scale[BINS];
  __shared__ unsigned long long g_lds[BINS];
  __shared__ float red[NT_PIX / 64];
  const int i = blockIdx.y, t = threadIdx.x;
  const ImgDesc d = desc[i];
  const int64_t P0 = (int64_t)blockIdx.x * tile_px;
  if (P0 >= d.npix) return;  // uniform: this image has fewer tiles
  const int64_t P1 = min(P0 + tile_px, d.npix);
  const float* mt = m_tab + (size_t)i * BINS;
  for (int v = t; v < BINS; v += NT_PIX) {
    scale[v] = v ? mt[v] / (float)(v * (BINS - 1)) : 0.f;
    g_lds[v] = 0ull;
  }
  __syncthreads();
  const float black = mt[0] / (float)(BINS - 1);
  const gptr<const float> tg = to_global(reinterpret_cast<const float*>(d.out));
  // p below is a multiple of PX (tile_px is), so a full step of a tight
  // image starts 16-byte aligned in both arrays
  const bool vec = d.in_vec && (reinterpret_cast<uintptr_t>(d.out) & 15u) == 0;
  float sq = 0.f;
  int cur = -1;
  long long run = 0;
  for (int64_t p = P0 + (int64_t)t * PX; p < P1; p += (int64_t)NT_PIX * PX) {
    const int n = (int)min((int64_t)PX, P1 - p);
    if (vec && n == PX) {
      const gptr<const v4u> src = to_global(reinterpret_cast<const v4u*>(d.in + 3 * p));
      const gptr<const v4u> tsrc = to_global(reinterpret_cast<const v4u*>(d.out + 12 * p));
      uint32_t w[12];
      float tv[48];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const v4u a = src[q];
        w[4 * q] = a.x;
        w[4 * q + 1] = a.y;
        w[4 * q + 2] = a.z;
        w[4 * q + 3] = a.w;
      }
#pragma unroll
      for (int q = 0; q < 12; ++q) {
        const v4u b = tsrc[q];
        tv[4 * q] = __uint_as_float(b.x);
        tv[4 * q + 1] = __uint_as_float(b.y);
        tv[4 * q + 2] = __uint_as_float(b.z);
        tv[4 * q + 3] = __uint_as_float(b.w);
      }
#pragma unroll
      for (int k = 0; k < PX; ++k) {
        const uint32_t c0 = (w[(3 * k) >> 2] >> (8 * ((3 * k) & 3))) & 0xffu;
        const uint32_t c1 = (w[(3 * k + 1) >> 2] >> (8 * ((3 * k + 1) & 3))) & 0xffu;
        const uint32_t c2 = (w[(3 * k + 2) >> 2] >> (8 * ((3 * k + 2) & 3))) & 0xffu;
        soft_pixel(c0, c1, c2, tv + 3 * k, scale, black, sq, cur, run, g_lds);
      }
    } else {
      for (int k = 0; k < n; ++k) {
        const int64_t q = p + k;
        const int64_t y = q / d.W;
        const int x = (int)(q - y * d.W);
        const gptr<const uint8_t> px = to_global(d.in + y * d.in_stride) + 3 * x;
        soft_pixel(px[0], px[1], px[2], tg + 3 * q, scale, black, sq, cur, run, g_lds);
      }
    }
  }
  if (cur >= 0 && run) atomicAdd(&g_lds[cur], (unsigned long long)run);
  const float tot = block_sum<NT_PIX>(sq, red);
  __syncthreads();
  unsigned long long* out = acc + (size_t)i * (BINS + 1);
  for (int v = t; v < BINS; v += NT_PIX)
    if (g_lds[v]) atomicAdd(out + v, g_lds[v]);
  if (t == 0) atomicAdd(out + BINS, (unsigned long long)__double2ll_rn((double)tot * LOSS_SCALE));
}

// ---------------------------------------------------------------------------
// dLoss/dm(v) -> dLoss/dh~ (one workgroup per image)
// ---------------------------------------------------------------------------

// m(v) = k - 1/2 + (u - lo) / (hi - lo) with lo = F~(k-1), hi = F~(k):
//   dm/dlo = (u - hi) / (hi - lo)^2,  dm/dhi = -(u - lo) / (hi - lo)^2;
// F~(j) = C(j) / C(l-1):  dF~(j)/dh~_i = ([i <= j] - F~(j)) / C(l-1).
__global__ __launch_bounds__(DIFF_BINS) void k_softgrad(const uint32_t* hv, const float* target,
                                                        const unsigned long long* acc, double* loss,
                                                        float* dtarget) {
  constexpr int BINS = DIFF_BINS;
  __shared__ SoftSmem sm;
  const int i = blockIdx.x, t = threadIdx.x;
  const uint32_t* hS = hv + (size_t)i * BINS;
  uint64_t N;
  const double S = soft_cdfs(hS, target + (size_t)i * BINS, sm, N);
  const unsigned long long* a = acc + (size_t)i * (BINS + 1);
  const double inv3N = 1.0 / (3.0 * (double)N);
  {
    const double G = (double)(long long)a[t] / G_SCALE;
    double lo, hi;
    const int k = soft_branch(sm, sm.u[t], lo, hi);
    const double m = (double)k - 0.5 + (sm.u[t] - lo) / (hi - lo);
    const bool clamped = m < 0.0 || m > (double)(BINS - 1);
    const double dLdm = clamped ? 0.0 : 2.0 * G * inv3N / (double)(t ? t * (BINS - 1) : (BINS - 1));
    const double dm = hS[t] ? dLdm : 0.0;
    sm.dm[t] = dm;
    // this level's terms of dLoss/dF~(k - 1) and dLoss/dF~(k); levels of
    // zero weight add none
    int kt = -1;
    double t1 = 0.0, t2 = 0.0;
    if (dm != 0.0) {
      const double w = hi - lo;
      t1 = dm * (sm.u[t] - hi) / (w * w);
      t2 = dm * -(sm.u[t] - lo) / (w * w);
      kt = k;
    }
    sm.kv[t] = kt;
    sm.t1[t] = t1;
    sm.t2[t] = t2;
  }
  __syncthreads();
  {
    // dLoss/dF~(t): the terms that name level t, added in level order (a
    // level names t either as its k or as its k - 1), which is the order of
    // one sequential sweep over the levels: the sums do not depend on the
    // thread count
    double g = 0.0;
    for (int v0 = 0; v0 < BINS; v0 += 16) {
      int kvv[16];
#pragma unroll
      for (int u = 0; u < 16; ++u) kvv[u] = sm.kv[v0 + u];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        if (kvv[u] == t) g += sm.t2[v0 + u];
        else if (kvv[u] == t + 1) g += sm.t1[v0 + u];
      }
    }
    sm.gF[t] = g;
  }
  __syncthreads();
  // the normalisation F~ = C / C(l-1): the dot product and the suffix sums
  // are sequential (one thread, fixed order); the divisions are per level
  if (t == 0) {
    double dot = 0.0;
#pragma unroll 16
    for (int k = 0; k < BINS; ++k) dot += sm.gF[k] * sm.F[k];
    double suffix = 0.0;
#pragma unroll 16
    for (int k = BINS - 1; k >= 0; --k) {
      suffix += sm.gF[k];
      sm.suf[k] = suffix;
    }
    sm.dot = dot;
    loss[i] = (double)(long long)a[BINS] / LOSS_SCALE * inv3N;
  }
  __syncthreads();
  dtarget[(size_t)i * BINS + t] = (float)((sm.suf[t] - sm.dot) / S);
}

// ---------------------------------------------------------------------------
// reverse pass of the solve (one workgroup per image, one thread per level)
// ---------------------------------------------------------------------------

// The quantities of one forward pass that its reverse reads (the others, L^2,
// rho and R' R, follow from these and the pass's state by one operation).
struct PassRec {
  float dcl[DIFF_BINS], u[DIFF_BINS], rp[DIFF_BINS], v[DIFF_BINS], lp[DIFF_BINS];
  float Q, P, Sl, Sr;
};
// Passes of a checkpoint segment whose quantities are kept from its
// recomputation for its reverse (longer segments recompute them).
constexpr int KEEP_MAX = 10;

struct VjpSmem : SolveCore<DIFF_BINS, NT_VJP> {
  float segl[SEG_MAX][DIFF_BINS], segr[SEG_MAX][DIFF_BINS];  // states of the current segment (compacted)
  float lt[DIFF_BINS], rt[DIFF_BINS];                        // state of the pass being reversed
  float dcl[DIFF_BINS], rh[DIFF_BINS];                       // class totals and rho by class
  float u[DIFF_BINS], rp[DIFF_BINS], v[DIFF_BINS], lp[DIFF_BINS];            // u_b, R', v_a, L'
  float l2[DIFF_BINS], w[DIFF_BINS];                         // L^2, R' R
  float lb[DIFF_BINS], rb[DIFF_BINS];                        // adjoints of the state
  float lbp[DIFF_BINS], rbp[DIFF_BINS];                      // adjoints of L', R'
  float vb[DIFF_BINS], ub[DIFF_BINS];                        // adjoints of v, u
  float ta[DIFF_BINS], tb[DIFF_BINS];                        // gather results
  float rhb[DIFF_BINS];                              // adjoint of rho, then of d
  float gH[DIFF_BINS];                               // dLoss/dh~ (dense)
  double theta[DIFF_BINS];                           // Eq. (17) on A
  double qc1[DIFF_BINS + 1], qc2[DIFF_BINS + 1];     // running sums over B (class sums)
  double part[NT_VJP];                               // lane partials of the class sums
  float redv[NT_VJP / 64], redv2[NT_VJP / 64];
  double redd[NT_VJP / 64];
  float sc_Q, sc_P, sc_Sl, sc_Sr;
  PassRec rec[KEEP_MAX];  // passes 0 .. E-2 of the current segment
};

// out[o] = sum_k x[k] * tab[cls(o, k)] for o < nout, k < nin: G lanes per
// output (a power of two), lane k of the group taking a contiguous slice of
// the inputs, summed in fixed order (slice, then the group's DPP sum).
template <typename ClassFn>
__device__ inline void lane_gather(int nout, int nin, const float* x, const float* tab, float* out, ClassFn cls) {
  const int t = threadIdx.x;
  const int G = nout <= NT_VJP ? pow2_floor64(NT_VJP / max(nout, 1)) : 1;
  const int L = (nin + G - 1) / G;
  for (int base = 0; base < nout * G; base += NT_VJP) {
    if (base + (t & ~63) >= nout * G) break;  // whole wave past the outputs
    const int q = base + t;
    const int o = min(q / G, nout - 1), k = q & (G - 1);
    const int k0 = k * L, k1 = min(k0 + L, nin);
    float a4[4] = {0.f, 0.f, 0.f, 0.f};
    int kk = k0;
    // four inputs at a time, their reads issued together; input kk always
    // goes to partial sum (kk - k0) mod 4
    for (; kk + 4 <= k1; kk += 4) {
      float xv[4], tv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        xv[u] = x[kk + u];
        tv[u] = tab[cls(o, kk + u)];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) a4[u] = fmaf(xv[u], tv[u], a4[u]);
    }
    for (; kk < k1; ++kk) a4[(kk - k0) & 3] = fmaf(x[kk], tab[cls(o, kk)], a4[(kk - k0) & 3]);
    float acc = group_sum_last((a4[0] + a4[1]) + (a4[2] + a4[3]), G);
    if (k == G - 1 && q / G < nout) out[o] = acc;
  }
}

// out[j] = sum_i x[i] * tab[class(A_i, B_j)] for j < nB
template <typename ClassFn>
__device__ inline void col_gather(const VjpSmem& sm, const float* x, const float* tab, float* out, ClassFn cls) {
  lane_gather(sm.nB, sm.nA, x, tab, out, [&](int j, int i) { return cls(i, j); });
}

// out[i] = sum_j y[j] * tab[class(A_i, B_j)] for i < nA
template <typename ClassFn>
__device__ inline void row_gather(const VjpSmem& sm, const float* y, const float* tab, float* out, ClassFn cls) {
  lane_gather(sm.nA, sm.nB, y, tab, out, [&](int i, int j) { return cls(i, j); });
}

// Exclusive prefix sums, in FP64, of q1[0..n) followed by a zero (n + 1
// values) into dst, and of q2 into dst2 when given, in the association order
// of block_scan over NT threads with one value per thread (n + 1 <= NT):
// chunks of 64 values scanned by wave sums, each chunk offset by the totals
// of the chunks before it added in order.  Wave 0 does all of it, so no
// barrier is needed before the scan, one after.
template <int NT>
__device__ inline void scan_levels(const float* q1, const float* q2, int n, double* dst, double* dst2) {
  static_assert(DIFF_BINS + 1 <= NT, "one value per thread of the block form");
  const int t = threadIdx.x;
  const int m = n + 1;
  if (t < 64) {
    double base1 = 0.0, base2 = 0.0;
    for (int c = 0; c * 64 < m; ++c) {
      const int i = c * 64 + t;
      double l1 = 0.0, l2 = 0.0;
      if (i < m) {
        l1 += i < n ? (double)q1[i] : 0.0;
        if (q2) l2 += i < n ? (double)q2[i] : 0.0;
      }
      const double i1 = wave_scan(l1);
      const double i2 = q2 ? wave_scan(l2) : 0.0;
      if (i < m) {
        dst[i] = base1 + i1 - l1;
        if (q2) dst2[i] = base2 + i2 - l2;
      }
      base1 += read_lane(i1, 63);
      if (q2) base2 += read_lane(i2, 63);
    }
  }
  __syncthreads();
}

// out[m] = sum over the cells (i, j) of class m of p1[i] q1[j] + p2[i] q2[j]
// (the second term only with TWO); classes with s_m = 0 get 0.  Rows of a
// class contribute runs of B, summed as differences of FP64 running sums of
// q1, q2; the (class, row) pairs are spread over balanced lanes (class q
// takes rows q..nA-1) and each class adds its lanes' partials in order.
template <bool TWO>
__device__ inline void class_sums(VjpSmem& sm, const ClassLanes& cl, const float* p1, const float* q1,
                                  const float* p2, const float* q2, float* out) {
  const int t = threadIdx.x;
  const int nA = sm.nA, nB = sm.nB;
  for (int m = t; m < DIFF_BINS; m += NT_VJP) out[m] = 0.f;
  scan_levels<NT_VJP>(q1, TWO ? q2 : nullptr, nB, sm.qc1, sm.qc2);
  double acc = 0.0;
  if (cl.q >= 0) {
    const int m = sm.A[cl.q];
    for (int i = cl.q + cl.k; i < nA; i += cl.g) {
      int jlo, jhi;
      class_run_upper<DIFF_BINS>(sm, i, m, jlo, jhi);  // empty: jlo = jhi
      acc = fma((double)p1[i], sm.qc1[jhi] - sm.qc1[jlo], acc);
      if (TWO) acc = fma((double)p2[i], sm.qc2[jhi] - sm.qc2[jlo], acc);
    }
  }
  sm.part[t] = acc;
  __syncthreads();
  if (cl.q >= 0 && cl.k == 0) {
    // the class's lane partials in lane order, read eight at a time
    double d = 0.0;
    int x = 0;
    for (; x + 8 <= cl.g; x += 8) {
      double pv[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) pv[u] = sm.part[t + x + u];
#pragma unroll
      for (int u = 0; u < 8; ++u) d += pv[u];
    }
    for (; x < cl.g; ++x) d += sm.part[t + x];
    out[sm.A[cl.q]] = (float)d;
  }
  __syncthreads();
}

struct IdxClass {
  const VjpSmem& sm;
  // the FP32 form of index(a, b): the same class as the integer formula for
  // every pair of levels at 256 levels
  __device__ int operator()(int i, int j) const { return (int)class_of(sm.af[i], sm.bq[j]); }
};
struct Idx1Class {
  const VjpSmem& sm;
  __device__ int operator()(int i, int j) const {
    return (int)floor(sm.theta[i] * (double)sm.B[j] + 0.5);  // Eq. (19), as in the forward
  }
};

// The quantities of one pass from the state (lt, rt): d, rho (Eq. 11),
// u and R' (Eq. 13), v and L' (Eq. 12), and the sums Q, P, Sl, Sr.
__device__ void vjp_forward_pass(VjpSmem& sm, const ClassLanes& cl, const SolveParams& p) {
  const int t = threadIdx.x;
  const int nA = sm.nA, nB = sm.nB;
  class_sums<false>(sm, cl, sm.lt, sm.rt, nullptr, nullptr, sm.dcl);
  const float l2 = t < nA ? sm.lt[t] * sm.lt[t] : 0.f;
  if (t < nA) sm.l2[t] = l2;
  if (t < DIFF_BINS) sm.rh[t] = sm.dcl[t] > 0.f ? sm.sd[t] / sm.dcl[t] : 0.f;
  const float Q = block_sum<NT_VJP>(l2, sm.redv);  // synchronises
  col_gather(sm, sm.l2, sm.rh, sm.u, IdxClass{sm});
  __syncthreads();
  float rpv = 0.f;
  if (t < nB) {
    rpv = (sm.rt[t] * sm.u[t] + p.beta * sm.gc[t]) / (Q + p.beta);
    sm.rp[t] = rpv;
    sm.w[t] = rpv * sm.rt[t];
  }
  float Sr = rpv, P = rpv * rpv;
  block_sum2<NT_VJP>(Sr, P, sm.redv, sm.redv2);
  row_gather(sm, sm.w, sm.rh, sm.v, IdxClass{sm});
  __syncthreads();
  float lpv = 0.f;
  if (t < nA) {
    lpv = (sm.lt[t] * sm.v[t] + p.alpha * sm.sc[t]) / (P + p.alpha);
    sm.lp[t] = lpv;
  }
  const float Sl = block_sum<NT_VJP>(lpv, sm.redv);
  if (t == 0) {
    sm.sc_Q = Q;
    sm.sc_P = P;
    sm.sc_Sl = Sl;
    sm.sc_Sr = Sr;
  }
  __syncthreads();
}

__device__ void save_pass(VjpSmem& sm, PassRec& r) {
  const int t = threadIdx.x;
  if (t < DIFF_BINS) r.dcl[t] = sm.dcl[t];
  if (t < sm.nB) {
    r.u[t] = sm.u[t];
    r.rp[t] = sm.rp[t];
  }
  if (t < sm.nA) {
    r.v[t] = sm.v[t];
    r.lp[t] = sm.lp[t];
  }
  if (t == 0) {
    r.Q = sm.sc_Q;
    r.P = sm.sc_P;
    r.Sl = sm.sc_Sl;
    r.Sr = sm.sc_Sr;
  }
}

// What vjp_forward_pass leaves for the state (lt, rt), from its record: the
// derived arrays by the same operations as there.
__device__ void load_pass(VjpSmem& sm, const PassRec& r) {
  const int t = threadIdx.x;
  if (t < DIFF_BINS) {
    const float d = r.dcl[t];
    sm.dcl[t] = d;
    sm.rh[t] = d > 0.f ? sm.sd[t] / d : 0.f;
  }
  if (t < sm.nA) {
    sm.l2[t] = sm.lt[t] * sm.lt[t];
    sm.v[t] = r.v[t];
    sm.lp[t] = r.lp[t];
  }
  if (t < sm.nB) {
    const float rpv = r.rp[t];
    sm.u[t] = r.u[t];
    sm.rp[t] = rpv;
    sm.w[t] = rpv * sm.rt[t];
  }
  if (t == 0) {
    sm.sc_Q = r.Q;
    sm.sc_P = r.P;
    sm.sc_Sl = r.Sl;
    sm.sc_Sr = r.Sr;
  }
  __syncthreads();
}

// Reverse of one pass: (lb, rb) = adjoints of the normalised outputs on
// entry, of the pass's input state (lt, rt) on exit.  Adds the pass's
// contributions to dalpha, dbeta (every thread holds the same totals).
__device__ void vjp_backward_pass(VjpSmem& sm, const ClassLanes& cl, const SolveParams& p, double& dalpha,
                                  double& dbeta) {
  const int t = threadIdx.x;
  const int nA = sm.nA, nB = sm.nB;
  const float Q = sm.sc_Q, P = sm.sc_P, Sl = sm.sc_Sl, Sr = sm.sc_Sr;
  const float Dl = P + p.alpha, Dr = Q + p.beta;
  // Eqs. (14), (15): L+ = L'/Sl, R+ = R'/Sr
  float dotl = t < nA ? sm.lb[t] * sm.lp[t] / Sl : 0.f, dotr = t < nB ? sm.rb[t] * sm.rp[t] / Sr : 0.f;
  block_sum2<NT_VJP>(dotl, dotr, sm.redv, sm.redv2);
  float lbp = 0.f, rbp = 0.f;
  if (t < nA) lbp = (sm.lb[t] - dotl) / Sl;
  if (t < nB) rbp = (sm.rb[t] - dotr) / Sr;
  // Eq. (12): L' = (L v + alpha s) / (P + alpha)
  double da = t < nA ? (double)lbp * (double)(sm.sc[t] - sm.lp[t]) / Dl : 0.0;
  float Pb = t < nA ? lbp * sm.lp[t] / Dl : 0.f;
  block_sum2<NT_VJP>(da, Pb, sm.redd, sm.redv);
  Pb = -Pb;
  dalpha += da;
  if (t < nA) {
    sm.vb[t] = lbp * sm.lt[t] / Dl;
    sm.lb[t] = lbp * sm.v[t] / Dl;  // direct term; more below
  }
  if (t < nB) rbp += 2.f * Pb * sm.rp[t];
  __syncthreads();
  // v_a = sum_b R'_b R_b rho(a,b): y_b = sum_a vbar_a rho(a,b)
  col_gather(sm, sm.vb, sm.rh, sm.tb, IdxClass{sm});
  __syncthreads();
  if (t < nB) {
    rbp += sm.rt[t] * sm.tb[t];
    sm.rb[t] = sm.rp[t] * sm.tb[t];
    sm.rbp[t] = rbp;
  }
  // Eq. (13): R' = (R u + beta g) / (Q + beta)
  double db = t < nB ? (double)rbp * (double)(sm.gc[t] - sm.rp[t]) / Dr : 0.0;
  float Qb = t < nB ? rbp * sm.rp[t] / Dr : 0.f;
  block_sum2<NT_VJP>(db, Qb, sm.redd, sm.redv);
  Qb = -Qb;
  dbeta += db;
  if (t < nB) {
    sm.ub[t] = rbp * sm.rt[t] / Dr;
    sm.rb[t] += rbp * sm.u[t] / Dr;
  }
  if (t < nA) sm.lb[t] += 2.f * Qb * sm.lt[t];
  __syncthreads();
  // u_b = sum_a L_a^2 rho(a,b): z_a = sum_b ubar_b rho(a,b)
  row_gather(sm, sm.ub, sm.rh, sm.ta, IdxClass{sm});
  // rho-bar_m = sum over class m of vbar_a R'_b R_b + L_a^2 ubar_b
  class_sums<true>(sm, cl, sm.vb, sm.w, sm.l2, sm.ub, sm.rhb);
  if (t < nA) sm.lb[t] += 2.f * sm.lt[t] * sm.ta[t];
  // rho = s / d: d-bar = -rho-bar rho / d
  if (t < DIFF_BINS) sm.rhb[t] = sm.dcl[t] > 0.f ? -sm.rhb[t] * sm.rh[t] / sm.dcl[t] : 0.f;
  __syncthreads();
  // d_m = sum over class m of L_a R_b
  row_gather(sm, sm.rt, sm.rhb, sm.ta, IdxClass{sm});
  col_gather(sm, sm.lt, sm.rhb, sm.tb, IdxClass{sm});
  __syncthreads();
  if (t < nA) sm.lb[t] += sm.ta[t];
  if (t < nB) sm.rb[t] += sm.tb[t];
  __syncthreads();
}

// dtarget: dLoss/dh~ [n][256]; ckpt: dense (L, R) per checkpoint; writes
// dalpha[i], dbeta[i].
__global__ __launch_bounds__(NT_VJP) void k_solve_vjp(const uint32_t* hv, const uint32_t* hg, SolveParams p,
                                                      int ncp, const float* ckpt, const float* dtarget,
                                                      double* dalpha, double* dbeta, uint32_t* flags) {
  constexpr int BINS = DIFF_BINS;
  __shared__ VjpSmem sm;
  const int img = blockIdx.x, t = threadIdx.x;
  const uint64_t N = solve_setup<BINS, NT_VJP>(hv + (size_t)img * BINS, hg + (size_t)img * BINS, -1, sm, flags);
  const int nA = sm.nA, nB = sm.nB, E = p.ckpt_every;
  if (nA == 0 || nB == 0) {  // no mass (flagged by the setup): h~ is 0 and so is its gradient
    if (t == 0) {
      dalpha[img] = 0.0;
      dbeta[img] = 0.0;
    }
    return;
  }
  const float* ck = ckpt + (size_t)img * ncp * 2 * BINS;
  if (t < nA) {
    const int a = sm.A[t];
    sm.theta[t] = a ? pow((double)a / (double)(BINS - 1), p.inv_gamma) : 0.0;  // Eq. (17)
  }
  if (t < BINS) sm.gH[t] = dtarget[(size_t)img * BINS + t];
  if (t < BINS) {
    sm.af[t] = t < nA ? (float)sm.A[t] : 0.f;
    sm.bq[t] = t < nB ? (float)sm.B[t] / (float)(BINS - 1) : 0.f;
  }
  const ClassLanes cl = class_lanes<NT_VJP>(nA, t);
  // final state
  const float* last = ck + (size_t)(ncp - 1) * 2 * BINS;
  if (t < nA) sm.lt[t] = last[sm.A[t]];
  if (t < nB) sm.rt[t] = last[BINS + sm.B[t]];
  __syncthreads();
  // Eq. (20): h~_k = N sum over idx1(a,b) = k of L_a R_b
  row_gather(sm, sm.rt, sm.gH, sm.ta, Idx1Class{sm});
  col_gather(sm, sm.lt, sm.gH, sm.tb, Idx1Class{sm});
  __syncthreads();
  const float Nf = (float)N;
  if (t < nA) sm.lb[t] = Nf * sm.ta[t];
  if (t < nB) sm.rb[t] = Nf * sm.tb[t];
  __syncthreads();
  double da = 0.0, db = 0.0;
  const bool keep = E - 1 <= KEEP_MAX;
  for (int seg = ncp - 2; seg >= 0; --seg) {
    const float* c0 = ck + (size_t)seg * 2 * BINS;
    if (t < nA) sm.segl[0][t] = c0[sm.A[t]];
    if (t < nB) sm.segr[0][t] = c0[BINS + sm.B[t]];
    __syncthreads();
    // recompute the states of the segment
    for (int q = 1; q < E; ++q) {
      if (t < nA) sm.lt[t] = sm.segl[q - 1][t];
      if (t < nB) sm.rt[t] = sm.segr[q - 1][t];
      __syncthreads();
      vjp_forward_pass(sm, cl, p);
      if (keep) save_pass(sm, sm.rec[q - 1]);
      if (t < nA) sm.segl[q][t] = sm.lp[t] / sm.sc_Sl;
      if (t < nB) sm.segr[q][t] = sm.rp[t] / sm.sc_Sr;
      __syncthreads();
    }
    for (int q = E - 1; q >= 0; --q) {
      if (t < nA) sm.lt[t] = sm.segl[q][t];
      if (t < nB) sm.rt[t] = sm.segr[q][t];
      __syncthreads();
      if (keep && q < E - 1)
        load_pass(sm, sm.rec[q]);
      else
        vjp_forward_pass(sm, cl, p);
      vjp_backward_pass(sm, cl, p, da, db);
    }
  }
  if (t == 0) {
    dalpha[img] = da;
    dbeta[img] = db;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

namespace launch {

hipError_t solve_ckpt(int n, const uint32_t* hv, const uint32_t* hg, const SolveParams& p, int ncp, float* ckpt,
                      float* target, uint32_t* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_solve_ckpt, dim3(n), dim3(NT_SOLVE), 0, s, hv, hg, p, ncp, ckpt, target, flags);
  return hipGetLastError();
}

hipError_t softmatch(int n, const ImgDesc* desc, int64_t max_npix, const uint32_t* hv, const float* target,
                     float* m_tab, unsigned long long* acc, double* loss, float* dtarget, hipStream_t s) {
  hipLaunchKernelGGL(k_softmap, dim3(n), dim3(DIFF_BINS), 0, s, hv, target, m_tab);
  hipError_t e = fill_u32(reinterpret_cast<uint32_t*>(acc), (int64_t)n * (DIFF_BINS + 1) * 2, 0u, s);
  if (e != hipSuccess) return e;
  const int64_t tile_px = (int64_t)NT_PIX * 16 * 8;
  const int64_t tiles = (max_npix + tile_px - 1) / tile_px;
  hipLaunchKernelGGL(k_softloss, dim3((unsigned)tiles, n), dim3(NT_PIX), 0, s, desc, m_tab, tile_px, acc);
  hipLaunchKernelGGL(k_softgrad, dim3(n), dim3(DIFF_BINS), 0, s, hv, target, acc, loss, dtarget);
  return hipGetLastError();
}

hipError_t solve_vjp(int n, const uint32_t* hv, const uint32_t* hg, const SolveParams& p, int ncp, const float* ckpt,
                     const float* dtarget, double* dalpha, double* dbeta, uint32_t* flags, hipStream_t s) {
  hipLaunchKernelGGL(k_solve_vjp, dim3(n), dim3(NT_VJP), 0, s, hv, hg, p, ncp, ckpt, dtarget, dalpha, dbeta, flags);
  return hipGetLastError();
}

int diff_seg_max() { return SEG_MAX; }

}  // namespace launch
}  // namespace hr
