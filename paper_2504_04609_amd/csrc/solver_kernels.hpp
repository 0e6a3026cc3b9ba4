// Device side of the OTLM scaling loop (Algorithm 1): the GEMM epilogues that
// carry each elementwise update, plus set-up, convergence and output kernels.
//
// Internal layout: every per-spectrum array is [B, ld] row-major FP32 with the
// bin dimension padded to np (multiple of 16) and the dictionary dimension to
// kp (multiple of 16); padded entries are kept at exactly 0 so they never
// contribute to a product.  Notation follows the paper with u_1 -> v
// (target-side scaling) and u_2 -> u (source-side scaling).
#pragma once
#include <hip/hip_runtime.h>
#include "omega.hpp"

enum { FIT_BALANCED = 0, FIT_KL = 1, FIT_TV = 2, FIT_L2 = 3, FIT_L2_TV = 4, FIT_POISSON = 5 };
enum { PEN_NONE = 0, PEN_L1 = 1, PEN_L2SQ = 2, PEN_EN = 3 };

constexpr float OTLM_R_CLAMP = 1.0e30f;

// FP32 -> BF16 bits, round to nearest even (NaN stays NaN).
__device__ __forceinline__ unsigned short f32_to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

// Elementwise FP32 -> BF16 copy (start of a BF16 phase).
__global__ void convert_f32_to_bf16(const float* __restrict__ x, unsigned short* __restrict__ y, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    y[i] = f32_to_bf16(x[i]);
}

// K = exp(-C / eps) rounded to BF16, zero padded to [np, np] (transpose = 1: K^T).
__global__ void build_kernel_bf16(const double* __restrict__ C, int n, int np, double inv_eps, int transpose,
                                  unsigned short* __restrict__ K) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= np || i >= np) return;
  float v = 0.f;
  if (i < n && j < n) v = (float)exp(-(transpose ? C[(size_t)j * n + i] : C[(size_t)i * n + j]) * inv_eps);
  K[(size_t)i * np + j] = f32_to_bf16(v);
}

// ---------------------------------------------------------------------------
// s = K v epilogue (Algorithm 1, source update, first half).
// Stores s and r = log(s / a) with a = D w from the previous weight step
// (Table 2: Z's normalisation (D w')_i; bins with a = 0 carry no dictionary
// mass and contribute 0).  On check iterations it also accumulates the
// source-marginal violation sum_i |u_i s_i - a_i| and sum_i a_i, where u is the
// previous source scaling, so u o (K v) - D w measures how far the current plan
// is from Q1 = D w.
struct EpiSrc {
  static constexpr int NRED = 2;
  static constexpr bool RED_IS_MAX[2] = {false, false};
  float* S;
  float* R;
  const float* A;
  const float* U;
  float* part_num;
  float* part_den;
  int ld, n_valid, ntiles;
  bool do_red;
  __device__ __forceinline__ void elem(int m, int n, float s, float* red) const {
    const size_t o = (size_t)m * ld + n;
    if (n >= n_valid) {
      S[o] = 0.f;
      if (R) R[o] = 0.f;
      return;
    }
    const float a = A[o];
    S[o] = s;
    if (R) {
      float r = 0.f;
      if (a > 0.f) r = fminf(fmaxf(logf(s / a), -OTLM_R_CLAMP), OTLM_R_CLAMP);
      R[o] = r;
    }
    if (do_red) {
      red[0] += fabsf(U[o] * s - a);
      red[1] += a;
    }
  }
  __device__ __forceinline__ void row_partial(int m, int tile, const float* v) const {
    part_num[(size_t)m * ntiles + tile] = v[0];
    part_den[(size_t)m * ntiles + tile] = v[1];
  }
};

// ---------------------------------------------------------------------------
// Weight step epilogue: c = (R D)_j = sum_i D_ij log(s_i / a_i).
// Table 2 / Appendix A: nu_j = log w'_j + c_j / x_j and
//   none:        w_j = exp(nu_j)
//   l1:          w_j = exp(nu_j - alpha / (eps x_j))
//   squared l2:  w_j = omega(nu_j + log g_j) / g_j,              g_j = alpha / (eps x_j)
//   elastic net: w_j = omega(nu_j - alpha/(eps x_j) + log g_j) / g_j,  g_j = beta / (eps x_j)
// colc holds per column [1/x_j, shift_j, g_j, log g_j].  Frozen spectra keep
// their weights.
struct EpiWupd {
  static constexpr int NRED = 0;
  static constexpr bool RED_IS_MAX[2] = {false, false};
  float* W;
  const float4* colc;
  const int* done;
  const int* mm_until;  // when not null only rows with it <= mm_until[m] take the step
  int it;
  int ld, k_valid, pen;
  bool do_red;
  __device__ __forceinline__ void elem(int m, int j, float c, float*) const {
    const size_t o = (size_t)m * ld + j;
    if (j >= k_valid) {
      W[o] = 0.f;
      return;
    }
    const float wold = W[o];
    const float4 cc = colc[j];
    const float nu = logf(wold) + c * cc.x;
    float w;
    if (pen == PEN_NONE) {
      w = expf(nu);
    } else if (pen == PEN_L1) {
      w = expf(nu - cc.y);
    } else {  // PEN_L2SQ (shift 0) and PEN_EN share the Lambert-W form
      w = wright_omega<float>(nu - cc.y + cc.w) / cc.z;
    }
    if (!done[m] && (!mm_until || it <= mm_until[m])) W[o] = w;
  }
  __device__ __forceinline__ void row_partial(int, int, const float*) const {}
};

// ---------------------------------------------------------------------------
// a = D w epilogue, then u = a / s (Algorithm 1: u_2 <- X w / K u_1).
struct EpiUscale {
  static constexpr int NRED = 0;
  static constexpr bool RED_IS_MAX[2] = {false, false};
  float* A;
  float* U;
  const float* S;
  int ld, n_valid;
  bool do_red;
  unsigned short* Ubf;  // BF16 shadow of u for a BF16 product (null: none)
  __device__ __forceinline__ void elem(int m, int n, float a, float*) const {
    const size_t o = (size_t)m * ld + n;
    if (n >= n_valid) {
      A[o] = 0.f;
      U[o] = 0.f;
      if (Ubf) Ubf[o] = 0;
      return;
    }
    a = fmaxf(a, 0.f);
    A[o] = a;
    const float u = a > 0.f ? a / S[o] : 0.f;
    U[o] = u;
    if (Ubf) Ubf[o] = f32_to_bf16(u);
  }
  __device__ __forceinline__ void row_partial(int, int, const float*) const {}
};

// Plain store epilogue (a = D w at set-up).
struct EpiStore {
  static constexpr int NRED = 0;
  static constexpr bool RED_IS_MAX[2] = {false, false};
  float* C;
  int ld, n_valid;
  bool do_red;
  __device__ __forceinline__ void elem(int m, int n, float c, float*) const {
    C[(size_t)m * ld + n] = n < n_valid ? c : 0.f;
  }
  __device__ __forceinline__ void row_partial(int, int, const float*) const {}
};

// ---------------------------------------------------------------------------
// Target step (Table 1), for t = (K^T u)_j and data y_j, returns v_j = p_j / t_j.
struct ProxConsts {
  int fit;
  float kappa;        // KL: lam / (lam + eps)
  float lam_eps;      // lam / eps
  float lam2_eps;     // lam2 / eps
  float eps_lam;      // eps / lam
  float log_lam_eps;  // log(lam / eps)
};

__device__ __forceinline__ float target_scaling(const ProxConsts& pc, float t, float y) {
  if (!(t > 0.f)) return 1.f;  // no transported mass reaches this bin: leave v = 1
  const float lt = logf(t);
  switch (pc.fit) {
    case FIT_BALANCED:
      return y / t;
    case FIT_KL:  // p = t^{eps/(eps+lam)} y^{lam/(eps+lam)}  ->  v = (y / t)^{lam/(eps+lam)}
      return y > 0.f ? expf(pc.kappa * (logf(y) - lt)) : 0.f;
    case FIT_TV: {  // p = min(t e^{lam/eps}, max(t e^{-lam/eps}, y))
      const float ly = y > 0.f ? logf(y) : -INFINITY;
      return expf(fminf(fmaxf(ly - lt, -pc.lam_eps), pc.lam_eps));
    }
    case FIT_L2: {  // p = (eps/lam) W0((lam/eps) t e^{lam y / eps})
      const float p = pc.eps_lam * wright_omega<float>(pc.log_lam_eps + lt + pc.lam_eps * y);
      return p / t;
    }
    case FIT_L2_TV: {  // tau = prox_TV(t), p = prox_L2(tau)
      const float ly = y > 0.f ? logf(y) : -INFINITY;
      const float ltau = lt + fminf(fmaxf(ly - lt, -pc.lam2_eps), pc.lam2_eps);
      const float p = pc.eps_lam * wright_omega<float>(pc.log_lam_eps + ltau + pc.lam_eps * y);
      return p / t;
    }
    case FIT_POISSON: {  // p = (lam/eps) y / W0((lam/eps) (y/t) e^{lam/eps})
      if (!(y > 0.f)) return 0.f;
      const float p = pc.lam_eps * y / wright_omega<float>(pc.log_lam_eps + logf(y) - lt + pc.lam_eps);
      return p / t;
    }
  }
  return 1.f;
}

struct EpiProx {
  static constexpr int NRED = 0;
  static constexpr bool RED_IS_MAX[2] = {false, false};
  float* V;
  const float* Y;
  const int* done;
  ProxConsts pc;
  int ld, ldy, n_valid;
  bool do_red;
  unsigned short* Vbf;  // BF16 shadow of v for a BF16 product (null: none)
  __device__ __forceinline__ void elem(int m, int n, float t, float*) const {
    const size_t o = (size_t)m * ld + n;
    if (n >= n_valid) {
      V[o] = 0.f;
      if (Vbf) Vbf[o] = 0;
      return;
    }
    if (done[m]) return;
    const float v = target_scaling(pc, t, Y[(size_t)m * ldy + n]);
    V[o] = v;
    if (Vbf) Vbf[o] = f32_to_bf16(v);
  }
  __device__ __forceinline__ void row_partial(int, int, const float*) const {}
};

// ---------------------------------------------------------------------------
// Set-up and bookkeeping kernels.

// K = exp(-C / eps) in FP64, rounded to FP32, zero-padded to [np, np].
// With transpose=1 the output is K^T.
__global__ void build_kernel_f32(const double* __restrict__ C, int n, int np, double inv_eps, int transpose,
                                 float* __restrict__ K) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= np || i >= np) return;
  float v = 0.f;
  if (i < n && j < n) v = (float)exp(-(transpose ? C[(size_t)j * n + i] : C[(size_t)i * n + j]) * inv_eps);
  K[(size_t)i * np + j] = v;
}

// Dictionary copies: Dp [np, kp] (= D, zero padded), DTp [kp, np] (= D^T),
// per-column constants colc[j] = {1/x_j, shift_j, gamma_j, log gamma_j} and
// the rows holding its nonzero entries, band[j] = [lo, hi) ([0, 0) if none).
__global__ void prep_dictionary(const float* __restrict__ D, int n, int k, int np, int kp, int pen, double eps,
                                double alpha, double beta, float* __restrict__ Dp, float* __restrict__ DTp,
                                float4* __restrict__ colc, int2* __restrict__ band, int* __restrict__ bad) {
  const int j = blockIdx.x;
  if (j >= kp) return;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    const float d = (i < n && j < k) ? D[(size_t)i * k + j] : 0.f;
    Dp[(size_t)i * kp + j] = d;
    DTp[(size_t)j * np + i] = d;
    if (!(d >= 0.f) || !isfinite(d)) bad[0] = 1;
  }
  if (threadIdx.x == 0) {
    float4 c = {0.f, 0.f, 1.f, 0.f};
    int lo = n, hi = 0;
    if (j < k) {
      double x = 0.0;
      for (int i = 0; i < n; ++i) {
        const float d = D[(size_t)i * k + j];
        x += (double)d;
        if (d != 0.f) {
          lo = min(lo, i);
          hi = i + 1;
        }
      }
      if (!(x > 0.0)) bad[0] = 1;
      double shift = 0.0, gam = 1.0;
      if (pen == PEN_L1) shift = alpha / (eps * x);
      if (pen == PEN_L2SQ) gam = alpha / (eps * x);
      if (pen == PEN_EN) {
        shift = alpha / (eps * x);
        gam = beta / (eps * x);
      }
      c = make_float4((float)(1.0 / x), (float)shift, (float)gam, (float)log(gam));
    }
    colc[j] = c;
    band[j] = lo < hi ? make_int2(lo, hi) : make_int2(0, 0);
  }
}

// Per-spectrum set-up: validity of y, total mass, and the initial state
// (cold: v = 1, w0_j = sum(y) / (k x_j); warm: v = exp(logV), w = W).
// One workgroup per spectrum.
__global__ void init_state(const float* __restrict__ Y, const float* __restrict__ Win,
                           const float* __restrict__ logVin, const float4* __restrict__ colc, int n, int k,
                           int np, int kp, int warm, float* __restrict__ V, float* __restrict__ W,
                           float* __restrict__ U, int* __restrict__ done, int* __restrict__ status,
                           int* __restrict__ iters, float* __restrict__ ew_prev, float* __restrict__ ew_best,
                           int* __restrict__ stall, int* __restrict__ mm_until, int mm_warmup,
                           int* __restrict__ xflags, int* __restrict__ bad) {
  const int b = blockIdx.x;
  __shared__ double ssum[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    const size_t o = (size_t)b * np + i;
    if (i < n) {
      const float y = Y[(size_t)b * n + i];
      if (!(y >= 0.f) || !isfinite(y)) bad[0] = 1;
      acc += (double)y;
      V[o] = warm ? expf(logVin[(size_t)b * n + i]) : 1.f;
    } else {
      V[o] = 0.f;
    }
    U[o] = 0.f;
  }
  ssum[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) ssum[threadIdx.x] += ssum[threadIdx.x + s];
    __syncthreads();
  }
  const double mass = ssum[0];
  for (int j = threadIdx.x; j < kp; j += blockDim.x) {
    float w = 0.f;
    if (j < k) w = warm ? Win[(size_t)b * k + j] : (float)(mass / k * (double)colc[j].x);
    W[(size_t)b * kp + j] = w;
  }
  if (threadIdx.x == 0) {
    done[b] = 0;
    status[b] = 0;
    iters[b] = 0;
    ew_prev[b] = 0.f;
    ew_best[b] = INFINITY;
    stall[b] = 0;
    mm_until[b] = warm ? 0 : mm_warmup;
    xflags[b] = 0;
  }
}

// Fallback of a warm start: at the first convergence test, a spectrum whose
// weight change over the interval exceeds `probe` relative to the weights in
// the l1 norm, sum|w - w_start| / sum|w| (pln / pld; a good prediction errs on
// a few weights, a bad one on all of them), or is not finite, is restarted
// from the cold start (v = 1, w0_j = sum(y)/(k x_j), u = 0), takes MM steps up
// to iteration it + mm_warmup, and is flagged (bit 16 of xflags).  The caller
// recomputes a = D w afterwards.  One workgroup per spectrum.
__global__ void warm_fallback(const float* __restrict__ pln, const float* __restrict__ pld, float probe,
                              const float* __restrict__ Y, const float4* __restrict__ colc, int n, int k, int np,
                              int kp, int it, int mm_warmup, float* __restrict__ V, unsigned short* __restrict__ Vbf,
                              float* __restrict__ W, float* __restrict__ Wsnap, float* __restrict__ U,
                              int* __restrict__ done, int* __restrict__ status, float* __restrict__ ew_prev,
                              float* __restrict__ ew_best, int* __restrict__ stall, int* __restrict__ mm_until,
                              int* __restrict__ xflags, int* __restrict__ count) {
  const int b = blockIdx.x;
  const float d = pld[b] > 0.f ? pln[b] / pld[b] : 0.f;
  if (d <= probe) return;  // also skips nothing for NaN: NaN fails the comparison and falls back
  __shared__ double ssum[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += (double)Y[(size_t)b * n + i];
  ssum[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) ssum[threadIdx.x] += ssum[threadIdx.x + s];
    __syncthreads();
  }
  const double mass = ssum[0];
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    const size_t o = (size_t)b * np + i;
    V[o] = i < n ? 1.f : 0.f;
    if (Vbf) Vbf[o] = i < n ? (unsigned short)0x3f80 : (unsigned short)0;  // BF16 1.0
    U[o] = 0.f;
  }
  for (int j = threadIdx.x; j < kp; j += blockDim.x) {
    const float w = j < k ? (float)(mass / k * (double)colc[j].x) : 0.f;
    W[(size_t)b * kp + j] = w;
    Wsnap[(size_t)b * kp + j] = w;
  }
  if (threadIdx.x == 0) {
    done[b] = 0;
    status[b] = 0;
    ew_prev[b] = 0.f;
    ew_best[b] = INFINITY;
    stall[b] = 0;
    mm_until[b] = it + mm_warmup;
    xflags[b] |= 16;
    atomicAdd(count, 1);
  }
}

// Scaling range test of a bulk phase (FP32 state): an active spectrum with
// |log u_i| > tau or |log v_i| > tau for some bin stops its bulk phase and
// continues in the FP64 phase, whose state has the range of exp(+-709); it is
// flagged (bit 32 of xflags) and leaves the active count.  One wave per
// spectrum.
__global__ __launch_bounds__(256) void range_check(const float* __restrict__ U, const float* __restrict__ V, int n,
                                                   int np, int B, float tau, int it, int* __restrict__ done,
                                                   int* __restrict__ status, int* __restrict__ iters,
                                                   int* __restrict__ xflags, int* __restrict__ active) {
  const int b = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (b >= B || done[b]) return;
  float m = 0.f;
  for (int i = lane; i < n; i += 64) {
    const float u = U[(size_t)b * np + i], v = V[(size_t)b * np + i];
    if (u > 0.f) m = fmaxf(m, fabsf(logf(u)));
    if (v > 0.f) m = fmaxf(m, fabsf(logf(v)));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if (lane == 0 && m > tau) {
    done[b] = 1;
    status[b] = 32;
    iters[b] = it;
    xflags[b] |= 32;
    atomicSub(active, 1);
  }
}

// Active spectra after a convergence test (and the warm-start fallback and
// range promotion that follow it): rows[0 .. c) = the b with done[b] == 0 in
// increasing order, and flags[0] = c, the count the host reads.  One
// workgroup, wave ballots.
__global__ __launch_bounds__(1024) void compact_active(const int* __restrict__ done, int B, int* __restrict__ rows,
                                                        int* __restrict__ flags) {
  __shared__ int wsum[16];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int base = 0;
  for (int c0 = 0; c0 < B; c0 += 1024) {
    const int r = c0 + tid;
    const bool on = r < B && !done[r];
    const unsigned long long m = __ballot(on);
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wave] = __popcll(m);
    __syncthreads();
    int off = 0, tot = 0;
    for (int w = 0; w < 16; ++w) {
      off += w < wave ? wsum[w] : 0;
      tot += wsum[w];
    }
    if (on) rows[base + off + before] = r;
    base += tot;
    __syncthreads();
  }
  if (tid == 0) flags[0] = base;
}

// Weight change over a check interval, per spectrum: max_j |w_j - w^snap_j|
// and max_j |w_j|, where w^snap holds the weights at the previous test (the
// stopping rule), and, when pln is not null, sum_j |w_j - w^snap_j| and
// sum_j |w_j| (the warm-start probe); then w^snap = w.  With init = 1 it only
// takes the snapshot (start of a phase).  NaN propagates into the maxima and
// the sums.  One wave per spectrum.
__device__ __forceinline__ double nan_max(double a, double b) { return (a > b || a != a) ? a : b; }

template <class T>
__global__ __launch_bounds__(256) void interval_change(const T* __restrict__ W, int ld, int k, int B,
                                                       T* __restrict__ snap, int init, float* __restrict__ pwn,
                                                       float* __restrict__ pwd, float* __restrict__ pln,
                                                       float* __restrict__ pld) {
  const int b = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (b >= B) return;
  double dw = 0.0, wm = 0.0, ds = 0.0, ws = 0.0;
  for (int j = lane; j < k; j += 64) {
    const size_t o = (size_t)b * ld + j;
    const T w = W[o];
    const double dj = fabs((double)w - (double)snap[o]);
    dw = nan_max(dw, dj);
    wm = nan_max(wm, fabs((double)w));
    ds += dj;
    ws += fabs((double)w);
    snap[o] = w;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    dw = nan_max(dw, __shfl_xor(dw, off, 64));
    wm = nan_max(wm, __shfl_xor(wm, off, 64));
    ds += __shfl_xor(ds, off, 64);
    ws += __shfl_xor(ws, off, 64);
  }
  if (lane == 0 && !init) {
    pwn[b] = (float)dw;
    pwd[b] = (float)wm;
    if (pln) {
      pln[b] = (float)ds;
      pld[b] = (float)ws;
    }
  }
}

// Convergence test for every spectrum (the stopping rule of "while not
// converged").  e_src = sum|u s - a| / sum a, assembled from the per-tile
// partials in a fixed order, and d = max|w - w^snap| / max|w|, the relative
// weight change over the check interval.  For a linearly converging iteration
// the interval changes shrink geometrically, rho = d / d_prev, and the
// distance to the limit is d rho / (1 - rho) (the a-posteriori bound of the
// c-step map; exact for a geometric sequence).  A spectrum stops when
// e_src <= tol and either that bound is <= tol, or d has reached the resolution
// `floor` of the phase's precision without shrinking since the last test (the
// iteration no longer moves w beyond its rounding noise; a change below the
// floor that still shrinks is real, slow contraction and the bound decides).
// A spectrum whose d has not improved on its best value for OTLM_STALL_CHECKS
// tests has reached the noise floor of its precision on an ill-conditioned
// problem: it stops with status 8.  One workgroup; also counts the spectra
// still active into *active.  The iteration index recorded for a stopping
// spectrum is `it` (or *it_dev when it_dev is not null) plus it_base[b] when
// it_base is not null.
constexpr int OTLM_STALL_CHECKS = 6;
__global__ void check_convergence(const float* __restrict__ psn, const float* __restrict__ psd, int nts,
                                  const float* __restrict__ pwn, const float* __restrict__ pwd, int B, float tol,
                                  float floor_w, int it, float* __restrict__ ew_prev, float* __restrict__ ew_best,
                                  int* __restrict__ stall, int* __restrict__ done, int* __restrict__ iters,
                                  int* __restrict__ status, int* __restrict__ active,
                                  const int* __restrict__ it_dev, const int* __restrict__ it_base) {
  __shared__ int cnt[1024];
  if (it_dev) it = it_dev[0];  // iteration index kept on the device (captured chunks)
  int count = 0;
  for (int b = threadIdx.x; b < B; b += blockDim.x) {
    if (!done[b]) {
      float num = 0.f, den = 0.f;
      for (int t = 0; t < nts; ++t) {
        num += psn[(size_t)b * nts + t];
        den += psd[(size_t)b * nts + t];
      }
      const float dw = pwn[b], wm = pwd[b];
      const float esrc = den > 0.f ? num / den : 0.f;
      const float ew = wm > 0.f ? dw / wm : 0.f;
      const float prev = ew_prev[b];
      ew_prev[b] = ew;
      float bound = INFINITY;
      const bool shrinking = prev > 0.f && ew < prev;
      if (ew == 0.f) {
        bound = 0.f;
      } else if (shrinking) {
        const float rho = ew / prev;
        bound = ew * rho / (1.f - rho);
      }
      int st = 0;
      if (ew < ew_best[b]) {
        ew_best[b] = ew;
        stall[b] = 0;
      } else {
        stall[b] += 1;
      }
      if (!isfinite(num + den + dw + wm)) st = 4;
      else if (esrc <= tol && (bound <= tol || (ew <= floor_w && !shrinking))) st = 1;
      else if (stall[b] >= OTLM_STALL_CHECKS) st = 8;
      if (st) {
        done[b] = 1;
        status[b] = st;
        iters[b] = it + (it_base ? it_base[b] : 0);
      } else {
        ++count;
      }
    }
  }
  cnt[threadIdx.x] = count;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) cnt[threadIdx.x] += cnt[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) active[0] = cnt[0];
}

// Outputs: W (unpadded), log u, log v, iteration counts and status flags.
__global__ void write_outputs(const float* __restrict__ Wst, const float* __restrict__ U,
                              const float* __restrict__ V, const int* __restrict__ done,
                              const int* __restrict__ st, const int* __restrict__ it_in,
                              const int* __restrict__ xflags, const int* __restrict__ it_base, int n, int k,
                              int np, int kp, int max_iter, float* __restrict__ W, float* __restrict__ logU,
                              float* __restrict__ logV, int* __restrict__ iters, int* __restrict__ status) {
  const int b = blockIdx.x;
  for (int j = threadIdx.x; j < k; j += blockDim.x) W[(size_t)b * k + j] = Wst[(size_t)b * kp + j];
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    if (logU) logU[(size_t)b * n + i] = logf(U[(size_t)b * np + i]);
    logV[(size_t)b * n + i] = logf(V[(size_t)b * np + i]);
  }
  if (threadIdx.x == 0) {
    if (iters) iters[b] = done[b] ? it_in[b] : max_iter + it_base[b];
    if (status) status[b] = (done[b] ? st[b] : 2) | xflags[b];
  }
}
