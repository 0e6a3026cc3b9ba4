// FP64 evaluation of the OTLM objective, its Fenchel dual and the optimality
// residuals at a given (w, log u, log v) -- eq. OTLM in the scaling form
// eps KL(Q||K) + F1(Q1) + F2(Q^T 1), with Q = diag(u) K diag(v).  Not on the
// solve path: it certifies a solution.
#pragma once
#include <hip/hip_runtime.h>
#include "solver_kernels.hpp"

// K = exp(-C / eps) in FP64 (also K^T when requested), unpadded [n, n].
__global__ void build_kernel_f64(const double* __restrict__ C, int n, double inv_eps, int transpose,
                                 double* __restrict__ K) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= n) return;
  K[(size_t)i * n + j] = exp(-(transpose ? C[(size_t)j * n + i] : C[(size_t)i * n + j]) * inv_eps);
}

// K = exp(-C / eps) in FP64, zero padded to [np, np] (refinement products).
__global__ void build_kernel_f64p(const double* __restrict__ C, int n, int np, double inv_eps, int transpose,
                                  double* __restrict__ K) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= np || i >= np) return;
  double v = 0.0;
  if (i < n && j < n) v = exp(-(transpose ? C[(size_t)j * n + i] : C[(size_t)i * n + j]) * inv_eps);
  K[(size_t)i * np + j] = v;
}

__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Per row i of spectrum b: s_i = (K v)_i, t_i = (K^T u)_i, q_i = u_i (C o K v)_i.
// One wave64 per row, lanes stride over the row (coalesced).
__global__ void objective_products(const double* __restrict__ K, const double* __restrict__ KT,
                                   const double* __restrict__ C, const float* __restrict__ logU,
                                   const float* __restrict__ logV, int n, double* __restrict__ s,
                                   double* __restrict__ t, double* __restrict__ q) {
  const int b = blockIdx.y;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const float* lu = logU + (size_t)b * n;
  const float* lv = logV + (size_t)b * n;
  double as = 0.0, at = 0.0, aq = 0.0;
  for (int j = lane; j < n; j += 64) {
    const double vj = exp((double)lv[j]);
    const double uj = exp((double)lu[j]);
    const double kij = K[(size_t)i * n + j];
    as += kij * vj;
    aq += C[(size_t)i * n + j] * kij * vj;
    at += KT[(size_t)i * n + j] * uj;
  }
  as = wave_sum_f64(as);
  at = wave_sum_f64(at);
  aq = wave_sum_f64(aq);
  if (lane == 0) {
    const double ui = exp((double)lu[i]);
    s[(size_t)b * n + i] = as;
    t[(size_t)b * n + i] = at;
    q[(size_t)b * n + i] = ui * aq;
  }
}

__device__ double block_sum_f64(double v, double* sh) {
  v = wave_sum_f64(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
  return r;
}

__device__ double block_max_f64(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double r = sh[0];
  for (int i = 1; i < (int)(blockDim.x >> 6); ++i) r = fmax(r, sh[i]);
  return r;
}

struct ObjParams {
  int n, k, fit, pen;
  double eps, lam, lam2, alpha, beta, sumK;
};

// F2*(-g_j) for one bin (F2 = lam L(. | y) on m >= 0).
__device__ __forceinline__ double datafit_conj_neg(const ObjParams& p, double g, double y) {
  const double z = -g;
  switch (p.fit) {
    case FIT_KL: return p.lam * y * (exp(z / p.lam) - 1.0);
    case FIT_L2: return (y + z / p.lam >= 0.0) ? z * y + z * z / (2.0 * p.lam) : -0.5 * p.lam * y * y;
    case FIT_TV: return z <= p.lam ? fmax(z * y, -p.lam * y) : INFINITY;
    case FIT_L2_TV: {
      double m = y;
      if (z > p.lam2) m = y + (z - p.lam2) / p.lam;
      else if (z < -p.lam2) m = y + (z + p.lam2) / p.lam;
      m = fmax(m, 0.0);
      return z * m - 0.5 * p.lam * (m - y) * (m - y) - p.lam2 * fabs(m - y);
    }
  }
  return NAN;
}

__device__ __forceinline__ double datafit_value(const ObjParams& p, double m, double y) {
  switch (p.fit) {
    case FIT_KL: return p.lam * ((m > 0.0 ? m * log(m / y) : 0.0) - m + y);
    case FIT_TV: return p.lam * fabs(m - y);
    case FIT_L2: return 0.5 * p.lam * (m - y) * (m - y);
    case FIT_L2_TV: return 0.5 * p.lam * (m - y) * (m - y) + p.lam2 * fabs(m - y);
    case FIT_POISSON: return -p.lam * ((y > 0.0 ? y * log(m) : 0.0) - m);
    case FIT_BALANCED: return 0.0;
  }
  return NAN;
}

// dist(-g, dF2(m)) / lam for one bin (target stationarity).
__device__ __forceinline__ double target_residual(const ObjParams& p, double g, double m, double y) {
  switch (p.fit) {
    case FIT_KL: return fabs(-g - p.lam * log(m / y)) / p.lam;
    case FIT_L2: return fabs(-g - p.lam * (m - y)) / p.lam;
    case FIT_TV:
    case FIT_L2_TV: {
      const double lt = p.fit == FIT_TV ? p.lam : p.lam2;
      const double zz = -g - (p.fit == FIT_TV ? 0.0 : p.lam * (m - y));
      const bool on = fabs(m - y) <= 1e-12 * fmax(fabs(y), 1e-300);
      const double r = on ? fmax(fabs(zz) - lt, 0.0) : fabs(zz - lt * (m > y ? 1.0 : -1.0));
      return r / p.lam;
    }
  }
  return 0.0;
}

// One workgroup per spectrum: assembles [primal, dual, <C,Q>, src, tgt, wkkt].
__global__ void objective_reduce(ObjParams p, const float* __restrict__ D, const float* __restrict__ Y,
                                 const float* __restrict__ W, const float* __restrict__ logU,
                                 const float* __restrict__ logV, const double* __restrict__ s,
                                 const double* __restrict__ t, const double* __restrict__ q,
                                 double* __restrict__ out) {
  __shared__ double sh[16];
  const int b = blockIdx.x, n = p.n, k = p.k;
  const float* lu = logU + (size_t)b * n;
  const float* lv = logV + (size_t)b * n;
  const float* y = Y + (size_t)b * n;
  const float* w = W + (size_t)b * k;
  double la = 0, lm = 0, sa = 0, fit = 0, conj2 = 0, us = 0, cq = 0, srcn = 0, srcd = 0, tgt = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double ui = exp((double)lu[i]), vi = exp((double)lv[i]);
    const double si = s[(size_t)b * n + i], ti = t[(size_t)b * n + i];
    const double a = ui * si, m = vi * ti, yi = y[i];
    if (a > 0.0) la += a * (double)lu[i];
    if (m > 0.0) lm += m * (double)lv[i];
    sa += a;
    fit += datafit_value(p, m, yi);
    conj2 += datafit_conj_neg(p, p.eps * (double)lv[i], yi);
    us += a;
    cq += q[(size_t)b * n + i];
    double dw = 0.0;
    for (int j = 0; j < k; ++j) dw += (double)D[(size_t)i * k + j] * (double)w[j];
    srcn += fabs(a - dw);
    srcd += dw;
    tgt = fmax(tgt, target_residual(p, p.eps * (double)lv[i], m, yi));
  }
  la = block_sum_f64(la, sh);
  lm = block_sum_f64(lm, sh);
  sa = block_sum_f64(sa, sh);
  fit = block_sum_f64(fit, sh);
  conj2 = block_sum_f64(conj2, sh);
  us = block_sum_f64(us, sh);
  cq = block_sum_f64(cq, sh);
  srcn = block_sum_f64(srcn, sh);
  srcd = block_sum_f64(srcd, sh);
  tgt = block_max_f64(tgt, sh);
  // weights: D^T f with f = eps log u (bins with u = 0 carry D_ij = 0)
  double pen = 0.0, conj1 = 0.0, wk = 0.0;
  for (int j = 0; j < k; ++j) {
    double df = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const double l = (double)lu[i];
      if (isfinite(l)) df += (double)D[(size_t)i * k + j] * p.eps * l;
    }
    df = block_sum_f64(df, sh);
    const double wj = (double)w[j];
    double rp = 0.0;
    if (p.pen == PEN_L1) {
      pen += p.alpha * wj;
      rp = p.alpha;
    } else if (p.pen == PEN_L2SQ) {
      pen += 0.5 * p.alpha * wj * wj;
      rp = p.alpha * wj;
      conj1 += fmax(0.0, -df) * fmax(0.0, -df) / (2.0 * p.alpha);
    } else if (p.pen == PEN_EN) {
      pen += p.alpha * wj + 0.5 * p.beta * wj * wj;
      rp = p.alpha + p.beta * wj;
      conj1 += fmax(0.0, -df - p.alpha) * fmax(0.0, -df - p.alpha) / (2.0 * p.beta);
    }
    wk = fmax(wk, fabs(fmin(wj, rp + df)));
  }
  if (threadIdx.x == 0) {
    double* o = out + (size_t)b * 6;
    o[0] = p.eps * (la + lm - sa + p.sumK) + fit + pen;
    o[1] = -conj1 - conj2 - p.eps * (us - p.sumK);
    o[2] = cq;
    o[3] = srcn / srcd;
    o[4] = tgt;
    o[5] = wk;
  }
}
