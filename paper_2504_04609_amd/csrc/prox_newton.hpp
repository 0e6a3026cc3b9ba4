// Exact weight proximal step on the GPU:
//
//   w = argmin_{w >= 0}  alpha R(w) + eps KL(D w || s)          (ProxP)
//
// the problem that the single MM step of Table 2 only decreases.  The paper
// allows the MM iteration to be run to convergence instead of one step
// (subsection "Iterative Algorithm for OTLM"); on dictionaries with strongly
// overlapping columns a multiplicative step crawls along the flat directions,
// so this kernel solves the same convex problem by an active-set Newton method:
//   gradient  g = alpha R'(w) + eps D^T log(D w / s)
//   Hessian   H = alpha R'' + eps D^T diag(1 / D w) D          (free weights only)
// Newton step on the free weights, ratio test to the first weight reaching 0
// (it joins the active set), Armijo backtracking, and release of the active
// weight with the most negative gradient once the free gradient vanishes.
// Weights that are exactly 0 are the active set, so the state carried between
// outer iterations is just W.
//
// One workgroup (256 threads) per spectrum, everything in FP64 (the Hessian of
// an overlapping Gaussian dictionary has condition numbers near 1e12).  LDS
// holds s, a = D w and 1/sqrt(a) or log(a/s) for the n bins, the 64 x 64
// Hessian / Cholesky factor and an 8-bin slab of scaled dictionary rows:
// (16 + sizeof(s)) n + 39.5 KB, so n <= 1024 fits the 64 KB a workgroup gets
// by default in both the FP32-state and the FP64-state (refinement) variants.
#pragma once
#include <hip/hip_runtime.h>
#include "solver_kernels.hpp"

constexpr int PN_THREADS = 256;
constexpr int PN_K = 64;    // largest dictionary handled by this kernel
constexpr int PN_CH = 8;    // bins per slab in the Hessian build
constexpr int PN_HLD = PN_K + 1;

template <class TS, class TW>
struct ProxNewtonArgs {
  const TS* S;         // [B, ld_s]  s = K v
  TW* W;               // [B, ld_w]  weights (in: start, out: prox)
  const float* Dp;     // [np, ld_d] dictionary, zero padded
  const float4* colc;  // per column {1/x_j, ...}
  const int* done;
  float* pwn;          // e_w partials, one tile per spectrum
  float* pwd;
  int* nit;            // Newton iterations done, accumulated per spectrum
  int ld_s, ld_w, ld_d, n, k, pen, max_newton;
  double eps, alpha, beta, gtol;
};

__device__ __forceinline__ double pn_block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

__device__ __forceinline__ double pn_block_min(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
}

// penalty value alpha R(w) and derivatives, per weight
__device__ __forceinline__ double pn_pen(int pen, double w, double alpha, double beta) {
  if (pen == PEN_L1) return alpha * w;
  if (pen == PEN_L2SQ) return 0.5 * alpha * w * w;
  if (pen == PEN_EN) return alpha * w + 0.5 * beta * w * w;
  return 0.0;
}
__device__ __forceinline__ double pn_pen_grad(int pen, double w, double alpha, double beta) {
  if (pen == PEN_L1) return alpha;
  if (pen == PEN_L2SQ) return alpha * w;
  if (pen == PEN_EN) return alpha + beta * w;
  return 0.0;
}

// V(w) = eps sum_i (a_i log(a_i/s_i) - a_i + s_i) + sum_j alpha R(w_j), a = D w
// (bins with a = 0 give s_i); stores a when `a` is not null.
template <class TS, class TW>
__device__ double pn_eval(const ProxNewtonArgs<TS, TW>& p, const double* w, const TS* s, double* a, double* red) {
  const int n = p.n, k = p.k;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += PN_THREADS) {
    const float* drow = p.Dp + (size_t)i * p.ld_d;
    double ai = 0.0;
    for (int j = 0; j < k; ++j) ai += (double)drow[j] * w[j];
    if (a) a[i] = ai;
    const double si = (double)s[i];
    acc += (ai > 0.0 ? ai * log(ai / si) : 0.0) - ai + si;
  }
  double v = p.eps * pn_block_sum(acc, red);
  double pv = 0.0;
  for (int j = 0; j < k; ++j) pv += pn_pen(p.pen, w[j], p.alpha, p.beta);
  return v + pv;
}

template <class TS, class TW>
__global__ __launch_bounds__(PN_THREADS) void prox_newton_kernel(ProxNewtonArgs<TS, TW> p) {
  const int b = blockIdx.x;
  if (p.done[b]) return;
  extern __shared__ double smem[];
  const int n = p.n, k = p.k, tid = threadIdx.x;
  double* a = smem;                    // [n]  D w at the current point
  double* l = a + n;                   // [n]  log(a/s) or 1/sqrt(a)
  double* H = l + n;                   // [64][65]
  double* Ms = H + PN_K * PN_HLD;      // [PN_CH][64]
  double* w = Ms + PN_CH * PN_K;       // [64]
  double* wt = w + PN_K;               // [64]
  double* g = wt + PN_K;               // [64]
  double* d = g + PN_K;                // [64]
  double* red = d + PN_K;              // [8]
  TS* s = reinterpret_cast<TS*>(red + 8);  // [n]
  __shared__ int act[PN_K];
  __shared__ int ctl[4];

  const TS* srow = p.S + (size_t)b * p.ld_s;
  TW* wrow = p.W + (size_t)b * p.ld_w;
  for (int i = tid; i < n; i += PN_THREADS) s[i] = srow[i];
  for (int j = tid; j < PN_K; j += PN_THREADS) {
    const double wj = j < k ? (double)wrow[j] : 0.0;
    w[j] = wj > 0.0 ? wj : 0.0;
    act[j] = (j < k && wj > 0.0) ? 0 : 1;   // padded columns stay active at 0
  }
  __syncthreads();
  const double tiny = 1e-300;
  const double gscale = fmax(fmax(p.alpha, p.eps), 1e-300) * p.gtol;
  const double hpen = p.pen == PEN_L2SQ ? p.alpha : (p.pen == PEN_EN ? p.beta : 0.0);

  int it = 0;
  for (; it < p.max_newton; ++it) {
    const double f = pn_eval(p, w, s, a, red);   // also a = D w
    // ---- gradient: g_j = alpha R'(w_j) + eps sum_i D_ij log(a_i / s_i)
    for (int i = tid; i < n; i += PN_THREADS) l[i] = log(fmax(a[i], tiny) / (double)s[i]);
    __syncthreads();
    {
      const int j = tid & 63, q = tid >> 6;
      double part = 0.0;
      if (j < k)
        for (int i = q; i < n; i += 4) part += (double)p.Dp[(size_t)i * p.ld_d + j] * l[i];
      Ms[q * PN_K + j] = part;
      __syncthreads();
      if (tid < PN_K) {
        const double gj = Ms[tid] + Ms[PN_K + tid] + Ms[2 * PN_K + tid] + Ms[3 * PN_K + tid];
        g[tid] = tid < k ? pn_pen_grad(p.pen, w[tid], p.alpha, p.beta) + p.eps * gj : 0.0;
      }
      __syncthreads();
    }
    // ---- optimality of the free set; release the most negative active gradient
    if (tid == 0) {
      double kkt = 0.0, gmin = 0.0;
      int jmin = -1;
      for (int j = 0; j < k; ++j) {
        if (!act[j]) kkt = fmax(kkt, fabs(g[j]));
        else if (g[j] < gmin) {
          gmin = g[j];
          jmin = j;
        }
      }
      int stop = 0;
      if (kkt <= gscale) {
        if (jmin >= 0 && gmin < -gscale) act[jmin] = 0;
        else stop = 1;
      }
      ctl[0] = stop;
    }
    __syncthreads();
    if (ctl[0]) break;

    // ---- Hessian on the free set: H = eps D^T diag(1/a) D + hpen I
    for (int i = tid; i < n; i += PN_THREADS) l[i] = 1.0 / sqrt(fmax(a[i], tiny));
    {
      const int q = tid >> 6, blk = tid & 63, bj = blk >> 3, bl = blk & 7;
      double acc[8][8];
#pragma unroll
      for (int x = 0; x < 8; ++x)
#pragma unroll
        for (int y = 0; y < 8; ++y) acc[x][y] = 0.0;
      for (int c0 = 0; c0 < n; c0 += PN_CH) {
        __syncthreads();
        for (int e = tid; e < PN_CH * PN_K; e += PN_THREADS) {
          const int r = e >> 6, j = e & 63, i = c0 + r;
          Ms[e] = (i < n && j < k) ? (double)p.Dp[(size_t)i * p.ld_d + j] * l[i] : 0.0;
        }
        __syncthreads();
        for (int r = q; r < PN_CH; r += 4) {
          const double* row = Ms + r * PN_K;
          double xa[8], xb[8];
#pragma unroll
          for (int x = 0; x < 8; ++x) {
            xa[x] = row[bj * 8 + x];
            xb[x] = row[bl * 8 + x];
          }
#pragma unroll
          for (int x = 0; x < 8; ++x)
#pragma unroll
            for (int y = 0; y < 8; ++y) acc[x][y] += xa[x] * xb[y];
        }
      }
      // fold the four bin groups into H (sequentially, one group at a time)
      for (int grp = 0; grp < 4; ++grp) {
        __syncthreads();
        if (q == grp) {
#pragma unroll
          for (int x = 0; x < 8; ++x)
#pragma unroll
            for (int y = 0; y < 8; ++y) {
              double* h = &H[(bj * 8 + x) * PN_HLD + bl * 8 + y];
              *h = (grp == 0 ? 0.0 : *h) + acc[x][y];
            }
        }
      }
      __syncthreads();
    }
    // scale, add the penalty curvature, and pin the active weights (identity rows)
    for (int e = tid; e < PN_K * PN_K; e += PN_THREADS) {
      const int r = e >> 6, c = e & 63;
      double h = p.eps * H[r * PN_HLD + c];
      if (act[r] || act[c]) h = (r == c) ? 1.0 : 0.0;
      else if (r == c) h += hpen;
      H[r * PN_HLD + c] = h;
    }
    __syncthreads();
    // ---- Cholesky H = L L^T (lower triangle, in place)
    for (int c = 0; c < PN_K; ++c) {
      if (tid == 0) {
        const double dgl = H[c * PN_HLD + c];
        H[c * PN_HLD + c] = sqrt(dgl > 0.0 ? dgl : 1e-300);
      }
      __syncthreads();
      const double piv = H[c * PN_HLD + c];
      for (int r = c + 1 + tid; r < PN_K; r += PN_THREADS) H[r * PN_HLD + c] /= piv;
      __syncthreads();
      const int m = PN_K - 1 - c;
      for (int e = tid; e < m * m; e += PN_THREADS) {
        const int r = c + 1 + e / m, cc = c + 1 + e % m;
        if (cc <= r) H[r * PN_HLD + cc] -= H[r * PN_HLD + c] * H[cc * PN_HLD + c];
      }
      __syncthreads();
    }
    // ---- solve L L^T d = -g (active rows have g = 0 -> d = 0)
    if (tid < PN_K) d[tid] = act[tid] ? 0.0 : -g[tid];
    __syncthreads();
    for (int c = 0; c < PN_K; ++c) {  // forward: L y = -g
      if (tid == 0) d[c] /= H[c * PN_HLD + c];
      __syncthreads();
      for (int r = c + 1 + tid; r < PN_K; r += PN_THREADS) d[r] -= H[r * PN_HLD + c] * d[c];
      __syncthreads();
    }
    for (int c = PN_K - 1; c >= 0; --c) {  // backward: L^T d = y
      if (tid == 0) d[c] /= H[c * PN_HLD + c];
      __syncthreads();
      for (int r = tid; r < c; r += PN_THREADS) d[r] -= H[c * PN_HLD + r] * d[c];
      __syncthreads();
    }
    // ---- ratio test and Armijo backtracking
    double slope = 0.0, tmax = INFINITY;
    {
      const double sl = (tid < PN_K && !act[tid]) ? g[tid] * d[tid] : 0.0;
      const double tm = (tid < PN_K && !act[tid] && d[tid] < 0.0) ? -w[tid] / d[tid] : INFINITY;
      slope = pn_block_sum(sl, red);
      tmax = pn_block_min(tm, red);
    }
    if (!(slope < 0.0)) break;
    double t = fmin(1.0, tmax), fn = 0.0;
    bool accepted = false;
    for (int ls = 0; ls < 60; ++ls) {
      if (tid < PN_K) wt[tid] = act[tid] ? 0.0 : fmax(w[tid] + t * d[tid], 0.0);
      __syncthreads();
      fn = pn_eval(p, wt, s, nullptr, red);
      if (fn <= f + 1e-4 * t * slope) {
        accepted = true;
        break;
      }
      t *= 0.5;
    }
    if (!accepted) break;
    const bool hit = (t == tmax);
    if (tid < PN_K) {
      double wn = wt[tid];
      // the weights that stop the ratio test join the active set at exactly 0
      if (hit && !act[tid] && d[tid] < 0.0 && -w[tid] / d[tid] <= tmax * (1.0 + 1e-12)) {
        act[tid] = 1;
        wn = 0.0;
      }
      w[tid] = wn;
    }
    __syncthreads();
  }

  // ---- write back and the weight-change reductions for the convergence test
  double dw = 0.0, wm = 0.0;
  if (tid < k) {
    const TW wold = wrow[tid];
    const TW wnew = (TW)w[tid];
    wrow[tid] = wnew;
    dw = fabs((double)wnew - (double)wold);
    wm = fabs((double)wnew);
  }
  if (tid < PN_K && tid >= k && tid < p.ld_w) wrow[tid] = (TW)0;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    dw = fmax(dw, __shfl_xor(dw, off, 64));
    wm = fmax(wm, __shfl_xor(wm, off, 64));
  }
  if (tid == 0) {
    p.pwn[b] = (float)dw;
    p.pwd[b] = (float)wm;
    p.nit[b] += it;
  }
}

inline size_t prox_newton_smem(int n, size_t s_bytes) {
  return sizeof(double) * ((size_t)2 * n + PN_K * PN_HLD + PN_CH * PN_K + 4 * PN_K + 8) + s_bytes * (size_t)n;
}
