// Device side of the ragged batch: spectra of different lengths n_b, each with
// its own dictionary D_b [n_b, k_b], solved together by Algorithm 1.
//
// Spectra that share a grid share a Gibbs kernel and form a group; the kernel
// products of all groups run as one grouped MFMA GEMM per product (S = V K^T
// with the source epilogue, T = U K with the target prox epilogue).  The
// dictionary work, which differs per spectrum, is one fused workgroup per
// spectrum: r = log(s / a), the MM weight step of Table 2 (repeated `inner`
// times at fixed s), a = D w and u = a / s.
//
// Dictionaries are kept transposed (D_b^T, [k_b, n_b], each column contiguous)
// together with the band [lo_j, hi_j) that holds every nonzero of column j.
// Products with D touch only the band: for the Gaussian-peak dictionaries of
// the ragged workload (peaks cut at 5 sigma) that is 10-50% of the column.
// Entries inside the band that are zero are used as stored, so the products
// are exact for any nonnegative D.
#pragma once
#include <hip/hip_runtime.h>
#include "omega.hpp"
#include "gemm_nt.hpp"
#include "solver_kernels.hpp"

// One spectrum of a ragged solve, in solve order (groups of equal grid, the
// largest n first; input order inside a group).
struct RgSpec {
  int b;          // input index
  int n, k, np;   // bins, dictionary columns, row stride of the group's [rows, np] arrays
  long long st;   // offset of the spectrum's row in the state arrays
  long long yin;  // offset of y_b, log u_b, log v_b in the packed input/output vectors
  long long din;  // offset of D_b ([n, k] row-major) in the packed input
  long long dt;   // offset of D_b^T ([k, n]) in the transposed copy
  long long col;  // offset of the spectrum's columns in the column tables and the weight state
  long long win;  // offset of w_b in the packed input/output weights
  long long dp;   // offset of D_b ([n, 64] row-major if k <= 64, else [n, 128]; zero padded) for the
                  // Newton prox; -1: none
};

constexpr int RG_THREADS = 256;
// Threads of the weight step per spectrum (256: many spectra in flight in the
// bulk of a solve; the slow tail takes the Newton prox instead).
#ifndef RG_WS_THREADS
#define RG_WS_THREADS 256
#endif
constexpr int RG_MAX_K = 256;
constexpr int RG_MAX_N = 4096;
constexpr int RG_TILE_ROWS = 32;

__device__ __forceinline__ float rg_wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// a_i = sum_j D_ij w_j for the spectrum's bins, summed over j in ascending
// order (entries outside a column's band are exact zeros and add nothing).
__device__ __forceinline__ void rg_dict_apply(const float* __restrict__ DTb, const int2* bnd, const float* w, int n,
                                              int k, float* a) {
  // Loads are unconditional (a load under a per-lane branch drains the wait
  // counter): a column whose band misses the wave's 64 bins is read at one bin
  // just outside its band, the same address for every lane (an exact zero,
  // one cache line), 16 loads in flight
  const int lane = threadIdx.x & 63;
  for (int i0 = threadIdx.x - lane; i0 < n; i0 += blockDim.x) {
    const int ic = min(i0 + lane, n - 1);
    float acc = 0.f;
    int j = 0;
    for (; j + 16 <= k; j += 16) {
      float d[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int2 bj = bnd[j + q];
        const int idx = (bj.x < i0 + 64 && bj.y > i0) ? ic : (bj.y <= i0 ? bj.y : bj.x - 1);
        d[q] = DTb[(size_t)(j + q) * n + idx];
      }
#pragma unroll
      for (int q = 0; q < 16; ++q) acc = fmaf(d[q], w[j + q], acc);
    }
    for (; j < k; ++j) {
      const int2 bj = bnd[j];
      const int idx = (bj.x < i0 + 64 && bj.y > i0) ? ic : (bj.y <= i0 ? bj.y : bj.x - 1);
      acc = fmaf(DTb[(size_t)j * n + idx], w[j], acc);
    }
    if (i0 + lane < n) a[i0 + lane] = acc;
  }
}

// Transposed copy of every D_b, the band of each column, and the per-column
// constants of the weight step {1/x_j, shift_j, gamma_j, log gamma_j}
// (x_j = sum_i D_ij, summed in FP64 in row order); nband[q] = sum_j band
// length.  Flags negative or non-finite entries and empty columns in bad[0].
// One workgroup per spectrum.
__global__ __launch_bounds__(RG_THREADS) void rg_prep_dict(const RgSpec* __restrict__ spec, const float* __restrict__ D,
                                                          int pen, double eps, double alpha, double beta,
                                                          float* __restrict__ DT, float* __restrict__ Dp,
                                                          float4* __restrict__ colc, int2* __restrict__ band,
                                                          int* __restrict__ nband, int* __restrict__ bad) {
  __shared__ int nb_s;
  if (threadIdx.x == 0) nb_s = 0;
  const RgSpec sp = spec[blockIdx.x];
  const int n = sp.n, k = sp.k, ks = k | 1;  // odd LDS stride: conflict-free column reads
  __shared__ float tile[RG_TILE_ROWS * (RG_MAX_K + 1)];
  const float* Db = D + sp.din;
  float* DTb = DT + sp.dt;
  const int j = threadIdx.x;
  double x = 0.0;
  int lo = n, hi = 0, badl = 0;
  for (int i0 = 0; i0 < n; i0 += RG_TILE_ROWS) {
    const int rows = min(RG_TILE_ROWS, n - i0);
    __syncthreads();
    for (int e = threadIdx.x; e < rows * k; e += blockDim.x) {
      const int r = e / k, c = e - r * k;
      tile[r * ks + c] = Db[(size_t)(i0 + r) * k + c];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < rows * k; e += blockDim.x) {
      const int c = e / rows, r = e - c * rows;
      DTb[(size_t)c * n + i0 + r] = tile[r * ks + c];
    }
    if (sp.dp >= 0) {  // row-major copy with 64 or 128 columns for the Newton prox
      const int wdt = k <= 64 ? 64 : 128;
      for (int e = threadIdx.x; e < rows * wdt; e += blockDim.x) {
        const int r = e / wdt, c = e - r * wdt;
        Dp[sp.dp + (size_t)(i0 + r) * wdt + c] = c < k ? tile[r * ks + c] : 0.f;
      }
    }
    if (j < k) {
      for (int r = 0; r < rows; ++r) {
        const float d = tile[r * ks + j];
        if (!(d >= 0.f) || !isfinite(d)) badl = 1;
        if (d != 0.f) {
          lo = min(lo, i0 + r);
          hi = i0 + r + 1;
        }
        x += (double)d;
      }
    }
  }
  if (j < k) {
    if (!(x > 0.0)) badl = 1;
    double shift = 0.0, gam = 1.0;
    if (pen == PEN_L1) shift = alpha / (eps * x);
    if (pen == PEN_L2SQ) gam = alpha / (eps * x);
    if (pen == PEN_EN) {
      shift = alpha / (eps * x);
      gam = beta / (eps * x);
    }
    colc[sp.col + j] = make_float4((float)(1.0 / x), (float)shift, (float)gam, (float)log(gam));
    band[sp.col + j] = make_int2(lo < hi ? lo : 0, lo < hi ? hi : 0);
    if (lo < hi) atomicAdd(&nb_s, hi - lo);
    if (badl) bad[0] = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0) nband[blockIdx.x] = nb_s;
}

// Per-spectrum start: y copied into the group layout (zero padded), the
// initial scalings and weights (cold: v = 1, w0_j = sum(y) / (k x_j); warm:
// v = exp(log v_in), w = w_in), a = D w0 and the convergence bookkeeping.
__global__ __launch_bounds__(RG_THREADS) void rg_init(const RgSpec* __restrict__ spec, const float* __restrict__ Y,
                                                     const float* __restrict__ Win, const float* __restrict__ logVin,
                                                     const float* __restrict__ DT, const float4* __restrict__ colc,
                                                     const int2* __restrict__ band, int warm, float* __restrict__ Yg,
                                                     float* __restrict__ V, float* __restrict__ U,
                                                     float* __restrict__ A, float* __restrict__ Wst,
                                                     int* __restrict__ done, int* __restrict__ status,
                                                     int* __restrict__ iters, float* __restrict__ ew_prev,
                                                     float* __restrict__ ew_best, int* __restrict__ stall,
                                                     int* __restrict__ bad) {
  const int q = blockIdx.x;
  const RgSpec sp = spec[q];
  const int n = sp.n, k = sp.k, np = sp.np;
  __shared__ double ssum[RG_THREADS];
  __shared__ float w[RG_MAX_K];
  __shared__ int2 bnd[RG_MAX_K];
  extern __shared__ float a_s[];
  double acc = 0.0;
  int badl = 0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    const size_t o = (size_t)sp.st + i;
    float y = 0.f, v = 0.f;
    if (i < n) {
      y = Y[sp.yin + i];
      if (!(y >= 0.f) || !isfinite(y)) badl = 1;
      acc += (double)y;
      v = warm ? expf(logVin[sp.yin + i]) : 1.f;
    }
    Yg[o] = y;
    V[o] = v;
    U[o] = 0.f;
  }
  if (badl) bad[0] = 1;
  ssum[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) ssum[threadIdx.x] += ssum[threadIdx.x + s];
    __syncthreads();
  }
  const double mass = ssum[0];
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    const float wj = warm ? Win[sp.win + j] : (float)(mass / k * (double)colc[sp.col + j].x);
    w[j] = wj;
    Wst[sp.col + j] = wj;
    bnd[j] = band[sp.col + j];
  }
  __syncthreads();
  rg_dict_apply(DT + sp.dt, bnd, w, n, k, a_s);
  __syncthreads();
  for (int i = threadIdx.x; i < np; i += blockDim.x) A[(size_t)sp.st + i] = i < n ? fmaxf(a_s[i], 0.f) : 0.f;
  if (threadIdx.x == 0) {
    done[q] = 0;
    status[q] = 0;
    iters[q] = 0;
    ew_prev[q] = 0.f;
    ew_best[q] = INFINITY;
    stall[q] = 0;
  }
}

// Weight step of one outer iteration for one spectrum (one workgroup each), at
// the s = K v of this iteration:
//   repeat `inner` times:  r_i = log(s_i / a_i)   (0 where a_i = 0)
//                          c_j = sum_i D_ij r_i;  w_j <- MM step (Table 2 / Appendix A)
//                          a = D w
//   u = a / s.
// Every repetition is one majorize-minimize step on the same ProxP problem, so
// the fixed point is that of the single step; more steps move w further per
// kernel product.  Frozen spectra keep their state.  A spectrum whose weights
// the Newton prox updates (dp >= 0 and *it_dev > newton_after) takes no MM
// step here: only a = D w and u = a / s at its new weights.
__global__ __launch_bounds__(RG_WS_THREADS) void rg_weight_step(const RgSpec* __restrict__ spec,
                                                            const float* __restrict__ DT,
                                                            const float4* __restrict__ colc,
                                                            const int2* __restrict__ band, int pen, int inner,
                                                            const float* __restrict__ S, float* __restrict__ A,
                                                            float* __restrict__ U, float* __restrict__ Wst,
                                                            const int* __restrict__ done,
                                                            const int* __restrict__ nband,
                                                            unsigned long long* __restrict__ work,
                                                            const int* __restrict__ it_dev, int newton_after) {
  const int q = blockIdx.x;
  if (done[q]) return;
  const RgSpec sp = spec[q];
  if (sp.dp >= 0 && newton_after >= 0 && it_dev[0] > newton_after) inner = 0;
  if (work && threadIdx.x == 0)  // algorithmic bytes: s, a in; a, u out; the band of D once; w in and out
    atomicAdd(work, 4ull * (4ull * sp.n + (unsigned long long)nband[q] + 2ull * sp.k));
  const int n = sp.n, k = sp.k, np = sp.np;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
  extern __shared__ float sm[];
  float* s_s = sm;
  float* a_s = sm + np;
  float* r_s = sm + 2 * np;
  __shared__ float w[RG_MAX_K];
  __shared__ float4 cc[RG_MAX_K];
  __shared__ int2 bnd[RG_MAX_K];
  const float* DTb = DT + sp.dt;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    s_s[i] = S[(size_t)sp.st + i];
    a_s[i] = A[(size_t)sp.st + i];
  }
  for (int j = threadIdx.x; j < k; j += blockDim.x) {
    w[j] = Wst[sp.col + j];
    cc[j] = colc[sp.col + j];
    bnd[j] = band[sp.col + j];
  }
  __syncthreads();
  if (inner == 0) {  // weights from the Newton prox: a = D w
    __syncthreads();
    rg_dict_apply(DTb, bnd, w, n, k, a_s);
    __syncthreads();
  }
  for (int t = 0; t < inner; ++t) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
      const float a = a_s[i];
      r_s[i] = a > 0.f ? fminf(fmaxf(logf(s_s[i] / a), -OTLM_R_CLAMP), OTLM_R_CLAMP) : 0.f;
    }
    __syncthreads();
    for (int j = wave; j < k; j += nwaves) {
      const int2 bj = bnd[j];
      const float* col = DTb + (size_t)j * n;
      // the band in 64-bin chunks, 8 unconditional loads in flight (clamped
      // into the column; bins past the band read exact zeros, bins past the
      // last get r = 0)
      float acc[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) acc[q] = 0.f;
      for (int i0 = bj.x; i0 < bj.y; i0 += 512) {
        float d[8], rv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int i = i0 + 64 * q + lane;
          const int ic = min(i, n - 1);
          d[q] = col[ic];
          rv[q] = r_s[ic] * (float)(i < n);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) acc[q] = fmaf(d[q], rv[q], acc[q]);
      }
      const float c = rg_wave_sum(((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7])));
      if (lane == 0) {
        const float4 cj = cc[j];
        const float wold = w[j];
        const float nu = logf(wold) + c * cj.x;
        float wn;
        if (pen == PEN_NONE) wn = expf(nu);
        else if (pen == PEN_L1) wn = expf(nu - cj.y);
        else wn = wright_omega<float>(nu - cj.y + cj.w) / cj.z;
        w[j] = wn;
      }
    }
    __syncthreads();
    rg_dict_apply(DTb, bnd, w, n, k, a_s);
    __syncthreads();
  }
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    float a = 0.f, u = 0.f;
    if (i < n) {
      a = fmaxf(a_s[i], 0.f);
      u = a > 0.f ? a / s_s[i] : 0.f;
    }
    A[(size_t)sp.st + i] = a;
    U[(size_t)sp.st + i] = u;
  }
  for (int j = threadIdx.x; j < k; j += blockDim.x) Wst[sp.col + j] = w[j];
}

// Weight change over a check interval for every spectrum of a ragged batch
// (the packed counterpart of interval_change): max_j |w_j - w^snap_j| and
// max_j |w_j|, then w^snap = w; init = 1 only takes the snapshot.  One wave
// per spectrum.
__global__ __launch_bounds__(256) void rg_interval_change(const RgSpec* __restrict__ spec, int B,
                                                          const float* __restrict__ Wst, float* __restrict__ snap,
                                                          int init, float* __restrict__ pwn,
                                                          float* __restrict__ pwd) {
  const int q = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (q >= B) return;
  const long long col = spec[q].col;
  const int k = spec[q].k;
  double dw = 0.0, wm = 0.0;
  for (int j = lane; j < k; j += 64) {
    const float w = Wst[col + j];
    dw = nan_max(dw, fabs((double)w - (double)snap[col + j]));
    wm = nan_max(wm, fabs((double)w));
    snap[col + j] = w;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    dw = nan_max(dw, __shfl_xor(dw, off, 64));
    wm = nan_max(wm, __shfl_xor(wm, off, 64));
  }
  if (lane == 0 && !init) {
    pwn[q] = (float)dw;
    pwd[q] = (float)wm;
  }
}

// Static description of the groups for the active-row compaction.
struct RgGroups {
  int ngroups;
  int row0[GEMM_MAX_GROUPS];  // first spectrum of the group (solve order)
  int rows[GEMM_MAX_GROUPS];  // spectra in the group
  int np[GEMM_MAX_GROUPS];    // row stride = GEMM N
};

// Active-row lists of the grouped products, rebuilt after every convergence
// test: for group g the rows (group-relative, ascending) of the spectra not
// yet stopped go to rows[row0_g ...], their count to act->nact[g], and the
// grid offsets of the group's BM x BN tiles to act->tile0.  Stable wave-ballot
// compaction in chunks of 1024 rows.  One workgroup of 1024 threads.
__global__ __launch_bounds__(1024) void rg_compact(const int* __restrict__ done, RgGroups gi, int bm, int bn,
                                                  GemmActive* __restrict__ act, int* __restrict__ rows) {
  __shared__ int wsum[16];
  __shared__ int nact_s[GEMM_MAX_GROUPS];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int g = 0; g < gi.ngroups; ++g) {
    int base = 0;
    for (int c0 = 0; c0 < gi.rows[g]; c0 += 1024) {
      const int r = c0 + tid;
      const bool on = r < gi.rows[g] && !done[gi.row0[g] + r];
      const unsigned long long m = __ballot(on);
      const int before = __popcll(m & ((1ull << lane) - 1ull));
      if (lane == 0) wsum[wave] = __popcll(m);
      __syncthreads();
      int off = 0, tot = 0;
      for (int w = 0; w < 16; ++w) {
        off += w < wave ? wsum[w] : 0;
        tot += wsum[w];
      }
      if (on) rows[gi.row0[g] + base + off + before] = r;
      base += tot;
      __syncthreads();
    }
    if (tid == 0) nact_s[g] = base;
  }
  __syncthreads();
  if (tid == 0) {
    int t = 0;
    for (int g = 0; g < GEMM_MAX_GROUPS; ++g) {
      act->tile0[g] = t;
      const bool used = g < gi.ngroups;
      const int na = used ? nact_s[g] : 0;
      act->nact[g] = na;
      act->row0[g] = used ? gi.row0[g] : 0;
      if (used) t += ((na + bm - 1) / bm) * ((gi.np[g] + bn - 1) / bn);
    }
    act->tile0[GEMM_MAX_GROUPS] = t;
  }
}

// Iteration counter of a captured chunk: the convergence kernel reads it to
// record the iteration at which each spectrum stopped.
__global__ void rg_advance(int* __restrict__ it, int c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) it[0] += c;
}

// Outputs in input order: packed w, log u, log v; iterations and status.
__global__ __launch_bounds__(RG_THREADS) void rg_write_outputs(const RgSpec* __restrict__ spec,
                                                              const float* __restrict__ Wst,
                                                              const float* __restrict__ U,
                                                              const float* __restrict__ V,
                                                              const int* __restrict__ done,
                                                              const int* __restrict__ st,
                                                              const int* __restrict__ it_in, int last,
                                                              float* __restrict__ W, float* __restrict__ logU,
                                                              float* __restrict__ logV, int* __restrict__ iters,
                                                              int* __restrict__ status) {
  const int q = blockIdx.x;
  const RgSpec sp = spec[q];
  for (int j = threadIdx.x; j < sp.k; j += blockDim.x) W[sp.win + j] = Wst[sp.col + j];
  for (int i = threadIdx.x; i < sp.n; i += blockDim.x) {
    if (logU) logU[sp.yin + i] = logf(U[(size_t)sp.st + i]);
    logV[sp.yin + i] = logf(V[(size_t)sp.st + i]);
  }
  if (threadIdx.x == 0) {
    if (iters) iters[sp.b] = done[q] ? it_in[q] : last;
    if (status) status[sp.b] = done[q] ? st[q] : 2;
  }
}
