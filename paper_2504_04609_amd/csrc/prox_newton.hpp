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
// weight with the most negative gradient once the free gradient is small next
// to it.  Weights that are exactly 0 are the active set, so the state carried
// between outer iterations is just W.
//
// One workgroup (256 threads, 4 wave64s) per spectrum, everything in FP64 (the
// Hessian of an overlapping Gaussian dictionary has condition numbers near
// 1e12).  LDS holds s and two pairs (a = D w, log(a/s)) for the n bins, the
// current point's and the line search's, and the 64 x 64 Hessian:
// (4 sizeof(a) + sizeof(s)) n + 37 KB, 78 KB at n = 1024 (two workgroups per CU).
// An accepted trial point keeps the a, log(a/s) and objective value the line
// search computed, so a Newton iteration after a line-search step starts
// without another pass over the dictionary.
// The dictionary is streamed from L2 with many independent loads in flight
// (D^T for the bin sweeps, D for the column sweeps).  The 64-wide Hessian is
// built on the FP64 matrix cores (its lower-triangle 16 x 16 blocks, each wave
// over a quarter of the bins, every dictionary entry read once); the Cholesky
// factorisation runs by 16 x 16 tiles and the two triangular solves in one wave,
// one row per lane.
//
// Factor reuse: the Hessian depends on the weights only (through a = D w), not
// on s, so a Cholesky factor stays accurate while w barely moves, as it does
// between late outer iterations.  Each spectrum keeps its last factor, the
// weights it was built at and its free set in global memory; a Newton
// iteration reuses it (a chord step, still safeguarded by the ratio test and
// Armijo) when the free set is the same and max|w - w_H| <= reuse_tol max|w_H|
// and the previous step, if it reused the factor, at least halved the free-set
// gradient; otherwise it builds and factors the Hessian anew.
#pragma once
#include <hip/hip_runtime.h>
#include <type_traits>
#include "gemm_nt_f64.hpp"
#include "solver_kernels.hpp"

constexpr int PN_THREADS = 256;
constexpr int PN_K = 64;    // largest dictionary handled by this kernel
constexpr int PN_HLD = PN_K + 1;
constexpr int PN_MAXB = 4;  // bins per thread in bin sweeps of a batch: n <= 1024
constexpr int PN_MAXB_RAGGED = 8;  // the same for ragged batches: n <= 2048

// Per-spectrum layout of a ragged batch (ProxNewtonArgs::rg; null for a batch
// that shares one dictionary and the strides of the arguments).
struct PnSpec {
  long long s_off;   // start of s_b in S
  long long w_off;   // start of w_b in W (packed, k_b entries)
  long long dp_off;  // start of D_b in Dp: [n_b, 64] row-major, columns >= k_b zero
  long long dt_off;  // start of D_b^T in DTp: [k_b, n_b]
  int n, k;
};

template <class TS, class TW>
struct ProxNewtonArgs {
  const TS* S;         // [B, ld_s]  s = K v
  TW* W;               // [B, ld_w]  weights (in: start, out: prox)
  const float* Dp;     // [np, ld_d] dictionary, zero padded
  const float* DTp;    // [kp, ld_dt] its transpose (coalesced column sweeps)
  const float4* colc;  // per column {1/x_j, ...}
  const int* done;
  const int* mm_until;  // spectra with it <= mm_until[b] take the MM step instead (null: none)
  int it;
  int* nit;
  int* nfac;                   // Hessian factorisations, accumulated per spectrum
  int* nent;                   // free-set Hessian entries m (m + 1) / 2 built, accumulated per spectrum (null: none)
  unsigned long long* flops;   // algorithmic flops of all spectra, accumulated (null: none): per Newton iteration
                               // 6 n k, per free-set Hessian entry built 2 n
  void* Lg;                    // last Cholesky factor per spectrum, lg_stride bytes each (null: no reuse)
  size_t lg_stride;
  double* wH;                  // [B][128] weights at that factorisation
  unsigned long long* maskH;   // [B][2] its active set (bit j: w_j pinned at 0)
  int* validH;                 // [B] 1 when the stored factor may be used
  double reuse_tol;
  const PnSpec* rg;            // ragged layout (null: batch layout)
  const int2* band;            // per dictionary column its rows with nonzero entries, [lo, hi) (null: unknown;
                               // batch: [k], ragged: indexed like W); orders the free weights of the 64-wide prox
  const int* it_dev;           // ragged: the iteration counter ...
  int newton_after;            // ... spectra take the prox once it exceeds this
  int ld_s, ld_w, ld_d, ld_dt, n, k, pen, max_newton;
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

// Wave-local synchronisation for LDS traffic among the lanes of one wave.
__device__ __forceinline__ void pn_wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Buffer resource over nfloats floats at p (raw, unswizzled; word 3 as CDNA
// expects).  Loads through it take one 32-bit lane offset and a wave-uniform
// offset instead of a 64-bit address per lane, so many can be in flight.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t pn_rsrc(const float* p, long long nfloats) {
  const long long bytes = nfloats * 4;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(p), (short)0,
                                           (int)(bytes < 0x7fffffffLL ? bytes : 0x7fffffffLL), 0x00020000);
}
// p[(voff + soff) / 4] with voff per lane and soff wave-uniform (bytes); every
// caller keeps voff + soff inside the buffer.
__device__ __forceinline__ float pn_ld(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

// Value of v in lane `src` (wave-uniform) for every lane of the wave.
__device__ __forceinline__ double pn_readlane(double v, int src) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Right-looking Cholesky of the 16 columns C0 .. C0 + 15 of the (already
// updated) lower triangle of a 64 x 64 matrix H in LDS, in one wave: lane r
// holds row r's entries of those columns, column entries reach the other
// lanes by v_readlane, and the rows below the block are eliminated with it
// (the panel of L under the diagonal block).  Each finished column is stored
// at once; lanes above the diagonal store 0 into the unused upper triangle,
// which keeps the code free of divergent branches.
template <int C0>
__device__ __forceinline__ void pn_chol_panel(double* H, int HLD, int lane) {
  double h[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) h[j] = C0 + j <= lane ? H[lane * HLD + C0 + j] : 0.0;
#pragma unroll
  for (int c = 0; c < 16; ++c) {
    const double hcc = fmax(pn_readlane(h[c], C0 + c), 1e-300);
    const double inv = rsqrt(hcc);  // 1 / L_cc
    const double lrc = lane > C0 + c ? h[c] * inv : 0.0;
    h[c] = lane == C0 + c ? hcc * inv : lrc;
#pragma unroll
    for (int q = c + 1; q < 16; ++q) h[q] -= lrc * pn_readlane(lrc, C0 + q);
    H[lane * HLD + C0 + c] = h[c];
  }
}

// Schur update of the trailing lower triangle of that matrix after the panel
// at columns R0 - 16 .. R0 - 1:  H[i][j] -= sum_c L[i][c] L[j][c]  for
// R0 <= j <= i < R0 + 16 nb (nb <= (64 - R0) / 16 block rows, wave-uniform),
// on the FP64 matrix cores (16 x 16 blocks, 4 columns of the panel per
// step), in one wave.
template <int R0>
__device__ __forceinline__ void pn_chol_schur(double* H, int HLD, int lane, int nb) {
  constexpr int NB = (64 - R0) / 16, NBLK = NB * (NB + 1) / 2, C0 = R0 - 16;
  const int c16 = lane & 15, ks = lane >> 4;
  nb = __builtin_amdgcn_readfirstlane(nb);
  f64x4 acc[NBLK];
#pragma unroll
  for (int x = 0; x < NBLK; ++x) acc[x] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int c0 = 0; c0 < 16; c0 += 4) {
    double xv[NB];  // L[R0 + 16 bi + lane%16][C0 + c0 + lane/16]: A and B operands alike
#pragma unroll
    for (int bi = 0; bi < NB; ++bi) xv[bi] = bi < nb ? H[(R0 + 16 * bi + c16) * HLD + C0 + c0 + ks] : 0.0;
    int x = 0;
#pragma unroll
    for (int bi = 0; bi < NB; ++bi)
#pragma unroll
      for (int bj = 0; bj <= bi; ++bj, ++x)
        if (bi < nb) acc[x] = __builtin_amdgcn_mfma_f64_16x16x4f64(xv[bi], xv[bj], acc[x], 0, 0, 0);
  }
  int x = 0;
#pragma unroll
  for (int bi = 0; bi < NB; ++bi)
#pragma unroll
    for (int bj = 0; bj <= bi; ++bj, ++x)
      if (bi < nb)
#pragma unroll
        for (int r = 0; r < 4; ++r) H[(R0 + 16 * bi + ks + 4 * r) * HLD + R0 + 16 * bj + c16] -= acc[x][r];
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
// (bins with a = 0 give s_i); stores a and l = log(max(a, tiny) / s), the
// factor of the gradient.  Each thread owns up to MAXB bins and keeps their
// sums independent so the D^T loads overlap.
template <int MAXB, class TS, class TW, class TL>
__device__ __forceinline__ double pn_eval(const ProxNewtonArgs<TS, TW>& p, const float* DTp, int ld_dt, int n, int k,
                          const double* w, const TS* s, TL* a, TL* l, double tiny, double* red) {
  double ai[MAXB];
  int vo[MAXB];  // byte offsets of this thread's bins in a row of D^T, clamped into the row
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    ai[q] = 0.0;
    vo[q] = min((int)threadIdx.x + q * PN_THREADS, n - 1) * 4;
  }
  const __amdgpu_buffer_rsrc_t rs = pn_rsrc(DTp, (long long)k * ld_dt);
  constexpr int CW = MAXB <= 4 ? 16 : 8;  // columns per step: CW * MAXB independent loads in flight
  int j = 0;
  for (; j + CW <= k; j += CW) {
    float dv[CW][MAXB];
#pragma unroll
    for (int u = 0; u < CW; ++u)
#pragma unroll
      for (int q = 0; q < MAXB; ++q) dv[u][q] = pn_ld(rs, vo[q], (j + u) * ld_dt * 4);
#pragma unroll
    for (int u = 0; u < CW; ++u) {
      const double wj = w[j + u];
#pragma unroll
      for (int q = 0; q < MAXB; ++q) ai[q] += (double)dv[u][q] * wj;
    }
  }
  for (; j < k; ++j) {
    const double wj = w[j];
#pragma unroll
    for (int q = 0; q < MAXB; ++q) ai[q] += (double)pn_ld(rs, vo[q], j * ld_dt * 4) * wj;
  }
  double acc = 0.0;
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int i = threadIdx.x + q * PN_THREADS;
    if (i < n) {
      const double si = (double)s[i];
      const double lg = log(fmax(ai[q], tiny) / si);
      a[i] = (TL)ai[q];
      l[i] = (TL)lg;
      acc += (ai[q] > 0.0 ? ai[q] * lg : 0.0) - ai[q] + si;
    }
  }
  acc *= p.eps;
  if ((int)threadIdx.x < k) acc += pn_pen(p.pen, w[threadIdx.x], p.alpha, p.beta);
  return pn_block_sum(acc, red);
}

// Template parameters: MAXB bins per thread (n <= 256 MAXB); TL storage of a
// and of log(a/s) or 1/a in LDS (double for a batch, float for the n <= 2048
// of a ragged batch); KMAX the dictionary width the Hessian is laid out for
// (64, or 128 for ragged spectra with 64 < k <= 128, where the FP64 Hessian
// and n = 2048 would not fit the 160 KB of LDS); TH the Hessian and Cholesky
// type (double; float for KMAX = 128: FP32-state ragged solves whose ridge
// penalty bounds the Hessian's condition number).
template <class TS, class TW, class TL, int MAXB, int KMAX = PN_K, class TH = double>
__global__ __launch_bounds__(PN_THREADS, 2) void prox_newton_kernel(ProxNewtonArgs<TS, TW> p) {
  static_assert(KMAX == 64 || KMAX == 128, "dictionary width");
  static_assert(KMAX == 128 || sizeof(TH) == 8, "the 64-wide Hessian is built in FP64");
  constexpr int HLD = KMAX + 1, RPL = KMAX / 64;  // Hessian row stride; rows per lane in the solves
  const int b = blockIdx.x;
  if (p.done[b] || (p.mm_until && p.it <= p.mm_until[b])) return;
  int n = p.n, k = p.k, ld_d = p.ld_d, ld_dt = p.ld_dt, ld_w = p.ld_w;
  const float* Dp = p.Dp;
  const float* DTp = p.DTp;
  const int2* band = p.band;
  const TS* srow = p.S + (size_t)b * p.ld_s;
  TW* wrow = p.W + (size_t)b * p.ld_w;
  if (p.rg) {  // ragged: this spectrum's own sizes and arrays, once it is past its MM iterations
    const PnSpec sp = p.rg[b];
    if (sp.dp_off < 0 || p.it_dev[0] <= p.newton_after) return;
    if ((KMAX == 64) != (sp.k <= 64)) return;  // the other width's kernel takes it
    n = sp.n;
    k = sp.k;
    ld_d = KMAX;
    ld_dt = sp.n;
    ld_w = sp.k;
    Dp = p.Dp + sp.dp_off;
    DTp = p.DTp + sp.dt_off;
    srow = p.S + sp.s_off;
    wrow = p.W + sp.w_off;
    if (band) band += sp.w_off;
  }
  extern __shared__ double smem[];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  TH* H = reinterpret_cast<TH*>(smem);                     // [KMAX][KMAX + 1]
  double* w = reinterpret_cast<double*>(H + KMAX * HLD);   // [KMAX]
  double* wt = w + KMAX;                                   // [KMAX]
  double* g = wt + KMAX;                                   // [KMAX]
  double* d = g + KMAX;                                    // [KMAX]
  double* gp = d + KMAX;                                   // [4][KMAX] gradient partials
  double* red = gp + 4 * KMAX;                             // [8]
  // two (a = D w, l = log(a/s)) pairs: the current point's and the line
  // search's, swapped when a trial point is accepted; the Hessian build takes
  // the trial pair's l for 1/a
  TL* a = reinterpret_cast<TL*>(red + 8);                  // [n]
  TL* l = a + n;                                           // [n]
  TL* at = l + n;                                          // [n]
  TL* lt = at + n;                                         // [n]
  TS* s = reinterpret_cast<TS*>(lt + n);                   // [n]
  __shared__ int act[KMAX];
  __shared__ int perm[KMAX];  // 64-wide: the free weights in column order (compact positions)
  __shared__ int ord_s[KMAX]; // 64-wide: column order, by the midpoint of the nonzero rows (ties: index)
  __shared__ int2 prng_s[4];  // 64-wide: per panel of 16 compact positions, the rows [lo, hi) of its nonzeros
  __shared__ int2 grng_s[4];  // 64-wide: the same per group of 16 positions of the column order
  __shared__ int cmp_s[2];    // [0] number of free weights m, [1] compact position of a released weight
  __shared__ double rt_s[2];  // slope g.d and ratio-test step of this iteration
  __shared__ int ctl[4];
  __shared__ double wHs[KMAX];             // weights of the factor held in H
  __shared__ unsigned long long hmask_s[RPL];  // its active set
  __shared__ int hstate[2];               // [0] H holds a usable factor, [1] it was rebuilt here
  __shared__ double hrel_diag_s;          // Hessian diagonal entry of a released weight
  __shared__ int force_rebuild;           // the last reused factor gave no descent
  double kkt_prev = 0.0;                  // (wave 0) the free gradient of the previous iteration
  int last_reused = 0;                    // (wave 0) the previous step used a reused factor
  int nfac = 0;
  int nent = 0;  // (thread 0) lower-triangle entries of the free-set Hessians built

  for (int i = tid; i < n; i += PN_THREADS) s[i] = srow[i];
  if constexpr (KMAX == 64) {
    // Columns ordered by where their nonzero rows sit: a panel of 16 neighbours
    // then covers few bins, so the Hessian skips the steps where a panel
    // holds only zeros and the gradient sweeps a group's rows only (rank
    // sort, lane j ranks column j; then the rows of each group of 16)
    if (wave == 0) {
      const int2 bj = lane < k && band ? band[lane] : make_int2(0, n);
      const int key = lane < k ? (band ? bj.x + bj.y : lane) : 0x7fffffff;
      int rank = 0;
#pragma unroll 8
      for (int i = 0; i < 64; ++i) {
        const int ki = __builtin_amdgcn_readlane(key, i);
        rank += (ki < key || (ki == key && i < lane)) ? 1 : 0;
      }
      ord_s[rank] = lane;
#pragma unroll
      for (int gq = 0; gq < 4; ++gq) {
        int lo = (lane < k && (rank >> 4) == gq) ? bj.x : 0x7fffffff;
        int hi = (lane < k && (rank >> 4) == gq) ? bj.y : 0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          lo = min(lo, __shfl_xor(lo, off, 64));
          hi = max(hi, __shfl_xor(hi, off, 64));
        }
        if (lane == 0) grng_s[gq] = make_int2(lo, hi);
      }
    }
  }
  for (int j = tid; j < KMAX; j += PN_THREADS) {
    const double wj = j < k ? (double)wrow[j] : 0.0;
    w[j] = wj > 0.0 ? wj : 0.0;
    act[j] = (j < k && wj > 0.0) ? 0 : 1;   // padded columns stay active at 0
    g[j] = 0.0;                             // (the gradient sweep writes j < k only)
  }
  const bool reuse_on = p.Lg && p.reuse_tol > 0.0;
  TH* Lb = reuse_on ? reinterpret_cast<TH*>(reinterpret_cast<char*>(p.Lg) + (size_t)b * p.lg_stride) : nullptr;
  if (tid == 0) {
    hstate[0] = reuse_on && p.validH[b];
    hstate[1] = 0;
    force_rebuild = 0;
    for (int m = 0; m < RPL; ++m) hmask_s[m] = reuse_on ? p.maskH[(size_t)b * 2 + m] : 0ull;
  }
  __syncthreads();
  if (hstate[0]) {  // the factor of the previous launch
    for (int e = tid; e < KMAX * KMAX; e += PN_THREADS) H[(e / KMAX) * HLD + (e % KMAX)] = Lb[e];
    if (tid < KMAX) wHs[tid] = p.wH[(size_t)b * 128 + tid];
  }
  __syncthreads();
  const double tiny = sizeof(TL) == 4 ? 1e-30 : 1e-300;
  const TH tinyh = sizeof(TH) == 4 ? (TH)1e-30 : (TH)1e-300;
  const double gscale = fmax(fmax(p.alpha, p.eps), 1e-300) * p.gtol;
  const double hpen = p.pen == PEN_L2SQ ? p.alpha : (p.pen == PEN_EN ? p.beta : 0.0);

  int it = 0;
  double f = 0.0;          // V(w); with a and l valid for w when have_f
  bool have_f = false;
  for (; it < p.max_newton; ++it) {
    if (!have_f) f = pn_eval<MAXB>(p, DTp, ld_dt, n, k, w, s, a, l, tiny, red);  // block_sum synchronises
    have_f = true;
    // ---- gradient: g_j = alpha R'(w_j) + eps sum_i D_ij log(a_i / s_i)
    // Column groups of 16 (G = ceil(k/16), at most 4 per pass; a 128-wide
    // dictionary takes two passes), lanes over bins: coalesced rows of D^T and
    // each l_i read once; with G <= 2 the P = 4/G waves of a group split the
    // 64-bin blocks and their partial sums meet in LDS.  The 16 column sums of
    // a wave leave the 64 lanes by a halving butterfly (17 shuffles), lane l
    // ending with column l / 4.
    {
      const __amdgpu_buffer_rsrc_t rs = pn_rsrc(DTp, (long long)k * ld_dt);
      const int G = min((k + 15) >> 4, 4);
      const int P = G == 1 ? 4 : (G == 2 ? 2 : 1);
      const int wv = __builtin_amdgcn_readfirstlane(wave);
      const int cg = wv % G, bp = wv / G;
#pragma unroll
      for (int cb0 = 0; cb0 < KMAX; cb0 += 64) {
        const int cb = cb0 + 16 * cg;
        if (bp < P && cb < k) {
          // positions cb + jj of the column order (64-wide: ord_s, else the
          // index) and the 64-bin blocks holding the group's nonzero rows
          int roff[16];
#pragma unroll
          for (int jj = 0; jj < 16; ++jj) {
            const int x = min(cb + jj, k - 1);
            roff[jj] = __builtin_amdgcn_readfirstlane((KMAX == 64 ? ord_s[x] : x) * ld_dt * 4);
          }
          int b_lo = 0, b_hi = (n + 63) >> 6;
          if constexpr (KMAX == 64) {
            const int2 gr = grng_s[cg];
            b_lo = __builtin_amdgcn_readfirstlane(gr.y > gr.x ? gr.x >> 6 : 0);
            b_hi = __builtin_amdgcn_readfirstlane(gr.y > gr.x ? (gr.y + 63) >> 6 : 0);
          }
          double acc[16];  // positions cb + jj (those past k read position k - 1 and are dropped)
#pragma unroll
          for (int jj = 0; jj < 16; ++jj) acc[jj] = 0.0;
          for (int blk = b_lo + 2 * bp; blk < b_hi; blk += 2 * P) {  // two 64-bin blocks: 32 loads in flight
            double li[2];
            float dv[2][16];
#pragma unroll
            for (int sb = 0; sb < 2; ++sb) {
              const int i = 64 * (blk + sb) + lane;
              const double lv = (double)l[min(i, n - 1)];  // unconditional (clamped) read, then masked
              li[sb] = (i < n && blk + sb < b_hi) ? lv : 0.0;
              const int vo = min(i, n - 1) * 4;
#pragma unroll
              for (int jj = 0; jj < 16; ++jj) dv[sb][jj] = pn_ld(rs, vo, roff[jj]);
            }
#pragma unroll
            for (int sb = 0; sb < 2; ++sb)
#pragma unroll
              for (int jj = 0; jj < 16; ++jj) acc[jj] += (double)dv[sb][jj] * li[sb];
          }
#pragma unroll
          for (int o = 32, v = 16; o >= 4; o >>= 1, v >>= 1) {
            const bool up = (lane & o) != 0;  // keeps the upper half of the values
#pragma unroll
            for (int h = 0; h < v / 2; ++h) {
              const double send = up ? acc[h] : acc[h + v / 2];
              const double keep = up ? acc[h + v / 2] : acc[h];
              acc[h] = keep + __shfl_xor(send, o, 64);
            }
          }
          acc[0] += __shfl_xor(acc[0], 2, 64);
          acc[0] += __shfl_xor(acc[0], 1, 64);
          const int xq = cb + (lane >> 2);
          const int j = KMAX == 64 ? ord_s[xq & (KMAX - 1)] : xq;  // (positions >= k keep their index)
          if ((lane & 3) == 0 && xq < KMAX) {
            if (P == 1) g[j] = j < k ? pn_pen_grad(p.pen, w[j], p.alpha, p.beta) + p.eps * acc[0] : 0.0;
            else gp[bp * KMAX + j] = acc[0];
          }
        }
      }
      if (P > 1) {  // k <= 32: sum the bin parts in part order
        __syncthreads();
        if (tid < KMAX) {
          double gj = 0.0;
          for (int q = 0; q < P; ++q) gj += gp[q * KMAX + tid];
          g[tid] = tid < k ? pn_pen_grad(p.pen, w[tid], p.alpha, p.beta) + p.eps * gj : 0.0;
        }
      }
      __syncthreads();
    }
    // ---- optimality of the free set, release of the most negative active
    // gradient, and whether the factor held in H serves this step: wave 0 by
    // butterfly reductions, so every lane ends with the same values
    if (wave == 0) {
      double kkt = 0.0, gmin = 0.0;
      int jmin = 0x7fffffff;  // (gmin, jmin): the smallest (g_j, j) over active j with g_j < 0
#pragma unroll
      for (int cc = 0; cc < RPL; ++cc) {
        const int j = lane + 64 * cc;
        if (j < k) {
          const double gj = g[j];
          if (!act[j]) {
            kkt = fmax(kkt, fabs(gj));
          } else if (gj < gmin) {
            gmin = gj;
            jmin = j;
          }
        }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        kkt = fmax(kkt, __shfl_xor(kkt, off, 64));
        const double og = __shfl_xor(gmin, off, 64);
        const int oj = __shfl_xor(jmin, off, 64);
        if (og < gmin || (og == gmin && oj < jmin)) {
          gmin = og;
          jmin = oj;
        }
      }
      const bool cand = jmin != 0x7fffffff && gmin < -gscale;
      int stop = 0, rel = -1, next = cand ? jmin : -1;  // next: release candidate if no descent is left
      if (kkt <= gscale && !cand) {
        stop = 1;
      } else if (cand && kkt <= fmax(gscale, 0.1 * fabs(gmin))) {
        rel = jmin;
        next = -1;
      }
      int reuse = 0;
      unsigned long long mask[RPL];
      if (!stop) {
        bool same = true;
#pragma unroll
        for (int cc = 0; cc < RPL; ++cc) {
          const int j = lane + 64 * cc;
          mask[cc] = __ballot(j < k && act[j] && j != rel);
          same = same && mask[cc] == hmask_s[cc];
        }
        // a step on a reused factor that did not halve the free gradient: refactor
        const bool poor = (last_reused && kkt > 0.5 * kkt_prev) || force_rebuild;
        if (hstate[0] && rel < 0 && same && !poor) {
          double dm = 0.0, wm = 0.0;
#pragma unroll
          for (int cc = 0; cc < RPL; ++cc) {
            const int j = lane + 64 * cc;
            if (j < k) {
              dm = fmax(dm, fabs(w[j] - wHs[j]));
              wm = fmax(wm, fabs(wHs[j]));
            }
          }
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) {
            dm = fmax(dm, __shfl_xor(dm, off, 64));
            wm = fmax(wm, __shfl_xor(wm, off, 64));
          }
          reuse = dm <= p.reuse_tol * wm;
        }
        last_reused = reuse;
        kkt_prev = kkt;
      }
      if constexpr (KMAX == 64) {  // compact positions of the free weights (after the release)
        if (!stop) {
          const int oj = ord_s[lane];  // the column at position lane of the order
          const bool fr = lane < k && (!act[oj] || oj == rel);
          const unsigned long long fm = __ballot(fr);
          const int x = __builtin_amdgcn_mbcnt_hi((unsigned)(fm >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)fm, 0u));
          if (fr) perm[x] = oj;
          if (fr && oj == rel) cmp_s[1] = x;
          if (lane == 0) cmp_s[0] = __popcll(fm);
          const int2 bj = (fr && band) ? band[oj] : make_int2(0, n);
#pragma unroll
          for (int pp = 0; pp < 4; ++pp) {
            int lo = (fr && (x >> 4) == pp) ? bj.x : 0x7fffffff, hi = (fr && (x >> 4) == pp) ? bj.y : 0;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
              lo = min(lo, __shfl_xor(lo, off, 64));
              hi = max(hi, __shfl_xor(hi, off, 64));
            }
            if (lane == 0) prng_s[pp] = make_int2(lo, hi);
          }
        }
      }
      if (lane == 0) {
        ctl[0] = stop;
        ctl[1] = rel;
        ctl[2] = next;
        ctl[3] = reuse;
        if (!stop) {
          if (rel >= 0) act[rel] = 0;
          force_rebuild = 0;
          if (!reuse)
            for (int m = 0; m < RPL; ++m) hmask_s[m] = mask[m];
        }
      }
    }
    __syncthreads();
    if (ctl[0]) break;
    const int released = ctl[1];
    if (!ctl[3]) {
      // ---- Hessian on the free set: H = eps D^T diag(1/a) D + hpen I
      TL* ra = lt;  // 1 / a_i (the trial buffer is free until the line search)
      for (int i = tid; i < n; i += PN_THREADS) ra[i] = (TL)(1.0 / fmax((double)a[i], tiny));
      __syncthreads();
      if constexpr (KMAX == 64 && sizeof(TH) == 8) {
        // FP64 matrix cores on the free weights only, in compact order: with m
        // free weights and NP = ceil(m / 16) panels, the NP (NP + 1) / 2 lower
        // 16 x 16 blocks (p >= q).  In a 4-bin step st lane l supplies bin
        // 4 st + l/16 and the column of the free weight at compact position
        // 16 p + l%16 of every panel p, as the A operand (scaled by 1 / a_i)
        // and as the B operand.
        const int m = cmp_s[0];
        const int c16 = lane & 15, ks = lane >> 4;
        const __amdgpu_buffer_rsrc_t rd = pn_rsrc(Dp, (long long)n * ld_d);
        int colb[4];  // byte offset of this lane's column in each panel (-1: padding)
#pragma unroll
        for (int pp = 0; pp < 4; ++pp) colb[pp] = 16 * pp + c16 < m ? perm[16 * pp + c16] * 4 : -1;
        auto hessian = [&](auto np_c) {
          constexpr int NP = decltype(np_c)::value, NBLK = NP * (NP + 1) / 2;
          f64x4 acc[NBLK];
#pragma unroll
          for (int x = 0; x < NBLK; ++x) acc[x] = f64x4{0.0, 0.0, 0.0, 0.0};
          // Wave w takes the 4-bin steps w, w + 4, ... of the bins where some
          // panel has nonzeros, four steps in flight; in a step a block's
          // matrix-core operation is skipped when either panel holds only zeros
          // there (a wave-uniform test: the skipped terms are exact zeros)
          int lo_all = 0x7fffffff, hi_all = 0;
#pragma unroll
          for (int pp = 0; pp < NP; ++pp) {
            lo_all = min(lo_all, prng_s[pp].x);
            hi_all = max(hi_all, prng_s[pp].y);
          }
          // (no nonzero rows: no steps; the prologue still loads, at clamped bins)
          const bool rows = hi_all > lo_all;
          const int st_lo = rows ? lo_all >> 2 : 0, st_hi = rows ? (hi_all + 3) >> 2 : 0;
          // Loads are unconditional at clamped addresses and their values are
          // used as loaded (a select on them, or a load under a branch, makes
          // the wait counters drain every step): a bin past the last or past
          // the steps' range gets the scale 0, which zeroes its terms through
          // the A operand, and padding positions (a clamped column) only reach
          // rows and columns >= m, which the last pass below overwrites
          auto load_step = [&](int st, float (&v)[NP], double& sc) __attribute__((always_inline)) {
            const int i = 4 * st + ks;
            const int ro = min(i, n - 1) * ld_d * 4;
#pragma unroll
            for (int pp = 0; pp < NP; ++pp) v[pp] = pn_ld(rd, ro + max(colb[pp], 0), 0);
            // (a product with a 0/1 mask, not a select, keeps the read unconditional)
            sc = (double)ra[min(i, n - 1)] * (double)(st < st_hi && i < n);
          };
          auto mfma_step = [&](const float (&v)[NP], double sc) __attribute__((always_inline)) {
            double bq[NP], ap[NP];
            bool nz[NP];  // the scaled panel has a nonzero entry (wave-uniform)
#pragma unroll
            for (int pp = 0; pp < NP; ++pp) {
              bq[pp] = (double)v[pp];
              ap[pp] = bq[pp] * sc;
              nz[pp] = __ballot(ap[pp] != 0.0) != 0ull;
            }
            int x = 0;
#pragma unroll
            for (int pp = 0; pp < NP; ++pp)
#pragma unroll
              for (int qq = 0; qq <= pp; ++qq, ++x)
                if (nz[pp] && nz[qq]) acc[x] = __builtin_amdgcn_mfma_f64_16x16x4f64(ap[pp], bq[qq], acc[x], 0, 0, 0);
          };
          // double buffer of two steps each: each half issues the other
          // buffer's loads first, so the buffer consumed next is the oldest one
          // in flight on every path into the loop (a loop whose first use is
          // the newest load makes the compiler drain the wait counter there)
          float v0[NP], v1[NP], v2[NP], v3[NP];
          double s0, s1, s2, s3;
          int st = st_lo + __builtin_amdgcn_readfirstlane(wave);
          load_step(st, v0, s0);
          load_step(st + 4, v1, s1);
          for (; st < st_hi; st += 16) {
            load_step(st + 8, v2, s2);
            load_step(st + 12, v3, s3);
            mfma_step(v0, s0);
            mfma_step(v1, s1);
            load_step(st + 16, v0, s0);
            load_step(st + 20, v1, s1);
            mfma_step(v2, s2);
            mfma_step(v3, s3);
          }
          // sum the four waves' partial blocks into H in wave order (lane l,
          // register r holds block row l/16 + 4 r, block column l%16); the last
          // pass scales, adds the penalty curvature and makes the padding
          // positions m .. 16 NP - 1 identity rows
          for (int src = 0; src < 4; ++src) {
            if (wave == src) {
              int x = 0;
#pragma unroll
              for (int pp = 0; pp < NP; ++pp)
#pragma unroll
                for (int qq = 0; qq <= pp; ++qq, ++x)
#pragma unroll
                  for (int r = 0; r < 4; ++r) {
                    const int row = 16 * pp + ks + 4 * r, col = 16 * qq + c16;
                    TH* h = &H[row * HLD + col];
                    double v = (src == 0 ? 0.0 : (double)*h) + acc[x][r];
                    if (src == 3) {
                      v *= p.eps;
                      if (row >= m || col >= m) v = (row == col) ? 1.0 : 0.0;
                      else if (row == col) v += hpen;
                    }
                    *h = (TH)v;
                  }
            }
            __syncthreads();
          }
        };
        switch ((m + 15) >> 4) {
          case 0:
          case 1: hessian(std::integral_constant<int, 1>{}); break;
          case 2: hessian(std::integral_constant<int, 2>{}); break;
          case 3: hessian(std::integral_constant<int, 3>{}); break;
          default: hessian(std::integral_constant<int, 4>{}); break;
        }
      } else {
        // FP32 matrix cores (v_mfma_f32_32x32x2_f32): the 10 lower 32 x 32 blocks
        // (p >= q) of the 4 x 4 block grid, 2 or 3 per wave over all bins, so no
        // cross-wave sum: wave 0 (0,0) (1,0) (1,1); 1 (2,0) (2,1) (2,2); 2 (3,0)
        // (3,1); 3 (3,2) (3,3).  In a step lane l supplies bin 2 st + l/32 and
        // column 32 p + l%32 of panel p, as the A operand (scaled by 1 / a_i)
        // and as the B operand; lane l, register r of a block hold its row
        // 8 (r/4) + 4 (l/32) + r%4, column l%32.
        const int l32 = lane & 31, kh = lane >> 5;
        const int nst = (n + 1) >> 1;
        const __amdgpu_buffer_rsrc_t rd = pn_rsrc(Dp, (long long)n * ld_d);
        auto run = [&](auto w_c) {
          constexpr int W = decltype(w_c)::value;
          constexpr int NB = W < 2 ? 3 : 2;
          constexpr int BP[4][3] = {{0, 1, 1}, {2, 2, 2}, {3, 3, 0}, {3, 3, 0}};
          constexpr int BQ[4][3] = {{0, 0, 1}, {0, 1, 2}, {0, 1, 0}, {2, 3, 0}};
          typedef float f32x16 __attribute__((ext_vector_type(16)));
          f32x16 acc[NB];
#pragma unroll
          for (int x = 0; x < NB; ++x)
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[x][r] = 0.f;
          // loads unconditional at clamped addresses and used as loaded (a bin
          // past the last gets the scale 0, which zeroes its terms through the
          // A operand): loads under a branch drain the wait counter every step
          auto load_step = [&](int st, float (&v)[4], float& sc) {
            const int i = 2 * st + kh;
            const int ro = (min(i, n - 1) * ld_d + l32) * 4;
#pragma unroll
            for (int pp = 0; pp < 4; ++pp) {
              bool need = false;
#pragma unroll
              for (int x = 0; x < NB; ++x) need = need || BP[W][x] == pp || BQ[W][x] == pp;
              v[pp] = need ? pn_ld(rd, ro, 128 * pp) : 0.f;
            }
            sc = (float)ra[min(i, n - 1)] * (float)(i < n);
          };
          auto mfma_step = [&](const float (&v)[4], float sc) {
#pragma unroll
            for (int x = 0; x < NB; ++x)
              acc[x] = __builtin_amdgcn_mfma_f32_32x32x2f32(v[BP[W][x]] * sc, v[BQ[W][x]], acc[x], 0, 0, 0);
          };
          float v0[4], v1[4], s0, s1;
          load_step(0, v0, s0);
          load_step(1, v1, s1);
          for (int st = 0; st < nst; st += 2) {
            mfma_step(v0, s0);
            load_step(st + 2, v0, s0);
            mfma_step(v1, s1);
            load_step(st + 3, v1, s1);
          }
#pragma unroll
          for (int x = 0; x < NB; ++x)
#pragma unroll
            for (int r = 0; r < 16; ++r)
              H[(32 * BP[W][x] + 8 * (r >> 2) + 4 * kh + (r & 3)) * HLD + 32 * BQ[W][x] + l32] = (TH)acc[x][r];
        };
        switch (__builtin_amdgcn_readfirstlane(wave)) {
          case 0: run(std::integral_constant<int, 0>{}); break;
          case 1: run(std::integral_constant<int, 1>{}); break;
          case 2: run(std::integral_constant<int, 2>{}); break;
          default: run(std::integral_constant<int, 3>{}); break;
        }
        __syncthreads();
      }
      if constexpr (KMAX == 64) {
        // ---- Cholesky H = L L^T of the compact 16 NP x 16 NP matrix (lower
        // triangle in place) in wave 0: 16-column panels in registers, each
        // followed by the Schur update of the trailing lower triangle on the
        // matrix cores.  Rows past 16 NP hold stale values; they are eliminated
        // along (in their own lanes) but never read.
        if (wave == 0) {
          const int np16 = __builtin_amdgcn_readfirstlane(max((cmp_s[0] + 15) >> 4, 1));
          if (lane == 0) hrel_diag_s = released >= 0 ? (double)H[cmp_s[1] * HLD + cmp_s[1]] : 1.0;
          pn_chol_panel<0>(H, HLD, lane);
          if (np16 > 1) {
            pn_wave_sync();
            pn_chol_schur<16>(H, HLD, lane, np16 - 1);
            pn_wave_sync();
            pn_chol_panel<16>(H, HLD, lane);
            if (np16 > 2) {
              pn_wave_sync();
              pn_chol_schur<32>(H, HLD, lane, np16 - 2);
              pn_wave_sync();
              pn_chol_panel<32>(H, HLD, lane);
              if (np16 > 3) {
                pn_wave_sync();
                pn_chol_schur<48>(H, HLD, lane, 1);
                pn_wave_sync();
                pn_chol_panel<48>(H, HLD, lane);
              }
            }
          }
        }
        __syncthreads();
      } else {
        // scale, add the penalty curvature, and pin the active weights (identity rows)
        for (int e = tid; e < KMAX * KMAX; e += PN_THREADS) {
          const int r = e / KMAX, c = e % KMAX;
          if (c > r) continue;  // the factorisation and the solves read the lower triangle only
          double h = p.eps * (double)H[r * HLD + c];
          if (act[r] || act[c]) h = (r == c) ? 1.0 : 0.0;
          else if (r == c) h += hpen;
          H[r * HLD + c] = (TH)h;
        }
        __syncthreads();
        if (tid == 0) hrel_diag_s = released >= 0 ? (double)H[released * HLD + released] : 1.0;
        __syncthreads();

        // ---- Cholesky H = L L^T (lower triangle in place) by 16 x 16 tiles: factor
        // the diagonal tile in one wave, solve the panel below it (one thread per
        // row), update the trailing lower triangle (all threads).
        for (int kk = 0; kk < KMAX; kk += 16) {
          if (wave == 0 && lane < 16) {
            const int r = kk + lane;
            TH* Hr = H + r * HLD;
            for (int c = kk; c < kk + 16; ++c) {
              TH acc = 0;
              if (r >= c) {
                const TH* Hc = H + c * HLD;
                acc = Hr[c];
                for (int q = kk; q < c; ++q) acc -= Hr[q] * Hc[q];
              }
              if (r == c) Hr[c] = sqrt(acc > (TH)0 ? acc : tinyh);
              pn_wave_sync();
              if (r > c) Hr[c] = acc / H[c * HLD + c];
              pn_wave_sync();
            }
          }
          __syncthreads();
          for (int r = kk + 16 + tid; r < KMAX; r += PN_THREADS) {
            TH* Hr = H + r * HLD;
            for (int c = kk; c < kk + 16; ++c) {
              const TH* Hc = H + c * HLD;
              TH acc = Hr[c];
              for (int q = kk; q < c; ++q) acc -= Hr[q] * Hc[q];
              Hr[c] = acc / Hc[c];
            }
          }
          __syncthreads();
          const int m = KMAX - kk - 16;
          for (int e = tid; e < m * m; e += PN_THREADS) {
            const int r = kk + 16 + e / m, c = kk + 16 + e % m;
            if (c <= r) {
              const TH* Hr = H + r * HLD;
              const TH* Hc = H + c * HLD;
              TH s0 = 0, s1 = 0;
  #pragma unroll
              for (int q = 0; q < 16; q += 2) {
                s0 += Hr[kk + q] * Hc[kk + q];
                s1 += Hr[kk + q + 1] * Hc[kk + q + 1];
              }
              H[r * HLD + c] -= s0 + s1;
            }
          }
          __syncthreads();
        }
      }
      if (tid < KMAX) wHs[tid] = w[tid];
      if (tid == 0) {
        hstate[0] = 1;
        hstate[1] = 1;
      }
      ++nfac;
      if (tid == 0) {
        int m = 0;
        if constexpr (KMAX == 64) {
          m = cmp_s[0];
        } else {
          for (int j = 0; j < k; ++j) m += !act[j];
        }
        nent += m * (m + 1) / 2;
      }
      __syncthreads();
    }
    const double hdiag_released = released >= 0 ? hrel_diag_s : 1.0;

    // ---- solve L L^T d = -g in wave 0
    if (wave == 0) {
      if constexpr (KMAX == 64) {
        // compact positions: lane x works on the free weight perm[x] (x < m);
        // lane x keeps row x of L (forward), then column x (backward), 16
        // entries at a time in registers; y_c and 1 / L_cc reach the other
        // lanes by v_readlane
        const int m = cmp_s[0];
        const int nrow = __builtin_amdgcn_readfirstlane(max((m + 15) >> 4, 1)) * 16;
        const int x = lane;
        const int jx = x < m ? perm[x] : 0;
        const double inv_r = 1.0 / (double)H[x * HLD + x];
        double yv = x < m ? -g[jx] : 0.0;
#pragma unroll
        for (int cb = 0; cb < 64; cb += 16) {
          if (cb < nrow) {
            double lr[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) lr[u] = cb + u < x ? (double)H[x * HLD + cb + u] : 0.0;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
              const double yc = pn_readlane(yv, cb + u) * pn_readlane(inv_r, cb + u);
              yv = x == cb + u ? yc : yv - lr[u] * yc;
            }
          }
          __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int cb = 48; cb >= 0; cb -= 16) {
          if (cb < nrow) {
            double lc[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) lc[u] = cb + u > x ? (double)H[(cb + u) * HLD + x] : 0.0;
#pragma unroll
            for (int u = 15; u >= 0; --u) {
              const double dc = pn_readlane(yv, cb + u) * pn_readlane(inv_r, cb + u);
              yv = x == cb + u ? dc : yv - lc[u] * dc;
            }
          }
          __builtin_amdgcn_sched_barrier(0);
        }
        // weights at 0 cannot decrease; a released weight swamped by the coupling
        // takes its own Newton coordinate step instead
        if (x < m && w[jx] <= 0.0 && yv < 0.0) yv = 0.0;
        const double yr = __shfl(yv, released >= 0 ? cmp_s[1] : 0, 64);
        if (released >= 0 && yr <= 0.0) yv = (x < m && jx == released) ? -g[jx] / hdiag_released : 0.0;
        if (act[lane]) d[lane] = 0.0;
        if (x < m) d[jx] = yv;
        // ratio test inputs: slope g.d and the step to the first free weight reaching 0
        double sl = x < m ? g[jx] * yv : 0.0;
        double tm = (x < m && yv < 0.0) ? -w[jx] / yv : INFINITY;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          sl += __shfl_xor(sl, off, 64);
          tm = fmin(tm, __shfl_xor(tm, off, 64));
        }
        if (lane == 0) {
          rt_s[0] = sl;
          rt_s[1] = tm;
        }
      } else {
        // lane owns rows lane + 64 rr; forward: L y = -g ; backward: L^T d = y
        // (active rows: g = 0, L row = e_r); y_c and 1 / L_cc broadcast by
        // v_readlane
        double y[RPL], inv[RPL];
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
          const int r = lane + 64 * rr;
          y[rr] = act[r] ? 0.0 : -g[r];
          inv[rr] = 1.0 / (double)H[r * HLD + r];
        }
        for (int cb = 0; cb < KMAX; cb += 8) {  // L rows 8 entries at a time, read ahead of the chain
          TH lr[RPL][8];
#pragma unroll
          for (int rr = 0; rr < RPL; ++rr)
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const int r = lane + 64 * rr;
              const TH v = H[r * HLD + cb + u];
              lr[rr][u] = cb + u < r ? v : (TH)0;
            }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            const int c = cb + u;
            const double yc = pn_readlane(c < 64 ? y[0] : y[RPL - 1], c & 63) *
                              pn_readlane(c < 64 ? inv[0] : inv[RPL - 1], c & 63);
#pragma unroll
            for (int rr = 0; rr < RPL; ++rr) y[rr] = lane + 64 * rr == c ? yc : y[rr] - (double)lr[rr][u] * yc;
          }
        }
        for (int cb = KMAX - 8; cb >= 0; cb -= 8) {
          TH lc[RPL][8];
#pragma unroll
          for (int rr = 0; rr < RPL; ++rr)
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const int r = lane + 64 * rr;
              const TH v = H[(cb + u) * HLD + r];
              lc[rr][u] = cb + u > r ? v : (TH)0;
            }
#pragma unroll
          for (int u = 7; u >= 0; --u) {
            const int c = cb + u;
            const double dc = pn_readlane(c < 64 ? y[0] : y[RPL - 1], c & 63) *
                              pn_readlane(c < 64 ? inv[0] : inv[RPL - 1], c & 63);
#pragma unroll
            for (int rr = 0; rr < RPL; ++rr) y[rr] = lane + 64 * rr == c ? dc : y[rr] - (double)lc[rr][u] * dc;
          }
        }
        // weights at 0 cannot decrease; a released weight swamped by the coupling
        // takes its own Newton coordinate step instead
        const int rel = released >= 0 ? released : 0;
        double yr = 0.0;
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
          const int r = lane + 64 * rr;
          if (w[r] <= 0.0 && y[rr] < 0.0) y[rr] = 0.0;
          const double v = __shfl(y[rr], rel & 63, 64);
          if ((rel >> 6) == rr) yr = v;
        }
        double sl = 0.0, tm = INFINITY;
#pragma unroll
        for (int rr = 0; rr < RPL; ++rr) {
          const int r = lane + 64 * rr;
          double yv = y[rr];
          if (released >= 0 && yr <= 0.0) yv = (r == released) ? -g[r] / hdiag_released : 0.0;
          yv = act[r] ? 0.0 : yv;
          d[r] = yv;
          if (!act[r]) {  // ratio test inputs, as in the 64-wide path
            sl += g[r] * yv;
            if (yv < 0.0) tm = fmin(tm, -w[r] / yv);
          }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
          sl += __shfl_xor(sl, off, 64);
          tm = fmin(tm, __shfl_xor(tm, off, 64));
        }
        if (lane == 0) {
          rt_s[0] = sl;
          rt_s[1] = tm;
        }
      }
    }
    __syncthreads();

    // ---- ratio test and Armijo backtracking
    const double slope = rt_s[0], tmax = rt_s[1];  // reduced by wave 0 with the solve
    bool accepted = false, evaluated = false;
    double t = fmin(1.0, tmax), fn = 0.0;
    // trial point w + t d clipped at 0; at t = tmax the weights that stop the
    // ratio test land exactly on 0 (they join the active set if it is accepted)
    auto trial = [&](double tt) {
      if (tid < KMAX) {
        double v = act[tid] ? 0.0 : fmax(w[tid] + tt * d[tid], 0.0);
        if (tt == tmax && !act[tid] && d[tid] < 0.0 && -w[tid] / d[tid] <= tmax * (1.0 + 1e-12)) v = 0.0;
        wt[tid] = v;
      }
      __syncthreads();
    };
    if (slope < 0.0 && -slope <= 1e-14 * fabs(f)) {
      // the predicted decrease is below what V can resolve in FP64: the point is
      // optimal to working precision on this free set, take the step untested
      trial(t);
      accepted = true;
    } else if (slope < 0.0) {
      for (int ls = 0; ls < 30; ++ls) {
        trial(t);
        fn = pn_eval<MAXB>(p, DTp, ld_dt, n, k, wt, s, at, lt, tiny, red);
        if (fn <= f + 1e-4 * t * slope) {
          accepted = evaluated = true;
          break;
        }
        t *= 0.5;
      }
    }
    if (!accepted && ctl[3]) {  // the step on a reused factor failed: retry with a fresh factor
      __syncthreads();
      if (tid == 0) force_rebuild = 1;
      __syncthreads();
      continue;
    }
    if (!accepted) {  // no descent left on this free set: release the candidate, or stop
      const int cand = ctl[2];
      __syncthreads();
      if (cand >= 0) {
        if (tid == 0) act[cand] = 0;
        __syncthreads();
        continue;
      }
      break;
    }
    if (tid < KMAX) {
      if (t == tmax && !act[tid] && d[tid] < 0.0 && -w[tid] / d[tid] <= tmax * (1.0 + 1e-12)) act[tid] = 1;
      w[tid] = wt[tid];
    }
    if (evaluated) {  // the accepted trial's a, l and V are the new point's
      TL* x = a;
      a = at;
      at = x;
      x = l;
      l = lt;
      lt = x;
      f = fn;
    } else {
      have_f = false;
    }
    __syncthreads();
  }

  // ---- write back (and the last factor, for the next launch)
  if (tid < k) wrow[tid] = (TW)w[tid];
  if (tid < KMAX && tid >= k && tid < ld_w) wrow[tid] = (TW)0;
  if (tid == 0) {
    p.nit[b] += it;
    if (p.nfac) p.nfac[b] += nfac;
    if (p.nent) p.nent[b] += nent;
    if (p.flops) atomicAdd(p.flops, 6ull * (unsigned long long)it * n * k + 2ull * (unsigned long long)nent * n);
  }
  if (reuse_on && hstate[1]) {
    for (int e = tid; e < KMAX * KMAX; e += PN_THREADS) Lb[e] = H[(e / KMAX) * HLD + (e % KMAX)];
    if (tid < KMAX) p.wH[(size_t)b * 128 + tid] = wHs[tid];
    if (tid == 0) {
      for (int m = 0; m < RPL; ++m) p.maskH[(size_t)b * 2 + m] = hmask_s[m];
      p.validH[b] = 1;
    }
  }
}

// Largest dynamic LDS of one workgroup (the 160 KB of a CU less the kernel's
// static arrays, which take under 1 KB).
constexpr size_t PN_LDS_MAX = 160 * 1024 - 1024;

// Dynamic LDS of prox_newton_kernel<..., KMAX, TH> for n bins, s elements of
// s_bytes and a / l elements of l_bytes.
template <int KMAX = PN_K, class TH = double>
inline size_t prox_newton_smem(int n, size_t s_bytes, size_t l_bytes = sizeof(double)) {
  return sizeof(TH) * (size_t)KMAX * (KMAX + 1) + sizeof(double) * (8 * (size_t)KMAX + 8) +
         (4 * l_bytes + s_bytes) * (size_t)n;
}
