// FP64 counterparts of the scaling-loop epilogues (refinement phase) and the
// conversions between the FP32 and FP64 state.  Same algebra as
// solver_kernels.hpp (Algorithm 1 with the Table 1 proxes), evaluated in
// double precision.
#pragma once
#include <hip/hip_runtime.h>
#include "omega.hpp"
#include "solver_kernels.hpp"

struct ProxConsts64 {
  int fit;
  double kappa, lam_eps, lam2_eps, eps_lam, log_lam_eps;
};

__device__ __forceinline__ double target_scaling64(const ProxConsts64& pc, double t, double y) {
  if (!(t > 0.0)) return 1.0;
  const double lt = log(t);
  switch (pc.fit) {
    case FIT_BALANCED:
      return y / t;
    case FIT_KL:
      return y > 0.0 ? exp(pc.kappa * (log(y) - lt)) : 0.0;
    case FIT_TV: {
      const double ly = y > 0.0 ? log(y) : -INFINITY;
      return exp(fmin(fmax(ly - lt, -pc.lam_eps), pc.lam_eps));
    }
    case FIT_L2: {
      const double p = pc.eps_lam * wright_omega<double>(pc.log_lam_eps + lt + pc.lam_eps * y);
      return p / t;
    }
    case FIT_L2_TV: {
      const double ly = y > 0.0 ? log(y) : -INFINITY;
      const double ltau = lt + fmin(fmax(ly - lt, -pc.lam2_eps), pc.lam2_eps);
      const double p = pc.eps_lam * wright_omega<double>(pc.log_lam_eps + ltau + pc.lam_eps * y);
      return p / t;
    }
    case FIT_POISSON: {
      if (!(y > 0.0)) return 0.0;
      const double p = pc.lam_eps * y / wright_omega<double>(pc.log_lam_eps + log(y) - lt + pc.lam_eps);
      return p / t;
    }
  }
  return 1.0;
}

// s = K v; on test iterations the source-violation partials (as in EpiSrc).
struct EpiSrc64 {
  static constexpr int NRED = 2;
  static constexpr bool RED_IS_MAX[2] = {false, false};
  double* S;
  const double* A;
  const double* U;
  float* part_num;
  float* part_den;
  int ld, n_valid, ntiles;
  bool do_red;
  __device__ __forceinline__ void elem(int m, int n, double s, double* red) const {
    const size_t o = (size_t)m * ld + n;
    if (n >= n_valid) {
      S[o] = 0.0;
      return;
    }
    S[o] = s;
    if (do_red) {
      const double a = A[o];
      red[0] += fabs(U[o] * s - a);
      red[1] += a;
    }
  }
  __device__ __forceinline__ void row_partial(int m, int tile, const double* v) const {
    part_num[(size_t)m * ntiles + tile] = (float)v[0];
    part_den[(size_t)m * ntiles + tile] = (float)v[1];
  }
};

// a = D w, u = a / s
struct EpiUscale64 {
  static constexpr int NRED = 0;
  static constexpr bool RED_IS_MAX[2] = {false, false};
  double* A;
  double* U;
  const double* S;
  int ld, n_valid;
  bool do_red;
  __device__ __forceinline__ void elem(int m, int n, double a, double*) const {
    const size_t o = (size_t)m * ld + n;
    if (n >= n_valid) {
      A[o] = 0.0;
      U[o] = 0.0;
      return;
    }
    a = fmax(a, 0.0);
    A[o] = a;
    U[o] = a > 0.0 ? a / S[o] : 0.0;
  }
  __device__ __forceinline__ void row_partial(int, int, const double*) const {}
};

// t = K^T u, v = prox_L(t | y) / t
struct EpiProx64 {
  static constexpr int NRED = 0;
  static constexpr bool RED_IS_MAX[2] = {false, false};
  double* V;
  const float* Y;
  const int* done;
  ProxConsts64 pc;
  int ld, ldy, n_valid;
  bool do_red;
  __device__ __forceinline__ void elem(int m, int n, double t, double*) const {
    const size_t o = (size_t)m * ld + n;
    if (n >= n_valid) {
      V[o] = 0.0;
      return;
    }
    if (done[m]) return;
    V[o] = target_scaling64(pc, t, (double)Y[(size_t)m * ldy + n]);
  }
  __device__ __forceinline__ void row_partial(int, int, const double*) const {}
};

// Elementwise conversions between state precisions.
__global__ void convert_f32_to_f64(const float* __restrict__ x, double* __restrict__ y, size_t count) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
    y[i] = (double)x[i];
}

// Outputs from the FP64 state.
__global__ void write_outputs64(const double* __restrict__ Wst, const double* __restrict__ U,
                                const double* __restrict__ V, const int* __restrict__ done,
                                const int* __restrict__ st, const int* __restrict__ it_in,
                                const int* __restrict__ xflags, const int* __restrict__ it_base, int n, int k,
                                int np, int kp, int last_iter, float* __restrict__ W, float* __restrict__ logU,
                                float* __restrict__ logV, int* __restrict__ iters, int* __restrict__ status) {
  const int b = blockIdx.x;
  for (int j = threadIdx.x; j < k; j += blockDim.x) W[(size_t)b * k + j] = (float)Wst[(size_t)b * kp + j];
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    if (logU) logU[(size_t)b * n + i] = (float)log(U[(size_t)b * np + i]);
    logV[(size_t)b * n + i] = (float)log(V[(size_t)b * np + i]);
  }
  if (threadIdx.x == 0) {
    if (iters) iters[b] = done[b] ? it_in[b] : last_iter + it_base[b];
    if (status) status[b] = (done[b] ? st[b] : 2) | xflags[b];
  }
}

// Start of a refinement phase: every spectrum that has not failed becomes
// active again (its bulk-phase test used a looser tolerance).
// it_base[b] becomes the spectrum's own bulk iteration count minus `last` (the
// iteration at which the bulk phase ended for the batch), so that iteration
// indices of the refinement phase plus it_base count the spectrum's own
// iterations.
__global__ void reopen_spectra(int B, int last, int* __restrict__ done, int* __restrict__ status,
                               const int* __restrict__ iters, int* __restrict__ it_base, float* __restrict__ ew_prev,
                               float* __restrict__ ew_best, int* __restrict__ stall) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  it_base[b] = (done[b] ? iters[b] : last) - last;
  if (status[b] != 4) {
    done[b] = 0;
    status[b] = 0;
  }
  ew_prev[b] = 0.f;
  ew_best[b] = INFINITY;
  stall[b] = 0;
}
