// Device side of the warm-start network: a multilayer perceptron
//   x -> GELU(x W1^T + b1) -> GELU(. W2^T + b2) -> . W3^T + b3
// that maps a (standardised) target spectrum to a standardised prediction of
// the solver's fixed point (log u, log v, w).  Weights are [out, in] row-major;
// the flat parameter vector is [W1, b1, W2, b2, W3, b3].
//
// Every layer is one MFMA GEMM with the elementwise work in its epilogue:
// forward  Z_l = H_{l-1} W_l^T (+ b_l, GELU)                 (A, Bt k-contiguous)
// backward dH_{l-1} = dZ_l W_l   (then x GELU'(Z_{l-1}))      (B stored [Kd, N])
//          dW_l = dZ_l^T H_{l-1}                               (A and B stored [Kd, .])
// GELU is the exact form z Phi(z) (erf).  The loss is the weighted mean squared
// error over all outputs of standardised targets, (clamp(t, +-T_CLAMP) - mu) / sd.
#pragma once
#include <hip/hip_runtime.h>
#include "solver_kernels.hpp"

constexpr float MLP_T_CLAMP = 50.0f;
constexpr double MLP_SD_FLOOR = 1e-6;

__device__ __forceinline__ float mlp_gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float mlp_gelu_prime(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// hidden layer: z = c + b_n; keeps z for the backward pass (Z may be null) and
// stores GELU(z) in FP32 (H) and/or BF16 (Hbf)
struct EpiBiasGelu {
  static constexpr int NRED = 0;
  static constexpr bool RED_IS_MAX[2] = {false, false};
  const float* bias;
  float* Z;
  float* H;
  unsigned short* Hbf;
  int ld;
  bool do_red;
  __device__ __forceinline__ void elem(int m, int n, float c, float*) const {
    const float z = c + bias[n];
    const size_t o = (size_t)m * ld + n;
    if (Z) Z[o] = z;
    const float h = mlp_gelu(z);
    if (H) H[o] = h;
    if (Hbf) Hbf[o] = f32_to_bf16(h);
  }
  __device__ __forceinline__ void row_partial(int, int, const float*) const {}
};

// output layer in training: z = c + b_n, residual r = z - t^ with the
// standardised target t^ of row idx[m] (idx null: row m); with the output
// weight om_n it stores the loss gradient dZ = scale om_n r (scale = 2 / (B O))
// and the per-tile sum of om_n r^2
struct EpiLossOut {
  static constexpr int NRED = 1;
  static constexpr bool RED_IS_MAX[2] = {false, false};
  const float* bias;
  const float* T;
  const int* idx;
  int ldt;
  const float* mu;
  const float* sd;
  const float* om;
  float* dZ;
  int ld;
  float scale;
  float* part;
  int ntiles;
  bool do_red;
  __device__ __forceinline__ void elem(int m, int n, float c, float* red) const {
    const int row = idx ? idx[m] : m;
    const float t = fminf(fmaxf(T[(size_t)row * ldt + n], -MLP_T_CLAMP), MLP_T_CLAMP);
    const float r = (c + bias[n]) - (t - mu[n]) / sd[n];
    const float w = om[n];
    dZ[(size_t)m * ld + n] = scale * w * r;
    red[0] += w * r * r;
  }
  __device__ __forceinline__ void row_partial(int m, int tile, const float* v) const {
    part[(size_t)m * ntiles + tile] = v[0];
  }
};

// backward through GELU: dZ = c * GELU'(Z)
struct EpiGeluBack {
  static constexpr int NRED = 0;
  static constexpr bool RED_IS_MAX[2] = {false, false};
  const float* Z;
  float* dZ;
  int ld;
  bool do_red;
  __device__ __forceinline__ void elem(int m, int n, float c, float*) const {
    const size_t o = (size_t)m * ld + n;
    dZ[o] = c * mlp_gelu_prime(Z[o]);
  }
  __device__ __forceinline__ void row_partial(int, int, const float*) const {}
};

// output layer at inference: prediction p = (c + b_n) sd_n + mu_n in raw
// units, split by column into log u [n_u], log v [n_v] and w (clamped >= 0)
struct EpiOutSplit {
  static constexpr int NRED = 0;
  static constexpr bool RED_IS_MAX[2] = {false, false};
  const float* bias;
  const float* mu;
  const float* sd;
  int n_u, n_v, k_w;
  float* logU;
  float* logV;
  float* W;
  bool do_red;
  __device__ __forceinline__ void elem(int m, int n, float c, float*) const {
    const float p = (c + bias[n]) * sd[n] + mu[n];
    if (n < n_u) {
      if (logU) logU[(size_t)m * n_u + n] = p;
    } else if (n < n_u + n_v) {
      logV[(size_t)m * n_v + (n - n_u)] = p;
    } else {
      W[(size_t)m * k_w + (n - n_u - n_v)] = fmaxf(p, 0.f);
    }
  }
  __device__ __forceinline__ void row_partial(int, int, const float*) const {}
};

// x^ = (y - mu) / sd for rows idx[b] (idx null: row b) of Y, into FP32 and/or BF16.
__global__ __launch_bounds__(256) void mlp_gather_norm(const float* __restrict__ Y, int ldy,
                                                       const int* __restrict__ idx, int B, int cols,
                                                       const float* __restrict__ mu, const float* __restrict__ sd,
                                                       float* __restrict__ X, unsigned short* __restrict__ Xbf) {
  const int b = blockIdx.x;
  if (b >= B) return;
  const size_t row = idx ? (size_t)idx[b] : (size_t)b;
  for (int i = threadIdx.x; i < cols; i += blockDim.x) {
    const float x = (Y[row * ldy + i] - mu[i]) / sd[i];
    if (X) X[(size_t)b * cols + i] = x;
    if (Xbf) Xbf[(size_t)b * cols + i] = f32_to_bf16(x);
  }
}

// Column statistics, pass 1: per chunk of rows (rows chunk, chunk + nchunk,
// ...) and column, the FP64 sums of a and a^2 of the clamped values.
__global__ __launch_bounds__(256) void mlp_stats_partial(const float* __restrict__ A, long long rows, int cols,
                                                         int nchunk, float clamp, double* __restrict__ s1,
                                                         double* __restrict__ s2) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x, chunk = blockIdx.y;
  if (c >= cols) return;
  double a1 = 0.0, a2 = 0.0;
  for (long long r = chunk; r < rows; r += nchunk) {
    float a = A[(size_t)r * cols + c];
    if (clamp > 0.f) a = fminf(fmaxf(a, -clamp), clamp);
    a1 += (double)a;
    a2 += (double)a * (double)a;
  }
  s1[(size_t)chunk * cols + c] = a1;
  s2[(size_t)chunk * cols + c] = a2;
}

// pass 2: mean and floored standard deviation per column (chunks summed in order)
__global__ __launch_bounds__(256) void mlp_stats_final(const double* __restrict__ s1, const double* __restrict__ s2,
                                                       long long rows, int cols, int nchunk, float* __restrict__ mu,
                                                       float* __restrict__ sd) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double a1 = 0.0, a2 = 0.0;
  for (int k = 0; k < nchunk; ++k) {
    a1 += s1[(size_t)k * cols + c];
    a2 += s2[(size_t)k * cols + c];
  }
  const double m = a1 / (double)rows;
  const double var = fmax(a2 / (double)rows - m * m, 0.0);
  mu[c] = (float)m;
  sd[c] = (float)fmax(sqrt(var), MLP_SD_FLOOR);
}

// bias gradient: db_o = sum_b dZ[b, o] (rows in order, FP64 accumulate)
__global__ __launch_bounds__(256) void mlp_col_sum(const float* __restrict__ dZ, int B, int cols,
                                                   float* __restrict__ db) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= cols) return;
  double acc = 0.0;
  for (int b = 0; b < B; ++b) acc += (double)dZ[(size_t)b * cols + c];
  db[c] = (float)acc;
}

// loss = sum of the per-(row, tile) partials / (B O), summed in a fixed order
__global__ __launch_bounds__(256) void mlp_loss_reduce(const float* __restrict__ part, int count, double inv,
                                                       float* __restrict__ loss) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < count; i += blockDim.x) acc += (double)part[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = (float)(sh[0] * inv);
}

// AdamW with decoupled weight decay on every parameter; bc1 = 1 - b1^t,
// bc2 = 1 - b2^t for the step count t.
__global__ __launch_bounds__(256) void mlp_adamw(float* __restrict__ theta, const float* __restrict__ g,
                                                 float* __restrict__ m, float* __restrict__ v, long long count,
                                                 float lr, float b1, float b2, float eps, float wd, float bc1,
                                                 float bc2) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < count;
       i += (long long)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float p = theta[i];
    theta[i] = p - lr * ((mi / bc1) / (sqrtf(vi / bc2) + eps) + wd * p);
  }
}
