// FP64 "NT" GEMM on CDNA4 matrix cores (v_mfma_f64_16x16x4_f64) with the same
// fused-epilogue contract as gemm_nt_f32:
//
//   C[m, n] = sum_k A[m, k] * Bt[n, k]      (A: [M, Kd], Bt: [N, Kd], row-major)
//
// Used by the FP64 refinement phase, where the kernel products must carry more
// than FP32's 24 bits: on dictionaries with strongly overlapping columns the
// weight prox amplifies the relative error of s = K v by 1e2..1e4.
//
// Tiling: 256 threads = 4 wave64s in 2 x 2; workgroup tile 64 x 64, each wave
// 32 x 32 = 2 x 2 fragments of 16 x 16.  k stages of 16 go through LDS with rows
// padded to 18 doubles; within a stage the four 16-lane groups h supply
// k = 4h .. 4h+3, so each lane reads its operands with 128-bit LDS loads.
#pragma once
#include <hip/hip_runtime.h>

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

constexpr int G64_BM = 64, G64_BN = 64, G64_BK = 16, G64_LD = 18;

struct GemmArgs64 {
  const double* A;
  int lda;
  const double* Bt;
  int ldb;
  int M, N, Kd;
};

template <bool IS_MAX>
__device__ __forceinline__ double red_op64(double a, double b) {
  return IS_MAX ? fmax(a, b) : a + b;
}

// rowidx (may be null): rows 0 .. g.M - 1 of the product are rows rowidx[m]
// of A and of the epilogue (the active spectra of a batch).
template <class Epi>
__global__ __launch_bounds__(256) void gemm_nt_f64(GemmArgs64 g, Epi epi, const int* __restrict__ rowidx) {
  constexpr int BM = G64_BM, BN = G64_BN, BK = G64_BK, LD = G64_LD;
  __shared__ __attribute__((aligned(16))) double As[2][BM * LD];
  __shared__ __attribute__((aligned(16))) double Bs[2][BN * LD];
  __shared__ double red_s[2][BM][2];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1, h = lane >> 4, l16 = lane & 15;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;

  // global loads: a 64 x 16 tile = 512 pairs of doubles, 2 per thread per operand
  f64x2 ra[2], rb[2];
  const double* arow[2];  // A row of each staged pair (null: beyond M)
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int idx = tid + q * 256, r = idx >> 3, gm = m0 + r;
    arow[q] = gm < g.M ? g.A + (size_t)(rowidx ? rowidx[gm] : gm) * g.lda : nullptr;
  }
  auto gload = [&](int kt) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int idx = tid + q * 256, r = idx >> 3, c = (idx & 7) * 2;
      const int gn = n0 + r;
      ra[q] = arow[q] ? *reinterpret_cast<const f64x2*>(arow[q] + kt * BK + c) : f64x2{0.0, 0.0};
      rb[q] = gn < g.N ? *reinterpret_cast<const f64x2*>(g.Bt + (size_t)gn * g.ldb + kt * BK + c) : f64x2{0.0, 0.0};
    }
  };
  auto swrite = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int idx = tid + q * 256, r = idx >> 3, c = (idx & 7) * 2;
      *reinterpret_cast<f64x2*>(&As[buf][r * LD + c]) = ra[q];
      *reinterpret_cast<f64x2*>(&Bs[buf][r * LD + c]) = rb[q];
    }
  };

  f64x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};

  const int nk = g.Kd / BK;
  gload(0);
  swrite(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) gload(kt + 1);
    f64x4 a[2], b[2];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      const double* pa = &As[cur][(wm * 32 + f * 16 + l16) * LD + h * 4];
      const double* pb = &Bs[cur][(wn * 32 + f * 16 + l16) * LD + h * 4];
      f64x2 a0 = *reinterpret_cast<const f64x2*>(pa), a1 = *reinterpret_cast<const f64x2*>(pa + 2);
      f64x2 b0 = *reinterpret_cast<const f64x2*>(pb), b1 = *reinterpret_cast<const f64x2*>(pb + 2);
      a[f] = f64x4{a0[0], a0[1], a1[0], a1[1]};
      b[f] = f64x4{b0[0], b0[1], b1[0], b1[1]};
    }
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int fm = 0; fm < 2; ++fm)
#pragma unroll
        for (int fn = 0; fn < 2; ++fn)
          acc[fm][fn] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[fm][p], b[fn][p], acc[fm][fn], 0, 0, 0);
    if (kt + 1 < nk) swrite(cur ^ 1);
    __syncthreads();
  }

  // 16x16 f64 accumulator layout: lane l, register r holds row l/16 + 4 r,
  // column l%16 of its fragment.
#pragma unroll
  for (int fm = 0; fm < 2; ++fm) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = wm * 32 + fm * 16 + h + 4 * r;
      const int m = m0 + row;
      double red[2] = {0.0, 0.0};
      if (m < g.M) {
        const int mr = rowidx ? rowidx[m] : m;
#pragma unroll
        for (int fn = 0; fn < 2; ++fn) {
          const int n = n0 + wn * 32 + fn * 16 + l16;
          if (n < g.N) epi.elem(mr, n, acc[fm][fn][r], red);
        }
      }
      if constexpr (Epi::NRED > 0) {
        if (epi.do_red) {
#pragma unroll
          for (int off = 1; off < 16; off <<= 1) {
            red[0] = red_op64<Epi::RED_IS_MAX[0]>(red[0], __shfl_xor(red[0], off, 64));
            red[1] = red_op64<Epi::RED_IS_MAX[1]>(red[1], __shfl_xor(red[1], off, 64));
          }
          if (l16 == 0) {
            red_s[wn][row][0] = red[0];
            red_s[wn][row][1] = red[1];
          }
        }
      }
    }
  }
  if constexpr (Epi::NRED > 0) {
    if (epi.do_red) {
      __syncthreads();
      for (int row = tid; row < BM; row += 256) {
        const int m = m0 + row;
        if (m < g.M) {
          double v[2];
          v[0] = red_op64<Epi::RED_IS_MAX[0]>(red_s[0][row][0], red_s[1][row][0]);
          v[1] = red_op64<Epi::RED_IS_MAX[1]>(red_s[0][row][1], red_s[1][row][1]);
          epi.row_partial(rowidx ? rowidx[m] : m, blockIdx.x, v);
        }
      }
    }
  }
}
