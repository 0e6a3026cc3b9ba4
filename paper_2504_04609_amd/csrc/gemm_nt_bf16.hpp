// BF16 "NT" GEMM with FP32 accumulation on CDNA4 matrix cores
// (v_mfma_f32_32x32x16_bf16), same fused-epilogue contract as gemm_nt_f32:
//
//   C[m, n] = sum_k A[m, k] * Bt[n, k]      (A: [M, Kd], Bt: [N, Kd], BF16, row-major)
//
// Used for the kernel products s = K v and t = K^T u of a BF16 bulk phase: the
// scaling vectors and K are rounded to BF16 (8-bit mantissa), the sums are
// accumulated in FP32, and the result feeds the same FP32 epilogues.
//
// Tiling: 256 threads = 4 wave64s in 2 x 2; workgroup tile 128 x 128, each
// wave 64 x 64 = 2 x 2 fragments of 32 x 32.  k advances in stages of 32
// staged in LDS with rows padded to 40 elements (80 bytes, so the 128-bit reads
// of eight consecutive lanes hit distinct banks); in MFMA step kk of a stage the
// lanes of half h supply k = 16 kk + 8 h .. +7, read with one 128-bit load.
#pragma once
#include <hip/hip_runtime.h>
#include "gemm_nt.hpp"
#include "solver_kernels.hpp"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

constexpr int GB_BM = 128, GB_BN = 128, GB_BK = 32, GB_LD = 40;

struct GemmArgsBf16 {
  const unsigned short* A;
  int lda;
  const unsigned short* Bt;
  int ldb;
  int M, N, Kd;
};

// BM rows per tile (128, or 64: FM = BM / 64 fragments of 32 rows per wave),
// BN = 128 columns.
template <class Epi, int BM = GB_BM>
__global__ __launch_bounds__(256) void gemm_nt_bf16(GemmArgsBf16 g, Epi epi) {
  static_assert(BM == 128 || BM == 64, "tile rows");
  constexpr int BN = GB_BN, BK = GB_BK, LD = GB_LD, FM = BM / 64;
  __shared__ __attribute__((aligned(16))) unsigned short As[2][BM * LD];
  __shared__ __attribute__((aligned(16))) unsigned short Bs[2][BN * LD];
  __shared__ float red_s[2][BM][2];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1, h = lane >> 5, l32 = lane & 31;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;

  // a 128 x 32 tile is 512 chunks of 8 elements: two per thread (one for a
  // 64-row A tile)
  u16x8 ra[FM], rb[2];
  auto gload = [&](int kt) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int idx = tid + q * 256, r = idx >> 2, c = (idx & 3) * 8;
      const int gm = m0 + r, gn = n0 + r;
      if (q < FM)
        ra[q] = gm < g.M ? *reinterpret_cast<const u16x8*>(g.A + (size_t)gm * g.lda + kt * BK + c) : u16x8{};
      rb[q] = gn < g.N ? *reinterpret_cast<const u16x8*>(g.Bt + (size_t)gn * g.ldb + kt * BK + c) : u16x8{};
    }
  };
  auto swrite = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int idx = tid + q * 256, r = idx >> 2, c = (idx & 3) * 8;
      if (q < FM) *reinterpret_cast<u16x8*>(&As[buf][r * LD + c]) = ra[q];
      *reinterpret_cast<u16x8*>(&Bs[buf][r * LD + c]) = rb[q];
    }
  };

  f32x16 acc[FM][2];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  const int nk = g.Kd / BK;
  gload(0);
  swrite(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) gload(kt + 1);
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      bf16x8 a[FM], b[2];
#pragma unroll
      for (int f = 0; f < FM; ++f)
        a[f] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(
                                              &As[cur][(wm * (BM / 2) + f * 32 + l32) * LD + kk * 16 + h * 8]));
#pragma unroll
      for (int f = 0; f < 2; ++f)
        b[f] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8*>(
                                              &Bs[cur][(wn * 64 + f * 32 + l32) * LD + kk * 16 + h * 8]));
#pragma unroll
      for (int fm = 0; fm < FM; ++fm)
#pragma unroll
        for (int fn = 0; fn < 2; ++fn)
          acc[fm][fn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[fm], b[fn], acc[fm][fn], 0, 0, 0);
    }
    if (kt + 1 < nk) swrite(cur ^ 1);
    __syncthreads();
  }

  // 32x32 accumulator layout: lane l, register r holds row 8*(r/4) + 4*(l/32) + r%4,
  // column l%32 of its fragment.
#pragma unroll
  for (int fm = 0; fm < FM; ++fm) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = wm * (BM / 2) + fm * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
      const int m = m0 + row;
      float red[2] = {0.f, 0.f};
      if (m < g.M) {
#pragma unroll
        for (int fn = 0; fn < 2; ++fn) {
          const int n = n0 + wn * 64 + fn * 32 + l32;
          if (n < g.N) epi.elem(m, n, acc[fm][fn][r], red);
        }
      }
      if constexpr (Epi::NRED > 0) {
        if (epi.do_red) {
          red[0] = half_wave_reduce<Epi::RED_IS_MAX[0]>(red[0]);
          if constexpr (Epi::NRED > 1) red[1] = half_wave_reduce<Epi::RED_IS_MAX[1]>(red[1]);
          if (l32 == 0) {
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
          float v[2];
          v[0] = red_op<Epi::RED_IS_MAX[0]>(red_s[0][row][0], red_s[1][row][0]);
          v[1] = red_op<Epi::RED_IS_MAX[1]>(red_s[0][row][1], red_s[1][row][1]);
          epi.row_partial(m, blockIdx.x, v);
        }
      }
    }
  }
}
