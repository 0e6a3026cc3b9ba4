// FP32 "NT" GEMM on CDNA4 matrix cores with a fused, per-element epilogue.
//
//   C[m, n] = sum_k A[m, k] * Bt[n, k]        (A: [M, Kd], Bt: [N, Kd], both row-major)
//
// Both operands are read along k, which is the layout every product of the
// scaling loop needs without a transpose: S = V K^T reads K itself, T = U K
// reads K^T (the same array when the cost is symmetric), the dictionary
// products read D or D^T.
//
// Tiling: a 256-thread workgroup (4 wave64s in a 2 x 2 grid) owns a BM x BN
// output tile; each wave owns (BM/2) x (BN/2) as 32 x 32 fragments of
// v_mfma_f32_32x32x2_f32.  k advances in stages of 16; each stage is staged in
// LDS with rows padded to 20 floats so that the 128-bit LDS reads of a
// half-wave hit distinct banks, and the next stage is prefetched into registers
// while the current one is multiplied (one barrier per stage).  Inside a stage
// the lanes of half h supply k = 8h .. 8h+7, so each lane reads its operands
// with two 128-bit LDS loads; the k order only permutes the sum.
//
// Requirements (checked by the host): lda, ldb multiples of 4, 16-byte aligned
// base pointers, Kd a multiple of 16 (operands are zero-padded), M, N >= 1.
// Rows of A beyond M and rows of Bt beyond N are read as zero.
//
// Epilogue contract (Epi):
//   static constexpr int NRED;                 // 0..2 row reductions
//   static constexpr bool RED_IS_MAX[2];      // max (true) or sum (false)
//   bool do_red;                               // runtime switch for the reductions
//   __device__ void elem(int m, int n, float c, float* red) const;
//   __device__ void row_partial(int m, int tile, const float* red) const;
// elem() is called once for every (m < M, n < N); row_partial() once per row
// m < M of the tile with the reductions over the tile's columns.
#pragma once
#include <hip/hip_runtime.h>

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int GEMM_BK = 16;
constexpr int GEMM_LDS_LD = 20;

struct GemmArgs {
  const float* A;
  int lda;
  const float* Bt;
  int ldb;
  int M, N, Kd;
};

template <bool IS_MAX>
__device__ __forceinline__ float red_op(float a, float b) {
  return IS_MAX ? fmaxf(a, b) : a + b;
}

template <bool IS_MAX>
__device__ __forceinline__ float half_wave_reduce(float v) {
#pragma unroll
  for (int off = 1; off < 32; off <<= 1) v = red_op<IS_MAX>(v, __shfl_xor(v, off, 64));
  return v;
}

// One BM x BN output tile at (m0, n0); `tile` is the column-tile index passed
// to row_partial().  Shared by the plain and the grouped launches.  With a row
// index (rowidx != null) the tile's rows m0.. are positions in that list: A
// row rowidx[m] is read and the epilogue sees row rowidx[m] (gathered rows).
//
// Layouts: by default both operands are k-contiguous (A [M, Kd], Bt [N, Kd]).
// TA = true reads A stored [Kd, M] (element (m, k) at A[k * lda + m]) and
// TB = true reads B stored [Kd, N] (element (n, k) at Bt[k * ldb + n]); such
// operands are loaded 4 consecutive m (or n) at a time and transposed into the
// same LDS layout, so the MFMA core is shared.  Those layouts need M (resp. N)
// a multiple of 4 and take no row index.
template <int BM, int BN, class Epi, bool TA = false, bool TB = false>
__device__ __forceinline__ void gemm_nt_f32_tile(const GemmArgs& g, const Epi& epi, int m0, int n0, int tile,
                                                 const int* __restrict__ rowidx = nullptr) {
  constexpr int BK = GEMM_BK, LD = GEMM_LDS_LD;
  constexpr int WM = BM / 2, WN = BN / 2, FM = WM / 32, FN = WN / 32;
  constexpr int A_V4 = BM * (BK / 4) / 256;
  constexpr int B_V4 = BN * (BK / 4) / 256;
  static_assert(FM >= 1 && FN >= 1 && A_V4 >= 1 && B_V4 >= 1, "tile too small");

  __shared__ __attribute__((aligned(16))) float As[2][BM * LD];
  __shared__ __attribute__((aligned(16))) float Bs[2][BN * LD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1, h = lane >> 5, l32 = lane & 31;

  f32x4 ra[A_V4], rb[B_V4];
  const float* arow[A_V4];  // A row of each staged chunk (null: beyond M)
  if constexpr (!TA) {
#pragma unroll
    for (int q = 0; q < A_V4; ++q) {
      const int idx = tid + q * 256, r = idx >> 2, c = (idx & 3) * 4, gr = m0 + r;
      arow[q] = gr < g.M ? g.A + (size_t)(rowidx ? rowidx[gr] : gr) * g.lda + c : nullptr;
    }
  }
  constexpr f32x4 zero4 = {0.f, 0.f, 0.f, 0.f};
  auto gload = [&](int kt) {
#pragma unroll
    for (int q = 0; q < A_V4; ++q) {
      if constexpr (!TA) {
        ra[q] = arow[q] ? *reinterpret_cast<const f32x4*>(arow[q] + kt * BK) : zero4;
      } else {
        const int idx = tid + q * 256, kr = idx / (BM / 4), mc = (idx % (BM / 4)) * 4, gm = m0 + mc;
        ra[q] = gm < g.M ? *reinterpret_cast<const f32x4*>(g.A + (size_t)(kt * BK + kr) * g.lda + gm) : zero4;
      }
    }
#pragma unroll
    for (int q = 0; q < B_V4; ++q) {
      if constexpr (!TB) {
        const int idx = tid + q * 256, r = idx >> 2, c = (idx & 3) * 4, gr = n0 + r;
        rb[q] = gr < g.N ? *reinterpret_cast<const f32x4*>(g.Bt + (size_t)gr * g.ldb + kt * BK + c) : zero4;
      } else {
        const int idx = tid + q * 256, kr = idx / (BN / 4), nc = (idx % (BN / 4)) * 4, gn = n0 + nc;
        rb[q] = gn < g.N ? *reinterpret_cast<const f32x4*>(g.Bt + (size_t)(kt * BK + kr) * g.ldb + gn) : zero4;
      }
    }
  };
  auto swrite = [&](int buf) {
#pragma unroll
    for (int q = 0; q < A_V4; ++q) {
      if constexpr (!TA) {
        const int idx = tid + q * 256, r = idx >> 2, c = (idx & 3) * 4;
        *reinterpret_cast<f32x4*>(&As[buf][r * LD + c]) = ra[q];
      } else {
        const int idx = tid + q * 256, kr = idx / (BM / 4), mc = (idx % (BM / 4)) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) As[buf][(mc + j) * LD + kr] = ra[q][j];
      }
    }
#pragma unroll
    for (int q = 0; q < B_V4; ++q) {
      if constexpr (!TB) {
        const int idx = tid + q * 256, r = idx >> 2, c = (idx & 3) * 4;
        *reinterpret_cast<f32x4*>(&Bs[buf][r * LD + c]) = rb[q];
      } else {
        const int idx = tid + q * 256, kr = idx / (BN / 4), nc = (idx % (BN / 4)) * 4;
#pragma unroll
        for (int j = 0; j < 4; ++j) Bs[buf][(nc + j) * LD + kr] = rb[q][j];
      }
    }
  };

  f32x16 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][j][r] = 0.f;

  const int nk = g.Kd / BK;
  gload(0);
  swrite(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) gload(kt + 1);
    f32x4 a[FM][2], b[FN][2];
#pragma unroll
    for (int fm = 0; fm < FM; ++fm) {
      const float* pa = &As[cur][(wm * WM + fm * 32 + l32) * LD + h * 8];
      a[fm][0] = *reinterpret_cast<const f32x4*>(pa);
      a[fm][1] = *reinterpret_cast<const f32x4*>(pa + 4);
    }
#pragma unroll
    for (int fn = 0; fn < FN; ++fn) {
      const float* pb = &Bs[cur][(wn * WN + fn * 32 + l32) * LD + h * 8];
      b[fn][0] = *reinterpret_cast<const f32x4*>(pb);
      b[fn][1] = *reinterpret_cast<const f32x4*>(pb + 4);
    }
#pragma unroll
    for (int p = 0; p < 8; ++p)
#pragma unroll
      for (int fm = 0; fm < FM; ++fm)
#pragma unroll
        for (int fn = 0; fn < FN; ++fn)
          acc[fm][fn] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[fm][p >> 2][p & 3], b[fn][p >> 2][p & 3],
                                                              acc[fm][fn], 0, 0, 0);
    if (kt + 1 < nk) swrite(cur ^ 1);
    __syncthreads();
  }

  // Epilogue.  32x32 accumulator layout: lane l, register r holds
  // row 8*(r/4) + 4*(l/32) + r%4 and column l%32 of its fragment.
  __shared__ float red_s[2][BM][2];
#pragma unroll
  for (int fm = 0; fm < FM; ++fm) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = wm * WM + fm * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
      const int m = m0 + row;
      float red[2] = {0.f, 0.f};
      if (m < g.M) {
        const int mr = rowidx ? rowidx[m] : m;
#pragma unroll
        for (int fn = 0; fn < FN; ++fn) {
          const int n = n0 + wn * WN + fn * 32 + l32;
          if (n < g.N) epi.elem(mr, n, acc[fm][fn][r], red);
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
          epi.row_partial(rowidx ? rowidx[m] : m, tile, v);
        }
      }
    }
  }
}

// rowidx (may be null): rows 0 .. g.M - 1 of the product are rows rowidx[m]
// of A and of the epilogue (the active spectra of a batch).
template <int BM, int BN, class Epi>
__global__ __launch_bounds__(256) void gemm_nt_f32(GemmArgs g, Epi epi, const int* __restrict__ rowidx) {
  gemm_nt_f32_tile<BM, BN, Epi>(g, epi, blockIdx.y * BM, blockIdx.x * BN, blockIdx.x, rowidx);
}

// Any of the four operand layouts (see gemm_nt_f32_tile).
template <int BM, int BN, bool TA, bool TB, class Epi>
__global__ __launch_bounds__(256) void gemm_f32_layout(GemmArgs g, Epi epi) {
  gemm_nt_f32_tile<BM, BN, Epi, TA, TB>(g, epi, blockIdx.y * BM, blockIdx.x * BN, blockIdx.x);
}

// Grouped launch: up to GEMM_MAX_GROUPS independent products (each with its
// own operands, sizes and epilogue) in one grid.  Group q owns the linear
// workgroup range [tile0[q], tile0[q+1]); inside it the column tile runs
// fastest, so consecutive workgroups share the A rows and the round-robin
// placement of workgroups on the chip's 8 XCDs gives each XCD a fixed subset of
// the Bt column blocks, which then stay in that XCD's L2.  Groups are ordered
// by the caller (largest products first) so that the long tiles start first.
constexpr int GEMM_MAX_GROUPS = 8;
template <class Epi>
struct GemmGroups {
  int ngroups;
  int tile0[GEMM_MAX_GROUPS + 1];
  int ntn[GEMM_MAX_GROUPS];
  int nvalid[GEMM_MAX_GROUPS];  // unpadded N = Kd of the group (work count only)
  GemmArgs g[GEMM_MAX_GROUPS];
  Epi epi[GEMM_MAX_GROUPS];
};

template <int BM, int BN, class Epi>
__global__ __launch_bounds__(256) void gemm_nt_f32_grouped(GemmGroups<Epi> p) {
  const int L = blockIdx.x;
  int q = 0;
#pragma unroll
  for (int i = 1; i < GEMM_MAX_GROUPS; ++i) q += (i < p.ngroups && L >= p.tile0[i]) ? 1 : 0;
  const int t = L - p.tile0[q], tm = t / p.ntn[q], tn = t - tm * p.ntn[q];
  gemm_nt_f32_tile<BM, BN, Epi>(p.g[q], p.epi[q], tm * BM, tn * BN, tn);
}

// Active rows of a grouped product, rebuilt on the device between launches:
// group q multiplies only the nact[q] rows listed at rows[row0[q]..] (row
// numbers inside the group), in tiles tile0[q] .. tile0[q+1] - 1 of the grid.
// The grid is sized for every row; workgroups past tile0[ngroups] exit.
struct GemmActive {
  int nact[GEMM_MAX_GROUPS];
  int row0[GEMM_MAX_GROUPS];
  int tile0[GEMM_MAX_GROUPS + 1];
};

// work (nullable): the launch adds its algorithmic multiply-adds,
// sum_q nact[q] nvalid[q]^2, for profiling.
template <int BM, int BN, class Epi>
__global__ __launch_bounds__(256) void gemm_nt_f32_grouped_active(GemmGroups<Epi> p, const GemmActive* __restrict__ act,
                                                                  const int* __restrict__ rows,
                                                                  unsigned long long* __restrict__ work) {
  const int L = blockIdx.x;
  if (work && L == 0 && threadIdx.x == 0) {
    unsigned long long macs = 0;
    for (int q = 0; q < p.ngroups; ++q)
      macs += (unsigned long long)act->nact[q] * (unsigned long long)p.nvalid[q] * (unsigned long long)p.nvalid[q];
    atomicAdd(work, macs);
  }
  if (L >= act->tile0[p.ngroups]) return;
  int q = 0;
#pragma unroll
  for (int i = 1; i < GEMM_MAX_GROUPS; ++i) q += (i < p.ngroups && L >= act->tile0[i]) ? 1 : 0;
  const int t = L - act->tile0[q], tm = t / p.ntn[q], tn = t - tm * p.ntn[q];
  GemmArgs g = p.g[q];
  g.M = act->nact[q];
  gemm_nt_f32_tile<BM, BN, Epi>(g, p.epi[q], tm * BM, tn * BN, tn, rows + act->row0[q]);
}
