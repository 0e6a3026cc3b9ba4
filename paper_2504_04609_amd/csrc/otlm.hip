// libotlm: C-ABI and host engine of the batched OTLM scaling solver (gfx950).
//
// One call of otlm_solve_batch runs Algorithm 1 ("Scaling Algorithm for OTLM")
// for B spectra that share the Gibbs kernel K and the dictionary D.  Per
// iteration it issues four MFMA GEMM launches, each with the elementwise
// update of that step fused into its epilogue:
//   1. S = V K^T      -> s, r = log(s / a)              (kernel product, Table 2 input)
//   2. G = R D        -> w = wMMstep(...)                (Table 2 / Appendix A)
//   3. A = W D^T      -> a = D w, u = a / s              (source scaling)
//   4. T = U K        -> v = prox_L(t | y) / t           (Table 1, target scaling)
// and, every check_every iterations, one convergence kernel whose active-count
// is the only value read back by the host inside the loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/otlm.h"
#include "gemm_nt.hpp"
#include "gemm_nt_f64.hpp"
#include "gemm_nt_bf16.hpp"
#include "objective_kernels.hpp"
#include "prox_newton.hpp"
#include "ragged_kernels.hpp"
#include "mlp_kernels.hpp"
#include "solver_kernels.hpp"
#include "solver_kernels64.hpp"

namespace {

#define OTLM_HIP(call)                                      \
  do {                                                      \
    hipError_t e_ = (call);                                 \
    if (e_ != hipSuccess) {                                 \
      std::fprintf(stderr, "libotlm: %s failed: %s (%s:%d)\n", #call, hipGetErrorString(e_), __FILE__, __LINE__); \
      return OTLM_E_HIP;                                    \
    }                                                       \
  } while (0)

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

struct Workspace {
  int64_t B = 0, np = 0, kp = 0;
  float *V = nullptr, *S = nullptr, *R = nullptr, *A = nullptr, *U = nullptr, *W = nullptr;
  float *Dp = nullptr, *DTp = nullptr;
  float4* colc = nullptr;
  int2* band = nullptr;  // rows of the nonzero entries of each dictionary column
  float *psn = nullptr, *psd = nullptr, *pwn = nullptr, *pwd = nullptr;
  float *pln = nullptr, *pld = nullptr;  // l1 weight change and l1 weights of the last interval (warm-start probe)
  float* Wsnap = nullptr;  // weights at the previous convergence test
  int *done = nullptr, *iters = nullptr, *status = nullptr, *flags = nullptr;
  float* ew_prev = nullptr;
  float* ew_best = nullptr;
  int* stall = nullptr;
  int* nit = nullptr;    // Newton iterations per spectrum, FP32-state prox
  int* nit64 = nullptr;  // the same, FP64-state prox
  int* nfac = nullptr;   // Hessian factorisations per spectrum, FP32-state prox
  int* nfac64 = nullptr; // the same, FP64-state prox
  int* nent = nullptr;   // free-set Hessian entries built per spectrum, FP32-state prox
  int* nent64 = nullptr; // the same, FP64-state prox
  // stored Cholesky factors of the weight prox (factor reuse), allocated on demand
  int64_t fac_B = 0;
  double *Lg = nullptr, *wH = nullptr;
  unsigned long long* maskH = nullptr;
  int* validH = nullptr;
  int* mm_until = nullptr;  // last iteration of each spectrum's MM warm-up (exact weight prox)
  int* xflags = nullptr;    // status bits set on the way: 16 warm start replaced, 32 range promotion
  int* it_base = nullptr;   // per-spectrum offset of refinement-phase iteration indices
  int* act_rows = nullptr;  // active spectra after the last convergence test (compacted products)
  unsigned short *Vbf = nullptr, *Ubf = nullptr;
  // FP64 refinement state
  int64_t B64 = 0;
  double *V64 = nullptr, *S64 = nullptr, *A64 = nullptr, *U64 = nullptr, *W64 = nullptr, *Dp64 = nullptr;
  double* Wsnap64 = nullptr;
  std::vector<void*> allocs64;
  double *os = nullptr, *ot = nullptr, *oq = nullptr;
  int64_t obj_B = 0;
  int* host_flags = nullptr;  // pinned: [0] active count, [1] bad-input flag
  std::vector<void*> allocs;

  void release() {
    for (void* p : allocs) (void)hipFree(p);
    allocs.clear();
    for (void* q : {(void*)Lg, (void*)wH, (void*)maskH, (void*)validH})
      if (q) (void)hipFree(q);
    if (host_flags) (void)hipHostFree(host_flags);
    host_flags = nullptr;
    B = np = kp = 0;
    V = S = R = A = U = W = Dp = DTp = psn = psd = pwn = pwd = pln = pld = Wsnap = nullptr;
    colc = nullptr;
    band = nullptr;
    done = iters = status = flags = nullptr;
    ew_prev = nullptr;
    ew_best = nullptr;
    stall = nullptr;
    nit = nit64 = nfac = nfac64 = nent = nent64 = nullptr;
    fac_B = 0;
    Lg = wH = nullptr;
    maskH = nullptr;
    validH = nullptr;
    mm_until = xflags = it_base = act_rows = nullptr;
    Vbf = Ubf = nullptr;
  }
  void release64() {
    for (void* p : allocs64) (void)hipFree(p);
    allocs64.clear();
    B64 = 0;
    V64 = S64 = A64 = U64 = W64 = Dp64 = Wsnap64 = nullptr;
  }
  void release_obj() {
    if (os) (void)hipFree(os);
    if (ot) (void)hipFree(ot);
    if (oq) (void)hipFree(oq);
    os = ot = oq = nullptr;
    obj_B = 0;
  }
};

// In the exact weight-prox mode the first iterations take the MM step: from a
// cold start s = K 1 carries far more mass than y and an exact prox there
// drives weights to scales that Newton leaves only slowly.
constexpr int OTLM_MM_WARMUP = 3;
// A Newton iteration of the weight prox reuses the spectrum's last Cholesky
// factor while the free set is unchanged and the weights moved by at most this
// fraction of max|w| since it was built (0: always refactor).
#ifndef OTLM_HESS_REUSE
#define OTLM_HESS_REUSE 1e-2
#endif
// Scaled gradient tolerance of the Newton weight prox during an FP32 bulk phase
// that an FP64 refinement will follow (the outer iterate is itself only good to
// ~1e-5 there); the FP64 phase and FP32-only solves use 1e-13.
#ifndef OTLM_BULK_GTOL
#define OTLM_BULK_GTOL 1e-9
#endif
constexpr float OTLM_FP32_FLOOR = 4.76837158e-7f;  // 2^-21: weight changes below it are FP32 noise
constexpr float OTLM_FP64_FLOOR = 1e-13f;          // the same for the FP64 state
constexpr float OTLM_BF16_FLOOR = 3.0e-4f;         // ~2^-12: BF16 products move w by about this much
constexpr int MAX_TILES = 256;
// kernel classes timed by otlm_profile_* (order documented in include/otlm.h)
enum { PROF_KV32 = 0, PROF_W32, PROF_U32, PROF_KTU32, PROF_CHECK, PROF_KV64, PROF_W64, PROF_U64, PROF_KTU64,
       PROF_KVBF, PROF_KTUBF, PROF_WMM32, OTLM_PROF_CLASSES };  // per-row partial slots: np / 64 <= 256 column tiles

}  // namespace

struct otlm_kernel_s {
  int device = 0;
  int64_t n = 0, np = 0;
  double eps = 0.0;
  int symmetric = 0;
  float* K = nullptr;     // [np, np] FP32, zero padded
  float* KT = nullptr;    // == K when symmetric
  double* K64 = nullptr;  // [n, n] FP64
  double* KT64 = nullptr; // == K64 when symmetric
  double* K64p = nullptr;  // [np, np] FP64, zero padded (refinement products)
  unsigned short* Kbf = nullptr;   // [np, np] BF16 (bulk-phase products)
  unsigned short* KTbf = nullptr;  // == Kbf when symmetric
  double* KT64p = nullptr; // == K64p when symmetric
  double sumK = 0.0;
  Workspace ws;
  // kernel timing (otlm_profile_*)
  bool profile = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[OTLM_PROF_CLASSES];
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
  double prof_ms[OTLM_PROF_CLASSES] = {};
  int64_t prof_n[OTLM_PROF_CLASSES] = {};
  int64_t prof_newton[6] = {0, 0, 0, 0, 0, 0};  // weight prox: Newton iterations FP32 / FP64 state, then
                                                 // factorisations, then free-set Hessian entries built
};

namespace {

template <class T>
int dev_alloc(Workspace& ws, T** p, size_t count) {
  void* q = nullptr;
  if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return OTLM_E_NOMEM;
  ws.allocs.push_back(q);
  *p = static_cast<T*>(q);
  return OTLM_OK;
}

int ensure_workspace(otlm_kernel k, int64_t B, int64_t kp) {
  Workspace& ws = k->ws;
  if (ws.B >= B && ws.kp >= kp && ws.np == k->np && ws.host_flags) return OTLM_OK;
  ws.release();
  const int64_t np = k->np;
  const size_t bn = (size_t)B * np, bk = (size_t)B * kp;
  int rc = OTLM_OK;
  rc |= dev_alloc(ws, &ws.V, bn);
  rc |= dev_alloc(ws, &ws.S, bn);
  rc |= dev_alloc(ws, &ws.R, bn);
  rc |= dev_alloc(ws, &ws.A, bn);
  rc |= dev_alloc(ws, &ws.U, bn);
  rc |= dev_alloc(ws, &ws.W, bk);
  rc |= dev_alloc(ws, &ws.Dp, (size_t)np * kp);
  rc |= dev_alloc(ws, &ws.DTp, (size_t)kp * np);
  rc |= dev_alloc(ws, &ws.colc, (size_t)kp);
  rc |= dev_alloc(ws, &ws.band, (size_t)kp);
  rc |= dev_alloc(ws, &ws.psn, (size_t)B * MAX_TILES);
  rc |= dev_alloc(ws, &ws.psd, (size_t)B * MAX_TILES);
  rc |= dev_alloc(ws, &ws.pwn, (size_t)B);
  rc |= dev_alloc(ws, &ws.pwd, (size_t)B);
  rc |= dev_alloc(ws, &ws.pln, (size_t)B);
  rc |= dev_alloc(ws, &ws.pld, (size_t)B);
  rc |= dev_alloc(ws, &ws.Wsnap, bk);
  rc |= dev_alloc(ws, &ws.done, (size_t)B);
  rc |= dev_alloc(ws, &ws.iters, (size_t)B);
  rc |= dev_alloc(ws, &ws.status, (size_t)B);
  rc |= dev_alloc(ws, &ws.flags, 4);
  rc |= dev_alloc(ws, &ws.ew_prev, (size_t)B);
  rc |= dev_alloc(ws, &ws.ew_best, (size_t)B);
  rc |= dev_alloc(ws, &ws.stall, (size_t)B);
  rc |= dev_alloc(ws, &ws.nit, (size_t)B);
  rc |= dev_alloc(ws, &ws.nit64, (size_t)B);
  rc |= dev_alloc(ws, &ws.nfac, (size_t)B);
  rc |= dev_alloc(ws, &ws.nfac64, (size_t)B);
  rc |= dev_alloc(ws, &ws.nent, (size_t)B);
  rc |= dev_alloc(ws, &ws.nent64, (size_t)B);
  rc |= dev_alloc(ws, &ws.mm_until, (size_t)B);
  rc |= dev_alloc(ws, &ws.xflags, (size_t)B);
  rc |= dev_alloc(ws, &ws.it_base, (size_t)B);
  rc |= dev_alloc(ws, &ws.act_rows, (size_t)B);
  rc |= dev_alloc(ws, &ws.Vbf, bn);
  rc |= dev_alloc(ws, &ws.Ubf, bn);
  if (rc != OTLM_OK) {
    ws.release();
    return OTLM_E_NOMEM;
  }
  if (hipHostMalloc((void**)&ws.host_flags, 4 * sizeof(int)) != hipSuccess) {
    ws.release();
    return OTLM_E_NOMEM;
  }
  ws.B = B;
  ws.np = np;
  ws.kp = kp;
  return OTLM_OK;
}

// Tile shapes of the four products (chosen per problem size).
// rowidx (may be null): the g.M product rows are rows rowidx[0 .. g.M) of A
// and of the epilogue.
template <class Epi>
void gemm(int bm, int bn, const GemmArgs& g, const Epi& e, hipStream_t s, const int* rowidx = nullptr) {
  auto launch = [&](auto kern, int BM, int BN) {
    dim3 grid((unsigned)((g.N + BN - 1) / BN), (unsigned)((g.M + BM - 1) / BM));
    hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, g, e, rowidx);
  };
  if (bm == 128 && bn == 128) launch(gemm_nt_f32<128, 128, Epi>, 128, 128);
  else if (bm == 128 && bn == 64) launch(gemm_nt_f32<128, 64, Epi>, 128, 64);
  else if (bm == 64 && bn == 128) launch(gemm_nt_f32<64, 128, Epi>, 64, 128);
  else launch(gemm_nt_f32<64, 64, Epi>, 64, 64);
}

// Bracket one launch with events when profiling is on.
struct ProfScope {
  otlm_kernel k;
  int cls;
  hipStream_t s;
  std::pair<hipEvent_t, hipEvent_t> e{nullptr, nullptr};
  ProfScope(otlm_kernel k_, int cls_, hipStream_t s_) : k(k_), cls(cls_), s(s_) {
    if (!k->profile) return;
    if (!k->ev_pool.empty()) {
      e = k->ev_pool.back();
      k->ev_pool.pop_back();
    } else if (hipEventCreate(&e.first) != hipSuccess || hipEventCreate(&e.second) != hipSuccess) {
      e = {nullptr, nullptr};
      return;
    }
    (void)hipEventRecord(e.first, s);
  }
  ~ProfScope() {
    if (!e.first) return;
    (void)hipEventRecord(e.second, s);
    k->ev[cls].push_back(e);
  }
};

// Fold recorded event pairs into the running means (synchronises the events).
void prof_collect(otlm_kernel k) {
  for (int c = 0; c < OTLM_PROF_CLASSES; ++c) {
    for (auto& e : k->ev[c]) {
      float ms = 0.f;
      if (hipEventSynchronize(e.second) == hipSuccess && hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) {
        k->prof_ms[c] += ms;
        k->prof_n[c] += 1;
      }
      k->ev_pool.push_back(e);
    }
    k->ev[c].clear();
  }
}

bool params_valid(const otlm_params* p, double kernel_eps) {
  if (!p) return false;
  if (!(p->eps > 0.0) || std::fabs(p->eps - kernel_eps) > 1e-12 * kernel_eps) return false;
  if (!(p->lambda >= 0.0) || !(p->lambda2 >= 0.0) || !(p->alpha >= 0.0) || !(p->beta >= 0.0)) return false;
  if (!(p->tol >= 0.0) || p->max_iter < 1 || p->check_every < 1) return false;
  if (p->fit < OTLM_FIT_BALANCED || p->fit > OTLM_FIT_POISSON) return false;
  if (p->pen < OTLM_PEN_NONE || p->pen > OTLM_PEN_ELASTIC) return false;
  if (p->pen == OTLM_PEN_L2SQ && !(p->alpha > 0.0)) return false;
  if (p->pen == OTLM_PEN_ELASTIC && !(p->beta > 0.0)) return false;
  if ((p->fit == OTLM_FIT_L2 || p->fit == OTLM_FIT_L2_TV || p->fit == OTLM_FIT_POISSON) && !(p->lambda > 0.0))
    return false;
  if (p->warm != 0 && p->warm != 1) return false;
  if (p->wstep != OTLM_WSTEP_MM && p->wstep != OTLM_WSTEP_EXACT) return false;
  if (p->wstep == OTLM_WSTEP_EXACT && p->inner_max < 1) return false;
  if (p->prec != OTLM_PREC_FP32 && p->prec != OTLM_PREC_BF16) return false;
  if (p->refine < OTLM_REFINE_NONE || p->refine > OTLM_REFINE_FP64) return false;
  if (p->refine != OTLM_REFINE_NONE && p->refine_sweeps < 1) return false;
  if (p->refine_check_every < 0) return false;
  if (!(p->bulk_tol >= 0.0) || !(p->warm_probe >= 0.0) || !(p->absorb_tau >= 0.0)) return false;
  return true;
}

}  // namespace

extern "C" {

void otlm_default_params(otlm_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->eps = 1.0;
  p->lambda = 1.0;
  p->tol = 1e-6;
  p->max_iter = 1000;
  p->check_every = 10;
  p->fit = OTLM_FIT_KL;
  p->pen = OTLM_PEN_NONE;
  p->prec = OTLM_PREC_FP32;
  p->refine = OTLM_REFINE_NONE;
  p->refine_sweeps = 200;
  p->bulk_tol = 1e-4;
  p->absorb_tau = 30.0;
  p->wstep = OTLM_WSTEP_MM;
  p->inner_max = 5;
  p->refine_check_every = 2;
}

const char* otlm_status_str(int code) {
  switch (code) {
    case OTLM_OK: return "ok";
    case OTLM_E_INVALID: return "invalid argument";
    case OTLM_E_HIP: return "HIP runtime error";
    case OTLM_E_NOMEM: return "out of device memory";
    case OTLM_E_UNSUPPORTED: return "unsupported request";
  }
  return "unknown status";
}

int otlm_make_kernel(const double* C, int64_t n, double eps, void* stream, otlm_kernel* out) {
  if (!C || !out || n < 1 || n > 16384 || !(eps > 0.0) || !std::isfinite(eps)) return OTLM_E_INVALID;
  *out = nullptr;
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto* k = new (std::nothrow) otlm_kernel_s();
  if (!k) return OTLM_E_NOMEM;
  OTLM_HIP(hipGetDevice(&k->device));
  k->n = n;
  k->np = round_up(n, 64);
  k->eps = eps;
  // symmetry test on the host (C is read once at set-up)
  std::vector<double> hc((size_t)n * n);
  if (hipMemcpyAsync(hc.data(), C, hc.size() * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    delete k;
    return OTLM_E_HIP;
  }
  bool sym = true, finite = true;
  for (int64_t i = 0; i < n && finite; ++i)
    for (int64_t j = 0; j < n; ++j) {
      const double c = hc[(size_t)i * n + j];
      if (std::isnan(c) || c == -INFINITY) { finite = false; break; }
      if (j > i && c != hc[(size_t)j * n + i]) sym = false;
    }
  if (!finite) {
    delete k;
    return OTLM_E_INVALID;
  }
  k->symmetric = sym ? 1 : 0;
  const size_t npp = (size_t)k->np * k->np;
  if (hipMalloc(&k->K, npp * sizeof(float)) != hipSuccess ||
      hipMalloc(&k->K64, (size_t)n * n * sizeof(double)) != hipSuccess ||
      hipMalloc(&k->K64p, npp * sizeof(double)) != hipSuccess ||
      hipMalloc(&k->Kbf, npp * sizeof(unsigned short)) != hipSuccess) {
    otlm_free_kernel(k);
    return OTLM_E_NOMEM;
  }
  if (sym) {
    k->KT = k->K;
    k->KT64 = k->K64;
    k->KT64p = k->K64p;
    k->KTbf = k->Kbf;
  } else if (hipMalloc(&k->KT, npp * sizeof(float)) != hipSuccess ||
             hipMalloc(&k->KT64, (size_t)n * n * sizeof(double)) != hipSuccess ||
             hipMalloc(&k->KT64p, npp * sizeof(double)) != hipSuccess ||
             hipMalloc(&k->KTbf, npp * sizeof(unsigned short)) != hipSuccess) {
    otlm_free_kernel(k);
    return OTLM_E_NOMEM;
  }
  const double inv = 1.0 / eps;
  dim3 g32((unsigned)((k->np + 255) / 256), (unsigned)k->np), g64((unsigned)((n + 255) / 256), (unsigned)n);
  hipLaunchKernelGGL(build_kernel_f32, g32, dim3(256), 0, s, C, (int)n, (int)k->np, inv, 0, k->K);
  hipLaunchKernelGGL(build_kernel_f64, g64, dim3(256), 0, s, C, (int)n, inv, 0, k->K64);
  hipLaunchKernelGGL(build_kernel_f64p, g32, dim3(256), 0, s, C, (int)n, (int)k->np, inv, 0, k->K64p);
  hipLaunchKernelGGL(build_kernel_bf16, g32, dim3(256), 0, s, C, (int)n, (int)k->np, inv, 0, k->Kbf);
  if (!sym) {
    hipLaunchKernelGGL(build_kernel_f32, g32, dim3(256), 0, s, C, (int)n, (int)k->np, inv, 1, k->KT);
    hipLaunchKernelGGL(build_kernel_f64, g64, dim3(256), 0, s, C, (int)n, inv, 1, k->KT64);
    hipLaunchKernelGGL(build_kernel_f64p, g32, dim3(256), 0, s, C, (int)n, (int)k->np, inv, 1, k->KT64p);
    hipLaunchKernelGGL(build_kernel_bf16, g32, dim3(256), 0, s, C, (int)n, (int)k->np, inv, 1, k->KTbf);
  }
  if (hipGetLastError() != hipSuccess) {
    otlm_free_kernel(k);
    return OTLM_E_HIP;
  }
  double sum = 0.0;
  for (size_t i = 0; i < hc.size(); ++i) sum += std::exp(-hc[i] * inv);
  k->sumK = sum;
  if (hipStreamSynchronize(s) != hipSuccess) {
    otlm_free_kernel(k);
    return OTLM_E_HIP;
  }
  *out = k;
  return OTLM_OK;
}

int otlm_profile_enable(otlm_kernel k, int32_t on) {
  if (!k) return OTLM_E_INVALID;
  prof_collect(k);
  for (int c = 0; c < OTLM_PROF_CLASSES; ++c) {
    k->prof_ms[c] = 0.0;
    k->prof_n[c] = 0;
  }
  for (int q = 0; q < 6; ++q) k->prof_newton[q] = 0;
  k->profile = on != 0;
  return OTLM_OK;
}

int otlm_profile_read(otlm_kernel k, double* ms, int64_t* count, int64_t* newton_iters) {
  if (!k) return OTLM_E_INVALID;
  prof_collect(k);
  if (newton_iters)
    for (int q = 0; q < 6; ++q) newton_iters[q] = k->prof_newton[q];
  for (int c = 0; c < OTLM_PROF_CLASSES; ++c) {
    if (ms) ms[c] = k->prof_n[c] ? k->prof_ms[c] / (double)k->prof_n[c] : 0.0;
    if (count) count[c] = k->prof_n[c];
  }
  return OTLM_OK;
}

int otlm_free_kernel(otlm_kernel k) {
  if (!k) return OTLM_OK;
  (void)hipDeviceSynchronize();
  prof_collect(k);
  for (auto& e : k->ev_pool) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  k->ws.release();
  k->ws.release64();
  k->ws.release_obj();
  if (k->KT64p && k->KT64p != k->K64p) (void)hipFree(k->KT64p);
  if (k->KTbf && k->KTbf != k->Kbf) (void)hipFree(k->KTbf);
  if (k->Kbf) (void)hipFree(k->Kbf);
  if (k->K64p) (void)hipFree(k->K64p);
  if (k->KT && k->KT != k->K) (void)hipFree(k->KT);
  if (k->K) (void)hipFree(k->K);
  if (k->KT64 && k->KT64 != k->K64) (void)hipFree(k->KT64);
  if (k->K64) (void)hipFree(k->K64);
  delete k;
  return OTLM_OK;
}

int otlm_kernel_info(otlm_kernel k, int64_t* n, int32_t* symmetric, double* eps) {
  if (!k) return OTLM_E_INVALID;
  if (n) *n = k->n;
  if (symmetric) *symmetric = k->symmetric;
  if (eps) *eps = k->eps;
  return OTLM_OK;
}

int otlm_solve_batch(otlm_kernel k, const float* D, int64_t kdim, const float* Y, int64_t B,
                     const otlm_params* p, float* W, float* logU, float* logV, int32_t* iters,
                     int32_t* status, void* stream) {
  if (!k || !params_valid(p, k->eps)) return OTLM_E_INVALID;
  if (B < 0 || kdim < 1 || kdim > 256) return OTLM_E_INVALID;
  if (B == 0) return OTLM_OK;
  if (!D || !Y || !W || !logV) return OTLM_E_INVALID;
  if (B > (1 << 24)) return OTLM_E_INVALID;
  const bool exact = p->wstep == OTLM_WSTEP_EXACT;
  const bool fp64 = p->refine == OTLM_REFINE_FP64;
  if (exact && (kdim > PN_K || prox_newton_smem((int)k->n, sizeof(double)) > PN_LDS_MAX)) return OTLM_E_UNSUPPORTED;
  if (exact) {  // the Newton kernels take more than the default 64 KB of dynamic LDS
    const size_t sm32 = prox_newton_smem((int)k->n, sizeof(float)), sm64 = prox_newton_smem((int)k->n, sizeof(double));
    if (hipFuncSetAttribute((const void*)prox_newton_kernel<float, float, double, PN_MAXB>,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm32) != hipSuccess ||
        (fp64 && hipFuncSetAttribute((const void*)prox_newton_kernel<double, double, double, PN_MAXB>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm64) != hipSuccess))
      return OTLM_E_HIP;
  }
  if (fp64 && !exact) return OTLM_E_UNSUPPORTED;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t n = k->n, np = k->np, kp = round_up(kdim, 64);
  int rc = ensure_workspace(k, B, kp);
  if (rc != OTLM_OK) return rc;
  Workspace& ws = k->ws;
  if (fp64 && ws.B64 < B) {
    ws.release64();
    const size_t bn = (size_t)B * np;
    auto al = [&](double** q, size_t c) {
      void* v = nullptr;
      if (hipMalloc(&v, c * sizeof(double)) != hipSuccess) return false;
      ws.allocs64.push_back(v);
      *q = static_cast<double*>(v);
      return true;
    };
    if (!al(&ws.V64, bn) || !al(&ws.S64, bn) || !al(&ws.A64, bn) || !al(&ws.U64, bn) ||
        !al(&ws.W64, (size_t)B * kp) || !al(&ws.Dp64, (size_t)np * kp) || !al(&ws.Wsnap64, (size_t)B * kp)) {
      ws.release64();
      return OTLM_E_NOMEM;
    }
    ws.B64 = B;
  }

  OTLM_HIP(hipMemsetAsync(ws.flags, 0, 4 * sizeof(int), s));
  bool reuse = false;
  if (exact) {
    OTLM_HIP(hipMemsetAsync(ws.nit, 0, (size_t)B * sizeof(int), s));
    OTLM_HIP(hipMemsetAsync(ws.nit64, 0, (size_t)B * sizeof(int), s));
    OTLM_HIP(hipMemsetAsync(ws.nfac, 0, (size_t)B * sizeof(int), s));
    OTLM_HIP(hipMemsetAsync(ws.nfac64, 0, (size_t)B * sizeof(int), s));
    OTLM_HIP(hipMemsetAsync(ws.nent, 0, (size_t)B * sizeof(int), s));
    OTLM_HIP(hipMemsetAsync(ws.nent64, 0, (size_t)B * sizeof(int), s));
    if (OTLM_HESS_REUSE > 0.0 && ws.fac_B < B) {  // factor storage: 32 KB per spectrum; without it, no reuse
      for (void* q : {(void*)ws.Lg, (void*)ws.wH, (void*)ws.maskH, (void*)ws.validH})
        if (q) (void)hipFree(q);
      ws.Lg = ws.wH = nullptr;
      ws.maskH = nullptr;
      ws.validH = nullptr;
      ws.fac_B = 0;
      if (hipMalloc(&ws.Lg, (size_t)B * PN_K * PN_K * sizeof(double)) == hipSuccess &&
          hipMalloc(&ws.wH, (size_t)B * 128 * sizeof(double)) == hipSuccess &&
          hipMalloc(&ws.maskH, (size_t)B * 2 * sizeof(unsigned long long)) == hipSuccess &&
          hipMalloc(&ws.validH, (size_t)B * sizeof(int)) == hipSuccess) {
        ws.fac_B = B;
      } else {
        (void)hipGetLastError();
      }
    }
    reuse = OTLM_HESS_REUSE > 0.0 && ws.fac_B >= B;
    if (reuse) OTLM_HIP(hipMemsetAsync(ws.validH, 0, (size_t)B * sizeof(int), s));
  }
  OTLM_HIP(hipMemsetAsync(ws.it_base, 0, (size_t)B * sizeof(int), s));
  hipLaunchKernelGGL(prep_dictionary, dim3((unsigned)kp), dim3(256), 0, s, D, (int)n, (int)kdim, (int)np, (int)kp,
                     p->pen, p->eps, p->alpha, p->beta, ws.Dp, ws.DTp, ws.colc, ws.band, ws.flags + 1);
  hipLaunchKernelGGL(init_state, dim3((unsigned)B), dim3(256), 0, s, Y, (const float*)W, (const float*)logV,
                     (const float4*)ws.colc, (int)n, (int)kdim, (int)np, (int)kp, p->warm, ws.V, ws.W, ws.U,
                     ws.done, ws.status, ws.iters, ws.ew_prev, ws.ew_best, ws.stall, ws.mm_until,
                     exact ? OTLM_MM_WARMUP : 0, ws.xflags, ws.flags + 1);
  OTLM_HIP(hipGetLastError());
  OTLM_HIP(hipMemcpyAsync(ws.host_flags, ws.flags, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  OTLM_HIP(hipStreamSynchronize(s));
  if (ws.host_flags[1]) return OTLM_E_INVALID;  // negative / non-finite D or Y, or an empty column

  const int M = (int)B;
  {  // a = D w for the start
    GemmArgs g{ws.W, (int)kp, ws.Dp, (int)kp, M, (int)np, (int)kp};
    EpiStore e{ws.A, (int)np, (int)n, false};
    gemm(64, 128, g, e, s);
  }
  // 64 x 128 tiles: at B = 4096, n = 1024 the 512 tiles put two workgroups on
  // every CU (128 x 128 tiles give one, with nothing to cover its latencies)
  const int bm_k = 64, bn_k = 128;
  const int nts = (int)((np + bn_k - 1) / bn_k);
  const int bn_w = kp >= 128 ? 128 : 64;
  ProxConsts pc;
  pc.fit = p->fit;
  pc.kappa = (float)(p->lambda / (p->lambda + p->eps));
  pc.lam_eps = (float)(p->lambda / p->eps);
  pc.lam2_eps = (float)(p->lambda2 / p->eps);
  pc.eps_lam = p->lambda > 0 ? (float)(p->eps / p->lambda) : 0.f;
  pc.log_lam_eps = p->lambda > 0 ? (float)std::log(p->lambda / p->eps) : 0.f;
  ProxConsts64 pc64;
  pc64.fit = p->fit;
  pc64.kappa = p->lambda / (p->lambda + p->eps);
  pc64.lam_eps = p->lambda / p->eps;
  pc64.lam2_eps = p->lambda2 / p->eps;
  pc64.eps_lam = p->lambda > 0 ? p->eps / p->lambda : 0.0;
  pc64.log_lam_eps = p->lambda > 0 ? std::log(p->lambda / p->eps) : 0.0;

  auto prox_args32 = [&]() {
    ProxNewtonArgs<float, float> a;
    a.S = ws.S; a.W = ws.W; a.Dp = ws.Dp; a.DTp = ws.DTp; a.ld_dt = (int)np; a.colc = ws.colc; a.done = ws.done;
    a.mm_until = ws.mm_until; a.it = 0;
    a.nfac = ws.nfac; a.nent = ws.nent; a.flops = nullptr; a.Lg = reuse ? ws.Lg : nullptr; a.lg_stride = (size_t)PN_K * PN_K * sizeof(double); a.wH = ws.wH; a.maskH = ws.maskH; a.validH = ws.validH;
    a.reuse_tol = OTLM_HESS_REUSE;
    a.rg = nullptr; a.band = ws.band; a.it_dev = nullptr; a.newton_after = 0;
    a.ld_s = (int)np; a.ld_w = (int)kp; a.ld_d = (int)kp; a.n = (int)n; a.k = (int)kdim; a.pen = p->pen;
    a.max_newton = p->inner_max; a.eps = p->eps; a.alpha = p->alpha; a.beta = p->beta;
    a.gtol = fp64 ? OTLM_BULK_GTOL : 1e-13;
    a.nit = ws.nit;
    return a;
  };
  auto prox_args64 = [&]() {
    ProxNewtonArgs<double, double> a;
    a.S = ws.S64; a.W = ws.W64; a.Dp = ws.Dp; a.DTp = ws.DTp; a.ld_dt = (int)np; a.colc = ws.colc; a.done = ws.done;
    a.mm_until = nullptr; a.it = 0;
    a.nfac = ws.nfac64; a.nent = ws.nent64; a.flops = nullptr; a.Lg = reuse ? ws.Lg : nullptr; a.lg_stride = (size_t)PN_K * PN_K * sizeof(double); a.wH = ws.wH; a.maskH = ws.maskH; a.validH = ws.validH;
    a.reuse_tol = OTLM_HESS_REUSE;
    a.rg = nullptr; a.band = ws.band; a.it_dev = nullptr; a.newton_after = 0;
    a.ld_s = (int)np; a.ld_w = (int)kp; a.ld_d = (int)kp; a.n = (int)n; a.k = (int)kdim; a.pen = p->pen;
    a.max_newton = p->inner_max; a.eps = p->eps; a.alpha = p->alpha; a.beta = p->beta; a.gtol = 1e-13;
    a.nit = ws.nit64;
    return a;
  };

  // Last iteration at which some spectrum still takes the MM step in the exact
  // mode (cold starts: OTLM_MM_WARMUP; warm starts: none; a fallback restarts it).
  int mm_until_max = (exact && !p->warm) ? OTLM_MM_WARMUP : 0;
  // Rows of the FP32 / FP64 kernel products: all spectra at the start of a
  // phase, then the active ones listed after each convergence test (spectra
  // that stopped are frozen, so their rows need no products).  The products
  // take 64-row tiles, and K^T u 64 x 64 ones once the active rows fall to half
  // the batch, to keep the tile count up.
  int Ma = M;
  const int* arows = nullptr;
  // One FP32 iteration (bulk phase or FP32 refinement); `it` counts from 1 over the whole solve.
  auto iterate32 = [&](int it, bool chk, bool bf16) {
    const bool mm_step = !exact || it <= mm_until_max;
    {  // s = K v, r = log(s / a)
      EpiSrc e{ws.S, mm_step ? ws.R : nullptr, ws.A, ws.U, ws.psn, ws.psd, (int)np, (int)n, nts, chk};
      if (bf16) {
        ProfScope ps(k, PROF_KVBF, s);
        GemmArgsBf16 g{ws.Vbf, (int)np, k->Kbf, (int)np, M, (int)np, (int)np};
        dim3 grid((unsigned)((np + GB_BN - 1) / GB_BN), (unsigned)((B + 63) / 64));
        hipLaunchKernelGGL((gemm_nt_bf16<EpiSrc, 64>), grid, dim3(256), 0, s, g, e);
      } else {
        ProfScope ps(k, PROF_KV32, s);
        GemmArgs g{ws.V, (int)np, k->K, (int)np, Ma, (int)np, (int)np};
        gemm(bm_k, bn_k, g, e, s, arows);
      }
    }
    if (exact) {  // weight prox solved by active-set Newton (spectra past their MM warm-up)
      ProfScope ps(k, PROF_W32, s);
      auto kern = prox_newton_kernel<float, float, double, PN_MAXB>;
      auto a = prox_args32();
      a.it = it;
      hipLaunchKernelGGL(kern, dim3((unsigned)B), dim3(PN_THREADS), prox_newton_smem((int)n, sizeof(float)), s, a);
    }
    if (mm_step) {  // MM weight step (every spectrum, or those in their warm-up)
      ProfScope ps(k, exact ? PROF_WMM32 : PROF_W32, s);
      GemmArgs g{ws.R, (int)np, ws.DTp, (int)np, Ma, (int)kp, (int)np};
      EpiWupd e{ws.W, ws.colc, ws.done, exact ? ws.mm_until : nullptr, it, (int)kp, (int)kdim, p->pen, false};
      gemm(64, bn_w, g, e, s, arows);
    }
    {  // a = D w, u = a / s
      ProfScope ps(k, PROF_U32, s);
      GemmArgs g{ws.W, (int)kp, ws.Dp, (int)kp, Ma, (int)np, (int)kp};
      EpiUscale e{ws.A, ws.U, ws.S, (int)np, (int)n, false, bf16 ? ws.Ubf : nullptr};
      gemm(64, 128, g, e, s, arows);
    }
    {  // t = K^T u, v = prox(t | y) / t
      EpiProx e{ws.V, Y, ws.done, pc, (int)np, (int)n, (int)n, false, bf16 ? ws.Vbf : nullptr};
      if (bf16) {
        ProfScope ps(k, PROF_KTUBF, s);
        GemmArgsBf16 g{ws.Ubf, (int)np, k->KTbf, (int)np, M, (int)np, (int)np};
        dim3 grid((unsigned)((np + GB_BN - 1) / GB_BN), (unsigned)((B + 63) / 64));
        hipLaunchKernelGGL((gemm_nt_bf16<EpiProx, 64>), grid, dim3(256), 0, s, g, e);
      } else {
        ProfScope ps(k, PROF_KTU32, s);
        GemmArgs g{ws.U, (int)np, k->KT, (int)np, Ma, (int)np, (int)np};
        if (2 * Ma <= M) gemm(64, 64, g, e, s, arows);
        else gemm(bm_k, bn_k, g, e, s, arows);
      }
    }
  };
  // One FP64 iteration (refinement phase, exact weight prox).
  auto iterate64 = [&](int, bool chk) {
    const int ntiles64 = (int)((np + G64_BN - 1) / G64_BN);
    dim3 grid_n((unsigned)((np + G64_BN - 1) / G64_BN), (unsigned)((Ma + G64_BM - 1) / G64_BM));
    {
      ProfScope ps(k, PROF_KV64, s);
      GemmArgs64 g{ws.V64, (int)np, k->K64p, (int)np, Ma, (int)np, (int)np};
      EpiSrc64 e{ws.S64, ws.A64, ws.U64, ws.psn, ws.psd, (int)np, (int)n, ntiles64, chk};
      hipLaunchKernelGGL(gemm_nt_f64<EpiSrc64>, grid_n, dim3(256), 0, s, g, e, arows);
    }
    {
      ProfScope ps(k, PROF_W64, s);
      auto kern = prox_newton_kernel<double, double, double, PN_MAXB>;
      hipLaunchKernelGGL(kern, dim3((unsigned)B), dim3(PN_THREADS),
                         prox_newton_smem((int)n, sizeof(double)), s, prox_args64());
    }
    {
      ProfScope ps(k, PROF_U64, s);
      GemmArgs64 g{ws.W64, (int)kp, ws.Dp64, (int)kp, Ma, (int)np, (int)kp};
      EpiUscale64 e{ws.A64, ws.U64, ws.S64, (int)np, (int)n, false};
      hipLaunchKernelGGL(gemm_nt_f64<EpiUscale64>, grid_n, dim3(256), 0, s, g, e, arows);
    }
    {
      ProfScope ps(k, PROF_KTU64, s);
      GemmArgs64 g{ws.U64, (int)np, k->KT64p, (int)np, Ma, (int)np, (int)np};
      EpiProx64 e{ws.V64, Y, ws.done, pc64, (int)np, (int)n, (int)n, false};
      hipLaunchKernelGGL(gemm_nt_f64<EpiProx64>, grid_n, dim3(256), 0, s, g, e, arows);
    }
  };
  // Runs one phase; returns the last iteration index or a negative status.
  // Weight change since the previous test (init: snapshot at the phase start).
  auto weight_change = [&](bool use64, int init) {
    const dim3 grid((unsigned)((B + 3) / 4));
    if (use64) {
      auto kern = interval_change<double>;
      hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, ws.W64, (int)kp, (int)kdim, M, ws.Wsnap64, init, ws.pwn,
                         ws.pwd, ws.pln, ws.pld);
    } else {
      auto kern = interval_change<float>;
      hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, ws.W, (int)kp, (int)kdim, M, ws.Wsnap, init, ws.pwn, ws.pwd,
                         ws.pln, ws.pld);
    }
  };
  // range promotion of the FP32 bulk phase (needs the FP64 phase to continue in)
  const bool absorb = fp64 && p->absorb_tau > 0.0;
  // probe: test the warm start at the first convergence test of this phase
  auto run_phase = [&](int it0, int cap, double tol, float floor_w, bool use64, bool bf16, int nts_phase,
                       bool probe, int cadence) -> int {
    int it = it0;
    if (tol > 0.0) weight_change(use64, 1);
    bool first_check = true;
    Ma = M;  // every spectrum of the phase is active until its first test
    arows = nullptr;
    for (int j = 1; j <= cap; ++j) {
      it = it0 + j;
      const bool chk = (tol > 0.0) && (j % cadence == 0 || j == cap);
      if (use64) iterate64(it, chk);
      else iterate32(it, chk, bf16);
      if (chk) {
        {
          ProfScope ps(k, PROF_CHECK, s);
          weight_change(use64, 0);
          hipLaunchKernelGGL(check_convergence, dim3(1), dim3(1024), 0, s, ws.psn, ws.psd, nts_phase, ws.pwn, ws.pwd,
                             M, (float)tol, floor_w, it, ws.ew_prev, ws.ew_best, ws.stall, ws.done, ws.iters,
                             ws.status, ws.flags, nullptr, (const int*)ws.it_base);
        }
        const bool fb = probe && first_check;
        if (fb)
          hipLaunchKernelGGL(warm_fallback, dim3((unsigned)B), dim3(256), 0, s, (const float*)ws.pln,
                             (const float*)ws.pld, (float)p->warm_probe, Y, (const float4*)ws.colc, (int)n,
                             (int)kdim, (int)np, (int)kp, it, exact ? OTLM_MM_WARMUP : 0, ws.V,
                             bf16 ? ws.Vbf : nullptr, ws.W, ws.Wsnap, ws.U, ws.done, ws.status, ws.ew_prev,
                             ws.ew_best, ws.stall, ws.mm_until, ws.xflags, ws.flags + 2);
        first_check = false;
        if (absorb && !use64)
          hipLaunchKernelGGL(range_check, dim3((unsigned)((B + 3) / 4)), dim3(256), 0, s, (const float*)ws.U,
                             (const float*)ws.V, (int)n, (int)np, M, (float)p->absorb_tau, it, ws.done, ws.status,
                             ws.iters, ws.xflags, ws.flags);
        // the active list, and its count in flags[0], after every change of done
        hipLaunchKernelGGL(compact_active, dim3(1), dim3(1024), 0, s, (const int*)ws.done, M, ws.act_rows, ws.flags);
        if (hipGetLastError() != hipSuccess) return OTLM_E_HIP;
        if (hipMemcpyAsync(ws.host_flags, ws.flags, 3 * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
          return OTLM_E_HIP;
        Ma = ws.host_flags[0] > 0 ? ws.host_flags[0] : M;
        arows = Ma < M ? ws.act_rows : nullptr;
        if (fb && ws.host_flags[2] > 0) {  // restarted spectra: a = D w0, and their MM warm-up
          GemmArgs g{ws.W, (int)kp, ws.Dp, (int)kp, M, (int)np, (int)kp};
          EpiStore e{ws.A, (int)np, (int)n, false};
          gemm(64, 128, g, e, s);
          if (exact) mm_until_max = it + OTLM_MM_WARMUP;
          continue;
        }
        if (ws.host_flags[0] == 0) break;
      }
    }
    return hipGetLastError() == hipSuccess ? it : OTLM_E_HIP;
  };

  const bool refine = p->refine != OTLM_REFINE_NONE;
  const bool bulk_bf16 = p->prec == OTLM_PREC_BF16;
  if (bulk_bf16) {
    hipLaunchKernelGGL(convert_f32_to_bf16, dim3(1024), dim3(256), 0, s, ws.V, ws.Vbf, (size_t)B * np);
    OTLM_HIP(hipGetLastError());
  }
  const bool probe = p->warm && p->warm_probe > 0.0;
  int last = run_phase(0, p->max_iter, refine ? p->bulk_tol : p->tol, bulk_bf16 ? OTLM_BF16_FLOOR : OTLM_FP32_FLOOR,
                       false, bulk_bf16, nts, probe, p->check_every);
  const int refine_cadence = p->refine_check_every > 0 ? p->refine_check_every : p->check_every;
  if (last < 0) return last;
  bool state64 = false;
  if (refine) {
    hipLaunchKernelGGL(reopen_spectra, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, s, M, last, ws.done,
                       ws.status, (const int*)ws.iters, ws.it_base, ws.ew_prev, ws.ew_best, ws.stall);
    if (fp64) {
      const size_t bn = (size_t)B * np;
      hipLaunchKernelGGL(convert_f32_to_f64, dim3(1024), dim3(256), 0, s, ws.V, ws.V64, bn);
      hipLaunchKernelGGL(convert_f32_to_f64, dim3(1024), dim3(256), 0, s, ws.U, ws.U64, bn);
      hipLaunchKernelGGL(convert_f32_to_f64, dim3(1024), dim3(256), 0, s, ws.A, ws.A64, bn);
      hipLaunchKernelGGL(convert_f32_to_f64, dim3(1024), dim3(256), 0, s, ws.W, ws.W64, (size_t)B * kp);
      hipLaunchKernelGGL(convert_f32_to_f64, dim3(1024), dim3(256), 0, s, ws.Dp, ws.Dp64, (size_t)np * kp);
      OTLM_HIP(hipGetLastError());
      const int nts64 = (int)((np + G64_BN - 1) / G64_BN);
      last = run_phase(std::max(last, mm_until_max), p->refine_sweeps, p->tol, OTLM_FP64_FLOOR, true, false, nts64,
                       false, refine_cadence);
      state64 = true;
    } else {
      last = run_phase(std::max(last, mm_until_max), p->refine_sweeps, p->tol, OTLM_FP32_FLOOR, false, false, nts,
                       false, refine_cadence);
    }
    if (last < 0) return last;
  }
  if (state64)
    hipLaunchKernelGGL(write_outputs64, dim3((unsigned)B), dim3(256), 0, s, ws.W64, ws.U64, ws.V64, ws.done,
                       ws.status, ws.iters, (const int*)ws.xflags, (const int*)ws.it_base, (int)n, (int)kdim, (int)np, (int)kp, last, W, logU, logV, iters, status);
  else
    hipLaunchKernelGGL(write_outputs, dim3((unsigned)B), dim3(256), 0, s, ws.W, ws.U, ws.V, ws.done, ws.status,
                       ws.iters, (const int*)ws.xflags, (const int*)ws.it_base, (int)n, (int)kdim, (int)np, (int)kp, last, W, logU, logV, iters, status);
  OTLM_HIP(hipGetLastError());
  if (k->profile && exact) {  // Newton iteration count for the roofline of the prox kernel
    std::vector<int> h((size_t)B);
    std::vector<int> h64((size_t)B), f32((size_t)B), f64((size_t)B), e32((size_t)B), e64((size_t)B);
    OTLM_HIP(hipMemcpyAsync(h.data(), ws.nit, (size_t)B * sizeof(int), hipMemcpyDeviceToHost, s));
    OTLM_HIP(hipMemcpyAsync(h64.data(), ws.nit64, (size_t)B * sizeof(int), hipMemcpyDeviceToHost, s));
    OTLM_HIP(hipMemcpyAsync(f32.data(), ws.nfac, (size_t)B * sizeof(int), hipMemcpyDeviceToHost, s));
    OTLM_HIP(hipMemcpyAsync(f64.data(), ws.nfac64, (size_t)B * sizeof(int), hipMemcpyDeviceToHost, s));
    OTLM_HIP(hipMemcpyAsync(e32.data(), ws.nent, (size_t)B * sizeof(int), hipMemcpyDeviceToHost, s));
    OTLM_HIP(hipMemcpyAsync(e64.data(), ws.nent64, (size_t)B * sizeof(int), hipMemcpyDeviceToHost, s));
    OTLM_HIP(hipStreamSynchronize(s));
    for (int v : h) k->prof_newton[0] += v;
    for (int v : h64) k->prof_newton[1] += v;
    for (int v : f32) k->prof_newton[2] += v;
    for (int v : f64) k->prof_newton[3] += v;
    for (int v : e32) k->prof_newton[4] += v;
    for (int v : e64) k->prof_newton[5] += v;
  }
  return OTLM_OK;
}

int otlm_objective(otlm_kernel k, const double* C, const float* D, int64_t kdim, const float* Y, int64_t B,
                   const otlm_params* p, const float* W, const float* logU, const float* logV, double* out,
                   void* stream) {
  if (!k || !params_valid(p, k->eps)) return OTLM_E_INVALID;
  if (B < 0 || kdim < 1 || kdim > 256) return OTLM_E_INVALID;
  if (B == 0) return OTLM_OK;
  if (!C || !D || !Y || !W || !logU || !logV || !out) return OTLM_E_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Workspace& ws = k->ws;
  const int64_t n = k->n;
  if (ws.obj_B < B) {
    ws.release_obj();
    if (hipMalloc(&ws.os, (size_t)B * n * sizeof(double)) != hipSuccess ||
        hipMalloc(&ws.ot, (size_t)B * n * sizeof(double)) != hipSuccess ||
        hipMalloc(&ws.oq, (size_t)B * n * sizeof(double)) != hipSuccess) {
      ws.release_obj();
      return OTLM_E_NOMEM;
    }
    ws.obj_B = B;
  }
  hipLaunchKernelGGL(objective_products, dim3((unsigned)((n + 3) / 4), (unsigned)B), dim3(256), 0, s, k->K64,
                     k->KT64, C, logU, logV, (int)n, ws.os, ws.ot, ws.oq);
  ObjParams op{(int)n, (int)kdim, p->fit, p->pen, p->eps, p->lambda, p->lambda2, p->alpha, p->beta, k->sumK};
  hipLaunchKernelGGL(objective_reduce, dim3((unsigned)B), dim3(256), 0, s, op, D, Y, W, logU, logV, ws.os, ws.ot,
                     ws.oq, out);
  OTLM_HIP(hipGetLastError());
  return OTLM_OK;
}

}  // extern "C"

#include "ragged.hpp"
#include "mlp.hpp"
