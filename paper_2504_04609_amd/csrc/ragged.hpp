// Host engine of the ragged batch (otlm_ragged_*): part of the libotlm
// translation unit, included at the end of otlm.hip.
//
// A plan fixes the batch structure (which Gibbs kernel, hence grid, each
// spectrum uses and its dictionary size), the parameters and the GEMM tile
// shape.  It groups the spectra by kernel (largest n first), lays the
// per-spectrum state out as one [rows, np] block per group, picks the tile
// shape of the grouped kernel products by timing the candidates on the real
// shapes, and captures one check interval of Algorithm 1 (check_every
// iterations plus the convergence test) as a HIP graph.  A solve then copies
// the caller's dictionaries and targets into the plan's layout and replays the
// graph until every spectrum has stopped; the host reads back one integer per
// interval.

namespace {

constexpr int RG_TILES[4][2] = {{128, 128}, {128, 64}, {64, 128}, {64, 64}};
enum { RG_PROF_KV = 0, RG_PROF_W, RG_PROF_KTU, RG_PROF_CHECK, RG_PROF_NEWTON, RG_PROF_CLASSES };
// Newton prox of the ragged path: inner iterations per launch and scaled
// gradient tolerance (FP32 state, a and log(a/s) held in FP32).
constexpr int RG_NEWTON_MAX = 5;
constexpr double RG_NEWTON_GTOL = 1e-7;
constexpr size_t RG_LG_STRIDE = 65536;  // bytes of stored factor per spectrum: 64^2 FP64 or 128^2 FP32

}  // namespace

struct otlm_ragged_s {
  int device = 0;
  int64_t B = 0;
  otlm_params p{};
  ProxConsts pc{};
  struct Group {
    const otlm_kernel_s* K;
    int n, np, rows;
    int64_t row0, base;  // first spectrum (solve order) and offset of its row in the state arrays
  };
  int ngroups = 0;
  Group grp[GEMM_MAX_GROUPS];
  std::vector<RgSpec> hspec;
  int64_t tot_state = 0, tot_cols = 0, tot_dt = 0, tot_bins = 0;
  int npmax = 0, ts = 0;  // largest row stride; partial slots per spectrum (np / 64)
  RgSpec* spec = nullptr;
  float *V = nullptr, *S = nullptr, *A = nullptr, *U = nullptr, *Yg = nullptr, *Wst = nullptr, *DT = nullptr;
  float* Wsnap = nullptr;  // weights at the previous convergence test
  GemmActive* act = nullptr;  // active rows of the grouped products (device)
  int* nband = nullptr;       // band entries of each spectrum's dictionary
  // Newton prox of the spectra still active after newton_after iterations (k <= 64, n <= 2048)
  int newton_after = -1;
  int n_newton = 0, nmax64 = 0, nmax128 = 0;  // spectra that may take it; largest n with k <= 64 / k > 64
  size_t smem64 = 0, smem128 = 0;
  int64_t tot_dp = 0;
  float* Dp = nullptr;
  PnSpec* pnspec = nullptr;
  double *Lg = nullptr, *wH = nullptr;
  unsigned long long* maskH = nullptr;
  int *validH = nullptr, *nit = nullptr, *nfac = nullptr;
  unsigned long long* work = nullptr;  // profiling: [0] kernel-product MACs, [1] weight-step bytes, [2] Newton flops
  int* act_rows = nullptr;
  RgGroups gi{};
  float4* colc = nullptr;
  int2* band = nullptr;
  float *psn = nullptr, *psd = nullptr, *pwn = nullptr, *pwd = nullptr, *ew_prev = nullptr, *ew_best = nullptr;
  int *done = nullptr, *iters = nullptr, *status = nullptr, *flags = nullptr, *stall = nullptr, *it_dev = nullptr;
  int* host_flags = nullptr;
  int64_t bytes = 0;
  int tile = 0;
  double tune_ms[4] = {};
  bool use_graph = true;
  hipStream_t cap = nullptr;
  hipGraphExec_t exec = nullptr;
  int exec_c = 0;
  std::vector<void*> allocs;
  bool profile = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[RG_PROF_CLASSES], pool;
  double prof_ms[RG_PROF_CLASSES] = {};
  int64_t prof_n[RG_PROF_CLASSES] = {};

  template <class T>
  bool alloc(T** q, size_t count) {
    void* v = nullptr;
    if (hipMalloc(&v, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return false;
    allocs.push_back(v);
    bytes += (int64_t)(std::max<size_t>(count, 1) * sizeof(T));
    *q = static_cast<T*>(v);
    return true;
  }
  void release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    exec = nullptr;
    if (cap) (void)hipStreamDestroy(cap);
    cap = nullptr;
    for (void* v : allocs) (void)hipFree(v);
    allocs.clear();
    if (host_flags) (void)hipHostFree(host_flags);
    host_flags = nullptr;
    for (int c = 0; c < RG_PROF_CLASSES; ++c) {
      for (auto& e : ev[c]) pool.push_back(e);
      ev[c].clear();
    }
    for (auto& e : pool) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    pool.clear();
  }
};

namespace {

struct RgProfScope {
  otlm_ragged_s* r;
  int cls;
  hipStream_t s;
  std::pair<hipEvent_t, hipEvent_t> e{nullptr, nullptr};
  RgProfScope(otlm_ragged_s* r_, int cls_, hipStream_t s_) : r(r_), cls(cls_), s(s_) {
    if (!r->profile) return;
    if (!r->pool.empty()) {
      e = r->pool.back();
      r->pool.pop_back();
    } else if (hipEventCreate(&e.first) != hipSuccess || hipEventCreate(&e.second) != hipSuccess) {
      e = {nullptr, nullptr};
      return;
    }
    (void)hipEventRecord(e.first, s);
  }
  ~RgProfScope() {
    if (!e.first) return;
    (void)hipEventRecord(e.second, s);
    r->ev[cls].push_back(e);
  }
};

void rg_prof_collect(otlm_ragged_s* r) {
  for (int c = 0; c < RG_PROF_CLASSES; ++c) {
    for (auto& e : r->ev[c]) {
      float ms = 0.f;
      if (hipEventSynchronize(e.second) == hipSuccess && hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) {
        r->prof_ms[c] += ms;
        r->prof_n[c] += 1;
      }
      r->pool.push_back(e);
    }
    r->ev[c].clear();
  }
}

// Grouped product over every group: transposed = false gives S = V K^T (A
// operand V), true gives T = U K (operand U, Bt = K^T).
template <class Epi, class MakeEpi>
GemmGroups<Epi> rg_groups(const otlm_ragged_s* r, int bm, int bn, bool transposed, const float* Aop, MakeEpi mk) {
  GemmGroups<Epi> gg{};
  gg.ngroups = r->ngroups;
  int t = 0;
  for (int g = 0; g < GEMM_MAX_GROUPS; ++g) {
    gg.tile0[g] = t;
    if (g >= r->ngroups) continue;
    const auto& G = r->grp[g];
    const int ntm = (G.rows + bm - 1) / bm, ntn = (G.np + bn - 1) / bn;
    gg.ntn[g] = ntn;
    gg.nvalid[g] = G.n;
    gg.g[g] = GemmArgs{Aop + G.base, G.np, transposed ? G.K->KT : G.K->K, G.np, G.rows, G.np, G.np};
    gg.epi[g] = mk(g);
    t += ntm * ntn;
  }
  gg.tile0[GEMM_MAX_GROUPS] = t;
  return gg;
}

// Grouped product over the active rows; the grid covers every row and the
// workgroups beyond the active tiles exit.
template <class Epi>
void rg_launch(const otlm_ragged_s* r, int tile, const GemmGroups<Epi>& gg, hipStream_t s) {
  const dim3 grid((unsigned)gg.tile0[GEMM_MAX_GROUPS]), block(256);
  unsigned long long* work = r->profile ? r->work : nullptr;
  if (tile == 0) {
    auto kern = gemm_nt_f32_grouped_active<128, 128, Epi>;
    hipLaunchKernelGGL(kern, grid, block, 0, s, gg, (const GemmActive*)r->act, (const int*)r->act_rows, work);
  } else if (tile == 1) {
    auto kern = gemm_nt_f32_grouped_active<128, 64, Epi>;
    hipLaunchKernelGGL(kern, grid, block, 0, s, gg, (const GemmActive*)r->act, (const int*)r->act_rows, work);
  } else if (tile == 2) {
    auto kern = gemm_nt_f32_grouped_active<64, 128, Epi>;
    hipLaunchKernelGGL(kern, grid, block, 0, s, gg, (const GemmActive*)r->act, (const int*)r->act_rows, work);
  } else {
    auto kern = gemm_nt_f32_grouped_active<64, 64, Epi>;
    hipLaunchKernelGGL(kern, grid, block, 0, s, gg, (const GemmActive*)r->act, (const int*)r->act_rows, work);
  }
}

// Rebuild the active-row lists for tile shape `tile` from the done flags.
void rg_compact_rows(otlm_ragged_s* r, int tile, hipStream_t s) {
  hipLaunchKernelGGL(rg_compact, dim3(1), dim3(1024), 0, s, (const int*)r->done, r->gi, RG_TILES[tile][0],
                     RG_TILES[tile][1], r->act, r->act_rows);
}

void rg_product_s(otlm_ragged_s* r, int tile, bool chk, hipStream_t s) {
  auto gg = rg_groups<EpiSrc>(r, RG_TILES[tile][0], RG_TILES[tile][1], false, r->V, [&](int g) {
    const auto& G = r->grp[g];
    return EpiSrc{r->S + G.base, nullptr, r->A + G.base, r->U + G.base, r->psn + G.row0 * r->ts,
                  r->psd + G.row0 * r->ts, G.np, G.n, r->ts, chk};
  });
  rg_launch(r, tile, gg, s);
}

void rg_product_t(otlm_ragged_s* r, int tile, hipStream_t s) {
  auto gg = rg_groups<EpiProx>(r, RG_TILES[tile][0], RG_TILES[tile][1], true, r->U, [&](int g) {
    const auto& G = r->grp[g];
    return EpiProx{r->V + G.base, r->Yg + G.base, r->done + G.row0, r->pc, G.np, G.np, G.n, false, nullptr};
  });
  rg_launch(r, tile, gg, s);
}

// One outer iteration of Algorithm 1 over the whole ragged batch.
void rg_iterate(otlm_ragged_s* r, bool chk, hipStream_t s) {
  {
    RgProfScope ps(r, RG_PROF_KV, s);
    rg_product_s(r, r->tile, chk, s);
  }
  if (r->n_newton > 0) {
    RgProfScope ps(r, RG_PROF_NEWTON, s);
    ProxNewtonArgs<float, float> a{};
    a.S = r->S; a.W = r->Wst; a.Dp = r->Dp; a.DTp = r->DT; a.colc = r->colc; a.done = r->done;
    a.mm_until = nullptr; a.it = 0; a.nit = r->nit; a.nfac = r->nfac;
    a.Lg = r->Lg; a.lg_stride = RG_LG_STRIDE; a.wH = r->wH; a.maskH = r->maskH; a.validH = r->validH;
    a.reuse_tol = OTLM_HESS_REUSE;
    a.rg = r->pnspec; a.band = r->band; a.it_dev = r->it_dev; a.newton_after = r->newton_after;
    a.flops = r->profile ? r->work + 2 : nullptr;
    a.pen = r->p.pen; a.max_newton = RG_NEWTON_MAX; a.eps = r->p.eps; a.alpha = r->p.alpha; a.beta = r->p.beta;
    a.gtol = RG_NEWTON_GTOL;
    if (r->nmax64) {
      auto kern = prox_newton_kernel<float, float, float, PN_MAXB_RAGGED, 64, double>;
      hipLaunchKernelGGL(kern, dim3((unsigned)r->B), dim3(PN_THREADS), r->smem64, s, a);
    }
    if (r->nmax128) {
      auto kern = prox_newton_kernel<float, float, float, PN_MAXB_RAGGED, 128, float>;
      hipLaunchKernelGGL(kern, dim3((unsigned)r->B), dim3(PN_THREADS), r->smem128, s, a);
    }
  }
  {
    RgProfScope ps(r, RG_PROF_W, s);
    hipLaunchKernelGGL(rg_weight_step, dim3((unsigned)r->B), dim3(RG_WS_THREADS), 3 * (size_t)r->npmax * sizeof(float),
                       s, r->spec, r->DT, r->colc, r->band, r->p.pen, r->p.inner_max, r->S, r->A, r->U, r->Wst,
                       r->done, (const int*)r->nband, r->profile ? r->work + 1 : nullptr, (const int*)r->it_dev,
                       r->n_newton > 0 ? r->newton_after : -1);
  }
  {
    RgProfScope ps(r, RG_PROF_KTU, s);
    rg_product_t(r, r->tile, s);
  }
}

// One check interval: c iterations, the last one accumulating the convergence
// partials, then the convergence test (when a tolerance is set) and the new
// active-row lists.
void rg_chunk(otlm_ragged_s* r, int c, hipStream_t s) {
  const bool test = r->p.tol > 0.0;
  hipLaunchKernelGGL(rg_advance, dim3(1), dim3(64), 0, s, r->it_dev, c);
  for (int j = 1; j <= c; ++j) rg_iterate(r, test && j == c, s);
  if (test) {
    RgProfScope ps(r, RG_PROF_CHECK, s);
    hipLaunchKernelGGL(rg_interval_change, dim3((unsigned)((r->B + 3) / 4)), dim3(256), 0, s, r->spec, (int)r->B,
                       r->Wst, r->Wsnap, 0, r->pwn, r->pwd);
    hipLaunchKernelGGL(check_convergence, dim3(1), dim3(1024), 0, s, r->psn, r->psd, r->ts, r->pwn, r->pwd,
                       (int)r->B, (float)r->p.tol, OTLM_FP32_FLOOR, 0, r->ew_prev, r->ew_best, r->stall, r->done,
                       r->iters, r->status, r->flags, r->it_dev, (const int*)nullptr);
    rg_compact_rows(r, r->tile, s);
  }
}

int rg_autotune(otlm_ragged_s* r, int forced, hipStream_t s) {
  if (forced >= 0) {
    r->tile = forced;
    return OTLM_OK;
  }
  hipEvent_t e0, e1;
  OTLM_HIP(hipEventCreate(&e0));
  OTLM_HIP(hipEventCreate(&e1));
  int best = 0;
  for (int t = 0; t < 4; ++t) {
    rg_compact_rows(r, t, s);
    rg_product_s(r, t, false, s);
    (void)hipEventRecord(e0, s);
    for (int rep = 0; rep < 3; ++rep) rg_product_s(r, t, false, s);
    (void)hipEventRecord(e1, s);
    float ms = 0.f;
    if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return OTLM_E_HIP;
    }
    r->tune_ms[t] = ms / 3.0;
    if (r->tune_ms[t] < r->tune_ms[best]) best = t;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  r->tile = best;
  return hipGetLastError() == hipSuccess ? OTLM_OK : OTLM_E_HIP;
}

int rg_capture(otlm_ragged_s* r, int c) {
  if (r->exec) (void)hipGraphExecDestroy(r->exec);
  r->exec = nullptr;
  if (!r->cap) OTLM_HIP(hipStreamCreateWithFlags(&r->cap, hipStreamNonBlocking));
  const bool prof = r->profile;
  r->profile = false;
  OTLM_HIP(hipStreamBeginCapture(r->cap, hipStreamCaptureModeThreadLocal));
  rg_chunk(r, c, r->cap);
  hipGraph_t graph = nullptr;
  const hipError_t e = hipStreamEndCapture(r->cap, &graph);
  r->profile = prof;
  if (e != hipSuccess || !graph) {
    std::fprintf(stderr, "libotlm: graph capture failed: %s\n", hipGetErrorString(e));
    return OTLM_E_HIP;
  }
  const hipError_t ei = hipGraphInstantiate(&r->exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (ei != hipSuccess) {
    r->exec = nullptr;
    std::fprintf(stderr, "libotlm: graph instantiation failed: %s\n", hipGetErrorString(ei));
    return OTLM_E_HIP;
  }
  r->exec_c = c;
  return OTLM_OK;
}

}  // namespace

extern "C" {

void otlm_ragged_default_opts(otlm_ragged_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->use_graph = 1;
  o->tile = -1;
  o->newton_after = 15;
}

int otlm_ragged_create(const otlm_kernel* kernels, int32_t nkernels, const int32_t* kernel_of, const int32_t* kdim,
                       int64_t B, const otlm_params* p, const otlm_ragged_opts* opts, void* stream,
                       otlm_ragged* out) {
  if (!out) return OTLM_E_INVALID;
  *out = nullptr;
  if (!kernels || !kernel_of || !kdim || !p || nkernels < 1 || nkernels > GEMM_MAX_GROUPS) return OTLM_E_INVALID;
  if (B < 1 || B > (1 << 22)) return OTLM_E_INVALID;
  otlm_ragged_opts o;
  otlm_ragged_default_opts(&o);
  if (opts) o = *opts;
  if (o.tile < -1 || o.tile > 3 || o.newton_after < -1) return OTLM_E_INVALID;
  for (int g = 0; g < nkernels; ++g) {
    if (!kernels[g] || !params_valid(p, kernels[g]->eps)) return OTLM_E_INVALID;
    if (kernels[g]->n > RG_MAX_N) return OTLM_E_UNSUPPORTED;
  }
  if (p->wstep != OTLM_WSTEP_MM || p->prec != OTLM_PREC_FP32 || p->refine != OTLM_REFINE_NONE)
    return OTLM_E_UNSUPPORTED;
  if (p->inner_max < 1 || p->inner_max > 64) return OTLM_E_INVALID;
  std::vector<int64_t> used(nkernels, 0);
  for (int64_t b = 0; b < B; ++b) {
    if (kernel_of[b] < 0 || kernel_of[b] >= nkernels || kdim[b] < 1 || kdim[b] > RG_MAX_K) return OTLM_E_INVALID;
    used[kernel_of[b]] += 1;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto* r = new (std::nothrow) otlm_ragged_s();
  if (!r) return OTLM_E_NOMEM;
  auto fail = [&](int rc) {
    r->release();
    delete r;
    return rc;
  };
  if (hipGetDevice(&r->device) != hipSuccess) return fail(OTLM_E_HIP);
  r->B = B;
  r->p = *p;
  r->use_graph = o.use_graph != 0;
  r->newton_after = o.newton_after;
  r->pc.fit = p->fit;
  r->pc.kappa = (float)(p->lambda / (p->lambda + p->eps));
  r->pc.lam_eps = (float)(p->lambda / p->eps);
  r->pc.lam2_eps = (float)(p->lambda2 / p->eps);
  r->pc.eps_lam = p->lambda > 0 ? (float)(p->eps / p->lambda) : 0.f;
  r->pc.log_lam_eps = p->lambda > 0 ? (float)std::log(p->lambda / p->eps) : 0.f;

  // groups: kernels in use, the largest n first
  std::vector<int> order;
  for (int g = 0; g < nkernels; ++g)
    if (used[g]) order.push_back(g);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return kernels[a]->n > kernels[b]->n; });
  std::vector<int> group_of_kernel(nkernels, -1);
  r->ngroups = (int)order.size();
  int64_t row0 = 0, base = 0;
  for (int g = 0; g < r->ngroups; ++g) {
    const otlm_kernel_s* K = kernels[order[g]];
    group_of_kernel[order[g]] = g;
    r->grp[g] = {K, (int)K->n, (int)K->np, (int)used[order[g]], row0, base};
    r->gi.row0[g] = (int)row0;
    r->gi.rows[g] = (int)used[order[g]];
    r->gi.np[g] = (int)K->np;
    row0 += used[order[g]];
    base += used[order[g]] * K->np;
    r->npmax = std::max(r->npmax, (int)K->np);
  }
  r->tot_state = base;
  r->gi.ngroups = r->ngroups;
  r->ts = (r->npmax + 63) / 64;
  // offsets of the packed inputs (input order)
  std::vector<int64_t> yin(B), din(B), win(B);
  int64_t oy = 0, od = 0, ow = 0;
  for (int64_t b = 0; b < B; ++b) {
    const int64_t n = kernels[kernel_of[b]]->n;
    yin[b] = oy;
    din[b] = od;
    win[b] = ow;
    oy += n;
    od += n * kdim[b];
    ow += kdim[b];
  }
  r->tot_bins = oy;
  r->tot_cols = ow;
  r->tot_dt = od;
  // solve order
  r->hspec.resize(B);
  std::vector<int64_t> next_row(r->ngroups);
  for (int g = 0; g < r->ngroups; ++g) next_row[g] = r->grp[g].row0;
  std::vector<int64_t> q_of(B);
  for (int64_t b = 0; b < B; ++b) q_of[b] = next_row[group_of_kernel[kernel_of[b]]]++;
  std::vector<int64_t> b_of(B);
  for (int64_t b = 0; b < B; ++b) b_of[q_of[b]] = b;
  int64_t odt = 0, ocol = 0, odp = 0;
  for (int64_t q = 0; q < B; ++q) {
    const int64_t b = b_of[q];
    const int g = group_of_kernel[kernel_of[b]];
    const auto& G = r->grp[g];
    RgSpec& sp = r->hspec[q];
    sp.b = (int)b;
    sp.n = G.n;
    sp.k = kdim[b];
    sp.np = G.np;
    sp.st = G.base + (q - G.row0) * G.np;
    sp.yin = yin[b];
    sp.din = din[b];
    sp.dt = odt;
    sp.col = ocol;
    sp.win = win[b];
    odt += (int64_t)G.n * kdim[b];
    ocol += kdim[b];
    sp.dp = -1;
    if (r->newton_after >= 0 && sp.k <= 128 && sp.n <= PN_THREADS * PN_MAXB_RAGGED) {
      sp.dp = odp;
      odp += (int64_t)sp.n * (sp.k <= 64 ? 64 : 128);
      r->n_newton += 1;
      if (sp.k <= 64) r->nmax64 = std::max(r->nmax64, sp.n);
      else r->nmax128 = std::max(r->nmax128, sp.n);
    }
  }
  r->tot_dp = odp;
  r->smem64 = r->nmax64 ? prox_newton_smem<64, double>(r->nmax64, sizeof(float), sizeof(float)) : 0;
  r->smem128 = r->nmax128 ? prox_newton_smem<128, float>(r->nmax128, sizeof(float), sizeof(float)) : 0;
  if (r->smem64 > 65536 &&
      hipFuncSetAttribute((const void*)prox_newton_kernel<float, float, float, PN_MAXB_RAGGED, 64, double>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)r->smem64) != hipSuccess)
    return fail(OTLM_E_HIP);
  if (r->smem128 > 65536 &&
      hipFuncSetAttribute((const void*)prox_newton_kernel<float, float, float, PN_MAXB_RAGGED, 128, float>,
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)r->smem128) != hipSuccess)
    return fail(OTLM_E_HIP);
  std::vector<PnSpec> hpn(B);
  for (int64_t q = 0; q < B; ++q) {
    const RgSpec& sp = r->hspec[q];
    hpn[q] = PnSpec{sp.st, sp.col, sp.dp, sp.dt, sp.n, sp.k};
  }

  bool ok = r->alloc(&r->spec, B) && r->alloc(&r->V, r->tot_state) && r->alloc(&r->S, r->tot_state) &&
            r->alloc(&r->A, r->tot_state) && r->alloc(&r->U, r->tot_state) && r->alloc(&r->Yg, r->tot_state) &&
            r->alloc(&r->Wst, r->tot_cols) && r->alloc(&r->Wsnap, r->tot_cols) && r->alloc(&r->DT, r->tot_dt) && r->alloc(&r->colc, r->tot_cols) &&
            r->alloc(&r->band, r->tot_cols) && r->alloc(&r->psn, B * r->ts) && r->alloc(&r->psd, B * r->ts) &&
            r->alloc(&r->pwn, B) && r->alloc(&r->pwd, B) && r->alloc(&r->ew_prev, B) && r->alloc(&r->ew_best, B) &&
            r->alloc(&r->done, B) && r->alloc(&r->iters, B) && r->alloc(&r->status, B) && r->alloc(&r->flags, 4) &&
            r->alloc(&r->stall, B) && r->alloc(&r->it_dev, 1) && r->alloc(&r->act, 1) &&
            r->alloc(&r->act_rows, B) && r->alloc(&r->nband, B) && r->alloc(&r->work, 3) &&
            r->alloc(&r->Dp, r->tot_dp) && r->alloc(&r->pnspec, B) && r->alloc(&r->nit, B) &&
            r->alloc(&r->nfac, B) && r->alloc(&r->validH, B) && r->alloc(&r->maskH, 2 * B) &&
            r->alloc(&r->wH, r->n_newton ? B * 128 : 1) &&
            r->alloc(&r->Lg, r->n_newton ? (size_t)B * (RG_LG_STRIDE / sizeof(double)) : 1);
  if (!ok) return fail(OTLM_E_NOMEM);
  if (hipHostMalloc((void**)&r->host_flags, 4 * sizeof(int)) != hipSuccess) return fail(OTLM_E_NOMEM);
  const size_t sb = (size_t)r->tot_state * sizeof(float);
  if (hipMemcpyAsync(r->spec, r->hspec.data(), (size_t)B * sizeof(RgSpec), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(r->pnspec, hpn.data(), (size_t)B * sizeof(PnSpec), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemsetAsync(r->nit, 0, (size_t)B * sizeof(int), s) != hipSuccess ||
      hipMemsetAsync(r->nfac, 0, (size_t)B * sizeof(int), s) != hipSuccess ||
      hipMemsetAsync(r->V, 0, sb, s) != hipSuccess || hipMemsetAsync(r->A, 0, sb, s) != hipSuccess ||
      hipMemsetAsync(r->U, 0, sb, s) != hipSuccess || hipMemsetAsync(r->done, 0, (size_t)B * sizeof(int), s) != hipSuccess)
    return fail(OTLM_E_HIP);
  int rc = rg_autotune(r, o.tile, s);
  if (rc != OTLM_OK) return fail(rc);
  // partial slots beyond a group's column tiles are never written: keep them 0
  if (hipMemsetAsync(r->psn, 0, (size_t)B * r->ts * sizeof(float), s) != hipSuccess ||
      hipMemsetAsync(r->psd, 0, (size_t)B * r->ts * sizeof(float), s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(OTLM_E_HIP);
  if (r->use_graph) {
    rc = rg_capture(r, std::min(p->check_every, p->max_iter));
    if (rc != OTLM_OK) return fail(rc);
  }
  *out = r;
  return OTLM_OK;
}

int otlm_ragged_solve(otlm_ragged r, const float* D, const float* Y, float* W, float* logU, float* logV,
                      int32_t* iters, int32_t* status, void* stream) {
  if (!r || !D || !Y || !W || !logV) return OTLM_E_INVALID;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != r->device) return OTLM_E_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const otlm_params& p = r->p;
  OTLM_HIP(hipMemsetAsync(r->flags, 0, 4 * sizeof(int), s));
  OTLM_HIP(hipMemsetAsync(r->it_dev, 0, sizeof(int), s));
  hipLaunchKernelGGL(rg_prep_dict, dim3((unsigned)r->B), dim3(RG_THREADS), 0, s, r->spec, D, p.pen, p.eps, p.alpha,
                     p.beta, r->DT, r->Dp, r->colc, r->band, r->nband, r->flags + 1);
  OTLM_HIP(hipMemsetAsync(r->validH, 0, (size_t)r->B * sizeof(int), s));
  hipLaunchKernelGGL(rg_init, dim3((unsigned)r->B), dim3(RG_THREADS), (size_t)r->npmax * sizeof(float), s, r->spec, Y,
                     (const float*)W, (const float*)logV, r->DT, r->colc, r->band, p.warm, r->Yg, r->V, r->U, r->A,
                     r->Wst, r->done, r->status, r->iters, r->ew_prev, r->ew_best, r->stall, r->flags + 1);
  hipLaunchKernelGGL(rg_interval_change, dim3((unsigned)((r->B + 3) / 4)), dim3(256), 0, s, r->spec, (int)r->B, r->Wst,
                     r->Wsnap, 1, r->pwn, r->pwd);
  rg_compact_rows(r, r->tile, s);
  OTLM_HIP(hipGetLastError());
  OTLM_HIP(hipMemcpyAsync(r->host_flags, r->flags, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  OTLM_HIP(hipStreamSynchronize(s));
  if (r->host_flags[1]) return OTLM_E_INVALID;  // negative / non-finite D or Y, or an empty column

  const int c = std::min(p.check_every, p.max_iter);
  const bool graph = r->use_graph && r->exec && !r->profile && r->exec_c == c;
  int last = 0;
  while (last < p.max_iter) {
    const int cc = std::min(c, p.max_iter - last);
    if (graph && cc == c) OTLM_HIP(hipGraphLaunch(r->exec, s));
    else rg_chunk(r, cc, s);
    OTLM_HIP(hipGetLastError());
    last += cc;
    if (p.tol > 0.0) {
      OTLM_HIP(hipMemcpyAsync(r->host_flags, r->flags, sizeof(int), hipMemcpyDeviceToHost, s));
      OTLM_HIP(hipStreamSynchronize(s));
      if (r->host_flags[0] == 0) break;
    }
  }
  hipLaunchKernelGGL(rg_write_outputs, dim3((unsigned)r->B), dim3(RG_THREADS), 0, s, r->spec, r->Wst, r->U, r->V,
                     r->done, r->status, r->iters, last, W, logU, logV, iters, status);
  OTLM_HIP(hipGetLastError());
  return OTLM_OK;
}

int otlm_ragged_info(otlm_ragged r, int32_t* tile_bm, int32_t* tile_bn, double* tune_ms, int64_t* sizes) {
  if (!r) return OTLM_E_INVALID;
  if (tile_bm) *tile_bm = RG_TILES[r->tile][0];
  if (tile_bn) *tile_bn = RG_TILES[r->tile][1];
  if (tune_ms)
    for (int t = 0; t < 4; ++t) tune_ms[t] = r->tune_ms[t];
  if (sizes) {
    sizes[0] = r->tot_bins;
    sizes[1] = r->tot_cols;
    sizes[2] = r->tot_dt;
    sizes[3] = r->bytes;
  }
  return OTLM_OK;
}

int otlm_ragged_profile_enable(otlm_ragged r, int32_t on) {
  if (!r) return OTLM_E_INVALID;
  rg_prof_collect(r);
  OTLM_HIP(hipMemset(r->work, 0, 3 * sizeof(unsigned long long)));
  for (int c = 0; c < RG_PROF_CLASSES; ++c) {
    r->prof_ms[c] = 0.0;
    r->prof_n[c] = 0;
  }
  r->profile = on != 0;
  return OTLM_OK;
}

int otlm_ragged_profile_read(otlm_ragged r, double* ms, int64_t* count, int64_t* work) {
  if (!r) return OTLM_E_INVALID;
  rg_prof_collect(r);
  if (work) {
    unsigned long long h[3] = {0, 0, 0};
    OTLM_HIP(hipDeviceSynchronize());
    OTLM_HIP(hipMemcpy(h, r->work, sizeof(h), hipMemcpyDeviceToHost));
    work[0] = (int64_t)h[0];
    work[1] = (int64_t)h[1];
    work[2] = (int64_t)h[2];
  }
  for (int c = 0; c < RG_PROF_CLASSES; ++c) {
    if (ms) ms[c] = r->prof_n[c] ? r->prof_ms[c] / (double)r->prof_n[c] : 0.0;
    if (count) count[c] = r->prof_n[c];
  }
  return OTLM_OK;
}

int otlm_ragged_free(otlm_ragged r) {
  if (!r) return OTLM_OK;
  (void)hipDeviceSynchronize();
  rg_prof_collect(r);
  r->release();
  delete r;
  return OTLM_OK;
}

}  // extern "C"
