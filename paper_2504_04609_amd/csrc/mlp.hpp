// Host engine of the warm-start network (otlm_mlp_*): part of the libotlm
// translation unit, included at the end of otlm.hip.
//
// The object owns the FP32 parameters, their gradient and AdamW moments, BF16
// copies of the weight matrices for inference, the standardisation statistics
// and an activation workspace sized for the largest batch seen.  Training is
// driven by the caller one minibatch at a time (row indices into a training set
// that stays in device memory); every step runs 3 forward GEMMs, 5 backward
// GEMMs, 3 bias reductions, the loss reduction and one AdamW update.

struct otlm_mlp_s {
  int device = 0;
  int dims[4] = {0, 0, 0, 0};
  int64_t nparam = 0;
  int64_t off[6] = {};  // W1, b1, W2, b2, W3, b3
  float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  unsigned short* wbf = nullptr;  // BF16 W1 | W2 | W3
  bool bf_valid = false;
  float *in_mu = nullptr, *in_sd = nullptr, *out_mu = nullptr, *out_sd = nullptr;
  float* out_w = nullptr;  // loss weight of every output
  int64_t step = 0;
  // activation workspace for `cap` rows
  int64_t cap = 0;
  float *X = nullptr, *Z1 = nullptr, *H1 = nullptr, *Z2 = nullptr, *H2 = nullptr;
  float *dZ1 = nullptr, *dZ2 = nullptr, *dZ3 = nullptr, *part = nullptr;
  unsigned short *Xbf = nullptr, *H1bf = nullptr, *H2bf = nullptr;
  std::vector<void*> allocs, ws_allocs;

  void release_ws() {
    for (void* p : ws_allocs) (void)hipFree(p);
    ws_allocs.clear();
    cap = 0;
  }
  void release() {
    release_ws();
    for (void* p : allocs) (void)hipFree(p);
    allocs.clear();
  }
};

namespace {

constexpr int MLP_BN = 64;  // column tile of the training GEMMs (loss partial slots per row)

template <class T>
bool mlp_alloc(std::vector<void*>& list, T** q, size_t count) {
  void* v = nullptr;
  if (hipMalloc(&v, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess) return false;
  list.push_back(v);
  *q = static_cast<T*>(v);
  return true;
}

int mlp_ensure_ws(otlm_mlp_s* m, int64_t rows) {
  if (m->cap >= rows) return OTLM_OK;
  m->release_ws();
  const int in = m->dims[0], h1 = m->dims[1], h2 = m->dims[2], out = m->dims[3];
  auto& L = m->ws_allocs;
  const size_t r = (size_t)rows;
  bool ok = mlp_alloc(L, &m->X, r * in) && mlp_alloc(L, &m->Z1, r * h1) && mlp_alloc(L, &m->H1, r * h1) &&
            mlp_alloc(L, &m->Z2, r * h2) && mlp_alloc(L, &m->H2, r * h2) && mlp_alloc(L, &m->dZ1, r * h1) &&
            mlp_alloc(L, &m->dZ2, r * h2) && mlp_alloc(L, &m->dZ3, r * out) &&
            mlp_alloc(L, &m->part, r * ((out + MLP_BN - 1) / MLP_BN)) && mlp_alloc(L, &m->Xbf, r * in) &&
            mlp_alloc(L, &m->H1bf, r * h1) && mlp_alloc(L, &m->H2bf, r * h2);
  if (!ok) {
    m->release_ws();
    return OTLM_E_NOMEM;
  }
  m->cap = rows;
  return OTLM_OK;
}

template <bool TA, bool TB, class Epi>
void mlp_gemm(const GemmArgs& g, const Epi& e, hipStream_t s) {
  auto kern = gemm_f32_layout<64, MLP_BN, TA, TB, Epi>;
  const dim3 grid((unsigned)((g.N + MLP_BN - 1) / MLP_BN), (unsigned)((g.M + 63) / 64));
  hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, g, e);
}

// Forward and backward of one minibatch: rows idx[0..B) of X [*, in] and T [*, out];
// fills m->grad and, when loss is not null, the mean squared error.
int mlp_forward_backward(otlm_mlp_s* m, const float* Xraw, const float* T, const int* idx, int B, float* loss,
                         hipStream_t s) {
  const int in = m->dims[0], h1 = m->dims[1], h2 = m->dims[2], out = m->dims[3];
  const float* W1 = m->theta + m->off[0];
  const float* b1 = m->theta + m->off[1];
  const float* W2 = m->theta + m->off[2];
  const float* b2 = m->theta + m->off[3];
  const float* W3 = m->theta + m->off[4];
  const float* b3 = m->theta + m->off[5];
  const int ntiles = (out + MLP_BN - 1) / MLP_BN;
  hipLaunchKernelGGL(mlp_gather_norm, dim3((unsigned)B), dim3(256), 0, s, Xraw, in, idx, B, in,
                     (const float*)m->in_mu, (const float*)m->in_sd, m->X, (unsigned short*)nullptr);
  mlp_gemm<false, false>(GemmArgs{m->X, in, W1, in, B, h1, in}, EpiBiasGelu{b1, m->Z1, m->H1, nullptr, h1, false}, s);
  mlp_gemm<false, false>(GemmArgs{m->H1, h1, W2, h1, B, h2, h1}, EpiBiasGelu{b2, m->Z2, m->H2, nullptr, h2, false},
                         s);
  mlp_gemm<false, false>(GemmArgs{m->H2, h2, W3, h2, B, out, h2},
                         EpiLossOut{b3, T, idx, out, m->out_mu, m->out_sd, m->out_w, m->dZ3, out,
                                    (float)(2.0 / ((double)B * out)), m->part, ntiles, true},
                         s);
  // backward
  float* g = m->grad;
  mlp_gemm<true, true>(GemmArgs{m->dZ3, out, m->H2, h2, out, h2, B}, EpiStore{g + m->off[4], h2, h2, false}, s);
  hipLaunchKernelGGL(mlp_col_sum, dim3((unsigned)((out + 255) / 256)), dim3(256), 0, s, (const float*)m->dZ3, B, out,
                     g + m->off[5]);
  mlp_gemm<false, true>(GemmArgs{m->dZ3, out, W3, h2, B, h2, out}, EpiGeluBack{m->Z2, m->dZ2, h2, false}, s);
  mlp_gemm<true, true>(GemmArgs{m->dZ2, h2, m->H1, h1, h2, h1, B}, EpiStore{g + m->off[2], h1, h1, false}, s);
  hipLaunchKernelGGL(mlp_col_sum, dim3((unsigned)((h2 + 255) / 256)), dim3(256), 0, s, (const float*)m->dZ2, B, h2,
                     g + m->off[3]);
  mlp_gemm<false, true>(GemmArgs{m->dZ2, h2, W2, h1, B, h1, h2}, EpiGeluBack{m->Z1, m->dZ1, h1, false}, s);
  mlp_gemm<true, true>(GemmArgs{m->dZ1, h1, m->X, in, h1, in, B}, EpiStore{g + m->off[0], in, in, false}, s);
  hipLaunchKernelGGL(mlp_col_sum, dim3((unsigned)((h1 + 255) / 256)), dim3(256), 0, s, (const float*)m->dZ1, B, h1,
                     g + m->off[1]);
  if (loss)
    hipLaunchKernelGGL(mlp_loss_reduce, dim3(1), dim3(256), 0, s, (const float*)m->part, B * ntiles,
                       1.0 / ((double)B * out), loss);
  return hipGetLastError() == hipSuccess ? OTLM_OK : OTLM_E_HIP;
}

bool mlp_check_train_args(otlm_mlp_s* m, const float* X, const float* T, const int32_t* idx, int64_t B) {
  return m && X && T && idx && B >= 16 && B % 16 == 0 && B <= (1 << 20);
}

}  // namespace

extern "C" {

int otlm_mlp_create(const int32_t* dims, const float* theta, void* stream, otlm_mlp* out) {
  if (!out) return OTLM_E_INVALID;
  *out = nullptr;
  if (!dims || !theta) return OTLM_E_INVALID;
  for (int l = 0; l < 3; ++l)
    if (dims[l] < 32 || dims[l] > 16384 || dims[l] % 32) return OTLM_E_INVALID;
  if (dims[3] < 16 || dims[3] > 65536 || dims[3] % 16) return OTLM_E_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  auto* m = new (std::nothrow) otlm_mlp_s();
  if (!m) return OTLM_E_NOMEM;
  auto fail = [&](int rc) {
    m->release();
    delete m;
    return rc;
  };
  if (hipGetDevice(&m->device) != hipSuccess) return fail(OTLM_E_HIP);
  for (int l = 0; l < 4; ++l) m->dims[l] = dims[l];
  int64_t o = 0;
  for (int l = 0; l < 3; ++l) {
    m->off[2 * l] = o;
    o += (int64_t)dims[l + 1] * dims[l];
    m->off[2 * l + 1] = o;
    o += dims[l + 1];
  }
  m->nparam = o;
  const int64_t nw = (int64_t)dims[1] * dims[0] + (int64_t)dims[2] * dims[1] + (int64_t)dims[3] * dims[2];
  auto& L = m->allocs;
  if (!(mlp_alloc(L, &m->theta, o) && mlp_alloc(L, &m->grad, o) && mlp_alloc(L, &m->m, o) &&
        mlp_alloc(L, &m->v, o) && mlp_alloc(L, &m->wbf, nw) && mlp_alloc(L, &m->in_mu, dims[0]) &&
        mlp_alloc(L, &m->in_sd, dims[0]) && mlp_alloc(L, &m->out_mu, dims[3]) && mlp_alloc(L, &m->out_sd, dims[3]) &&
        mlp_alloc(L, &m->out_w, dims[3])))
    return fail(OTLM_E_NOMEM);
  std::vector<float> zeros(std::max(dims[0], dims[3]), 0.f), ones(std::max(dims[0], dims[3]), 1.f);
  if (hipMemcpyAsync(m->theta, theta, (size_t)o * sizeof(float), hipMemcpyDefault, s) != hipSuccess ||
      hipMemsetAsync(m->m, 0, (size_t)o * sizeof(float), s) != hipSuccess ||
      hipMemsetAsync(m->v, 0, (size_t)o * sizeof(float), s) != hipSuccess ||
      hipMemsetAsync(m->grad, 0, (size_t)o * sizeof(float), s) != hipSuccess ||
      hipMemcpyAsync(m->in_mu, zeros.data(), dims[0] * sizeof(float), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(m->in_sd, ones.data(), dims[0] * sizeof(float), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(m->out_mu, zeros.data(), dims[3] * sizeof(float), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(m->out_sd, ones.data(), dims[3] * sizeof(float), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(m->out_w, ones.data(), dims[3] * sizeof(float), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(OTLM_E_HIP);
  *out = m;
  return OTLM_OK;
}

int otlm_mlp_info(otlm_mlp m, int32_t* dims, int64_t* nparam, int64_t* step) {
  if (!m) return OTLM_E_INVALID;
  if (dims)
    for (int l = 0; l < 4; ++l) dims[l] = m->dims[l];
  if (nparam) *nparam = m->nparam;
  if (step) *step = m->step;
  return OTLM_OK;
}

int otlm_mlp_set_norm(otlm_mlp m, const float* X, const float* T, int64_t N, void* stream) {
  if (!m || !X || !T || N < 1) return OTLM_E_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nchunk = 64;
  const int cmax = std::max(m->dims[0], m->dims[3]);
  double *s1 = nullptr, *s2 = nullptr;
  if (hipMalloc(&s1, (size_t)nchunk * cmax * sizeof(double)) != hipSuccess) return OTLM_E_NOMEM;
  if (hipMalloc(&s2, (size_t)nchunk * cmax * sizeof(double)) != hipSuccess) {
    (void)hipFree(s1);
    return OTLM_E_NOMEM;
  }
  auto stats = [&](const float* A, int cols, float clamp, float* mu, float* sd) {
    hipLaunchKernelGGL(mlp_stats_partial, dim3((unsigned)((cols + 255) / 256), (unsigned)nchunk), dim3(256), 0, s, A,
                       (long long)N, cols, nchunk, clamp, s1, s2);
    hipLaunchKernelGGL(mlp_stats_final, dim3((unsigned)((cols + 255) / 256)), dim3(256), 0, s, (const double*)s1,
                       (const double*)s2, (long long)N, cols, nchunk, mu, sd);
  };
  stats(X, m->dims[0], 0.f, m->in_mu, m->in_sd);
  stats(T, m->dims[3], MLP_T_CLAMP, m->out_mu, m->out_sd);
  const hipError_t e1 = hipGetLastError();
  const hipError_t e2 = hipStreamSynchronize(s);
  (void)hipFree(s1);
  (void)hipFree(s2);
  return (e1 == hipSuccess && e2 == hipSuccess) ? OTLM_OK : OTLM_E_HIP;
}

int otlm_mlp_set_loss_weights(otlm_mlp m, const float* weights, void* stream) {
  if (!m || !weights) return OTLM_E_INVALID;
  std::vector<float> h((size_t)m->dims[3]);
  hipStream_t s = static_cast<hipStream_t>(stream);
  OTLM_HIP(hipMemcpyAsync(h.data(), weights, h.size() * sizeof(float), hipMemcpyDefault, s));
  OTLM_HIP(hipStreamSynchronize(s));
  for (float w : h)
    if (!(w >= 0.f) || !std::isfinite(w)) return OTLM_E_INVALID;
  OTLM_HIP(hipMemcpyAsync(m->out_w, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice, s));
  OTLM_HIP(hipStreamSynchronize(s));
  return OTLM_OK;
}

int otlm_mlp_set_norm_stats(otlm_mlp m, const float* in_mu, const float* in_sd, const float* out_mu,
                            const float* out_sd, void* stream) {
  if (!m || !in_mu || !in_sd || !out_mu || !out_sd) return OTLM_E_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t bi = (size_t)m->dims[0] * sizeof(float), bo = (size_t)m->dims[3] * sizeof(float);
  std::vector<float> sd((size_t)std::max(m->dims[0], m->dims[3]));
  for (int pass = 0; pass < 2; ++pass) {  // standard deviations must be positive and finite
    const size_t cnt = pass ? (size_t)m->dims[3] : (size_t)m->dims[0];
    OTLM_HIP(hipMemcpyAsync(sd.data(), pass ? out_sd : in_sd, cnt * sizeof(float), hipMemcpyDefault, s));
    OTLM_HIP(hipStreamSynchronize(s));
    for (size_t i = 0; i < cnt; ++i)
      if (!(sd[i] > 0.f) || !std::isfinite(sd[i])) return OTLM_E_INVALID;
  }
  OTLM_HIP(hipMemcpyAsync(m->in_mu, in_mu, bi, hipMemcpyDefault, s));
  OTLM_HIP(hipMemcpyAsync(m->in_sd, in_sd, bi, hipMemcpyDefault, s));
  OTLM_HIP(hipMemcpyAsync(m->out_mu, out_mu, bo, hipMemcpyDefault, s));
  OTLM_HIP(hipMemcpyAsync(m->out_sd, out_sd, bo, hipMemcpyDefault, s));
  OTLM_HIP(hipStreamSynchronize(s));
  return OTLM_OK;
}

int otlm_mlp_get_norm(otlm_mlp m, float* in_mu, float* in_sd, float* out_mu, float* out_sd, void* stream) {
  if (!m) return OTLM_E_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const size_t bi = (size_t)m->dims[0] * sizeof(float), bo = (size_t)m->dims[3] * sizeof(float);
  if (in_mu) OTLM_HIP(hipMemcpyAsync(in_mu, m->in_mu, bi, hipMemcpyDefault, s));
  if (in_sd) OTLM_HIP(hipMemcpyAsync(in_sd, m->in_sd, bi, hipMemcpyDefault, s));
  if (out_mu) OTLM_HIP(hipMemcpyAsync(out_mu, m->out_mu, bo, hipMemcpyDefault, s));
  if (out_sd) OTLM_HIP(hipMemcpyAsync(out_sd, m->out_sd, bo, hipMemcpyDefault, s));
  return OTLM_OK;
}

int otlm_mlp_grad(otlm_mlp m, const float* X, const float* T, const int32_t* idx, int64_t B, float* grad,
                  float* loss, void* stream) {
  if (!mlp_check_train_args(m, X, T, idx, B)) return OTLM_E_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc = mlp_ensure_ws(m, B);
  if (rc != OTLM_OK) return rc;
  rc = mlp_forward_backward(m, X, T, idx, (int)B, loss, s);
  if (rc != OTLM_OK) return rc;
  if (grad) OTLM_HIP(hipMemcpyAsync(grad, m->grad, (size_t)m->nparam * sizeof(float), hipMemcpyDefault, s));
  return OTLM_OK;
}

int otlm_mlp_train_step(otlm_mlp m, const float* X, const float* T, const int32_t* idx, int64_t B,
                        const otlm_adamw* h, float* loss, void* stream) {
  if (!mlp_check_train_args(m, X, T, idx, B) || !h) return OTLM_E_INVALID;
  if (!(h->lr >= 0.0) || !(h->beta1 >= 0.0 && h->beta1 < 1.0) || !(h->beta2 >= 0.0 && h->beta2 < 1.0) ||
      !(h->eps > 0.0) || !(h->weight_decay >= 0.0))
    return OTLM_E_INVALID;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc = mlp_ensure_ws(m, B);
  if (rc != OTLM_OK) return rc;
  rc = mlp_forward_backward(m, X, T, idx, (int)B, loss, s);
  if (rc != OTLM_OK) return rc;
  m->step += 1;
  const double bc1 = 1.0 - std::pow(h->beta1, (double)m->step), bc2 = 1.0 - std::pow(h->beta2, (double)m->step);
  hipLaunchKernelGGL(mlp_adamw, dim3(1024), dim3(256), 0, s, m->theta, (const float*)m->grad, m->m, m->v,
                     (long long)m->nparam, (float)h->lr, (float)h->beta1, (float)h->beta2, (float)h->eps,
                     (float)h->weight_decay, (float)bc1, (float)bc2);
  m->bf_valid = false;
  OTLM_HIP(hipGetLastError());
  return OTLM_OK;
}

int otlm_mlp_get_params(otlm_mlp m, float* theta, void* stream) {
  if (!m || !theta) return OTLM_E_INVALID;
  OTLM_HIP(hipMemcpyAsync(theta, m->theta, (size_t)m->nparam * sizeof(float), hipMemcpyDefault,
                          static_cast<hipStream_t>(stream)));
  return OTLM_OK;
}

int otlm_mlp_set_params(otlm_mlp m, const float* theta, void* stream) {
  if (!m || !theta) return OTLM_E_INVALID;
  OTLM_HIP(hipMemcpyAsync(m->theta, theta, (size_t)m->nparam * sizeof(float), hipMemcpyDefault,
                          static_cast<hipStream_t>(stream)));
  m->bf_valid = false;
  return OTLM_OK;
}

int otlm_mlp_infer(otlm_mlp m, const float* Y, int64_t B, int32_t prec, int32_t n_u, int32_t n_v, float* logU,
                   float* logV, float* W, void* stream) {
  if (!m || !Y || !logV || !W || B < 0 || B > (1 << 24)) return OTLM_E_INVALID;
  if (prec != OTLM_PREC_FP32 && prec != OTLM_PREC_BF16) return OTLM_E_INVALID;
  const int in = m->dims[0], h1 = m->dims[1], h2 = m->dims[2], out = m->dims[3];
  if (n_u < 0 || n_v < 1 || n_u + n_v >= out) return OTLM_E_INVALID;
  if (B == 0) return OTLM_OK;
  hipStream_t s = static_cast<hipStream_t>(stream);
  int rc = mlp_ensure_ws(m, B);
  if (rc != OTLM_OK) return rc;
  const float* b1 = m->theta + m->off[1];
  const float* b2 = m->theta + m->off[3];
  const float* b3 = m->theta + m->off[5];
  const EpiOutSplit eo{b3, m->out_mu, m->out_sd, n_u, n_v, out - n_u - n_v, logU, logV, W, false};
  const int M = (int)B;
  if (prec == OTLM_PREC_FP32) {
    hipLaunchKernelGGL(mlp_gather_norm, dim3((unsigned)M), dim3(256), 0, s, Y, in, (const int*)nullptr, M, in,
                       (const float*)m->in_mu, (const float*)m->in_sd, m->X, (unsigned short*)nullptr);
    mlp_gemm<false, false>(GemmArgs{m->X, in, m->theta + m->off[0], in, M, h1, in},
                           EpiBiasGelu{b1, nullptr, m->H1, nullptr, h1, false}, s);
    mlp_gemm<false, false>(GemmArgs{m->H1, h1, m->theta + m->off[2], h1, M, h2, h1},
                           EpiBiasGelu{b2, nullptr, m->H2, nullptr, h2, false}, s);
    mlp_gemm<false, false>(GemmArgs{m->H2, h2, m->theta + m->off[4], h2, M, out, h2}, eo, s);
  } else {
    unsigned short* w1 = m->wbf;
    unsigned short* w2 = w1 + (size_t)h1 * in;
    unsigned short* w3 = w2 + (size_t)h2 * h1;
    if (!m->bf_valid) {
      hipLaunchKernelGGL(convert_f32_to_bf16, dim3(512), dim3(256), 0, s, (const float*)(m->theta + m->off[0]), w1,
                         (size_t)h1 * in);
      hipLaunchKernelGGL(convert_f32_to_bf16, dim3(512), dim3(256), 0, s, (const float*)(m->theta + m->off[2]), w2,
                         (size_t)h2 * h1);
      hipLaunchKernelGGL(convert_f32_to_bf16, dim3(512), dim3(256), 0, s, (const float*)(m->theta + m->off[4]), w3,
                         (size_t)out * h2);
      m->bf_valid = true;
    }
    hipLaunchKernelGGL(mlp_gather_norm, dim3((unsigned)M), dim3(256), 0, s, Y, in, (const int*)nullptr, M, in,
                       (const float*)m->in_mu, (const float*)m->in_sd, (float*)nullptr, m->Xbf);
    auto bf = [&](const unsigned short* A, int lda, const unsigned short* Bt, int N, int Kd, auto epi) {
      using E = decltype(epi);
      auto kern = gemm_nt_bf16<E>;
      const dim3 grid((unsigned)((N + GB_BN - 1) / GB_BN), (unsigned)((M + GB_BM - 1) / GB_BM));
      hipLaunchKernelGGL(kern, grid, dim3(256), 0, s, GemmArgsBf16{A, lda, Bt, Kd, M, N, Kd}, epi);
    };
    bf(m->Xbf, in, w1, h1, in, EpiBiasGelu{b1, nullptr, nullptr, m->H1bf, h1, false});
    bf(m->H1bf, h1, w2, h2, h1, EpiBiasGelu{b2, nullptr, nullptr, m->H2bf, h2, false});
    bf(m->H2bf, h2, w3, out, h2, eo);
  }
  OTLM_HIP(hipGetLastError());
  return OTLM_OK;
}

int otlm_mlp_free(otlm_mlp m) {
  if (!m) return OTLM_OK;
  (void)hipDeviceSynchronize();
  m->release();
  delete m;
  return OTLM_OK;
}

}  // extern "C"
