"""GPU parity of libotlm against the FP64 oracle, through the C-ABI.

Both sides get the same inputs: the FP32-rounded dictionary and targets (cast
back to FP64 for the oracle) and the same FP64 cost.  Tolerances:
* fixed point (ridge penalty, which converges in a few hundred iterations):
  relative weight error ||w - w*||_2 / ||w*||_2 <= 1e-5;
* fixed iteration count on the l1 workload (which does not converge in any
  practical number of single MM steps): the FP32 path drifts from FP64 along
  the flat directions of the weight problem, about 4e-6 after 20 iterations
  when the same loop is run in NumPy float32; the bound is 2.5e-5.
"""
import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as orc
from dictionaries import gapped_dictionary
from paper_2504_04609_amd import otlm, synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def rel_err(w, ref):
    return np.linalg.norm(w - ref, axis=-1) / np.linalg.norm(ref, axis=-1)


def as_f32(a):
    return np.asarray(a, dtype=np.float32)


def gpu(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def setup(wl, idx):
    dic = wl.dictionary()
    D32 = as_f32(dic.D)
    Y32 = as_f32(wl.targets(idx, dic=dic))
    C = wl.cost()
    return D32, Y32, C


def oracle_solve(C, D32, Y32, wl, **kw):
    K = orc.gibbs_kernel(C, wl.eps)
    return orc.solve(K, D32.astype(np.float64), Y32.astype(np.float64), fit=wl.fit, pen=wl.pen, eps=wl.eps,
                     lam=wl.lam, alpha=wl.alpha, lam2=wl.lam2, beta=wl.beta, **kw)


def gpu_solve(C, D32, Y32, wl, **kw):
    kern = otlm.GibbsKernel(gpu(C, torch.float64), wl.eps)
    p = otlm.SolveParams(eps=wl.eps, fit=wl.fit, pen=wl.pen, lam=wl.lam, lam2=wl.lam2, alpha=wl.alpha,
                         beta=wl.beta, **kw)
    out = kern.solve(gpu(D32), gpu(Y32), p)
    torch.cuda.synchronize()
    res = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    return kern, res


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    otlm.load()


def test_identity_dictionary_closed_form():
    """D = I, no penalty, one iteration: w = K 1, u = 1, v = (y / K^T 1)^{lam/(lam+eps)}."""
    n, eps, lam = 96, 0.02, 0.7
    x = synth.grid(n)
    C = synth.sq_cost(x, x)
    y = as_f32(np.random.default_rng(0).uniform(0.1, 1.0, (3, n)))
    wl = synth.Workload("identity", n=n, k=n, B=3, eps=eps, fit="kl", pen="none", lam=lam, alpha=0.0)
    _, res = gpu_solve(C, np.eye(n, dtype=np.float32), y, wl, tol=0.0, max_iter=1)
    K = np.exp(-C / eps)
    np.testing.assert_allclose(res["W"], np.broadcast_to(K.sum(1), (3, n)), rtol=2e-6)
    np.testing.assert_allclose(res["logU"], 0.0, atol=2e-6)
    np.testing.assert_allclose(np.exp(res["logV"]), (y / K.sum(0)) ** (lam / (lam + eps)), rtol=5e-6)
    assert np.all(res["status"] == otlm.STATUS_MAX_ITER) and np.all(res["iters"] == 1)


def test_single_target_fixed_point():
    """n = 200, k = 10, eps = 0.01, KL, ridge 1e-3: converged weights within 1e-5."""
    wl = synth.CONFIG1
    D32, Y32, C = setup(wl, [0])
    ref = oracle_solve(C, D32, Y32, wl, max_iter=5000, tol=1e-13)
    assert ref["converged"][0]
    _, res = gpu_solve(C, D32, Y32, wl, tol=1e-6, max_iter=3000, check_every=10)
    assert res["status"][0] == otlm.STATUS_CONVERGED
    assert res["iters"][0] % 10 == 0 and res["iters"][0] < 3000
    assert rel_err(res["W"], ref["W"])[0] <= 1e-5


def test_ridge_batch_fixed_point_ragged():
    """Ridge penalty at n = 1024, k = 64 converges: 37 spectra (ragged M tile)."""
    import dataclasses
    wl = dataclasses.replace(synth.CONFIG2, pen="l2sq", alpha=1e-3, B=37)
    D32, Y32, C = setup(wl, range(37))
    ref = oracle_solve(C, D32, Y32, wl, max_iter=3000, tol=1e-12)
    assert ref["converged"].all()
    _, res = gpu_solve(C, D32, Y32, wl, tol=1e-6, max_iter=3000, check_every=10)
    assert np.all(res["status"] == otlm.STATUS_CONVERGED)
    assert rel_err(res["W"], ref["W"]).max() <= 1e-5


def test_l1_path_parity_config2_slice():
    """l1 workload (n = 1024, k = 64, eps = 0.005), 67 spectra, 20 iterations."""
    wl = synth.CONFIG2
    idx = list(range(67))
    D32, Y32, C = setup(wl, idx)
    ref = oracle_solve(C, D32, Y32, wl, max_iter=20, tol=0.0)
    _, res = gpu_solve(C, D32, Y32, wl, tol=0.0, max_iter=20)
    assert rel_err(res["W"], ref["W"]).max() <= 2.5e-5
    lv_ref = ref["logV"]
    assert np.max(np.abs(res["logV"] - lv_ref)) <= 2e-4
    cov = np.isfinite(ref["logU"])
    assert np.array_equal(np.isfinite(res["logU"]), cov)
    assert np.max(np.abs(res["logU"][cov] - ref["logU"][cov])) <= 2e-4


FITS = ["kl", "tv", "l2", "l2tv", "balanced", "poisson"]
PENS = ["none", "l1", "l2sq", "en"]


@pytest.mark.parametrize("fit", FITS)
@pytest.mark.parametrize("pen", PENS)
def test_every_datafit_and_penalty(fit, pen):
    """Path parity after 30 iterations, n = 200 (ragged bin tile), k = 10, B = 5."""
    import dataclasses
    wl = dataclasses.replace(synth.CONFIG1, fit=fit, pen=pen, B=5, lam=1.0, lam2=0.1, alpha=2e-3, beta=1e-3,
                             gain=(0.8, 1.2))
    D32, Y32, C = setup(wl, range(5))
    ref = oracle_solve(C, D32, Y32, wl, max_iter=30, tol=0.0)
    _, res = gpu_solve(C, D32, Y32, wl, tol=0.0, max_iter=30)
    assert np.all(np.isfinite(res["W"]))
    assert rel_err(res["W"], ref["W"]).max() <= 5e-5, (fit, pen)


def test_asymmetric_cost():
    n, k, eps = 128, 6, 0.02
    dic = synth.make_dictionary(n, k, 9)
    x = dic.x
    C = synth.sq_cost(x, x) + 0.05 * x[:, None] * (1.0 - x[None, :])
    wl = synth.Workload("asym", n=n, k=k, B=4, eps=eps, fit="kl", pen="l2sq", lam=1.0, alpha=1e-3, seed=9,
                        shift=0.02, gain=(0.9, 1.1))
    Y32 = as_f32(wl.targets(range(4), dic=dic))
    D32 = as_f32(dic.D)
    kern, res = gpu_solve(C, D32, Y32, wl, tol=0.0, max_iter=25)
    assert kern.info()[1] is False
    ref = oracle_solve(C, D32, Y32, wl, max_iter=25, tol=0.0)
    assert rel_err(res["W"], ref["W"]).max() <= 2e-5


def test_objective_matches_oracle():
    wl = synth.CONFIG1
    D32, Y32, C = setup(wl, [0])
    kern, res = gpu_solve(C, D32, Y32, wl, tol=1e-6, max_iter=3000)
    p = otlm.SolveParams(eps=wl.eps, fit=wl.fit, pen=wl.pen, lam=wl.lam, alpha=wl.alpha)
    out = kern.objective(gpu(C, torch.float64), gpu(D32), gpu(Y32), p, gpu(res["W"]), gpu(res["logU"]),
                         gpu(res["logV"])).cpu().numpy()[0]
    K = orc.gibbs_kernel(C, wl.eps)
    ref = orc.objective(K, C, D32.astype(np.float64), Y32.astype(np.float64), res["W"].astype(np.float64),
                        res["logU"].astype(np.float64), res["logV"].astype(np.float64), fit=wl.fit, pen=wl.pen,
                        eps=wl.eps, lam=wl.lam, alpha=wl.alpha)[0]
    np.testing.assert_allclose(out[:3], ref[:3], rtol=1e-10)
    np.testing.assert_allclose(out[3:], ref[3:], rtol=1e-6, atol=1e-12)
    # and the converged FP32 point is near-optimal
    assert abs(out[0] - out[1]) <= 1e-5 * abs(out[0])
    assert out[3] < 1e-5


def test_deterministic_and_batch_independent():
    wl = synth.CONFIG2
    D32, Y32, C = setup(wl, range(40))
    kern = otlm.GibbsKernel(gpu(C, torch.float64), wl.eps)
    p = otlm.SolveParams(eps=wl.eps, fit=wl.fit, pen=wl.pen, lam=wl.lam, alpha=wl.alpha, tol=1e-4, max_iter=60,
                         check_every=5)
    a = kern.solve(gpu(D32), gpu(Y32), p)
    b = kern.solve(gpu(D32), gpu(Y32), p)
    c = kern.solve(gpu(D32), gpu(Y32[7:9]), p)
    torch.cuda.synchronize()
    assert torch.equal(a["W"], b["W"]) and torch.equal(a["logV"], b["logV"])
    assert torch.equal(a["W"][7:9], c["W"]) and torch.equal(a["iters"][7:9], c["iters"])


def test_warm_start_continues_the_path():
    wl = synth.CONFIG2
    D32, Y32, C = setup(wl, range(8))
    kern = otlm.GibbsKernel(gpu(C, torch.float64), wl.eps)
    mk = lambda n, warm=False: otlm.SolveParams(eps=wl.eps, fit=wl.fit, pen=wl.pen, lam=wl.lam, alpha=wl.alpha,
                                                tol=0.0, max_iter=n, warm=warm)
    full = kern.solve(gpu(D32), gpu(Y32), mk(30))
    half = kern.solve(gpu(D32), gpu(Y32), mk(15))
    rest = kern.solve(gpu(D32), gpu(Y32), mk(15, True), W=half["W"].clone(), logV=half["logV"].clone())
    torch.cuda.synchronize()
    err = rel_err(rest["W"].cpu().numpy(), full["W"].cpu().numpy())
    assert err.max() <= 1e-5


def test_invalid_inputs_are_rejected():
    wl = synth.CONFIG1
    D32, Y32, C = setup(wl, [0])
    kern = otlm.GibbsKernel(gpu(C, torch.float64), wl.eps)
    p = otlm.SolveParams(eps=wl.eps, fit=wl.fit, pen=wl.pen, lam=wl.lam, alpha=wl.alpha)
    bad = D32.copy()
    bad[3, 2] = -1.0
    with pytest.raises(otlm.OtlmError):
        kern.solve(gpu(bad), gpu(Y32), p)
    with pytest.raises(otlm.OtlmError):
        kern.solve(gpu(D32), gpu(Y32), otlm.SolveParams(eps=wl.eps * 2, fit="kl", pen="none"))
    empty = D32.copy()
    empty[:, 4] = 0.0
    with pytest.raises(otlm.OtlmError):
        kern.solve(gpu(empty), gpu(Y32), p)
    out = kern.solve(gpu(D32), gpu(Y32[:0]), p)
    assert out["W"].shape == (0, D32.shape[1])


def test_full_size_sampled_parity():
    """B = 4096, n = 1024, k = 64 (the benchmark launch), 20 iterations; 6 sampled
    spectra compared one by one with the oracle."""
    wl = synth.CONFIG2
    D32, Y32, C = setup(wl, None)
    _, res = gpu_solve(C, D32, Y32, wl, tol=0.0, max_iter=20)
    rng = np.random.default_rng(3)
    pick = np.sort(rng.choice(wl.B, 6, replace=False))
    ref = oracle_solve(C, D32, Y32[pick], wl, max_iter=20, tol=0.0)
    assert rel_err(res["W"][pick], ref["W"]).max() <= 2.5e-5


# ---------------------------------------------------------------- exact weight prox
def test_exact_prox_l1_fixed_point():
    """l1 workload with the weight prox solved exactly each iteration, FP32 state:
    every spectrum converges; its weights sit at the FP32 floor of this
    ill-conditioned dictionary (the weight prox amplifies the 1e-7 relative error
    of s = K v by up to ~1e3), so the bound is 1e-3 per spectrum and 2e-5 for the
    median; the FP64 refinement test below asks for 1e-5 on every spectrum."""
    wl = synth.CONFIG2
    idx = list(range(19))
    D32, Y32, C = setup(wl, idx)
    ref = oracle_solve(C, D32, Y32, wl, max_iter=400, tol=1e-10, mode="exact")
    assert ref["converged"].all()
    _, res = gpu_solve(C, D32, Y32, wl, tol=1e-6, max_iter=400, check_every=5, wstep="exact", inner_max=5)
    assert np.all((res["status"] == otlm.STATUS_CONVERGED) | (res["status"] == otlm.STATUS_STAGNATED)), res["iters"]
    err = rel_err(res["W"], ref["W"])
    assert err.max() <= 1e-3 and np.median(err) <= 2e-5, err
    # the l1 solution is sparse: exact zeros on the GPU where the oracle has zeros
    assert np.array_equal(res["W"] == 0, ref["W"] == 0) or np.all(res["W"][ref["W"] == 0] < 1e-6 * res["W"].max())


def test_exact_prox_ridge_agrees_with_mm_fixed_point():
    import dataclasses
    wl = dataclasses.replace(synth.CONFIG2, pen="l2sq", alpha=1e-3, B=9)
    D32, Y32, C = setup(wl, range(9))
    _, a = gpu_solve(C, D32, Y32, wl, tol=1e-6, max_iter=3000, wstep="exact")
    _, b = gpu_solve(C, D32, Y32, wl, tol=1e-6, max_iter=3000, wstep="mm")
    assert np.all(a["status"] == otlm.STATUS_CONVERGED) and np.all(b["status"] == otlm.STATUS_CONVERGED)
    assert rel_err(a["W"], b["W"]).max() <= 1e-5


@pytest.mark.parametrize("k,pen,alpha", [(5, "l1", 1e-2), (16, "l1", 1e-2), (17, "l1", 1e-2), (33, "l1", 1e-2),
                                         (48, "l1", 1e-2), (63, "l1", 1e-2), (40, "l2sq", 1e-3), (63, "l2sq", 1e-3)])
def test_exact_prox_every_dictionary_width(k, pen, alpha):
    """Exact weight prox with FP64 refinement for dictionary widths on both sides
    of the kernel's 16-column boundaries: the gradient splits bins over the idle
    waves (k <= 32), leaves one wave idle (33..48) or uses all four (> 48); the l1
    free sets (5..27 weights) take 1 or 2 compact Hessian panels, the ridge ones
    (every weight free) 3 or 4.  n = 200 leaves a ragged tail in every bin sweep.
    Bar: 1e-5 on every spectrum."""
    wl = synth.Workload(f"width{k}", n=200, k=k, B=6, eps=0.01, fit="kl", pen=pen, lam=1.0, alpha=alpha, seed=21)
    D32, Y32, C = setup(wl, range(wl.B))
    ref = oracle_solve(C, D32, Y32, wl, max_iter=600, tol=1e-11, mode="exact")
    assert ref["converged"].all()
    _, res = gpu_solve(C, D32, Y32, wl, tol=1e-9, bulk_tol=1e-4, max_iter=400, check_every=5, wstep="exact",
                       inner_max=8, refine="fp64", refine_sweeps=300)
    assert np.all(res["status"] == otlm.STATUS_CONVERGED), res["status"]
    err = rel_err(res["W"], ref["W"])
    assert err.max() <= 1e-5, err


@pytest.mark.parametrize("k,pen,alpha", [(40, "l2sq", 1e-3), (64, "l2sq", 1e-3), (64, "l1", 1e-2)])
def test_exact_prox_gapped_dictionary(k, pen, alpha):
    """The Newton prox orders the free weights by where their columns' nonzero
    rows sit and skips the Hessian's all-zero block-steps (and the gradient's
    empty bin blocks); columns with interior gaps, dense columns and columns at
    the grid's ends, shuffled, must still reach the oracle (FP64 refinement,
    bar 1e-5 on every spectrum)."""
    wl = synth.Workload(f"gapped{k}", n=200, k=k, B=6, eps=0.01, fit="kl", pen=pen, lam=1.0, alpha=alpha, seed=23)
    D32 = gapped_dictionary(wl.n, k, 31)
    rng = np.random.default_rng(32)
    W = rng.exponential(1.0, (wl.B, k))
    Y32 = as_f32(W @ D32.T.astype(np.float64) + np.abs(rng.normal(0.0, 1e-3, (wl.B, wl.n))))
    C = wl.cost()
    ref = oracle_solve(C, D32, Y32, wl, max_iter=600, tol=1e-11, mode="exact")
    assert ref["converged"].all()
    _, res = gpu_solve(C, D32, Y32, wl, tol=1e-9, bulk_tol=1e-4, max_iter=400, check_every=5, wstep="exact",
                       inner_max=8, refine="fp64", refine_sweeps=300)
    assert np.all(res["status"] == otlm.STATUS_CONVERGED), res["status"]
    err = rel_err(res["W"], ref["W"])
    assert err.max() <= 1e-5, err


def test_exact_prox_column_order_invariance():
    """Permuting the dictionary's columns permutes the weights: the prox orders
    its free weights by where the columns' nonzero rows sit (ties by index), so
    the two solves differ only in rounding (FP64 refinement to tol 1e-9)."""
    wl = synth.Workload("perm48", n=200, k=48, B=6, eps=0.01, fit="kl", pen="l1", lam=1.0, alpha=1e-2, seed=25)
    D32, Y32, C = setup(wl, range(wl.B))
    perm = np.random.default_rng(26).permutation(wl.k)
    kw = dict(tol=1e-9, bulk_tol=1e-4, max_iter=400, check_every=5, wstep="exact", inner_max=8, refine="fp64",
              refine_sweeps=300)
    _, a = gpu_solve(C, D32, Y32, wl, **kw)
    _, b = gpu_solve(C, np.ascontiguousarray(D32[:, perm]), Y32, wl, **kw)
    assert (a["status"] == otlm.STATUS_CONVERGED).all() and (b["status"] == otlm.STATUS_CONVERGED).all()
    assert rel_err(b["W"], a["W"][:, perm]).max() <= 2e-6


def test_exact_prox_rejects_large_dictionaries():
    n, k = 128, 80
    dic = synth.make_dictionary(n, k, 4)
    wl = synth.Workload("k80", n=n, k=k, B=2, eps=0.01, fit="kl", pen="l1", lam=1.0, alpha=1e-2, seed=4)
    Y32 = as_f32(wl.targets(range(2), dic=dic))
    kern = otlm.GibbsKernel(gpu(wl.cost(), torch.float64), wl.eps)
    p = otlm.SolveParams(eps=wl.eps, fit="kl", pen="l1", alpha=1e-2, wstep="exact")
    with pytest.raises(otlm.OtlmError, match="unsupported"):
        kern.solve(gpu(as_f32(dic.D)), gpu(Y32), p)


def test_exact_prox_full_size_sampled():
    """B = 4096 (the benchmark launch), exact weight prox, 5 sampled spectra."""
    wl = synth.CONFIG2
    D32, Y32, C = setup(wl, None)
    _, res = gpu_solve(C, D32, Y32, wl, tol=1e-6, max_iter=400, check_every=5, wstep="exact", inner_max=5)
    ok = (res["status"] == otlm.STATUS_CONVERGED) | (res["status"] == otlm.STATUS_STAGNATED)
    assert ok.all() and np.mean(res["status"] == otlm.STATUS_CONVERGED) >= 0.8
    pick = np.sort(np.random.default_rng(3).choice(wl.B, 5, replace=False))
    ref = oracle_solve(C, D32, Y32[pick], wl, max_iter=400, tol=1e-10, mode="exact")
    assert rel_err(res["W"][pick], ref["W"]).max() <= 1e-3


def test_fp64_refinement_reaches_oracle_l1():
    """Exact weight prox, FP32 bulk phase to 1e-4 then FP64 refinement: every
    spectrum of a 19-spectrum l1 slice within 1e-5 of the oracle (the FP32 state
    alone plateaus at 1e-5..1e-3 on this dictionary)."""
    wl = synth.CONFIG2
    idx = list(range(19))
    D32, Y32, C = setup(wl, idx)
    ref = oracle_solve(C, D32, Y32, wl, max_iter=400, tol=1e-10, mode="exact")
    _, res = gpu_solve(C, D32, Y32, wl, tol=1e-9, bulk_tol=1e-4, max_iter=300, check_every=5, wstep="exact",
                       inner_max=5, refine="fp64", refine_sweeps=200)
    assert np.all(res["status"] == otlm.STATUS_CONVERGED), res["iters"]
    err = rel_err(res["W"], ref["W"])
    assert err.max() <= 1e-5, err


def test_fp64_refinement_full_size_sampled():
    """B = 4096 with FP64 refinement: all spectra converge to tol 1e-9; 5 sampled
    spectra within 1e-5 of the oracle."""
    wl = synth.CONFIG2
    D32, Y32, C = setup(wl, None)
    _, res = gpu_solve(C, D32, Y32, wl, tol=1e-9, bulk_tol=1e-4, max_iter=300, check_every=5, wstep="exact",
                       inner_max=5, refine="fp64", refine_sweeps=200)
    assert np.all(res["status"] == otlm.STATUS_CONVERGED), np.unique(res["status"], return_counts=True)
    pick = np.sort(np.random.default_rng(3).choice(wl.B, 5, replace=False))
    ref = oracle_solve(C, D32, Y32[pick], wl, max_iter=400, tol=1e-10, mode="exact")
    assert rel_err(res["W"][pick], ref["W"]).max() <= 1e-5


# ---------------------------------------------------------------- BF16 bulk phase
def test_bf16_products_closed_form():
    """D = I, one iteration with BF16 kernel products: w = K 1 and
    v = (y / K^T 1)^{lam/(lam+eps)} within the BF16 rounding of K (2^-9 per
    entry, all terms positive, so the sums carry at most that relative error)."""
    n, eps, lam = 96, 0.02, 0.7
    x = synth.grid(n)
    C = synth.sq_cost(x, x)
    y = as_f32(np.random.default_rng(0).uniform(0.1, 1.0, (3, n)))
    wl = synth.Workload("identity", n=n, k=n, B=3, eps=eps, fit="kl", pen="none", lam=lam, alpha=0.0)
    _, res = gpu_solve(C, np.eye(n, dtype=np.float32), y, wl, tol=0.0, max_iter=1, prec="bf16")
    K = np.exp(-C / eps)
    np.testing.assert_allclose(res["W"], np.broadcast_to(K.sum(1), (3, n)), rtol=2 ** -8)
    np.testing.assert_allclose(np.exp(res["logV"]), (y / K.sum(0)) ** (lam / (lam + eps)), rtol=2 ** -8)


def test_bf16_bulk_then_fp64_reaches_oracle_l1():
    wl = synth.CONFIG2
    idx = list(range(19))
    D32, Y32, C = setup(wl, idx)
    ref = oracle_solve(C, D32, Y32, wl, max_iter=400, tol=1e-10, mode="exact")
    _, res = gpu_solve(C, D32, Y32, wl, tol=1e-9, bulk_tol=1e-3, max_iter=300, check_every=5, wstep="exact",
                       inner_max=5, prec="bf16", refine="fp64", refine_sweeps=300)
    assert np.all(res["status"] == otlm.STATUS_CONVERGED), res["iters"]
    assert rel_err(res["W"], ref["W"]).max() <= 1e-5


def test_bf16_bulk_then_fp32_ridge():
    """Ridge workload, MM steps: BF16 bulk then FP32 sweeps reach the oracle's
    fixed point to 1e-5 (ridge keeps the weight problem well conditioned)."""
    import dataclasses
    wl = dataclasses.replace(synth.CONFIG2, pen="l2sq", alpha=1e-3, B=21)
    D32, Y32, C = setup(wl, range(21))
    ref = oracle_solve(C, D32, Y32, wl, max_iter=3000, tol=1e-12)
    _, res = gpu_solve(C, D32, Y32, wl, tol=1e-6, bulk_tol=1e-3, max_iter=2000, check_every=10, prec="bf16",
                       refine="fp32", refine_sweeps=2000)
    assert np.all(res["status"] == otlm.STATUS_CONVERGED)
    assert rel_err(res["W"], ref["W"]).max() <= 1e-5


def test_small_eps_range_promotion_reaches_oracle():
    """eps = 0.001: BF16 bulk products, FP64 refinement.  With the range test
    forced low (|log u| > 5, below the |log u| ~ 10-12 these spectra reach) every
    spectrum leaves the bulk phase early for the FP64 state and still reaches the
    oracle; with the default threshold (30) none is moved."""
    wl = synth.CONFIG3
    idx = [0, 5, 9, 123]
    D32, Y32, C = setup(wl, idx)
    common = dict(tol=1e-9, bulk_tol=1e-3, max_iter=400, check_every=5, wstep="exact", inner_max=5, prec="bf16",
                  refine="fp64", refine_sweeps=300)
    ref = oracle_solve(C, D32, Y32, wl, max_iter=800, tol=1e-11, mode="exact")
    _, low = gpu_solve(C, D32, Y32, wl, absorb_tau=5.0, **common)
    assert (low["status"] & otlm.STATUS_ABSORBED).all() and (low["status"] & otlm.STATUS_CONVERGED).all()
    assert rel_err(low["W"], ref["W"]).max() <= 1e-5
    _, std = gpu_solve(C, D32, Y32, wl, **common)
    assert not (std["status"] & otlm.STATUS_ABSORBED).any() and (std["status"] & otlm.STATUS_CONVERGED).all()
    assert rel_err(std["W"], ref["W"]).max() <= 1e-5
