"""GPU parity of the ragged batch (otlm_ragged_*) against the FP64 oracle.

Every spectrum has its own grid length and dictionary.  The oracle solves each
spectrum on its own (Algorithm 1 with the exact weight prox, run to tol 1e-12,
whose fixed point is the one of the single MM step) from the same FP32-rounded
inputs cast to FP64.  Bar: relative l2 weight error <= 1e-5 in the FP32 path.

The small cases mix grid lengths that are not multiples of the 64-bin padding
(ragged tails), dictionaries from 3 to 130 columns and groups of 1 to ~10
spectra, so the grouped products run partial tiles in both dimensions.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as orc
from dictionaries import gapped_dictionary
from paper_2504_04609_amd import otlm, synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SMALL = synth.RaggedWorkload(name="ragged_small", B=24, ns=(96, 200, 320), ks=(3, 17, 40, 70, 130), seed=11)


def gpu(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def rel_err(w, ref):
    return float(np.linalg.norm(w - ref) / np.linalg.norm(ref))


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    otlm.load()


def params(wl, **kw):
    base = dict(eps=wl.eps, fit=wl.fit, pen=wl.pen, lam=wl.lam, lam2=wl.lam2, alpha=wl.alpha, beta=wl.beta,
                tol=1e-6, max_iter=3000, check_every=10, inner_max=4)
    base.update(kw)
    return otlm.SolveParams(**base)


class Ragged:
    """Packed inputs of a ragged workload plus its kernels on the GPU."""

    def __init__(self, wl, idx=None):
        self.wl = wl
        self.kernel_of, self.ns, self.kdim, self.D, self.Y = wl.pack(idx)
        self.C = {n: wl.cost(n) for n in self.ns}
        self.kernels = [otlm.GibbsKernel(gpu(self.C[n], torch.float64), wl.eps) for n in self.ns]
        self.Dt, self.Yt = gpu(self.D), gpu(self.Y)
        n = np.array(self.ns)[self.kernel_of]
        self.y_off = np.concatenate([[0], np.cumsum(n)])
        self.w_off = np.concatenate([[0], np.cumsum(self.kdim)])
        self.d_off = np.concatenate([[0], np.cumsum(n * self.kdim)])

    def plan(self, p, **kw):
        return otlm.RaggedPlan(self.kernels, self.kernel_of, self.kdim, p, **kw)

    def solve(self, p, **kw):
        plan = self.plan(p, **kw)
        out = plan.solve(self.Dt, self.Yt)
        torch.cuda.synchronize()
        res = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
        return plan, res

    def spectrum(self, b):
        n = self.ns[self.kernel_of[b]]
        k = int(self.kdim[b])
        D = self.D[self.d_off[b]:self.d_off[b + 1]].reshape(n, k).astype(np.float64)
        y = self.Y[self.y_off[b]:self.y_off[b + 1]].astype(np.float64)
        return n, k, D, y

    def w(self, res, b):
        return res["W"][self.w_off[b]:self.w_off[b + 1]]

    def logv(self, res, b):
        return res["logV"][self.y_off[b]:self.y_off[b + 1]]

    def oracle(self, b, **kw):
        n, k, D, y = self.spectrum(b)
        wl = self.wl
        K = orc.gibbs_kernel(self.C[n], wl.eps)
        args = dict(fit=wl.fit, pen=wl.pen, eps=wl.eps, lam=wl.lam, lam2=wl.lam2, alpha=wl.alpha, beta=wl.beta,
                    max_iter=2000, tol=1e-12, mode="exact")
        args.update(kw)
        return orc.solve(K, D, y[None], **args)


@pytest.fixture(scope="module")
def small():
    return Ragged(SMALL)


def test_small_ragged_batch_reaches_oracle(small):
    plan, res = small.solve(params(SMALL))
    assert (res["status"] == otlm.STATUS_CONVERGED).all(), res["status"]
    errs, verrs = [], []
    for b in range(SMALL.B):
        ref = small.oracle(b)
        errs.append(rel_err(small.w(res, b), ref["W"][0]))
        verrs.append(np.abs(small.logv(res, b) - ref["logV"][0]).max())
    print("tile", plan.info()["tile"], "max w err", max(errs), "max logv err", max(verrs))
    assert max(errs) <= 1e-5, errs
    assert max(verrs) <= 1e-3, verrs


def test_graph_replay_equals_eager_launches(small):
    p = params(SMALL)
    _, a = small.solve(p, use_graph=True, tile=0)
    _, b = small.solve(p, use_graph=False, tile=0)
    for key in ("W", "logU", "logV", "iters", "status"):
        np.testing.assert_array_equal(a[key], b[key], err_msg=key)


@pytest.mark.parametrize("tile", [0, 1, 2, 3])
def test_every_tile_shape_reaches_oracle(small, tile):
    plan, res = small.solve(params(SMALL), tile=tile)
    assert plan.info()["tile"] == otlm.RAGGED_TILES[tile]
    for b in (0, 5, 11, 23):
        assert rel_err(small.w(res, b), small.oracle(b)["W"][0]) <= 1e-5


def test_input_order_does_not_change_a_spectrum(small):
    """Rows of the grouped products and the per-spectrum weight steps are
    independent: a permuted batch gives every spectrum bitwise the same result
    (same tile shape)."""
    p = params(SMALL)
    _, a = small.solve(p, tile=0)
    perm = np.random.default_rng(5).permutation(SMALL.B)
    sub = Ragged(SMALL, perm)
    _, b = sub.solve(p, tile=0)
    for j, bi in enumerate(perm):
        np.testing.assert_array_equal(sub.w(b, j), small.w(a, bi))
        np.testing.assert_array_equal(sub.logv(b, j), small.logv(a, bi))
        assert b["iters"][j] == a["iters"][bi]


def test_inner_steps_keep_the_fixed_point(small):
    """One and eight MM steps per iteration converge to the same weights (the
    repetitions change the path, not the limit); more steps need fewer
    iterations.  MM steps only (no Newton prox after some iterations)."""
    _, one = small.solve(params(SMALL, inner_max=1), newton_after=-1)
    _, eight = small.solve(params(SMALL, inner_max=8), newton_after=-1)
    for b in range(0, SMALL.B, 3):
        ref = small.oracle(b)["W"][0]
        assert rel_err(small.w(one, b), ref) <= 1e-5
        assert rel_err(small.w(eight, b), ref) <= 1e-5
    assert eight["iters"].mean() < 0.5 * one["iters"].mean()


def test_single_mm_step_path_matches_oracle(small):
    """Fixed iteration count (tol 0): with one MM step per iteration (and no
    Newton prox) the GPU follows the oracle's single-step path, not only its
    limit."""
    _, res = small.solve(params(SMALL, inner_max=1, tol=0.0, max_iter=25), newton_after=-1)
    assert (res["iters"] == 25).all() and (res["status"] == otlm.STATUS_MAX_ITER).all()
    for b in (1, 7, 19):
        ref = small.oracle(b, mode="single", max_iter=25, tol=0.0)
        assert rel_err(small.w(res, b), ref["W"][0]) <= 2e-5


def test_warm_start_from_the_solution(small):
    p = params(SMALL)
    plan, res = small.solve(p)
    pw = params(SMALL, warm=True)
    plan2 = small.plan(pw)
    W = gpu(res["W"])
    logV = gpu(res["logV"])
    out = plan2.solve(small.Dt, small.Yt, W=W, logV=logV)
    torch.cuda.synchronize()
    w2 = out["W"].cpu().numpy()
    # a restart from an FP32 fixed point stays inside its rounding-noise ball
    # and stops within two tests
    assert out["iters"].cpu().numpy().max() <= 2 * p.check_every
    for b in range(SMALL.B):
        assert rel_err(small.w({"W": w2}, b), small.w(res, b)) <= 1e-5
    for b in (0, 6, 13):
        assert rel_err(small.w({"W": w2}, b), small.oracle(b)["W"][0]) <= 1e-5


def test_invalid_requests_are_rejected(small):
    p = params(SMALL)
    with pytest.raises(otlm.OtlmError):
        otlm.RaggedPlan(small.kernels, small.kernel_of * 0 + len(small.kernels), small.kdim, p)
    with pytest.raises(otlm.OtlmError):
        small.plan(params(SMALL, eps=SMALL.eps * 2))
    with pytest.raises(otlm.OtlmError, match="unsupported"):
        small.plan(params(SMALL, wstep="exact"))
    with pytest.raises(otlm.OtlmError, match="unsupported"):
        small.plan(params(SMALL, prec="bf16"))
    bad = small.kdim.copy()
    bad[0] = 300
    with pytest.raises(otlm.OtlmError):
        otlm.RaggedPlan(small.kernels, small.kernel_of, bad, p)
    plan = small.plan(p)
    D = small.Dt.clone()
    D[int(small.d_off[3]) + 1] = -1.0
    with pytest.raises(otlm.OtlmError, match="invalid"):
        plan.solve(D, small.Yt)
    Y = small.Yt.clone()
    Y[5] = float("nan")
    with pytest.raises(otlm.OtlmError, match="invalid"):
        plan.solve(small.Dt, Y)
    D = small.Dt.clone()
    n, k, _, _ = small.spectrum(2)
    D[int(small.d_off[2]):int(small.d_off[3])].view(n, k)[:, 1] = 0.0  # empty column
    with pytest.raises(otlm.OtlmError, match="invalid"):
        plan.solve(D, small.Yt)


def test_ragged_workload_full_size_sampled():
    """8192 spectra, n in {256..2048}, k in {16..128}, own dictionaries: every
    spectrum stops on the convergence test, and a stratified sample (one per
    (n, k) cell) matches the oracle to 1e-5."""
    wl = synth.CONFIG4
    full = Ragged(wl)
    plan, res = full.solve(params(wl))
    info = plan.info()
    print("tile", info["tile"], "tune ms", info["tune_ms"], "iters mean", res["iters"].mean())
    assert (res["status"] == otlm.STATUS_CONVERGED).mean() >= 0.99
    sizes = list(zip(np.array(full.ns)[full.kernel_of], full.kdim))
    pick = {}
    for b, cell in enumerate(sizes):
        pick.setdefault(cell, b)
    errs = [rel_err(full.w(res, b), full.oracle(b)["W"][0]) for b in pick.values()]
    print("sampled max err", max(errs))
    assert len(errs) == 16 and max(errs) <= 1e-5


def test_newton_weight_prox_reaches_oracle(small):
    """Spectra with k <= 128 switch to the exact weight prox after 3 MM
    iterations (FP64 Hessian up to k = 64, FP32 up to 128; k = 130 stays on MM
    steps): every spectrum still reaches the oracle, in far fewer iterations."""
    _, mm = small.solve(params(SMALL), newton_after=-1)
    plan, nt = small.solve(params(SMALL), newton_after=3)
    assert (nt["status"] == otlm.STATUS_CONVERGED).all()
    for b in range(SMALL.B):
        assert rel_err(small.w(nt, b), small.oracle(b)["W"][0]) <= 1e-5, b
    newton = np.array([k <= 128 for k in small.kdim])
    print("mean iterations MM", mm["iters"][newton].mean(), "Newton", nt["iters"][newton].mean())
    assert nt["iters"][newton].mean() < 0.7 * mm["iters"][newton].mean()
    np.testing.assert_array_equal(nt["iters"][~newton], mm["iters"][~newton])


def test_newton_graph_replay_equals_eager(small):
    p = params(SMALL)
    _, a = small.solve(p, use_graph=True, tile=0, newton_after=3)
    _, b = small.solve(p, use_graph=False, tile=0, newton_after=3)
    for key in ("W", "logV", "iters", "status"):
        np.testing.assert_array_equal(a[key], b[key], err_msg=key)


def test_gapped_dictionaries_reach_oracle():
    """Own dictionaries with interior gaps, dense columns and narrow columns near
    the grid's ends (shuffled, no two alike), widths on both Newton kernels (40,
    64; 100 on the 128-wide one): the banded MM steps, the column order of the
    64-wide prox and the skipped Hessian block-steps must still reach the oracle
    (bar 1e-5)."""
    wl = SMALL
    n = 200
    ks = [40, 64, 100, 64]
    Ds = [gapped_dictionary(n, k, 40 + i) for i, k in enumerate(ks)]
    rng = np.random.default_rng(41)
    Ys = [(rng.exponential(1.0, k) @ D.T.astype(np.float64) + np.abs(rng.normal(0.0, 1e-3, n))).astype(np.float32)
          for D, k in zip(Ds, ks)]
    C = wl.cost(n)
    kern = otlm.GibbsKernel(gpu(C, torch.float64), wl.eps)
    kernel_of = np.zeros(len(ks), dtype=np.int32)
    kdim = np.array(ks, dtype=np.int32)
    plan = otlm.RaggedPlan([kern], kernel_of, kdim, params(wl), newton_after=3)
    out = plan.solve(gpu(np.concatenate([D.ravel() for D in Ds])), gpu(np.concatenate(Ys)))
    torch.cuda.synchronize()
    assert (out["status"].cpu().numpy() == otlm.STATUS_CONVERGED).all()
    W = out["W"].cpu().numpy()
    off = np.concatenate([[0], np.cumsum(ks)])
    K = orc.gibbs_kernel(C, wl.eps)
    for b, (D, y) in enumerate(zip(Ds, Ys)):
        ref = orc.solve(K, D.astype(np.float64), y.astype(np.float64)[None], fit=wl.fit, pen=wl.pen, eps=wl.eps,
                        lam=wl.lam, lam2=wl.lam2, alpha=wl.alpha, beta=wl.beta, max_iter=2000, tol=1e-12,
                        mode="exact")["W"][0]
        assert rel_err(W[off[b]:off[b + 1]], ref) <= 1e-5, b

