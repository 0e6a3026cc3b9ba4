"""What the trained warm-start network gains, end to end on the GPU.

A network 1024 -> 512 -> 512 -> 2112 is trained with the library's kernels on
50 000 solver-generated (y, log u, log v, w) triples of the held-out-eps
workload (n = 1024, k = 64, KL, l1 1e-2, eps = 0.002), then 512 held-out
targets are solved cold and from its BF16 predictions.  Both arms must reach
the FP64 oracle to 1e-5 on sampled spectra; the warm arm must do markedly
less Newton work; garbage starts must fall back to the cold start.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as orc
from paper_2504_04609_amd import otlm, synth, warmstart

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
N_TRAIN, N_EVAL = 50_000, 512
DIMS = (1024, 512, 512, 2 * 1024 + 64)


@pytest.fixture(scope="module")
def setup():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    ev, tr = synth.CONFIG5_EVAL, synth.CONFIG5_TRAIN
    dic = ev.dictionary()
    Ye = ev.targets_fast(range(N_EVAL), dic=dic, device=DEV)
    Yt = tr.targets_fast(range(N_TRAIN), dic=dic, device=DEV)
    D = torch.as_tensor(dic.D.astype(np.float32), device=DEV)
    C = ev.cost()
    kern = otlm.GibbsKernel(torch.as_tensor(C, device=DEV), ev.eps)
    base = dict(eps=ev.eps, fit=ev.fit, pen=ev.pen, lam=ev.lam, alpha=ev.alpha, check_every=5, max_iter=400,
                wstep="exact", inner_max=5, refine="fp64")
    out = warmstart.solve_in_chunks(kern, D, Yt, otlm.SolveParams(**base, tol=1e-8, bulk_tol=1e-4, refine_sweeps=200))
    assert (out["status"] == otlm.STATUS_CONVERGED).all()
    T = warmstart.training_targets(out)
    net = otlm.WarmStartMLP(DIMS, synth.mlp_init(DIMS, 21))
    net.set_norm(Yt, T)
    net.set_loss_weights(np.concatenate([np.zeros(1024), np.ones(1024), np.full(64, 16.0)]))
    hist = warmstart.train(net, Yt, T, 20, batch=256, lr=1e-3, weight_decay=1e-4, seed=1)
    assert hist[-1] < 0.5 * hist[0]
    return dict(ev=ev, dic=dic, Ye=Ye, D=D, C=C, kern=kern, net=net, base=base)


def params(s, **kw):
    return otlm.SolveParams(**s["base"], tol=1e-9, bulk_tol=1e-4, refine_sweeps=300, **kw)


def solve_profiled(s, p, W=None, logV=None):
    kern = s["kern"]
    kern.profile(True)
    out = kern.solve(s["D"], s["Ye"], p, W=W, logV=logV) if W is not None else kern.solve(s["D"], s["Ye"], p)
    torch.cuda.synchronize()
    prof = kern.profile_read()
    kern.profile(False)
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}, prof


def rel(a, b):
    return np.linalg.norm(a - b, axis=-1) / np.linalg.norm(b, axis=-1)


def test_warm_start_gains_over_cold(setup):
    s = setup
    cold, pc = solve_profiled(s, params(s))
    _, logV, W = s["net"].infer(s["Ye"], 1024, 1024, prec="bf16")
    warm, pw = solve_profiled(s, params(s, warm=True, warm_probe=0.5), W=W, logV=logV)
    print(f"cold: {cold['iters'].mean():.1f} iterations, {pc['newton_iters']} Newton; "
          f"warm: {warm['iters'].mean():.1f} iterations, {pw['newton_iters']} Newton, "
          f"{int(np.sum(warm['status'] & otlm.STATUS_FALLBACK > 0))} fallbacks")
    assert (cold["status"] & otlm.STATUS_CONVERGED).all() and (warm["status"] & otlm.STATUS_CONVERGED).all()
    assert warm["iters"].mean() < 0.85 * cold["iters"].mean()
    assert pw["newton_iters"] < 0.8 * pc["newton_iters"]
    # both arms reach the oracle
    ev = s["ev"]
    K = orc.gibbs_kernel(s["C"], ev.eps)
    Y = s["Ye"].cpu().numpy().astype(np.float64)
    pick = np.random.default_rng(3).choice(N_EVAL, 4, replace=False)
    ref = orc.solve(K, s["dic"].D.astype(np.float32).astype(np.float64), Y[pick], fit=ev.fit, pen=ev.pen,
                    eps=ev.eps, lam=ev.lam, alpha=ev.alpha, max_iter=600, tol=1e-10, mode="exact")["W"]
    assert rel(cold["W"][pick], ref).max() <= 1e-5
    assert rel(warm["W"][pick], ref).max() <= 1e-5


def test_garbage_start_falls_back_to_cold(setup):
    s = setup
    rng = np.random.default_rng(0)
    W = torch.as_tensor(rng.uniform(0, 2, (N_EVAL, 64)).astype(np.float32), device=DEV)
    logV = torch.as_tensor(rng.normal(0, 3, (N_EVAL, 1024)).astype(np.float32), device=DEV)
    warm, _ = solve_profiled(s, params(s, warm=True, warm_probe=0.5), W=W, logV=logV)
    cold, _ = solve_profiled(s, params(s))
    assert (warm["status"] & otlm.STATUS_FALLBACK > 0).all()
    assert (warm["status"] & otlm.STATUS_CONVERGED > 0).all()
    assert rel(warm["W"], cold["W"]).max() <= 1e-6


def test_without_probe_the_prediction_is_kept(setup):
    s = setup
    _, logV, W = s["net"].infer(s["Ye"], 1024, 1024, prec="bf16")
    warm, _ = solve_profiled(s, params(s, warm=True, warm_probe=0.0), W=W, logV=logV)
    assert not (warm["status"] & otlm.STATUS_FALLBACK).any()
    assert (warm["status"] & otlm.STATUS_CONVERGED).all()
