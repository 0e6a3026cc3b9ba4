"""Benchmark: spectra solved per second on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--sample S]

Headline workload (held-out targets of the learned-warm-start workload): 4096
synthetic spectra, n = 1024 bins, k = 64 Gaussian peaks (the batched
workload's generator and dictionary), squared-distance cost, eps = 0.002, KL
datafit (lambda = 1), l1 penalty 1e-2.  Inputs are resident in HBM and K is
prebuilt before the timed region; one step is one solve of the whole batch
through the C-ABI (for the warm arms: the network's BF16 inference plus the
solve, including any fallback restarts).

Before the timed region the warm-start network (1024 -> 512 -> 512 -> 2112,
GELU) is trained on the GPU with the library's kernels on 200 000 targets of
the same generator (other seeds), solved by the library itself; generation,
solve and training times are reported apart.

A spectrum counts as solved when its weights are within 1e-5 (relative l2) of
the FP64 oracle's fixed point.  The oracle solves S sampled spectra (seed 3)
to tol 1e-10; the solved fraction of the sample scales the batch.  That oracle
run is also the CPU baseline (timed on the host cores it used).

Arms (through the C-ABI):
  paper_mm          Algorithm 1 as printed: one MM weight step per iteration,
                    FP32, cold, 300 iterations (it does not converge here)
  fp32_cold         weight prox solved exactly per iteration (Newton), FP32, cold
  fp32_64_cold      the same with an FP64 refinement phase (cold baseline)
  bf16_64_cold      BF16 kernel products in the bulk phase, FP64 refinement, cold
  bf16warm_fp32_64  BF16 network inference -> warm start (probe 0.5) -> FP32
                    bulk -> FP64 refinement  (headline)
  bf16warm_bf16_64  the same with BF16 bulk kernel products

Secondary rows: "batched" (the batched workload, eps = 0.005, cold FP32 +
FP64), "small_eps" (the same at eps = 0.001: BF16 bulk + 20 FP32 refinement
sweeps, BF16 bulk + FP64 refinement, FP32 bulk + FP64 refinement, each with its
weight-error quantiles on 256 oracle-checked spectra; skip with --no-small-eps)
and "ragged" (skip with --no-ragged): 8192 spectra with their own grid
length n in {256, 512, 1024, 2048} and dictionary (k in {16..128} Gaussian
peaks), L2 + TV datafit (1.0, 0.1), ridge 1e-3, eps 0.005, FP32, solved by one
otlm_ragged plan (grouped kernel products, banded dictionary steps with 4 MM
steps per iteration, graph-replayed check intervals), checked against the
oracle on one spectrum per (n, k) cell.

Prints one JSON line; the roofline entry is the kernel class with the largest
total time in the headline arm, timed with HIP events on the solve's stream
inside the timed region.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32_mfma": 157.3, "fp64_mfma": 78.6, "fp64_vector": 78.6, "bf16_mfma": 2500.0}  # TFLOP/s, MI355X
HEADLINE = "bf16warm_fp32_64"
# HBM traffic of the dominant kernel, from rocprofv3 FETCH_SIZE / WRITE_SIZE runs
# calibrated on a plain copy; valid only for the kernel source, the solver engine
# and the benchmark settings it was taken with (their sha256 together)
PMC_TRAFFIC = os.path.join(ROOT, "profiles", "pmc_traffic_prox_newton_fp32_warm_n1024_k64_B4096.txt")
PMC_SOURCES = [os.path.join(ROOT, "paper_2504_04609_amd", "csrc", "prox_newton.hpp"),
               os.path.join(ROOT, "paper_2504_04609_amd", "csrc", "otlm.hip"),
               os.path.abspath(__file__)]
# the same for the ragged row's kernels (MM weight step; Newton prox, both widths)
PMC_TRAFFIC_RAGGED = {
    "per-spectrum weight step": os.path.join(ROOT, "profiles", "pmc_traffic_rg_weight_step_ragged_8192.txt"),
    "prox_newton_kernel<float, float, float> (64- and 128-wide launches)":
        os.path.join(ROOT, "profiles", "pmc_traffic_prox_newton_ragged_8192.txt")}
PMC_SOURCES_RAGGED = [os.path.join(ROOT, "paper_2504_04609_amd", "csrc", f)
                      for f in ("prox_newton.hpp", "otlm.hip", "ragged.hpp", "ragged_kernels.hpp")] + \
                     [os.path.abspath(__file__)]
COPY_BYTES = 256 << 20
BASELINE_ARM = "fp32_64_cold"
# warm-start probe: l1 relative weight change over the first test interval. On the
# held-out set the network's starts stay below 0.64, random starts (w ~ U(0, 2),
# log v ~ N(0, 3)) start at 1.0 and weights 3x too large at 0.6 (median 2.0)
PROBE = 0.8


def kernel_nonzero_fraction(C, eps):
    """Fraction of K = exp(-C/eps) entries that are FP32-normal (algorithmic work)."""
    K32 = np.exp(-C / eps).astype(np.float32)
    return float(np.mean(K32 >= np.finfo(np.float32).tiny))


def cores_used():
    try:
        from threadpoolctl import threadpool_info
        return max([int(i.get("num_threads", 1)) for i in threadpool_info()] or [1])
    except Exception:
        return os.cpu_count() or 1


def arm_params(name, wl, otlm):
    base = dict(eps=wl.eps, fit=wl.fit, pen=wl.pen, lam=wl.lam, alpha=wl.alpha, check_every=5)
    # up to 8 Newton iterations of the weight prox per outer iteration (measured best on
    # this workload: 5 -> 66.6 ms, 8 -> 62.9 ms, 12 -> 65.4 ms per cold FP32+FP64 solve)
    exact = dict(base, max_iter=400, wstep="exact", inner_max=8)
    # refined arms stop when the estimated remaining weight change is below 1e-7
    # relative (100x inside the 1e-5 criterion), testing every 2 refinement
    # iterations (the library default)
    if name == "paper_mm":
        return otlm.SolveParams(**base, tol=0.0, max_iter=300, wstep="mm")
    if name == "fp32_cold":  # (FP32 alone does best with 5 Newton iterations: 62 ms, 74 ms with 8)
        return otlm.SolveParams(**dict(exact, inner_max=5), tol=1e-6)
    if name == "fp32_64_cold":
        return otlm.SolveParams(**exact, tol=1e-7, bulk_tol=1e-4, refine="fp64", refine_sweeps=300)
    if name == "bf16_64_cold":
        return otlm.SolveParams(**exact, tol=1e-7, bulk_tol=1e-3, prec="bf16", refine="fp64", refine_sweeps=300)
    if name == "bf16warm_fp32_64":
        return otlm.SolveParams(**exact, tol=1e-7, bulk_tol=1e-4, refine="fp64", refine_sweeps=300, warm=True,
                                warm_probe=PROBE)
    if name == "bf16warm_bf16_64":
        return otlm.SolveParams(**exact, tol=1e-7, bulk_tol=1e-3, prec="bf16", refine="fp64", refine_sweeps=300,
                                warm=True, warm_probe=PROBE)
    raise ValueError(name)


def sources_digest(paths=None):
    """sha256 over the files that decide the measured kernel's launches."""
    import hashlib
    h = hashlib.sha256()
    for path in (PMC_SOURCES if paths is None else paths):
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def pmc_traffic(kernel, path=None, sources=None):
    """Bytes per launch of `kernel` from the committed counter summary, or None
    when there is none or the kernel, the engine or the benchmark settings have
    changed since it was taken."""
    try:
        with open(PMC_TRAFFIC if path is None else path) as f:
            kv = dict(ln.split(":", 1) for ln in f if ":" in ln and not ln.startswith("#"))
        digest = sources_digest(sources)
    except OSError:
        return None
    kv = {a.strip(): b.strip() for a, b in kv.items()}
    if kv.get("kernel") != kernel or kv.get("sources_sha256") != digest:
        return None
    return float(kv["hbm_bytes_per_launch"])


def copy_calibration(torch):
    """One elementwise copy of COPY_BYTES (read COPY_BYTES, write COPY_BYTES),
    three times: the reference dispatch for the FETCH_SIZE / WRITE_SIZE scale."""
    src = torch.empty(COPY_BYTES // 4, dtype=torch.float32, device="cuda:0").uniform_()
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": COPY_BYTES, "copy_bytes_written": COPY_BYTES, "dispatches": 3}),
          flush=True)


def roofline(prof, B, n, k, phi):
    """Roofline entry for the kernel class with the largest total time."""
    totals = {c: v[0] * v[1] for c, v in prof.items() if isinstance(v, tuple)}
    dom = max(totals, key=totals.get)
    ms, cnt = prof[dom]
    entry = {"kernel": dom, "ms_per_launch": ms, "launches": cnt, "traffic": None}
    if dom in ("kv_product", "ktu_product", "kv_product_f64", "ktu_product_f64", "kv_product_bf16",
               "ktu_product_bf16"):
        flops = 2.0 * B * n * n * phi
        peak = {"f64": PEAK["fp64_mfma"], "bf16": PEAK["bf16_mfma"]}.get(dom.rsplit("_", 1)[-1], PEAK["fp32_mfma"])
        entry.update(bound="mfma", unit="TFLOP/s", peak=peak, flops_per_launch=flops)
    elif dom in ("weight_step", "weight_prox_f64") and prof["newton_iters"] > 0:
        # Newton on the weight prox (FP64 arithmetic): every Newton iteration and
        # spectrum takes ~6 n k flop (a = D w and the objective, the gradient, one
        # line-search evaluation); an iteration that factors anew adds its free-set
        # Hessian, 2 n flop per lower-triangle entry (m (m + 1) / 2 entries for m
        # free weights; the Cholesky factorisation, m^3 / 3 < 3 % of that, is not
        # counted); the counts are those of this kernel (FP32- or FP64-state) over
        # its timed launches.
        sfx = "fp32" if dom == "weight_step" else "fp64"
        nit, nfac = prof["newton_iters_" + sfx], prof["factorisations_" + sfx]
        nent = prof["hessian_entries_" + sfx]
        flops = (nit * 6.0 * n * k + nent * 2.0 * n) / max(cnt, 1)
        entry.update(newton_iters=nit, factorisations=nfac, hessian_entries=nent)
        entry["kernel"] = "prox_newton_kernel<float, float>" if dom == "weight_step" else \
            "prox_newton_kernel<double, double>"
        entry["traffic"] = pmc_traffic(entry["kernel"])
        entry.update(bound="alu", unit="TFLOP/s", peak=PEAK["fp64_vector"], flops_per_launch=flops)
    else:
        flops = 2.0 * B * n * k
        entry.update(bound="mfma", unit="TFLOP/s", peak=PEAK["fp32_mfma"], flops_per_launch=flops)
    entry["achieved"] = entry["flops_per_launch"] / (ms * 1e-3) / 1e12
    entry["frac"] = entry["achieved"] / entry["peak"]
    return entry


def timed(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    times = []
    out = None
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    return 1e3 * statistics.median(times), [1e3 * t for t in times], out


def oracle_reference(orc, C, wl, D, Y):
    """FP64 oracle fixed points of the rows of Y (exact weight prox, tol 1e-10)."""
    K = orc.gibbs_kernel(C, wl.eps)
    t0 = time.perf_counter()
    ref = orc.solve(K, D.astype(np.float64), Y.astype(np.float64), fit=wl.fit, pen=wl.pen, eps=wl.eps, lam=wl.lam,
                    alpha=wl.alpha, max_iter=600, tol=1e-10, mode="exact")
    return ref["W"], time.perf_counter() - t0


def check(W, ref):
    err = np.linalg.norm(W.astype(np.float64) - ref, axis=1) / np.linalg.norm(ref, axis=1)
    return {"fraction": float(np.mean(err <= 1e-5)), "max_err": float(err.max()), "median_err": float(np.median(err))}


def train_network(args, otlm, synth, warmstart, torch, kern, Dt, log):
    """Training triples from the solver, then GPU training; returns (net, info)."""
    tr = synth.CONFIG5_TRAIN
    dic = tr.dictionary()
    info = {"train_spectra": args.train, "epochs": args.epochs, "batch": 256, "lr": 1e-3, "weight_decay": 1e-4,
            "loss_weights": "log u 0, log v 1, w 16"}
    t0 = time.perf_counter()
    Yt = tr.targets_fast(range(args.train), dic=dic, device="cuda:0")
    torch.cuda.synchronize()
    info["generate_s"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    p = otlm.SolveParams(eps=tr.eps, fit=tr.fit, pen=tr.pen, lam=tr.lam, alpha=tr.alpha, check_every=5,
                         max_iter=400, wstep="exact", inner_max=8, tol=1e-8, bulk_tol=1e-4, refine="fp64",
                         refine_sweeps=300)
    out = warmstart.solve_in_chunks(kern, Dt, Yt, p)
    torch.cuda.synchronize()
    info["solve_s"] = time.perf_counter() - t0
    info["solve_converged_fraction"] = float((out["status"] & otlm.STATUS_CONVERGED > 0).float().mean())
    T = warmstart.training_targets(out)
    del out
    n = tr.n
    dims = (n, 512, 512, 2 * n + tr.k)
    net = otlm.WarmStartMLP(dims, synth.mlp_init(dims, 21))
    net.set_norm(Yt, T)
    net.set_loss_weights(np.concatenate([np.zeros(n), np.ones(n), np.full(tr.k, 16.0)]).astype(np.float32))
    t0 = time.perf_counter()
    hist = warmstart.train(net, Yt, T, args.epochs, batch=256, lr=1e-3, weight_decay=1e-4, seed=1)
    torch.cuda.synchronize()
    info["train_s"] = time.perf_counter() - t0
    info["loss_first_last_epoch"] = [hist[0], hist[-1]]
    log(f"# network: {info['train_spectra']} triples solved in {info['solve_s']:.1f} s, "
        f"{args.epochs} epochs in {info['train_s']:.1f} s, loss {hist[0]:.4g} -> {hist[-1]:.4g}")
    return net, info


def batched_row(args, otlm, synth, torch, orc):
    """The batched workload (eps = 0.005), cold FP32 bulk + FP64 refinement."""
    wl = synth.CONFIG2
    dic = wl.dictionary()
    D = dic.D.astype(np.float32)
    Y = wl.targets(dic=dic).astype(np.float32)
    C = wl.cost()
    kern = otlm.GibbsKernel(torch.as_tensor(C, device="cuda:0"), wl.eps)
    Dt, Yt = torch.as_tensor(D, device="cuda:0"), torch.as_tensor(Y, device="cuda:0")
    p = arm_params("fp32_64_cold", wl, otlm)
    ms, _, out = timed(lambda: kern.solve(Dt, Yt, p), max(1, min(args.steps, 3)), args.warmup, torch)
    row = {"workload": wl.name, "B": wl.B, "n": wl.n, "k": wl.k, "eps": wl.eps, "arm": "fp32_64_cold",
           "ms_per_solve": ms, "iters_mean": float(out["iters"].float().mean())}
    if orc is not None:
        pick = np.sort(np.random.default_rng(3).choice(wl.B, 4, replace=False))
        ref, _ = oracle_reference(orc, C, wl, D, Y[pick])
        row["check"] = check(out["W"].cpu().numpy()[pick], ref)
        row["spectra_solved_per_s"] = wl.B * row["check"]["fraction"] / (ms * 1e-3)
    kern.close()
    return row


SMALL_EPS_ARMS = ("bf16_32", "bf16_64", "fp32_64")


def small_eps_row(args, otlm, synth, torch, orc):
    """The small-eps workload (the batched one at eps = 0.001), cold: BF16 bulk
    products then 20 FP32 refinement sweeps, BF16 bulk then FP64 refinement (with
    range promotion above |log u| = 30), and FP32 bulk then FP64 refinement.  The
    weight error of each arm against the FP64 oracle on 256 sampled spectra."""
    wl = synth.CONFIG3
    dic = wl.dictionary()
    D = dic.D.astype(np.float32)
    C = wl.cost()
    Dt = torch.as_tensor(D, device="cuda:0")
    Yt = wl.targets_fast(dic=dic, device="cuda:0")
    kern = otlm.GibbsKernel(torch.as_tensor(C, device="cuda:0"), wl.eps)
    exact = dict(eps=wl.eps, fit=wl.fit, pen=wl.pen, lam=wl.lam, alpha=wl.alpha, check_every=5, max_iter=400,
                 wstep="exact", inner_max=8, tol=1e-7)
    params = {"bf16_32": otlm.SolveParams(**exact, bulk_tol=1e-3, prec="bf16", refine="fp32", refine_sweeps=20),
              "bf16_64": otlm.SolveParams(**exact, bulk_tol=1e-3, prec="bf16", refine="fp64", refine_sweeps=300),
              "fp32_64": otlm.SolveParams(**exact, bulk_tol=1e-4, refine="fp64", refine_sweeps=300)}
    row = {"workload": wl.name, "B": wl.B, "n": wl.n, "k": wl.k, "eps": wl.eps, "arms": {}}
    W = {}
    for arm in SMALL_EPS_ARMS:
        ms, _, out = timed(lambda p=params[arm]: kern.solve(Dt, Yt, p), max(1, min(args.steps, 3)), args.warmup,
                           torch)
        st = out["status"].cpu().numpy()
        W[arm] = out["W"].cpu().numpy()
        row["arms"][arm] = {"ms_per_solve": ms, "iters_mean": float(out["iters"].float().mean()),
                            "status_counts": {int(s): int(c) for s, c in zip(*np.unique(st, return_counts=True))},
                            "absorbed": int(np.sum(st & otlm.STATUS_ABSORBED > 0))}
    if orc is not None:
        pick = np.sort(np.random.default_rng(3).choice(wl.B, min(256, wl.B), replace=False))
        ref, dt = oracle_reference(orc, C, wl, D, Yt.cpu().numpy()[pick])
        row["oracle_sample"] = {"spectra": len(pick), "seconds": dt}
        for arm in SMALL_EPS_ARMS:
            a = row["arms"][arm]
            err = np.linalg.norm(W[arm][pick].astype(np.float64) - ref, axis=1) / np.linalg.norm(ref, axis=1)
            a["check"] = check(W[arm][pick], ref)
            a["err_quantiles_50_90_99_max"] = [float(x) for x in np.quantile(err, [0.5, 0.9, 0.99, 1.0])]
            a["spectra_solved_per_s"] = wl.B * a["check"]["fraction"] / (a["ms_per_solve"] * 1e-3)
    kern.close()
    return row


def ragged_row(args, otlm, synth, torch):
    """Ragged batch: time per solve, spectra/s, sampled oracle check, roofline."""
    wl = synth.CONFIG4
    kernel_of, ns, kdim, D, Y = wl.pack()
    dev = "cuda:0"
    kernels = [otlm.GibbsKernel(torch.as_tensor(wl.cost(n), device=dev), wl.eps) for n in ns]
    Dt, Yt = torch.as_tensor(D, device=dev), torch.as_tensor(Y, device=dev)
    params = otlm.SolveParams(eps=wl.eps, fit=wl.fit, pen=wl.pen, lam=wl.lam, lam2=wl.lam2, alpha=wl.alpha,
                              tol=1e-6, max_iter=3000, check_every=10, inner_max=3)
    plan = otlm.RaggedPlan(kernels, kernel_of, kdim, params)
    for _ in range(args.warmup):
        plan.solve(Dt, Yt)
    torch.cuda.synchronize()
    times = []
    for _ in range(max(1, min(args.steps, 3))):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = plan.solve(Dt, Yt)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    ms = 1e3 * statistics.median(times)
    W = out["W"].cpu().numpy()
    iters = out["iters"].cpu().numpy()
    status = out["status"].cpu().numpy()
    # kernel classes and algorithmic work from one eager, event-timed solve
    plan.profile(True)
    plan.solve(Dt, Yt)
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile(False)
    info = plan.info()
    (kv_ms, kv_n), (ws_ms, ws_n), (kt_ms, kt_n) = prof["kv_product"], prof["weight_step"], prof["ktu_product"]
    prod_ms = (kv_ms * kv_n + kt_ms * kt_n) / max(kv_n + kt_n, 1)
    prod = {"kernel": "grouped kernel products (s = K v, t = K^T u)", "bound": "mfma", "unit": "TFLOP/s",
            "peak": PEAK["fp32_mfma"], "ms_per_launch": prod_ms, "launches": kv_n + kt_n, "traffic": None,
            "flops_per_launch": 2.0 * prof["product_macs"] / max(kv_n + kt_n, 1)}
    prod["achieved"] = prod["flops_per_launch"] / (prod_ms * 1e-3) / 1e12
    wstep = {"kernel": "per-spectrum weight step", "bound": "hbm", "unit": "GB/s", "peak": 8000.0,
             "ms_per_launch": ws_ms, "launches": ws_n, "traffic": None,
             "bytes_per_launch": prof["weight_step_bytes"] / max(ws_n, 1)}
    wstep["achieved"] = wstep["bytes_per_launch"] / (ws_ms * 1e-3) / 1e9
    nt_ms, nt_n = prof["weight_prox_newton"]
    newton = {"kernel": "prox_newton_kernel<float, float, float> (64- and 128-wide launches)", "bound": "alu",
              "unit": "TFLOP/s", "peak": PEAK["fp64_vector"], "ms_per_launch": nt_ms, "launches": nt_n,
              "traffic": None, "flops_per_launch": prof["newton_flops"] / max(nt_n, 1)}
    newton["achieved"] = newton["flops_per_launch"] / (max(nt_ms, 1e-9) * 1e-3) / 1e12
    entries = (prod, wstep, newton)
    for e in entries:
        e["frac"] = e["achieved"] / e["peak"]
        if e["kernel"] in PMC_TRAFFIC_RAGGED:
            e["traffic"] = pmc_traffic(e["kernel"], PMC_TRAFFIC_RAGGED[e["kernel"]], PMC_SOURCES_RAGGED)
    dominant = max(entries, key=lambda e: e["ms_per_launch"] * e["launches"])
    row = {"workload": wl.name, "B": wl.B, "n": list(ns), "k": sorted(set(int(x) for x in kdim)),
           "datafit": "l2+tv", "lambda": wl.lam, "lambda2": wl.lam2, "penalty": "l2sq", "alpha": wl.alpha,
           "eps": wl.eps, "dtype": "f32", "inner_mm_steps": 3, "tile": info["tile"], "tile_tune_ms": info["tune_ms"],
           "ms_per_solve": ms, "ms_all": [1e3 * t for t in times], "spectra_per_s": wl.B / (ms * 1e-3),
           "iters_mean": float(iters.mean()), "iters_max": int(iters.max()),
           "iters_quantiles_50_90_99": [float(x) for x in np.quantile(iters, [0.5, 0.9, 0.99])],
           "status_counts": {int(a): int(b) for a, b in zip(*np.unique(status, return_counts=True))},
           "kernels_ms_per_launch": {c: v[0] for c, v in prof.items() if isinstance(v, tuple)},
           "kernel_launches": {c: v[1] for c, v in prof.items() if isinstance(v, tuple)},
           "roofline": dominant, "roofline_other": [e for e in entries if e is not dominant]}
    if not args.no_cpu:
        import oracle as orc
        n_of = np.array(ns)[kernel_of]
        w_off = np.concatenate([[0], np.cumsum(kdim)])
        d_off = np.concatenate([[0], np.cumsum(n_of * kdim)])
        y_off = np.concatenate([[0], np.cumsum(n_of)])
        pick = {}
        for b in range(wl.B):
            pick.setdefault((int(n_of[b]), int(kdim[b])), b)
        errs = []
        for (n, k), b in sorted(pick.items()):
            K = orc.gibbs_kernel(wl.cost(n), wl.eps)
            Db = D[d_off[b]:d_off[b + 1]].reshape(n, k).astype(np.float64)
            yb = Y[y_off[b]:y_off[b + 1]].astype(np.float64)
            ref = orc.solve(K, Db, yb[None], fit=wl.fit, pen=wl.pen, eps=wl.eps, lam=wl.lam, lam2=wl.lam2,
                            alpha=wl.alpha, max_iter=2000, tol=1e-12, mode="exact")["W"][0]
            w = W[w_off[b]:w_off[b + 1]].astype(np.float64)
            errs.append(float(np.linalg.norm(w - ref) / np.linalg.norm(ref)))
        row["check"] = {"spectra": len(errs), "sample": "first spectrum of every (n, k) cell",
                        "max_err": max(errs), "median_err": float(np.median(errs)),
                        "fraction_le_1e-5": float(np.mean(np.array(errs) <= 1e-5))}
    plan.close()
    print(f"# ragged: {ms:.1f} ms/solve, mean iters {row['iters_mean']:.1f}, max {row['iters_max']}",
          file=sys.stderr, flush=True)
    return row


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sample", type=int, default=512,
                    help="held-out spectra checked against the oracle (also the CPU-baseline sample)")
    ap.add_argument("--train", type=int, default=200_000, help="training triples for the network")
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--save-net", default=None, help="write the trained network to this .npz")
    ap.add_argument("--load-net", default=None, help="use a network saved by --save-net instead of training")
    ap.add_argument("--arms", default="paper_mm,fp32_cold,fp32_64_cold,bf16_64_cold,bf16warm_bf16_64,"
                                      "bf16warm_fp32_64")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle (profiling runs)")
    ap.add_argument("--no-ragged", action="store_true", help="skip the ragged-batch row")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-workload row")
    ap.add_argument("--no-small-eps", action="store_true", help="skip the small-eps (0.001) row")
    ap.add_argument("--ragged-only", action="store_true", help="run only the ragged-batch row")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (scale for the HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported here (the spectra are "
              "independent, so each GPU would solve its own share of the batch).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2504_04609_amd import otlm, synth, warmstart
    log = lambda msg: print(msg, file=sys.stderr, flush=True)  # noqa: E731

    if args.copy_calibration:
        copy_calibration(torch)
        return
    if args.ragged_only:
        print(json.dumps({"ragged": ragged_row(args, otlm, synth, torch)}), flush=True)
        return

    wl = synth.CONFIG5_EVAL
    B, n, k = wl.B, wl.n, wl.k
    dic = wl.dictionary()
    D = dic.D.astype(np.float32)
    C = wl.cost()
    dev = "cuda:0"
    Dt = torch.as_tensor(D, device=dev)
    Yt = wl.targets_fast(dic=dic, device=dev)
    Y = Yt.cpu().numpy()
    kern = otlm.GibbsKernel(torch.as_tensor(C, device=dev), wl.eps)
    phi = kernel_nonzero_fraction(C, wl.eps)
    arms = [a for a in args.arms.split(",") if a]
    headline = HEADLINE if HEADLINE in arms else arms[-1]
    net, net_info = None, None
    if any("warm" in a for a in arms):
        if args.load_net:
            net, net_info = warmstart.load_network(args.load_net), {"loaded_from": args.load_net}
        else:
            net, net_info = train_network(args, otlm, synth, warmstart, torch, kern, Dt, log)
            if args.save_net:
                warmstart.save_network(net, args.save_net)

    results = {}
    for arm in arms:
        params = arm_params(arm, wl, otlm)
        if params.warm:
            fn = lambda p=params: warmstart.warm_solve(kern, net, Dt, Yt, p, n, infer_prec="bf16")  # noqa: E731
        else:
            fn = lambda p=params: kern.solve(Dt, Yt, p)  # noqa: E731
        if arm == headline:  # kernel classes timed with events inside the timed steps
            for _ in range(args.warmup):
                fn()
            torch.cuda.synchronize()
            kern.profile(True)
            ms, ms_all, out = timed(fn, args.steps, 0, torch)
            prof = kern.profile_read()
            kern.profile(False)
        else:
            ms, ms_all, out = timed(fn, args.steps, args.warmup, torch)
            prof = None
        status = out["status"].cpu().numpy()
        results[arm] = {"ms_median": ms, "ms_all": ms_all, "W": out["W"].cpu().numpy(),
                        "iters_mean": float(out["iters"].float().mean()),
                        "status_counts": {int(s): int(c) for s, c in zip(*np.unique(status, return_counts=True))},
                        "fallbacks": int(np.sum(status & otlm.STATUS_FALLBACK > 0)), "prof": prof}
        log(f"# {arm}: {ms:.1f} ms/solve, mean iters {results[arm]['iters_mean']:.1f}, "
            f"status {results[arm]['status_counts']}")
    infer_ms = None
    if net is not None:
        infer_ms, _, _ = timed(lambda: net.infer(Yt, n, n, prec="bf16"), 5, 1, torch)

    # verification against the oracle on a sample (also the CPU baseline)
    cpu, orc = None, None
    solved = {a: None for a in arms}
    if not args.no_cpu:
        import oracle as orc
        pick = np.sort(np.random.default_rng(3).choice(B, args.sample, replace=False))
        ref, dt = oracle_reference(orc, C, wl, D, Y[pick])
        cpu = {"value": args.sample / dt, "unit": "spectra/s", "cores": cores_used(), "kind": "oracle",
               "sample": f"{args.sample} held-out spectra (seed 3) solved to tol 1e-10 from a cold start, FP64, "
                         "exact weight prox", "seconds": dt}
        for arm in arms:
            solved[arm] = check(results[arm]["W"][pick], ref)

    def value_of(arm):
        frac = solved[arm]["fraction"] if solved[arm] is not None else float("nan")
        return B * frac / (results[arm]["ms_median"] * 1e-3)

    h = results[headline]
    line = {
        "metric": "spectra solved/s to 1e-5 weight err, n=1024 k=64: plain FP32 vs BF16+warm",
        "value": value_of(headline),
        "unit": "spectra/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_median"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16+f32+f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "B": B, "n": n, "k": k, "eps": wl.eps, "datafit": "kl", "lambda": wl.lam,
                   "penalty": "l1", "alpha": wl.alpha, "arm": headline, "warm_probe": PROBE,
                   "solved_criterion": "rel l2 weight error <= 1e-5 vs FP64 oracle (tol 1e-10), sampled"},
        "roofline": roofline(h["prof"], B, n, k, phi) if h["prof"] else None,
        "arms": {a: {"ms_per_solve": r["ms_median"], "spectra_solved_per_s": value_of(a),
                     "iters_mean": r["iters_mean"], "status_counts": r["status_counts"],
                     "fallbacks": r["fallbacks"], "check": solved[a]} for a, r in results.items()},
        "nonzero_fraction_K": phi,
    }
    if h["prof"]:
        line["kernels_ms_per_launch"] = {c: v[0] for c, v in h["prof"].items() if isinstance(v, tuple) and v[1]}
        line["kernel_launches"] = {c: v[1] for c, v in h["prof"].items() if isinstance(v, tuple) and v[1]}
        line["newton_iters"] = h["prof"]["newton_iters"]
    for base in (BASELINE_ARM, "fp32_cold"):
        if base in results and solved[base] and solved[headline] and value_of(base) > 0:
            line[f"speedup_vs_{base}"] = value_of(headline) / value_of(base)
    if net_info is not None:
        net_info["bf16_infer_ms"] = infer_ms
        line["network"] = net_info
    if cpu is not None:
        line["cpu_baseline"] = cpu
    if not args.no_batched:
        line["batched"] = batched_row(args, otlm, synth, torch, orc)
    if not args.no_small_eps:
        line["small_eps"] = small_eps_row(args, otlm, synth, torch, orc)
    if not args.no_ragged:
        line["ragged"] = ragged_row(args, otlm, synth, torch)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
