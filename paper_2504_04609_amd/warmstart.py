"""Warm-start pipeline around libotlm (argument marshalling and loops only).

1. Training triples: the solver itself solves the training targets; the
   network's target row for spectrum y is [log u | log v | w] of the solution.
2. Training: minibatch AdamW steps of otlm_mlp_train_step over a training set
   held in device memory, cosine learning-rate decay, seeded shuffles.
3. Warm solve: otlm_mlp_infer (BF16 by default) writes the predicted log v and
   w straight into the warm-start arrays of otlm_solve_batch, whose probe
   restarts from the cold start every spectrum whose prediction is too far off.
"""
from __future__ import annotations

import math

from . import otlm


def solve_in_chunks(kern, D, Y, params, chunk: int = 8192):
    """otlm_solve_batch over Y in chunks; returns the concatenated outputs."""
    import torch
    parts = []
    for s in range(0, Y.shape[0], chunk):
        parts.append(kern.solve(D, Y[s:s + chunk].contiguous(), params))
    return {key: (torch.cat([p[key] for p in parts]) if parts[0][key] is not None else None)
            for key in parts[0]}


def training_targets(out):
    """Network targets [B, 2n + k] = [log u | log v | w] of solver outputs."""
    import torch
    return torch.cat([out["logU"], out["logV"], out["W"]], dim=1).contiguous()


def train(net, X, T, epochs: int, batch: int = 256, lr: float = 1e-3, lr_min: float = 1e-5,
          weight_decay: float = 1e-4, seed: int = 0, log=None):
    """AdamW training with the library's kernels; returns the mean minibatch
    loss of every epoch.  The learning rate follows a cosine from lr to lr_min."""
    import torch
    N = X.shape[0]
    steps = N // batch
    if steps < 1:
        raise ValueError("training set smaller than one minibatch")
    gen = torch.Generator(device=X.device).manual_seed(seed)
    losses = torch.empty(steps, device=X.device, dtype=torch.float32)
    total = epochs * steps
    history = []
    t = 0
    for e in range(epochs):
        perm = torch.randperm(N, device=X.device, generator=gen).to(torch.int32)
        for s in range(steps):
            rate = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * t / total))
            net.train_step(X, T, perm[s * batch:(s + 1) * batch], lr=rate, weight_decay=weight_decay,
                           loss=losses[s:s + 1])
            t += 1
        history.append(float(losses.mean().cpu()))
        if log:
            log(f"epoch {e + 1}/{epochs}: loss {history[-1]:.4g}")
    return history


def save_network(net, path):
    """Parameters and standardisation of a network, as an .npz file."""
    import numpy as np
    i_mu, i_sd, o_mu, o_sd = [t.cpu().numpy() for t in net.get_norm()]
    np.savez(path, dims=np.array(net.dims, dtype=np.int32), theta=net.params().cpu().numpy(), in_mu=i_mu,
             in_sd=i_sd, out_mu=o_mu, out_sd=o_sd)


def load_network(path):
    """A network written by save_network (no pickled objects are read)."""
    import numpy as np
    with np.load(path, allow_pickle=False) as f:
        net = otlm.WarmStartMLP(tuple(int(d) for d in f["dims"]), f["theta"])
        net.set_norm_stats(f["in_mu"], f["in_sd"], f["out_mu"], f["out_sd"])
    return net


def warm_solve(kern, net, D, Y, params, n: int, infer_prec: str = "bf16"):
    """Predict (log v, w) with the network, then solve from there; params must
    have warm=True (and usually warm_probe > 0)."""
    if not params.warm:
        raise ValueError("warm_solve needs params.warm = True")
    _, logV, W = net.infer(Y, n, n, prec=infer_prec)
    return kern.solve(D, Y, params, W=W, logV=logV)
