"""Seeded synthetic inputs for the OTLM solver.

This module only draws inputs: bin grids, squared-distance costs, Gaussian-peak
dictionaries and perturbed target spectra.  It contains none of the solver's
arithmetic (no Gibbs kernel, no scaling updates), so that the GPU path and the
FP64 reference can both be fed from it without sharing any of the method.

Workload recipes (readings of the problem statement, section "Optimal Transport
Linear Models"; the dictionary/target construction mirrors the spectroscopy
demonstration and the scaling-test appendix):

* bins: ``x_i = (i + 1/2) / n`` on [0, 1];
* cost: ``C_ij = (x_i - x_j)^2``;
* dictionary column j: Gaussian with centre ``c_j ~ U[0.1, 0.9]`` and standard
  deviation ``sigma_j ~ U[0.01, 0.05]``, truncated at ``|x - c_j| > 5 sigma_j``
  and normalised to unit discrete mass;
* target: every peak centre moved by one per-spectrum shift ``delta``, the
  shifted truncated Gaussians renormalised to unit mass, mixed with weights
  ``w_true ~ Exp(1)``, multiplied by a gain ``g`` and given ``|N(0, 1e-3)|``
  noise per bin (so every bin is strictly positive).

Every spectrum b of a workload draws from its own stream
``PCG64(SeedSequence([seed, b]))`` so any single spectrum of a large batch can be
regenerated on its own; the dictionary draws from ``SeedSequence([seed, DICT])``.
"""
from __future__ import annotations

import dataclasses
import numpy as np

DICT_STREAM = 1 << 30


def rng_for(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(stream)])))


def grid(n: int) -> np.ndarray:
    """Bin centres of an n-bin grid on [0, 1]."""
    return (np.arange(n, dtype=np.float64) + 0.5) / n


def sq_cost(x_src: np.ndarray, x_tgt: np.ndarray) -> np.ndarray:
    """Squared-distance cost matrix, FP64, [len(x_src), len(x_tgt)]."""
    return (x_src[:, None] - x_tgt[None, :]) ** 2


def gaussian_peaks(x: np.ndarray, centres: np.ndarray, sigmas: np.ndarray,
                   trunc: float = 5.0) -> np.ndarray:
    """Unit-mass truncated Gaussian columns, [len(x), len(centres)], FP64."""
    d = x[:, None] - centres[None, :]
    g = np.exp(-0.5 * (d / sigmas[None, :]) ** 2)
    g[np.abs(d) > trunc * sigmas[None, :]] = 0.0
    mass = g.sum(axis=0, keepdims=True)
    if np.any(mass <= 0):
        raise ValueError("a peak has no support on the grid")
    return g / mass


@dataclasses.dataclass
class Dictionary:
    x: np.ndarray        # [n] bin centres
    centres: np.ndarray  # [k]
    sigmas: np.ndarray   # [k]
    D: np.ndarray        # [n, k] FP64, unit-mass columns


def make_dictionary(n: int, k: int, seed: int) -> Dictionary:
    rng = rng_for(seed, DICT_STREAM)
    x = grid(n)
    c = rng.uniform(0.1, 0.9, k)
    s = rng.uniform(0.01, 0.05, k)
    return Dictionary(x, c, s, gaussian_peaks(x, c, s))


def make_target(d: Dictionary, seed: int, b: int, shift: float,
                gain: tuple[float, float], noise: float = 1e-3):
    """One perturbed target spectrum; returns (y [n], w_true [k], delta, g)."""
    rng = rng_for(seed, b)
    k = d.centres.size
    w_true = rng.exponential(1.0, k)
    delta = rng.uniform(-shift, shift) if shift > 0 else 0.0
    g = rng.uniform(gain[0], gain[1]) if gain[1] > gain[0] else gain[0]
    eta = np.abs(rng.normal(0.0, noise, d.x.size))
    y = g * (gaussian_peaks(d.x, d.centres + delta, d.sigmas) @ w_true) + eta
    return y, w_true, delta, g


@dataclasses.dataclass
class Workload:
    name: str
    n: int
    k: int
    B: int
    eps: float
    fit: str            # 'kl' | 'tv' | 'l2' | 'l2tv' | 'balanced'
    pen: str            # 'none' | 'l1' | 'l2sq' | 'en'
    lam: float
    alpha: float
    lam2: float = 0.0
    beta: float = 0.0
    seed: int = 0
    shift: float = 0.0
    gain: tuple = (1.0, 1.0)
    dict_seed: int | None = None

    def dictionary(self) -> Dictionary:
        return make_dictionary(self.n, self.k, self.seed if self.dict_seed is None else self.dict_seed)

    def targets(self, idx=None, dic: Dictionary | None = None) -> np.ndarray:
        """Targets [len(idx), n] FP64 (all B spectra when idx is None)."""
        dic = dic or self.dictionary()
        idx = range(self.B) if idx is None else idx
        return np.stack([make_target(dic, self.seed, int(b), self.shift, self.gain)[0] for b in idx])

    def targets_fast(self, idx=None, dic: Dictionary | None = None, device: str = "cpu", chunk: int = 2048):
        """The same targets as targets(), as a torch FP32 tensor on `device`: the
        per-spectrum random draws are taken exactly as make_target takes them
        and the shifted peaks are evaluated in FP64 with torch in chunks."""
        import torch
        dic = dic or self.dictionary()
        idx = list(range(self.B)) if idx is None else [int(b) for b in idx]
        k, n = dic.centres.size, dic.x.size
        x = torch.as_tensor(dic.x, dtype=torch.float64, device=device)
        c = torch.as_tensor(dic.centres, dtype=torch.float64, device=device)
        sg = torch.as_tensor(dic.sigmas, dtype=torch.float64, device=device)
        out = torch.empty((len(idx), n), dtype=torch.float32, device=device)
        for s0 in range(0, len(idx), chunk):
            part = idx[s0:s0 + chunk]
            w = np.empty((len(part), k))
            dg = np.empty((len(part), 2))
            eta = np.empty((len(part), n))
            for r, b in enumerate(part):
                rng = rng_for(self.seed, b)
                w[r] = rng.exponential(1.0, k)
                dg[r, 0] = rng.uniform(-self.shift, self.shift) if self.shift > 0 else 0.0
                dg[r, 1] = rng.uniform(self.gain[0], self.gain[1]) if self.gain[1] > self.gain[0] else self.gain[0]
                eta[r] = np.abs(rng.normal(0.0, 1e-3, n))
            wt = torch.as_tensor(w, device=device)
            delta = torch.as_tensor(dg[:, 0], device=device)
            gain = torch.as_tensor(dg[:, 1], device=device)
            d = x[None, :, None] - (c[None, None, :] + delta[:, None, None])      # [b, n, k]
            g = torch.exp(-0.5 * (d / sg[None, None, :]) ** 2)
            g = torch.where(d.abs() > 5.0 * sg[None, None, :], torch.zeros_like(g), g)
            g = g / g.sum(dim=1, keepdim=True)
            y = gain[:, None] * torch.einsum("bnk,bk->bn", g, wt) + torch.as_tensor(eta, device=device)
            out[s0:s0 + len(part)] = y.to(torch.float32)
        return out

    def cost(self) -> np.ndarray:
        x = grid(self.n)
        return sq_cost(x, x)


# The five workloads.  Unstated parameters: KL weight lambda = 1 wherever the
# datafit is KL; squared-l2 penalty is alpha/2 ||w||^2; l1 penalty is alpha ||w||_1.
CONFIG1 = Workload("single_n200_k10", n=200, k=10, B=1, eps=0.01, fit="kl", pen="l2sq",
                   lam=1.0, alpha=1e-3, seed=1, shift=0.02, gain=(1.0, 1.0))
CONFIG2 = Workload("batch_n1024_k64_l1", n=1024, k=64, B=4096, eps=0.005, fit="kl", pen="l1",
                   lam=1.0, alpha=1e-2, seed=2, shift=0.03, gain=(0.8, 1.2))
CONFIG3 = dataclasses.replace(CONFIG2, name="batch_n1024_k64_l1_eps1e-3", eps=0.001)
CONFIG5_EVAL = dataclasses.replace(CONFIG2, name="heldout_n1024_k64_l1_eps2e-3", eps=0.002,
                                   seed=6, dict_seed=2)
CONFIG5_TRAIN = dataclasses.replace(CONFIG5_EVAL, name="train_n1024_k64_l1_eps2e-3", B=200_000,
                                    seed=5)


# ---------------------------------------------------------------- ragged batch
RAGGED_NS = (256, 512, 1024, 2048)
RAGGED_KS = (16, 32, 64, 128)


@dataclasses.dataclass
class RaggedWorkload:
    """Spectra of uneven length, each with its own grid and dictionary.

    Spectrum b draws n_b from RAGGED_NS and k_b from RAGGED_KS, then its own
    dictionary (centres U[0.1, 0.9], sigmas U[0.01, 0.05], truncated at 5 sigma,
    unit mass) and a target built as for the single-target workload (one shift
    U[-shift, shift], gain 1, |N(0, 1e-3)| noise), all from PCG64(SeedSequence([seed, b])).
    """
    name: str = "ragged_8192_l2tv_ridge"
    B: int = 8192
    eps: float = 0.005
    fit: str = "l2tv"
    pen: str = "l2sq"
    lam: float = 1.0
    lam2: float = 0.1
    alpha: float = 1e-3
    beta: float = 0.0
    seed: int = 4
    shift: float = 0.02
    ns: tuple = RAGGED_NS
    ks: tuple = RAGGED_KS

    def spectrum(self, b: int):
        """(n, k, D [n, k] FP64, y [n] FP64) of spectrum b."""
        rng = rng_for(self.seed, b)
        n = int(rng.choice(self.ns))
        k = int(rng.choice(self.ks))
        x = grid(n)
        c = rng.uniform(0.1, 0.9, k)
        s = rng.uniform(0.01, 0.05, k)
        D = gaussian_peaks(x, c, s)
        w_true = rng.exponential(1.0, k)
        delta = rng.uniform(-self.shift, self.shift)
        eta = np.abs(rng.normal(0.0, 1e-3, n))
        y = gaussian_peaks(x, c + delta, s) @ w_true + eta
        return n, k, D, y

    def sizes(self, idx=None):
        """(n_b, k_b) for the spectra in idx, without building dictionaries."""
        idx = range(self.B) if idx is None else idx
        out = []
        for b in idx:
            rng = rng_for(self.seed, int(b))
            out.append((int(rng.choice(self.ns)), int(rng.choice(self.ks))))
        return out

    def cost(self, n: int) -> np.ndarray:
        """Squared-distance cost on the n-bin grid."""
        x = grid(n)
        return sq_cost(x, x)

    def pack(self, idx=None):
        """Packed FP32 inputs of the spectra in idx (input order): kernel index
        of each spectrum into the sorted list of distinct n, the list itself,
        k per spectrum, D_0 D_1 ... (each [n_b, k_b] row-major) and y_0 y_1 ..."""
        idx = list(range(self.B)) if idx is None else [int(b) for b in idx]
        specs = [self.spectrum(b) for b in idx]
        ns = sorted({sp[0] for sp in specs})
        kernel_of = np.array([ns.index(sp[0]) for sp in specs], dtype=np.int32)
        kdim = np.array([sp[1] for sp in specs], dtype=np.int32)
        D = np.concatenate([sp[2].astype(np.float32).ravel() for sp in specs])
        Y = np.concatenate([sp[3].astype(np.float32) for sp in specs])
        return kernel_of, ns, kdim, D, Y


CONFIG4 = RaggedWorkload()


# ---------------------------------------------------------------- warm-start network
def mlp_init(dims, seed: int) -> np.ndarray:
    """Initial flat parameters [W1, b1, W2, b2, W3, b3] of the warm-start network
    (W_l [out, in] row-major): every entry of layer l drawn U(-1/sqrt(in_l),
    1/sqrt(in_l)) from PCG64(SeedSequence([seed, l])), FP32."""
    parts = []
    for layer, (a, b) in enumerate(zip(dims[:-1], dims[1:])):
        rng = rng_for(seed, layer)
        bound = 1.0 / np.sqrt(a)
        parts.append(rng.uniform(-bound, bound, b * a))
        parts.append(rng.uniform(-bound, bound, b))
    return np.concatenate(parts).astype(np.float32)
