"""Synthetic dictionaries for tests beyond the Gaussian-peak generator (shared
by the batch and ragged GPU parity tests; no GPU or library code here)."""
import numpy as np


def gapped_dictionary(n, k, seed):
    """Columns of three kinds, in shuffled order: two separated bumps (zeros inside
    the column's band), a dense column (no zeros), and a narrow bump near either
    end of the grid; unit mass each, no two alike (with l1, repeated columns
    leave w undetermined)."""
    rng = np.random.default_rng(seed)
    x = (np.arange(n) + 0.5) / n
    D = np.zeros((n, k))
    for j in range(k):
        kind = j % 4
        if kind in (0, 1):
            c1, c2 = rng.uniform(0.05, 0.45), rng.uniform(0.55, 0.95)
            s1, s2 = rng.uniform(0.01, 0.04, 2)
            col = np.exp(-0.5 * ((x - c1) / s1) ** 2) * (np.abs(x - c1) < 4 * s1)
            col += np.exp(-0.5 * ((x - c2) / s2) ** 2) * (np.abs(x - c2) < 4 * s2)
        elif kind == 2:
            col = 0.05 + np.exp(-0.5 * ((x - rng.uniform(0.2, 0.8)) / rng.uniform(0.1, 0.3)) ** 2)
        else:
            c = rng.uniform(0.01, 0.05)
            c = c if rng.random() < 0.5 else 1.0 - c
            sd = rng.uniform(0.005, 0.015)
            col = np.exp(-0.5 * ((x - c) / sd) ** 2) * (np.abs(x - c) < 3 * sd)
        D[:, j] = col / col.sum()
    return np.ascontiguousarray(D[:, rng.permutation(k)], dtype=np.float32)
