"""Host checks of the ragged-batch input generator (no method arithmetic)."""
import numpy as np

from paper_2504_04609_amd import synth


def test_sizes_follow_the_spectrum_draws():
    wl = synth.CONFIG4
    idx = [0, 1, 17, 4095, 8191]
    sizes = wl.sizes(idx)
    for b, (n, k) in zip(idx, sizes):
        n2, k2, D, y = wl.spectrum(b)
        assert (n, k) == (n2, k2)
        assert n in synth.RAGGED_NS and k in synth.RAGGED_KS
        assert D.shape == (n, k) and y.shape == (n,)
        assert (D >= 0).all() and (y >= 0).all()
        np.testing.assert_allclose(D.sum(axis=0), 1.0, rtol=1e-12)  # unit-mass peaks
        # peaks are cut at 5 sigma: every column is zero outside one contiguous band
        for j in range(k):
            nz = np.flatnonzero(D[:, j])
            assert nz.size and nz[-1] - nz[0] + 1 == nz.size


def test_size_mix_is_uniform_over_the_cells():
    sizes = np.array(synth.CONFIG4.sizes(range(2000)))
    for col, values in ((0, synth.RAGGED_NS), (1, synth.RAGGED_KS)):
        counts = np.array([(sizes[:, col] == v).sum() for v in values])
        assert counts.min() > 400 and counts.max() < 600


def test_pack_layout():
    wl = synth.RaggedWorkload(name="t", B=7, ns=(32, 50), ks=(2, 5), seed=3)
    ko, ns, kd, D, Y = wl.pack()
    assert ns == sorted(set(ns)) and D.dtype == np.float32 and Y.dtype == np.float32
    n_of = np.array(ns)[ko]
    assert Y.size == n_of.sum() and D.size == (n_of * kd).sum()
    off_d = np.concatenate([[0], np.cumsum(n_of * kd)])
    off_y = np.concatenate([[0], np.cumsum(n_of)])
    for b in range(wl.B):
        n, k, Db, y = wl.spectrum(b)
        np.testing.assert_array_equal(D[off_d[b]:off_d[b + 1]].reshape(n, k), Db.astype(np.float32))
        np.testing.assert_array_equal(Y[off_y[b]:off_y[b + 1]], y.astype(np.float32))
    # a subset keeps the per-spectrum draws
    ko2, ns2, kd2, D2, Y2 = wl.pack([5, 2])
    assert list(kd2) == [kd[5], kd[2]]


def test_fast_targets_equal_the_reference_generator():
    import torch
    wl = synth.CONFIG5_TRAIN
    dic = wl.dictionary()
    idx = [0, 7, 199_999]
    ref = wl.targets(idx, dic=dic).astype(np.float32)
    fast = wl.targets_fast(idx, dic=dic, chunk=2).numpy()
    np.testing.assert_allclose(fast, ref, rtol=1e-6, atol=1e-9)
