"""GPU parity of the warm-start network kernels (otlm_mlp_*) against the FP64
oracle: forward pass, standardisation, loss and gradient (FP32 GPU vs FP64 CPU,
relative l2 error per parameter block <= 1e-4), AdamW steps, and BF16
inference against FP32 inference."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import mlp as omlp
from paper_2504_04609_amd import otlm, synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
DIMS = (96, 64, 32, 48)  # small widths that still span several 64-wide tiles


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    otlm.load()


def gpu(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def blocks(v, dims):
    return [np.asarray(b).ravel() for b in omlp.unpack(np.asarray(v, dtype=np.float64), dims)]


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def data(N, dims, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(2.0, 1.5, (N, dims[0])).astype(np.float32)
    T = rng.normal(-1.0, 3.0, (N, dims[3])).astype(np.float32)
    T[rng.random(T.shape) < 0.05] = -np.inf          # log u of bins without dictionary mass
    return X, T


def test_forward_fp32_matches_oracle():
    theta = synth.mlp_init(DIMS, 1)
    net = otlm.WarmStartMLP(DIMS, theta)
    Y = np.random.default_rng(2).normal(size=(70, DIMS[0])).astype(np.float32)
    logU = torch.empty((70, 16), device=DEV)
    _, logV, W = net.infer(gpu(Y), 16, 16, prec="fp32", logU=logU)
    torch.cuda.synchronize()
    Z, _ = omlp.forward(theta.astype(np.float64), DIMS, Y.astype(np.float64))
    np.testing.assert_allclose(logU.cpu().numpy(), Z[:, :16], rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(logV.cpu().numpy(), Z[:, 16:32], rtol=1e-5, atol=1e-5)
    np.testing.assert_allclose(W.cpu().numpy(), np.maximum(Z[:, 32:], 0.0), rtol=1e-5, atol=1e-5)


def test_standardisation_matches_oracle():
    net = otlm.WarmStartMLP(DIMS, synth.mlp_init(DIMS, 3))
    X, T = data(300, DIMS, 4)
    net.set_norm(gpu(X), gpu(T))
    i_mu, i_sd, o_mu, o_sd = [t.cpu().numpy() for t in net.get_norm()]
    mu, sd = omlp.column_stats(X)
    np.testing.assert_allclose(i_mu, mu, rtol=1e-6, atol=1e-6)
    np.testing.assert_allclose(i_sd, sd, rtol=1e-6)
    mu, sd = omlp.column_stats(T, clamp=omlp.T_CLAMP)
    np.testing.assert_allclose(o_mu, mu, rtol=1e-6, atol=1e-5)
    np.testing.assert_allclose(o_sd, sd, rtol=1e-6)


@pytest.mark.parametrize("B,weighted", [(16, False), (48, False), (32, True)])
def test_gradient_matches_oracle(B, weighted):
    theta = synth.mlp_init(DIMS, 5)
    net = otlm.WarmStartMLP(DIMS, theta)
    X, T = data(200, DIMS, 6)
    net.set_norm(gpu(X), gpu(T))
    om = None
    if weighted:
        om = np.concatenate([np.zeros(16), np.ones(16), np.full(16, 4.0)]).astype(np.float32)
        net.set_loss_weights(om)
    idx = np.random.default_rng(7).choice(200, B, replace=False).astype(np.int32)
    g, loss = net.grad(gpu(X), gpu(T), gpu(idx, torch.int32))
    torch.cuda.synchronize()
    i_mu, i_sd = omlp.column_stats(X)
    o_mu, o_sd = omlp.column_stats(T, clamp=omlp.T_CLAMP)
    Xh = omlp.standardise(X[idx], i_mu, i_sd)
    Th = omlp.standardise(T[idx], o_mu, o_sd, clamp=omlp.T_CLAMP)
    L, gref = omlp.loss_and_grad(theta.astype(np.float64), DIMS, Xh, Th, weights=om)
    assert float(loss.cpu()) == pytest.approx(L, rel=1e-5)
    for name, a, b in zip(("W1", "b1", "W2", "b2", "W3", "b3"), blocks(g.cpu().numpy(), DIMS), blocks(gref, DIMS)):
        assert rel(a, b) <= 1e-4, name


def test_adamw_steps_match_oracle():
    theta = synth.mlp_init(DIMS, 8)
    net = otlm.WarmStartMLP(DIMS, theta)
    X, T = data(64, DIMS, 9)
    net.set_norm(gpu(X), gpu(T))
    i_mu, i_sd = omlp.column_stats(X)
    o_mu, o_sd = omlp.column_stats(T, clamp=omlp.T_CLAMP)
    p = theta.astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    hp = dict(lr=3e-3, b1=0.9, b2=0.99, eps=1e-8, wd=1e-2)
    for t in range(1, 4):
        idx = np.arange(16 * (t - 1), 16 * t, dtype=np.int32)
        net.train_step(gpu(X), gpu(T), gpu(idx, torch.int32), lr=hp["lr"], beta1=hp["b1"], beta2=hp["b2"],
                       eps=hp["eps"], weight_decay=hp["wd"])
        _, g = omlp.loss_and_grad(p, DIMS, omlp.standardise(X[idx], i_mu, i_sd),
                                  omlp.standardise(T[idx], o_mu, o_sd, clamp=omlp.T_CLAMP))
        p, m, v = omlp.adamw(p, g, m, v, t, hp["lr"], hp["b1"], hp["b2"], hp["eps"], hp["wd"])
    got = net.params().cpu().numpy()
    # Adam's normalised step is sign-like for tiny gradients, so compare the
    # parameter change, not the gradient
    assert rel(got - theta, p - theta) <= 1e-3
    assert net.info()["step"] == 3


def test_bf16_inference_close_to_fp32():
    theta = synth.mlp_init(DIMS, 10)
    net = otlm.WarmStartMLP(DIMS, theta)
    Y = gpu(np.random.default_rng(11).normal(size=(300, DIMS[0])))
    _, v32, w32 = net.infer(Y, 16, 16, prec="fp32")
    _, v16, w16 = net.infer(Y, 16, 16, prec="bf16")
    torch.cuda.synchronize()
    assert rel(v16.cpu().numpy(), v32.cpu().numpy()) <= 2e-2
    assert rel(w16.cpu().numpy(), w32.cpu().numpy()) <= 3e-2


def test_training_trajectory_follows_oracle():
    """200 AdamW steps on the same minibatches: the GPU loss sequence and the
    final parameters follow the FP64 oracle's training run (FP32 rounding
    drifts slowly along the trajectory: 1e-2 relative), and the loss falls."""
    teacher = synth.mlp_init(DIMS, 12) * 3.0
    rng = np.random.default_rng(13)
    X = rng.normal(size=(512, DIMS[0])).astype(np.float32)
    T = omlp.forward(teacher.astype(np.float64), DIMS, X.astype(np.float64))[0].astype(np.float32)
    theta = synth.mlp_init(DIMS, 14)
    net = otlm.WarmStartMLP(DIMS, theta)
    Xt, Tt = gpu(X), gpu(T)
    net.set_norm(Xt, Tt)
    i_mu, i_sd = omlp.column_stats(X)
    o_mu, o_sd = omlp.column_stats(T, clamp=omlp.T_CLAMP)
    Xh, Th = omlp.standardise(X, i_mu, i_sd), omlp.standardise(T, o_mu, o_sd, clamp=omlp.T_CLAMP)
    p, m, v = theta.astype(np.float64), np.zeros(theta.size), np.zeros(theta.size)
    order = np.random.default_rng(15)
    loss = torch.empty(1, device=DEV)
    gpu_loss, ref_loss = [], []
    for t in range(1, 201):
        idx = order.choice(512, 64, replace=False).astype(np.int32)
        net.train_step(Xt, Tt, gpu(idx, torch.int32), lr=2e-3, loss=loss)
        L, g = omlp.loss_and_grad(p, DIMS, Xh[idx], Th[idx])
        p, m, v = omlp.adamw(p, g, m, v, t, 2e-3)
        if t in (1, 50, 100, 200):
            gpu_loss.append(float(loss.cpu()))
            ref_loss.append(L)
    print("gpu", gpu_loss, "oracle", ref_loss)
    np.testing.assert_allclose(gpu_loss, ref_loss, rtol=1e-2)
    assert rel(net.params().cpu().numpy(), p) <= 1e-2
    assert ref_loss[-1] < 0.5 * ref_loss[0]


def test_save_and_load_keep_the_predictions(tmp_path):
    from paper_2504_04609_amd import warmstart
    net = otlm.WarmStartMLP(DIMS, synth.mlp_init(DIMS, 16))
    X, T = data(128, DIMS, 17)
    net.set_norm(gpu(X), gpu(T))
    path = str(tmp_path / "net.npz")
    warmstart.save_network(net, path)
    net2 = warmstart.load_network(path)
    Y = gpu(X[:20])
    a = net.infer(Y, 16, 16, prec="fp32")
    b = net2.infer(Y, 16, 16, prec="fp32")
    torch.cuda.synchronize()
    np.testing.assert_array_equal(a[1].cpu().numpy(), b[1].cpu().numpy())
    np.testing.assert_array_equal(a[2].cpu().numpy(), b[2].cpu().numpy())
