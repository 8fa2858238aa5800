"""The weight-window network's GPU kernels (FP32 MFMA training, BF16 MFMA
inference, through the C ABI) against the FP64 NumPy oracle."""
import numpy as np
import pytest

from oracle import mlp_oracle as mo


def data(n, seed=0):
    rng = np.random.default_rng(seed)
    X = np.zeros((n, 8), dtype=np.float32)
    X[:, :3] = rng.uniform(0, 1, (n, 3))
    g = rng.integers(0, 2, n)
    X[np.arange(n), 3 + g] = 1.0
    t = (np.sin(3 * X[:, 0]) - 2 * X[:, 1] * X[:, 2] + 0.5 * g).astype(np.float32)
    w = rng.uniform(0.2, 1.0, n).astype(np.float32)
    w /= w.sum()
    return X, t, w


def dev(*arrs):
    import torch

    return [torch.as_tensor(a, device="cuda").contiguous() for a in arrs]


@pytest.mark.gpu
@pytest.mark.parametrize("n", [1, 16, 1000, 8003])
def test_gradient_matches_fp64_oracle(n):
    import paper_2305_07636_amd as m

    X, t, w = data(n)
    net = m.mcdc_mlp_create(seed=5)
    theta = net.get_params().astype(np.float64)
    L, g = net.grad(*dev(X, t, w))
    Lr, gr = mo.loss_and_grad(theta, X.astype(np.float64), t.astype(np.float64), w.astype(np.float64))
    print(f"[mlp] n={n} loss {L} vs {Lr}", flush=True)
    assert abs(L - Lr) <= 1e-4 * abs(Lr) + 1e-7
    err = np.abs(g - gr)
    assert err.max() <= 1e-4 * np.abs(gr).max(), (err.max(), np.abs(gr).max(), np.argmax(err))
    assert np.linalg.norm(g - gr) <= 1e-4 * np.linalg.norm(gr)


@pytest.mark.gpu
def test_gradient_is_deterministic():
    import paper_2305_07636_amd as m

    X, t, w = data(5000, 1)
    net = m.mcdc_mlp_create(seed=6)
    a = net.grad(*dev(X, t, w))[1]
    b = net.grad(*dev(X, t, w))[1]
    assert np.array_equal(a, b)


@pytest.mark.gpu
def test_training_tracks_fp64_oracle():
    import paper_2305_07636_amd as m

    X, t, w = data(2000, 2)
    net = m.mcdc_mlp_create(seed=7)
    theta0 = net.get_params().astype(np.float64)
    losses = net.train(*dev(X, t, w), steps=300, lr=2e-3)
    _, ref = mo.train(theta0, X.astype(np.float64), t.astype(np.float64), w.astype(np.float64), 300, 2e-3)
    print(f"[mlp] loss {losses[0]:.4g} -> {losses[-1]:.4g}, oracle {ref[0]:.4g} -> {ref[-1]:.4g}", flush=True)
    assert losses[-1] < 0.1 * losses[0]
    np.testing.assert_allclose(losses[:50], ref[:50], rtol=2e-3)
    assert abs(losses[-1] - ref[-1]) <= 0.05 * ref[-1]


@pytest.mark.gpu
@pytest.mark.parametrize("n", [1, 63, 8000])
def test_bf16_inference(n):
    import paper_2305_07636_amd as m

    X, t, w = data(n, 3)
    net = m.mcdc_mlp_create(seed=8)
    (Xd,) = dev(X)
    y = net.infer(Xd).cpu().numpy()
    theta = net.get_params().astype(np.float64)
    yb = mo.forward_bf16(theta, X.astype(np.float64))
    y64, _ = mo.forward(theta, X.astype(np.float64))
    scale = 1.0 + np.abs(y64).max()
    assert np.abs(y - yb).max() <= 1e-2 * scale, np.abs(y - yb).max()
    assert np.abs(y - y64).max() <= 3e-2 * scale, np.abs(y - y64).max()
