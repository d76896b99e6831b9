"""Pins of the surrogate-MLP oracle against library routines."""
import numpy as np
import torch

from oracle import mlp


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(size=20000) * 10.0 ** rng.integers(-8, 8, size=20000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.005859375, 3.0e38, -2.5e-39]])
    want = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x), want)


def _torch_net(P):
    p = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True)
         for k, v in mlp.unpack(P).items()}
    return p


def test_unrounded_forward_backward_match_torch_autograd():
    rng = np.random.default_rng(1)
    P = mlp.init_params(rng).astype(np.float64)
    P[mlp.NP - 3:] = rng.normal(size=3)  # nonzero output bias
    x = rng.normal(size=(37, 4))
    t = rng.normal(size=(37, 3))
    w = np.array([1.0, 0.5, 2.0])
    y, _ = mlp.forward(P, x, rounding=False)
    g, dx, loss = mlp.backward(P, x, t, w, rounding=False)
    p = _torch_net(P)
    xt = torch.tensor(x, requires_grad=True)
    z1 = xt @ p["W1"].T + p["b1"]
    h1 = torch.nn.functional.silu(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = torch.nn.functional.silu(z2)
    yt = h2 @ p["W3"].T + p["b3"]
    L = (torch.tensor(w) * (yt - torch.tensor(t)) ** 2).sum() / x.shape[0]
    L.backward()
    np.testing.assert_allclose(y, yt.detach().numpy(), rtol=1e-12, atol=1e-12)
    assert abs(loss - L.item()) < 1e-12 * abs(L.item())
    tg = np.concatenate([p[k].grad.numpy().reshape(-1) for k, _ in mlp.SHAPES])
    np.testing.assert_allclose(g, tg, rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(dx, xt.grad.numpy(), rtol=1e-10, atol=1e-13)


def test_rounded_network_is_close_to_unrounded():
    rng = np.random.default_rng(2)
    P = mlp.init_params(rng)
    x = rng.normal(size=(64, 4))
    ya, _ = mlp.forward(P, x, rounding=True)
    yb, _ = mlp.forward(P, x, rounding=False)
    assert np.max(np.abs(ya - yb)) < 0.05 * np.max(np.abs(yb)) + 1e-3


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(3)
    p0 = rng.normal(size=50)
    pt = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for step in range(1, 7):
        g = rng.normal(size=50)
        pt.grad = torch.tensor(g)
        opt.step()
        p, m, v = mlp.adam(p, g, m, v, step)
        np.testing.assert_allclose(p, pt.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_adam_first_step_is_lr_times_sign():
    g = np.array([3.0, -0.5, 1e-3])
    p, _, _ = mlp.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=1e-3, eps=1e-12)
    np.testing.assert_allclose(p, -1e-3 * np.sign(g), rtol=1e-8)
