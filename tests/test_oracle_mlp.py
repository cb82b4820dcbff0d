"""CPU pins of the surrogate network's oracle (oracle/mlp.py).

The oracle is checked against things other than itself:
- central finite differences of the loss (its gradient),
- torch's CPU float64 Linear/SiLU layers and autograd (an independent
  implementation of the same forward and backward),
- torch.optim.Adam (an independent implementation of Kingma & Ba's update),
- torch's float32 -> bfloat16 conversion (round to nearest, ties to even),
- closed forms: silu(0) = 0, silu'(0) = 1/2, the first Adam step has size lr.
"""

import numpy as np
import pytest
import torch

from oracle import mlp


def _theta(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, size=mlp.NPARAM)


def _data(seed, n=37):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, mlp.NIN))
    t = rng.normal(size=n)
    return X, t


def _torch_net(theta):
    p = mlp.unpack(theta)
    net = torch.nn.Sequential(torch.nn.Linear(6, 64), torch.nn.SiLU(), torch.nn.Linear(64, 64), torch.nn.SiLU(),
                              torch.nn.Linear(64, 1)).double()
    with torch.no_grad():
        for layer, (w, b) in zip((net[0], net[2], net[4]), (("W1", "b1"), ("W2", "b2"), ("W3", "b3"))):
            layer.weight.copy_(torch.from_numpy(p[w].copy()))
            layer.bias.copy_(torch.from_numpy(p[b].copy()))
    return net


def test_parameter_count_and_pack_roundtrip():
    assert mlp.NPARAM == 6 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 4673
    th = _theta(0)
    assert np.array_equal(mlp.pack(mlp.unpack(th)), th)


def test_silu_closed_forms():
    assert mlp.silu(np.array(0.0)) == 0.0
    assert mlp.silu_grad(np.array(0.0)) == 0.5
    assert abs(mlp.silu(np.array(40.0)) - 40.0) < 1e-15
    assert abs(mlp.silu(np.array(-40.0))) < 1e-15
    z = np.linspace(-6, 6, 25)
    h = 1e-6
    fd = (mlp.silu(z + h) - mlp.silu(z - h)) / (2 * h)
    assert np.max(np.abs(fd - mlp.silu_grad(z))) < 1e-9


def test_forward_matches_torch_layers():
    th = _theta(1)
    X, _ = _data(2)
    y, _ = mlp.forward(th, X)
    with torch.no_grad():
        ref = _torch_net(th)(torch.from_numpy(X)).numpy()[:, 0]
    assert np.max(np.abs(y - ref)) <= 1e-13 * max(1.0, np.abs(ref).max())


def test_gradient_matches_torch_autograd():
    th = _theta(3)
    X, t = _data(4)
    L, g = mlp.loss_and_grad(th, X, t)
    net = _torch_net(th)
    out = net(torch.from_numpy(X))[:, 0]
    lt = torch.mean((out - torch.from_numpy(t)) ** 2)
    lt.backward()
    ref = np.concatenate([net[0].weight.grad.numpy().ravel(), net[0].bias.grad.numpy(),
                          net[2].weight.grad.numpy().ravel(), net[2].bias.grad.numpy(),
                          net[4].weight.grad.numpy().ravel(), net[4].bias.grad.numpy()])
    assert abs(L - lt.item()) <= 1e-13 * abs(L)
    assert np.linalg.norm(g - ref) <= 1e-12 * np.linalg.norm(ref)


def test_gradient_matches_central_differences():
    th = _theta(5)
    X, t = _data(6, n=11)
    _, g = mlp.loss_and_grad(th, X, t)
    rng = np.random.default_rng(7)
    idx = np.concatenate([np.arange(0, 6), rng.choice(mlp.NPARAM, 60, replace=False), [mlp.NPARAM - 1]])
    h = 1e-6
    fd = np.empty(idx.size)
    for j, i in enumerate(idx):
        e = np.zeros(mlp.NPARAM)
        e[i] = h
        fd[j] = (mlp.loss(th + e, X, t) - mlp.loss(th - e, X, t)) / (2 * h)
    assert np.linalg.norm(fd - g[idx]) <= 1e-6 * np.linalg.norm(g[idx])


def test_adam_matches_torch_optimizer():
    th = _theta(8)
    X, t = _data(9)
    m = np.zeros(mlp.NPARAM)
    v = np.zeros(mlp.NPARAM)
    net = _torch_net(th)
    opt = torch.optim.Adam(net.parameters(), lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    cur = th.copy()
    for step in range(1, 6):
        _, g = mlp.loss_and_grad(cur, X, t)
        cur, m, v = mlp.adam(cur, g, m, v, step)
        opt.zero_grad()
        out = net(torch.from_numpy(X))[:, 0]
        torch.mean((out - torch.from_numpy(t)) ** 2).backward()
        opt.step()
    ref = np.concatenate([q.detach().numpy().ravel() for q in net.parameters()])
    assert np.max(np.abs(cur - ref)) <= 1e-13


def test_adam_first_step_has_size_lr():
    th = _theta(10)
    g = np.random.default_rng(11).normal(size=mlp.NPARAM)
    new, _, _ = mlp.adam(th, g, np.zeros_like(th), np.zeros_like(th), 1, lr=1e-3, eps=0.0)
    assert np.allclose(np.abs(new - th), 1e-3, rtol=1e-12)


def test_bf16_round_matches_torch_conversion():
    rng = np.random.default_rng(12)
    x = rng.normal(size=4096).astype(np.float32) * np.float32(10.0) ** rng.integers(-30, 30, 4096).astype(np.float32)
    # exact ties (low 16 bits = 0x8000) with even and odd kept bits, and special values
    ties = (np.arange(64, dtype=np.uint32) << 16 | 0x3F800000 | 0x8000).view(np.float32)
    special = np.array([0.0, -0.0, np.inf, -np.inf, 3.3895314e38, -3.3895314e38, 1e-45, 1.0, -1.0],
                       dtype=np.float32)
    x = np.concatenate([x, ties, special])
    got = mlp.bf16_round(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    nan = mlp.bf16_round(np.array([np.nan], dtype=np.float32))
    assert np.isnan(nan).all()


def test_truncation_error_label():
    g = np.zeros((6, 2, 2, 2))
    g[1, 0, 0, 0] = 4.0
    assert mlp.truncation_error(g, g) == mlp.FLOOR
    loc = g.copy()
    loc[3, 1, 1, 1] = 4e-3
    assert mlp.truncation_error(loc, g) == pytest.approx(-3.0, abs=1e-12)
    loc[3, 1, 1, 1] = 4e-30
    assert mlp.truncation_error(loc, g) == mlp.FLOOR


def test_features():
    f = mlp.features([0, 4, 100], [4, 16, 64], [0.5, 0.5, 1.0], [16, 20, 40], [0.1, 0.2, 0.3], [8, 16, 64])
    assert f.shape == (3, 6)
    assert np.allclose(f[:, 0], [0.0, 0.5, 0.02])
    assert np.allclose(f[:, 1], [2, 4, 6])
    assert np.allclose(f[:, 5], [3, 4, 6])
