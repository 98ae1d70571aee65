"""Pins for the FP64 network reference (no GPU): a forward pass worked by hand,
finite differences and an autograd run for the backward pass, torch's Adam
for the update, and planted mistakes that the pins catch."""
import numpy as np
import pytest
import torch

from oracle import mlp


def rand_problem(D=7, H=5, B=9, seed=0):
    rng = np.random.default_rng(seed)
    p = rng.standard_normal(mlp.nparams(D, H)) * 0.5
    X = rng.standard_normal((B, D))
    T = rng.standard_normal(B)
    return p, X, T


def test_forward_worked_example():
    # D = 2, H = 2: W1 = [[1, -1], [2, 0]], b1 = [0, -1]; W2 = [[1, 1], [-1, 0.5]],
    # b2 = [0.5, 0]; w3 = [2, -3], b3 = 0.25; x = (3, 1)
    # z1 = (3-1+0, 6+0-1) = (2, 5) -> a1 = (2, 5)
    # z2 = (2+5+0.5, -2+2.5+0) = (7.5, 0.5) -> a2 = (7.5, 0.5)
    # y = 2*7.5 - 3*0.5 + 0.25 = 13.75
    p = np.array([1, -1, 2, 0, 0, -1, 1, 1, -1, 0.5, 0.5, 0, 2, -3, 0.25], dtype=np.float64)
    y, (z1, a1, z2, a2) = mlp.forward(p, np.array([[3.0, 1.0]]), 2, 2)
    assert y[0] == 13.75
    # a negative pre-activation is cut: x = (-3, 1): z1 = (-4, -7) -> a1 = 0; z2 = (0.5, 0) -> y = 1.25
    y2, _ = mlp.forward(p, np.array([[-3.0, 1.0]]), 2, 2)
    assert y2[0] == 1.25


def test_gradient_matches_finite_differences():
    D, H = 7, 5
    p, X, T = rand_problem(D, H)
    g, _ = mlp.gradient(p, X, T, D, H)
    fd = mlp.finite_difference(p, X, T, D, H)
    assert np.max(np.abs(g - fd)) <= 1e-6 * max(1.0, np.max(np.abs(g)))


def test_gradient_matches_autograd():
    D, H = 6, 8
    p, X, T = rand_problem(D, H, B=13, seed=3)
    g, l = mlp.gradient(p, X, T, D, H)
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    o = 0
    W1 = pt[o:o + H * D].view(H, D); o += H * D
    b1 = pt[o:o + H]; o += H
    W2 = pt[o:o + H * H].view(H, H); o += H * H
    b2 = pt[o:o + H]; o += H
    w3 = pt[o:o + H]; o += H
    b3 = pt[o]
    Xt = torch.tensor(X)
    a1 = torch.relu(Xt @ W1.T + b1)
    a2 = torch.relu(a1 @ W2.T + b2)
    y = a2 @ w3 + b3
    lt = torch.mean((y - torch.tensor(T)) ** 2)
    lt.backward()
    assert abs(lt.item() - l) <= 1e-12 * max(1.0, abs(l))
    assert np.max(np.abs(pt.grad.numpy() - g)) <= 1e-12 * max(1.0, np.max(np.abs(g)))


def test_adam_matches_torch():
    rng = np.random.default_rng(5)
    p0 = rng.standard_normal(20)
    grads = [rng.standard_normal(20) for _ in range(4)]
    pt = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(20), np.zeros(20)
    for t, g in enumerate(grads, start=1):
        opt.zero_grad()
        pt.grad = torch.tensor(g)
        opt.step()
        p, m, v = mlp.adam_step(p, g, m, v, t, lr=1e-2)
    assert np.max(np.abs(p - pt.detach().numpy())) <= 1e-12


def test_planted_mistakes_fail_a_pin():
    D, H = 5, 4
    p, X, T = rand_problem(D, H, seed=7)
    fd = mlp.finite_difference(p, X, T, D, H)
    g, _ = mlp.gradient(p, X, T, D, H)

    def broken_relu_mask():   # derivative of relu applied at the wrong layer
        W1, b1, W2, b2, w3, b3 = mlp.unpack(p, D, H)
        y, (z1, a1, z2, a2) = mlp.forward(p, X, D, H)
        dy = 2.0 * (y - T) / X.shape[0]
        d2 = np.outer(dy, w3) * (z1 > 0)[:, :H]
        return d2.T @ a1

    def transposed_w2():
        W1, b1, W2, b2, w3, b3 = mlp.unpack(p, D, H)
        y, (z1, a1, z2, a2) = mlp.forward(p, X, D, H)
        dy = 2.0 * (y - T) / X.shape[0]
        d2 = np.outer(dy, w3) * (z2 > 0)
        d1 = (d2 @ W2.T) * (z1 > 0)
        return d1.T @ X

    o = H * D + H
    fd_W2 = fd[o:o + H * H].reshape(H, H)
    fd_W1 = fd[:H * D].reshape(H, D)
    assert np.max(np.abs(broken_relu_mask() - fd_W2)) > 1e-4
    assert np.max(np.abs(transposed_w2() - fd_W1)) > 1e-4
    # a missing 2/B factor
    assert np.max(np.abs(g / 2 - fd)) > 1e-4
