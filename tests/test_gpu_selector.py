"""The selector network's HIP kernels against the FP64 reference, training on
the GPU, and the learned tune mode with its fallbacks."""
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import mlp as ref
import paper_1501_07350_amd as offt
from paper_1501_07350_amd import selector
import synth

pytestmark = pytest.mark.gpu

D, H = selector.feature_dim(), 64


def problem(B=200, seed=0):
    rng = np.random.default_rng(seed)
    p = np.zeros(ref.nparams(D, H), dtype=np.float32)
    from paper_1501_07350_amd import _lib
    import ctypes
    _lib.load().offt_mlp_init_params(D, H, 77 + seed, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)))
    p[H * D:H * D + H] = rng.standard_normal(H).astype(np.float32) * 0.1     # non-zero b1
    X = rng.standard_normal((B, D)).astype(np.float32)
    T = rng.standard_normal(B).astype(np.float32)
    return p, X, T


def test_forward_matches_reference():
    p, X, T = problem()
    net = selector.Network(D, H, 256, params=p)
    y = net.forward(torch.from_numpy(X).cuda()).cpu().numpy()
    yr, _ = ref.forward(p.astype(np.float64), X.astype(np.float64), D, H)
    assert np.max(np.abs(y - yr)) <= 1e-5 * max(1.0, np.max(np.abs(yr)))
    # gathered rows
    idx = torch.tensor([5, 0, 199, 17], dtype=torch.int32, device="cuda")
    y2 = net.forward(torch.from_numpy(X).cuda(), idx).cpu().numpy()
    assert np.allclose(y2, y[[5, 0, 199, 17]], rtol=0, atol=0)


def test_gradient_matches_reference():
    p, X, T = problem(B=256, seed=1)
    net = selector.Network(D, H, 256, params=p)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    grad = torch.zeros(net.P, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    idx = torch.arange(256, dtype=torch.int32, device="cuda").flip(0)
    net.gradient(Xd, Td, idx, grad, loss)
    g = grad.cpu().numpy()
    order = idx.cpu().numpy()
    gr, lr = ref.gradient(p.astype(np.float64), X[order].astype(np.float64), T[order].astype(np.float64), D, H)
    assert abs(loss.item() - lr) <= 1e-5 * max(1.0, lr)
    assert np.max(np.abs(g - gr)) <= 1e-4 * max(1e-3, np.max(np.abs(gr)))
    # the reference backward itself is pinned by finite differences (CPU tests)


def test_adam_step_matches_reference():
    p, X, T = problem(B=64, seed=2)
    net = selector.Network(D, H, 64, params=p)
    rng = np.random.default_rng(3)
    m = np.zeros(p.size)
    v = np.zeros(p.size)
    pr = p.astype(np.float64)
    for t in (1, 2, 3):
        g = (rng.standard_normal(p.size) * 0.01).astype(np.float32)
        net.adam(torch.from_numpy(g).cuda(), lr=1e-3)
        pr, m, v = ref.adam_step(pr, g.astype(np.float64), m, v, t, lr=1e-3)
    assert np.max(np.abs(net.params() - pr)) <= 1e-6


def test_training_reduces_loss():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((2048, D)).astype(np.float32)
    w = rng.standard_normal(D)
    T = (np.tanh(X @ w / 5) + 0.1 * np.maximum(X[:, 0], 0)).astype(np.float32)
    net = selector.Network(D, H, 128, seed=9)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    grad = torch.zeros(net.P, dtype=torch.float32, device="cuda")
    y0 = net.forward(Xd).cpu().numpy()
    l0 = float(np.mean((y0 - T) ** 2))
    for ep in range(20):
        perm = torch.from_numpy(rng.permutation(2048).astype(np.int32)).cuda()
        for b0 in range(0, 2048, 128):
            net.gradient(Xd, Td, perm[b0:b0 + 128], grad)
            net.adam(grad, lr=3e-3)
    y1 = net.forward(Xd).cpu().numpy()
    l1 = float(np.mean((y1 - T) ** 2))
    print(f"loss {l0:.4f} -> {l1:.4f}")
    assert l1 < 0.2 * l0


def _write_random_weights(path, seed=5):
    rng = np.random.default_rng(seed)
    p = (rng.standard_normal(ref.nparams(D, H)) * 0.1).astype(np.float32)
    selector.write_weights(path, np.zeros(D), np.ones(D), 0.0, 1.0, p)
    return p


def test_host_choice_is_argmin_of_gpu_forward(tmp_path):
    wpath = str(tmp_path / "w.txt")
    p = _write_random_weights(wpath)
    net = selector.Network(D, H, 256, params=p)
    for dims, bt, dt in [((64, 48, 60), 1, 1), ((512, 512, 512), 1, 0), ((100, 3, 250), 2, 1)]:
        plans, feats = selector.candidates(dims, bt, dt)
        y = net.forward(torch.from_numpy(feats).cuda()).cpu().numpy()
        pick = selector.choose(wpath, dims, bt, dt)
        assert pick == plans[int(np.argmin(y))]
        host = selector.scores(wpath, feats)
        assert np.max(np.abs(host - y)) <= 1e-4 * max(1.0, np.max(np.abs(y)))


def test_learned_mode_and_fallbacks(tmp_path):
    shape = (48, 60, 80)
    x = synth.complex_grid(shape, torch.complex64, device="cuda")
    ref_y = oracle.fft3(x.cpu().numpy().astype(np.complex128))
    wpath = str(tmp_path / "w.txt")
    _write_random_weights(wpath)
    corrupt = str(tmp_path / "bad.txt")
    with open(corrupt, "w") as f:
        f.write("offt-selector 1\ndims 45 64\nmean 1 2 3\n")
    for wp in (wpath, corrupt, str(tmp_path / "missing.txt")):
        plan = offt.Plan(shape, dtype=torch.complex64, tune="learned", weights_path=wp)
        y = plan.forward(x)
        torch.cuda.synchronize()
        assert oracle.rel_l2(y.cpu().numpy(), ref_y) <= oracle.tolerance(x.numel(), True), wp
        plan.close()
