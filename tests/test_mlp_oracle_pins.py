"""Pins of the FP64 network oracle (oracle/mlp.py): bfloat16 rounding and
GELU against torch, gradients against finite differences and torch autograd,
Adam against torch.optim.Adam."""
import numpy as np
import pytest
import torch

from oracle import mlp


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e4, 100), rng.normal(0, 1e-6, 100),
                        [1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -8, 0.0, 65504.0]])
    ref = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x), ref)
    assert mlp.bf16(1 + 2 ** -8) == 1.0 and mlp.bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6


def test_gelu_matches_torch_tanh_form():
    z = np.linspace(-8, 8, 1001)
    ref = torch.nn.functional.gelu(torch.tensor(z), approximate="tanh").numpy()
    np.testing.assert_allclose(mlp.gelu(z), ref, rtol=1e-14, atol=1e-15)
    h = 1e-6
    np.testing.assert_allclose(mlp.gelu_grad(z), (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h), rtol=1e-7, atol=1e-9)


def _batch(B=64, seed=1):
    rng = np.random.default_rng(seed)
    x = np.zeros((B, mlp.N_IN_PAD))
    x[:, :mlp.N_IN] = rng.normal(0, 1, (B, mlp.N_IN))
    t = np.zeros((B, mlp.N_OUT_PAD))
    t[:, :mlp.N_OUT] = rng.normal(0, 1, (B, mlp.N_OUT))
    return x, t


def test_backward_matches_finite_differences():
    p = mlp.init_params(3)
    x, t = _batch(16)
    Y, c = mlp.forward(p, x, quantize=False)
    g = mlp.backward(p, c, Y, t, quantize=False)
    rng = np.random.default_rng(4)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in p[k].shape)
            if (k == "W1" and idx[0] >= mlp.N_IN) or (k in ("W3", "b3") and idx[-1] >= mlp.N_OUT):
                continue
            h = 1e-6
            pp = {kk: vv.copy() for kk, vv in p.items()}
            pm = {kk: vv.copy() for kk, vv in p.items()}
            pp[k][idx] += h
            pm[k][idx] -= h
            fd = (mlp.loss(mlp.forward(pp, x, False)[0], t) - mlp.loss(mlp.forward(pm, x, False)[0], t)) / (2 * h)
            assert g[k][idx] == pytest.approx(fd, rel=1e-6, abs=1e-10), (k, idx)


def test_backward_matches_torch_autograd():
    p = mlp.init_params(5)
    x, t = _batch(32, 6)
    tp = {k: torch.tensor(v, requires_grad=True) for k, v in p.items()}
    xt = torch.tensor(x)
    h1 = torch.nn.functional.gelu(xt @ tp["W1"] + tp["b1"], approximate="tanh")
    h2 = torch.nn.functional.gelu(h1 @ tp["W2"] + tp["b2"], approximate="tanh")
    y = h2 @ tp["W3"] + tp["b3"]
    l = ((y[:, :12] - torch.tensor(t[:, :12])) ** 2).mean()
    l.backward()
    Y, c = mlp.forward(p, x, quantize=False)
    assert mlp.loss(Y, t) == pytest.approx(l.item(), rel=1e-13)
    g = mlp.backward(p, c, Y, t, quantize=False)
    for k in p:
        ref = tp[k].grad.numpy().copy()
        if k == "W1":
            ref[mlp.N_IN:] = 0
        np.testing.assert_allclose(g[k], ref, rtol=1e-11, atol=1e-14)


def test_adam_matches_torch():
    p = mlp.init_params(7)
    x, t = _batch(32, 8)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(v) for k, v in p.items()}
    tp = {k: torch.tensor(val, requires_grad=True) for k, val in p.items()}
    opt = torch.optim.Adam(list(tp.values()), lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 4):
        Y, c = mlp.forward(p, x, quantize=False)
        g = mlp.backward(p, c, Y, t, quantize=False)
        mlp.adam_step(p, g, m, v, step, 1e-3)
        opt.zero_grad()
        for k in tp:
            tp[k].grad = torch.tensor(g[k])
        opt.step()
    for k in p:
        np.testing.assert_allclose(p[k], tp[k].detach().numpy(), rtol=1e-12, atol=1e-15)
