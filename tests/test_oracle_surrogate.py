"""Pins of the float64 surrogate reference (oracle/surrogate.py) against
independent routines: central finite differences, PyTorch's tanh-GELU and
Adam, scipy's Spearman, and PyTorch's bfloat16 rounding."""
import numpy as np
import pytest
import torch

from oracle import surrogate as S


def _small_params(seed=0, scale=1.0):
    p = S.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    p["b1"] = rng.normal(0, 0.1, S.N_H1).astype(np.float32)
    p["b2"] = rng.normal(0, 0.1, S.N_H2).astype(np.float32)
    p["b3"] = np.array([0.3], np.float32)
    return {k: (v * scale).astype(np.float64) for k, v in p.items()}


def _batch(n=6, seed=1, n_cat=64):
    rng = np.random.default_rng(seed)
    z = np.stack([rng.permutation(64) for _ in range(n)]).astype(np.uint8)
    return S.one_hot(z, n_cat), rng.normal(0, 1, n)


def test_one_hot_structure():
    rng = np.random.default_rng(0)
    z = np.full((5, 64), 0xFF, np.uint8)
    for b in range(5):
        z[b, :12] = rng.permutation(12)
    x = S.one_hot(z, 12).reshape(5, 64, 64)
    assert x.sum() == 5 * 12
    for b in range(5):
        for c in range(64):
            row = x[b, c]
            if c < 12:
                assert row.sum() == 1 and row[z[b, c]] == 1
            else:
                assert row.sum() == 0


def test_gelu_matches_torch():
    u = np.linspace(-8, 8, 2001)
    ref = torch.nn.functional.gelu(torch.from_numpy(u), approximate="tanh").numpy()
    np.testing.assert_allclose(S.gelu(u), ref, rtol=1e-12, atol=1e-14)
    # derivative against autograd
    t = torch.from_numpy(u).requires_grad_(True)
    torch.nn.functional.gelu(t, approximate="tanh").sum().backward()
    np.testing.assert_allclose(S.gelu_grad(u), t.grad.numpy(), rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("name", ["W1", "b1", "W2", "b2", "W3", "b3"])
def test_backward_finite_differences(name):
    p = _small_params()
    x, t = _batch()
    y, cache = S.forward(p, x)
    g = S.backward(p, cache, y, t)
    rng = np.random.default_rng(hash(name) % 1000)
    flat = p[name].reshape(-1)
    gflat = g[name].reshape(-1)
    if name == "W1":   # only rows touched by the one-hot input carry gradient
        rows = np.flatnonzero(x.sum(0))
        idx = [int(r) * S.N_H1 + int(c) for r, c in zip(rng.choice(rows, 8), rng.integers(0, S.N_H1, 8))]
    else:
        idx = rng.integers(0, flat.size, 8)
    h = 1e-5
    for i in idx:
        old = flat[i]
        flat[i] = old + h
        lp = S.loss(p, x, t)
        flat[i] = old - h
        lm = S.loss(p, x, t)
        flat[i] = old
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gflat[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (name, i, fd, gflat[i])


def test_backward_matches_autograd():
    p = _small_params(3)
    x, t = _batch(4, seed=9)
    y, cache = S.forward(p, x)
    g = S.backward(p, cache, y, t)
    tp = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    xt = torch.from_numpy(x)
    h1 = torch.nn.functional.gelu(xt @ tp["W1"] + tp["b1"], approximate="tanh")
    h2 = torch.nn.functional.gelu(h1 @ tp["W2"] + tp["b2"], approximate="tanh")
    yt = (h2 @ tp["W3"])[:, 0] + tp["b3"][0]
    ((yt - torch.from_numpy(t)) ** 2).mean().backward()
    for k in p:
        np.testing.assert_allclose(g[k], tp[k].grad.numpy(), rtol=1e-9, atol=1e-12)


def test_adam_matches_torch():
    rng = np.random.default_rng(5)
    w0 = rng.normal(size=(7, 3))
    p = {"w": w0.copy()}
    m = {"w": np.zeros_like(w0)}
    v = {"w": np.zeros_like(w0)}
    tw = torch.tensor(w0, requires_grad=True)
    opt = torch.optim.Adam([tw], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 6):
        g = rng.normal(size=w0.shape)
        S.adam_step(p, {"w": g}, m, v, step)
        opt.zero_grad()
        tw.grad = torch.tensor(g)
        opt.step()
        np.testing.assert_allclose(p["w"], tw.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(6)
    a = np.concatenate([rng.normal(size=10000).astype(np.float32),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.0078125, 3e38, -2.5e-38], np.float32)])
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(S.bf16_round(a), ref)


def test_spearman_matches_scipy():
    from scipy.stats import spearmanr
    rng = np.random.default_rng(7)
    a = rng.integers(0, 20, 300).astype(float)
    b = a + rng.normal(0, 5, 300)
    assert abs(S.spearman(a, b) - spearmanr(a, b).correlation) < 1e-12
