"""Pins of the predictor-network oracle: bfloat16 rounding against torch's
conversion, gradients against central finite differences, Adam against
torch.optim.Adam."""
import numpy as np
import pytest
import torch

from oracle import mlp


def test_parameter_count():
    assert mlp.n_params() == 5378


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000).astype(np.float32) * 10.0 ** rng.integers(-5, 5, 10000),
                        np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 0.0, 65504.0], np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(mlp.bf16_round(x), ref)


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(1)
    p = {k: v.astype(np.float64) + 0.1 * rng.standard_normal(v.shape) for k, v in mlp.init_params(2).items()}
    X = rng.standard_normal((7, 16))
    T = rng.standard_normal((7, 2))
    _, g = mlp.loss_and_grad(p, X, T, bf16=False)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = p[name].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = mlp.loss_and_grad(p, X, T, bf16=False)
            flat[idx] = old - h
            lm, _ = mlp.loss_and_grad(p, X, T, bf16=False)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert g[name].reshape(-1)[idx] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_bf16_forward_close_to_fp64():
    rng = np.random.default_rng(3)
    p = mlp.init_params(4)
    X = rng.standard_normal((32, 16)).astype(np.float32)
    y16, _ = mlp.forward(p, X, bf16=True)
    y64, _ = mlp.forward(p, X, bf16=False)
    assert np.abs(y16 - y64).max() <= 0.05 * np.abs(y64).max()


def test_adam_matches_torch():
    rng = np.random.default_rng(5)
    p = mlp.init_params(6)
    state = mlp.adam_init(p)
    tp = {k: torch.tensor(v, requires_grad=True) for k, v in p.items()}
    opt = torch.optim.Adam(list(tp.values()), lr=3e-3, betas=(mlp.ADAM_B1, mlp.ADAM_B2), eps=mlp.ADAM_EPS)
    for t in range(1, 4):
        g = {k: rng.standard_normal(v.shape).astype(np.float32) for k, v in p.items()}
        p = mlp.adam_step(p, g, state, 3e-3, t)
        opt.zero_grad()
        for k, v in tp.items():
            v.grad = torch.from_numpy(g[k])
        opt.step()
    for k in p:
        assert np.allclose(p[k], tp[k].detach().numpy(), rtol=1e-5, atol=1e-7)


def test_training_reduces_loss_on_a_smooth_target():
    rng = np.random.default_rng(7)
    X = rng.standard_normal((256, 16)).astype(np.float32)
    T = np.stack([np.tanh(X[:, 0] + 0.5 * X[:, 1]), 0.3 * X[:, 2] ** 2 - 0.2], axis=1).astype(np.float32)
    p = mlp.init_params(8)
    st = mlp.adam_init(p)
    l0, _ = mlp.loss_and_grad(p, X, T)
    for t in range(1, 301):
        _, g = mlp.loss_and_grad(p, X, T)
        p = mlp.adam_step(p, g, st, 3e-3, t)
    l1, _ = mlp.loss_and_grad(p, X, T)
    assert l1 < 0.2 * l0
