"""GPU parity of the predictor-network kernels (bf16 MFMA forward / backward,
Adam) against the numpy oracle with the same bfloat16 rounding."""
import numpy as np
import pytest

from gpu_common import ctx

pytestmark = pytest.mark.gpu


def _pack(p):
    return np.concatenate([p["W1"].ravel(), p["b1"], p["W2"].ravel(), p["b2"], p["W3"].ravel(), p["b3"]]).astype(
        np.float32)


def _unpack(v):
    v = np.asarray(v, np.float32)
    o, p = 0, {}
    for name, shape in (("W1", (16, 64)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (64, 2)),
                        ("b3", (2,))):
        n = int(np.prod(shape))
        p[name] = v[o:o + n].reshape(shape)
        o += n
    return p


@pytest.mark.parametrize("B", [1, 37, 64, 200])
def test_forward_matches_oracle(B):
    import paper_0912_4457_amd as nks
    from oracle import mlp
    rng = np.random.default_rng(B)
    p = {k: v + 0.05 * rng.standard_normal(v.shape).astype(np.float32) for k, v in mlp.init_params(3).items()}
    X = rng.standard_normal((B, 16)).astype(np.float32)
    y_ref, _ = mlp.forward(p, X, bf16=True)
    y = nks.mlp_forward(ctx(), _pack(p), X).cpu().numpy()
    err = np.abs(y - y_ref) / (np.abs(y_ref).max() + 1e-6)
    # float32 vs float64 accumulation can move a bf16 activation by one ulp (2^-8)
    assert np.median(err) < 1e-5 and err.max() < 2e-2


@pytest.mark.parametrize("B", [16, 130, 256])
def test_gradient_matches_oracle(B):
    import paper_0912_4457_amd as nks
    from oracle import mlp
    rng = np.random.default_rng(10 + B)
    p = {k: v + 0.05 * rng.standard_normal(v.shape).astype(np.float32) for k, v in mlp.init_params(4).items()}
    X = rng.standard_normal((B, 16)).astype(np.float32)
    T = rng.standard_normal((B, 2)).astype(np.float32)
    loss_ref, g_ref = mlp.loss_and_grad(p, X, T, bf16=True)
    loss, g = nks.mlp_backward(ctx(), _pack(p), X, T)
    g = _unpack(g.cpu().numpy())
    assert float(loss.cpu()) == pytest.approx(loss_ref, rel=1e-3)
    for k in g_ref:
        assert np.linalg.norm(g[k] - g_ref[k]) <= 2e-2 * np.linalg.norm(g_ref[k]) + 1e-7, k


def test_adam_step_matches_oracle():
    import torch
    import paper_0912_4457_amd as nks
    from oracle import mlp
    rng = np.random.default_rng(7)
    p = mlp.init_params(5)
    st = mlp.adam_init(p)
    P = torch.from_numpy(_pack(p)).cuda()
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    for t in range(1, 4):
        g = {k: rng.standard_normal(v.shape).astype(np.float32) for k, v in p.items()}
        p = mlp.adam_step(p, g, st, 1e-3, t)
        nks.mlp_adam_step(ctx(), P, torch.from_numpy(_pack(g)).cuda(), M, V, t, 1e-3)
    assert np.allclose(P.cpu().numpy(), _pack(p), rtol=1e-5, atol=1e-7)


def test_gpu_training_reduces_loss():
    import torch
    import paper_0912_4457_amd as nks
    from oracle import mlp
    rng = np.random.default_rng(9)
    X = rng.standard_normal((256, 16)).astype(np.float32)
    T = np.stack([np.tanh(X[:, 0] + 0.5 * X[:, 1]), 0.3 * X[:, 2] ** 2 - 0.2], axis=1).astype(np.float32)
    P = torch.from_numpy(_pack(mlp.init_params(8))).cuda()
    M = torch.zeros_like(P)
    V = torch.zeros_like(P)
    Xd, Td = torch.from_numpy(X).cuda(), torch.from_numpy(T).cuda()
    l0, _ = nks.mlp_backward(ctx(), P, Xd, Td)
    l0 = float(l0.cpu())
    for t in range(1, 301):
        _, g = nks.mlp_backward(ctx(), P, Xd, Td)
        nks.mlp_adam_step(ctx(), P, g, M, V, t, 3e-3)
    l1, _ = nks.mlp_backward(ctx(), P, Xd, Td)
    assert float(l1.cpu()) < 0.2 * l0
