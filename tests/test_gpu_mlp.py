"""GPU parity for the selector network's HIP kernels against the float64
reference: forward probabilities, gradients of the batch-mean loss, and Adam.
FP32 against float64: rtol 1e-4 with an absolute floor of 1e-6 (sums of at most
a few hundred FP32 terms)."""
import numpy as np
import pytest

from oracle import mlp

pytestmark = pytest.mark.gpu


def batch(n, seed):
    g = np.random.default_rng(seed)
    X = g.uniform(0, 1, size=(n, 12))
    is_join = g.uniform(size=n) < 0.5
    X[:, 0] = is_join
    mask = np.zeros((n, mlp.N_CLASSES))
    mask[np.ix_(is_join, mlp.JOIN_CLASSES)] = 1
    mask[np.ix_(~is_join, mlp.GROUPBY_CLASSES)] = 1
    y = np.where(is_join, np.array(mlp.JOIN_CLASSES)[g.integers(0, 3, size=n)],
                 np.array(mlp.GROUPBY_CLASSES)[g.integers(0, 4, size=n)])
    return X, mask, y


def to_dev(a, dt):
    import torch
    return torch.tensor(a, dtype=dt, device="cuda")


def test_forward_and_gradient_match_reference():
    import torch
    import paper_2312_00720_amd as gj
    X, mask, y = batch(300, 1)
    theta = mlp.init(2).astype(np.float32).astype(np.float64)
    p_ref, _ = mlp.forward(theta, X.astype(np.float32).astype(np.float64), mask)
    L_ref, g_ref = mlp.grad(theta, X.astype(np.float32).astype(np.float64), mask, y)
    P = to_dev(theta, torch.float32)
    Xd, Md, Yd = to_dev(X, torch.float32), to_dev(mask, torch.float32), to_dev(y, torch.int32)
    p = gj.mlp_forward(P, Xd, Md).cpu().numpy()
    np.testing.assert_allclose(p, p_ref, rtol=1e-4, atol=1e-6)
    loss, g = gj.mlp_grad(P, Xd, Md, Yd)
    assert abs(float(loss.cpu()) - L_ref) <= 1e-4 * abs(L_ref)
    g = g.cpu().numpy()
    np.testing.assert_allclose(g, g_ref, rtol=1e-4, atol=1e-6 + 1e-4 * np.abs(g_ref).max())
    # deterministic: the same call gives the same bits
    _, g2 = gj.mlp_grad(P, Xd, Md, Yd)
    assert np.array_equal(g, g2.cpu().numpy())


def test_adam_matches_reference():
    import torch
    import paper_2312_00720_amd as gj
    rng = np.random.default_rng(3)
    theta = rng.normal(size=mlp.N_PARAMS)
    g = rng.normal(size=mlp.N_PARAMS) * 0.1
    m = rng.normal(size=mlp.N_PARAMS) * 0.01
    v = np.abs(rng.normal(size=mlp.N_PARAMS)) * 0.01
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    want, wm, wv = mlp.adam(f32(theta), f32(g), f32(m), f32(v), 7, lr=1e-3)
    P, G, Md, Vd = (to_dev(a, torch.float32) for a in (theta, g, m, v))
    gj.mlp_adam(P, G, Md, Vd, 7, lr=1e-3)
    np.testing.assert_allclose(P.cpu().numpy(), want, rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(Md.cpu().numpy(), wm, rtol=1e-5, atol=1e-8)
    np.testing.assert_allclose(Vd.cpu().numpy(), wv, rtol=1e-5, atol=1e-9)


def test_training_on_gpu_learns_rule():
    import torch
    import paper_2312_00720_amd as gj
    g = np.random.default_rng(5)
    n = 2000
    X = g.uniform(0, 1, size=(n, 12))
    is_join = g.uniform(size=n) < 0.5
    X[:, 0] = is_join
    mask = np.zeros((n, mlp.N_CLASSES))
    mask[np.ix_(is_join, mlp.JOIN_CLASSES)] = 1
    mask[np.ix_(~is_join, mlp.GROUPBY_CLASSES)] = 1
    y = np.where(is_join, np.where(X[:, 8] > 0.25, 0, 1), np.where(X[:, 3] < 0.4, 2, 4))
    P = to_dev(mlp.init(6), torch.float32)
    Md = torch.zeros_like(P)
    Vd = torch.zeros_like(P)
    Xd, Mk, Yd = to_dev(X, torch.float32), to_dev(mask, torch.float32), to_dev(y, torch.int32)
    for t in range(1, 1501):
        b = torch.tensor(g.choice(n, 256, replace=False), device="cuda")
        _, gr = gj.mlp_grad(P, Xd[b].contiguous(), Mk[b].contiguous(), Yd[b].contiguous())
        gj.mlp_adam(P, gr, Md, Vd, t, lr=3e-3)
    pred = gj.mlp_forward(P, Xd, Mk).argmax(dim=1).cpu().numpy()
    assert float(np.mean(pred == y)) >= 0.99
