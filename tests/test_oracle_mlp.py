"""Pins for the float64 selector-network reference: central finite differences,
masking, and that a known rule is learned."""
import numpy as np

from oracle import mlp


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


def test_parameter_count():
    assert mlp.N_PARAMS == 64 * 12 + 64 + 64 * 64 + 64 + 7 * 64 + 7 == 5447


def test_gradient_matches_central_differences():
    X, mask, y = batch(16, 0)
    theta = mlp.init(1)
    _, g = mlp.grad(theta, X, mask, y)
    rng = np.random.default_rng(2)
    idx = rng.choice(mlp.N_PARAMS, size=60, replace=False)
    h = 1e-6
    for i in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        num = (mlp.loss(tp, X, mask, y) - mlp.loss(tm, X, mask, y)) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 * max(1.0, abs(num)) + 1e-9, (i, num, g[i])


def test_masked_classes_get_zero_probability():
    X, mask, y = batch(32, 3)
    p, _ = mlp.forward(mlp.init(4), X, mask)
    assert np.all(p[mask == 0] == 0)
    np.testing.assert_allclose(p.sum(axis=1), 1.0, rtol=1e-12)


def test_adam_matches_hand_computed_first_step():
    theta = np.array([1.0, -2.0])
    g = np.array([0.5, -0.25])
    new, m, v = mlp.adam(theta, g, np.zeros(2), np.zeros(2), 1, lr=0.1)
    # at t = 1 the bias-corrected moments are g and g^2, so the step is lr*sign(g)
    np.testing.assert_allclose(new, theta - 0.1 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_learns_a_linear_cost_rule():
    """Labels from a known rule: join -> GFTR iff feature 8 (match ratio) > 0.25;
    group-by -> hash if feature 3 (log2 g) < 0.4, partition otherwise."""
    g = np.random.default_rng(5)
    n = 2000
    X = g.uniform(0, 1, size=(n, 12))
    is_join = g.uniform(size=n) < 0.5
    X[:, 0] = is_join
    mask = np.zeros((n, mlp.N_CLASSES))
    mask[np.ix_(is_join, mlp.JOIN_CLASSES)] = 1
    mask[np.ix_(~is_join, mlp.GROUPBY_CLASSES)] = 1
    y = np.where(is_join, np.where(X[:, 8] > 0.25, 0, 1), np.where(X[:, 3] < 0.4, 2, 4))
    theta = mlp.init(6)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    for t in range(1, 1501):
        b = g.choice(n, 256, replace=False)
        _, gr = mlp.grad(theta, X[b], mask[b], y[b])
        theta, m, v = mlp.adam(theta, gr, m, v, t, lr=3e-3)
    acc = float(np.mean(mlp.predict(theta, X, mask) == y))
    assert acc >= 0.99, acc
