"""Pins of the FP64 reference MLP (forward, chain-rule gradients, Adam,
bf16 rounding) against independent definitions."""
import numpy as np
import pytest

from oracle import mlp


def _problem(seed=0, rows=40, F=8, H=16, O=2, groups=3):
    rng = np.random.default_rng(seed)
    p = mlp.init(F, H, O, seed=seed)
    for k in ("b1", "b2", "b3"):
        p[k] = rng.standard_normal(p[k].shape) * 0.1
    X = rng.standard_normal((rows, F))
    T = rng.standard_normal((rows, O))
    group = rng.integers(0, groups, rows)
    group[:groups] = np.arange(groups)
    return p, X, T, group


def test_forward_hand_computed():
    # 1 input, 2 hidden units per layer: every value written out by hand
    p = dict(W1=np.array([[2.0], [-1.0]]), b1=np.array([0.5, 0.25]),
             W2=np.array([[1.0, 3.0], [-2.0, 1.0]]), b2=np.array([0.0, 1.0]),
             W3=np.array([[1.0, -1.0], [0.5, 2.0]]), b3=np.array([0.1, -0.2]))
    y, _ = mlp.forward(p, np.array([[1.0], [-1.0]]))
    # x = 1: a1 = (2.5, -0.75) -> h1 = (2.5, 0); a2 = (2.5, -4) -> h2 = (2.5, 0)
    # x = -1: a1 = (-1.5, 1.25) -> h1 = (0, 1.25); a2 = (3.75, 2.25) -> h2 = (3.75, 2.25)
    assert np.allclose(y, [[2.6, 1.05], [1.6, 6.175]], atol=1e-14)


def test_group_weights_make_mean_relative_error():
    p, X, T, group = _problem()
    w = mlp.group_weights(T, group)
    L, _, y = mlp.loss_and_grad(p, X, T, w)
    G = group.max() + 1
    rel = [np.sum((y[group == g] - T[group == g]) ** 2) / np.sum(T[group == g] ** 2) for g in range(G)]
    assert L == pytest.approx(np.mean(rel), rel=1e-13)


def test_gradients_match_central_differences():
    p, X, T, group = _problem(seed=3)
    w = mlp.group_weights(T, group)
    _, g, _ = mlp.loss_and_grad(p, X, T, w)
    rng = np.random.default_rng(1)
    eps = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        idx = rng.choice(flat.size, min(12, flat.size), replace=False)
        for i in idx:
            old = flat[i]
            flat[i] = old + eps
            Lp, _, _ = mlp.loss_and_grad(p, X, T, w)
            flat[i] = old - eps
            Lm, _, _ = mlp.loss_and_grad(p, X, T, w)
            flat[i] = old
            fd = (Lp - Lm) / (2 * eps)
            an = g[k].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (k, i, fd, an)


def test_adam_matches_algorithm_on_a_quadratic():
    # minimises 0.5 |x - c|^2; first step moves every coordinate by lr
    # (bias-corrected m/sqrt(v) = sign(g)), and the iteration converges
    c = np.array([1.0, -2.0, 3.0])
    p = {"x": np.zeros(3)}
    m = {"x": np.zeros(3)}
    v = {"x": np.zeros(3)}
    mlp.adam_step(p, {"x": p["x"] - c}, m, v, 1, 0.1)
    assert np.allclose(p["x"], 0.1 * np.sign(c), atol=1e-7)
    for t in range(2, 3000):
        mlp.adam_step(p, {"x": p["x"] - c}, m, v, t, 0.01)
    assert np.allclose(p["x"], c, atol=1e-3)


def test_bf16_round_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(5)
    a = np.concatenate([rng.standard_normal(1000) * 10.0 ** rng.integers(-6, 6, 1000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.0078125, 1.01171875, 65504.0]])
    ref = torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16_round(a), ref)
