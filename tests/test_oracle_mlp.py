"""Pins of the FP64 reference network: finite differences, Adam closed form,
bfloat16 rounding."""
import numpy as np

from oracle import mlp


def small_params(seed=1):
    return mlp.init_params(n_in=7, n_h=9, n_out=5, seed=seed)


def loss_of(p, X, T):
    Y, _ = mlp.forward(p, X)
    return mlp.mse(Y, T)[0]


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    p = small_params()
    for k in ("b1", "b2", "b3"):
        p[k] = rng.normal(0, 0.3, size=p[k].shape)
    X = rng.normal(size=(6, 7))
    T = rng.normal(size=(6, 5))
    Y, cache = mlp.forward(p, X)
    _, dY = mlp.mse(Y, T)
    g = mlp.backward(cache, dY)
    h = 1e-6
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        num = np.zeros_like(p[k])
        for idx in np.ndindex(p[k].shape):
            old = p[k][idx]
            p[k][idx] = old + h
            lp = loss_of(p, X, T)
            p[k][idx] = old - h
            lm = loss_of(p, X, T)
            p[k][idx] = old
            num[idx] = (lp - lm) / (2 * h)
        assert np.max(np.abs(num - g[k])) <= 1e-7 * max(1e-3, np.max(np.abs(g[k])))
    # input gradient
    num = np.zeros_like(X)
    for idx in np.ndindex(X.shape):
        old = X[idx]
        X[idx] = old + h
        lp = loss_of(p, X, T)
        X[idx] = old - h
        lm = loss_of(p, X, T)
        X[idx] = old
        num[idx] = (lp - lm) / (2 * h)
    assert np.max(np.abs(num - g["X"])) <= 1e-7 * np.max(np.abs(g["X"]))


def test_silu_closed_forms():
    z = np.array([-30.0, -1.0, 0.0, 1.0, 30.0])
    assert np.allclose(mlp.silu(z), z / (1 + np.exp(-z)))
    assert mlp.silu_grad(np.array([0.0]))[0] == 0.5
    assert abs(mlp.silu_grad(np.array([40.0]))[0] - 1.0) < 1e-15


def test_first_adam_step_is_sign_step():
    # after one step with zero moments, each weight moves by lr * g / (|g| + eps)
    p = small_params()
    rng = np.random.default_rng(2)
    g = {k: rng.normal(size=v.shape) for k, v in p.items()}
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(v) for k, v in p.items()}
    p0 = {k: val.copy() for k, val in p.items()}
    mlp.adam_step(p, g, m, v, 1, 1e-3)
    for k in p:
        assert np.allclose(p0[k] - p[k], 1e-3 * g[k] / (np.abs(g[k]) + 1e-8), rtol=1e-12, atol=1e-18)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -2.5, 3.0e38], np.float32)
    r = mlp.bf16_round(vals)
    # 1 + 2^-8 is a tie between 1 and 1 + 2^-7: rounds to even (1.0);
    # 1 + 3*2^-8 ties between 1+2^-7 and 1+2^-6: rounds to even (1 + 2^-6)
    assert list(r[:4]) == [1.0, 1.0, 1.0 + 2 ** -7, 1.0 + 2 ** -6]
    assert r[4] == -2.5
    x = np.random.default_rng(0).normal(size=1000).astype(np.float32)
    assert np.max(np.abs(mlp.bf16_round(x) / x - 1)) <= 2 ** -8      # unit roundoff
