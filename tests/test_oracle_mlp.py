"""Pins of the FP64 network oracle: central-difference gradients, the
softmax cross-entropy gradient p - y, exact bfloat16 rounding, and Adam's
first step (which moves every weight by -lr sign(g))."""
import numpy as np
import pytest

from oracle import mlp


def _data(n=32, seed=0):
    rng = np.random.default_rng(seed)
    return rng.uniform(-1, 1, (n, 6)), rng.integers(0, 4, n)


def test_parameter_count():
    assert mlp.NPARAM == 34436


def test_gradient_central_differences():
    x, y = _data()
    th = mlp.he_uniform(3) * 0.5 + 0.01
    l0, g = mlp.backward(th, x, y)
    assert l0 == pytest.approx(mlp.loss(th, x, y), rel=1e-14)
    rng = np.random.default_rng(1)
    idx = np.concatenate([rng.choice(mlp.NPARAM, 60, replace=False),
                          [0, 767, 768, 17279, 33920, 34435]])
    for i in idx:
        h = 1e-6
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss(tp, x, y) - mlp.loss(tm, x, y)) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-9), i


def test_output_gradient_is_p_minus_y():
    x, y = _data(8)
    th = mlp.he_uniform(4)
    _, p, _ = mlp.forward(th, x)
    _, g = mlp.backward(th, x, y)
    L = mlp.unpack(g)
    onehot = np.eye(4)[y]
    assert np.allclose(L[3][1], (p - onehot).sum(axis=0) / len(y), atol=1e-15)


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 2 ** -7, 1.0 + 3 * 2 ** -8, -3.14159, 0.0, 1e-3])
    r = mlp.bf16(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                 # tie -> even
    assert r[2] == 1.0 + 2 ** -7
    assert r[3] == 1.0 + 2 ** -6       # tie -> even (up)
    assert r[4] == -3.140625
    for v in r:                        # exactly representable with 8 significant bits
        m, e = np.frexp(v)
        assert m * 2 ** 8 == np.round(m * 2 ** 8)


def test_adam_first_step():
    th = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -1e-3, 5.0])
    t1, m, v = mlp.adam_step(th, g, np.zeros(3), np.zeros(3), 1, lr=1e-3)
    assert np.allclose(t1 - th, -1e-3 * np.sign(g), rtol=1e-5)
