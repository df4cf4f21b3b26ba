"""Pins of the fp64 cost-model reference (oracle/mlp_oracle.py): a hand-computed
forward pass, the chain-rule gradient against central finite differences of
the loss, and the Adam update against its first step's closed form."""

import numpy as np
import pytest

from oracle import mlp_oracle as M


def test_forward_hand_computed():
    # 2 inputs -> 2 ReLU units -> 1 output
    dims = [2, 2, 1]
    W1 = [[1.0, -2.0], [0.5, 0.25]]
    b1 = [0.5, -1.0]
    W2 = [[3.0, -1.0]]
    b2 = [0.25]
    params = np.array(sum(W1, []) + b1 + sum(W2, []) + b2)
    x = np.array([[1.0, 1.0], [4.0, 2.0]])
    # row 0: z1 = (1 - 2 + .5, .5 + .25 - 1) = (-.5, -.25) -> relu 0, 0 -> y = .25
    # row 1: z1 = (4 - 4 + .5, 2 + .5 - 1) = (.5, 1.5) -> y = 1.5 - 1.5 + .25 = .25
    y, _, _ = M.forward(params, dims, x)
    assert np.allclose(y, [0.25, 0.25])
    y2, _, _ = M.forward(params, dims, np.array([[3.0, 0.0]]))
    # z1 = (3.5, 0.5) -> y = 10.5 - 0.5 + 0.25
    assert np.allclose(y2, [10.25])
    assert M.loss(params, dims, np.array([[3.0, 0.0]]), [0.25]) == pytest.approx(100.0 / 2)


def test_param_count():
    assert M.param_count(12, 64, 3) == 12 * 64 + 64 + 2 * (64 * 64 + 64) + 64 + 1


@pytest.mark.parametrize("depth,hidden", [(1, 5), (3, 8)])
def test_gradient_finite_differences(depth, hidden):
    rng = np.random.default_rng(depth * 10 + hidden)
    dims = M.layer_dims(4, hidden, depth)
    p = rng.normal(0, 0.7, M.param_count(4, hidden, depth))
    x = rng.normal(0, 1, (9, 4))
    t = rng.normal(0, 1, 9)
    g = M.gradient(p, dims, x, t)
    h = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (M.loss(p + e, dims, x, t) - M.loss(p - e, dims, x, t)) / (2 * h)
    assert np.allclose(g, fd, rtol=1e-5, atol=1e-7)


def test_gradient_catches_planted_mistake():
    # dropping the ReLU mask in the backward pass must break the finite-difference pin
    rng = np.random.default_rng(3)
    dims = M.layer_dims(3, 6, 2)
    p = rng.normal(0, 1, M.param_count(3, 6, 2))
    x = rng.normal(0, 1, (7, 3))
    t = rng.normal(0, 1, 7)
    layers = M.unpack(p, dims)
    y, zs, acts = M.forward(p, dims, x)
    dz = ((y - t) / len(y))[:, None]
    grads = [None] * len(layers)
    for k in range(len(layers) - 1, -1, -1):
        grads[k] = (dz.T @ acts[k], dz.sum(axis=0))
        if k:
            dz = dz @ layers[k][0]  # mask dropped
    bad = np.concatenate([np.concatenate([a.reshape(-1), b]) for a, b in grads])
    assert not np.allclose(bad, M.gradient(p, dims, x, t), rtol=1e-5, atol=1e-7)


def test_adam_first_step():
    # at step 1 the bias-corrected update is lr * g / (|g| + eps), i.e. about lr * sign(g)
    p = np.array([1.0, -2.0, 0.0])
    g = np.array([0.5, -3.0, 0.0])
    p1, m, v = M.adam(p, g, np.zeros(3), np.zeros(3), 1, 0.01)
    assert np.allclose(p1, [0.99, -1.99, 0.0], atol=1e-7)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
