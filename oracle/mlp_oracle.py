"""Test infrastructure, not part of the product: a plain fp64 numpy reference of
the cost-model perceptron (forward pass, mean-squared-error loss, gradient by
the chain rule, Adam update) used to check the HIP kernels.

The cost model is not in the paper; nothing here is pinned by a printed value.
The gradient is pinned by central finite differences of the loss, the forward
pass by a hand-computed two-layer case (tests/test_mlp_oracle.py).

Parameter layout (one flat array): for each layer, its weights (out x in,
row-major) then its biases.  Hidden layers apply ReLU; the last layer has one
output and no activation.  loss = sum_b (y_b - t_b)^2 / (2 B).
"""

import numpy as np


def layer_dims(in_features, hidden, depth):
    return [in_features] + [hidden] * depth + [1]


def param_count(in_features, hidden, depth):
    d = layer_dims(in_features, hidden, depth)
    return sum(d[k + 1] * d[k] + d[k + 1] for k in range(len(d) - 1))


def unpack(params, dims):
    """Flat parameter array -> list of (W (out, in), b (out,)) in fp64."""
    p = np.asarray(params, dtype=np.float64)
    out, pos = [], 0
    for k in range(len(dims) - 1):
        i, o = dims[k], dims[k + 1]
        W = p[pos: pos + o * i].reshape(o, i)
        pos += o * i
        b = p[pos: pos + o]
        pos += o
        out.append((W, b))
    assert pos == p.size
    return out


def forward(params, dims, x):
    """Outputs (B,) and the per-layer pre-activations and activations."""
    layers = unpack(params, dims)
    a = np.asarray(x, dtype=np.float64)
    zs, acts = [], [a]
    for k, (W, b) in enumerate(layers):
        z = a @ W.T + b
        zs.append(z)
        a = np.maximum(z, 0.0) if k + 1 < len(layers) else z
        acts.append(a)
    return a[:, 0], zs, acts


def loss(params, dims, x, t):
    y, _, _ = forward(params, dims, x)
    d = y - np.asarray(t, dtype=np.float64)
    return float(d @ d) / (2.0 * len(d))


def gradient(params, dims, x, t):
    """d loss / d params (flat, same layout) by the chain rule."""
    layers = unpack(params, dims)
    y, zs, acts = forward(params, dims, x)
    B = len(y)
    dz = ((y - np.asarray(t, dtype=np.float64)) / B)[:, None]  # d loss / d z of the output layer
    grads = [None] * len(layers)
    for k in range(len(layers) - 1, -1, -1):
        W, _ = layers[k]
        grads[k] = (dz.T @ acts[k], dz.sum(axis=0))
        if k:
            dz = (dz @ W) * (zs[k - 1] > 0)
    return np.concatenate([np.concatenate([gW.reshape(-1), gb]) for gW, gb in grads])


def adam(params, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015) with bias correction; returns (params, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mhat = m / (1 - b1 ** step)
    vhat = v / (1 - b2 ** step)
    return params - lr * mhat / (np.sqrt(vhat) + eps), m, v
