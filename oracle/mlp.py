"""FP64 reference of the learned configuration predictor (oracle; test
infrastructure only).

A multilayer perceptron maps workload features x (4 values) to scores over
the kernel configurations of the tuning space:

    h1 = relu(x W1 + b1)        W1: [4, 64]
    h2 = relu(h1 W2 + b2)       W2: [64, 64]
    z  = h2 W3 + b3             W3: [64, C]
    p  = softmax(z)

Training minimises the mean cross-entropy  L = -(1/B) sum_i sum_c y_ic log p_ic
against target distributions y (rows summing to one) by plain gradient
descent.  The paper names learning from tuning data as related and future
work (Sect. 2; Sect. 6); this module is the plain definition the GPU kernels
are checked against.
"""
from __future__ import annotations

import numpy as np


def init_params(rng: np.random.Generator, n_in: int, n_hidden: int, n_out: int) -> dict:
    """He-uniform weights, zero biases (FP64)."""
    def he(fan_in, fan_out):
        lim = np.sqrt(6.0 / fan_in)
        return rng.uniform(-lim, lim, (fan_in, fan_out))
    return {"W1": he(n_in, n_hidden), "b1": np.zeros(n_hidden),
            "W2": he(n_hidden, n_hidden), "b2": np.zeros(n_hidden),
            "W3": he(n_hidden, n_out), "b3": np.zeros(n_out)}


def forward(params: dict, x: np.ndarray):
    """Returns (p, cache) with p the softmax probabilities [B, C]."""
    x = np.asarray(x, dtype=np.float64)
    a1 = x @ params["W1"] + params["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ params["W2"] + params["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ params["W3"] + params["b3"]
    zs = z - z.max(axis=1, keepdims=True)
    e = np.exp(zs)
    p = e / e.sum(axis=1, keepdims=True)
    return p, (x, a1, h1, a2, h2, z)


def loss(params: dict, x: np.ndarray, y: np.ndarray) -> float:
    """Mean cross-entropy of softmax(z) against target distributions y."""
    p, _ = forward(params, x)
    return float(-np.sum(y * np.log(np.maximum(p, 1e-300))) / x.shape[0])


def backward(params: dict, x: np.ndarray, y: np.ndarray) -> dict:
    """Gradients of the mean cross-entropy with respect to every parameter."""
    p, (x, a1, h1, a2, h2, z) = forward(params, x)
    B = x.shape[0]
    dz = (p - y) / B                       # softmax + cross-entropy
    g = {"W3": h2.T @ dz, "b3": dz.sum(axis=0)}
    dh2 = dz @ params["W3"].T
    da2 = dh2 * (a2 > 0)
    g["W2"] = h1.T @ da2
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ params["W2"].T
    da1 = dh1 * (a1 > 0)
    g["W1"] = x.T @ da1
    g["b1"] = da1.sum(axis=0)
    return g


def sgd_step(params: dict, grads: dict, lr: float) -> dict:
    return {k: params[k] - lr * grads[k] for k in params}
