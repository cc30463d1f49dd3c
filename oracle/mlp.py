"""Oracle: the cost-model network in float64.  TEST INFRASTRUCTURE ONLY.

The paper feeds its shortest path a measured tuning profile of section times
(section 2, third paragraph).  The learned cost model replaces that profile
with a small fully connected network: inputs -> hidden ReLU layers -> one
linear output predicting ln(time in microseconds), trained on mean squared
error with Adam (Kingma and Ba, ICLR 2015: m <- b1 m + (1-b1) g,
v <- b2 v + (1-b2) g^2, step lr * m_hat / (sqrt(v_hat) + eps) with
m_hat = m / (1 - b1^t), v_hat = v / (1 - b2^t)).

Weights of layer l are W_l [out, in] (row major) and b_l [out]; a layer maps
x -> x W_l^T + b_l.  Everything here is plain numpy float64; matrix
products are numpy's.
"""
from __future__ import annotations

import numpy as np


def init_params(sizes, u):
    """He-uniform weights from the given uniform[-1,1) draws `u` (consumed in
    order: W_0 row-major, then W_1, ...); biases start at zero."""
    params, at = [], 0
    for i in range(len(sizes) - 1):
        fan_in, fan_out = sizes[i], sizes[i + 1]
        lim = np.sqrt(6.0 / fan_in)
        W = lim * np.asarray(u[at:at + fan_out * fan_in], np.float64).reshape(fan_out, fan_in)
        at += fan_out * fan_in
        params += [W, np.zeros(fan_out)]
    return params


def forward(params, x):
    """Returns (output [B], cache of pre-activations and activations)."""
    a = np.asarray(x, np.float64)
    acts, pres = [a], []
    L = len(params) // 2
    for l in range(L):
        W, b = params[2 * l], params[2 * l + 1]
        z = a @ W.T + b
        pres.append(z)
        a = np.maximum(z, 0.0) if l < L - 1 else z
        acts.append(a)
    return a[:, 0], (acts, pres)


def loss(params, x, y):
    out, _ = forward(params, x)
    return float(np.mean((out - y) ** 2))


def backward(params, x, y):
    """Gradients of the mean squared error with respect to every parameter."""
    out, (acts, pres) = forward(params, x)
    B = len(y)
    L = len(params) // 2
    grads = [None] * len(params)
    delta = (2.0 / B) * (out - np.asarray(y, np.float64))[:, None]   # dLoss/dz_last
    for l in range(L - 1, -1, -1):
        grads[2 * l] = delta.T @ acts[l]
        grads[2 * l + 1] = delta.sum(axis=0)
        if l > 0:
            delta = (delta @ params[2 * l]) * (pres[l - 1] > 0.0)
    return grads


class Adam:
    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [np.zeros_like(p) for p in params]
        self.v = [np.zeros_like(p) for p in params]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        for i, (p, g) in enumerate(zip(params, grads)):
            self.m[i] = self.b1 * self.m[i] + (1 - self.b1) * g
            self.v[i] = self.b2 * self.v[i] + (1 - self.b2) * g * g
            mh = self.m[i] / (1 - self.b1 ** self.t)
            vh = self.v[i] / (1 - self.b2 ** self.t)
            p -= self.lr * mh / (np.sqrt(vh) + self.eps)
