"""Oracle: the learned-closure network in plain FP64 numpy.

TEST INFRASTRUCTURE.  Only tests/, the smoke check and the benchmark's CPU
baseline may use anything under oracle/.  The product path never does.

Network (three dense layers, exact-erf GELU after the first two):
    z1 = W1 x + b1,  a1 = gelu(z1)
    z2 = W2 a1 + b2, a2 = gelu(z2)
    y  = W3 a2 + b3
Loss: mean squared error over the batch and the outputs.  The backward pass
is written out by hand (chain rule through each layer); Adam is the method of
Kingma & Ba with bias correction.

bf16=True rounds the operands of every matrix product to bfloat16 (round to
nearest, ties to even) before multiplying, and accumulates in FP64: the
precision the closure's specification fixes for its matrix products (BF16
operands, wide accumulation).  Biases, activations before rounding, the loss
and the optimiser stay in FP64.  bf16=False is the plain FP64 network, whose
gradient is the exact derivative of the loss.

Parameters live in a dict {W1, b1, W2, b2, W3, b3}; `flatten` gives the flat
blob order W1 (row-major, out x in), b1, W2, b2, W3, b3.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def bf16_round(a):
    """Round FP64 values to the nearest bfloat16 (ties to even), returned as
    FP64.  Inf/NaN pass through."""
    a = np.asarray(a, dtype=np.float64)
    out = np.empty_like(a)
    fin = np.isfinite(a)
    m, e = np.frexp(a[fin])  # a = m 2^e, 0.5 <= |m| < 1
    # bfloat16 keeps 8 significant bits: scale the mantissa to an integer
    # with 8 bits and round half to even (numpy's rint)
    out[fin] = np.ldexp(np.rint(np.ldexp(m, 8)), e - 8)
    out[~fin] = a[~fin]
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    """d gelu / dz = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def init(n_in, n_hidden, n_out, seed, fan_in=None):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases.  fan_in
    of the first layer may be smaller than n_in (padded inputs get zero
    weights)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    f1 = fan_in or n_in
    W1 = np.zeros((n_hidden, n_in))
    W1[:, :f1] = rng.uniform(-1, 1, size=(n_hidden, f1)) / math.sqrt(f1)
    W2 = rng.uniform(-1, 1, size=(n_hidden, n_hidden)) / math.sqrt(n_hidden)
    W3 = rng.uniform(-1, 1, size=(n_out, n_hidden)) / math.sqrt(n_hidden)
    return {"W1": W1, "b1": np.zeros(n_hidden), "W2": W2, "b2": np.zeros(n_hidden),
            "W3": W3, "b3": np.zeros(n_out)}


def flatten(p):
    return np.concatenate([np.asarray(p[k], dtype=np.float64).ravel() for k in NAMES])


def unflatten(flat, n_in, n_hidden, n_out):
    shapes = {"W1": (n_hidden, n_in), "b1": (n_hidden,), "W2": (n_hidden, n_hidden), "b2": (n_hidden,),
              "W3": (n_out, n_hidden), "b3": (n_out,)}
    out, o = {}, 0
    flat = np.asarray(flat, dtype=np.float64)
    for k in NAMES:
        n = int(np.prod(shapes[k]))
        out[k] = flat[o:o + n].reshape(shapes[k]).copy()
        o += n
    assert o == flat.size
    return out


def forward(p, X, bf16=False):
    """Outputs Y (batch x n_out) and the cache of the backward pass."""
    q = bf16_round if bf16 else (lambda a: a)
    Xq = q(X)
    W1, W2, W3 = q(p["W1"]), q(p["W2"]), q(p["W3"])
    z1 = Xq @ W1.T + p["b1"]
    a1 = q(gelu(z1))
    z2 = a1 @ W2.T + p["b2"]
    a2 = q(gelu(z2))
    Y = a2 @ W3.T + p["b3"]
    return Y, {"X": Xq, "W1": W1, "W2": W2, "W3": W3, "z1": z1, "a1": a1, "z2": z2, "a2": a2}


def loss(Y, T):
    return float(np.mean((Y - T) ** 2))


def backward(p, cache, Y, T, bf16=False):
    """Gradients of the mean squared error with respect to every parameter."""
    q = bf16_round if bf16 else (lambda a: a)
    B = Y.shape[0]
    dY = 2.0 * (Y - T) / (B * Y.shape[1])
    dYq = q(dY)
    g = {}
    g["W3"] = dYq.T @ cache["a2"]
    g["b3"] = dY.sum(axis=0)
    dZ2 = (dYq @ cache["W3"]) * gelu_grad(cache["z2"])
    dZ2q = q(dZ2)
    g["W2"] = dZ2q.T @ cache["a1"]
    g["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2q @ cache["W2"]) * gelu_grad(cache["z1"])
    dZ1q = q(dZ1)
    g["W1"] = dZ1q.T @ cache["X"]
    g["b1"] = dZ1.sum(axis=0)
    return g


class Adam:
    """Adam with bias correction (Kingma & Ba): m <- b1 m + (1 - b1) g,
    v <- b2 v + (1 - b2) g^2, p <- p - lr mhat / (sqrt(vhat) + eps)."""

    def __init__(self, params, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = {k: np.zeros_like(v) for k, v in params.items()}
        self.v = {k: np.zeros_like(v) for k, v in params.items()}
        self.t = 0

    def step(self, params, grads, lr=None):
        lr = self.lr if lr is None else lr
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for k in params:
            self.m[k] = self.b1 * self.m[k] + (1.0 - self.b1) * grads[k]
            self.v[k] = self.b2 * self.v[k] + (1.0 - self.b2) * grads[k] ** 2
            params[k] = params[k] - lr * (self.m[k] / c1) / (np.sqrt(self.v[k] / c2) + self.eps)
        return params
