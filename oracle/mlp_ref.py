"""FP64 reference of the learned warm start -- TEST INFRASTRUCTURE ONLY.

The paper has no learned component; the warm start is a small multilayer
perceptron that maps one time step's loads (and calendar phase) to the
converged voltages, so that the fixed-point iteration of Algorithm 1 starts
closer to its fixed point.  This module is the plain FP64 definition the GPU
kernels are checked against: forward pass, mean-squared-error loss, backward
pass and one AdamW step, written with numpy matrix products and nothing else.

Conventions (shared with the library only through this description):
  features  x = [50 P_1..50 P_n, 50 Q_1..50 Q_n, sin/cos(2 pi minute-of-day/1440),
                 sin/cos(2 pi day/365)],  day = floor(t/1440) mod 365
  layers    h_1 = gelu(x W_1^T + b_1), ..., y = h_L W_{L+1}^T + b_{L+1}, W_l is [out, in]
  gelu      x Phi(x) = x (1 + erf(x / sqrt 2)) / 2
  target    20 [Re(V - v_s), Im(V - v_s)] per PQ bus
  loss      mean over rows and outputs of (y - target)^2
  AdamW     m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; p -= lr (mhat/(sqrt(vhat)+eps) + wd p)
            with mhat = m/(1-b1^t), vhat = v/(1-b2^t)  (Loshchilov and Hutter, decoupled decay)
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

FEAT_SCALE = 50.0
OUT_SCALE = 20.0


def features(S: np.ndarray, t_index: np.ndarray) -> np.ndarray:
    S = np.asarray(S)
    t = np.asarray(t_index, np.float64)
    mod = (t % 1440.0) / 1440.0
    day = np.floor(t / 1440.0) % 365.0 / 365.0
    cal = np.stack([np.sin(2 * math.pi * mod), np.cos(2 * math.pi * mod),
                    np.sin(2 * math.pi * day), np.cos(2 * math.pi * day)], axis=1)
    return np.concatenate([FEAT_SCALE * S.real, FEAT_SCALE * S.imag, cal], axis=1)


def targets(V: np.ndarray, vs: complex = 1.0 + 0.0j) -> np.ndarray:
    D = np.asarray(V) - vs
    return OUT_SCALE * np.concatenate([D.real, D.imag], axis=1)


def to_voltage(y: np.ndarray, vs: complex = 1.0 + 0.0j) -> np.ndarray:
    n = y.shape[1] // 2
    return vs + (y[:, :n] + 1j * y[:, n:]) / OUT_SCALE


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def layer_sizes(n_in, hidden, layers, n_out):
    return [n_in] + [hidden] * layers + [n_out]


def unpack(params: np.ndarray, sizes):
    """Flat parameter vector -> [(W [out,in], b [out]) per layer] (views)."""
    out, o = [], 0
    for a, b in zip(sizes[:-1], sizes[1:]):
        W = params[o:o + a * b].reshape(b, a)
        o += a * b
        bb = params[o:o + b]
        o += b
        out.append((W, bb))
    assert o == params.size
    return out


def num_params(sizes):
    return sum(a * b + b for a, b in zip(sizes[:-1], sizes[1:]))


def forward(params, sizes, x):
    """Returns (y, cache) with cache = pre-activations and layer inputs."""
    layers = unpack(np.asarray(params, np.float64), sizes)
    h = np.asarray(x, np.float64)
    cache = []
    for l, (W, b) in enumerate(layers):
        z = h @ W.T + b
        cache.append((h, z))
        h = gelu(z) if l < len(layers) - 1 else z
    return h, cache


def loss_and_grad(params, sizes, x, t):
    """MSE loss and its gradient with respect to the flat parameter vector."""
    y, cache = forward(params, sizes, x)
    t = np.asarray(t, np.float64)
    diff = y - t
    loss = float(np.mean(diff * diff))
    layers = unpack(np.asarray(params, np.float64), sizes)
    grads = []
    dz = 2.0 * diff / diff.size
    for l in range(len(layers) - 1, -1, -1):
        h, z = cache[l]
        W, _ = layers[l]
        if l < len(layers) - 1:
            dz = dz * gelu_grad(z)
        grads.append((dz.T @ h, dz.sum(axis=0)))
        dz = dz @ W
    grads.reverse()
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return loss, flat


def adamw_step(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8, wd=1e-4):
    """One decoupled-weight-decay Adam step (in place on copies); returns (p, m, v)."""
    p = np.array(p, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    p -= lr * (mh / (np.sqrt(vh) + eps) + wd * p)
    return p, m, v
