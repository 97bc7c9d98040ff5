"""FP64 reference of the surrogate network (not part of the paper's method).

A fully connected network 11 -> 128 -> 128 -> 128 -> 1 with GELU after each hidden layer
and a linear output, trained on the mean squared error with Adam. It stands in for the
history integral of eq. (P-final). This module only defines the arithmetic (forward,
backward, loss, one Adam update) so that the GPU kernels can be checked against it.

Parameters are a list of (W, b) with W of shape (fan_in, fan_out). ``round_bf16`` emulates
the GPU's storage of weights and layer inputs in bfloat16 (round to nearest even).
"""
import numpy as np
from scipy.special import erf

LAYERS = (11, 128, 128, 128, 1)


def round_bf16(x):
    """Round FP64 values to the nearest bfloat16 (ties to even), returned as FP64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)


def forward(params, x, bf16=False):
    """Returns the output (n, 1) and the per-layer cache (inputs, pre-activations)."""
    cache = []
    h = np.asarray(x, dtype=np.float64)
    last = len(params) - 1
    for i, (w, b) in enumerate(params):
        hin = round_bf16(h) if bf16 else h
        wv = round_bf16(w) if bf16 else w
        z = hin @ wv + b
        cache.append((hin, z, wv))
        h = z if i == last else gelu(z)
    return h, cache


def backward(params, cache, dy):
    """Gradients of sum(dy * output) with respect to every (W, b)."""
    grads = [None] * len(params)
    g = np.asarray(dy, dtype=np.float64)
    last = len(params) - 1
    for i in range(last, -1, -1):
        hin, z, wv = cache[i]
        if i != last:
            g = g * gelu_grad(z)
        grads[i] = (hin.T @ g, g.sum(axis=0))
        g = g @ wv.T
    return grads


def mse_loss_and_grads(params, x, y, bf16=False):
    """L = mean over samples of (f(x) - y)^2 and its gradients."""
    out, cache = forward(params, x, bf16)
    r = out[:, 0] - np.asarray(y, dtype=np.float64)
    loss = float(np.mean(r * r))
    dy = (2.0 / len(r)) * r[:, None]
    return loss, backward(params, cache, dy)


def adam_update(params, grads, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (bias-corrected), returning new params, m, v."""
    new_p, new_m, new_v = [], [], []
    c1 = 1.0 - beta1 ** step
    c2 = 1.0 - beta2 ** step
    for (w, b), (gw, gb), (mw, mb), (vw, vb) in zip(params, grads, m, v):
        out = []
        for p, gp, mp, vp in ((w, gw, mw, vw), (b, gb, mb, vb)):
            mp = beta1 * mp + (1.0 - beta1) * gp
            vp = beta2 * vp + (1.0 - beta2) * gp * gp
            p = p - lr * (mp / c1) / (np.sqrt(vp / c2) + eps)
            out.append((p, mp, vp))
        new_p.append((out[0][0], out[1][0]))
        new_m.append((out[0][1], out[1][1]))
        new_v.append((out[0][2], out[1][2]))
    return new_p, new_m, new_v
