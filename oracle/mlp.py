"""FP64 reference of the surrogate network (not part of the paper's method).

A fully connected network 16 -> 128 -> 128 -> 128 -> 1 with GELU after each hidden layer
and a linear output, trained on the mean squared error with Adam. It stands in for the
history integral of eq. (P-final). This module defines the arithmetic (forward, backward,
loss, one Adam update) and the network's inputs, so that the GPU kernels can be checked
against it.

Parameters are a list of (W, b) with W of shape (fan_in, fan_out). ``round_bf16`` emulates
the GPU's storage of weights in bfloat16 (round to nearest even) and ``round_bf16x2`` its
layer inputs, kept as two bfloat16 parts hi = bf16(v), lo = bf16(v - hi).
"""
import numpy as np
from scipy.special import erf

LAYERS = (16, 128, 128, 128, 1)
# lags in ln a below the last stored node at which the stored history is sampled
LAGS = (0.0, 0.05, 0.1, 0.2, 0.35, 0.55, 0.8, 1.2, 2.1)


def features(k_mean, a_now, m_nu_total, hist_a, hist_pm_half, hist_pnu_half, pcdm_half,
             omega_m=0.3, n_species=3):
    """The network's inputs for every bin, (B, 16), or None when the stored history does not
    reach LAGS[-1] below its last node: ln k, ln a_now, M_nu, ln a_now - ln a_{n-1},
    P_nu^{1/2}(a_{n-1}) / P_cdm^{1/2}(a_now) (what the first iteration of Sec. 4.3 (iii) puts
    into the current node), ln(a_now / a_0), ln(k (s(a_now) - s(a_{n-1})) T_nu0 / m) (the
    free-streaming kernel's argument across the last interval, m = M_nu / n_species, s of
    the matter + Lambda background), then A(ln a_{n-1} - lag) / P_cdm^{1/2}(a_now) for each
    lag, with A the stored P_M^{1/2} linear in ln a between the stored nodes (the reading
    of the history integral)."""
    from .background import T_NU0, superconformal_interval
    lna = np.log(np.asarray(hist_a, dtype=np.float64))
    pm = np.asarray(hist_pm_half, dtype=np.float64)
    pn = np.asarray(hist_pnu_half, dtype=np.float64)
    k = np.asarray(k_mean, dtype=np.float64)
    if len(lna) < 2 or lna[-1] - LAGS[-1] < lna[0]:
        return None
    B = len(k)
    ds_last = superconformal_interval(float(np.exp(lna[-1])), float(a_now), omega_m)
    x_last = k * ds_last * T_NU0 / (m_nu_total / n_species)
    cols = [np.log(k), np.full(B, np.log(a_now)), np.full(B, float(m_nu_total)),
            np.full(B, np.log(a_now) - lna[-1]), pn[-1] / pcdm_half,
            np.full(B, np.log(a_now) - lna[0]), np.log(x_last)]
    for lag in LAGS:
        u = lna[-1] - lag
        cols.append(np.array([np.interp(u, lna, pm[:, b]) for b in range(B)]) / pcdm_half)
    return np.stack(cols, axis=1)


def round_bf16(x):
    """Round FP64 values to the nearest bfloat16 (ties to even), returned as FP64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def round_bf16x2(x):
    """v as the sum of its two bfloat16 parts, hi = bf16(v) and lo = bf16(v - hi) (the
    difference taken in FP32, as on the GPU)."""
    f = np.asarray(x, dtype=np.float32).astype(np.float64)
    hi = round_bf16(f)
    lo = round_bf16((f.astype(np.float32) - hi.astype(np.float32)).astype(np.float64))
    return hi + lo


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
        hin = round_bf16x2(h) if bf16 else h
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
