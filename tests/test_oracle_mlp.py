"""Pins of the oracle's surrogate network: backward pass against central finite
differences, the bfloat16 rounding against its bit-level definition, and Adam against a
hand-stepped scalar case (CPU)."""
import numpy as np
import pytest

from oracle import mlp


def _params(seed, layers=(11, 16, 16, 16, 1)):
    rng = np.random.default_rng(seed)
    return [(rng.standard_normal((a, b)) / np.sqrt(a), 0.1 * rng.standard_normal(b))
            for a, b in zip(layers[:-1], layers[1:])]


def test_backward_matches_finite_differences():
    params = _params(0)
    rng = np.random.default_rng(1)
    x = rng.standard_normal((7, 11))
    y = rng.standard_normal(7)
    _, grads = mlp.mse_loss_and_grads(params, x, y)
    h = 1e-5
    worst = 0.0
    for li, (w, b) in enumerate(params):
        for arr, g in ((w, grads[li][0]), (b, grads[li][1])):
            flat = arr.reshape(-1)
            gflat = g.reshape(-1)
            for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp, _ = mlp.mse_loss_and_grads(params, x, y)
                flat[idx] = old - h
                lm, _ = mlp.mse_loss_and_grads(params, x, y)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                worst = max(worst, abs(fd - gflat[idx]) / max(1e-3, abs(fd)))
    assert worst < 1e-6


def test_gelu_derivative_matches_finite_differences():
    x = np.linspace(-6, 6, 101)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(x), fd, atol=1e-8)
    assert mlp.gelu(0.0) == 0.0 and mlp.gelu(30.0) == pytest.approx(30.0)


def test_bf16_rounding_definition():
    # bfloat16 keeps 8 significant bits; 1 + 2^-8 is a tie and rounds to even (1.0);
    # 1 + 3*2^-8 rounds up to 1 + 2^-6.
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -2.5, 3.0e-3, 0.0])
    got = mlp.round_bf16(vals)
    assert got[0] == 1.0 and got[1] == 1.0 and got[2] == 1.0 + 2 ** -6 and got[3] == -2.5
    assert got[4] == pytest.approx(3.0e-3, rel=2 ** -8) and got[5] == 0.0
    # values already representable are unchanged
    rep = np.array([1.5, 0.15625, -96.0])
    assert np.array_equal(mlp.round_bf16(rep), rep)


def test_adam_first_step_moves_by_lr_times_sign():
    params = [(np.array([[1.0]]), np.array([0.5]))]
    grads = [(np.array([[0.3]]), np.array([-2.0]))]
    zeros = [(np.zeros((1, 1)), np.zeros(1))]
    p, m, v = mlp.adam_update(params, grads, zeros, zeros, 1, 0.01)
    # bias-corrected m/sqrt(v) = g/|g| on the first step
    assert p[0][0][0, 0] == pytest.approx(1.0 - 0.01, rel=1e-6)
    assert p[0][1][0] == pytest.approx(0.5 + 0.01, rel=1e-6)


def test_layer_sizes_give_35329_parameters():
    n = sum(a * b + b for a, b in zip(mlp.LAYERS[:-1], mlp.LAYERS[1:]))
    assert n == 35329


def test_features_sample_the_history_at_lags_in_ln_a():
    """A history linear in ln a is sampled exactly at every lag whatever the node spacing
    (irregular nodes here); lag 0 is the last stored node itself; the gap input is
    ln a_now - ln a_{n-1}; a history shorter than the longest lag has no inputs."""
    rng = np.random.default_rng(3)
    lna = np.sort(np.concatenate([[np.log(0.01)], rng.uniform(np.log(0.01), np.log(0.9), 60),
                                  [np.log(0.9)]]))
    a_nodes = np.exp(lna)
    k = np.array([0.02, 0.2, 2.0])
    slope, icpt = np.array([0.8, 1.3, 2.0]), np.array([5.0, 3.0, 1.0])
    hist = icpt[None, :] + slope[None, :] * lna[:, None]          # linear in ln a
    pcdm_half = np.array([4.0, 2.0, 0.5])
    pnu = 0.5 * hist
    f = mlp.features(k, 1.0, 0.3, a_nodes, hist, pnu, pcdm_half)
    assert f.shape == (3, 16)
    assert np.allclose(f[:, 0], np.log(k)) and np.all(f[:, 1] == 0.0) and np.all(f[:, 2] == 0.3)
    assert np.allclose(f[:, 3], -np.log(0.9), rtol=0, atol=1e-15)
    assert np.array_equal(f[:, 4], pnu[-1] / pcdm_half)
    assert np.allclose(f[:, 5], -np.log(0.01), rtol=1e-15)
    # the kernel argument across the last interval, with s from its closed-form integral
    from oracle import background as bg
    from scipy import integrate
    ds = integrate.quad(lambda a: 1.0 / (a ** 3 * bg.hubble_rate(a, 0.3)), 0.9, 1.0,
                        epsrel=1e-13)[0]
    assert np.allclose(f[:, 6], np.log(k * ds * bg.T_NU0 / 0.1), rtol=1e-9)
    for m, lag in enumerate(mlp.LAGS):
        want = (icpt + slope * (np.log(0.9) - lag)) / pcdm_half
        assert np.allclose(f[:, 7 + m], want, rtol=1e-13, atol=0)
    assert np.array_equal(f[:, 7], hist[-1] / pcdm_half)
    # the same linear history on a regular grid gives the same inputs
    reg = np.linspace(np.log(0.01), np.log(0.9), 25)
    lin = icpt + slope * reg[:, None]
    f2 = mlp.features(k, 1.0, 0.3, np.exp(reg), lin, 0.5 * lin, pcdm_half)
    assert np.allclose(f2, f, rtol=1e-12, atol=1e-14)
    # not enough history: 2.0 in ln a below the last node
    short = np.linspace(np.log(0.9) - 2.0, np.log(0.9), 30)
    assert mlp.features(k, 1.0, 0.3, np.exp(short), np.ones((30, 3)), np.ones((30, 3)),
                        pcdm_half) is None
