"""Pins of the oracle's time-stepping loop (the loop of Sec. 4.3 repeated, leapfrog in s) (CPU).

* Einstein-de Sitter, no neutrinos, a plane-wave Zel'dovich displacement: before shell
  crossing the Zel'dovich solution is exact in one dimension, so the displacement grows as
  D = a and the velocity u = dx/ds = a^2 H f psi with f = 1. The loop must converge to it at
  second order in the step (kick-drift-kick), down to the PM force's own 1e-4 error.
* A uniform lattice moving as a whole feels no force: it drifts by u (s(a1) - s(a0)).
* The PM force sums to zero, so the total momentum is conserved to rounding.
* Every step stores its node: the history grows by one row per step, at the step's a.
"""
import numpy as np
import pytest

from oracle import background as bg
from oracle import step as ostep

N, L = 16, 64.0
CELL = L / N


def _lattice():
    idx = np.stack(np.meshgrid(*(np.arange(N),) * 3, indexing="ij"), -1).reshape(-1, 3)
    return (idx + 0.5) * CELL


def _empty_history(nb=8, a=0.05):
    return dict(a=np.array([a]), pm_half=np.zeros((1, nb)), pnu_half=np.zeros((1, nb)),
                pnu_half_init=np.zeros(nb), theta_over_delta_init=np.zeros(nb))


def _plane_wave_run(n_steps, a0=0.1, a1=0.3, amp=0.05 * CELL):
    q = _lattice()
    kx = 2 * np.pi / L
    psi = np.zeros_like(q)
    psi[:, 0] = amp * np.sin(kx * q[:, 0])
    x = np.mod(q + psi, L)
    u = a0 ** 2 * float(bg.hubble_rate(a0, 1.0)) * psi
    hist = _empty_history()
    g = ostep.full_step(x, N, L, 8, hist, a0, 0.0, omega_m=1.0)["acc"]
    x1, u1, _, h1 = ostep.advance(x, u, g, hist, np.geomspace(a0, a1, n_steps + 1), N, L, 8,
                                  0.0, omega_m=1.0)
    d = np.mod(x1 - q + L / 2, L) - L / 2
    grow = a1 / a0
    d_amp = 2 * np.mean(d[:, 0] * np.sin(kx * q[:, 0])) / (amp * grow) - 1
    u_amp = (2 * np.mean(u1[:, 0] * np.sin(kx * q[:, 0]))
             / (a1 ** 2 * float(bg.hubble_rate(a1, 1.0)) * amp * grow) - 1)
    return d_amp, u_amp, u1, h1


def test_eds_plane_wave_grows_as_a_at_second_order():
    errs = []
    for n in (2, 4, 8, 16):
        d_err, u_err, _, _ = _plane_wave_run(n)
        errs.append(abs(d_err))
    errs = np.array(errs)
    assert errs[-1] < 1e-3
    ratio = errs[:-1] / errs[1:]
    assert np.all((ratio > 3.4) & (ratio < 4.3)), ratio
    assert abs(u_err) < 5e-4


def test_transverse_components_stay_unperturbed():
    _, _, u1, _ = _plane_wave_run(4)
    assert np.abs(u1[:, 1:]).max() < 1e-12 * np.abs(u1[:, 0]).max()


def test_uniform_drift_and_momentum():
    q = _lattice()
    u0 = np.array([3e-4, -1e-4, 2e-4])
    vel = np.tile(u0, (len(q), 1))
    hist = _empty_history()
    a0, a1 = 0.2, 0.5
    g = ostep.full_step(q, N, L, 8, hist, a0, 0.0)["acc"]
    assert np.abs(g).max() < 1e-12
    steps = np.geomspace(a0, a1, 4)
    x1, u1, _, h1 = ostep.advance(q, vel, g, hist, steps, N, L, 8, 0.0)
    ds = bg.superconformal_interval(a0, a1, 0.3)
    shift = np.mod(x1 - q + L / 2, L) - L / 2
    assert np.allclose(shift, np.tile(u0 * ds, (len(q), 1)), rtol=1e-9, atol=1e-12)
    assert np.allclose(u1, vel, rtol=0, atol=1e-15)
    assert len(h1["a"]) == 1 + 3 and np.allclose(h1["a"][1:], steps[1:])


def test_total_momentum_is_conserved_with_neutrinos():
    from synth import log_spaced_nodes, synthetic_history, zeldovich_ics
    a0 = 0.1
    pos, vel = zeldovich_ics(16, L, 0.3, 5, a0)
    sp = ostep.spectrum(pos, N, L, 8)
    nodes = log_spaced_nodes(0.01, a0, 10)
    hist = synthetic_history(sp["k_mean"], np.sqrt(sp["p_cdm"]), nodes, 0.3)   # nodes < a0
    r = ostep.full_step(pos, N, L, 8, hist, a0, 0.3)
    hist["a"] = np.append(hist["a"], a0)
    hist["pm_half"] = np.vstack([hist["pm_half"], r["pm_half_now"]])
    hist["pnu_half"] = np.vstack([hist["pnu_half"], r["pnu_half"]])
    x1, u1, g1, h1 = ostep.advance(pos, vel, r["acc"], hist, np.geomspace(a0, 0.2, 4), N, L, 8,
                                   0.3)
    p0 = vel.astype(np.float64).sum(0)
    assert np.abs(u1.sum(0) - p0).max() < 1e-12 * np.abs(u1).sum(0).max()
    assert len(h1["a"]) == len(hist["a"]) + 3
    assert np.all(h1["pnu_half"][-1] > 0)
