"""The second-order displacement of the input generator (CPU).

Closed forms of second-order Lagrangian perturbation theory (psi2 = -(3/7) grad phi2,
lap phi2 = sum_{i<j} (phi1_ii phi1_jj - phi1_ij^2), psi1 = -grad phi1):
* one plane wave has no second-order displacement (the Zel'dovich solution is exact in 1-D);
* two crossed plane waves phi1 = A cos(kx) + B cos(ky) give phi2 = -(A B k^2 / 2) cos kx cos ky,
  so psi2 = -(3/14) A B k^3 (sin kx cos ky, cos kx sin ky, 0): with A, B > 0 the lines
  x = pi/k and y = pi/k are overdense, and the correction moves matter towards the line
  where both are (infall enhanced at second order).
"""
import numpy as np

from synth.ics import second_order_displacement, zeldovich_ics

N, L = 16, 64.0


def _lattice():
    g = (np.arange(N) + 0.5) * (L / N)
    return np.stack(np.meshgrid(g, g, g, indexing="ij"), -1)


def test_single_plane_wave_has_no_second_order_term():
    q = _lattice()
    k = 2 * np.pi / L * 2
    psi1 = np.zeros_like(q)
    psi1[..., 0] = 0.3 * np.sin(k * q[..., 0])
    psi2 = second_order_displacement(psi1, L)
    assert np.abs(psi2).max() < 1e-15


def test_crossed_plane_waves_closed_form():
    q = _lattice()
    k = 2 * np.pi / L * 3
    a, b = 0.4, -0.25
    psi1 = np.zeros_like(q)
    psi1[..., 0] = a * k * np.sin(k * q[..., 0])          # -d/dx of A cos(kx)
    psi1[..., 1] = b * k * np.sin(k * q[..., 1])
    psi2 = second_order_displacement(psi1, L)
    c = -(3.0 / 14.0) * a * b * k ** 3
    want_x = c * np.sin(k * q[..., 0]) * np.cos(k * q[..., 1])
    want_y = c * np.cos(k * q[..., 0]) * np.sin(k * q[..., 1])
    scale = abs(c)
    assert np.abs(psi2[..., 0] - want_x).max() < 1e-12 * scale
    assert np.abs(psi2[..., 1] - want_y).max() < 1e-12 * scale
    assert np.abs(psi2[..., 2]).max() < 1e-12 * scale
    # direction: both amplitudes positive, just left of x = pi/k on the line y = pi/k
    a2, b2 = 0.4, 0.25
    psi1[..., 1] = b2 * k * np.sin(k * q[..., 1])
    psi1[..., 0] = a2 * k * np.sin(k * q[..., 0])
    psi2 = second_order_displacement(psi1, L)
    x = q[:, 0, 0, 0]
    ix = np.argmin(np.where(x < np.pi / k, np.pi / k - x, np.inf))   # nearest site left of the line
    iy = np.argmin(np.abs(q[0, :, 0, 1] - np.pi / k))
    assert psi2[ix, iy, 0, 0] > 0


def test_second_order_ics_are_a_small_correction_in_both_orders():
    for order in ("morton", "c"):
        p1, v1 = zeldovich_ics(16, L, 0.3, 3, 0.1, order=order)
        p2, v2 = zeldovich_ics(16, L, 0.3, 3, 0.1, order=order, second_order=True)
        d = np.mod(p2 - p1 + L / 2, L) - L / 2
        rms = np.sqrt((d.astype(np.float64) ** 2).sum(1).mean()) / (L / 16)
        assert 1e-4 < rms < 0.05                         # second order in 0.3 cells
        assert np.all((p2 >= 0) & (p2 < L))
        assert np.abs(v2 - v1).max() < 0.2 * np.abs(v1).max()
