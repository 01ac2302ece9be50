"""Pins of the oracle's mapping and field part (mesh map and Eq. (2) of
Sec. 2.1) against closed forms and exact discrete identities."""
import math

import numpy as np
import pytest

from ecpic_inputs import C_LIGHT, CHI01, EPS0, MU0


def _grid(og, nr=16, nz=12, R=0.02, L=0.015, xi_a=2.0, dt=1e-11, **kw):
    return og.Grid(nr, nz, R, L, xi_a, dt, EPS0, MU0, **kw)


def test_mapping_closed_form(og):
    # r = 2 s sqrt(xi xi_a) below xi_a, s (xi + xi_a) above; s = R/(nr + xi_a)
    g = _grid(og, nr=20, xi_a=2.0, R=0.1)
    s = 0.1 / 22.0
    xi = np.array([0.0, 0.3, 1.0, 1.999, 2.0, 2.5, 7.0, 20.0])
    r = g.r_of_xi(xi)
    ref = np.where(xi < 2, 2 * s * np.sqrt(xi * 2.0), s * (xi + 2.0))
    np.testing.assert_allclose(r, ref, rtol=1e-15, atol=0)
    assert g.r_of_xi(20.0) == pytest.approx(0.1, rel=1e-15)
    # r J_r is the constant 2 s^2 xi_a in the square-root region (axis regular)
    xs = np.array([0.01, 0.5, 1.3, 1.99])
    np.testing.assert_allclose(g.r_of_xi(xs) * g.jr_of_xi(xs), 2 * s * s * 2.0, rtol=1e-14)
    # C^1 at xi_a, inverse map
    eps = 1e-9
    assert abs(g.r_of_xi(2 - eps) - g.r_of_xi(2 + eps)) < 3 * s * eps
    assert g.jr_of_xi(2 - 1e-12) == pytest.approx(s, rel=1e-11)
    xr = np.linspace(0.0, 20.0, 101)
    np.testing.assert_allclose(g.xi_of_r(g.r_of_xi(xr)), xr, rtol=1e-13, atol=1e-13)
    # uniform mesh when xi_a = 0
    g0 = _grid(og, nr=10, xi_a=0.0, R=0.1)
    np.testing.assert_allclose(g0.r_of_xi(np.arange(11.0)), np.arange(11) * 0.01, rtol=1e-15)


def test_dual_volumes_tile_the_cylinder(og):
    # z-edge dual areas are annuli between consecutive cell-centre radii and the
    # ring volumes of the cells sum to pi R^2 L only up to the midpoint rule,
    # while the dual annuli sum exactly to pi r_{nr-1/2}^2.
    g = _grid(og, nr=24, nz=10, R=0.05, L=0.02, xi_a=2.0)
    T = g.tables()
    wz = T["wz"] * (0.02 / 10) / EPS0  # A*_z
    assert wz.sum() == pytest.approx(math.pi * T["rh"][-1] ** 2, rel=1e-13)
    assert T["rn"][0] == 0.0 and T["rn"][-1] == pytest.approx(0.05, rel=1e-15)


def test_div_curl_is_zero(og):
    g = _grid(og)
    rng = np.random.default_rng(3)
    h = rng.standard_normal(g.nr * g.nz)
    kr, kz = g.curl_h(h)
    d = g.div(kr, kz).reshape(g.nr + 1, g.nz + 1)
    # every node that is not on a PEC wall (z walls or side wall)
    inner = d[: g.nr, 1: g.nz]
    assert np.abs(inner).max() <= 1e-12 * np.abs(kr).max()


def test_ampere_is_minus_weighted_transpose_of_faraday(og):
    # sum_cells 2 pi r_{i+1/2} h (C u) = - sum_interior edges u (K h): the exact
    # discrete Poynting identity behind energy conservation.
    g = _grid(og)
    rng = np.random.default_rng(4)
    ur = rng.standard_normal(g.nr * (g.nz + 1))
    uz = rng.standard_normal((g.nr + 1) * g.nz)
    urv = ur.reshape(g.nr, g.nz + 1)
    urv[:, 0] = 0
    urv[:, -1] = 0
    uz.reshape(g.nr + 1, g.nz)[-1, :] = 0
    h = rng.standard_normal(g.nr * g.nz)
    ce = g.curl_e(ur, uz).reshape(g.nr, g.nz)
    rh = g.tables()["rh"]
    lhs = np.sum(2 * np.pi * rh[:, None] * h.reshape(g.nr, g.nz) * ce)
    kr, kz = g.curl_h(h)
    rhs = -(np.dot(ur, kr) + np.dot(uz, kz))
    assert lhs == pytest.approx(rhs, rel=1e-12)


def test_vacuum_energy_is_conserved(og):
    # Crank-Nicolson with PEC walls and no current conserves W_E + W_B exactly
    g = _grid(og, nr=12, nz=10, dt=3e-11)
    rng = np.random.default_rng(5)
    ur = rng.standard_normal(g.nr * (g.nz + 1))
    uz = rng.standard_normal((g.nr + 1) * g.nz)
    ur.reshape(g.nr, g.nz + 1)[:, [0, -1]] = 0
    uz.reshape(g.nr + 1, g.nz)[-1, :] = 0
    h = rng.standard_normal(g.nr * g.nz) * 1e-3
    Ir, Iz = g.zeros_r(), g.zeros_z()
    W0 = g.energy_e(ur, uz) + g.energy_b(h)
    for n in range(40):
        ur, uz, h = g.field_solve(ur, uz, h, Ir, Iz, n * g.dt)
    W1 = g.energy_e(ur, uz) + g.energy_b(h)
    assert W1 == pytest.approx(W0, rel=1e-12)


def _tm0m0_frequency(og, nr, nz, xi_a, m, nsteps=240, dt=1e-11, R=0.02, L=0.02):
    """Measured angular frequency of the TM_0m0 mode of the empty cavity."""
    from scipy.special import jn_zeros
    chi = jn_zeros(0, m)[m - 1]
    g = og.Grid(nr, nz, R, L, xi_a, dt, EPS0, MU0)
    rn = g.tables()["rn"]
    from scipy.special import j0
    uz = np.zeros((nr + 1) * nz)
    prof = j0(chi * rn / R)
    prof[-1] = 0.0
    uz[:] = np.repeat(prof, nz) * (L / nz)
    ur, h = g.zeros_r(), g.zeros_h()
    Ir, Iz = g.zeros_r(), g.zeros_z()
    w = np.repeat(prof, nz)
    sig = []
    for n in range(nsteps):
        sig.append(np.dot(uz, w))
        ur, uz, h = g.field_solve(ur, uz, h, Ir, Iz, n * dt)
    s = np.array(sig)
    # for one dominant discrete mode: s[n+1] + s[n-1] = 2 cos(w dt) s[n]
    cwd = np.dot(s[1:-1], s[2:] + s[:-2]) / (2 * np.dot(s[1:-1], s[1:-1]))
    w_num = math.acos(cwd) / dt
    w_h = 2.0 / dt * math.tan(w_num * dt / 2)  # undo the CN frequency map
    return w_num, w_h, C_LIGHT * chi / R


@pytest.mark.parametrize("m", [1, 2])
def test_tm_cavity_mode_converges_to_bessel_zero(og, m):
    # TM_0m0 of a PEC cylinder: omega = c chi_0m / R (chi from the Bessel zeros)
    errs = []
    for nr in (16, 32, 64):
        _, w_h, w_exact = _tm0m0_frequency(og, nr, 8, 0.0, m)
        errs.append(abs(w_h / w_exact - 1.0))
    assert errs[-1] < 2e-3
    # second order on the uniform mesh: ratio ~4 per halving
    assert 3.0 < errs[0] / errs[1] < 5.0 and 3.0 < errs[1] / errs[2] < 5.0


def test_tm_cavity_mode_with_axis_map(og):
    w_num, w_h, w_exact = _tm0m0_frequency(og, 32, 8, 2.0, 1)
    assert abs(w_h / w_exact - 1.0) < 5e-3
    # the CN shift itself: omega_num = (2/dt) atan(omega dt / 2), ~ -1.06 % here
    shift = (2 / 1e-11) * math.atan(w_exact * 1e-11 / 2) / w_exact - 1
    assert abs(w_num / w_exact - 1 - shift) < 5e-3
    assert CHI01 == pytest.approx(2.404825557695773)


def test_field_solve_satisfies_the_cn_equations(og):
    # residuals of Faraday and Ampere written directly (not via elimination)
    g = _grid(og, nr=10, nz=8, dt=2e-11, drive_amp=(50.0,), drive_freq=(1e9,), drive_phase=(0.3,))
    rng = np.random.default_rng(8)
    nr, nz = g.nr, g.nz
    ur0 = rng.standard_normal(nr * (nz + 1))
    uz0 = rng.standard_normal((nr + 1) * nz)
    ur0.reshape(nr, nz + 1)[:, [0, -1]] = 0
    ur0.reshape(nr, nz + 1)[nr - 1, 0] = g.drive(0.7e-9)
    uz0.reshape(nr + 1, nz)[-1, :] = 0
    h0 = rng.standard_normal(nr * nz) * 1e-2
    Ir = rng.standard_normal(nr * (nz + 1)) * 1e-3
    Iz = rng.standard_normal((nr + 1) * nz) * 1e-3
    t = 0.7e-9
    ur1, uz1, h1 = g.field_solve(ur0, uz0, h0, Ir, Iz, t)
    T = g.tables()
    urh, uzh, hh = 0.5 * (ur0 + ur1), 0.5 * (uz0 + uz1), 0.5 * (h0 + h1)
    # Faraday: mu A_c (h1-h0)/dt = C u^{1/2}
    far = MU0 * np.repeat(T["area"], nz) * (h1 - h0) / g.dt - g.curl_e(urh, uzh)
    assert np.abs(far).max() < 1e-12 * np.abs(g.curl_e(urh, uzh)).max()
    # Ampere on interior edges: (eps A*/l)(u1-u0)/dt = K h^{1/2} - I
    kr, kz = g.curl_h(hh)
    amp_r = (np.repeat(T["wr"], nz + 1) * (ur1 - ur0) / g.dt - kr + Ir).reshape(nr, nz + 1)[:, 1:-1]
    amp_z = (np.repeat(np.append(T["wz"], 0), nz) * (uz1 - uz0) / g.dt - kz + Iz).reshape(nr + 1, nz)[:-1]
    scale = np.abs(kr).max() + np.abs(Ir).max()
    assert np.abs(amp_r).max() < 1e-11 * scale and np.abs(amp_z).max() < 1e-11 * scale
    # boundary edges take the wall / drive values at t + dt
    assert ur1.reshape(nr, nz + 1)[nr - 1, 0] == pytest.approx(50 * math.sin(2 * math.pi * 1e9 * (t + g.dt) + 0.3))
    assert np.all(uz1.reshape(nr + 1, nz)[-1] == 0)
