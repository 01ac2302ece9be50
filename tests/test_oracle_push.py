"""Pins of the oracle's particle push (Eq. (4), mid-point centring, split at
cell crossings) and charge-conserving deposit (Eq. (3), m = 1), Sec. 2.1."""
import math

import numpy as np
import pytest

from ecpic_inputs import EPS0, ME, MU0, QE


def _grid(og, nr=16, nz=12, R=0.02, L=0.015, xi_a=2.0, dt=1e-11, **kw):
    return og.Grid(nr, nz, R, L, xi_a, dt, EPS0, MU0, **kw)


def _bilinear_charge(nr, nz, xi, eta, qw):
    """Node charge with logical bilinear weights, written independently."""
    Q = np.zeros((nr + 1, nz + 1))
    i = np.clip(np.floor(xi).astype(int), 0, nr - 1)
    j = np.clip(np.floor(eta).astype(int), 0, nz - 1)
    a, b = xi - i, eta - j
    np.add.at(Q, (i, j), qw * (1 - a) * (1 - b))
    np.add.at(Q, (i + 1, j), qw * a * (1 - b))
    np.add.at(Q, (i, j + 1), qw * (1 - a) * b)
    np.add.at(Q, (i + 1, j + 1), qw * a * b)
    return Q


def _random_fields(g, rng, amp=30.0):
    ur = rng.standard_normal(g.nr * (g.nz + 1)) * amp
    uz = rng.standard_normal((g.nr + 1) * g.nz) * amp
    ur.reshape(g.nr, g.nz + 1)[:, [0, -1]] = 0
    uz.reshape(g.nr + 1, g.nz)[-1, :] = 0
    return ur, uz


def _electrons(og, g, rng, n, vth):
    xi = rng.random(n) * g.nr
    eta = rng.random(n) * g.nz
    v = rng.standard_normal((3, n)) * vth
    return og.Species(-QE, ME, 1e5, xi, eta, v[0], v[1], v[2], np.arange(n, dtype=np.uint64))


def test_charge_continuity_including_walls(og):
    # Delta Q + dt div I = 0 at every node (wall nodes with their absorbed charge)
    g = _grid(og, dt=1e-10)
    rng = np.random.default_rng(11)
    ur, uz = _random_fields(g, rng)
    sp = _electrons(og, g, rng, 4000, 1e7)  # fast: many crossings and wall hits
    qw = sp.q * sp.w
    Q0 = _bilinear_charge(g.nr, g.nz, sp.xi[: sp.n], sp.eta[: sp.n], qw)
    st = og.State(g)
    Ir, Iz, rc, stats = g.push_deposit(sp, ur, uz, commit=True, state=st)
    assert rc == 0 and stats["n_crossings"] > 500 and sp.n < 4000
    Q1 = _bilinear_charge(g.nr, g.nz, sp.xi[: sp.n], sp.eta[: sp.n], qw)
    Q1[:, 0] += st.wall_bot
    Q1[:, -1] += st.wall_top
    Q1[-1, :] += st.wall_side
    divI = g.div(Ir, Iz).reshape(g.nr + 1, g.nz + 1)
    res = Q1 - Q0 + g.dt * divI
    assert np.abs(res).max() <= 1e-13 * np.abs(Q0).max()
    # and the walls did receive charge
    assert abs(st.wall_bot.sum() + st.wall_top.sum() + st.wall_side.sum()) > 0


def test_work_equals_deposited_power_per_particle(og):
    # 1/2 m (v'^2 - v^2) = dt * sum u . I for every single particle (energy
    # exchange identity of the gather/deposit pair)
    g = _grid(og, dt=1e-10)
    rng = np.random.default_rng(12)
    ur, uz = _random_fields(g, rng, amp=50.0)
    worst = 0.0
    n_cross = 0
    for k in range(300):
        sp = _electrons(og, g, rng, 1, 2e6)
        v0 = np.array([sp.vr[0], sp.vt[0], sp.vz[0]])
        Ir, Iz, rc, st = g.push_deposit(sp, ur, uz, commit=True, state=og.State(g))
        n_cross += st["n_crossings"]
        if sp.n == 0:
            continue  # absorbed: its energy left with it
        v1 = np.array([sp.vr[0], sp.vt[0], sp.vz[0]])
        dke = 0.5 * sp.m * sp.w * (v1 @ v1 - v0 @ v0)
        work = g.dt * (ur @ Ir + uz @ Iz)
        worst = max(worst, abs(dke - work) / (0.5 * sp.m * sp.w * (v0 @ v0)))
    assert n_cross > 20
    assert worst < 1e-12


def test_angular_momentum_exact_in_linear_region(og):
    # no field: r' v_theta' = r v_theta at every sub-step of the linear map
    g = _grid(og, nr=40, nz=10, R=0.04, xi_a=2.0)
    rng = np.random.default_rng(13)
    ur, uz = g.zeros_r(), g.zeros_z()
    for k in range(50):
        xi = 10 + rng.random() * 25
        sp = og.Species(-QE, ME, 1.0, [xi], [5.0], [rng.normal() * 2e6], [rng.normal() * 2e6],
                        [rng.normal() * 1e5], [0])
        L0 = g.r_of_xi(sp.xi[0]) * sp.vt[0]
        E0 = sp.vr[0] ** 2 + sp.vt[0] ** 2 + sp.vz[0] ** 2
        for n in range(5):
            g.push_deposit(sp, ur, uz, commit=True, state=og.State(g))
            if sp.n == 0 or sp.xi[0] < 2.5:
                break
        if sp.n == 0 or sp.xi[0] < 2.5:
            continue
        assert g.r_of_xi(sp.xi[0]) * sp.vt[0] == pytest.approx(L0, rel=1e-13)
        assert sp.vr[0] ** 2 + sp.vt[0] ** 2 + sp.vz[0] ** 2 == pytest.approx(E0, rel=1e-13)


def _gyrate(og, dt, nsteps, B, r0, v):
    g = og.Grid(200, 4, 0.2, 0.004, 2.0, dt, EPS0, MU0, bz_ext=B)
    ur, uz = g.zeros_r(), g.zeros_z()
    sp = og.Species(-QE, ME, 1.0, [g.xi_of_r(r0)], [2.0], [v[0]], [v[1]], [v[2]], [0])
    traj = []
    for n in range(nsteps):
        g.push_deposit(sp, ur, uz, commit=True, state=og.State(g))
        traj.append((g.r_of_xi(sp.xi[0]), sp.vr[0], sp.vt[0], sp.vz[0]))
    return np.array(traj)


def test_uniform_bz_gyration(og):
    # electron in uniform B_z: closed circle in the x-y plane; |v| and the
    # canonical angular momentum m r v_t + q B r^2 / 2 are conserved exactly,
    # the orbit matches the analytic circle to O(dt^2).
    B = 0.01
    wc = QE * B / ME                      # cyclotron frequency
    r0, v = 0.05, (3e5, 4e5, 0.0)
    T = 2 * math.pi / wc
    dt = T / 100
    n = 100
    tr = _gyrate(og, dt, n, B, r0, v)
    speed = np.sqrt(tr[:, 1] ** 2 + tr[:, 2] ** 2 + tr[:, 3] ** 2)
    np.testing.assert_allclose(speed, 5e5, rtol=1e-12)
    ptheta = ME * tr[:, 0] * tr[:, 2] + (-QE) * B * tr[:, 0] ** 2 / 2
    p0 = ME * r0 * v[1] + (-QE) * B * r0 ** 2 / 2
    np.testing.assert_allclose(ptheta, p0, rtol=1e-11)

    def exact_r(t):
        # x-y motion of charge -e in B_z: velocity rotates at +wc
        x0, y0 = r0, 0.0
        vx0, vy0 = v[0], v[1]
        c, s = np.cos(wc * t), np.sin(wc * t)
        x = x0 + (vx0 * s - vy0 * (1 - c)) / wc
        y = y0 + (vy0 * s + vx0 * (1 - c)) / wc
        return np.hypot(x, y)

    errs = []
    for m in (1, 2):
        trm = _gyrate(og, dt / m, n * m, B, r0, v)
        t = dt / m * np.arange(1, n * m + 1)
        errs.append(np.abs(trm[:, 0] - exact_r(t)).max() / r0)
    assert errs[0] < 1e-2
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_exb_rigid_rotation_is_a_discrete_fixed_point(og):
    # E_r = E0 r / R plus B_z: a circular orbit about the axis with
    # w^2 + wc w + (q/m) E0 / R = 0 stays exactly circular
    B, E0, R = 0.02, -2.0e4, 0.1
    q, m = -QE, ME
    wc = q * B / m
    disc = wc * wc - 4 * (q / m) * E0 / R
    w = (-wc + math.sqrt(disc)) / 2
    g = og.Grid(100, 4, R, 0.004, 2.0, 2e-11, EPS0, MU0, bz_ext=B, er_ext=E0)
    ur, uz = g.zeros_r(), g.zeros_z()
    r0 = 0.06
    sp = og.Species(q, m, 1.0, [g.xi_of_r(r0)], [2.0], [0.0], [w * r0], [0.0], [0])
    for n in range(200):
        g.push_deposit(sp, ur, uz, commit=True, state=og.State(g))
    assert g.r_of_xi(sp.xi[0]) == pytest.approx(r0, rel=1e-12)
    assert abs(sp.vr[0]) < 1e-9 * abs(w * r0)
    assert sp.vt[0] == pytest.approx(w * r0, rel=1e-12)


def test_axis_reflection_and_wall_absorption(og):
    g = _grid(og, nr=8, nz=8, R=0.008, L=0.008)
    ur, uz = g.zeros_r(), g.zeros_z()
    # straight at the axis with no angular momentum: mirrored, speed kept
    sp = og.Species(-QE, ME, 1.0, [0.3], [4.0], [-5e6], [0.0], [1e4], [0])
    st = og.State(g)
    for n in range(30):
        g.push_deposit(sp, ur, uz, commit=True, state=st)
    assert sp.n == 1 and sp.vr[0] > 0
    assert sp.vr[0] ** 2 + sp.vz[0] ** 2 == pytest.approx(25e12 + 1e8, rel=1e-13)
    # into the bottom wall: absorbed, with its charge on the two wall nodes
    sp = og.Species(-QE, ME, 2.0, [3.25], [0.02], [0.0], [0.0], [-5e6], [0])
    st = og.State(g)
    g.push_deposit(sp, ur, uz, commit=True, state=st)
    assert sp.n == 0
    assert st.wall_bot[3] == pytest.approx(-2 * QE * 0.75) and st.wall_bot[4] == pytest.approx(-2 * QE * 0.25)


def test_uncommitted_pass_leaves_state(og):
    g = _grid(og)
    rng = np.random.default_rng(14)
    ur, uz = _random_fields(g, rng)
    sp = _electrons(og, g, rng, 500, 1e6)
    before = sp.view()
    g.push_deposit(sp, ur, uz, commit=False)
    after = sp.view()
    for k in before:
        assert np.array_equal(before[k], after[k])


def _exb_orbit(og, dt, nsteps, B, E0, R, r0, vt0, dvr):
    g = og.Grid(100, 4, R, 0.004, 2.0, dt, EPS0, MU0, bz_ext=B, er_ext=E0)
    ur, uz = g.zeros_r(), g.zeros_z()
    sp = og.Species(-QE, ME, 1.0, [g.xi_of_r(r0)], [2.0], [dvr], [vt0], [0.0], [0])
    r = [r0]
    for n in range(nsteps):
        g.push_deposit(sp, ur, uz, commit=True, state=og.State(g))
        assert sp.n == 1
        r.append(g.r_of_xi(sp.xi[0]))
    return np.array(r)


def _sinusoid_frequency(s, dt):
    # s_n = c + A cos(W n dt + p): the differences d_n obey
    # d_{n+1} + d_{n-1} = 2 cos(W dt) d_n; least squares for cos(W dt)
    d = np.diff(s)
    x, y = d[1:-1], d[2:] + d[:-2]
    c = np.dot(x, y) / (2 * np.dot(x, x))
    return math.acos(c) / dt


def test_exb_epicyclic_frequency_is_second_order(og):
    # E_r = E0 r / R plus uniform B_z.  In x + i y = zeta the motion is linear:
    # zeta'' = k zeta - i wc zeta' with k = (q/m) E0 / R, wc = q B / m, so every
    # orbit is a sum of two circular modes exp(i w t), w^2 + wc w + k = 0, and
    # r^2 = |zeta|^2 oscillates at the difference of the roots,
    # W = sqrt(wc^2 - 4k), at any amplitude.  Start on the slow (E x B) rigid
    # rotation and kick v_r: the measured frequency of r^2 converges to W at
    # second order in dt.
    B, E0, R = 0.02, -2.0e4, 0.1
    q, m = -QE, ME
    wc = q * B / m
    k = (q / m) * E0 / R
    W = math.sqrt(wc * wc - 4 * k)
    w_slow = (-wc - math.copysign(W, -wc)) / 2   # the root of smaller modulus
    assert abs(w_slow) < 0.01 * abs(wc)
    r0 = 0.06
    T = 2 * math.pi / W
    errs = []
    for dt in (T / 24, T / 48, T / 96):
        n = int(round(4 * T / dt))
        r = _exb_orbit(og, dt, n, B, E0, R, r0, w_slow * r0, 0.3 * abs(w_slow) * r0)
        assert np.ptp(r) > 1e-3 * r0   # the kick excites the fast mode
        errs.append(abs(_sinusoid_frequency(r * r, dt) / W - 1))
    assert errs[0] < 1e-2
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_orbit_that_turns_at_a_face_takes_a_halved_substep(og):
    """tests/golden/grazing_particle.npz (written by make_grazing_fixture.py
    from the oracle's own run): the electron's free sub-step leaves its cell
    across the eta face, but its orbit turns there, so no face can be
    reached consistently.  The sub-step is taken again at half the length:
    the push succeeds, charge is conserved to round-off and the work done
    equals the deposited power (the identities every sub-step keeps)."""
    import os
    d = np.load(os.path.join(os.path.dirname(__file__), "golden", "grazing_particle.npz"))
    g = og.Grid(32, 32, 0.02, 0.02, 2.0, 5e-11, EPS0, MU0, port_i=24, port_eps=3.8)
    q, m, w = float(d["q"]), float(d["m"]), float(d["w"])
    sp = og.Species(q, m, w, d["xi"], d["eta"], d["vr"], d["vt"], d["vz"], d["uid"], cap=2)
    qw = q * w
    Q0 = _bilinear_charge(32, 32, sp.xi[:1], sp.eta[:1], qw)
    e0 = 0.5 * m * w * (sp.vr[0] ** 2 + sp.vt[0] ** 2 + sp.vz[0] ** 2)
    Ir, Iz, rc, st = g.push_deposit(sp, d["ur_h"], d["uz_h"], commit=True, state=og.State(g))
    assert rc == 0 and st["n_errors"] == 0 and st["n_halvings"] >= 1 and sp.n == 1
    Q1 = _bilinear_charge(32, 32, sp.xi[:1], sp.eta[:1], qw)
    res = Q1 - Q0 + g.dt * g.div(Ir, Iz).reshape(33, 33)
    assert np.abs(res).max() <= 1e-13 * abs(qw)
    e1 = 0.5 * m * w * (sp.vr[0] ** 2 + sp.vt[0] ** 2 + sp.vz[0] ** 2)
    pw = g.dt * (np.dot(d["ur_h"], Ir) + np.dot(d["uz_h"], Iz))
    assert abs((e1 - e0) - pw) <= 1e-10 * e0
