"""Pins of the oracle's full implicit step (Picard iteration of the coupled
system, Sec. 2.1): exact invariants, energy balance within the nonlinear
tolerance, the cold-plasma oscillation frequency and a brute-force Newton
solution of the same discrete equations."""
import math

import numpy as np
import pytest

import ecpic_inputs as E
from ecpic_inputs import EPS0, ME, MU0, QE

from brute_force import TinyCase


def _bilinear_charge(nr, nz, sp):
    Q = np.zeros((nr + 1, nz + 1))
    for s in sp:
        xi, eta = s.xi[: s.n], s.eta[: s.n]
        i = np.clip(np.floor(xi).astype(int), 0, nr - 1)
        j = np.clip(np.floor(eta).astype(int), 0, nz - 1)
        a, b = xi - i, eta - j
        qw = s.q * s.w
        np.add.at(Q, (i, j), qw * (1 - a) * (1 - b))
        np.add.at(Q, (i + 1, j), qw * a * (1 - b))
        np.add.at(Q, (i, j + 1), qw * (1 - a) * b)
        np.add.at(Q, (i + 1, j + 1), qw * a * b)
    return Q


def _c1_small(og, **over):
    w = E.workload("c1", **over)
    g = og.grid_from_workload(w)
    parts = E.make_particles(w)
    sp = og.species_from_workload(g, parts)
    return w, g, sp


def test_c1_invariants_over_ten_steps(og):
    w, g, sp = _c1_small(og)
    st = og.State(g)
    nr, nz = g.nr, g.nz
    Q0 = _bilinear_charge(nr, nz, sp)
    G0 = g.gauss(st.ur, st.uz).reshape(nr + 1, nz + 1)
    ke0 = sum(0.5 * s.m * s.w * np.sum(s.vr[: s.n] ** 2 + s.vt[: s.n] ** 2 + s.vz[: s.n] ** 2) for s in sp)
    W_prev = ke0
    qscale = abs(sp[0].q * sp[0].w) * w.ppc
    for n in range(w.steps):
        d = g.step(st, sp, tol=w.tol)
        assert d["rc"] == 0 and d["converged"] and d["n_errors"] == 0
        assert d["residual"][-1] <= w.tol
        # Gauss's law is an invariant of the charge-conserving step at every
        # node off the conducting walls, independently of convergence
        Q = _bilinear_charge(nr, nz, sp)
        G = g.gauss(st.ur, st.uz).reshape(nr + 1, nz + 1)
        dev = (G - Q) - (G0 - Q0)
        assert np.abs(dev[:nr, 1:nz]).max() < 1e-12 * qscale
        # energy balance: kinetic + field + absorbed is conserved to ~ tol
        W = sum(d["ke"][:2]) + d["we"] + d["wb"]
        bal = W - W_prev + d["w_absorbed"]
        assert abs(bal) <= 10 * w.tol * W_prev
        # particle work and field-side exchange agree to the Picard tolerance
        assert abs(d["w_particles"] - d["w_field_io"]) <= 10 * w.tol * W_prev
        W_prev = W


def test_fixed_iteration_mode_matches_tolerance_mode(og):
    w, g, sp = _c1_small(og)
    st = og.State(g)
    sp2 = [s.copy() for s in sp]
    st2 = st.copy()
    d = g.step(st, sp, tol=w.tol)
    d2 = g.step(st2, sp2, fixed_iter=d["iters"])
    assert d2["iters"] == d["iters"]
    assert np.array_equal(st.ur, st2.ur) and np.array_equal(st.h, st2.h)
    for a, b in zip(sp, sp2):
        assert np.array_equal(a.xi[: a.n], b.xi[: b.n])


def test_not_converged_leaves_state(og):
    w, g, sp = _c1_small(og)
    st = og.State(g)
    before = [s.view() for s in sp]
    d = g.step(st, sp, tol=1e-30, max_iter=2)
    assert d["rc"] == -4 and not d["converged"]
    assert st.step == 0 and np.all(st.ur == 0)
    for s, b in zip(sp, before):
        assert np.array_equal(s.xi[: s.n], b["xi"])


def test_drive_and_collisions_energy_balance(og):
    # a driven, collisional plasma: kinetic + field + absorbed + collisional
    # loss - drive work is conserved to the Picard tolerance
    w = E.Workload("t", 24, 16, 0.03, 0.01, n0=1e16, profile="j0sin", ppc=8,
                   drive_amp=(100.0,), drive_freq=(100e6,), pressure_pa=10.0, seed=21,
                   dt=1e-11, tol=1e-11)
    g = og.grid_from_workload(w)
    sp = og.species_from_workload(g, E.make_particles(w), extra_cap=0.5)
    st = og.State(g)
    nr, nz = g.nr, g.nz
    mcc = w.mcc_params()
    mcc["eps_max_ev"] = 1000.0
    Q0 = _bilinear_charge(nr, nz, sp)
    G0 = g.gauss(st.ur, st.uz).reshape(nr + 1, nz + 1)
    W_prev = sum(0.5 * s.m * s.w * np.sum(s.vr[: s.n] ** 2 + s.vt[: s.n] ** 2 + s.vz[: s.n] ** 2) for s in sp)
    tot_coll = 0
    drive = 0.0
    for n in range(12):
        d = g.step(st, sp, mcc=mcc, tol=w.tol)
        assert d["rc"] == 0 and d["n_errors"] == 0
        W = sum(d["ke"][:2]) + d["we"] + d["wb"]
        bal = W - W_prev + d["w_absorbed"] + d["w_coll"] - d["w_drive"]
        assert abs(bal) <= 10 * w.tol * W_prev + 1e-9 * abs(d["w_drive"])
        tot_coll += sum(d["n_coll"][:2])
        drive += abs(d["w_drive"])
        W_prev = W
        Q = _bilinear_charge(nr, nz, sp)
        G = g.gauss(st.ur, st.uz).reshape(nr + 1, nz + 1)
        dev = (G - Q) - (G0 - Q0)
        assert np.abs(dev[: nr - 1, 1:nz]).max() < 1e-12 * abs(sp[0].q * sp[0].w) * w.ppc
    assert tot_coll > 0 and drive > 0


def test_cold_plasma_oscillation_frequency(og):
    # immobile ions, cold electrons with v = v0 grad(psi): an exact
    # electrostatic eigenmode of the cavity; it oscillates at omega_pe, shifted
    # by the mid-point rule to (2/dt) atan(omega_pe dt / 2)
    n0, dt = 1e15, 1e-10
    w = E.Workload("cold", 32, 32, 0.02, 0.02, n0=n0, xi_a=2.0, dt=dt)
    g = og.grid_from_workload(w)
    parts = E.cold_mode_particles(w, 128 * 128, v0=2.0)
    e = g.species(parts[0])
    ions = g.species(parts[1], mobile=False)
    sp = [e, ions]
    st = og.State(g)
    wpe = math.sqrt(n0 * QE * QE / (EPS0 * ME))
    from scipy.special import j0, j1
    k, kz = E.CHI01 / w.R, math.pi / w.L

    def proj():
        r = g.r_of_xi(e.xi[: e.n])
        z = e.eta[: e.n] * (w.L / w.nz)
        gr = -k * j1(k * r) * np.sin(kz * z)
        gz = kz * j0(k * r) * np.cos(kz * z)
        return np.sum(e.vr[: e.n] * gr + e.vz[: e.n] * gz)

    sig = [proj()]
    for n in range(70):
        d = g.step(st, sp, tol=1e-10)
        assert d["rc"] == 0
        sig.append(proj())
    s = np.array(sig)
    cwd = np.dot(s[1:-1], s[2:] + s[:-2]) / (2 * np.dot(s[1:-1], s[1:-1]))
    w_num = math.acos(cwd) / dt
    w_expect = 2 / dt * math.atan(wpe * dt / 2)
    assert abs(w_num / w_expect - 1) < 0.02
    # the mode is curl-free: the magnetic energy stays negligible
    assert d["wb"] < 1e-6 * d["we"]


def test_brute_force_newton_agrees_with_picard(og):
    nr, nz, R, L, xa, dt = 4, 4, 0.004, 0.004, 2.0, 2e-11
    tiny = TinyCase(nr, nz, R, L, xa, dt, EPS0, MU0)
    g = og.Grid(nr, nz, R, L, xa, dt, EPS0, MU0)
    rng = np.random.default_rng(31)
    st = og.State(g)
    ur0 = rng.standard_normal((nr, nz + 1)) * 5.0
    ur0[:, [0, -1]] = 0
    uz0 = rng.standard_normal((nr + 1, nz)) * 5.0
    uz0[-1] = 0
    h0 = rng.standard_normal((nr, nz)) * 1e-2
    st.ur[:] = ur0.ravel()
    st.uz[:] = uz0.ravel()
    st.h[:] = h0.ravel()
    st.ur_prev[:] = st.ur
    st.uz_prev[:] = st.uz
    # four slow, heavy-weight electrons well inside their cells (one in the
    # square-root region of the map), strong enough to move the field
    xs = [(0.45, 1.5), (1.6, 2.4), (2.5, 0.6), (3.4, 3.5)]
    vs = rng.standard_normal((4, 3)) * 2e4
    wgt = 3e6
    sp = og.Species(-QE, ME, wgt, [x for x, _ in xs], [e for _, e in xs], vs[:, 0], vs[:, 1],
                    vs[:, 2], np.arange(4, dtype=np.uint64))
    parts = [(-QE, ME, wgt, (x, e, v[0], v[1], v[2])) for (x, e), v in zip(xs, vs)]
    ur1, uz1, h1, P1 = tiny.solve(ur0, uz0, h0, parts)
    d = g.step(st, [sp], fixed_iter=40)
    assert d["rc"] == 0
    # the currents matter: the field moved by more than the vacuum evolution
    assert np.abs(ur1 - ur0).max() > 1e-3
    rel = lambda a, b: np.abs(a - b).max() / np.abs(b).max()
    assert rel(st.ur.reshape(nr, nz + 1), ur1) < 1e-11
    assert rel(st.uz.reshape(nr + 1, nz), uz1) < 1e-11
    assert rel(st.h.reshape(nr, nz), h1) < 1e-11
    for k in range(4):
        assert abs(sp.xi[k] - P1[k, 0]) < 1e-12 and abs(sp.eta[k] - P1[k, 1]) < 1e-12
        vmax = np.abs(P1[k, 2:]).max()
        assert np.abs(np.array([sp.vr[k], sp.vt[k], sp.vz[k]]) - P1[k, 2:]).max() < 1e-11 * vmax


def test_device_input_generator_draws_the_same_distributions():
    # the GPU recipe (run here on the CPU device) against the host one: the
    # same profile, weights and Maxwellians, another random stream
    import torch
    from scipy import stats
    w = E.workload("c2")
    a = E.make_particles_device(w, device="cpu", n=100_000)
    b = E.make_particles(w, n=100_000)
    for k in range(2):
        assert a[k]["w"] == b[k]["w"] and a[k]["q"] == b[k]["q"]
        for key in ("r", "z", "vr", "vt", "vz"):
            x = a[k][key].numpy()
            assert stats.ks_2samp(x, b[k][key]).pvalue > 1e-4, (k, key)
        assert torch.equal(a[0]["r"], a[1]["r"])  # pair loading
    assert float(a[0]["r"].min()) > 0 and float(a[0]["r"].max()) < w.R
