"""Pins of the oracle's TEM port (Sec. 2.1, Eqs. (5)-(7)): the drive enters
through a coaxial line meeting the bottom wall over r_p <= r <= R, with the
Mur condition for the outgoing wave and the incoming wave set from the
electrode potential; the electrostatic model's port is the Dirichlet wall
with the static coaxial potential (Sec. 2.2).

What pins it, apart from the oracle's own arithmetic:
* the discrete energy balance, exact with the power through the mouth
  (a wrong half-face capacitance or boundary-field update breaks it);
* the mouth voltage of a vacuum cavity driven well below its resonances
  against the lumped circuit of a line (impedance eta ln(R/r_p) / 2 pi)
  closed by the cavity's capacitance: amplitude and phase lag (the factor
  two of the incoming wave, its sign and the line impedance each move them
  by a factor of two or more);
* absorption: after a burst that ends at zero the field energy never rises
  and drains away, where the closed cavity of the delta gap keeps it;
* the electrostatic wall profile against the formula of Sec. 2.2 computed
  here from the node radii;
* the EM model with the port tending to the electrostatic one as c grows,
  to first order in c / c* (the line impedance scales as 1/c*);
* energy balance and Gauss's law with plasma, collisions and the blocking
  capacitor in both models."""
import math

import numpy as np
import pytest

import ecpic_inputs as E

from test_oracle_step import _bilinear_charge

EPS0, MU0 = E.EPS0, E.MU0


def _vacuum(og, ip, eps_r, f, model="em", t_end=0.0, nr=24, nz=8, R=0.12, L=0.005, dt=1e-10):
    return og.Grid(nr, nz, R, L, 2.0, dt, EPS0, MU0, drive_amp=(100.0,), drive_freq=(f,),
                   drive_t_end=t_end, port_i=ip, port_eps=eps_r, model=model)


def test_port_tables_follow_the_coaxial_profile(og):
    g = _vacuum(og, 20, 1.0, 78e6)
    kappa, prof = g.port_tables()
    rn = g.tables()["rn"]
    rp, R = rn[20], g.R
    # Sec. 2.2: phi(r) = phi_0 ln(r / r_max) / ln(r_p / r_max) across the mouth
    want = np.array([1.0 if i <= 20 else math.log(rn[i] / R) / math.log(rp / R)
                     for i in range(g.nr + 1)])
    assert np.allclose(prof, want, rtol=0, atol=1e-15)
    # edge shares are the profile's drops and add up to the whole voltage
    assert np.allclose(kappa[20:], prof[20:-1] - prof[21:], rtol=0, atol=1e-15)
    assert np.all(kappa[:20] == 0) and abs(kappa.sum() - 1.0) < 1e-14


def test_port_energy_balance_is_exact_in_vacuum(og):
    g = _vacuum(og, 20, 3.8, 150e6)
    st = og.State(g)
    W0, worst = 0.0, 0.0
    for n in range(300):
        d = g.step(st, [], tol=1e-13, max_iter=30)
        assert d["rc"] == 0
        W = d["we"] + d["wb"]
        worst = max(worst, abs(W - W0 - d["w_drive"]) / max(W, 1e-300))
        W0 = W
    assert worst < 1e-12, worst


def _mouth_amp_lag(og, ip, eps_r, f):
    dt = 1e-10
    g = _vacuum(og, ip, eps_r, f, dt=dt)
    st = og.State(g)
    n = int(round(6 / (f * dt)))
    v = np.zeros(n)
    for k in range(n):
        d = g.step(st, [], tol=1e-13, max_iter=30)
        assert d["rc"] == 0
        v[k] = d["port_v"]
    t = dt * np.arange(1, n + 1)
    sel = t > 3 / f      # the line's transient (time constant Z0 C ~ 1 ns) is gone
    A = np.stack([np.sin(2 * math.pi * f * t[sel]), np.cos(2 * math.pi * f * t[sel])], 1)
    (s, c), *_ = np.linalg.lstsq(A, v[sel], rcond=None)
    return math.hypot(s, c) / 100.0, math.atan2(-c, s)


def _lumped(og, ip, eps_r, f):
    """Line impedance and the cavity's capacitance seen from the electrode:
    the charge on its face per volt in the static electrostatic solution."""
    ges = _vacuum(og, ip, eps_r, 1e3, model="es")
    t = ges.tables()
    ur1, uz1, _ = ges.field_solve(ges.zeros_r(), ges.zeros_z(), ges.zeros_h(), ges.zeros_r(),
                                  ges.zeros_z(), 0.0)
    v1 = ges.drive(ges.dt)
    uz = uz1.reshape(ges.nr + 1, ges.nz)
    C = sum(t["wz"][i] * uz[i, 0] for i in range(ip + 1)) / v1
    eta = math.sqrt(MU0 / (EPS0 * eps_r))
    Z0 = eta * math.log(ges.R / t["rn"][ip]) / (2 * math.pi)
    return 2 * math.pi * f * C * Z0


@pytest.mark.parametrize("eps_r,f", [(1.0, 78e6), (4.0, 78e6), (1.0, 30e6)])
def test_mouth_voltage_follows_the_line_and_cavity_circuit(og, eps_r, f):
    """A line of impedance Z0 closed by a capacitance C passes the incoming
    wave's doubled voltage as phi / (1 + j w C Z0): amplitude
    1/sqrt(1 + x^2) and lag atan(x), x = w C Z0.  The cavity (12 cm across,
    5 mm high) is far below its first resonance; its mouth and fringe add a
    few percent of capacitance the face charge misses."""
    x = _lumped(og, 20, eps_r, f)
    amp, lag = _mouth_amp_lag(og, 20, eps_r, f)
    assert abs(amp * math.sqrt(1 + x * x) - 1.0) < 0.015, (amp, x)
    assert 1.0 < lag / math.atan(x) < 1.12, (lag, math.atan(x))


def test_port_absorbs_what_the_closed_cavity_keeps(og):
    """A two-period burst that ends at zero: through the port the field
    energy never rises afterwards and drains to ~1e-8 of its peak; with the
    delta gap the closed cavity keeps it (to the Picard tolerance over 300
    steps)."""
    f, dt = 200e6, 1e-10
    out = {}
    for ip in (20, 0):
        g = _vacuum(og, ip, 1.0, f, t_end=2 / f, dt=dt)
        st = og.State(g)
        Wp, Wmax, rise, W_end = 0.0, 0.0, 0.0, None
        for k in range(400):
            d = g.step(st, [], tol=1e-13, max_iter=30)
            assert d["rc"] == 0
            W = d["we"] + d["wb"]
            if st.t > 2 / f + dt / 2:
                rise = max(rise, (W - Wp) / Wmax)
                W_end = W_end or Wp
            Wmax, Wp = max(Wmax, W), W
        out[ip] = (rise, W / W_end)
    rise, left = out[20]
    assert rise <= 1e-14 and left < 1e-6, out
    rise, left = out[0]
    assert abs(left - 1.0) < 1e-10, out


def _plasma(og, model, cap=0.0, cf=1.0, tol=1e-11, pressure=10.0):
    w = E.Workload("port", 24, 16, 0.03, 0.01, n0=1e16, profile="j0sin", ppc=8,
                   drive_amp=(100.0,), drive_freq=(100e6,), seed=23, dt=1e-11, tol=tol,
                   pressure_pa=pressure, port_i=18, port_eps=3.8)
    g = og.grid_from_workload(w, model=model, cap=cap, mu=MU0 / cf ** 2)
    sp = og.species_from_workload(g, E.make_particles(w), extra_cap=0.5)
    return w, g, sp


@pytest.mark.parametrize("model,cap", [("em", 0.0), ("em", 1e-10), ("es", 0.0), ("es", 1e-10)])
def test_port_steps_balance_energy_and_keep_gauss_law(og, model, cap):
    w, g, sp = _plasma(og, model, cap)
    st = og.State(g)
    nr, nz = g.nr, g.nz
    mcc = w.mcc_params()
    W_prev = sum(0.5 * s.m * s.w * np.sum(s.vr[: s.n] ** 2 + s.vt[: s.n] ** 2 + s.vz[: s.n] ** 2)
                 for s in sp)
    qscale = abs(sp[0].q * sp[0].w) * w.ppc
    kappa, _ = g.port_tables()
    coll = 0
    for n in range(10):
        d = g.step(st, sp, mcc=mcc, tol=w.tol)
        assert d["rc"] == 0 and d["n_errors"] == 0
        W = sum(d["ke"][:2]) + d["we"] + d["wb"]
        bal = W - W_prev + d["w_absorbed"] + d["w_coll"] - d["w_drive"]
        assert abs(bal) <= 10 * w.tol * W_prev + 1e-9 * abs(d["w_drive"]), (n, bal)
        W_prev = W
        coll += sum(d["n_coll"][:2])
        Q = _bilinear_charge(nr, nz, sp)
        G = g.gauss(st.ur, st.uz).reshape(nr + 1, nz + 1)
        # every node off the walls (the port's nodes pass charge to the line)
        assert np.abs(G - Q)[:nr, 1:nz].max() < 1e-12 * qscale
        phi = d["phi"] if cap > 0 else g.drive(st.t)
        ub = st.ur.reshape(nr, nz + 1)[18:, 0]
        if model == "es":
            assert np.allclose(ub, phi * kappa[18:], rtol=0, atol=1e-12 * abs(phi))
        assert abs(d["port_v"] - ub.sum()) <= 1e-12 * np.abs(ub).sum()
    assert coll > 0


def test_em_port_tends_to_the_electrostatic_port(og):
    """Sec. 3.3 with the paper's drive: EM with mu / c*^2, the port and the
    blocking capacitor against the electrostatic model with its port; the
    fields and the electrode potential approach it as c / c* (first order,
    the line impedance being proportional to 1 / c*)."""
    def run(model, cf):
        _, g, sp = _plasma(og, model, cap=1e-10, cf=cf, tol=1e-12, pressure=0.0)
        st = og.State(g)
        out = []
        for _ in range(4):
            assert g.step(st, sp, tol=1e-12)["rc"] == 0
            out.append((st.ur.copy(), st.uz.copy(), st.phi))
        return out

    es = run("es", 1.0)
    errs = {}
    for cf in (100.0, 1000.0):
        em = run("em", cf)
        ef = max(max(np.abs(a[0] - b[0]).max() / np.abs(b[0]).max(),
                     np.abs(a[1] - b[1]).max() / np.abs(b[1]).max()) for a, b in zip(em, es))
        ep = max(abs(a[2] - b[2]) / abs(b[2]) for a, b in zip(em, es))
        errs[cf] = (ef, ep)
    assert errs[1000.0][0] < 1e-3 and errs[1000.0][1] < 2e-4, errs
    for q in (0, 1):
        assert 6 < errs[100.0][q] / errs[1000.0][q] < 15, errs


def test_em_electrode_current_is_the_ampere_loop_at_the_rim(og):
    """Eq. (6)'s electrode current, summed over the face's z-edges, equals
    2 pi r h^{n+1/2} on the first port cell (Ampere's law telescoped over
    the face), the form the GPU evaluates."""
    _, g, sp = _plasma(og, "em", cap=1e-10, pressure=0.0)
    st = og.State(g)
    nz = g.nz
    rh = g.tables()["rh"]
    for _ in range(3):
        h0, q0 = st.h.copy(), st.q_cap
        assert g.step(st, sp, tol=1e-12)["rc"] == 0
        ie = (st.q_cap - q0) / g.dt
        hh = 0.5 * (h0[18 * nz] + st.h[18 * nz])
        assert abs(ie - 2 * math.pi * rh[18] * hh) <= 1e-12 * abs(ie), (ie, hh)
