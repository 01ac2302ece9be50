"""Pins of the oracle's blocking-capacitor circuit (Sec. 2.1, Eq. (6)): the
powered electrode is driven through a capacitor C, and its potential follows
from the capacitor charge and the current the electrode sends into the
domain.  Without plasma the electrode and the domain form a capacitive
divider, phi = V C / (C + C_e), exact for the electrostatic model and the
quasi-static limit of the EM one; the generator's work splits into the work
through the gap and the capacitor's energy; with plasma the asymmetric
cavity charges the capacitor to a negative self-bias."""
import math

import numpy as np
import pytest

import ecpic_inputs as E

F = 50e6


def _vacuum(f=F):
    return E.Workload("v", 16, 16, 0.02, 0.02, dt=1e-10, drive_amp=(100.0,), drive_freq=(f,))


def _electrode_capacitance(og, w):
    """C_e: the charge on the powered plate's nodes per volt of plate
    potential, from one electrostatic solve of a plate step with no current
    (its Gauss charge, from the mesh tables)."""
    g = og.grid_from_workload(w, model="es", drive_amp=(1.0,), drive_freq=(w.drive_freq[0],),
                              drive_phase=(0.0,))
    t = g.tables()
    u1 = g.field_solve(g.zeros_r(), g.zeros_z(), g.zeros_h(), g.zeros_r(), g.zeros_z(), 0.0)
    uz = u1[1].reshape(w.nr + 1, w.nz)
    return float(np.sum(t["wz"] * uz[: w.nr, 0])) / (g.drive(w.dt) - g.drive(0.0))


def _divider_error(og, model, f=F, steps=200):
    w = _vacuum(f)
    ce = _electrode_capacitance(og, w)
    cap = 10.0 * ce
    g = og.grid_from_workload(w, model=model, cap=cap)
    st = og.State(g)
    err, bal = 0.0, 0.0
    for _ in range(steps):
        q0 = st.q_cap
        d = g.step(st, [], tol=1e-12)
        assert d["rc"] == 0
        v = g.drive(st.t)
        err = max(err, abs(st.phi - v * cap / (cap + ce)) / 100.0)
        # the capacitor's charge is C (V - phi), and the generator's work is
        # the work through the gap plus the capacitor's energy change
        assert abs(st.q_cap - cap * (v - st.phi)) <= 1e-10 * cap * 100.0
        de = (st.q_cap ** 2 - q0 ** 2) / (2.0 * cap)
        bal = max(bal, abs(d["w_gen"] - d["w_drive"] - de) / max(abs(d["w_gen"]), 1e-300))
    return err, bal


def test_electrostatic_vacuum_divider_is_exact(og):
    err, bal = _divider_error(og, "es")
    assert err < 1e-10
    assert bal < 1e-9


def test_em_vacuum_divider_is_quasi_static(og):
    """The EM cavity's first resonance is near 6 GHz.  At 50 MHz the divider
    holds up to the cavity's ringing: the drive's switch-on (slope 2 pi f A)
    excites the cavity modes, which the lossless scheme keeps, at an
    amplitude of order f / f_res of the drive's.  Halving f halves the
    deviation; the time step does not change it."""
    e50, bal = _divider_error(og, "em", F)
    e25, _ = _divider_error(og, "em", F / 2, steps=400)
    assert e50 < 1e-3 and bal < 1e-9
    assert 1.6 < e50 / e25 < 2.5


@pytest.mark.parametrize("model", ["es", "em"])
def test_self_bias_with_plasma(og, model):
    """Two 50 MHz periods of a 3e15 m^-3 plasma: the domain's energy balance
    holds with the gap's work, the circuit's with the generator's, and the
    electrode settles at a negative mean potential (the grounded wall and
    top plate are the larger electrode)."""
    w = E.Workload("p", 16, 16, 0.02, 0.02, n0=3e15, ppc=8, dt=5e-11, drive_amp=(100.0,),
                   drive_freq=(F,), seed=3, tol=1e-11)
    ce = _electrode_capacitance(og, w)
    cap = 10.0 * ce
    g = og.grid_from_workload(w, model=model, cap=cap)
    sp = og.species_from_workload(g, E.make_particles(w), extra_cap=0.5)
    st = og.State(g)
    W_prev = sum(0.5 * s.m * s.w * np.sum(s.vr[: s.n] ** 2 + s.vt[: s.n] ** 2 + s.vz[: s.n] ** 2)
                 for s in sp)
    phis = []
    per = int(round(1.0 / (F * w.dt)))
    for n in range(2 * per):
        q0 = st.q_cap
        d = g.step(st, sp, tol=w.tol)
        assert d["rc"] == 0
        W = sum(d["ke"][:2]) + d["we"] + d["wb"]
        assert abs(W - W_prev + d["w_absorbed"] - d["w_drive"]) <= 10 * w.tol * W_prev + \
            1e-9 * abs(d["w_drive"])
        W_prev = W
        de = (st.q_cap ** 2 - q0 ** 2) / (2.0 * cap)
        assert abs(d["w_gen"] - d["w_drive"] - de) <= 1e-8 * abs(d["w_gen"]) + 1e-9 * abs(de) + 1e-30
        phis.append(st.phi)
    bias = float(np.mean(phis[per:]))
    assert -60.0 < bias < -20.0, bias
