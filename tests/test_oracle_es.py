"""Pins of the oracle's electrostatic model (Sec. 2.2, Eq. (8)): the mapped
Poisson solve driven by the charge-conserving current, checked against
Gauss's law coded independently, the absence of circulation, the energy
balance with the source's work, the EM model's approach to it as c grows
(Sec. 3.3), and its own surface-mode lines against Eq. (10) (Sec. 3.1)."""
import math

import numpy as np
import pytest

import ecpic_inputs as E
from oracle import surface_modes as sm

from test_oracle_step import _bilinear_charge


def _driven(og, model="es", cf=1.0, **over):
    w = E.Workload("es", 24, 16, 0.03, 0.01, n0=1e16, profile="j0sin", ppc=8,
                   drive_amp=(100.0,), drive_freq=(100e6,), seed=23, dt=1e-11, tol=1e-12)
    for k, v in over.items():
        setattr(w, k, v)
    g = og.grid_from_workload(w, model=model, mu=E.MU0 / cf ** 2)
    sp = og.species_from_workload(g, E.make_particles(w), extra_cap=0.5)
    return w, g, sp


def _gauss_np(g, ur, uz):
    """Sum over the edges leaving each node of (eps A*/l) u, from the mesh
    tables (written here, apart from the oracle's own operator)."""
    nr, nz = g.nr, g.nz
    t = g.tables()
    wr, wz = t["wr"], t["wz"]
    ur = ur.reshape(nr, nz + 1)
    uz = uz.reshape(nr + 1, nz)
    G = np.zeros((nr + 1, nz + 1))
    fr = wr[:, None] * ur
    fz = np.vstack([wz[:, None] * uz[:nr], np.zeros((1, nz))])
    G[:nr, :] += fr
    G[1:, :] -= fr
    G[:, :nz] += fz
    G[:, 1:] -= fz
    return G


def test_es_solve_obeys_gauss_law_and_has_no_circulation(og):
    """Two solves from random currents (from a zero field at t = 0, where the
    drive is zero too, then from the first result): at every free node the
    field's Gauss charge changes by -dt div I; no cell has circulation; the
    plates and the side wall keep their values; h is zero."""
    w, g, _ = _driven(og)
    nr, nz = g.nr, g.nz
    rng = np.random.default_rng(3)
    ur0 = np.zeros(nr * (nz + 1))
    uz0 = np.zeros((nr + 1) * nz)
    ur0, uz0, _ = g.field_solve(ur0, uz0, g.zeros_h(), rng.standard_normal(ur0.size),
                                rng.standard_normal(uz0.size), 0.0)
    Ir = rng.standard_normal(nr * (nz + 1))
    Iz = rng.standard_normal((nr + 1) * nz)
    t = w.dt
    ur1, uz1, h1 = g.field_solve(ur0, uz0, g.zeros_h(), Ir, Iz, t)
    G = _gauss_np(g, ur1, uz1) - _gauss_np(g, ur0, uz0)
    div = np.zeros((nr + 1, nz + 1))
    Ir2, Iz2 = Ir.reshape(nr, nz + 1), Iz.reshape(nr + 1, nz)
    div[:nr, :] += Ir2
    div[1:, :] -= Ir2
    div[:, :nz] += Iz2
    div[:, 1:] -= Iz2
    scale = w.dt * np.abs(div).max()
    assert np.abs(G + w.dt * div)[:nr, 1:nz].max() < 1e-12 * scale
    assert np.abs(g.curl_e(ur1, uz1)).max() < 1e-12 * np.abs(ur1).max()
    u = ur1.reshape(nr, nz + 1)
    assert u[nr - 1, 0] == g.drive(t + w.dt)
    assert np.all(u[: nr - 1, 0] == 0) and np.all(u[:, nz] == 0)
    assert np.all(uz1.reshape(nr + 1, nz)[nr] == 0)
    assert np.all(h1 == 0)


def test_es_steps_keep_gauss_law_and_balance_energy(og):
    """Driven, collisional steps: Gauss's law against the particles' charge
    at every free node, and kinetic + field + absorbed + collisional - source
    work conserved to the Picard tolerance."""
    w, g, sp = _driven(og, pressure_pa=10.0, tol=1e-11)
    st = og.State(g)
    nr, nz = g.nr, g.nz
    mcc = w.mcc_params()
    W_prev = sum(0.5 * s.m * s.w * np.sum(s.vr[: s.n] ** 2 + s.vt[: s.n] ** 2 + s.vz[: s.n] ** 2)
                 for s in sp)
    qscale = abs(sp[0].q * sp[0].w) * w.ppc
    drive = 0.0
    coll = 0
    for n in range(12):
        d = g.step(st, sp, mcc=mcc, tol=w.tol)
        assert d["rc"] == 0 and d["n_errors"] == 0
        assert d["wb"] == 0.0
        W = sum(d["ke"][:2]) + d["we"]
        bal = W - W_prev + d["w_absorbed"] + d["w_coll"] - d["w_drive"]
        assert abs(bal) <= 10 * w.tol * W_prev + 1e-9 * abs(d["w_drive"]), (n, bal)
        W_prev = W
        drive += abs(d["w_drive"])
        coll += sum(d["n_coll"][:2])
        Q = _bilinear_charge(nr, nz, sp)
        G = _gauss_np(g, st.ur, st.uz)
        assert np.abs(G - Q)[:nr, 1:nz].max() < 1e-12 * qscale
        assert np.abs(g.curl_e(st.ur, st.uz)).max() < 1e-12 * np.abs(st.ur).max()
    assert drive > 0 and coll > 0


def test_em_fields_approach_es_as_c_grows(og):
    """Sec. 3.3: the EM model with mu / c*^2 tends to the ES one; the
    difference falls as (c / c*)^2."""
    _, ges, sp_es = _driven(og)
    st_es = og.State(ges)
    errs = {}
    runs = {cf: _driven(og, model="em", cf=cf) for cf in (100.0, 1000.0)}
    states = {cf: og.State(r[1]) for cf, r in runs.items()}
    for n in range(4):
        assert ges.step(st_es, sp_es, tol=1e-12)["rc"] == 0
        for cf, (_, g, sp) in runs.items():
            assert g.step(states[cf], sp, tol=1e-12)["rc"] == 0
            e = max(np.abs(states[cf].ur - st_es.ur).max() / np.abs(st_es.ur).max(),
                    np.abs(states[cf].uz - st_es.uz).max() / np.abs(st_es.uz).max())
            errs[cf] = max(errs.get(cf, 0.0), e)
    assert errs[1000.0] < 2e-5
    assert 50 < errs[100.0] / errs[1000.0] < 200


@pytest.fixture(scope="module")
def es_slab(og, inputs):
    w = inputs.workload("slab_small")
    g = og.grid_from_workload(w, model="es", omp=True)
    e, i = inputs.slab_particles(w)
    sp = [g.species(e, cap=len(e["r"]) + 16, role=1),
          g.species(i, mobile=False, cap=len(i["r"]) + 16, role=2)]
    st = og.State(g)
    jb = int(1e-3 / (w.L / w.nz))
    bot = np.zeros((w.steps, w.nr + 1))
    top = np.zeros((w.steps, w.nr + 1))
    for k in range(w.steps):
        assert g.step(st, sp, None, tol=w.tol, max_iter=50)["rc"] == 0
        uz = st.uz.reshape(w.nr + 1, w.nz)
        bot[k] = uz[:, jb]
        top[k] = uz[:, w.nz - 1 - jb]
    first = int(math.ceil(w.drive_t_end / w.dt))
    return w, g.r_of_xi(np.arange(w.nr + 1.0)), bot[first:], top[first:]


@pytest.mark.parametrize("m,fam", [(1, "symmetric"), (1, "antisymmetric"), (2, "symmetric"),
                                   (3, "symmetric"), (3, "antisymmetric")])
def test_es_surface_mode_lines_follow_eq10(es_slab, m, fam):
    w, r, bot, top = es_slab
    sym, anti = sm.mode_series(bot, top, r, w.R, m)
    x = sym if fam == "symmetric" else anti
    got = 2 * math.pi * sm.peak_frequency(x, w.dt, 20e6, 1.5e9)
    want = sm.es_frequency(sm.bessel_zeros(0, m)[m - 1] / w.R, w.n0, w.gap, w.L / 2, fam)
    tol = 0.01 if m == 1 else 0.025
    assert abs(got / want - 1.0) < tol, (m, fam, got / 2 / math.pi, want / 2 / math.pi)
