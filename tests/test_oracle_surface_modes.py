"""Surface-mode dispersion (Sec. 3.1; Appendix A): pins of the analytic
relations and of the Fourier-Bessel projection, then the oracle's own
EM PIC run of the quiet slab cavity against the Eq. (9) roots, and the
c -> 10 c run (mu / 100, Sec. 3.3) against the Eq. (10) limit."""
import math

import numpy as np
import pytest

from oracle import surface_modes as sm

N0, S, HALF = 1e16, 1.8e-3, 0.015   # Sec. 3.1: 1e16 m^-3, 1.8 mm sheaths, 3 cm gap
R = 0.15
FAM = ("symmetric", "antisymmetric")


def test_skin_depth_matches_the_printed_value():
    # Sec. 3.1 quotes c / w_pe ~ 5.3 cm at these parameters
    assert abs(sm.C0 / sm.omega_pe(N0) - 0.053) < 0.001


def test_electrostatic_limits():
    wpe = sm.omega_pe(N0)
    d = HALF - S
    # k -> 0: symmetric branch cuts off at the plasma series resonance
    assert math.isclose(sm.es_frequency(1e-4, N0, S, HALF, "symmetric"),
                        sm.psr_frequency(N0, S, HALF), rel_tol=1e-6)
    # antisymmetric branch starts linearly: w ~ w_pe k sqrt(s d)
    k = 1e-3
    assert math.isclose(sm.es_frequency(k, N0, S, HALF, "antisymmetric"),
                        wpe * k * math.sqrt(S * d), rel_tol=1e-5)
    # short waves: both families approach the planar surface-plasmon w_pe / sqrt 2
    for fam in FAM:
        assert math.isclose(sm.es_frequency(1e5, N0, S, HALF, fam), wpe / math.sqrt(2),
                            rel_tol=1e-9)


@pytest.mark.parametrize("fam", FAM)
def test_em_relation_tends_to_the_electrostatic_one(fam):
    for chi in sm.bessel_zeros(0, 4):
        k = chi / R
        w_em = sm.em_frequency(k, N0, S, HALF, c=1e4 * sm.C0, family=fam)
        assert math.isclose(w_em, sm.es_frequency(k, N0, S, HALF, fam), rel_tol=1e-6)


def test_em_symmetric_long_wavelength_phase_velocity():
    """Small k and w: alpha tanh(alpha s) -> alpha^2 s, beta -> 1/delta, so the
    symmetric relation gives w/k = c / sqrt(1 + delta tanh(d / delta) / s); for
    delta >> d that is the transmission-line speed c sqrt(s / l)."""
    delta = sm.C0 / sm.omega_pe(N0)
    d = HALF - S
    v = sm.C0 / math.sqrt(1.0 + delta * math.tanh(d / delta) / S)
    for k in (0.01, 0.05):
        w = sm.em_frequency(k, N0, S, HALF, family="symmetric")
        assert math.isclose(w / k, v, rel_tol=2e-4)


def test_em_against_es_at_the_cavity_wave_numbers():
    """The statements of Sec. 3.1 for these parameters: the antisymmetric
    branch hardly changes between EM and ES, the symmetric one drops well
    below the ES cut-off at m = 1."""
    for m, chi in enumerate(sm.bessel_zeros(0, 3), 1):
        k = chi / R
        a_em = sm.em_frequency(k, N0, S, HALF, family="antisymmetric")
        a_es = sm.es_frequency(k, N0, S, HALF, "antisymmetric")
        assert abs(a_em / a_es - 1.0) < 0.02
    k1 = sm.bessel_zeros(0, 1)[0] / R
    s_em = sm.em_frequency(k1, N0, S, HALF, family="symmetric")
    assert s_em < 0.7 * sm.es_frequency(k1, N0, S, HALF, "symmetric")
    assert s_em < sm.psr_frequency(N0, S, HALF)


def test_fourier_bessel_recovers_a_known_series(og):
    """Orthogonality of the Appendix A basis under the r-weighted product:
    a two-term J0 series and a one-term J1 series come back term by term
    (trapezoid error ~1e-3 on 129 mapped radii)."""
    g = og.Grid(128, 4, R, 0.03, 2.0, 1e-11, sm.EPS0, 4e-7 * math.pi)
    r = g.r_of_xi(np.arange(129.0))
    chi0 = sm.bessel_zeros(0, 4)
    chi1 = sm.bessel_zeros(1, 4)
    from scipy.special import j0, j1
    f = 2.0 * j0(chi0[0] * r / R) - 0.5 * j0(chi0[2] * r / R)
    got = [sm.fourier_bessel(f, r, R, m, 0) for m in (1, 2, 3, 4)]
    assert np.allclose(got, [2.0, 0.0, -0.5, 0.0], atol=1e-3)
    f1 = 0.7 * j1(chi1[1] * r / R)
    got = [sm.fourier_bessel(f1, r, R, m, 1) for m in (1, 2, 3)]
    assert np.allclose(got, [0.0, 0.7, 0.0], atol=1e-4)
    # a stack of samples is projected row by row
    one = sm.fourier_bessel(f, r, R, 1, 0)
    two = sm.fourier_bessel(np.stack([f, 3.0 * f]), r, R, 1, 0)
    assert np.allclose(two, [one, 3.0 * one])


def _slab_run(og, inputs, c_factor):
    """The oracle on the quiet slab cavity: E_z edge voltages 1 mm from each
    plate after every step."""
    w = inputs.workload("slab_small")
    g = og.grid_from_workload(w, mu=inputs.MU0 / c_factor ** 2, omp=True)
    e, i = inputs.slab_particles(w)
    sp = [g.species(e, cap=len(e["r"]) + 16, role=1),
          g.species(i, mobile=False, cap=len(i["r"]) + 16, role=2)]
    st = og.State(g)
    jb = int(1e-3 / (w.L / w.nz))
    bot = np.zeros((w.steps, w.nr + 1))
    top = np.zeros((w.steps, w.nr + 1))
    for k in range(w.steps):
        d = g.step(st, sp, None, tol=w.tol, max_iter=50)
        assert d["rc"] == 0, d
        uz = st.uz.reshape(w.nr + 1, w.nz)
        bot[k] = uz[:, jb]
        top[k] = uz[:, w.nz - 1 - jb]
    first = int(math.ceil(w.drive_t_end / w.dt))
    return w, g.r_of_xi(np.arange(w.nr + 1.0)), bot[first:], top[first:]


# (radial mode, family) pairs whose line dominates its projected spectrum
_LINES = [(1, "symmetric"), (1, "antisymmetric"), (2, "symmetric"), (3, "symmetric"),
          (3, "antisymmetric")]


@pytest.fixture(scope="module")
def slab_runs(og, inputs):
    return {cf: _slab_run(og, inputs, cf) for cf in (1.0, 10.0)}


def _measured(run, m, fam):
    w, r, bot, top = run
    sym, anti = sm.mode_series(bot, top, r, w.R, m)
    x = sym if fam == "symmetric" else anti
    return 2 * math.pi * sm.peak_frequency(x, w.dt, 20e6, 1.5e9)


@pytest.mark.parametrize("m,fam", _LINES)
def test_oracle_pic_follows_the_em_dispersion(slab_runs, m, fam):
    run = slab_runs[1.0]
    w = run[0]
    k = sm.bessel_zeros(0, m)[m - 1] / w.R
    want = sm.em_frequency(k, w.n0, w.gap, w.L / 2, family=fam)
    got = _measured(run, m, fam)
    tol = 0.01 if m == 1 else 0.025
    assert abs(got / want - 1.0) < tol, (m, fam, got / 2 / math.pi, want / 2 / math.pi)


@pytest.mark.parametrize("m,fam", _LINES)
def test_oracle_pic_with_faster_light_moves_to_the_es_curve(slab_runs, m, fam):
    """mu / 100 makes c* = 10 c: the lines follow Eq. (9) at c*, which is
    within a percent of Eq. (10)."""
    run = slab_runs[10.0]
    w = run[0]
    k = sm.bessel_zeros(0, m)[m - 1] / w.R
    want = sm.em_frequency(k, w.n0, w.gap, w.L / 2, c=10 * sm.C0, family=fam)
    got = _measured(run, m, fam)
    tol = 0.01 if m == 1 else 0.025
    assert abs(got / want - 1.0) < tol, (m, fam, got / 2 / math.pi, want / 2 / math.pi)
    es = sm.es_frequency(k, w.n0, w.gap, w.L / 2, fam)
    assert abs(got / es - 1.0) < tol + 0.01


def test_symmetric_m1_line_leaves_the_knee_as_c_grows(slab_runs):
    """Sec. 3.1 / 3.3: the EM symmetric m = 1 line sits far below the ES
    cut-off; with c* = 10 c it moves up to it."""
    em = _measured(slab_runs[1.0], 1, "symmetric")
    fast = _measured(slab_runs[10.0], 1, "symmetric")
    w = slab_runs[1.0][0]
    psr = sm.psr_frequency(w.n0, w.gap, w.L / 2)
    assert em < 0.75 * psr
    assert fast > 0.95 * psr
