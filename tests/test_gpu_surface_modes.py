"""Surface-mode dispersion on the HIP path (Sec. 3.1; Sec. 3.3 for the
faster-light runs).

1. Parity: the first steps of the quiet slab cavity (cold electrons,
   immobile ions, 20-harmonic sawtooth burst on the drive gap), GPU against
   the oracle at the 1e-12 bar of the other step-parity tests.
2. Physics: the cavity rung for 300 ns on the GPU.  E_z 1 mm from each plate
   is projected on J0(chi_0m r / R) (Appendix A), split into the even and odd
   combinations, and Fourier transformed; the lines must sit on the roots of
   Eq. (9) (and, with c* = 10 c and 100 c, move onto Eq. (10)).
"""
import math
import sys

import numpy as np
import pytest

import ecpic_inputs as E
from oracle import surface_modes as sm

pytestmark = pytest.mark.gpu


def _flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def test_slab_step_parity(og, torch_cuda):
    """Whole steps on the slab cavity with 1 eV electrons and the burst cut
    after 5 of 12 steps (the drive's end time is exercised).  The cold
    cavity itself is checked pass by pass below: there its first currents
    are so small that the oracle's own position rounding decides them."""
    import paper_2212_08836_amd as P
    from test_gpu_parity import _step_parity
    _flush("step parity, slab cavity 64 x 100, 1 eV electrons, burst of 5 steps, immobile ions")
    w = E.workload("slab", Te_eV=1.0)
    w.drive_t_end = 5 * w.dt
    parts = E.slab_particles(w)
    worst = _step_parity(og, P, w, parts, 12, mobile=(True, False), running_scale=True)
    _flush(f"  worst {worst:.2e}")


def test_cold_slab_first_pass_currents(og, torch_cuda):
    """The cold cavity's first push in the drive's vacuum field: currents at
    1e-12 of the largest plus the floor of the oracle's global-coordinate
    displacements (a few 1e-13 A here, against 2e-5 A of current)."""
    import paper_2212_08836_amd as P
    from test_gpu_parity import _currents_ok
    w = E.workload("slab")
    parts = E.slab_particles(w)
    g = og.grid_from_workload(w)
    sp = g.species(parts[0], cap=len(parts[0]["r"]) + 16, role=1)
    u1 = g.field_solve(g.zeros_r(), g.zeros_z(), g.zeros_h(), g.zeros_r(), g.zeros_z(), 0.0)
    urh, uzh = u1[0] / 2, u1[1] / 2
    Iro, Izo, rc, _ = g.push_deposit(sp, urh, uzh)
    assert rc == 0
    ctx = P.context_from_workload(w)
    P.load_workload_species(ctx, parts, mobile=(True, False))
    ctx.set_half_field(urh, uzh)
    Irg, Izg = ctx.push_deposit()
    assert _currents_ok((Irg, Izg), (Iro, Izo), w, [parts[0]], "cold slab first pass")


def _gpu_ring(torch, P, w, c_factor, model="em"):
    """Run the cavity on the GPU; the E_z edge voltages 1 mm from each plate
    after every step, gathered on the device from the bound field tensors."""
    dev = torch.device("cuda")
    f64 = torch.float64
    ctx = P.context_from_workload(w, mu=E.MU0 / c_factor ** 2, model=model)
    P.load_workload_species(ctx, E.slab_particles(w), mobile=(True, False))
    nr, nz = w.nr, w.nz
    ur = torch.zeros(nr * (nz + 1), dtype=f64, device=dev)
    uz = torch.zeros((nr + 1) * nz, dtype=f64, device=dev)
    h = torch.zeros(nr * nz, dtype=f64, device=dev)
    ctx.bind_fields(ur, uz, h, torch.zeros_like(ur), torch.zeros_like(uz), torch.zeros_like(h))
    jb = int(1e-3 / (w.L / nz))
    first = int(math.ceil(w.drive_t_end / w.dt))
    rec = torch.zeros((w.steps, 2, nr + 1), dtype=f64, device=dev)
    uz2 = uz.view(nr + 1, nz)
    iters = retried = 0
    for k in range(w.steps):
        try:
            d = ctx.step(tol=w.tol, max_iter=50)
        except P.EcpicError as e:
            # a Picard cycle held up by a flipping particle event (the step
            # is left uncommitted): the same step with a fixed count
            if e.status != P.ECPIC_ENOTCONV:
                raise
            retried += 1
            d = ctx.step(fixed_iter=12)
        iters += d["iters"]
        rec[k, 0] = uz2[:, jb]
        rec[k, 1] = uz2[:, nz - 1 - jb]
        if k % 5000 == 4999:
            _flush(f"  c* = {c_factor:g} c: step {k + 1}, mean iterations {iters / (k + 1):.2f}")
    torch.cuda.synchronize()
    assert retried <= w.steps // 1000, retried
    out = rec.cpu().numpy()
    ctx.bind_fields(None, None, None, None, None, None)
    return out[first:, 0], out[first:, 1]


def _radii(og, w):
    g = og.grid_from_workload(w, push_only=True)
    return g.r_of_xi(np.arange(w.nr + 1.0))


@pytest.fixture(scope="module")
def rings(og, torch_cuda):
    import paper_2212_08836_amd as P
    w = E.workload("slab")
    r = _radii(og, w)
    out = {}
    for cf in (1.0, 10.0, 100.0):
        _flush(f"surface-mode cavity 64 x 100, {w.steps} steps, c* = {cf:g} c")
        out[cf] = _gpu_ring(torch_cuda, P, w, cf)
    _flush(f"surface-mode cavity 64 x 100, {w.steps} steps, electrostatic model")
    out["es"] = _gpu_ring(torch_cuda, P, w, 1.0, model="es")
    return w, r, out


def _line(w, r, bot, top, m, fam):
    sym, anti = sm.mode_series(bot, top, r, w.R, m)
    x = sym if fam == "symmetric" else anti
    return 2 * math.pi * sm.peak_frequency(x, w.dt, 20e6, 1.5e9)


_LINES = [(1, "symmetric"), (1, "antisymmetric"), (2, "symmetric"), (2, "antisymmetric"),
          (3, "symmetric"), (3, "antisymmetric")]


def _tol(m, fam):
    """1 % for m = 1, 2.5 % for the other lines that dominate their projected
    spectra (the lines the oracle's test checks).  The m = 2 antisymmetric
    line does not dominate its spectrum: from run to run (the order of the
    FP64 current atomics differs) its peak pick has landed from 140 to 150
    MHz against 152.8, so it is printed and not checked (None)."""
    if m == 1:
        return 0.01
    return None if (m, fam) == (2, "antisymmetric") else 0.025


@pytest.mark.parametrize("cf", [1.0, 10.0, 100.0])
def test_lines_follow_the_dispersion_relation(rings, cf):
    w, r, out = rings
    bot, top = out[cf]
    worst = 0.0
    bad = []
    for m, fam in _LINES:
        k = sm.bessel_zeros(0, m)[m - 1] / w.R
        want = sm.em_frequency(k, w.n0, w.gap, w.L / 2, c=cf * sm.C0, family=fam)
        es = sm.es_frequency(k, w.n0, w.gap, w.L / 2, fam)
        got = _line(w, r, bot, top, m, fam)
        _flush(f"  c*={cf:g}c m={m} {fam:13s}: PIC {got / 2e6 / math.pi:8.2f} MHz, "
               f"Eq.(9) {want / 2e6 / math.pi:8.2f}, Eq.(10) {es / 2e6 / math.pi:8.2f}")
        if _tol(m, fam) is None:
            continue
        if not abs(got / want - 1.0) < _tol(m, fam):
            bad.append((m, fam))
        worst = max(worst, abs(got / want - 1.0))
    _flush(f"  worst relative line offset {worst:.4f}")
    assert not bad, bad


def test_electrostatic_model_lines_follow_eq10(rings):
    """The same cavity with the electrostatic model (Sec. 2.2): its lines
    sit on Eq. (10)."""
    w, r, out = rings
    bot, top = out["es"]
    bad = []
    for m, fam in _LINES:
        k = sm.bessel_zeros(0, m)[m - 1] / w.R
        want = sm.es_frequency(k, w.n0, w.gap, w.L / 2, fam)
        got = _line(w, r, bot, top, m, fam)
        _flush(f"  ES m={m} {fam:13s}: PIC {got / 2e6 / math.pi:8.2f} MHz, "
               f"Eq.(10) {want / 2e6 / math.pi:8.2f}")
        if _tol(m, fam) is not None and not abs(got / want - 1.0) < _tol(m, fam):
            bad.append((m, fam))
    assert not bad, bad


def test_symmetric_m1_line_moves_to_the_electrostatic_cutoff(rings):
    w, r, out = rings
    lines = [_line(w, r, *out[cf], 1, "symmetric") for cf in (1.0, 10.0, 100.0)]
    es = sm.es_frequency(sm.bessel_zeros(0, 1)[0] / w.R, w.n0, w.gap, w.L / 2, "symmetric")
    assert lines[0] < 0.75 * es
    assert lines[0] < lines[1] <= lines[2] * 1.002
    assert abs(lines[2] / es - 1.0) < 0.01
