"""The electrostatic model on the HIP path (Sec. 2.2, Eq. (8)): the
DST/tridiagonal Poisson update against the oracle's banded Cholesky, whole
steps against the oracle (driven, collisional, sorted), and the Gauss law
and absence of circulation of the GPU's own fields."""
import sys

import numpy as np
import pytest

import ecpic_inputs as E

from test_gpu_parity import TOL, _rel, _step_parity

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


@pytest.mark.parametrize("shape", [(8, 2, 2.0), (13, 7, 2.0), (70, 33, 2.0), (256, 128, 2.0),
                                   (300, 65, 0.0), (1024, 512, 2.0)])
def test_es_field_solve_parity(og, torch_cuda, shape):
    import paper_2212_08836_amd as P
    nr, nz, xa = shape
    _flush(f"ES field_solve parity {shape}")
    w = E.Workload("f", nr, nz, 0.05, 0.03, xi_a=xa, dt=2e-11, drive_amp=(150.0,),
                   drive_freq=(90e6,), drive_phase=(0.4,))
    g = og.grid_from_workload(w, model="es")
    ctx = P.context_from_workload(w, model="es")
    rng = np.random.default_rng(nr * 1000 + nz)
    ur0 = rng.standard_normal(nr * (nz + 1)) * 20
    uz0 = rng.standard_normal((nr + 1) * nz) * 20
    ur0.reshape(nr, nz + 1)[:, [0, -1]] = 0
    uz0.reshape(nr + 1, nz)[-1] = 0
    h0 = np.zeros(nr * nz)
    Ir = rng.standard_normal(nr * (nz + 1)) * 1e-2
    Iz = rng.standard_normal((nr + 1) * nz) * 1e-2
    t = 3.3e-9
    a = ctx.field_solve(ur0, uz0, h0, Ir, Iz, t)
    b = g.field_solve(ur0, uz0, h0, Ir, Iz, t)
    for x, y in zip(a[:2], b[:2]):
        assert _rel(x, y) < TOL
    assert np.all(a[2] == 0)


def test_es_step_parity_driven_collisional(og, torch_cuda):
    import paper_2212_08836_amd as P
    _flush("ES step parity, driven + MCC, sort every 3 steps")
    w = E.Workload("es", 48, 24, 0.03, 0.012, n0=1e16, profile="j0sin", ppc=12,
                   drive_amp=(200.0,), drive_freq=(100e6,), pressure_pa=60.0, seed=14,
                   dt=1e-11, tol=1e-10)
    parts = E.make_particles(w)
    for k in ("vr", "vt", "vz"):
        parts[0][k] = parts[0][k] * 3.0
    worst = _step_parity(og, P, w, parts, 8, mcc=w.mcc_params(), sort_every=3, model="es")
    _flush(f"  worst {worst:.2e}")


def test_es_step_parity_c1_tolerance_mode(og, torch_cuda):
    import paper_2212_08836_amd as P
    _flush("ES step parity c1, immobile ions")
    w = E.workload("c1")
    _step_parity(og, P, w, E.make_particles(w), 6, model="es", mobile=(True, False))


def test_es_gpu_fields_obey_gauss_and_have_no_circulation(og, torch_cuda):
    """After GPU steps of a driven plasma: the field's Gauss charge equals the
    particles' node charge at every free node, and no cell has circulation
    (both evaluated by the oracle's operators on the GPU's output)."""
    import paper_2212_08836_amd as P
    w = E.Workload("es", 64, 32, 0.03, 0.012, n0=1e16, profile="j0sin", ppc=16,
                   drive_amp=(200.0,), drive_freq=(100e6,), seed=15, dt=1e-11, tol=1e-10)
    g = og.grid_from_workload(w, model="es")
    ctx = P.context_from_workload(w, model="es")
    P.load_workload_species(ctx, E.make_particles(w), extra_cap=0.2)
    for _ in range(10):
        ctx.step(tol=w.tol)
    ur, uz, h = ctx.get_fields()
    q, _, _, _ = ctx.node_charge()
    G = g.gauss(ur, uz).reshape(w.nr + 1, w.nz + 1)
    Q = np.asarray(q).reshape(w.nr + 1, w.nz + 1)
    qscale = np.abs(Q).max()
    dev = np.abs(G - Q)[: w.nr, 1: w.nz].max()
    _flush(f"  Gauss deviation {dev:.3e} of max node charge {qscale:.3e}")
    assert dev < 1e-10 * qscale
    assert np.abs(g.curl_e(ur, uz)).max() < 1e-12 * np.abs(ur).max()
    assert np.all(h == 0)
