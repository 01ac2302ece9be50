"""The mixed-precision path (FP32 push on int32 cell + FP32 offsets, FP64
currents, field solve, residual and energy accounting) against the FP64 path.

Bar: from a common state, one implicit step of each path, the fields at
t^{n+1} agree to 1e-5 relative (norm-wise max|a-b| / max|b| per array), and
both converge to the same Picard tolerance.  The FP64 GPU path itself matches
the CPU oracle to 1e-12 (test_gpu_parity.py), so it stands for the oracle
here.  Trajectories of the two paths diverge over many steps (the system is
chaotic), so the bound is per step from a shared state.
"""
import math
import sys

import numpy as np
import pytest

import ecpic_inputs as E

pytestmark = pytest.mark.gpu

FIELD_TOL = 1e-5


def _flush(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rel(a, b):
    den = np.abs(b).max()
    return np.abs(a - b).max() / den if den > 0 else np.abs(a).max()


def _r_of_xi(w, xi):
    # the radial map of the logical grid: 2 s sqrt(xi xi_a) below xi_a,
    # s (xi + xi_a) above, s = R / (nr + xi_a)
    s = w.R / (w.nr + w.xi_a)
    xi = np.asarray(xi, dtype=np.float64)
    lin = s * (xi + w.xi_a)
    sq = 2.0 * s * np.sqrt(np.maximum(xi, 0.0) * w.xi_a)
    return np.where(xi < w.xi_a, sq, lin)


def _state_of(ctx, w):
    parts = []
    for sid in range(2):
        d = ctx.read_particles(sid)
        parts.append(dict(r=_r_of_xi(w, d["xi"]), z=d["eta"] * (w.L / w.nz), vr=d["vr"],
                          vt=d["vt"], vz=d["vz"], uid=d["uid"]))
    return parts, ctx.get_fields()


def _fresh(P, w, precision, parts, fields, caps, qmw, t, step, mcc):
    ctx = P.context_from_workload(w, precision=precision)
    for sid, d in enumerate(parts):
        q, m, wt = qmw[sid]
        ctx.add_species(q, m, wt, caps[sid], True)
        ctx.load_particles(sid, d["r"], d["z"], d["vr"], d["vt"], d["vz"], d["uid"])
    ur, uz, h = fields
    ctx.set_fields(ur, uz, h, None, None, t=t, step=step)
    if mcc:
        ctx.set_mcc(mcc)
    return ctx


def _one_step_compare(P, w, warm_steps, mcc, bound=FIELD_TOL):
    parts0 = E.make_particles(w)
    qmw = [(d["q"], d["m"], d["w"]) for d in parts0]
    caps = [int(len(d["r"]) * 1.3) + 256 for d in parts0]
    run = P.context_from_workload(w)
    P.load_workload_species(run, parts0, extra_cap=0.3)
    if mcc:
        run.set_mcc(mcc)
    for k in range(warm_steps):
        run.step(tol=w.tol, sort_every=4, stats=False)
    st = run.diagnostics()
    parts, fields = _state_of(run, w)
    run.close()
    d64 = _fresh(P, w, "fp64", parts, fields, caps, qmw, st["t"], st["step"], mcc)
    mix = _fresh(P, w, "mixed", parts, fields, caps, qmw, st["t"], st["step"], mcc)
    s64 = d64.step(tol=w.tol)
    smx = mix.step(tol=w.tol)
    f64, fmx = d64.get_fields(), mix.get_fields()
    errs = [_rel(a, b) for a, b in zip(fmx, f64)]
    incs = [_rel(a - f0, b - f0) for a, b, f0 in zip(fmx, f64, fields)]
    _flush(f"  {w.name}: after {warm_steps} steps, one step: field rel err "
           f"ur {errs[0]:.2e} uz {errs[1]:.2e} h {errs[2]:.2e}; increment rel err "
           f"{incs[0]:.2e} {incs[1]:.2e} {incs[2]:.2e}; iters fp64 {s64['iters']} mixed "
           f"{smx['iters']}, residual {s64['residual'][s64['iters'] - 1]:.2e} / "
           f"{smx['residual'][smx['iters'] - 1]:.2e}")
    assert s64["converged"] == 1 and smx["converged"] == 1
    assert s64["residual"][s64["iters"] - 1] <= w.tol
    assert smx["residual"][smx["iters"] - 1] <= w.tol
    assert max(errs) <= bound, errs
    # particle counts and energies follow the FP64 path closely
    assert abs(smx["n_alive"][0] - s64["n_alive"][0]) <= max(2, 1e-5 * s64["n_alive"][0])
    ke64, kem = s64["ke"][0], smx["ke"][0]
    assert abs(kem - ke64) <= 1e-5 * abs(ke64)
    d64.close()
    mix.close()
    return max(errs)


def test_mixed_one_step_c1(torch_cuda):
    import paper_2212_08836_amd as P
    _flush("mixed vs fp64, c1")
    w = E.workload("c1")
    _one_step_compare(P, w, 6, None)
    _one_step_compare(P, w, 12, None)


def test_mixed_first_step_from_zero_field(torch_cuda):
    # from zero fields and a quasi-neutral start, the field after one step is
    # the small residue of cancelling thermal currents; its relative error is
    # the FP32 rounding of the offsets amplified by that cancellation
    import paper_2212_08836_amd as P
    _flush("mixed vs fp64, c1 first step")
    w = E.workload("c1")
    _one_step_compare(P, w, 0, None, bound=1e-4)


def test_mixed_one_step_c2(torch_cuda):
    # the bench workload at full size, after the discharge has run a while
    import paper_2212_08836_amd as P
    _flush("mixed vs fp64, c2")
    w = E.workload("c2")
    _one_step_compare(P, w, 20, w.mcc_params())


def test_mixed_one_step_c3(torch_cuda):
    # the mixed-precision workload at full size (512x256 cells, 128
    # particles per cell per species, about 33.5M particles)
    import paper_2212_08836_amd as P
    _flush("mixed vs fp64, c3")
    w = E.workload("c3")
    _one_step_compare(P, w, 8, w.mcc_params())


def test_mixed_one_step_long_rows(torch_cuda):
    # 384 cells along z: the slow pass's tile spans part of a row only
    import paper_2212_08836_amd as P
    _flush("mixed vs fp64, 32 x 384")
    w = E.Workload("long", 32, 384, 0.05, 0.03, n0=1e16, profile="j0sin", ppc=8,
                   drive_amp=(200.0,), drive_freq=(100e6,), pressure_pa=5.0, seed=21)
    _one_step_compare(P, w, 10, w.mcc_params())


def test_mixed_deposit_conserves_charge(og, torch_cuda):
    # continuity of the mixed deposit: the currents are those of the FP32
    # displacements before the new offsets are rounded to FP32 for storage,
    # so Delta Q + dt div I = 0 holds to the rounding of the stored offsets
    # (half an FP32 ulp of a cell per particle), not to FP64 round-off
    import paper_2212_08836_amd as P
    w = E.workload("c1")
    parts = E.make_particles(w)
    ctx = P.context_from_workload(w, precision="mixed")
    P.load_workload_species(ctx, parts, extra_cap=0.3)
    g = og.grid_from_workload(w)
    rng = np.random.default_rng(5)
    nr, nz = w.nr, w.nz
    urh = rng.standard_normal(nr * (nz + 1)) * 2.0
    uzh = rng.standard_normal((nr + 1) * nz) * 2.0
    urh.reshape(nr, nz + 1)[:, [0, -1]] = 0
    uzh.reshape(nr + 1, nz)[-1] = 0
    ctx.set_half_field(urh, uzh)
    q0, _, _, _ = ctx.node_charge()
    Ir, Iz = ctx.push_deposit(commit=True)
    q1, bot, top, side = ctx.node_charge()
    dq = (q1 - q0).reshape(nr + 1, nz + 1)
    dq[:, 0] += bot
    dq[:, -1] += top
    dq[-1, :] += side
    div = g.div(Ir, Iz).reshape(nr + 1, nz + 1)
    qscale = abs(parts[0]["q"] * parts[0]["w"]) * w.ppc
    assert np.abs(Ir).max() > 0
    worst = np.abs(dq + w.dt * div).max() / qscale
    _flush(f"  mixed continuity residual {worst:.2e} of the cell charge scale")
    # each node sees at most ~4 ppc particles per species, each off by at
    # most 2^-25 of a cell in either offset
    assert worst < 8 * 2.0 ** -25


def _mixed_vs_oracle(og, P, w, warm_steps, mcc):
    """From a common state (the FP64 GPU path after warm_steps), one step of
    the mixed path and one of the CPU oracle; returns the worst field error."""
    parts0 = E.make_particles(w)
    qmw = [(d["q"], d["m"], d["w"]) for d in parts0]
    caps = [int(len(d["r"]) * 1.3) + 256 for d in parts0]
    run = P.context_from_workload(w)
    P.load_workload_species(run, parts0, extra_cap=0.3)
    if mcc:
        run.set_mcc(mcc)
    for k in range(warm_steps):
        run.step(tol=w.tol, sort_every=4, stats=False)
    st = run.diagnostics()
    parts, fields = _state_of(run, w)
    run.close()
    mix = _fresh(P, w, "mixed", parts, fields, caps, qmw, st["t"], st["step"], mcc)
    g = og.grid_from_workload(w)
    sp = [g.species(dict(parts[k], q=qmw[k][0], m=qmw[k][1], w=qmw[k][2]), cap=caps[k],
                    role=k + 1) for k in range(2)]
    ost = og.State(g)
    ost.ur, ost.uz, ost.h = (f.copy() for f in fields)
    ost.ur_prev, ost.uz_prev = ost.ur.copy(), ost.uz.copy()
    ost.t, ost.step = st["t"], st["step"]
    d_o = g.step(ost, sp, mcc=mcc, tol=w.tol)
    d_m = mix.step(tol=w.tol)
    assert d_o["rc"] == 0 and d_m["converged"] == 1
    assert d_m["residual"][d_m["iters"] - 1] <= w.tol
    errs = [_rel(a, b) for a, b in zip(mix.get_fields(), (ost.ur, ost.uz, ost.h))]
    _flush(f"  {w.name}: mixed vs oracle after {warm_steps} steps: field rel err "
           f"{errs[0]:.2e} {errs[1]:.2e} {errs[2]:.2e}; iters oracle {d_o['iters']} "
           f"mixed {d_m['iters']}")
    mix.close()
    return max(errs)


def test_mixed_one_step_against_the_oracle(og, torch_cuda):
    # the 1e-5 bar against the CPU oracle itself (not only the FP64 GPU path)
    import paper_2212_08836_amd as P
    _flush("mixed vs oracle, c1 and a reduced c2")
    assert _mixed_vs_oracle(og, P, E.workload("c1"), 6, None) <= FIELD_TOL
    w = E.workload("c2", ppc=8)
    assert _mixed_vs_oracle(og, P, w, 10, w.mcc_params()) <= FIELD_TOL
