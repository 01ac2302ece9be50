"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bar: 1e-12 relative, norm-wise per array (max |a-b| / max |b|), with
positions as absolute differences in cell units and velocities relative to
the largest speed; the
Picard iteration count is pinned to the oracle's in each step so that both
sides run the same iterates.  Particles are compared keyed by species and id.
"""
import math
import sys

import numpy as np
import pytest

import ecpic_inputs as E

pytestmark = pytest.mark.gpu

TOL = 1e-12


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
    a, b = np.asarray(a), np.asarray(b)
    den = np.abs(b).max()
    if den == 0:
        return np.abs(a).max()
    return np.abs(a - b).max() / den


def _currents_ok(Ig, Io, w, parts, what=""):
    """Current parity: 1e-12 of the largest current, plus the floor the
    oracle's positions set.  The oracle keeps global logical positions
    (xi up to nr, eta up to nz), so each sub-step's displacement, the
    difference of two stored positions, carries the rounding of a number of
    that size: up to ulp(max(nr, nz)) cells, i.e. (q w / dt) ulp amperes per
    particle.  The GPU forms displacements from cell offsets in [0, 1].  The
    floor is that per-particle bound times the square root of the particles
    that deposit on one edge (at most those of four cells), times 2."""
    n_cell = 0
    for d in parts:
        if len(d["r"]):
            n_cell = max(n_cell, _max_per_cell(w, d))
    unit = sum(abs(d["q"] * d["w"]) for d in parts) / w.dt
    floor = 2.0 * unit * np.spacing(float(max(w.nr, w.nz))) * math.sqrt(4 * max(n_cell, 1))
    worst = 0.0
    for a, b in zip(Ig, Io):
        err = np.abs(a - b).max()
        bound = 1e-12 * np.abs(b).max() + floor
        worst = max(worst, err / bound)
    _flush(f"  {what} currents: worst error {worst:.2f} of the bar (floor {floor:.2e} A)")
    return worst <= 1.0


def _max_per_cell(w, d):
    s = w.R / (w.nr + w.xi_a)
    r = np.asarray(d["r"])
    xi = np.where(r < 2 * s * w.xi_a, r * r / (4 * s * s * max(w.xi_a, 1e-300)), r / s - w.xi_a)
    i = np.clip(np.floor(xi).astype(np.int64), 0, w.nr - 1)
    j = np.clip(np.floor(np.asarray(d["z"]) / (w.L / w.nz)).astype(np.int64), 0, w.nz - 1)
    return int(np.bincount(i * w.nz + j, minlength=w.nr * w.nz).max())


def _by_uid(d):
    o = np.argsort(d["uid"], kind="stable")
    return {k: v[o] for k, v in d.items()}


def _cmp_species(gpu, ora, what=""):
    g, o = _by_uid(gpu), _by_uid(ora)
    assert len(g["uid"]) == len(o["uid"]), f"{what}: count {len(g['uid'])} vs {len(o['uid'])}"
    assert np.array_equal(g["uid"], o["uid"]), what
    if len(o["uid"]) == 0:
        return 0.0
    worst = 0.0
    for k in ("xi", "eta"):  # absolute, in cell units
        worst = max(worst, np.abs(g[k] - o[k]).max())
    vmax = max(np.abs(o[k]).max() for k in ("vr", "vt", "vz"))
    vmax = vmax if vmax > 0 else 1.0  # all at rest: the differences must be 0
    for k in ("vr", "vt", "vz"):
        worst = max(worst, np.abs(g[k] - o[k]).max() / vmax)
    return worst


def _make_pair(w, og, P, parts, precision="fp64", extra_cap=0.3, mobile=(True, True),
               model="em", cap=0.0):
    g = og.grid_from_workload(w, model=model, cap=cap)
    sp = []
    for k, d in enumerate(parts):
        n = len(d["r"])
        sp.append(g.species(d, cap=int(n * (1 + extra_cap)) + 256, role=k + 1,
                            mobile=mobile[k]))
    ctx = P.context_from_workload(w, precision=precision, model=model, blocking_cap=cap)
    P.load_workload_species(ctx, parts, extra_cap=extra_cap, mobile=mobile)
    return g, sp, ctx


def test_load_read_roundtrip(og, torch_cuda):
    import paper_2212_08836_amd as P
    w = E.workload("c1")
    parts = E.make_particles(w)
    g, sp, ctx = _make_pair(w, og, P, parts)
    for k in range(2):
        d = ctx.read_particles(k)
        assert _cmp_species(d, sp[k].view(), "load") < 1e-14


# nr > 256 gives the per-mode scan 2, 4, 5 and (at the largest nr, 2048) 8
# rows per thread; 40 x 1024 has the longest rows a grid may have
@pytest.mark.parametrize("shape", [(32, 32, 2.0), (37, 29, 2.0), (70, 130, 0.0), (300, 16, 2.0),
                                   (512, 8, 2.0), (1024, 8, 2.0), (1100, 12, 0.0),
                                   (1024, 512, 2.0), (2048, 8, 2.0), (40, 1024, 2.0)])
def test_field_solve_parity(og, torch_cuda, shape):
    import paper_2212_08836_amd as P
    nr, nz, xa = shape
    _flush(f"field_solve parity {shape}")
    w = E.Workload("f", nr, nz, 0.05, 0.03, xi_a=xa, dt=2e-11, drive_amp=(150.0,),
                   drive_freq=(90e6,), drive_phase=(0.4,))
    g = og.grid_from_workload(w)
    ctx = P.context_from_workload(w)
    rng = np.random.default_rng(nr * 1000 + nz)
    ur0 = rng.standard_normal(nr * (nz + 1)) * 20
    uz0 = rng.standard_normal((nr + 1) * nz) * 20
    ur0.reshape(nr, nz + 1)[:, [0, -1]] = 0
    uz0.reshape(nr + 1, nz)[-1] = 0
    h0 = rng.standard_normal(nr * nz) * 0.1
    Ir = rng.standard_normal(nr * (nz + 1)) * 1e-2
    Iz = rng.standard_normal((nr + 1) * nz) * 1e-2
    t = 3.3e-9
    a = ctx.field_solve(ur0, uz0, h0, Ir, Iz, t)
    b = g.field_solve(ur0, uz0, h0, Ir, Iz, t)
    bar = max(TOL, _cn_condition(g, w) * 2.0 ** -53)
    errs = [_rel(x, y) for x, y in zip(a, b)]
    _flush(f"  errors {errs}, bar {bar:.2e}")
    assert max(errs) < bar


def _cn_condition(g, w):
    """Condition number of the SPD system for h^{n+1/2}: its extreme
    eigenvalues are those of the radial tridiagonal of the lowest and of the
    highest axial mode (the system separates in z).  Two backward-stable
    solves of it may differ by this times the unit roundoff; at 1024 x 512
    with dt = 20 ps it is 1.4e5 (c dt / dz = 100), below 1e4 on the smaller
    shapes."""
    from scipy.linalg import eigvalsh_tridiagonal
    t = g.tables()
    rh, wr, wz, area = t["rh"], t["wr"], t["wz"], t["area"]
    dt, mu = w.dt, E.MU0
    mi = 2 * math.pi * rh
    dzw, drw = 2 * wz / dt, 2 * wr / dt
    diag = mi * 2 * mu * area / dt + mi * mi / dzw
    diag[:-1] += mi[:-1] ** 2 / dzw[1:]
    off = -(2 * math.pi * rh[:-1]) * mi[1:] / dzw[1:]
    grad = mi * mi / drw
    lam = 2 - 2 * math.cos(math.pi * (w.nz - 1) / w.nz)
    lo = eigvalsh_tridiagonal(diag, off, select="i", select_range=(0, 0))[0]
    hi = eigvalsh_tridiagonal(diag + lam * grad, off, select="i",
                              select_range=(w.nr - 1, w.nr - 1))[0]
    return hi / lo


def test_push_deposit_parity_c1(og, torch_cuda):
    # one pass in a strong random half-step field, uncommitted then committed
    import paper_2212_08836_amd as P
    _flush("push_deposit parity c1")
    w = E.workload("c1", dt=4e-11)
    parts = E.make_particles(w)
    for d in parts[:1]:  # hot electrons: many crossings and some wall hits
        d["vr"] *= 4
        d["vz"] *= 4
    g, sp, ctx = _make_pair(w, og, P, parts)
    rng = np.random.default_rng(3)
    nr, nz = w.nr, w.nz
    urh = rng.standard_normal(nr * (nz + 1)) * 2.0
    uzh = rng.standard_normal((nr + 1) * nz) * 2.0
    urh.reshape(nr, nz + 1)[:, [0, -1]] = 0
    uzh.reshape(nr + 1, nz)[-1] = 0
    ctx.set_half_field(urh, uzh)
    Ir_g, Iz_g = ctx.push_deposit(commit=False)
    Ir_o, Iz_o = g.zeros_r(), g.zeros_z()
    stats = []
    for s in sp:
        _, _, rc, st = g.push_deposit(s, urh, uzh, commit=False, Ir=Ir_o, Iz=Iz_o)
        stats.append(st)
        assert rc == 0
    assert sum(s["n_crossings"] for s in stats) > 500
    assert _rel(Ir_g, Ir_o) < TOL and _rel(Iz_g, Iz_o) < TOL
    # committed pass: end states, absorption and wall charge
    Ir_g, Iz_g = ctx.push_deposit(commit=True)
    ost = og.State(g)
    for s in sp:
        g.push_deposit(s, urh, uzh, commit=True, state=ost)
    for k in range(2):
        assert _cmp_species(ctx.read_particles(k), sp[k].view(), f"species {k}") < TOL
    q, bot, top, side = ctx.node_charge()
    assert _rel(bot, ost.wall_bot) < TOL and _rel(top, ost.wall_top) < TOL
    assert _rel(side, ost.wall_side) < TOL


def _edge_particles(w):
    """Hand-placed electrons on the c1 grid: on cell faces and corners
    (moving out, in, along), in the square-root-map cells next to the axis
    and at the axis itself, heading out through every wall, fast enough to
    cross several cells in one step, and at rest.  The ions are empty."""
    s = w.R / (w.nr + w.xi_a)
    r_of = lambda xi: (2.0 * s * np.sqrt(xi * w.xi_a) if xi < w.xi_a else s * (xi + w.xi_a))
    dz = w.L / w.nz
    v = 4e6  # m/s: about 1.5 cells per 1e-11 s step radially in the linear cells
    rows = []
    for i, j in ((5, 7), (12, 3), (20, 28)):
        # slow normal motion off the face: a particle exactly on a face with
        # zero normal velocity, pushed out of both adjacent cells by their
        # fields, has no admissible sub-step (both sides report a failed push)
        for dv in ((v, 0, v), (-v, 0, -v), (1e3, 0, v), (v, 0, -1e3), (-1e3, v, 1e3)):
            rows.append((r_of(i), (j + 0.5) * dz) + dv)           # on an r-face
            rows.append((r_of(i + 0.5), j * dz) + dv)             # on a z-face
            rows.append((r_of(i), j * dz) + dv)                   # on a corner
    for xi in (1e-6, 0.3, 1.0, 1.7, 2.0, 2.4):                   # near the axis
        for dv in ((-v, 0, 0.3 * v), (v, 0.5 * v, 0), (-0.2 * v, 2 * v, -v)):
            rows.append((r_of(xi), 0.37 * w.L) + dv)
    rows.append((r_of(w.nr - 0.1), 0.5 * w.L, 3 * v, 0, 0))      # out through the side wall
    rows.append((r_of(9.5), 0.1 * dz, 0, 0, -3 * v))              # the bottom electrode
    rows.append((r_of(9.5), w.L - 0.1 * dz, 0, 0, 3 * v))         # the top electrode
    rows.append((r_of(w.nr - 0.05), 0.05 * dz, 2 * v, 0, -2 * v))  # a corner
    rows.append((r_of(14.25), 0.5 * w.L, 4 * v, v, 4 * v))        # several cells at once
    rows.append((r_of(14.25), 0.25 * w.L, 0, 0, 0))               # at rest
    a = np.array(rows, dtype=np.float64)
    base = E.make_particles(w)
    e = dict(q=base[0]["q"], m=base[0]["m"], w=base[0]["w"], r=a[:, 0].copy(), z=a[:, 1].copy(),
             vr=a[:, 2].copy(), vt=a[:, 3].copy(), vz=a[:, 4].copy(),
             uid=np.arange(len(a), dtype=np.uint64))
    empty = dict(q=base[1]["q"], m=base[1]["m"], w=base[1]["w"],
                 **{k: np.zeros(0) for k in ("r", "z", "vr", "vt", "vz")},
                 uid=np.zeros(0, dtype=np.uint64))
    return [e, empty]


def test_push_deposit_edge_cases(og, torch_cuda):
    import paper_2212_08836_amd as P
    _flush("push_deposit parity, edge cases")
    w = E.workload("c1")
    parts = _edge_particles(w)
    g, sp, ctx = _make_pair(w, og, P, parts)
    rng = np.random.default_rng(5)
    nr, nz = w.nr, w.nz
    urh = rng.standard_normal(nr * (nz + 1)) * 2.0
    uzh = rng.standard_normal((nr + 1) * nz) * 2.0
    urh.reshape(nr, nz + 1)[:, [0, -1]] = 0
    uzh.reshape(nr + 1, nz)[-1] = 0
    ctx.set_half_field(urh, uzh)
    Ir_g, Iz_g = ctx.push_deposit(commit=False)
    Ir_o, Iz_o = g.zeros_r(), g.zeros_z()
    cross = 0
    for s in sp:
        _, _, rc, st = g.push_deposit(s, urh, uzh, commit=False, Ir=Ir_o, Iz=Iz_o)
        assert rc == 0
        cross += st["n_crossings"]
    _flush(f"  {len(parts[0]['r'])} electrons, {cross} face crossings")
    assert cross >= 20  # 27 with these particles and fields
    assert _rel(Ir_g, Ir_o) < TOL and _rel(Iz_g, Iz_o) < TOL
    Ir_g, Iz_g = ctx.push_deposit(commit=True)
    ost = og.State(g)
    for s in sp:
        g.push_deposit(s, urh, uzh, commit=True, state=ost)
    assert _cmp_species(ctx.read_particles(0), sp[0].view(), "edge electrons") < TOL
    assert len(ctx.read_particles(1)["xi"]) == 0
    q, bot, top, side = ctx.node_charge()
    assert _rel(bot, ost.wall_bot) < TOL and _rel(top, ost.wall_top) < TOL
    assert _rel(side, ost.wall_side) < TOL
    assert np.abs(side).max() > 0 and np.abs(bot).max() > 0 and np.abs(top).max() > 0


def _push_deposit_case(og, P, w, parts, sort, seed=6, waves=0):
    """One push (then one committing push) of `parts` in random half-step
    fields against the oracle; returns the oracle's face-crossing count.
    waves: build of the plain slow pass (0 by size, 2 or 3 forced)."""
    g, sp, ctx = _make_pair(w, og, P, parts)
    ctx.set_option(P.ECPIC_OPT_QUEUE_WAVES, waves)
    if sort:
        ctx.sort()
    rng = np.random.default_rng(seed)
    nr, nz = w.nr, w.nz
    urh = rng.standard_normal(nr * (nz + 1)) * 2.0
    uzh = rng.standard_normal((nr + 1) * nz) * 2.0
    urh.reshape(nr, nz + 1)[:, [0, -1]] = 0
    uzh.reshape(nr + 1, nz)[-1] = 0
    ctx.set_half_field(urh, uzh)
    Ir_g, Iz_g = ctx.push_deposit(commit=False)
    Ir_o, Iz_o = g.zeros_r(), g.zeros_z()
    cross = 0
    for s in sp:
        _, _, rc, st = g.push_deposit(s, urh, uzh, commit=False, Ir=Ir_o, Iz=Iz_o)
        assert rc == 0
        cross += st["n_crossings"]
    _flush(f"  {cross} face crossings")
    assert _rel(Ir_g, Ir_o) < TOL and _rel(Iz_g, Iz_o) < TOL
    Ir_g, Iz_g = ctx.push_deposit(commit=True)
    ost = og.State(g)
    for s in sp:
        g.push_deposit(s, urh, uzh, commit=True, state=ost)
    for k in range(2):
        assert _cmp_species(ctx.read_particles(k), sp[k].view(), f"species {k}") < TOL
    q, bot, top, side = ctx.node_charge()
    assert _rel(bot, ost.wall_bot) < TOL and _rel(top, ost.wall_top) < TOL
    assert _rel(side, ost.wall_side) < TOL
    return cross


@pytest.mark.parametrize("sort,waves", [(False, 0), (True, 0), (False, 3), (True, 3)])
def test_push_deposit_many_crossers(og, torch_cuda, sort, waves):
    # electrons at 30x thermal speed (about 2.7 keV): about half of them leave
    # their cell, hundreds per fast-pass block, so the slow queue's records
    # are both staged and fetched again, and in cell order (sort) the slow
    # pass's tile takes most deposits while in load order most go to global
    # atomics
    import paper_2212_08836_amd as P
    _flush(f"push_deposit parity, fast electrons, sorted {sort}, slow-pass build {waves}")
    w = E.workload("c1")
    parts = E.make_particles(w, n=4096)
    for k in ("vr", "vt", "vz"):
        parts[0][k] = parts[0][k] * 30.0
    assert _push_deposit_case(og, P, w, parts, sort, waves=waves) > 2000  # 2266


@pytest.mark.parametrize("waves", [0, 3])
def test_push_deposit_long_rows(og, torch_cuda, waves):
    # 320 cells along z: the slow pass's tile spans part of a row only, so
    # crossings of r-faces leave it for global atomics
    import paper_2212_08836_amd as P
    _flush(f"push_deposit parity, 12 x 320 grid, slow-pass build {waves}")
    w = E.Workload("long", 12, 320, 0.01, 0.03, ppc=2, Te_eV=300.0)
    parts = E.make_particles(w)
    assert _push_deposit_case(og, P, w, parts, sort=True, waves=waves) > 3000


def test_step_parity_edge_cases(og, torch_cuda):
    # whole steps with the same particles (one species empty throughout)
    import paper_2212_08836_amd as P
    _flush("step parity, edge cases")
    w = E.workload("c1")
    _step_parity(og, P, w, _edge_particles(w), 3)


def _step_parity(og, P, w, parts, nsteps, mcc=None, sort_every=0, mobile=(True, True),
                 running_scale=False, model="em", cap=0.0, waves=0):
    """Steps on both sides with the oracle's iteration counts.  Fields are
    compared against their largest value in this step, or with running_scale
    in any step so far (for runs whose drive is switched off: the fields then
    fall to the plasma's response and keep the absolute rounding of the
    driven steps)."""
    g, sp, ctx = _make_pair(w, og, P, parts, mobile=mobile, model=model, cap=cap)
    if waves:
        ctx.set_option(P.ECPIC_OPT_QUEUE_WAVES, waves)
    st = og.State(g)
    if mcc:
        ctx.set_mcc(mcc)
    worst = 0.0
    scale = [0.0, 0.0, 0.0]
    for n in range(nsteps):
        d_o = g.step(st, sp, mcc=mcc, tol=w.tol)
        assert d_o["rc"] == 0
        d_g = ctx.step(fixed_iter=d_o["iters"], sort_every=sort_every)
        assert d_g["iters"] == d_o["iters"]
        # same iterates: residual history agrees
        for a, b in zip(d_g["residual"], d_o["residual"]):
            assert abs(a - b) <= 1e-9 * b + 1e-13
        ur, uz, h = ctx.get_fields()
        errs = []
        for q, (a, b) in enumerate(((ur, st.ur), (uz, st.uz), (h, st.h))):
            scale[q] = max(scale[q], np.abs(b).max()) if running_scale else np.abs(b).max()
            errs.append(np.abs(a - b).max() / scale[q] if scale[q] > 0 else np.abs(a).max())
        for k in range(len(sp)):
            errs.append(_cmp_species(ctx.read_particles(k), sp[k].view(), f"step {n} sp {k}"))
        worst = max(worst, max(errs))
        _flush(f"  step {n}: iters {d_o['iters']} worst rel {max(errs):.2e} "
               f"coll {d_o['n_coll'][:2]} ion {d_o['n_ionized']}")
        assert max(errs) < TOL, (n, errs)
        assert d_g["n_ionized"] == d_o["n_ionized"]
        assert d_g["n_coll"][:2] == d_o["n_coll"][:2]
        assert d_g["n_absorbed"][:2] == d_o["n_absorbed"][:2]
        # energy accounting (sums in a different order: 1e-10 relative)
        for key in ("we", "wb", "w_absorbed", "w_coll", "w_particles", "w_field_io"):
            assert d_g[key] == pytest.approx(d_o[key], rel=1e-10, abs=1e-30), key
        for k in range(2):
            assert d_g["ke"][k] == pytest.approx(d_o["ke"][k], rel=1e-12), "ke"
        assert d_g["w_drive"] == pytest.approx(d_o["w_drive"], rel=1e-9, abs=1e-30)
        if cap > 0.0:
            assert d_g["electrode_v"] == pytest.approx(st.phi, rel=1e-10, abs=1e-12)
            assert d_g["cap_charge"] == pytest.approx(st.q_cap, rel=1e-10, abs=1e-30)
            assert d_g["w_gen"] == pytest.approx(d_o["w_gen"], rel=1e-9, abs=1e-30)
        if w.port_i > 0:
            # the mouth voltage and the line's wall field at t^{n+1}
            assert d_g["port_v"] == pytest.approx(d_o["port_v"], rel=1e-10, abs=1e-12)
            hb = ctx.get_port_field()
            hs = np.abs(st.hb).max()
            assert np.abs(hb - st.hb).max() <= TOL * hs + 1e-300, "port H_b"
    return worst


def test_step_parity_c1(og, torch_cuda):
    import paper_2212_08836_amd as P
    _flush("step parity c1 (10 steps)")
    w = E.workload("c1")
    _step_parity(og, P, w, E.make_particles(w), w.steps)


@pytest.mark.parametrize("waves", [0, 3])
def test_step_parity_driven_collisional(og, torch_cuda, waves):
    # the c2 physics (drive, J0 sin profile, MCC) on a reduced grid; high
    # pressure so that every process occurs, with a sort every 3 steps; both
    # builds of the plain slow pass (two wavefronts per SIMD, and the three
    # the large workloads take)
    import paper_2212_08836_amd as P
    _flush(f"step parity driven + MCC, slow-pass build {waves}")
    w = E.Workload("c2s", 48, 24, 0.03, 0.012, n0=1e16, profile="j0sin", ppc=12,
                   drive_amp=(200.0,), drive_freq=(100e6,), pressure_pa=60.0, seed=12,
                   dt=1e-11, tol=1e-10)
    parts = E.make_particles(w)
    parts[0]["vr"] *= 3.0  # hotter electrons: ionisation within a few steps
    parts[0]["vt"] *= 3.0
    parts[0]["vz"] *= 3.0
    mcc = w.mcc_params()
    _step_parity(og, P, w, parts, 8, mcc=mcc, sort_every=3, waves=waves)


@pytest.mark.parametrize("waves", [0, 3])
def test_step_parity_immobile_ions_collisional(og, torch_cuda, waves):
    # one mobile species: the passes run one slot, the commit is never fused
    # (an immobile species' buffer would not flip), so every step ends with
    # the separate commit pass and its collision list
    import paper_2212_08836_amd as P
    _flush("step parity, immobile ions, MCC")
    w = E.Workload("c2s", 48, 24, 0.03, 0.012, n0=1e16, profile="j0sin", ppc=12,
                   drive_amp=(200.0,), drive_freq=(100e6,), pressure_pa=60.0, seed=13,
                   dt=1e-11, tol=1e-10)
    parts = E.make_particles(w)
    for k in ("vr", "vt", "vz"):
        parts[0][k] = parts[0][k] * 3.0
    _step_parity(og, P, w, parts, 4, mcc=w.mcc_params(), sort_every=2, mobile=(True, False),
                 waves=waves)


def test_collide_parity(og, torch_cuda):
    import paper_2212_08836_amd as P
    _flush("collide parity")
    w = E.Workload("mc", 16, 16, 0.02, 0.02, n0=1e16, ppc=64, Te_eV=30.0, Ti_eV=0.5,
                   pressure_pa=300.0, seed=4)
    parts = E.make_particles(w)
    g, sp, ctx = _make_pair(w, og, P, parts, extra_cap=1.0)
    mcc = w.mcc_params()
    for step in (5, 6):
        d_o = g.collide(sp, mcc, step)
        ctx.collide(mcc, step)
        assert d_o["n_ionized"] > 0 and d_o["n_coll"][1] > 0
        for k in range(2):
            assert _cmp_species(ctx.read_particles(k), sp[k].view(), f"collide sp {k}") < TOL


def test_sort_keeps_particles_and_orders_cells(og, torch_cuda):
    import paper_2212_08836_amd as P
    w = E.workload("c1")
    parts = E.make_particles(w)
    g, sp, ctx = _make_pair(w, og, P, parts)
    before = [ctx.read_particles(k) for k in range(2)]
    ctx.sort()
    for k in range(2):
        d = ctx.read_particles(k)
        cell = np.minimum(np.floor(d["xi"]).astype(int), w.nr - 1) * w.nz + \
            np.minimum(np.floor(d["eta"]).astype(int), w.nz - 1)
        assert np.all(np.diff(cell) >= 0)
        assert _cmp_species(d, before[k], "sort") == 0.0


def _order_ok(d, nr, nz):
    """Slots in cell order: the cell of each slot lies between the cells its
    position allows (a particle on a face reads as either neighbour)."""
    xi, eta = d["xi"], d["eta"]
    ilo = np.clip(np.ceil(xi).astype(np.int64) - 1, 0, nr - 1)
    ihi = np.clip(np.floor(xi).astype(np.int64), 0, nr - 1)
    jlo = np.clip(np.ceil(eta).astype(np.int64) - 1, 0, nz - 1)
    jhi = np.clip(np.floor(eta).astype(np.int64), 0, nz - 1)
    lo, hi = ilo * nz + jlo, ihi * nz + jhi
    return len(lo) < 2 or bool(np.all(np.maximum.accumulate(lo)[:-1] <= hi[1:]))


@pytest.mark.parametrize("name,precision", [("c2", "fp64"), ("c2", "mixed"), ("rows", "fp64"),
                                            ("rows", "mixed")])
def test_sort_after_drift(og, torch_cuda, name, precision):
    """The sort on the order a run leaves: sorted, then twelve steps without
    a sort, so that most particles are still near their block's cells and
    some have left for other rows (c2), and on the longest rows a grid may
    have (4 x 1024, hot electrons), where a block's cells and window span
    rows and drift across rows leaves the window.  Every particle is kept
    unchanged and the slots come out in cell order."""
    import paper_2212_08836_amd as P
    _flush(f"sort after drift, {name}, {precision}")
    if name == "c2":
        w = E.workload("c2")
    else:
        w = E.Workload("rows", 4, 1024, 0.004, 0.128, ppc=4, Te_eV=50.0, tol=1e-9)
    ctx = P.context_from_workload(w, precision=precision)
    P.load_workload_species(ctx, E.make_particles(w), extra_cap=0.3)
    ctx.sort()
    for k in range(2):
        assert _order_ok(ctx.read_particles(k), w.nr, w.nz)
    for _ in range(12):
        ctx.step(tol=w.tol, sort_every=0)
    before = [ctx.read_particles(k) for k in range(2)]
    assert not all(_order_ok(d, w.nr, w.nz) for d in before)
    ctx.sort()
    for k in range(2):
        d = ctx.read_particles(k)
        assert _order_ok(d, w.nr, w.nz), k
        assert _cmp_species(d, before[k], f"sort sp {k}") == 0.0


def test_sort_stride_sorts_a_species_at_every_kth_sort(og, torch_cuda):
    """ecpic_species_desc.sort_stride: with a sort every 2 steps and the ions
    at every 3rd of those sorts, the electrons come out in cell order after
    every sort, the ions only after steps 6, 12, ... (counted from step 0);
    both keep every particle."""
    import paper_2212_08836_amd as P
    _flush("sort stride")
    w = E.workload("c1")
    ctx = P.context_from_workload(w)
    P.load_workload_species(ctx, E.make_particles(w), extra_cap=0.3, sort_strides=(0, 3))
    n0 = [len(ctx.read_particles(k)["uid"]) for k in range(2)]
    assert not _order_ok(ctx.read_particles(1), w.nr, w.nz)  # load order
    for step in range(1, 7):
        ctx.step(tol=w.tol, sort_every=2)
        d = [ctx.read_particles(k) for k in range(2)]
        if step % 2 == 0:
            assert _order_ok(d[0], w.nr, w.nz), step
        assert _order_ok(d[1], w.nr, w.nz) == (step == 6), step
    assert len(d[1]["uid"]) <= n0[1]
    with pytest.raises(P.EcpicError) as e:
        ctx.add_species(E.QE, E.M_AR, 1.0, 100, True, -1)
    assert e.value.status == P.ECPIC_EINVAL


def _host_node_charge(ds, qs, ws, nr, nz):
    """Bilinear node charge of read-back particles (the plain definition)."""
    Q = np.zeros((nr + 1, nz + 1))
    for d, q, w in zip(ds, qs, ws):
        i = np.clip(np.floor(d["xi"]).astype(int), 0, nr - 1)
        j = np.clip(np.floor(d["eta"]).astype(int), 0, nz - 1)
        a, b = d["xi"] - i, d["eta"] - j
        np.add.at(Q, (i, j), q * w * (1 - a) * (1 - b))
        np.add.at(Q, (i + 1, j), q * w * a * (1 - b))
        np.add.at(Q, (i, j + 1), q * w * (1 - a) * b)
        np.add.at(Q, (i + 1, j + 1), q * w * a * b)
    return Q


@pytest.mark.parametrize("name,precision", [("c1", "fp64"), ("c1", "mixed"), ("rows", "fp64")])
def test_node_charge_matches_bilinear_weights(og, torch_cuda, name, precision):
    """The device's node charge (block-local sums in LDS over a block's cell
    window, global adds for slots outside it) against the bilinear
    definition on the host, on particles in load order (most slots outside
    their block's window), after a sort, and after steps without one."""
    import paper_2212_08836_amd as P
    _flush(f"node charge, {name}, {precision}")
    if name == "c1":
        w = E.workload("c1")
    else:
        w = E.Workload("rows", 4, 1024, 0.004, 0.128, ppc=4, Te_eV=50.0, tol=1e-9)
    parts = E.make_particles(w)
    ctx = P.context_from_workload(w, precision=precision)
    P.load_workload_species(ctx, parts, extra_cap=0.3)
    qs = [d["q"] for d in parts]
    ws = [d["w"] for d in parts]
    scale = abs(qs[0] * ws[0]) * w.ppc
    for stage in ("loaded", "sorted", "stepped"):
        if stage == "sorted":
            ctx.sort()
        elif stage == "stepped":
            for _ in range(6):
                ctx.step(tol=w.tol, sort_every=0)
        q, _, _, _ = ctx.node_charge()
        want = _host_node_charge([ctx.read_particles(k) for k in range(2)], qs, ws, w.nr, w.nz)
        err = np.abs(np.asarray(q).reshape(w.nr + 1, w.nz + 1) - want).max()
        assert err <= 1e-12 * scale, (stage, err, scale)


def test_c2_full_size_sampled(og, torch_cuda):
    # c2 at full size (256 x 128, 4.2M particles) in the configuration the
    # bench times: one committed pass in a strong half-step field; sampled
    # particles re-pushed one by one by the oracle, and exact charge
    # continity of the whole deposit checked on the GPU's own outputs.
    import paper_2212_08836_amd as P
    _flush("c2 full size sampled")
    w = E.workload("c2")
    parts = E.make_particles(w)
    ctx = P.context_from_workload(w)
    P.load_workload_species(ctx, parts)
    ctx.sort()
    g = og.grid_from_workload(w)
    nr, nz = w.nr, w.nz
    rng = np.random.default_rng(9)
    urh = rng.standard_normal(nr * (nz + 1)) * 3.0
    uzh = rng.standard_normal((nr + 1) * nz) * 3.0
    urh.reshape(nr, nz + 1)[:, [0, -1]] = 0
    urh.reshape(nr, nz + 1)[nr - 1, 0] = 100.0
    uzh.reshape(nr + 1, nz)[-1] = 0
    ctx.set_half_field(urh, uzh)
    before = [ctx.read_particles(k) for k in range(2)]
    q0, _, _, _ = ctx.node_charge()
    Ir, Iz = ctx.push_deposit(commit=True)
    q1, bot, top, side = ctx.node_charge()
    after = [ctx.read_particles(k) for k in range(2)]
    # continuity: Delta Q + dt div I = 0 at every node (walls with their charge)
    dq = (q1 - q0).reshape(nr + 1, nz + 1)
    dq[:, 0] += bot
    dq[:, -1] += top
    dq[-1, :] += side
    div = g.div(Ir, Iz).reshape(nr + 1, nz + 1)
    qscale = abs(parts[0]["q"] * parts[0]["w"]) * w.ppc
    assert np.abs(dq + w.dt * div).max() < 1e-11 * qscale
    # sampled particles: the oracle pushes each alone in the same field
    for k in range(2):
        b, a = _by_uid(before[k]), _by_uid(after[k])
        idx = rng.choice(len(b["uid"]), 3000, replace=False)
        s = og.Species(parts[k]["q"], parts[k]["m"], parts[k]["w"], b["xi"][idx], b["eta"][idx],
                       b["vr"][idx], b["vt"][idx], b["vz"][idx], b["uid"][idx])
        g.push_deposit(s, urh, uzh, commit=True, state=og.State(g))
        ov = s.view()
        keep = np.isin(a["uid"], ov["uid"])
        gv = {kk: v[keep] for kk, v in a.items()}
        assert _cmp_species(gv, ov, f"c2 sample sp {k}") < TOL


def test_c5_grid_sampled(og, torch_cuda):
    # the c5 grid (1024 x 512) at 64 particles per cell and species (67M
    # particles: the three-wavefront slow-pass build is chosen by size), drawn
    # on the GPU as the bench draws c5: one committed pass, exact continuity
    # of the whole deposit on the GPU's outputs, and 2000 sampled particles
    # per species re-pushed by the oracle
    import paper_2212_08836_amd as P
    _flush("c5 grid, 67M particles, sampled")
    w = E.workload("c5", ppc=64)
    parts = E.make_particles_device(w, device="cuda")
    ctx = P.context_from_workload(w)
    P.load_workload_species(ctx, parts)
    del parts
    ctx.sort()
    g = og.grid_from_workload(w, push_only=True)
    nr, nz = w.nr, w.nz
    urh, uzh = _c2_half_field(w, seed=15)
    ctx.set_half_field(urh, uzh)
    before = [ctx.read_particles(k) for k in range(2)]
    q0, _, _, _ = ctx.node_charge()
    Ir, Iz = ctx.push_deposit(commit=True)
    q1, bot, top, side = ctx.node_charge()
    after = [ctx.read_particles(k) for k in range(2)]
    dq = (q1 - q0).reshape(nr + 1, nz + 1)
    dq[:, 0] += bot
    dq[:, -1] += top
    dq[-1, :] += side
    div = g.div(Ir, Iz).reshape(nr + 1, nz + 1)
    # the charge of one cell's particles of one species
    qw = E.QE * (E._total_particles_phys(w) / w.n_per_species) * w.ppc
    err = np.abs(dq + w.dt * div).max()
    _flush(f"  continuity {err:.3e} against {qw:.3e} (charge of one cell's particles)")
    assert err < 1e-11 * qw
    rng = np.random.default_rng(21)
    for k in range(2):
        b = before[k]
        idx = rng.choice(len(b["uid"]), 2000, replace=False)
        q, m = (-E.QE, E.ME) if k == 0 else (E.QE, E.M_AR)
        s = og.Species(q, m, 1.0, b["xi"][idx], b["eta"][idx], b["vr"][idx], b["vt"][idx],
                       b["vz"][idx], b["uid"][idx])
        g.push_deposit(s, urh, uzh, commit=True, state=og.State(g))
        ov = s.view()
        a = after[k]
        sel = np.isin(a["uid"], ov["uid"])
        gv = _by_uid({kk: v[sel] for kk, v in a.items()})
        worst = _cmp_species(gv, ov, f"c5 sample sp {k}")
        _flush(f"  species {k}: sampled worst {worst:.2e}")
        assert worst < TOL


def _c2_half_field(w, seed=9):
    rng = np.random.default_rng(seed)
    nr, nz = w.nr, w.nz
    urh = rng.standard_normal(nr * (nz + 1)) * 3.0
    uzh = rng.standard_normal((nr + 1) * nz) * 3.0
    urh.reshape(nr, nz + 1)[:, [0, -1]] = 0
    urh.reshape(nr, nz + 1)[nr - 1, 0] = 100.0
    uzh.reshape(nr + 1, nz)[-1] = 0
    return urh, uzh


def test_c2_full_iteration_pass_currents(og, torch_cuda):
    # the bench's dominant pass at full size (4.19M particles, cell-sorted,
    # fast and slow pass): every current element against the oracle's push
    # of every particle
    import paper_2212_08836_amd as P
    _flush("c2 full-size iteration pass, every current")
    w = E.workload("c2")
    parts = E.make_particles(w)
    g, sp, ctx = _make_pair(w, og, P, parts, extra_cap=0.05)
    ctx.sort()
    urh, uzh = _c2_half_field(w)
    ctx.set_half_field(urh, uzh)
    Ir_g, Iz_g = ctx.push_deposit(commit=False)
    Ir_o, Iz_o = g.zeros_r(), g.zeros_z()
    cross = 0
    for s in sp:
        _, _, rc, st = g.push_deposit(s, urh, uzh, commit=False, Ir=Ir_o, Iz=Iz_o)
        assert rc == 0
        cross += st["n_crossings"]
    _flush(f"  {cross} face crossings; Ir {_rel(Ir_g, Ir_o):.2e}, Iz {_rel(Iz_g, Iz_o):.2e}")
    assert cross > 50_000
    assert _currents_ok((Ir_g, Iz_g), (Ir_o, Iz_o), w, parts, "c2 both species")


def test_c2_full_iteration_pass_currents_per_species(og, torch_cuda):
    # each species alone (the other immobile): the ions' currents are four
    # orders of magnitude below the electrons', so their parity shows the
    # position-rounding floor of the bar on its own
    import paper_2212_08836_amd as P
    _flush("c2 full-size iteration pass, per species")
    w = E.workload("c2")
    parts = E.make_particles(w)
    g = og.grid_from_workload(w)
    urh, uzh = _c2_half_field(w)
    for k in range(2):
        mob = (k == 0, k == 1)
        ctx = P.context_from_workload(w)
        P.load_workload_species(ctx, parts, extra_cap=0.05, mobile=mob)
        ctx.sort()
        ctx.set_half_field(urh, uzh)
        Ig = ctx.push_deposit(commit=False)
        s = g.species(parts[k], cap=len(parts[k]["r"]) + 256, role=k + 1)
        Io = (g.zeros_r(), g.zeros_z())
        _, _, rc, st = g.push_deposit(s, urh, uzh, commit=False, Ir=Io[0], Iz=Io[1])
        assert rc == 0
        assert _currents_ok(Ig, Io, w, [parts[k]], f"c2 species {k}")
        ctx.close()


def test_c2_full_step_tolerance_mode(og, torch_cuda):
    # one production step of the bench workload (100 MHz drive, 5 Pa MCC),
    # each side stopping on its own residual; fields, every particle, the
    # tallies, and the library's own charge-conservation check
    import paper_2212_08836_amd as P
    _flush("c2 full-size step, tolerance mode")
    w = E.workload("c2")
    parts = E.make_particles(w)
    g, sp, ctx = _make_pair(w, og, P, parts, extra_cap=0.05)
    mcc = w.mcc_params()
    ctx.set_mcc(mcc)
    st = og.State(g)
    for n in range(2):
        d_o = g.step(st, sp, mcc=mcc, tol=w.tol)
        assert d_o["rc"] == 0
        d_g = ctx.step(tol=w.tol, conservation=True)
        assert d_g["iters"] == d_o["iters"] and d_g["converged"] == 1
        for a, b in zip(d_g["residual"], d_o["residual"]):
            assert abs(a - b) <= 1e-9 * b + 1e-13
        ur, uz, h = ctx.get_fields()
        errs = [_rel(ur, st.ur), _rel(uz, st.uz), _rel(h, st.h)]
        for k in range(2):
            errs.append(_cmp_species(ctx.read_particles(k), sp[k].view(), f"c2 step {n} sp {k}"))
        assert d_g["n_ionized"] == d_o["n_ionized"]
        assert d_g["n_coll"][:2] == d_o["n_coll"][:2]
        assert d_g["n_absorbed"][:2] == d_o["n_absorbed"][:2]
        _flush(f"  step {n}: iters {d_o['iters']} worst {max(errs):.2e} continuity "
               f"{d_g['continuity_max'] / d_g['q_max']:.1e} gauss {d_g['gauss_max'] / d_g['q_max']:.1e}")
        assert max(errs) < TOL, errs
        assert d_g["continuity_max"] <= 1e-12 * d_g["q_max"]
        assert d_g["gauss_max"] <= 1e-12 * d_g["q_max"]


def test_step_tolerance_mode_c1(og, torch_cuda):
    # the production mode: both sides stop on their own residual; the GPU
    # enqueues each iteration ahead of the residual it waits for, so the
    # iteration after convergence must leave no trace (state, counts, timing)
    import paper_2212_08836_amd as P
    _flush("step parity c1, tolerance mode")
    w = E.workload("c1")
    g, sp, ctx = _make_pair(w, og, P, E.make_particles(w))
    st = og.State(g)
    ctx.set_profiling(True, kinds=("push", "push_commit", "field"))
    iters = 0
    for n in range(6):
        d_o = g.step(st, sp, tol=w.tol)
        d_g = ctx.step(tol=w.tol)
        assert d_g["iters"] == d_o["iters"] and d_g["converged"] == 1
        iters += d_g["iters"]
        for a, b in zip(d_g["residual"][:d_o["iters"]], d_o["residual"][:d_o["iters"]]):
            assert abs(a - b) <= 1e-9 * b + 1e-13
        ur, uz, h = ctx.get_fields()
        errs = [_rel(ur, st.ur), _rel(uz, st.uz), _rel(h, st.h)]
        for k in range(len(sp)):
            errs.append(_cmp_species(ctx.read_particles(k), sp[k].view(), f"step {n} sp {k}"))
        _flush(f"  step {n}: iters {d_o['iters']} worst rel {max(errs):.2e}")
        assert max(errs) < TOL, (n, errs)
    prof = ctx.profile()
    # both species go in one launch per pass; an iteration is either a plain
    # one or one that also commits
    assert prof["push"]["launches"] + prof["push_commit"]["launches"] == iters
    assert prof["field"]["launches"] == iters


def test_step_not_converged_leaves_state(og, torch_cuda):
    import paper_2212_08836_amd as P
    w = E.workload("c1")
    g, sp, ctx = _make_pair(w, og, P, E.make_particles(w))
    ctx.step(tol=w.tol)
    ur0, uz0, h0 = ctx.get_fields()
    parts0 = [ctx.read_particles(k) for k in range(2)]
    d = ctx.step(tol=1e-30, max_iter=3, check=False)
    assert d["rc"] == P.ECPIC_ENOTCONV and d["iters"] == 3 and d["converged"] == 0
    ur1, uz1, h1 = ctx.get_fields()
    assert np.array_equal(ur0, ur1) and np.array_equal(uz0, uz1) and np.array_equal(h0, h1)
    for k in range(2):
        assert _cmp_species(ctx.read_particles(k), parts0[k], "after ENOTCONV") == 0.0
    # the context is still usable: the same step in tolerance mode matches
    # the oracle run over the same two steps
    st = og.State(g)
    g.step(st, sp, tol=w.tol)
    d_o = g.step(st, sp, tol=w.tol)
    d_g = ctx.step(tol=w.tol)
    assert d_g["iters"] == d_o["iters"]
    ur, uz, h = ctx.get_fields()
    assert max(_rel(ur, st.ur), _rel(uz, st.uz), _rel(h, st.h)) < TOL


def test_step_tight_tolerance_discards_unaccepted_commits(og, torch_cuda):
    # with a tolerance near the round-off floor the residual trend now and
    # then predicts a last iteration that is not; such an iteration's
    # commit (into the other particle buffers) must leave no trace
    import paper_2212_08836_amd as P
    _flush("step parity c1, tolerance 1e-13")
    w = E.workload("c1")
    g, sp, ctx = _make_pair(w, og, P, E.make_particles(w))
    st = og.State(g)
    ctx.set_profiling(True, kinds=("push", "push_commit"))
    iters = 0
    for n in range(8):
        d_o = g.step(st, sp, tol=1e-13)
        d_g = ctx.step(tol=1e-13)
        assert d_g["iters"] == d_o["iters"] and d_g["converged"] == 1
        iters += d_g["iters"]
        ur, uz, h = ctx.get_fields()
        errs = [_rel(ur, st.ur), _rel(uz, st.uz), _rel(h, st.h)]
        for k in range(len(sp)):
            errs.append(_cmp_species(ctx.read_particles(k), sp[k].view(), f"step {n} sp {k}"))
        assert max(errs) < TOL, (n, errs)
        assert d_g["n_absorbed"][:2] == d_o["n_absorbed"][:2]
        for key in ("w_absorbed", "w_particles", "w_field_io"):
            assert d_g[key] == pytest.approx(d_o[key], rel=1e-10, abs=1e-30), key
    prof = ctx.profile()
    _flush(f"  iterations {iters}, committing iterations {prof['push_commit']['launches']} "
           f"for 8 steps")
    assert prof["push"]["launches"] + prof["push_commit"]["launches"] == iters
    # every launch timed: the counts agree with the timed launches
    for kind in ("push", "push_commit"):
        assert prof[kind]["calls"] == prof[kind]["launches"]
        assert prof[kind]["call_particles"] == prof[kind]["particles"]


def test_sampled_profiling_counts_every_launch(torch_cuda):
    # timing only every 3rd launch of a kind still counts every needed
    # launch (speculative iterations that turn out to be skipped excluded)
    import paper_2212_08836_amd as P
    w = E.workload("c1")
    ctx = P.context_from_workload(w)
    P.load_workload_species(ctx, E.make_particles(w), extra_cap=0.2)
    ctx.set_profiling(True, kinds=("push", "push_commit", "field"), every=3)
    iters = 0
    for k in range(6):
        d = ctx.step(tol=w.tol)
        iters += d["iters"]
    prof = ctx.profile()
    calls = prof["push"]["calls"] + prof["push_commit"]["calls"]
    timed = prof["push"]["launches"] + prof["push_commit"]["launches"]
    _flush(f"  sampled profiling: {iters} iterations, {calls} push passes counted, {timed} timed")
    assert calls == iters and prof["field"]["calls"] == iters
    assert 0 < timed < calls
    assert prof["push"]["ms"] > 0.0
    with pytest.raises(P.EcpicError):
        ctx.set_profiling(True, every=0)


def test_run_matches_oracle_steps(og, torch_cuda):
    # several steps in one library call (the next step's guess enqueued
    # ahead) give the oracle's steps
    import paper_2212_08836_amd as P
    _flush("run of 5 steps in one call vs the oracle, c1")
    w = E.workload("c1")
    g, sp, ctx = _make_pair(w, og, P, E.make_particles(w))
    st = og.State(g)
    for n in range(5):
        d_o = g.step(st, sp, tol=w.tol)
    d = ctx.run(5, tol=w.tol, stats=True)
    assert d["rc"] == 0 and d["done"] == 5
    assert d["iters"] == d_o["iters"] and d["converged"] == 1
    ur, uz, h = ctx.get_fields()
    errs = [_rel(ur, st.ur), _rel(uz, st.uz), _rel(h, st.h)]
    for k in range(len(sp)):
        errs.append(_cmp_species(ctx.read_particles(k), sp[k].view(), f"run sp {k}"))
    _flush(f"  after 5 steps: worst rel {max(errs):.2e}")
    assert max(errs) < TOL
    # a step that cannot converge stops the run and is reported
    d = ctx.run(3, tol=1e-30, max_iter=3, check=False)
    assert d["rc"] == P.ECPIC_ENOTCONV and d["done"] == 0
    ur1, uz1, h1 = ctx.get_fields()
    assert np.array_equal(ur, ur1) and np.array_equal(uz, uz1) and np.array_equal(h, h1)


def test_run_driven_collisional_matches_oracle(og, torch_cuda):
    # several steps in one call on the driven, collisional case: ionisation
    # appends particles in most steps, and the next step's guess is enqueued
    # before the host has read the appended counts
    import paper_2212_08836_amd as P
    _flush("run of 8 steps in one call vs the oracle, driven + MCC")
    w = E.Workload("c2s", 48, 24, 0.03, 0.012, n0=1e16, profile="j0sin", ppc=12,
                   drive_amp=(200.0,), drive_freq=(100e6,), pressure_pa=60.0, seed=12,
                   dt=1e-11, tol=1e-10)
    parts = E.make_particles(w)
    parts[0]["vr"] *= 3.0
    parts[0]["vt"] *= 3.0
    parts[0]["vz"] *= 3.0
    mcc = w.mcc_params()
    g, sp, ctx = _make_pair(w, og, P, parts)
    ctx.set_mcc(mcc)
    st = og.State(g)
    ion = 0
    for n in range(8):
        d_o = g.step(st, sp, mcc=mcc, tol=w.tol)
        assert d_o["rc"] == 0
        ion += d_o["n_ionized"]
    d = ctx.run(8, tol=w.tol, sort_every=5, stats=True)
    assert d["rc"] == 0 and d["done"] == 8 and d["iters"] == d_o["iters"]
    ur, uz, h = ctx.get_fields()
    errs = [_rel(ur, st.ur), _rel(uz, st.uz), _rel(h, st.h)]
    for k in range(len(sp)):
        errs.append(_cmp_species(ctx.read_particles(k), sp[k].view(), f"run sp {k}"))
    _flush(f"  after 8 steps ({ion} ionisations): worst rel {max(errs):.2e}")
    assert ion > 0
    assert max(errs) < TOL


@pytest.mark.parametrize("waves", [2, 3])
def test_orbit_that_turns_at_a_face(og, torch_cuda, waves):
    """The electron of tests/golden/grazing_particle.npz (from the oracle's
    own run): its free sub-step leaves the cell across the eta face, its orbit
    turns there and no face can be reached consistently, so the sub-step is
    taken again at half the length on both sides.  Both builds of the slow
    pass, uncommitted and committed, against the oracle."""
    import os
    import paper_2212_08836_amd as P
    d = np.load(os.path.join(os.path.dirname(__file__), "golden", "grazing_particle.npz"))
    w = E.Workload("p", 32, 32, 0.02, 0.02, dt=5e-11, port_i=24, port_eps=3.8)
    g0 = og.grid_from_workload(w)
    e = dict(q=float(d["q"]), m=float(d["m"]), w=float(d["w"]), r=g0.r_of_xi(d["xi"]),
             z=d["eta"] * (w.L / w.nz), vr=d["vr"].copy(), vt=d["vt"].copy(), vz=d["vz"].copy(),
             uid=d["uid"].copy())
    empty = {k: (v[:0] if isinstance(v, np.ndarray) else v) for k, v in e.items()}
    g, sp, ctx = _make_pair(w, og, P, [e, empty])
    ctx.set_option(P.ECPIC_OPT_QUEUE_WAVES, waves)
    ctx.set_half_field(d["ur_h"], d["uz_h"])
    Ir_g, Iz_g = ctx.push_deposit(commit=False)
    Ir_o, Iz_o, rc, st = g.push_deposit(sp[0], d["ur_h"], d["uz_h"], commit=False)
    assert rc == 0 and st["n_halvings"] >= 1 and st["n_errors"] == 0
    # the electron moves 7e-4 of a cell in eta near eta = 23: its z current
    # is at the floor of the oracle's global positions
    assert _currents_ok((Ir_g, Iz_g), (Ir_o, Iz_o), w, [e], "turning electron")
    ctx.push_deposit(commit=True)
    g.push_deposit(sp[0], d["ur_h"], d["uz_h"], commit=True, state=og.State(g))
    assert _cmp_species(ctx.read_particles(0), sp[0].view(), "turning electron") < TOL
