"""The C-ABI contract beyond parity: device memory that torch owns (a bound
workspace, fields bound in place), steps that must not commit (ECAPACITY,
ERANGE, ENOTCONV leave the state as it was), the overflow rules of the
stand-alone collision call, and the library's own charge-conservation check
(continuity and Gauss's law, Sec. 2.1).  Every failure here is forced from
the host through the arguments; no kernel is made to fault.
"""
import sys

import numpy as np
import pytest

import ecpic_inputs as E

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


def _snapshot(ctx, qscale):
    """Everything a committed step changes: particles, fields, wall charge,
    counts and clock.  qscale: the charge of one macro-particle (the node
    charge of a pair-loaded plasma is a sum of cancelling terms of that
    size)."""
    d = ctx.diagnostics()
    return dict(parts=[ctx.read_particles(k) for k in range(2)], fields=ctx.get_fields(),
                charge=ctx.node_charge(), t=d["t"], step=d["step"], n_alive=d["n_alive"][:2],
                qscale=qscale)


def _qscale(parts):
    return abs(parts[0]["q"] * parts[0]["w"])


def _by_uid(d):
    o = np.argsort(d["uid"], kind="stable")
    return {k: v[o] for k, v in d.items()}


def _same(a, b):
    """The state of one context before and after a call that must not
    change it: bitwise, except the node charge, which ecpic_node_charge sums
    anew with atomics (in an order that varies from call to call)."""
    assert a["t"] == b["t"] and a["step"] == b["step"] and a["n_alive"] == b["n_alive"]
    for x, y in zip(a["fields"] + a["charge"][1:], b["fields"] + b["charge"][1:]):
        assert np.array_equal(x, y)
    qa, qb = a["charge"][0], b["charge"][0]
    assert np.abs(qa - qb).max() <= 1e-13 * max(np.abs(qb).max(), a["qscale"])
    for pa, pb in zip(a["parts"], b["parts"]):
        for k in pa:
            assert np.array_equal(pa[k], pb[k]), k


def _rel(a, b):
    den = np.abs(b).max()
    return np.abs(a - b).max() / den if den > 0 else np.abs(a).max()


def _close(a, b, tol=1e-12):
    """Two contexts that ran the same steps: the current sums use atomics
    (their order varies between runs), so the states agree to round-off, not
    bitwise; positions absolute in cells, velocities relative to the largest."""
    assert a["t"] == b["t"] and a["step"] == b["step"] and a["n_alive"] == b["n_alive"]
    for x, y in zip(a["fields"] + a["charge"][1:], b["fields"] + b["charge"][1:]):
        assert _rel(x, y) <= tol
    qa, qb = a["charge"][0], b["charge"][0]
    assert np.abs(qa - qb).max() <= tol * max(np.abs(qb).max(), a["qscale"])
    for pa, pb in zip(a["parts"], b["parts"]):
        # particles born by ionisation are appended in the order their
        # slots were reserved, which varies: compare by identifier
        pa, pb = _by_uid(pa), _by_uid(pb)
        assert np.array_equal(pa["uid"], pb["uid"])
        for k in ("xi", "eta"):
            assert np.abs(pa[k] - pb[k]).max(initial=0.0) <= tol
        vmax = max(np.abs(pb[k]).max(initial=1.0) for k in ("vr", "vt", "vz"))
        for k in ("vr", "vt", "vz"):
            assert np.abs(pa[k] - pb[k]).max(initial=0.0) <= tol * vmax


def _same_iterates(da, db):
    assert da["iters"] == db["iters"]
    for x, y in zip(da["residual"], db["residual"]):
        assert abs(x - y) <= 1e-9 * y + 1e-13


def _context(P, w, parts, caps=None, workspace=False, precision="fp64"):
    ctx = P.context_from_workload(w, precision=precision)
    sids = []
    for k, d in enumerate(parts):
        cap = caps[k] if caps else len(d["r"]) + 256
        sids.append(ctx.add_species(d["q"], d["m"], d["w"], cap))
    if workspace:
        ctx.bind_workspace()
    for sid, d in zip(sids, parts):
        ctx.load_particles(sid, d["r"], d["z"], d["vr"], d["vt"], d["vz"], d["uid"])
    return ctx


def _driven(**over):
    # a small driven, collisional case: 24 x 24 cells, 200 V at 100 MHz
    return E.Workload("d", 24, 24, 0.02, 0.02, ppc=4, Te_eV=8.0, drive_amp=(200.0,),
                      drive_freq=(100e6,), pressure_pa=300.0, **over)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_bound_workspace_gives_the_same_steps(torch_cuda, precision):
    # the whole device region in one torch tensor: bitwise the same steps as
    # the library's own memory
    import paper_2212_08836_amd as P
    _flush(f"bound workspace, {precision}")
    w = _driven()
    parts = E.make_particles(w)
    a = _context(P, w, parts, precision=precision)
    b = _context(P, w, parts, workspace=True, precision=precision)
    nbytes = b.workspace_size()
    assert b.workspace is not None and b.workspace.numel() >= nbytes > 0
    for ctx in (a, b):
        ctx.set_mcc(w.mcc_params())
    for n in range(3):
        da = a.step(tol=w.tol, sort_every=2)
        db = b.step(tol=w.tol, sort_every=2)
        _same_iterates(da, db)
    _close(_snapshot(a, _qscale(parts)), _snapshot(b, _qscale(parts)))
    # binding comes before any device use, and once only
    with pytest.raises(P.EcpicError):
        b.bind_workspace()
    # a species cannot join a bound region
    with pytest.raises(P.EcpicError):
        b.add_species(parts[0]["q"], parts[0]["m"], parts[0]["w"], 10)
    a.close()
    b.close()


def test_workspace_too_small_is_refused(torch_cuda):
    import paper_2212_08836_amd as P
    w = _driven()
    ctx = P.context_from_workload(w)
    ctx.add_species(-E.QE, E.ME, 1.0, 1000)
    n = ctx.workspace_size()
    with pytest.raises(P.EcpicError) as e:
        ctx.bind_workspace(nbytes=n - 256)
    assert e.value.status == P.ECPIC_ENOMEM
    ctx.bind_workspace()  # the right size still binds
    ctx.close()


def test_bound_fields_hold_the_state_in_place(torch_cuda):
    import paper_2212_08836_amd as P
    torch = torch_cuda
    _flush("bound fields")
    w = _driven()
    parts = E.make_particles(w)
    a = _context(P, w, parts)
    b = _context(P, w, parts)
    for ctx in (a, b):
        ctx.set_mcc(w.mcc_params())
    # one step in each, then b's state moves into caller tensors
    a.step(tol=w.tol)
    b.step(tol=w.tol)
    ur, uz, h = [torch.from_numpy(x).cuda() for x in b.get_fields()]
    zr, zz, zh = b.zeros_r(), b.zeros_z(), b.zeros_h()
    # u^{n-1} is not readable through the ABI: a takes the same by a set
    # followed by one step from fields set with prev = current in both
    a.set_fields(*[x.cpu().numpy() for x in (ur, uz, h)], t=a.diagnostics()["t"], step=1)
    zr.copy_(ur)
    zz.copy_(uz)
    zh.copy_(h)
    b.bind_fields(ur, uz, h, zr, zz, zh)
    for n in range(3):
        da = a.step(tol=w.tol)
        db = b.step(tol=w.tol)
        _same_iterates(da, db)
        fa = a.get_fields()
        # the caller's tensors hold u^n after every step
        for x, y in zip(fa, (ur, uz, h)):
            assert _rel(y.cpu().numpy(), x) <= 1e-12
    prev = [x.clone() for x in (ur, uz, h)]
    da = a.step(tol=w.tol)
    db = b.step(tol=w.tol)
    for x, y in zip(prev, (zr, zz, zh)):
        assert torch.equal(x, y)  # and u^{n-1} in the prev tensors
    b.bind_fields(None, None, None, None, None, None)
    ur[:] = 0.0  # no longer the state
    _close(_snapshot(a, _qscale(parts)), _snapshot(b, _qscale(parts)))
    a.close()
    b.close()


def test_capacity_overflow_leaves_the_step_uncommitted(torch_cuda):
    # no spare capacity and ionising collisions: the step reports ECAPACITY
    # and leaves everything as it was; the next step (without collisions)
    # is the same as on a context that never saw the failed one
    import paper_2212_08836_amd as P
    _flush("ECAPACITY leaves the step uncommitted")
    w = _driven(seed=4)
    parts = E.make_particles(w)
    for k in ("vr", "vt", "vz"):
        parts[0][k] = parts[0][k] * 3.0  # about 70 eV: ionising
    caps = [len(parts[0]["r"]), len(parts[1]["r"])]
    a = _context(P, w, parts, caps=caps)
    b = _context(P, w, parts, caps=caps)
    for ctx in (a, b):
        ctx.step(tol=w.tol)  # one committed step without collisions
    before = _snapshot(a, _qscale(parts))
    a.set_mcc(w.mcc_params())
    d = a.step(tol=w.tol, check=False)
    assert d["rc"] == P.ECPIC_ECAPACITY and d["converged"] == 1
    _flush(f"  rejected step: {d['iters']} iterations")
    _same(_snapshot(a, _qscale(parts)), before)
    a.set_mcc(None)
    da = a.step(tol=w.tol)
    db = b.step(tol=w.tol)
    _same_iterates(da, db)
    _close(_snapshot(a, _qscale(parts)), _snapshot(b, _qscale(parts)))


def test_over_range_leaves_the_step_uncommitted(torch_cuda):
    # a null-collision bound below the electrons' energies: ERANGE, not
    # committed; with the bound raised the step is the one a fresh context
    # takes
    import paper_2212_08836_amd as P
    _flush("ERANGE leaves the step uncommitted")
    w = _driven(seed=6)
    parts = E.make_particles(w)
    a = _context(P, w, parts)
    b = _context(P, w, parts)
    mcc = w.mcc_params()
    a.set_mcc(dict(mcc, eps_max_ev=1.0))
    before = _snapshot(a, _qscale(parts))
    d = a.step(tol=w.tol, check=False)
    assert d["rc"] == P.ECPIC_ERANGE and d["n_over_range"] > 0
    _same(_snapshot(a, _qscale(parts)), before)
    a.set_mcc(mcc)
    b.set_mcc(mcc)
    da = a.step(tol=w.tol)
    db = b.step(tol=w.tol)
    _same_iterates(da, db)
    assert da["n_over_range"] == 0
    _close(_snapshot(a, _qscale(parts)), _snapshot(b, _qscale(parts)))


def test_not_converged_in_one_iteration(torch_cuda):
    import paper_2212_08836_amd as P
    w = _driven(seed=8)
    parts = E.make_particles(w)
    a = _context(P, w, parts)
    a.set_mcc(w.mcc_params())
    a.step(tol=w.tol)
    before = _snapshot(a, _qscale(parts))
    d = a.step(tol=w.tol, max_iter=1, check=False)
    assert d["rc"] == P.ECPIC_ENOTCONV and d["iters"] == 1 and d["converged"] == 0
    _same(_snapshot(a, _qscale(parts)), before)


def test_collide_overflow_applies_no_partial_pair(og, torch_cuda):
    # the stand-alone collision call with no room for new ions: every pair
    # that does not fit is dropped whole (its electron keeps its velocity),
    # no unwritten slot becomes a particle, and every other collision is the
    # oracle's (same draws)
    import paper_2212_08836_amd as P
    _flush("collide overflow")
    w = _driven(seed=10)
    parts = E.make_particles(w)
    for k in ("vr", "vt", "vz"):
        parts[0][k] = parts[0][k] * 3.0
    ne, ni = len(parts[0]["r"]), len(parts[1]["r"])
    ctx = _context(P, w, parts, caps=[ne + 64, ni])  # room for electrons only
    mcc = w.mcc_params()
    before = ctx.read_particles(0)
    with pytest.raises(P.EcpicError) as e:
        ctx.collide(mcc, 3)
    assert e.value.status == P.ECPIC_ECAPACITY
    el, ions = ctx.read_particles(0), ctx.read_particles(1)
    assert len(ions["uid"]) == ni   # no ion was added
    assert len(el["uid"]) == ne     # reserved electron slots are dead, not particles
    # the oracle with room for everything
    g = og.grid_from_workload(w)
    sp = [g.species(d, cap=3 * len(d["r"]) + 64, role=k + 1) for k, d in enumerate(parts)]
    og.Grid.collide(g, sp, mcc, 3)
    ov = sp[0].view()
    born = set(int(u) for u in ov["uid"][ne:])
    parents = {int(u) for u in before["uid"] if og.child_uid(int(u), 3) in born}
    assert len(parents) == len(born) > 0
    gi = {int(u): i for i, u in enumerate(el["uid"])}
    oi = {int(u): i for i, u in enumerate(ov["uid"][:ne])}
    bi = {int(u): i for i, u in enumerate(before["uid"])}
    vmax = max(np.abs(ov[k][:ne]).max() for k in ("vr", "vt", "vz"))
    for u in bi:
        a, o, b = gi[u], oi[u], bi[u]
        for k in ("vr", "vt", "vz"):
            if u in parents:
                assert el[k][a] == before[k][b]
            else:
                assert abs(el[k][a] - ov[k][o]) <= 1e-12 * vmax
    _flush(f"  {len(parents)} ionisations dropped whole, {ne - len(parents)} electrons as the oracle")


def test_conservation_check_c1_and_driven(og, torch_cuda):
    # the library's own continuity and Gauss residuals over checked steps
    import paper_2212_08836_amd as P
    torch = torch_cuda
    _flush("conservation check")
    for w, mcc in ((E.workload("c1"), None), (_driven(seed=12), "mcc")):
        parts = E.make_particles(w)
        ctx = _context(P, w, parts, caps=[2 * len(parts[0]["r"]), 2 * len(parts[1]["r"])])
        if mcc:
            ctx.set_mcc(w.mcc_params())
        for n in range(4):
            d = ctx.step(tol=w.tol, conservation=True, sort_every=3)
            assert d["q_max"] > 0
            _flush(f"  {w.name} step {n}: continuity {d['continuity_max'] / d['q_max']:.1e}, "
                   f"gauss {d['gauss_max'] / d['q_max']:.1e}")
            assert d["continuity_max"] <= 1e-13 * d["q_max"]
            assert d["gauss_max"] <= 1e-12 * d["q_max"]
        ctx.close()
    # a field change the step did not make is a Gauss violation the check sees
    w = E.workload("c1")
    parts = E.make_particles(w)
    ctx = _context(P, w, parts)
    ur, uz, h = (torch.zeros_like(x) for x in (ctx.zeros_r(), ctx.zeros_z(), ctx.zeros_h()))
    pr, pz, ph = (torch.zeros_like(x) for x in (ur, uz, h))
    ctx.bind_fields(ur, uz, h, pr, pz, ph)
    d = ctx.step(tol=w.tol, conservation=True)
    assert d["gauss_max"] <= 1e-12 * d["q_max"]
    uz.view(w.nr + 1, w.nz)[w.nr // 2, w.nz // 2] += 1.0  # 1 V on one z-edge
    d = ctx.step(tol=w.tol, conservation=True)
    assert d["gauss_max"] > 1e3 * d["q_max"] * 1e-12
    assert d["continuity_max"] <= 1e-13 * d["q_max"]
    ctx.close()
