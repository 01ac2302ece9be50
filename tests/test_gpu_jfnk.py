"""The Jacobian-free Newton-Krylov solver on the HIP path (Sec. 2.1 names
JFNK beside Picard): its answer against Picard's on the GPU and against the
oracle's JFNK, a fixed-count run against the oracle's, and the dense plasma
(omega_pe dt = 3.4) where Picard diverges and JFNK converges.

Bars: a forward-difference Jacobian carries the rounding of the map G
divided by the difference step (about 1e-16 / 1.5e-8 relative), so two
JFNK runs agree on their Newton corrections only to about 1e-8 of the
correction; the converged answer is unique only to within the tolerance,
so converged fields are compared at 1e-10."""
import math
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


def _ctx(P, w, krylov=20, model="em"):
    ctx = P.context_from_workload(w, model=model)
    ctx.set_option(P.ECPIC_OPT_JFNK_KRYLOV, krylov)
    P.load_workload_species(ctx, E.make_particles(w), extra_cap=0.5)
    return ctx


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


def test_jfnk_matches_picard_and_the_oracle(og, torch_cuda):
    import paper_2212_08836_amd as P
    _flush("JFNK against Picard (GPU) and the oracle's JFNK, c1, tol 1e-12")
    w = E.workload("c1")
    a = _ctx(P, w)
    b = _ctx(P, w)
    g = og.grid_from_workload(w)
    sp = og.species_from_workload(g, E.make_particles(w), extra_cap=0.5)
    st = og.State(g)
    for n in range(4):
        da = a.step(tol=1e-12)
        db = b.step(tol=1e-12, solver="jfnk", krylov=10, eta=1e-3)
        do = g.step(st, sp, tol=1e-12, solver="jfnk", krylov=10, eta=1e-3)
        assert do["rc"] == 0 and db["newton_iters"] >= 2
        _flush(f"  step {n}: Picard {da['iters']} passes, JFNK {db['iters']} passes / "
               f"{db['newton_iters']} Newton / {db['krylov_iters']} Krylov "
               f"(oracle {do['iters']}/{do['newton_iters']}/{do['krylov_iters']}), residuals "
               f"{np.array(db['residual'][:db['newton_iters']])}")
        fa, fb = a.get_fields(), b.get_fields()
        for x, y, z in zip(fa, fb, (st.ur, st.uz, st.h)):
            assert _rel(y, x) < 1e-10
            assert _rel(y, z) < 1e-10
        pa, pb = a.read_particles(0), b.read_particles(0)
        assert np.abs(pa["xi"] - pb["xi"]).max() < 1e-10


@pytest.mark.parametrize("krylov", [1, 4])
def test_jfnk_fixed_counts_against_the_oracle(og, torch_cuda, krylov):
    """Three Newton residual evaluations with exactly `krylov` GMRES
    iterations each.  With one Krylov direction the residual histories agree
    closely.  Later directions come from differences of nearly equal maps,
    whose noise (deposit order, inner-solve truncation) differs between the
    two implementations and is about 1e-8 of |v| against |J v - v| near 2e-5
    here; the Newton step's remaining residual (1e-7 of |u|) depends on it.
    There both must reach it, and the fields must agree at the step's bar."""
    import paper_2212_08836_amd as P
    _flush(f"JFNK fixed counts (3 Newton evaluations, {krylov} Krylov each) against the oracle")
    w = E.workload("c1")
    ctx = _ctx(P, w, krylov=krylov)
    g = og.grid_from_workload(w)
    sp = og.species_from_workload(g, E.make_particles(w), extra_cap=0.5)
    st = og.State(g)
    for n in range(3):
        d = ctx.step(fixed_iter=3, solver="jfnk", krylov=krylov)
        do = g.step(st, sp, fixed_iter=3, solver="jfnk", krylov=krylov)
        assert d["iters"] == do["iters"] == 1 + 2 * (krylov + 1)
        assert d["newton_iters"] == 3 and d["krylov_iters"] == 2 * krylov
        _flush(f"  step {n}: residuals {np.array(d['residual'][:3])}, "
               f"oracle {np.array(do['residual'][:3])}")
        assert abs(d["residual"][0] - do["residual"][0]) <= 1e-9 * do["residual"][0]
        if krylov == 1:
            # a residual near 1e-10 of |u| carries the two sides' rounding of
            # u (1e-14) at 1e-4 of itself
            for k, bar in ((1, 1e-5), (2, 1e-3)):
                assert abs(d["residual"][k] - do["residual"][k]) <= bar * do["residual"][k]
        else:
            assert d["residual"][1] < 1e-6 and d["residual"][2] < 1e-9
        f = ctx.get_fields()
        errs = [_rel(x, y) for x, y in zip(f, (st.ur, st.uz, st.h))]
        _flush(f"  field errors {errs}")
        assert max(errs) < 1e-10


def test_dense_plasma_picard_fails_jfnk_converges(og, torch_cuda):
    import paper_2212_08836_amd as P
    _flush("dense plasma, omega_pe dt = 3.4: Picard ENOTCONV, JFNK converges")
    w = E.workload("c1", n0=1e18, dt=6e-11, tol=1e-10)
    assert math.sqrt(w.n0 * E.QE ** 2 / (E.EPS0 * E.ME)) * w.dt > 3.0
    pic = _ctx(P, w)
    d = pic.step(tol=w.tol, max_iter=50, check=False)
    assert d["rc"] == P.ECPIC_ENOTCONV and d["residual"][49] > 0.5
    ctx = _ctx(P, w)
    g = og.grid_from_workload(w)
    W_prev = None
    for n in range(4):
        d = ctx.step(tol=w.tol, max_iter=20, solver="jfnk", krylov=20, eta=1e-4,
                     conservation=True)
        _flush(f"  step {n}: {d['iters']} passes, {d['newton_iters']} Newton, "
               f"{d['krylov_iters']} Krylov, residuals "
               f"{np.array(d['residual'][:d['newton_iters']])}, Gauss {d['gauss_max']:.2e} "
               f"of {d['q_max']:.2e}")
        assert d["rc"] == 0 and d["converged"]
        assert d["gauss_max"] < 1e-10 * d["q_max"]
        W = sum(d["ke"][:2]) + d["we"] + d["wb"]
        if W_prev is not None:
            assert abs(W - W_prev + d["w_absorbed"]) <= 10 * w.tol * W_prev
        W_prev = W
    ur, uz, _ = ctx.get_fields()
    q, _, _, _ = ctx.node_charge()
    G = g.gauss(ur, uz).reshape(w.nr + 1, w.nz + 1)
    Q = np.asarray(q).reshape(w.nr + 1, w.nz + 1)
    assert np.abs(G - Q)[: w.nr, 1: w.nz].max() < 1e-10 * np.abs(Q).max()


def test_jfnk_needs_reserved_space(torch_cuda):
    import paper_2212_08836_amd as P
    w = E.workload("c1")
    ctx = P.context_from_workload(w)
    P.load_workload_species(ctx, E.make_particles(w, n=256))
    d = ctx.step(solver="jfnk", krylov=4, check=False)
    assert d["rc"] == P.ECPIC_EINVAL
    with pytest.raises(Exception):
        ctx.set_option(P.ECPIC_OPT_JFNK_KRYLOV, 4)  # device memory already set up
