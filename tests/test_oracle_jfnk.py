"""Pins of the oracle's Jacobian-free Newton-Krylov solve of the implicit
step (Sec. 2.1 names JFNK beside Picard): it reaches Picard's answer where
Picard converges, with Newton's fast convergence, keeps Gauss's law and
the energy balance, and converges where Picard diverges (a plasma period
shorter than the step, omega_pe dt = 3.4)."""
import math

import numpy as np

import ecpic_inputs as E

from test_oracle_step import _bilinear_charge


def _setup(og, w):
    g = og.grid_from_workload(w)
    sp = og.species_from_workload(g, E.make_particles(w), extra_cap=0.5)
    return g, sp, og.State(g)


def test_jfnk_reaches_the_picard_answer(og):
    w = E.workload("c1")
    g1, sp1, st1 = _setup(og, w)
    g2, sp2, st2 = _setup(og, w)
    for n in range(3):
        a = g1.step(st1, sp1, tol=1e-12)
        b = g2.step(st2, sp2, tol=1e-12, solver="jfnk", krylov=10, eta=1e-3)
        assert a["rc"] == 0 and b["rc"] == 0
        # Newton: each residual at most about the square of the one before
        # (down to the forward-difference floor)
        r = b["residual"][: b["newton_iters"]]
        assert r[-1] <= 1e-12 and b["newton_iters"] <= 5
        for k in range(1, len(r) - 1):
            assert r[k + 1] <= 10.0 * r[k] ** 2 + 1e-12
        for x, y in ((st1.ur, st2.ur), (st1.uz, st2.uz), (st1.h, st2.h)):
            assert np.abs(x - y).max() <= 1e-11 * np.abs(x).max()
        for s1, s2 in zip(sp1, sp2):
            assert np.abs(s1.xi[: s1.n] - s2.xi[: s2.n]).max() < 1e-11
            vmax = np.abs(s1.vr[: s1.n]).max()
            assert np.abs(s1.vr[: s1.n] - s2.vr[: s2.n]).max() < 1e-11 * vmax


def test_jfnk_fixed_counts_are_deterministic(og):
    w = E.workload("c1")
    out = []
    for _ in range(2):
        g, sp, st = _setup(og, w)
        d = g.step(st, sp, fixed_iter=3, solver="jfnk", krylov=4)
        assert d["rc"] == 0 and d["newton_iters"] == 3 and d["krylov_iters"] == 8
        assert d["iters"] == 1 + 2 * (4 + 1)  # residual maps, Krylov maps, steps
        out.append(st.ur.copy())
    assert np.array_equal(out[0], out[1])


def test_dense_plasma_picard_diverges_jfnk_converges(og):
    w = E.workload("c1", n0=1e18, dt=6e-11, tol=1e-10)
    wpe = math.sqrt(w.n0 * E.QE ** 2 / (E.EPS0 * E.ME))
    assert wpe * w.dt > 3.0
    g, sp, st = _setup(og, w)
    d = g.step(st, sp, tol=w.tol, max_iter=50)
    assert d["rc"] == -4 and d["residual"][49] > 0.5
    g, sp, st = _setup(og, w)
    nr, nz = g.nr, g.nz
    W_prev = sum(0.5 * s.m * s.w * np.sum(s.vr[: s.n] ** 2 + s.vt[: s.n] ** 2 + s.vz[: s.n] ** 2)
                 for s in sp)
    qscale = abs(sp[0].q * sp[0].w) * w.ppc
    for n in range(3):
        d = g.step(st, sp, tol=w.tol, max_iter=20, solver="jfnk", krylov=20, eta=1e-4)
        assert d["rc"] == 0, (n, d["residual"][: d["newton_iters"]])
        W = sum(d["ke"][:2]) + d["we"] + d["wb"]
        assert abs(W - W_prev + d["w_absorbed"]) <= 10 * w.tol * W_prev
        W_prev = W
        Q = _bilinear_charge(nr, nz, sp)
        G = g.gauss(st.ur, st.uz).reshape(nr + 1, nz + 1)
        assert np.abs(G - Q)[:nr, 1:nz].max() < 1e-12 * qscale
