"""The OpenMP timing build of the oracle (the CPU baseline on all host
cores) computes what the single-threaded oracle computes: each particle is
pushed by the same code, only the currents are summed in another order."""
import numpy as np

import ecpic_inputs as E


def test_threaded_build_matches_the_serial_oracle(og):
    assert og.threads(omp=False) == 1
    w = E.workload("c2", ppc=2)
    parts = E.make_particles(w)
    res = []
    for omp in (False, True):
        g = og.grid_from_workload(w, omp=omp)
        sp = [g.species(d, cap=len(d["r"]) * 2 + 64, role=k + 1) for k, d in enumerate(parts)]
        st = og.State(g)
        mcc = w.mcc_params()
        ds = [g.step(st, sp, mcc=mcc, tol=w.tol) for _ in range(2)]
        res.append((st, sp, ds))
    (s0, p0, d0), (s1, p1, d1) = res
    for a, b in zip(d0, d1):
        assert a["iters"] == b["iters"] and a["rc"] == b["rc"] == 0
        for key in ("n_crossings", "n_substeps", "n_ionized"):
            assert a[key] == b[key], key
    for x, y in ((s0.ur, s1.ur), (s0.uz, s1.uz), (s0.h, s1.h)):
        assert np.abs(x - y).max() <= 1e-12 * np.abs(x).max()
    for a, b in zip(p0, p1):
        va, vb = a.view(), b.view()
        assert np.array_equal(va["uid"], vb["uid"])
        assert np.abs(va["xi"] - vb["xi"]).max() <= 1e-12
