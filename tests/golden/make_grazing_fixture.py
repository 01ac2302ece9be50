"""Writes grazing_particle.npz: an electron whose orbit turns at a face
within a step, with the half-step field it is pushed in.  It comes from the
oracle's own run of a 32 x 32 cavity (3e15 m^-3, 50 MHz through the TEM port
and a blocking capacitor, seed 9, tolerance 1e-11): at step 594 the free
sub-step of this electron leaves its cell across the eta face, but the
constrained crossing solve finds no consistent root.  Calls only the oracle
and the input generators."""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import ecpic_inputs as E  # noqa: E402
import oracle as og  # noqa: E402

STEP, INDEX = 594, 19319


def workload():
    return E.Workload("p", 32, 32, 0.02, 0.02, n0=3e15, ppc=32, dt=5e-11, drive_amp=(100.0,),
                      drive_freq=(50e6,), seed=9, tol=1e-11, port_i=24, port_eps=3.8)


def face_capacitance(w):
    g = og.Grid(w.nr, w.nz, w.R, w.L, w.xi_a, w.dt, E.EPS0, E.MU0, drive_amp=(1.0,),
                drive_freq=(1e3,), model="es", port_i=w.port_i, port_eps=w.port_eps)
    t = g.tables()
    _, uz1, _ = g.field_solve(g.zeros_r(), g.zeros_z(), g.zeros_h(), g.zeros_r(), g.zeros_z(), 0.0)
    uz = uz1.reshape(w.nr + 1, w.nz)
    return sum(t["wz"][i] * uz[i, 0] for i in range(w.port_i + 1)) / g.drive(w.dt)


def main():
    w = workload()
    g = og.grid_from_workload(w, cap=100.0 * face_capacitance(w), omp=True)
    sp = og.species_from_workload(g, E.make_particles(w), extra_cap=0.5)
    st = og.State(g)
    for n in range(STEP):
        assert g.step(st, sp, tol=w.tol, max_iter=50)["rc"] == 0, n
    e = sp[0].view()
    p = {k: np.array([e[k][INDEX]]) for k in ("xi", "eta", "vr", "vt", "vz", "uid")}
    ur0, uz0 = st.ur.copy(), st.uz.copy()
    assert g.step(st, sp, tol=w.tol, max_iter=50)["rc"] == 0
    np.savez(os.path.join(HERE, "grazing_particle.npz"), ur_h=0.5 * (ur0 + st.ur),
             uz_h=0.5 * (uz0 + st.uz), q=sp[0].q, m=sp[0].m, w=sp[0].w, **p)


if __name__ == "__main__":
    main()
