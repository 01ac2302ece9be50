"""FP64 CPU oracle of the implicit EM PIC/MCC step (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the bench
may import this package.  It wraps ``libecpic_oracle.so`` (plain C, built by
``build()`` with gcc) through ctypes and shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ecpic_oracle.c")
_LIB = os.path.join(_HERE, "libecpic_oracle.so")
# the same source with OpenMP: only for timing the CPU baseline on all cores
_LIB_OMP = os.path.join(_HERE, "libecpic_oracle_omp.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast-math), and
    its OpenMP timing build."""
    for out, extra in ((_LIB, []), (_LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(out):
            tmp = out + ".tmp"
            subprocess.run(["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-ffp-contract=off",
                            "-Wall", *extra, "-o", tmp, _SRC, "-lm"], check=True)
            os.replace(tmp, out)
    return _LIB


_libs = {}


def lib(omp: bool = False):
    """The oracle library; omp=True: the OpenMP timing build."""
    if omp not in _libs:
        path = _LIB_OMP if omp else _LIB
        if not os.path.exists(path):
            build(force=False)
        L = C.CDLL(path)
        _declare(L)
        _libs[omp] = L
    return _libs[omp]


def threads(omp: bool = False) -> int:
    """Threads a push pass of that build uses."""
    return int(lib(omp).og_threads())


class OgGrid(C.Structure):
    _fields_ = [("nr", C.c_int32), ("nz", C.c_int32), ("R", C.c_double), ("L", C.c_double),
                ("xi_a", C.c_double), ("dt", C.c_double), ("eps", C.c_double), ("mu", C.c_double),
                ("n_drive", C.c_int32), ("self_b", C.c_int32),
                ("drive_amp", C.c_double * 32), ("drive_freq", C.c_double * 32),
                ("drive_phase", C.c_double * 32), ("drive_t_end", C.c_double),
                ("bz_ext", C.c_double), ("er_ext", C.c_double),
                ("sub_tol", C.c_double), ("push_only", C.c_int32), ("model", C.c_int32),
                ("cap", C.c_double), ("port_i", C.c_int32), ("port_eps", C.c_double)]


_dp = C.POINTER(C.c_double)
_u64p = C.POINTER(C.c_uint64)


class OgSpecies(C.Structure):
    _fields_ = [("q", C.c_double), ("m", C.c_double), ("w", C.c_double), ("mobile", C.c_int32),
                ("mcc_role", C.c_int32), ("n", C.c_int64), ("cap", C.c_int64),
                ("xi", _dp), ("eta", _dp), ("vr", _dp), ("vt", _dp), ("vz", _dp), ("uid", _u64p)]


class OgState(C.Structure):
    _fields_ = [("ur", _dp), ("uz", _dp), ("h", _dp), ("ur_prev", _dp), ("uz_prev", _dp),
                ("wall_bot", _dp), ("wall_top", _dp), ("wall_side", _dp),
                ("t", C.c_double), ("step", C.c_int64), ("phi", C.c_double),
                ("phi_prev", C.c_double), ("q_cap", C.c_double), ("hb", _dp)]


class OgOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("fixed_iter", C.c_int32),
                ("solver", C.c_int32), ("krylov", C.c_int32), ("eta", C.c_double)]


class OgMcc(C.Structure):
    _fields_ = [("enabled", C.c_int32), ("electron_sid", C.c_int32), ("ion_sid", C.c_int32),
                ("pad", C.c_int32), ("n_gas", C.c_double), ("T_gas", C.c_double),
                ("m_gas", C.c_double), ("eps_max_ev", C.c_double), ("seed", C.c_uint64)]


class OgStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("residual", C.c_double * 64),
                ("ke", C.c_double * 4), ("we", C.c_double), ("wb", C.c_double),
                ("w_particles", C.c_double), ("w_field_io", C.c_double), ("w_drive", C.c_double),
                ("w_absorbed", C.c_double), ("w_coll", C.c_double),
                ("n_absorbed", C.c_int64 * 4), ("n_coll", C.c_int64 * 4), ("n_ionized", C.c_int64),
                ("n_substeps", C.c_int64), ("n_crossings", C.c_int64), ("n_halvings", C.c_int64),
                ("n_errors", C.c_int64), ("n_capped", C.c_int64), ("n_over_range", C.c_int64),
                ("newton_iters", C.c_int32), ("krylov_iters", C.c_int32),
                ("phi", C.c_double), ("q_cap", C.c_double), ("w_gen", C.c_double),
                ("port_v", C.c_double)]

    def as_dict(self) -> dict:
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            if hasattr(v, "__len__"):
                v = list(v)
            d[name] = v
        d["residual"] = d["residual"][: self.iters]
        return d


def _declare(L):
    vp = C.c_void_p
    L.og_create.argtypes = [C.POINTER(OgGrid), C.POINTER(vp)]
    L.og_create.restype = C.c_int
    L.og_destroy.argtypes = [vp]
    for f in ("og_r_of_xi", "og_jr_of_xi", "og_xi_of_r", "og_drive"):
        getattr(L, f).argtypes = [vp, C.c_double]
        getattr(L, f).restype = C.c_double
    L.og_tables.argtypes = [vp] + [_dp] * 6
    L.og_curl_e.argtypes = [vp, _dp, _dp, _dp]
    L.og_curl_h.argtypes = [vp, _dp, _dp, _dp]
    L.og_div.argtypes = [vp, _dp, _dp, _dp]
    L.og_field_solve.argtypes = [vp, _dp, _dp, _dp, _dp, _dp, C.c_double, _dp, _dp, _dp]
    L.og_push_deposit.argtypes = [vp, C.POINTER(OgSpecies), _dp, _dp, _dp, C.c_int, _dp, _dp,
                                  C.POINTER(OgState), C.POINTER(OgStats)]
    L.og_step.argtypes = [vp, C.POINTER(OgState), C.POINTER(OgSpecies), C.c_int32,
                          C.POINTER(OgMcc), C.POINTER(OgOpts), C.POINTER(OgStats)]
    L.og_collide.argtypes = [vp, C.POINTER(OgSpecies), C.c_int32, C.POINTER(OgMcc), C.c_int64,
                             C.POINTER(OgStats)]
    L.og_nu_max.argtypes = [C.POINTER(OgMcc), C.c_int32, C.c_double]
    L.og_nu_max.restype = C.c_double
    L.og_cross_sections.argtypes = [C.c_double, _dp, _dp, _dp]
    L.og_node_charge.argtypes = [vp, C.POINTER(OgSpecies), C.c_int32, _dp]
    L.og_gauss.argtypes = [vp, _dp, _dp, _dp]
    for f in ("og_energy_e", "og_energy_norm2"):
        getattr(L, f).argtypes = [vp, _dp, _dp]
        getattr(L, f).restype = C.c_double
    L.og_energy_b.argtypes = [vp, _dp]
    L.og_energy_b.restype = C.c_double
    L.og_kinetic.argtypes = [C.POINTER(OgSpecies)]
    L.og_kinetic.restype = C.c_double
    L.og_philox4x64_10.argtypes = [_u64p, _u64p, _u64p]
    L.og_child_uid.argtypes = [C.c_uint64, C.c_int64]
    L.og_child_uid.restype = C.c_uint64
    L.og_threads.argtypes = []
    L.og_threads.restype = C.c_int
    L.og_set_port_h.argtypes = [vp, _dp]
    L.og_get_port_h.argtypes = [vp, _dp]
    L.og_port_tables.argtypes = [vp, _dp, _dp]


def _p(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


class Species:
    """Particle arrays of one species (caller-owned, with spare capacity)."""

    def __init__(self, q, m, w, xi, eta, vr, vt, vz, uid, mobile=True, cap=None, role=0):
        n = len(xi)
        cap = max(cap or n, n, 1)
        self.q, self.m, self.w, self.mobile, self.role = float(q), float(m), float(w), bool(mobile), role
        self.n = n
        self.cap = cap

        def buf(a, dt=np.float64):
            b = np.zeros(cap, dtype=dt)
            b[:n] = a
            return b
        self.xi, self.eta = buf(xi), buf(eta)
        self.vr, self.vt, self.vz = buf(vr), buf(vt), buf(vz)
        self.uid = buf(uid, np.uint64)

    def struct(self) -> OgSpecies:
        return OgSpecies(self.q, self.m, self.w, int(self.mobile), int(self.role), self.n, self.cap,
                         _p(self.xi), _p(self.eta), _p(self.vr), _p(self.vt), _p(self.vz),
                         self.uid.ctypes.data_as(_u64p))

    def view(self) -> dict:
        n = self.n
        return dict(xi=self.xi[:n].copy(), eta=self.eta[:n].copy(), vr=self.vr[:n].copy(),
                    vt=self.vt[:n].copy(), vz=self.vz[:n].copy(), uid=self.uid[:n].copy())

    def copy(self) -> "Species":
        v = self.view()
        return Species(self.q, self.m, self.w, v["xi"], v["eta"], v["vr"], v["vt"], v["vz"],
                       v["uid"], self.mobile, self.cap, self.role)


class State:
    """Field state at t^n (plus u at t^{n-1}) and wall charge accumulators."""

    def __init__(self, grid: "Grid"):
        nr, nz = grid.nr, grid.nz
        self.ur = np.zeros(nr * (nz + 1))
        self.uz = np.zeros((nr + 1) * nz)
        self.h = np.zeros(nr * nz)
        self.ur_prev = np.zeros_like(self.ur)
        self.uz_prev = np.zeros_like(self.uz)
        self.wall_bot = np.zeros(nr + 1)
        self.wall_top = np.zeros(nr + 1)
        self.wall_side = np.zeros(nz + 1)
        self.t = 0.0
        self.step = 0
        self.phi = 0.0       # electrode potential (blocking capacitor)
        self.phi_prev = 0.0
        self.q_cap = 0.0     # capacitor charge
        self.hb = np.zeros(nr)  # port: H_theta on the wall under the port edges

    def struct(self) -> OgState:
        return OgState(_p(self.ur), _p(self.uz), _p(self.h), _p(self.ur_prev), _p(self.uz_prev),
                       _p(self.wall_bot), _p(self.wall_top), _p(self.wall_side), self.t, self.step,
                       self.phi, self.phi_prev, self.q_cap, _p(self.hb))

    def copy(self) -> "State":
        s = State.__new__(State)
        for k, v in self.__dict__.items():
            setattr(s, k, v.copy() if isinstance(v, np.ndarray) else v)
        return s


class Grid:
    """Mesh, mapping, field operators and the factorised H_theta system."""

    def __init__(self, nr, nz, R, L, xi_a, dt, eps, mu, drive_amp=(), drive_freq=(),
                 drive_phase=(), drive_t_end=0.0, self_b=False, bz_ext=0.0, er_ext=0.0,
                 sub_tol=0.0, omp=False, push_only=False, model="em", cap=0.0, port_i=0,
                 port_eps=1.0):
        L_ = lib(omp)
        g = OgGrid()
        g.nr, g.nz, g.R, g.L, g.xi_a, g.dt, g.eps, g.mu = nr, nz, R, L, xi_a, dt, eps, mu
        g.n_drive = len(drive_amp)
        for k in range(len(drive_amp)):
            g.drive_amp[k] = drive_amp[k]
            g.drive_freq[k] = drive_freq[k]
            g.drive_phase[k] = drive_phase[k] if k < len(drive_phase) else 0.0
        g.drive_t_end = drive_t_end
        g.self_b = int(self_b)
        g.bz_ext, g.er_ext, g.sub_tol = bz_ext, er_ext, sub_tol
        g.push_only = int(push_only)
        g.model = {"em": 0, "es": 1}[model]
        g.cap = cap
        g.port_i, g.port_eps = port_i, port_eps
        self.port_i, self.port_eps = port_i, port_eps
        self.desc = g
        self.nr, self.nz, self.R, self.L, self.xi_a, self.dt = nr, nz, R, L, xi_a, dt
        self.eps, self.mu = eps, mu
        self.model = model
        h = C.c_void_p()
        rc = L_.og_create(C.byref(g), C.byref(h))
        if rc != 0:
            raise RuntimeError(f"og_create failed: {rc}")
        self._h = h
        self._lib = L_

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.og_destroy(h)
            self._h = None

    # mapping
    def r_of_xi(self, xi):
        return np.vectorize(lambda x: self._lib.og_r_of_xi(self._h, float(x)))(xi)

    def jr_of_xi(self, xi):
        return np.vectorize(lambda x: self._lib.og_jr_of_xi(self._h, float(x)))(xi)

    def xi_of_r(self, r):
        return np.vectorize(lambda x: self._lib.og_xi_of_r(self._h, float(x)), otypes=[np.float64])(r)

    def drive(self, t: float) -> float:
        return self._lib.og_drive(self._h, float(t))

    def tables(self) -> dict:
        nr = self.nr
        rn, rh, a, wr, wz, vol = (np.zeros(nr + 1), np.zeros(nr), np.zeros(nr), np.zeros(nr),
                                  np.zeros(nr), np.zeros(nr))
        self._lib.og_tables(self._h, _p(rn), _p(rh), _p(a), _p(wr), _p(wz), _p(vol))
        return dict(rn=rn, rh=rh, area=a, wr=wr, wz=wz, vol=vol)

    # shapes
    def zeros_r(self):
        return np.zeros(self.nr * (self.nz + 1))

    def zeros_z(self):
        return np.zeros((self.nr + 1) * self.nz)

    def zeros_h(self):
        return np.zeros(self.nr * self.nz)

    def zeros_node(self):
        return np.zeros((self.nr + 1) * (self.nz + 1))

    # operators
    def curl_e(self, ur, uz):
        out = self.zeros_h()
        self._lib.og_curl_e(self._h, _p(ur), _p(uz), _p(out))
        return out

    def curl_h(self, h):
        kr, kz = self.zeros_r(), self.zeros_z()
        self._lib.og_curl_h(self._h, _p(h), _p(kr), _p(kz))
        return kr, kz

    def div(self, fr, fz):
        out = self.zeros_node()
        self._lib.og_div(self._h, _p(fr), _p(fz), _p(out))
        return out

    def gauss(self, ur, uz):
        out = self.zeros_node()
        self._lib.og_gauss(self._h, _p(ur), _p(uz), _p(out))
        return out

    def energy_e(self, ur, uz) -> float:
        return self._lib.og_energy_e(self._h, _p(ur), _p(uz))

    def energy_b(self, h) -> float:
        return self._lib.og_energy_b(self._h, _p(h))

    def energy_norm2(self, ur, uz) -> float:
        return self._lib.og_energy_norm2(self._h, _p(ur), _p(uz))

    def set_port_h(self, hb):
        """H_b at t of the port edges (used by the next field_solve)."""
        self._lib.og_set_port_h(self._h, _p(np.ascontiguousarray(hb, dtype=np.float64)))

    def get_port_h(self):
        """H_b at t + dt left by the last field_solve."""
        out = np.zeros(self.nr)
        self._lib.og_get_port_h(self._h, _p(out))
        return out

    def port_tables(self):
        """(kappa[nr], wall potential profile[nr+1]) of the port."""
        k, p = np.zeros(self.nr), np.zeros(self.nr + 1)
        self._lib.og_port_tables(self._h, _p(k), _p(p))
        return k, p

    def field_solve(self, ur0, uz0, h0, Ir, Iz, t):
        ur1, uz1, h1 = self.zeros_r(), self.zeros_z(), self.zeros_h()
        rc = self._lib.og_field_solve(self._h, _p(ur0), _p(uz0), _p(h0), _p(Ir), _p(Iz),
                                      float(t), _p(ur1), _p(uz1), _p(h1))
        assert rc == 0
        return ur1, uz1, h1

    def node_charge(self, species: Sequence[Species]):
        arr = (OgSpecies * len(species))(*[s.struct() for s in species])
        out = self.zeros_node()
        self._lib.og_node_charge(self._h, arr, len(species), _p(out))
        return out

    def push_deposit(self, sp: Species, ur_h, uz_h, h_h=None, commit=False, state=None,
                     Ir=None, Iz=None):
        Ir = self.zeros_r() if Ir is None else Ir
        Iz = self.zeros_z() if Iz is None else Iz
        st = OgStats()
        s = sp.struct()
        stc = state.struct() if state is not None else None
        rc = self._lib.og_push_deposit(self._h, C.byref(s), _p(ur_h), _p(uz_h), _p(h_h),
                                       int(commit), _p(Ir), _p(Iz),
                                       C.byref(stc) if stc is not None else None, C.byref(st))
        if commit:
            sp.n = s.n
        return Ir, Iz, rc, st.as_dict()

    def species(self, d: dict, mobile=True, cap=None, role=0) -> Species:
        """Species from an input-generator dict (physical r, z -> logical)."""
        xi = self.xi_of_r(d["r"])
        eta = d["z"] / (self.L / self.nz)
        return Species(d["q"], d["m"], d["w"], xi, eta, d["vr"], d["vt"], d["vz"], d["uid"],
                       mobile=mobile, cap=cap, role=role)

    def step(self, state: State, species: List[Species], mcc: Optional[dict] = None,
             tol=1e-10, max_iter=50, fixed_iter=0, solver="picard", krylov=10,
             eta=1e-4) -> dict:
        arr = (OgSpecies * len(species))(*[s.struct() for s in species])
        stc = state.struct()
        o = OgOpts(tol, max_iter, fixed_iter, {"picard": 0, "jfnk": 1}[solver], krylov, eta)
        m = make_mcc(mcc)
        st = OgStats()
        rc = self._lib.og_step(self._h, C.byref(stc), arr, len(species),
                               C.byref(m) if m is not None else None, C.byref(o), C.byref(st))
        for k, s in enumerate(species):
            s.n = arr[k].n
        state.t = stc.t
        state.step = stc.step
        state.phi, state.phi_prev, state.q_cap = stc.phi, stc.phi_prev, stc.q_cap
        d = st.as_dict()
        d["rc"] = rc
        return d

    def collide(self, species: List[Species], mcc: dict, step: int) -> dict:
        arr = (OgSpecies * len(species))(*[s.struct() for s in species])
        m = make_mcc(mcc)
        st = OgStats()
        rc = self._lib.og_collide(self._h, arr, len(species), C.byref(m), int(step), C.byref(st))
        for k, s in enumerate(species):
            s.n = arr[k].n
        d = st.as_dict()
        d["rc"] = rc
        return d


def make_mcc(mcc: Optional[dict]) -> Optional[OgMcc]:
    if mcc is None:
        return None
    return OgMcc(1, mcc.get("electron_sid", 0), mcc.get("ion_sid", 1), 0, mcc["n_gas"],
                 mcc["T_gas"], mcc["m_gas"], mcc["eps_max_ev"], mcc["seed"])


def nu_max(mcc: dict, role: int, m: float) -> float:
    return lib().og_nu_max(C.byref(make_mcc(mcc)), role, m)


def cross_sections(e: float):
    a, b, c = C.c_double(), C.c_double(), C.c_double()
    lib().og_cross_sections(float(e), C.byref(a), C.byref(b), C.byref(c))
    return a.value, b.value, c.value


def philox4x64_10(ctr: Sequence[int], key: Sequence[int]) -> List[int]:
    c = (C.c_uint64 * 4)(*[int(x) & (2**64 - 1) for x in ctr])
    k = (C.c_uint64 * 2)(*[int(x) & (2**64 - 1) for x in key])
    o = (C.c_uint64 * 4)()
    lib().og_philox4x64_10(c, k, o)
    return list(o)


def child_uid(parent: int, step: int) -> int:
    return int(lib().og_child_uid(int(parent), int(step)))


def grid_from_workload(w, **over) -> Grid:
    p = w.grid_params()
    p.update(over)
    return Grid(**p)


def species_from_workload(grid: Grid, parts: List[dict], extra_cap: float = 0.0):
    out = []
    for k, d in enumerate(parts):
        n = len(d["r"])
        out.append(grid.species(d, cap=int(n * (1.0 + extra_cap)) + 16, role=k + 1))
    return out
