"""MI355X (gfx950) hot path of the implicit energy- and charge-conserving EM
PIC/MCC method on an r-z grid: ctypes binding of ``libecpic.so``.

Argument marshalling only: every step of the path runs in the HIP kernels of
``csrc/``.  PyTorch supplies device memory and the stream.  Importing this
package never falls back to another implementation; when the library is
missing, :func:`lib` raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libecpic.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "ecpic.h")

ECPIC_FP64, ECPIC_MIXED = 0, 1
ECPIC_MODEL_EM, ECPIC_MODEL_ES = 0, 1
ECPIC_OPT_QUEUE_WAVES, ECPIC_OPT_NN_FORCE_FALLBACK, ECPIC_OPT_JFNK_KRYLOV = 0, 1, 2
ECPIC_SOLVER_PICARD, ECPIC_SOLVER_JFNK = 0, 1
_SOLVERS = {"picard": ECPIC_SOLVER_PICARD, "jfnk": ECPIC_SOLVER_JFNK}
ECPIC_OK, ECPIC_EINVAL, ECPIC_ENOMEM, ECPIC_EHIP, ECPIC_ENOTCONV = 0, -1, -2, -3, -4
ECPIC_EPUSH, ECPIC_ECAPACITY, ECPIC_ERANGE, ECPIC_ENOTIMPL = -5, -6, -7, -8
STATUS = {0: "ok", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENOTCONV", -5: "EPUSH",
          -6: "ECAPACITY", -7: "ERANGE", -8: "ENOTIMPL"}


class EcpicError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class GridDesc(C.Structure):
    _fields_ = [("nr", C.c_int32), ("nz", C.c_int32), ("R", C.c_double), ("L", C.c_double),
                ("xi_axis", C.c_double), ("dt", C.c_double), ("eps", C.c_double),
                ("mu", C.c_double), ("n_drive", C.c_int32), ("model", C.c_int32),
                ("drive_amp", C.c_double * 32), ("drive_freq", C.c_double * 32),
                ("drive_phase", C.c_double * 32), ("drive_t_end", C.c_double),
                ("blocking_cap", C.c_double), ("port_i", C.c_int32), ("port_eps", C.c_double)]


class SpeciesDesc(C.Structure):
    _fields_ = [("q", C.c_double), ("m", C.c_double), ("weight", C.c_double),
                ("capacity", C.c_int64), ("mobile", C.c_int32), ("sort_stride", C.c_int32)]


class MccDesc(C.Structure):
    _fields_ = [("enabled", C.c_int32), ("electron_sid", C.c_int32), ("ion_sid", C.c_int32),
                ("reserved", C.c_int32), ("n_gas", C.c_double), ("t_gas", C.c_double),
                ("m_gas", C.c_double), ("eps_max_ev", C.c_double), ("seed", C.c_uint64)]


class StepOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("fixed_iter", C.c_int32),
                ("sort_every", C.c_int32), ("use_nn", C.c_int32),
                ("check_conservation", C.c_int32), ("solver", C.c_int32),
                ("krylov", C.c_int32), ("eta", C.c_double)]


class FieldView(C.Structure):
    _fields_ = [("ur", C.c_void_p), ("uz", C.c_void_p), ("h", C.c_void_p),
                ("ur_prev", C.c_void_p), ("uz_prev", C.c_void_p), ("h_prev", C.c_void_p)]


class StepStats(C.Structure):
    _fields_ = [("iters", C.c_int32), ("converged", C.c_int32), ("used_nn", C.c_int32),
                ("nn_fallback", C.c_int32), ("residual", C.c_double * 64), ("ke", C.c_double * 4),
                ("we", C.c_double), ("wb", C.c_double), ("w_particles", C.c_double),
                ("w_field_io", C.c_double), ("w_drive", C.c_double), ("w_absorbed", C.c_double),
                ("w_coll", C.c_double), ("n_alive", C.c_int64 * 4), ("n_absorbed", C.c_int64 * 4),
                ("n_coll", C.c_int64 * 4), ("n_ionized", C.c_int64), ("n_substeps", C.c_int64),
                ("n_crossings", C.c_int64), ("n_errors", C.c_int64), ("n_over_range", C.c_int64),
                ("t", C.c_double), ("step", C.c_int64), ("continuity_max", C.c_double),
                ("gauss_max", C.c_double), ("q_max", C.c_double),
                ("newton_iters", C.c_int32), ("krylov_iters", C.c_int32),
                ("electrode_v", C.c_double), ("cap_charge", C.c_double), ("w_gen", C.c_double),
                ("port_v", C.c_double)]

    def as_dict(self) -> dict:
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if hasattr(v, "__len__") else v
        d["residual"] = d["residual"][: self.iters]
        return d


KERNEL_KINDS = ("push", "push_slow", "commit", "commit_slow", "field", "sort", "push_commit")


class Profile(C.Structure):
    _fields_ = [("launches", C.c_int64 * 7), ("ms", C.c_double * 7), ("bytes", C.c_double * 7),
                ("particles", C.c_int64 * 7), ("calls", C.c_int64 * 7),
                ("call_particles", C.c_int64 * 7)]

    def as_dict(self) -> dict:
        return {k: dict(launches=self.launches[i], ms=self.ms[i], bytes=self.bytes[i],
                        particles=self.particles[i], calls=self.calls[i],
                        call_particles=self.call_particles[i])
                for i, k in enumerate(KERNEL_KINDS)}


_lib = None
_vp, _dp, _fp = C.c_void_p, C.c_void_p, C.c_void_p


def lib() -> C.CDLL:
    """Load libecpic.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        st = C.c_int
        sig = {
            "ecpic_create": ([C.POINTER(GridDesc), C.c_int, _vp, C.POINTER(_vp)], st),
            "ecpic_destroy": ([_vp], st),
            "ecpic_workspace_size": ([_vp, C.POINTER(C.c_size_t)], st),
            "ecpic_bind_workspace": ([_vp, _vp, C.c_size_t], st),
            "ecpic_bind_fields": ([_vp, C.POINTER(FieldView)], st),
            "ecpic_add_species": ([_vp, C.POINTER(SpeciesDesc), C.POINTER(C.c_int32)], st),
            "ecpic_load_particles": ([_vp, C.c_int32] + [_dp] * 6 + [C.c_int64], st),
            "ecpic_read_particles": ([_vp, C.c_int32] + [_dp] * 6 + [C.c_int64,
                                                                      C.POINTER(C.c_int64)], st),
            "ecpic_set_fields": ([_vp] + [_dp] * 5 + [C.c_double, C.c_int64], st),
            "ecpic_get_fields": ([_vp, _dp, _dp, _dp], st),
            "ecpic_set_port_field": ([_vp, _dp], st),
            "ecpic_get_port_field": ([_vp, _dp], st),
            "ecpic_set_half_field": ([_vp, _dp, _dp], st),
            "ecpic_push_deposit": ([_vp, C.c_int32, _dp, _dp], st),
            "ecpic_field_solve": ([_vp] + [_dp] * 5 + [C.c_double] + [_dp] * 3, st),
            "ecpic_field_iterate": ([_vp, C.POINTER(C.c_double)], st),
            "ecpic_field_solve_noalloc": ([_vp] + [_dp] * 5 + [C.c_double] + [_dp] * 3, st),
            "ecpic_collide": ([_vp, C.POINTER(MccDesc), C.c_int64], st),
            "ecpic_set_mcc": ([_vp, C.POINTER(MccDesc)], st),
            "ecpic_step": ([_vp, C.POINTER(StepOpts), C.POINTER(StepStats)], st),
            "ecpic_run": ([_vp, C.POINTER(StepOpts), C.c_int32, C.POINTER(C.c_int32),
                           C.POINTER(StepStats)], st),
            "ecpic_sort": ([_vp], st),
            "ecpic_node_charge": ([_vp, _dp, _dp, _dp, _dp], st),
            "ecpic_diagnostics": ([_vp, C.POINTER(StepStats)], st),
            "ecpic_nn_param_count": ([], C.c_int64),
            "ecpic_nn_set_weights": ([_vp, _vp, C.POINTER(C.c_float)], st),
            "ecpic_nn_forward": ([_vp, _vp, _vp, _vp, C.c_int32], st),
            "ecpic_nn_grad": ([_vp, _vp, _vp, _vp, C.c_int32, _vp, C.POINTER(C.c_float)], st),
            "ecpic_nn_adam": ([_vp, _vp, _vp, _vp, _vp, C.c_float, C.c_int32], st),
            "ecpic_set_profiling": ([_vp, C.c_int32], st),
            "ecpic_set_option": ([_vp, C.c_int32, C.c_int64], st),
            "ecpic_set_profiling_every": ([_vp, C.c_int32], st),
            "ecpic_get_profile": ([_vp, C.POINTER(Profile)], st),
            "ecpic_last_error": ([_vp], C.c_char_p),
            "ecpic_status_string": ([C.c_int], C.c_char_p),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def header_symbols() -> list:
    """Names of the entry points declared in include/ecpic.h."""
    import re
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)  # drop comments
    return sorted(set(re.findall(r"\b(ecpic_[a-z0-9_]+)\s*\(", txt)))


def _ptr(t) -> Optional[int]:
    if t is None:
        return None
    return t.data_ptr()


class Context:
    """One grid + its species on the current HIP device and torch stream."""

    def __init__(self, nr, nz, R, L, xi_a, dt, eps, mu, drive_amp=(), drive_freq=(),
                 drive_phase=(), drive_t_end=0.0, precision: str = "fp64", device: str = "cuda",
                 model: str = "em", blocking_cap: float = 0.0, port_i: int = 0,
                 port_eps: float = 1.0):
        """The context allocates no device memory until its first device call;
        call :meth:`bind_workspace` after the last :meth:`add_species` to give
        it a torch-allocated region instead."""
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.nr, self.nz = nr, nz
        self.precision = precision
        g = GridDesc()
        g.nr, g.nz, g.R, g.L, g.xi_axis, g.dt, g.eps, g.mu = nr, nz, R, L, xi_a, dt, eps, mu
        g.n_drive = len(drive_amp)
        for k in range(len(drive_amp)):
            g.drive_amp[k] = drive_amp[k]
            g.drive_freq[k] = drive_freq[k]
            g.drive_phase[k] = drive_phase[k] if k < len(drive_phase) else 0.0
        g.drive_t_end = drive_t_end
        g.model = {"em": ECPIC_MODEL_EM, "es": ECPIC_MODEL_ES}[model]
        g.blocking_cap = blocking_cap
        g.port_i, g.port_eps = port_i, port_eps
        self.desc = g
        stream = torch.cuda.current_stream(self.device).cuda_stream
        h = _vp()
        self.L = lib()
        self._check(self.L.ecpic_create(C.byref(g), ECPIC_MIXED if precision == "mixed"
                                        else ECPIC_FP64, _vp(stream), C.byref(h)), None)
        self.h = h
        self.caps: Dict[int, int] = {}
        self.workspace = None
        self._bound_fields = None

    def _check(self, rc: int, h=None):
        if rc != 0:
            msg = self.L.ecpic_last_error(h if h is not None else getattr(self, "h", None))
            raise EcpicError(rc, (msg or b"").decode())
        return rc

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            self.torch.cuda.synchronize()
            self.L.ecpic_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- device memory owned by torch --
    def workspace_size(self) -> int:
        n = C.c_size_t()
        self._check(self.L.ecpic_workspace_size(self.h, C.byref(n)), self.h)
        return int(n.value)

    def bind_workspace(self, nbytes: Optional[int] = None):
        """Allocate the context's whole device region as one torch tensor and
        bind it (after the last add_species)."""
        t = self.torch
        n = self.workspace_size() if nbytes is None else int(nbytes)
        ws = t.empty(n + 256, dtype=t.uint8, device=self.device)
        off = (-ws.data_ptr()) % 256
        self._check(self.L.ecpic_bind_workspace(self.h, _vp(ws.data_ptr() + off), n), self.h)
        self.workspace = ws
        return ws

    def bind_fields(self, ur, uz, h, ur_prev, uz_prev, h_prev):
        """Keep u^n, u^{n-1} in these six torch FP64 device tensors (their
        contents become the state); None as ur unbinds."""
        if ur is None:
            self._check(self.L.ecpic_bind_fields(self.h, None), self.h)
            self._bound_fields = None
            return
        ts = (ur, uz, h, ur_prev, uz_prev, h_prev)
        for a in ts:
            assert a.is_cuda and a.dtype == self.torch.float64 and a.is_contiguous()
        assert ur.numel() == self.nr * (self.nz + 1) == ur_prev.numel()
        assert uz.numel() == (self.nr + 1) * self.nz == uz_prev.numel()
        assert h.numel() == self.nr * self.nz == h_prev.numel()
        v = FieldView(*[a.data_ptr() for a in ts])
        self._check(self.L.ecpic_bind_fields(self.h, C.byref(v)), self.h)
        self._bound_fields = ts

    # -- tensors --
    def _dev(self, a, dtype=None):
        t = self.torch
        if isinstance(a, np.ndarray):
            a = t.from_numpy(np.ascontiguousarray(a))
        return a.to(self.device, dtype=dtype).contiguous()

    def zeros_r(self):
        return self.torch.zeros(self.nr * (self.nz + 1), dtype=self.torch.float64,
                                device=self.device)

    def zeros_z(self):
        return self.torch.zeros((self.nr + 1) * self.nz, dtype=self.torch.float64,
                                device=self.device)

    def zeros_h(self):
        return self.torch.zeros(self.nr * self.nz, dtype=self.torch.float64, device=self.device)

    # -- species --
    def add_species(self, q, m, weight, capacity, mobile=True, sort_stride=0) -> int:
        d = SpeciesDesc(q, m, weight, int(capacity), int(bool(mobile)), int(sort_stride))
        sid = C.c_int32()
        self._check(self.L.ecpic_add_species(self.h, C.byref(d), C.byref(sid)), self.h)
        self.caps[sid.value] = int(capacity)
        return sid.value

    def load_particles(self, sid: int, r, z, vr, vt, vz, uid):
        f64 = self.torch.float64
        arrs = [self._dev(a, f64) for a in (r, z, vr, vt, vz)]
        u = uid if not isinstance(uid, np.ndarray) else uid.astype(np.int64)
        u = self._dev(u, self.torch.int64)
        self._keep = (arrs, u)
        self._check(self.L.ecpic_load_particles(self.h, sid, *[_ptr(a) for a in arrs], _ptr(u),
                                                len(arrs[0])), self.h)

    def read_particles(self, sid: int) -> dict:
        t = self.torch
        cap = self.caps[sid]
        outs = [t.empty(cap, dtype=t.float64, device=self.device) for _ in range(5)]
        uid = t.empty(cap, dtype=t.int64, device=self.device)
        n = C.c_int64()
        self._check(self.L.ecpic_read_particles(self.h, sid, *[_ptr(o) for o in outs], _ptr(uid),
                                                cap, C.byref(n)), self.h)
        n = n.value
        names = ("xi", "eta", "vr", "vt", "vz")
        d = {k: o[:n].cpu().numpy() for k, o in zip(names, outs)}
        d["uid"] = uid[:n].cpu().numpy().astype(np.uint64)
        return d

    # -- fields --
    def set_fields(self, ur, uz, h, ur_prev=None, uz_prev=None, t=0.0, step=0):
        f = self.torch.float64
        ts = [self._dev(a, f) if a is not None else None for a in (ur, uz, h, ur_prev, uz_prev)]
        self._check(self.L.ecpic_set_fields(self.h, *[_ptr(a) for a in ts], float(t), int(step)),
                    self.h)
        self.torch.cuda.synchronize()

    def get_fields(self):
        ur, uz, h = self.zeros_r(), self.zeros_z(), self.zeros_h()
        self._check(self.L.ecpic_get_fields(self.h, _ptr(ur), _ptr(uz), _ptr(h)), self.h)
        self.torch.cuda.synchronize()
        return ur.cpu().numpy(), uz.cpu().numpy(), h.cpu().numpy()

    def set_port_field(self, hb):
        """The TEM port's wall field H_b at t^n, [nr] (entries from port_i on)."""
        a = np.ascontiguousarray(hb, dtype=np.float64)
        assert a.size == self.nr
        self._check(self.L.ecpic_set_port_field(self.h, a.ctypes.data_as(_dp)), self.h)

    def get_port_field(self):
        out = np.zeros(self.nr)
        self._check(self.L.ecpic_get_port_field(self.h, out.ctypes.data_as(_dp)), self.h)
        return out

    def set_half_field(self, ur_h, uz_h):
        f = self.torch.float64
        a, b = self._dev(ur_h, f), self._dev(uz_h, f)
        self._check(self.L.ecpic_set_half_field(self.h, _ptr(a), _ptr(b)), self.h)
        self.torch.cuda.synchronize()

    def push_deposit(self, commit=False):
        Ir, Iz = self.zeros_r(), self.zeros_z()
        self._check(self.L.ecpic_push_deposit(self.h, int(commit), _ptr(Ir), _ptr(Iz)), self.h)
        self.torch.cuda.synchronize()
        return Ir.cpu().numpy(), Iz.cpu().numpy()

    def field_solve(self, ur0, uz0, h0, Ir, Iz, t):
        f = self.torch.float64
        ins = [self._dev(a, f) for a in (ur0, uz0, h0, Ir, Iz)]
        ur1, uz1, h1 = self.zeros_r(), self.zeros_z(), self.zeros_h()
        self._check(self.L.ecpic_field_solve(self.h, *[_ptr(a) for a in ins], float(t),
                                             _ptr(ur1), _ptr(uz1), _ptr(h1)), self.h)
        self.torch.cuda.synchronize()
        return ur1.cpu().numpy(), uz1.cpu().numpy(), h1.cpu().numpy()

    def field_solve_noalloc(self, ur0, uz0, h0, Ir, Iz, t, out=None):
        """ecpic_field_solve_noalloc on device tensors; out: (ur1, uz1, h1)
        device tensors to fill (allocated here when None).  Returns them."""
        f = self.torch.float64
        ins = [self._dev(a, f) for a in (ur0, uz0, h0, Ir, Iz)]
        outs = out if out is not None else (self.zeros_r(), self.zeros_z(), self.zeros_h())
        self._check(self.L.ecpic_field_solve_noalloc(self.h, *[_ptr(a) for a in ins], float(t),
                                                     *[_ptr(o) for o in outs]), self.h)
        return outs

    def field_iterate(self) -> float:
        r = C.c_double()
        self._check(self.L.ecpic_field_iterate(self.h, C.byref(r)), self.h)
        return r.value

    # -- collisions, step --
    @staticmethod
    def mcc_desc(mcc: Optional[dict]) -> MccDesc:
        if not mcc:
            return MccDesc()
        return MccDesc(1, mcc.get("electron_sid", 0), mcc.get("ion_sid", 1), 0, mcc["n_gas"],
                       mcc["T_gas"], mcc["m_gas"], mcc["eps_max_ev"], mcc["seed"])

    def set_mcc(self, mcc: Optional[dict]):
        d = self.mcc_desc(mcc)
        self._check(self.L.ecpic_set_mcc(self.h, C.byref(d)), self.h)

    def collide(self, mcc: dict, step: int):
        d = self.mcc_desc(mcc)
        self._check(self.L.ecpic_collide(self.h, C.byref(d), int(step)), self.h)

    def step(self, tol=1e-10, max_iter=50, fixed_iter=0, sort_every=0, use_nn=False,
             stats=True, check=True, conservation=False, solver="picard", krylov=10,
             eta=1e-4):
        o = StepOpts(tol, max_iter, fixed_iter, sort_every, int(use_nn), int(conservation),
                     _SOLVERS[solver], krylov, eta)
        if stats:
            s = StepStats()
            rc = self.L.ecpic_step(self.h, C.byref(o), C.byref(s))
            d = s.as_dict()
        else:
            rc = self.L.ecpic_step(self.h, C.byref(o), None)
            d = {}
        d["rc"] = rc
        if check and rc != 0:
            self._check(rc, self.h)
        return d

    def run(self, n_steps, tol=1e-10, max_iter=50, fixed_iter=0, sort_every=0, use_nn=False,
            stats=False, check=True, conservation=False, solver="picard", krylov=10,
            eta=1e-4):
        """n_steps implicit steps in the library (ecpic_run); returns the
        number done and, with stats, the last step's statistics."""
        o = StepOpts(tol, max_iter, fixed_iter, sort_every, int(use_nn), int(conservation),
                     _SOLVERS[solver], krylov, eta)
        done = C.c_int32(0)
        s = StepStats() if stats else None
        rc = self.L.ecpic_run(self.h, C.byref(o), int(n_steps), C.byref(done),
                              C.byref(s) if stats else None)
        d = s.as_dict() if stats else {}
        d["rc"], d["done"] = rc, done.value
        if check and rc != 0:
            self._check(rc, self.h)
        return d

    def sort(self):
        self._check(self.L.ecpic_sort(self.h), self.h)

    def node_charge(self):
        t = self.torch
        q = t.zeros((self.nr + 1) * (self.nz + 1), dtype=t.float64, device=self.device)
        b = t.zeros(self.nr + 1, dtype=t.float64, device=self.device)
        tp = t.zeros(self.nr + 1, dtype=t.float64, device=self.device)
        sd = t.zeros(self.nz + 1, dtype=t.float64, device=self.device)
        self._check(self.L.ecpic_node_charge(self.h, _ptr(q), _ptr(b), _ptr(tp), _ptr(sd)), self.h)
        t.cuda.synchronize()
        return q.cpu().numpy(), b.cpu().numpy(), tp.cpu().numpy(), sd.cpu().numpy()

    def set_option(self, option: int, value: int):
        self._check(self.L.ecpic_set_option(self.h, int(option), int(value)), self.h)

    def set_profiling(self, on: bool = True, kinds=None, every: int = 1):
        """Time launches with HIP events: every kind when `kinds` is None,
        else only the named ones (names of KERNEL_KINDS); only every
        `every`-th launch of a kind is timed, all are counted."""
        self._check(self.L.ecpic_set_profiling_every(self.h, int(every)), self.h)
        if not on:
            mask = 0
        elif kinds is None:
            mask = (1 << len(KERNEL_KINDS)) - 1
        else:
            mask = 0
            for k in kinds:
                mask |= 1 << KERNEL_KINDS.index(k)
        self._check(self.L.ecpic_set_profiling(self.h, mask), self.h)

    def profile(self) -> dict:
        p = Profile()
        self._check(self.L.ecpic_get_profile(self.h, C.byref(p)), self.h)
        return p.as_dict()

    # ---- learned initial guess (argument marshalling only) ----
    def nn_param_count(self) -> int:
        return int(self.L.ecpic_nn_param_count())

    def _f32(self, a):
        t = self.torch
        a = a if isinstance(a, t.Tensor) else t.as_tensor(np.asarray(a, dtype=np.float32))
        return a.to(device=self.device, dtype=t.float32).contiguous()

    def _bf16(self, a):
        t = self.torch
        a = a if isinstance(a, t.Tensor) else t.as_tensor(np.asarray(a, dtype=np.float32))
        if a.dtype != t.bfloat16:
            a = a.to(t.float32).to(t.bfloat16)
        return a.to(self.device).contiguous()

    def nn_set_weights(self, w, norm):
        """Install FP32 weights (canonical layout) and the 8 scales for
        step(use_nn=True); w=None uninstalls."""
        if w is None:
            self._check(self.L.ecpic_nn_set_weights(self.h, None, None), self.h)
            return
        wt = self._f32(w)
        nm = (C.c_float * 8)(*[float(v) for v in norm])
        self._check(self.L.ecpic_nn_set_weights(self.h, _ptr(wt), nm), self.h)
        self.torch.cuda.synchronize()

    def nn_forward(self, w, x):
        """x: [batch][6][nr+1][nz+1] (scaled); returns y [batch][2][nr+1][nz+1] FP32."""
        t = self.torch
        wt, xb = self._f32(w), self._bf16(x)
        b = xb.shape[0]
        y = t.empty((b, 2, self.nr + 1, self.nz + 1), dtype=t.float32, device=self.device)
        self._check(self.L.ecpic_nn_forward(self.h, _ptr(wt), _ptr(xb), _ptr(y), b), self.h)
        return y

    def nn_grad(self, w, x, target):
        """Loss and FP32 gradient of the mean squared error over the valid outputs."""
        t = self.torch
        wt, xb, tt = self._f32(w), self._bf16(x), self._f32(target)
        dw = t.empty(self.nn_param_count(), dtype=t.float32, device=self.device)
        loss = C.c_float()
        self._check(self.L.ecpic_nn_grad(self.h, _ptr(wt), _ptr(xb), _ptr(tt), xb.shape[0],
                                         _ptr(dw), C.byref(loss)), self.h)
        return dw, float(loss.value)

    def nn_adam(self, w, m, v, dw, lr, step):
        """In-place Adam step on device FP32 tensors w, m, v."""
        self._check(self.L.ecpic_nn_adam(self.h, _ptr(w), _ptr(m), _ptr(v), _ptr(dw),
                                         float(lr), int(step)), self.h)

    def diagnostics(self) -> dict:
        s = StepStats()
        self._check(self.L.ecpic_diagnostics(self.h, C.byref(s)), self.h)
        return s.as_dict()


def context_from_workload(w, precision="fp64", device="cuda", **over) -> Context:
    """A context for workload w (ecpic_inputs.Workload)."""
    p = w.grid_params()
    p.update(over)
    return Context(precision=precision, device=device, **p)


def load_workload_species(ctx: Context, parts, extra_cap: float = 0.0, mobile=(True, True),
                          workspace: bool = False, sort_strides=()):
    """Add the species of `parts` and load them; with workspace, the
    context's device region is one torch tensor bound before the load.
    sort_strides: per species, at which of the steps' sorts it is sorted
    (ecpic_species_desc.sort_stride; missing entries 0, every sort)."""
    sids = []
    for k, d in enumerate(parts):
        n = len(d["r"])
        cap = int(n * (1.0 + extra_cap)) + 256
        sid = ctx.add_species(d["q"], d["m"], d["w"], cap, mobile[k] if k < len(mobile) else True,
                              sort_strides[k] if k < len(sort_strides) else 0)
        sids.append(sid)
    if workspace:
        ctx.bind_workspace()
    for sid, d in zip(sids, parts):
        ctx.load_particles(sid, d["r"], d["z"], d["vr"], d["vt"], d["vz"], d["uid"])
    return sids
