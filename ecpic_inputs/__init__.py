"""Seeded synthetic inputs for the r-z PIC/MCC workloads.

This module holds configuration data and random initial conditions only: it
contains none of the method's arithmetic (no mapping, field, push, deposit or
collision code).  Both the CPU oracle and the HIP library consume what it
produces: particle positions in physical (r, z) coordinates and velocities in
m/s; each side converts positions to its own logical coordinates.

The workloads stand in for the paper's Testbench-B discharge (Sec. 2.1: a
cylindrical argon CCP, 3 cm gap, VHF drive, a few Pa), whose geometry files,
cross-section data and measurements are not available.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

# CODATA 2018 (exact SI values where defined)
QE = 1.602176634e-19
ME = 9.1093837015e-31
EPS0 = 8.8541878128e-12
MU0 = 1.25663706212e-6
KB = 1.380649e-23
AMU = 1.66053906660e-27
M_AR = 39.948 * AMU
C_LIGHT = 299792458.0
CHI01 = 2.404825557695773  # first zero of J0 (tabulated constant)


@dataclasses.dataclass
class Workload:
    name: str
    nr: int
    nz: int
    R: float
    L: float
    xi_a: float = 2.0
    dt: float = 1e-11
    drive_amp: tuple = ()
    drive_freq: tuple = ()
    drive_phase: tuple = ()
    drive_t_end: float = 0.0  # > 0: the drive is a burst that ends then
    n0: float = 1e15
    profile: str = "uniform"  # "uniform", "j0sin" or "slab"
    gap: float = 0.0  # slab: vacuum gap left at each electrode [m]
    n_rings: int = 0  # slab: lattice rings, equally spaced in r^2
    n_layers: int = 0  # slab: lattice layers, equally spaced in z
    ppc: int = 16  # macro-particles per cell per species
    Te_eV: float = 3.0
    Ti_eV: float = 0.026
    steps: int = 10
    tol: float = 1e-10
    pressure_pa: float = 0.0  # 0 = no collisions
    T_gas: float = 300.0
    eps_max_ev: float = 1000.0
    seed: int = 1
    port_i: int = 0  # > 0: the drive enters through a TEM port over r-edges port_i.. of the bottom wall
    port_eps: float = 1.0  # relative permittivity of the port's line

    @property
    def n_per_species(self) -> int:
        return self.ppc * self.nr * self.nz

    @property
    def n_gas(self) -> float:
        return self.pressure_pa / (KB * self.T_gas)

    def grid_params(self) -> dict:
        return dict(nr=self.nr, nz=self.nz, R=self.R, L=self.L, xi_a=self.xi_a,
                    dt=self.dt, eps=EPS0, mu=MU0,
                    drive_amp=tuple(self.drive_amp), drive_freq=tuple(self.drive_freq),
                    drive_phase=tuple(self.drive_phase) if self.drive_phase
                    else tuple(0.0 for _ in self.drive_amp),
                    drive_t_end=self.drive_t_end, port_i=self.port_i, port_eps=self.port_eps)

    def mcc_params(self) -> Optional[dict]:
        if self.pressure_pa <= 0:
            return None
        return dict(n_gas=self.n_gas, T_gas=self.T_gas, m_gas=M_AR,
                    eps_max_ev=self.eps_max_ev, seed=self.seed,
                    electron_sid=0, ion_sid=1)


WORKLOADS: Dict[str, Workload] = {
    # 32x32 cylinder, two Maxwellian species, zero fields, no drive, no MCC
    "c1": Workload("c1", 32, 32, 0.02, 0.02, n0=1e15, ppc=16, steps=10, tol=1e-10, seed=1),
    # VHF CCP slab, 256x128, 100 MHz 200 V, J0*sin density, MCC
    "c2": Workload("c2", 256, 128, 0.15, 0.03, n0=1e16, profile="j0sin", ppc=64,
                   drive_amp=(200.0,), drive_freq=(100e6,), steps=2000, tol=1e-10,
                   pressure_pa=5.0, seed=2),
    # mixed-precision scale-up, 512x256, 128 ppc
    "c3": Workload("c3", 512, 256, 0.25, 0.03, n0=1e16, profile="j0sin", ppc=128,
                   drive_amp=(200.0,), drive_freq=(100e6,), steps=5, tol=1e-10,
                   pressure_pa=5.0, seed=3),
    # largest single-GPU case, 1024x512, dual frequency
    "c5": Workload("c5", 1024, 512, 0.3, 0.03, n0=1e16, profile="j0sin", ppc=256,
                   drive_amp=(200.0, 200.0), drive_freq=(60e6, 13.56e6), steps=1000,
                   tol=1e-10, pressure_pa=5.0, seed=5),
}


def sawtooth_drive(amp: float, n_harm: int, freq: float):
    """Amplitudes and frequencies of the sawtooth-like excitation
    A sum_{n<=N} sin(2 pi n f t) / n (Sec. 3.1)."""
    return (tuple(amp / n for n in range(1, n_harm + 1)),
            tuple(n * freq for n in range(1, n_harm + 1)))


_SAW_AMP, _SAW_FREQ = sawtooth_drive(1.0, 20, 106e6)

# Surface-mode cavity (Sec. 3.1): a uniform 1e16 m^-3 plasma slab with
# immobile ions and cold electrons between two 1.8 mm vacuum gaps, excited by
# one period of the 106 MHz, 20-harmonic, 1 V sawtooth on the drive gap.
# The ring count puts at least two rings into each cell next to the axis.
WORKLOADS["slab_small"] = Workload(
    "slab_small", 24, 50, 0.15, 0.03, dt=5e-11, drive_amp=_SAW_AMP, drive_freq=_SAW_FREQ,
    drive_t_end=1.0 / 106e6, n0=1e16, profile="slab", gap=1.8e-3, n_rings=169, n_layers=44,
    Te_eV=0.0, Ti_eV=0.0, steps=3000, tol=1e-10, seed=11)
WORKLOADS["slab"] = Workload(
    "slab", 64, 100, 0.15, 0.03, dt=2e-11, drive_amp=_SAW_AMP, drive_freq=_SAW_FREQ,
    drive_t_end=1.0 / 106e6, n0=1e16, profile="slab", gap=1.8e-3, n_rings=1089, n_layers=176,
    Te_eV=0.0, Ti_eV=0.0, steps=15000, tol=1e-10, seed=12)


def workload(name: str, **over) -> Workload:
    w = dataclasses.replace(WORKLOADS[name])
    for k, v in over.items():
        setattr(w, k, v)
    return w


def _j0(x: np.ndarray) -> np.ndarray:
    from scipy.special import j0
    return j0(x)


def _total_particles_phys(w: Workload) -> float:
    """Physical number of electrons in the domain (integral of the density)."""
    if w.profile == "uniform":
        return w.n0 * math.pi * w.R ** 2 * w.L
    from scipy.integrate import quad
    from scipy.special import j0
    k = 2.405 / w.R
    ir, _ = quad(lambda r: max(j0(k * r), 0.0) * 2 * math.pi * r, 0.0, w.R, limit=200)
    iz = 2.0 * w.L / math.pi
    return w.n0 * ir * iz


def _positions(w: Workload, n: int, rng: np.random.Generator):
    """n positions, uniform in volume (r = R sqrt(U)), shaped by the profile."""
    if w.profile == "uniform":
        r = w.R * np.sqrt(rng.random(n))
        z = w.L * rng.random(n)
        return r, z
    k = 2.405 / w.R
    rs: List[np.ndarray] = []
    zs: List[np.ndarray] = []
    got = 0
    while got < n:
        m = int((n - got) * 2.2) + 1024
        r = w.R * np.sqrt(rng.random(m))
        z = w.L * rng.random(m)
        dens = np.clip(_j0(k * r), 0.0, None) * np.sin(math.pi * z / w.L)
        keep = rng.random(m) < dens
        rs.append(r[keep])
        zs.append(z[keep])
        got += int(keep.sum())
    return np.concatenate(rs)[:n], np.concatenate(zs)[:n]


def _interior(x: np.ndarray, hi: float) -> np.ndarray:
    """Keep loaded positions strictly inside (0, hi): a draw of exactly 0 is
    moved to the smallest positive double."""
    return np.clip(x, np.nextafter(0.0, 1.0), np.nextafter(hi, 0.0))


def make_particles(w: Workload, seed: Optional[int] = None, n: Optional[int] = None):
    """Electrons and Ar+ ions, pair-loaded (each ion at its electron's
    position, so the initial node charge is zero), Maxwellian velocities.

    Returns a list of two dicts (electrons, ions) with keys
    q, m, w, r, z, vr, vt, vz, uid.
    """
    seed = w.seed if seed is None else seed
    n = w.n_per_species if n is None else n
    rng = np.random.Generator(np.random.PCG64(seed))
    r, z = _positions(w, n, rng)
    r = _interior(r, w.R)
    z = _interior(z, w.L)
    weight = _total_particles_phys(w) / n
    out = []
    for q, m, T in ((-QE, ME, w.Te_eV), (QE, M_AR, w.Ti_eV)):
        sig = math.sqrt(T * QE / m)
        v = rng.standard_normal((3, n)) * sig
        out.append(dict(q=q, m=m, w=weight, r=r.copy(), z=z.copy(),
                        vr=v[0].copy(), vt=v[1].copy(), vz=v[2].copy(),
                        uid=np.arange(n, dtype=np.uint64)))
    return out


def cold_mode_particles(w: Workload, n: int, v0: float, seed: int = 7):
    """Cold electrons on a quiet (stratified) start with velocity v0 grad(psi),
    psi = J0(chi01 r / R) sin(pi z / L), plus immobile ions at the same
    positions.  Used for the cold-plasma oscillation check."""
    from scipy.special import j1
    rng = np.random.Generator(np.random.PCG64(seed))
    m_side = int(round(math.sqrt(n)))
    n = m_side * m_side
    a = (np.arange(m_side) + 0.5) / m_side
    ur, uz = np.meshgrid(a, a, indexing="ij")
    ur = ur.ravel() + (rng.random(n) - 0.5) * 1e-9
    uz = uz.ravel() + (rng.random(n) - 0.5) * 1e-9
    r = w.R * np.sqrt(ur)
    z = w.L * uz
    k = CHI01 / w.R
    kz = math.pi / w.L
    # grad psi = (-k J1(k r) sin(kz z), kz J0(k r) cos(kz z))
    vr = v0 * (-k * j1(k * r) * np.sin(kz * z))
    vz = v0 * (kz * _j0(k * r) * np.cos(kz * z))
    weight = w.n0 * math.pi * w.R ** 2 * w.L / n
    e = dict(q=-QE, m=ME, w=weight, r=r, z=z, vr=vr, vt=np.zeros(n), vz=vz,
             uid=np.arange(n, dtype=np.uint64))
    i = dict(q=QE, m=M_AR, w=weight, r=r.copy(), z=z.copy(), vr=np.zeros(n),
             vt=np.zeros(n), vz=np.zeros(n), uid=np.arange(n, dtype=np.uint64))
    return [e, i]


def slab_particles(w: Workload):
    """Quiet start for the surface-mode cavity: electrons on a lattice of
    n_rings rings equally spaced in r^2 (so equal volume per ring) times
    n_layers layers equally spaced in z over [gap, L - gap], each with an
    immobile ion at the same position (zero initial charge).  Velocities are
    drawn at Te_eV / Ti_eV (zero: a cold plasma).  Returns [electrons, ions]
    like make_particles; the ions are meant to be added with mobile = 0."""
    rng = np.random.Generator(np.random.PCG64(w.seed))
    u = (np.arange(w.n_rings) + 0.5) / w.n_rings
    zl = w.gap + (w.L - 2.0 * w.gap) * (np.arange(w.n_layers) + 0.5) / w.n_layers
    uu, zz = np.meshgrid(u, zl, indexing="ij")
    r = w.R * np.sqrt(uu.ravel())
    z = zz.ravel()
    n = r.size
    weight = w.n0 * math.pi * w.R ** 2 * (w.L - 2.0 * w.gap) / n
    out = []
    for q, m, T in ((-QE, ME, w.Te_eV), (QE, M_AR, w.Ti_eV)):
        sig = math.sqrt(T * QE / m)
        v = rng.standard_normal((3, n)) * sig
        out.append(dict(q=q, m=m, w=weight, r=r.copy(), z=z.copy(),
                        vr=v[0].copy(), vt=v[1].copy(), vz=v[2].copy(),
                        uid=np.arange(n, dtype=np.uint64)))
    return out


def make_particles_device(w: Workload, device="cuda", seed: Optional[int] = None,
                          n: Optional[int] = None):
    """The make_particles recipe drawn on the GPU with torch's seeded
    generator, for the workloads too large to draw on the host (c5: 268M
    particles): the same distributions (uniform-in-volume proposals shaped
    by the profile by rejection, pair loading, Maxwellians, 0-based ids) from
    another random stream.  Returns the two species as dicts of device
    tensors (FP64; ids int64)."""
    import torch
    seed = w.seed if seed is None else seed
    n = w.n_per_species if n is None else n
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    f64 = torch.float64
    k = 2.405 / w.R
    rs, zs, got = [], [], 0
    while got < n:
        m = int((n - got) * (1.0 if w.profile == "uniform" else 2.2)) + 1024
        r = w.R * torch.sqrt(torch.rand(m, generator=gen, device=device, dtype=f64))
        z = w.L * torch.rand(m, generator=gen, device=device, dtype=f64)
        if w.profile != "uniform":
            dens = torch.clamp(torch.special.bessel_j0(k * r), min=0.0) * torch.sin(math.pi * z / w.L)
            keep = torch.rand(m, generator=gen, device=device, dtype=f64) < dens
            r, z = r[keep], z[keep]
            del dens, keep
        rs.append(r)
        zs.append(z)
        got += int(r.numel())
    r = torch.cat(rs)[:n].clone()
    z = torch.cat(zs)[:n].clone()
    del rs, zs
    # strictly inside (0, R) x (0, L)
    r.clamp_(min=float(np.nextafter(0.0, 1.0)), max=float(np.nextafter(w.R, 0.0)))
    z.clamp_(min=float(np.nextafter(0.0, 1.0)), max=float(np.nextafter(w.L, 0.0)))
    weight = _total_particles_phys(w) / n
    out = []
    for q, m_, T in ((-QE, ME, w.Te_eV), (QE, M_AR, w.Ti_eV)):
        sig = math.sqrt(T * QE / m_)
        v = torch.randn((3, n), generator=gen, device=device, dtype=f64) * sig
        out.append(dict(q=q, m=m_, w=weight, r=r if not out else r.clone(),
                        z=z if not out else z.clone(), vr=v[0].clone(), vt=v[1].clone(),
                        vz=v[2].clone(), uid=torch.arange(n, device=device, dtype=torch.int64)))
        del v
    return out
