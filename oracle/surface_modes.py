"""Surface-mode analysis for the dispersion check of Sec. 3.1 (test
infrastructure only: imported by the tests, never by the library).

What it holds:

* the analytic dispersion relations of the two surface-mode families of a
  uniform cold plasma slab between two vacuum sheaths and two metal plates:
  the electromagnetic pair of Sec. 3.1, Eq. (9), and their electrostatic
  (c -> infinity) limit, Eq. (10);
* the Fourier-Bessel projection of Appendix A (coefficient c_m of
  F_m(r) = J_alpha(chi_{alpha,m} r / R));
* the Fourier-in-time peak pick used on a projected time series.

Notation follows Sec. 3.1: s is the sheath (vacuum gap) width, l the half
gap between the plates, d = l - s the plasma half-width, k the radial wave
number, eps_p = 1 - w_pe^2 / w^2 the relative plasma permittivity.  The paper
prints the attenuation constants with w_pe where the vacuum and plasma wave
equations give w: this module takes alpha^2 = k^2 - w^2/c^2 in the sheath and
beta^2 = k^2 - eps_p w^2/c^2 in the plasma (the forms whose c -> infinity
limit is Eq. (10), and which the long-wavelength limit below reproduces).

Eq. (9), multiplied through, is used in a form that stays real when alpha^2
or beta^2 is negative:

    symmetric:      T(beta^2, d) = -eps_p T(alpha^2, s)
    antisymmetric:  K(beta^2, d) = -eps_p T(alpha^2, s)

with T(x^2, w) = x tanh(x w) and K(x^2, w) = x coth(x w), both even in x
(x = i a gives -a tan(a w) and a cot(a w)).  "Symmetric" is the family whose
axial field is even about the mid-plane (equal sheath voltages, the coth(beta d)
relation), "antisymmetric" the odd one.
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np
from scipy.optimize import brentq
from scipy.special import jn_zeros, jv

# CODATA 2018
QE = 1.602176634e-19
ME = 9.1093837015e-31
EPS0 = 8.8541878128e-12
C0 = 299792458.0


def omega_pe(n0: float) -> float:
    """Electron plasma frequency [rad/s] at density n0 [m^-3]."""
    return math.sqrt(n0 * QE * QE / (EPS0 * ME))


def _t(x2: float, w: float) -> float:
    if x2 >= 0.0:
        x = math.sqrt(x2)
        return x * math.tanh(x * w)
    a = math.sqrt(-x2)
    return -a * math.tan(a * w)


def _k(x2: float, w: float) -> float:
    if x2 > 0.0:
        x = math.sqrt(x2)
        return x / math.tanh(x * w)
    if x2 == 0.0:
        return 1.0 / w
    a = math.sqrt(-x2)
    return a / math.tan(a * w)


def em_residual(w: float, k: float, n0: float, s: float, l: float, c: float,
                family: str) -> float:
    """Left minus right side of Eq. (9) in the real form above."""
    wpe = omega_pe(n0)
    d = l - s
    ep = 1.0 - wpe * wpe / (w * w)
    a2 = k * k - w * w / (c * c)
    b2 = k * k - ep * w * w / (c * c)
    lhs = _t(b2, d) if family == "symmetric" else _k(b2, d)
    return lhs + ep * _t(a2, s)


def em_frequency(k: float, n0: float, s: float, l: float, c: float = C0,
                 family: str = "symmetric") -> float:
    """The surface-mode root w(k) of Eq. (9) below w_pe [rad/s].

    The residual is scanned on a logarithmic grid over (1e-6, 1) w_pe and the
    sign change refined by Brent's method; exactly one root must exist."""
    if family not in ("symmetric", "antisymmetric"):
        raise ValueError(family)
    wpe = omega_pe(n0)
    grid = wpe * np.logspace(-6.0, math.log10(1.0 - 1e-12), 4001)
    f = np.array([em_residual(w, k, n0, s, l, c, family) for w in grid])
    idx = np.nonzero(np.sign(f[:-1]) * np.sign(f[1:]) < 0)[0]
    if len(idx) != 1:
        raise ValueError(f"{len(idx)} sign changes of the {family} relation at k={k}")
    i = int(idx[0])
    return brentq(em_residual, grid[i], grid[i + 1], args=(k, n0, s, l, c, family),
                  xtol=1e-12 * wpe, rtol=1e-14)


def es_frequency(k: float, n0: float, s: float, l: float,
                 family: str = "symmetric") -> float:
    """Eq. (10): the electrostatic surface-mode frequency [rad/s]."""
    wpe = omega_pe(n0)
    d = l - s
    cs = 1.0 / math.tanh(k * s)
    if family == "symmetric":
        cd = 1.0 / math.tanh(k * d)
        return wpe * math.sqrt(cd / (cs + cd))
    if family == "antisymmetric":
        td = math.tanh(k * d)
        return wpe * math.sqrt(td / (cs + td))
    raise ValueError(family)


def psr_frequency(n0: float, s: float, l: float) -> float:
    """Plasma series resonance w_pe sqrt(s / l), the k -> 0 cut-off of the
    electrostatic symmetric branch (Sec. 3.1)."""
    return omega_pe(n0) * math.sqrt(s / l)


def bessel_zeros(alpha: int, m: int) -> np.ndarray:
    """chi_{alpha,1..m}: the first m positive zeros of J_alpha."""
    return jn_zeros(alpha, m)


def fourier_bessel(f: np.ndarray, r: np.ndarray, R: float, m: int, alpha: int = 0) -> np.ndarray:
    """Appendix A: c_m = int_0^R r f F_m dr / int_0^R r F_m^2 dr with
    F_m = J_alpha(chi_{alpha,m} r / R), both integrals by the trapezoid rule
    over the sample radii r (ascending, r[0] = 0, r[-1] = R).  f has the
    radius as its last axis; the result drops that axis."""
    r = np.asarray(r, dtype=np.float64)
    chi = bessel_zeros(alpha, m)[m - 1]
    F = jv(alpha, chi * r / R)
    dr = np.diff(r)

    def trap(y):
        return ((y[..., :-1] + y[..., 1:]) * dr).sum(-1) / 2.0

    return trap(np.asarray(f) * (r * F)) / trap(r * F * F)


def spectrum(x: np.ndarray, dt: float, pad: int = 1 << 18):
    """Magnitude of the Hann-windowed, zero-padded FFT of the mean-free
    series x sampled every dt; returns (frequency [Hz], magnitude)."""
    x = np.asarray(x, dtype=np.float64)
    x = x - x.mean()
    n = max(pad, 1 << int(math.ceil(math.log2(len(x)))))
    mag = np.abs(np.fft.rfft(x * np.hanning(len(x)), n))
    return np.fft.rfftfreq(n, dt), mag


def peak_frequency(x: np.ndarray, dt: float, f_lo: float, f_hi: float) -> float:
    """Frequency [Hz] of the largest spectral line of x in [f_lo, f_hi]."""
    fr, mag = spectrum(x, dt)
    sel = (fr >= f_lo) & (fr <= f_hi)
    return float(fr[sel][np.argmax(mag[sel])])


def mode_series(bottom: np.ndarray, top: np.ndarray, r: Sequence[float], R: float, m: int):
    """Fourier-Bessel (alpha = 0) coefficient m over time of the even and the
    odd combination of E_z sampled at the same distance from the bottom and
    the top plate: (symmetric, antisymmetric) series."""
    b = np.asarray(bottom)
    t = np.asarray(top)
    return (fourier_bessel((b + t) / 2.0, r, R, m), fourier_bessel((b - t) / 2.0, r, R, m))
