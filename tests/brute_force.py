"""Brute-force solution of the coupled implicit step for a tiny case.

The discrete equations of Sec. 2.1 are written here directly in residual form
-- Faraday and Ampere (Eq. (2)) with mid-point centring on the Yee mesh, the
particle equations (Eq. (4)) at the mid-point, and the current of Eq. (3)
with m = 1 -- and solved all together by Newton's method with a dense
finite-difference Jacobian.  No elimination of the electric field, no Picard
iteration and no fixed point: an independent route to the same discrete
solution, for particles that stay in their cell during the step.
"""
from __future__ import annotations

import math

import numpy as np


class TinyCase:
    def __init__(self, nr, nz, R, L, xi_a, dt, eps, mu):
        self.nr, self.nz, self.R, self.L, self.xi_a = nr, nz, R, L, xi_a
        self.dt, self.eps, self.mu = dt, eps, mu
        self.s = R / (nr + xi_a)
        self.dz = L / nz
        self.rho = np.array([self.r(i + 0.5) for i in range(nr)])
        rn = np.array([self.r(i) for i in range(nr + 1)])
        self.ell = rn[1:] - rn[:-1]
        self.Ac = self.ell * self.dz
        self.Ar = 2 * math.pi * self.rho * self.dz
        rm = np.concatenate([[0.0], self.rho[:-1]])
        self.Az = math.pi * (self.rho ** 2 - rm ** 2)

    def r(self, xi):
        xa, s = self.xi_a, self.s
        return 2 * s * math.sqrt(xi * xa) if xi < xa else s * (xi + xa)

    def jr(self, xi):
        xa, s = self.xi_a, self.s
        return s * math.sqrt(xa / xi) if xi < xa else s

    # unknown layout: ur interior [nr][nz-1], uz interior [nr][nz], h [nr][nz],
    # then 5 per particle
    def split(self, X, npart):
        nr, nz = self.nr, self.nz
        a = nr * (nz - 1)
        b = a + nr * nz
        c = b + nr * nz
        ur = np.zeros((nr, nz + 1))
        ur[:, 1:nz] = X[:a].reshape(nr, nz - 1)
        uz = np.zeros((nr + 1, nz))
        uz[:nr] = X[a:b].reshape(nr, nz)
        h = X[b:c].reshape(nr, nz)
        P = X[c:].reshape(npart, 5)
        return ur, uz, h, P

    def residual(self, X, ur0, uz0, h0, parts):
        nr, nz, dt = self.nr, self.nz, self.dt
        ur1, uz1, h1, P1 = self.split(X, len(parts))
        urh, uzh, hh = 0.5 * (ur0 + ur1), 0.5 * (uz0 + uz1), 0.5 * (h0 + h1)
        Ir = np.zeros((nr, nz + 1))
        Iz = np.zeros((nr + 1, nz))
        res_p = []
        for (q, m, w, x0), x1 in zip(parts, P1):
            xi0, et0, vr0, vt0, vz0 = x0
            xi1, et1, vr1, vt1, vz1 = x1
            i, j = int(math.floor(xi0)), int(math.floor(et0))
            xb, eb = 0.5 * (xi0 + xi1), 0.5 * (et0 + et1)
            vrb, vtb, vzb = 0.5 * (vr0 + vr1), 0.5 * (vt0 + vt1), 0.5 * (vz0 + vz1)
            a, b = xb - i, eb - j
            Er = ((1 - b) * urh[i, j] + b * urh[i, j + 1]) / self.jr(xb)
            Ez = ((1 - a) * uzh[i, j] + a * uzh[i + 1, j]) / self.dz
            rb = self.r(xb)
            res_p += [(xi1 - xi0) / dt - vrb / self.jr(xb),
                      (et1 - et0) / dt - vzb / self.dz,
                      (vr1 - vr0) / dt - (q / m) * Er - vtb * vtb / rb,
                      (vt1 - vt0) / dt + vrb * vtb / rb,
                      (vz1 - vz0) / dt - (q / m) * Ez]
            c = q * w / dt
            Ir[i, j] += c * (xi1 - xi0) * (1 - b)
            Ir[i, j + 1] += c * (xi1 - xi0) * b
            Iz[i, j] += c * (et1 - et0) * (1 - a)
            Iz[i + 1, j] += c * (et1 - et0) * a
        far = np.zeros((nr, nz))
        for i in range(nr):
            for j in range(nz):
                far[i, j] = (self.mu * self.Ac[i] * (h1[i, j] - h0[i, j]) / dt
                             - (uzh[i + 1, j] - uzh[i, j] - urh[i, j + 1] + urh[i, j]))
        amp_r = np.zeros((nr, nz - 1))
        for i in range(nr):
            for j in range(1, nz):
                amp_r[i, j - 1] = (self.eps * self.Ar[i] / self.ell[i] * (ur1[i, j] - ur0[i, j]) / dt
                                   + 2 * math.pi * self.rho[i] * (hh[i, j] - hh[i, j - 1]) + Ir[i, j])
        amp_z = np.zeros((nr, nz))
        for i in range(nr):
            for j in range(nz):
                circ = 2 * math.pi * self.rho[i] * hh[i, j]
                if i > 0:
                    circ -= 2 * math.pi * self.rho[i - 1] * hh[i - 1, j]
                amp_z[i, j] = self.eps * self.Az[i] / self.dz * (uz1[i, j] - uz0[i, j]) / dt - circ + Iz[i, j]
        return np.concatenate([amp_r.ravel(), amp_z.ravel(), far.ravel(), np.array(res_p)])

    def solve(self, ur0, uz0, h0, parts, iters=30):
        nr, nz = self.nr, self.nz
        X = np.concatenate([ur0[:, 1:nz].ravel(), uz0[:nr].ravel(), h0.ravel(),
                            np.array([p[3] for p in parts]).ravel()])
        nf = nr * (nz - 1) + 2 * nr * nz
        scale = np.ones_like(X)
        scale[: nf - nr * nz] = max(np.abs(X[: nf - nr * nz]).max(), 1.0)
        scale[nf - nr * nz: nf] = max(np.abs(X[nf - nr * nz: nf]).max(), 1e-3)
        for k, p in enumerate(parts):
            vs = max(abs(p[3][2]), abs(p[3][3]), abs(p[3][4]), 1.0)
            scale[nf + 5 * k: nf + 5 * k + 5] = [1.0, 1.0, vs, vs, vs]
        for it in range(iters):
            F = self.residual(X, ur0, uz0, h0, parts)
            J = np.zeros((len(F), len(X)))
            for k in range(len(X)):
                d = 1e-6 * scale[k]
                Xp, Xm = X.copy(), X.copy()
                Xp[k] += d
                Xm[k] -= d
                J[:, k] = (self.residual(Xp, ur0, uz0, h0, parts) -
                           self.residual(Xm, ur0, uz0, h0, parts)) / (2 * d)
            dX = np.linalg.solve(J, -F)
            X = X + dX
            if np.all(np.abs(dX) <= 1e-15 * scale):
                break
        return self.split(X, len(parts))
