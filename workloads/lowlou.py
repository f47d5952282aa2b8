"""Low & Lou (1990) axisymmetric nonlinear force-free field, used as an exact solution.

This module only builds inputs and the exact reference field for checking; it contains none of the
DBIE arithmetic. The paper validates DBIE against this family of fields (Section 2.2, the benchmark
discussion around Table 1).

Construction (standard Low & Lou form, re-derived here):
  A(r, theta) = P(mu) / r^n,  mu = cos(theta),  Q(A) = a * A^(1 + 1/n)
  (1 - mu^2) P'' + n (n + 1) P + a^2 (1 + 1/n) P^(1 + 2/n) = 0,  P(-1) = P(1) = 0,  P'(-1) = P'(-1)_norm
  B_r = -P' / r^(n+2),  B_theta = n P / (r^(n+2) sin theta),  B_phi = a P |P|^(1/n) / (r^(n+2) sin theta)
The eigenvalue a^2 is found by shooting from both singular end points (regular series start) and
matching P, P' at mu = 0. m indexes the eigenvalues above a^2 = 0 in increasing order (m = 0 is the
linear profile a = 0). For integer n the a = 0 profile, (1 - mu^2) dP_n/dmu up to scale, already has
n - 1 interior zeros and each further eigenvalue adds one, so P_{n,m} has n - 1 + m interior zeros
(for n = 1 that is m, the usual count).
The field is placed in a frame tilted by Phi about the y axis, with the source a depth l below z = 0:
  X = x cos Phi - (z + l) sin Phi,  Y = y,  Z = x sin Phi + (z + l) cos Phi.
"""
from __future__ import annotations

import numpy as np
from scipy.integrate import solve_ivp
from scipy.optimize import brentq, fsolve


class LowLou:
    def __init__(self, n: int = 1, m: int = 1, l: float = 0.3, Phi: float = np.pi / 4,
                 dP_minus1: float = 10.0):
        self.n = int(n)
        self.m = int(m)
        self.l = float(l)
        self.Phi = float(Phi)
        self.dP = float(dP_minus1)
        self.a2, self._slope_plus = self._eigen()
        self.a = float(np.sqrt(self.a2))
        self._build_profile()

    # -- ODE ---------------------------------------------------------------------------------
    def _rhs(self, mu, y, a2):
        n = self.n
        P, Pp = y
        sp = np.sign(P) * np.abs(P) ** (1.0 + 2.0 / n)
        return [Pp, -(n * (n + 1) * P + a2 * (1.0 + 1.0 / n) * sp) / (1.0 - mu * mu)]

    def _start(self, slope, sgn, eps):
        # Near an end point, with s the distance to it, P = slope*s + d*s^2 and d = -n(n+1)slope/4
        d = -self.n * (self.n + 1) * slope / 4.0
        mu0 = sgn * (1.0 - eps)
        P0 = slope * eps + d * eps * eps
        Pp0 = -sgn * (slope + 2.0 * d * eps)
        return mu0, [P0, Pp0]

    def _side(self, a2, slope, sgn, eps, dense=False):
        mu0, y0 = self._start(slope, sgn, eps)
        return solve_ivp(self._rhs, (mu0, 0.0), y0, args=(a2,), rtol=1e-13, atol=1e-15,
                         method="DOP853", dense_output=dense)

    def _end_value(self, a2, eps=1e-6):
        mu0, y0 = self._start(self.dP, -1, eps)
        return solve_ivp(self._rhs, (mu0, 1.0 - eps), y0, args=(a2,), rtol=1e-11, atol=1e-13,
                         method="DOP853").y[0, -1]

    def _eigen(self, eps=1e-6):
        if self.m == 0:
            return 0.0, self.dP
        # bracket the m-th eigenvalue above 0 by the m-th sign change of the one-sided end value
        # P(1) over a scan in a^2 (started clear of the a = 0 root), then match two-sided
        grid = np.arange(0.01, 40.0, 0.05)
        prev = None
        bracket = None
        found = 0
        for a2 in grid:
            endv = self._end_value(a2, eps)
            if prev is not None and np.sign(endv) != np.sign(prev[1]):
                found += 1
                if found == self.m:
                    bracket = (prev[0], a2)
                    break
            prev = (a2, endv)
        if bracket is None:
            raise ValueError("eigenvalue bracket not found")
        a2_0 = brentq(lambda a: self._end_value(a, eps), *bracket, xtol=1e-10)
        # starting slope at +1 (in s = 1 - mu) from the one-sided profile near that end
        mu0, y0 = self._start(self.dP, -1, eps)
        near = solve_ivp(self._rhs, (mu0, 1.0 - 1e-3), y0, args=(a2_0,), rtol=1e-11, atol=1e-13,
                         method="DOP853").y[0, -1]
        c0 = near / 1e-3

        def F(v):
            a2, c = v
            L = self._side(a2, self.dP, -1, eps).y[:, -1]
            R = self._side(a2, c, +1, eps).y[:, -1]
            return L - R
        sol, info, ier, msg = fsolve(F, [a2_0, c0], xtol=1e-14, full_output=True)
        if ier != 1 and np.max(np.abs(F(sol))) > 1e-10:
            raise RuntimeError("eigenvalue matching failed: " + msg)
        return float(sol[0]), float(sol[1])

    def _build_profile(self, eps=1e-6):
        self._left = self._side(self.a2, self.dP, -1, eps, dense=True)
        self._right = self._side(self.a2, self._slope_plus, +1, eps, dense=True)
        self._eps = eps

    def P(self, mu):
        """P(mu) and P'(mu) on [-1, 1] (vectorised)."""
        mu = np.asarray(mu, dtype=np.float64)
        P = np.empty_like(mu)
        dP = np.empty_like(mu)
        eps = self._eps
        left = mu <= 0.0
        # inside the tiny end layers use the regular series
        for side, mask, slope, sgn in ((self._left, left, self.dP, -1),
                                       (self._right, ~left, self._slope_plus, +1)):
            if not np.any(mask):
                continue
            m = mu[mask]
            s = 1.0 - sgn * m
            d = -self.n * (self.n + 1) * slope / 4.0
            inner = s < eps
            Pv = np.empty_like(m)
            dPv = np.empty_like(m)
            if np.any(~inner):
                y = side.sol(m[~inner])
                Pv[~inner] = y[0]
                dPv[~inner] = y[1]
            if np.any(inner):
                si = s[inner]
                Pv[inner] = slope * si + d * si * si
                dPv[inner] = -sgn * (slope + 2.0 * d * si)
            P[mask] = Pv
            dP[mask] = dPv
        return P, dP

    # -- field -------------------------------------------------------------------------------
    def field(self, x, y, z):
        """Exact B = (Bx, By, Bz) at points (x, y, z); arrays broadcast together."""
        x, y, z = np.broadcast_arrays(np.asarray(x, np.float64), np.asarray(y, np.float64),
                                      np.asarray(z, np.float64))
        n = self.n
        cP, sP = np.cos(self.Phi), np.sin(self.Phi)
        zl = z + self.l
        X = x * cP - zl * sP
        Y = y
        Z = x * sP + zl * cP
        rho2 = X * X + Y * Y
        r = np.sqrt(rho2 + Z * Z)
        rho = np.sqrt(rho2)
        mu = Z / r
        sin_t = rho / r
        P, dP = self.P(mu)
        rn2 = r ** (n + 2)
        Br = -dP / rn2
        Bt = n * P / (rn2 * sin_t)
        Bp = self.a * P * np.abs(P) ** (1.0 / n) / (rn2 * sin_t)
        cph = X / rho
        sph = Y / rho
        BX = (Br * sin_t + Bt * mu) * cph - Bp * sph
        BY = (Br * sin_t + Bt * mu) * sph + Bp * cph
        BZ = Br * mu - Bt * sin_t
        Bx = BX * cP + BZ * sP
        By = BY
        Bz = -BX * sP + BZ * cP
        return np.stack([Bx, By, Bz])
