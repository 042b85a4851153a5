"""Exact solution of the Riemann problem for the 1D Euler equations of an ideal
gas (Toro, "Riemann Solvers and Numerical Methods for Fluid Dynamics", 3rd ed.,
2009, chapter 4), used to pin the oracle on Sod's shock tube (§5.1.2 of the
paper compares against an exact Riemann solver).

Pressure functions f_K(p) (Toro eq. 4.6-4.8): for p > p_K a shock,
    f_K = (p - p_K) sqrt(A_K / (p + B_K)),  A_K = 2/((g+1) rho_K),  B_K = (g-1)/(g+1) p_K,
otherwise a rarefaction,
    f_K = 2 c_K/(g-1) ((p/p_K)^((g-1)/(2g)) - 1).
The star pressure solves f_L(p) + f_R(p) + (u_R - u_L) = 0 and the star velocity
is u* = (u_L + u_R)/2 + (f_R(p*) - f_L(p*))/2 (Toro eq. 4.9). The solution is
sampled along rays x/t following Toro section 4.5.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


class ExactRiemann:
    def __init__(self, left, right, gamma=1.4):
        self.g = float(gamma)
        self.rL, self.uL, self.pL = map(float, left)
        self.rR, self.uR, self.pR = map(float, right)
        self.cL = math.sqrt(self.g * self.pL / self.rL)
        self.cR = math.sqrt(self.g * self.pR / self.rR)
        self._solve()

    def _f(self, p, rK, pK, cK):
        g = self.g
        if p > pK:
            A = 2.0 / ((g + 1.0) * rK)
            B = (g - 1.0) / (g + 1.0) * pK
            return (p - pK) * math.sqrt(A / (p + B))
        return 2.0 * cK / (g - 1.0) * ((p / pK) ** ((g - 1.0) / (2.0 * g)) - 1.0)

    def _solve(self):
        du = self.uR - self.uL
        fun = lambda p: (self._f(p, self.rL, self.pL, self.cL)
                         + self._f(p, self.rR, self.pR, self.cR) + du)
        hi = 10.0 * max(self.pL, self.pR)
        self.p_star = brentq(fun, 1e-12, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
        fL = self._f(self.p_star, self.rL, self.pL, self.cL)
        fR = self._f(self.p_star, self.rR, self.pR, self.cR)
        self.u_star = 0.5 * (self.uL + self.uR) + 0.5 * (fR - fL)
        g = self.g
        gm = (g - 1.0) / (g + 1.0)
        ps = self.p_star
        # star densities (Toro eq. 4.50/4.53 for shocks, 4.60 for rarefactions)
        if ps > self.pL:
            self.rho_star_L = self.rL * ((ps / self.pL + gm) / (gm * ps / self.pL + 1.0))
        else:
            self.rho_star_L = self.rL * (ps / self.pL) ** (1.0 / g)
        if ps > self.pR:
            self.rho_star_R = self.rR * ((ps / self.pR + gm) / (gm * ps / self.pR + 1.0))
        else:
            self.rho_star_R = self.rR * (ps / self.pR) ** (1.0 / g)

    def sample(self, xi):
        """Primitive state (rho, u, p) on the ray x/t = xi."""
        g = self.g
        ps, us = self.p_star, self.u_star
        if xi <= us:  # left of the contact
            rK, uK, pK, cK = self.rL, self.uL, self.pL, self.cL
            if ps > pK:  # left shock
                SL = uK - cK * math.sqrt((g + 1) / (2 * g) * ps / pK + (g - 1) / (2 * g))
                return (rK, uK, pK) if xi <= SL else (self.rho_star_L, us, ps)
            SHL = uK - cK
            cs = cK * (ps / pK) ** ((g - 1) / (2 * g))
            STL = us - cs
            if xi <= SHL:
                return (rK, uK, pK)
            if xi >= STL:
                return (self.rho_star_L, us, ps)
            c = 2.0 / (g + 1) * (cK + (g - 1) / 2 * (uK - xi))
            u = 2.0 / (g + 1) * (cK + (g - 1) / 2 * uK + xi)
            rho = rK * (c / cK) ** (2 / (g - 1))
            p = pK * (c / cK) ** (2 * g / (g - 1))
            return (rho, u, p)
        rK, uK, pK, cK = self.rR, self.uR, self.pR, self.cR
        if ps > pK:  # right shock
            SR = uK + cK * math.sqrt((g + 1) / (2 * g) * ps / pK + (g - 1) / (2 * g))
            return (rK, uK, pK) if xi >= SR else (self.rho_star_R, us, ps)
        SHR = uK + cK
        cs = cK * (ps / pK) ** ((g - 1) / (2 * g))
        STR = us + cs
        if xi >= SHR:
            return (rK, uK, pK)
        if xi <= STR:
            return (self.rho_star_R, us, ps)
        c = 2.0 / (g + 1) * (cK - (g - 1) / 2 * (uK - xi))
        u = 2.0 / (g + 1) * (-cK + (g - 1) / 2 * uK + xi)
        rho = rK * (c / cK) ** (2 / (g - 1))
        p = pK * (c / cK) ** (2 * g / (g - 1))
        return (rho, u, p)

    def shock_speed_right(self):
        g = self.g
        return self.uR + self.cR * math.sqrt((g + 1) / (2 * g) * self.p_star / self.pR + (g - 1) / (2 * g))

    def profile(self, x, t, x0=0.5):
        out = np.array([self.sample((xx - x0) / t) for xx in np.asarray(x, dtype=float)])
        return out[:, 0], out[:, 1], out[:, 2]

    def cell_average_profile(self, n, t, x0=0.5, sub=64):
        """Cell averages of the exact solution on n uniform cells of [0,1]."""
        dx = 1.0 / n
        xs = (np.arange(n * sub) + 0.5) * dx / sub
        r, u, p = self.profile(xs, t, x0)
        return (r.reshape(n, sub).mean(1), u.reshape(n, sub).mean(1), p.reshape(n, sub).mean(1))
