"""Exact solution of the Riemann problem for two stiffened gases.

Independent of the oracle: written from the textbook exact solver for the
Euler equations (Toro, Riemann Solvers and Numerical Methods for Fluid
Dynamics, ch. 4), with p replaced by p + pi_inf in the wave relations, which
is exact for the stiffened-gas EOS rho e = (p + gamma pi)/(gamma - 1).

For the five-equation model with a volume fraction that is piecewise
constant (it jumps only at the contact), each side is a single stiffened gas
with the mixture parameters gamma_m = 1 + 1/Gamma and pi_m = Pi/(Gamma + 1),
where Gamma = sum_k alpha_k/(gamma_k - 1), Pi = sum_k alpha_k gamma_k pi_k /
(gamma_k - 1).  `mixture_gas` returns those.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


def mixture_gas(alpha1, gamma, pi_inf):
    """Effective (gamma_m, pi_m) of the pressure-equilibrium mixture."""
    a = (alpha1, 1.0 - alpha1)
    G = sum(a[k] / (gamma[k] - 1.0) for k in range(2))
    P = sum(a[k] * gamma[k] * pi_inf[k] / (gamma[k] - 1.0) for k in range(2))
    return 1.0 + 1.0 / G, P / (G + 1.0)


class Side:
    def __init__(self, rho, u, p, gamma, pi):
        self.rho, self.u, self.p, self.g, self.pi = float(rho), float(u), float(p), float(gamma), float(pi)
        self.c = math.sqrt(self.g * (self.p + self.pi) / self.rho)

    def f(self, p):
        """Velocity jump function across the wave connecting this side to pressure p."""
        g, pi = self.g, self.pi
        if p > self.p:  # shock
            A = 2.0 / ((g + 1.0) * self.rho)
            B = (g - 1.0) / (g + 1.0) * (self.p + pi)
            return (p - self.p) * math.sqrt(A / (p + pi + B))
        # rarefaction
        return 2.0 * self.c / (g - 1.0) * (((p + pi) / (self.p + pi)) ** ((g - 1.0) / (2.0 * g)) - 1.0)

    def rho_star(self, ps):
        g, pi = self.g, self.pi
        r = (ps + pi) / (self.p + pi)
        if ps > self.p:
            k = (g - 1.0) / (g + 1.0)
            return self.rho * (r + k) / (k * r + 1.0)
        return self.rho * r ** (1.0 / g)


class ExactRiemann:
    """Exact Riemann solution between states L and R (each rho, u, p, gamma, pi)."""

    def __init__(self, L: Side, R: Side):
        self.L, self.R = L, R
        du = R.u - L.u

        def F(p):
            return L.f(p) + R.f(p) + du

        lo = -min(L.pi, R.pi) + 1e-12 * max(1.0, L.p, R.p)
        hi = max(L.p, R.p, 1.0)
        while F(hi) < 0.0:
            hi *= 2.0
        if F(lo) > 0.0:
            raise ValueError("vacuum generated")
        self.p_star = brentq(F, lo, hi, xtol=1e-14 * hi, rtol=1e-15, maxiter=500)
        ps = self.p_star
        self.u_star = 0.5 * (L.u + R.u) + 0.5 * (R.f(ps) - L.f(ps))
        self.rho_star_L = L.rho_star(ps)
        self.rho_star_R = R.rho_star(ps)

    def wave_speeds(self):
        """Dict of the characteristic speeds bounding each wave."""
        L, R, ps, us = self.L, self.R, self.p_star, self.u_star
        out = {}
        if ps > L.p:
            gL = L.g
            out["left_shock"] = L.u - L.c * math.sqrt((gL + 1) / (2 * gL) * (ps + L.pi) / (L.p + L.pi) + (gL - 1) / (2 * gL))
        else:
            cs = L.c * ((ps + L.pi) / (L.p + L.pi)) ** ((L.g - 1) / (2 * L.g))
            out["left_head"], out["left_tail"] = L.u - L.c, us - cs
        out["contact"] = us
        if ps > R.p:
            gR = R.g
            out["right_shock"] = R.u + R.c * math.sqrt((gR + 1) / (2 * gR) * (ps + R.pi) / (R.p + R.pi) + (gR - 1) / (2 * gR))
        else:
            cs = R.c * ((ps + R.pi) / (R.p + R.pi)) ** ((R.g - 1) / (2 * R.g))
            out["right_head"], out["right_tail"] = R.u + R.c, us + cs
        return out

    def sample(self, s):
        """(rho, u, p, side) at similarity coordinates s = x/t (array); side is
        0 left of the contact, 1 right of it."""
        s = np.asarray(s, dtype=np.float64)
        rho = np.empty_like(s)
        u = np.empty_like(s)
        p = np.empty_like(s)
        side = (s > self.u_star).astype(int)
        ws = self.wave_speeds()
        ps, us = self.p_star, self.u_star
        for K, sign in ((self.L, -1.0), (self.R, 1.0)):
            m = side == (0 if sign < 0 else 1)
            x = s[m]
            r = np.empty_like(x)
            uu = np.empty_like(x)
            pp = np.empty_like(x)
            rs = K.rho_star(ps)
            g, pi = K.g, K.pi
            if ps > K.p:
                shock = ws["left_shock" if sign < 0 else "right_shock"]
                outside = (x < shock) if sign < 0 else (x > shock)
                r[:] = np.where(outside, K.rho, rs)
                uu[:] = np.where(outside, K.u, us)
                pp[:] = np.where(outside, K.p, ps)
            else:
                head = ws["left_head" if sign < 0 else "right_head"]
                tail = ws["left_tail" if sign < 0 else "right_tail"]
                outside = (x < head) if sign < 0 else (x > head)
                star = (x > tail) if sign < 0 else (x < tail)
                fan = ~outside & ~star
                r[:] = np.where(outside, K.rho, rs)
                uu[:] = np.where(outside, K.u, us)
                pp[:] = np.where(outside, K.p, ps)
                xf = x[fan]
                # inside the fan (Toro eq. 4.56 / 4.63 with p -> p + pi)
                base = 2.0 / (g + 1.0) - sign * (g - 1.0) / ((g + 1.0) * K.c) * (K.u - xf)
                r[fan] = K.rho * base ** (2.0 / (g - 1.0))
                uu[fan] = 2.0 / (g + 1.0) * (-sign * K.c + (g - 1.0) / 2.0 * K.u + xf)
                pp[fan] = (K.p + pi) * base ** (2.0 * g / (g - 1.0)) - pi
            rho[m], u[m], p[m] = r, uu, pp
        return rho, u, p, side
