"""Exact solutions used to pin the oracle (test-side only).

* scalar advection: translation of the initial profile;
* Euler: the exact solution of the Riemann problem for a gamma-law gas
  (star pressure from the pressure function, solved by bisection, then
  sampling of shock / rarefaction / contact structure);
* shallow water: Ritter's dam break onto a dry bed.

Written from the gas-dynamics and shallow-water mathematics; nothing here is
shared with the oracle or the GPU library.
"""
from __future__ import annotations

import math

import numpy as np


# --------------------------------------------------------------------------
# Euler Riemann problem
# --------------------------------------------------------------------------

def _fK(p, rhoK, pK, cK, g):
    """Velocity jump across the wave that joins state K to pressure p."""
    if p > pK:  # shock: Rankine-Hugoniot
        A = 2.0 / ((g + 1.0) * rhoK)
        B = (g - 1.0) / (g + 1.0) * pK
        return (p - pK) * math.sqrt(A / (p + B))
    # rarefaction: isentropic, Riemann invariant
    return 2.0 * cK / (g - 1.0) * ((p / pK) ** ((g - 1.0) / (2.0 * g)) - 1.0)


def star_state(left, right, gamma=1.4, tol=1e-15):
    rL, uL, pL = left
    rR, uR, pR = right
    cL, cR = math.sqrt(gamma * pL / rL), math.sqrt(gamma * pR / rR)
    if uR - uL >= 2.0 * (cL + cR) / (gamma - 1.0):
        raise ValueError("vacuum is generated")

    def f(p):
        return _fK(p, rL, pL, cL, gamma) + _fK(p, rR, pR, cR, gamma) + (uR - uL)

    lo, hi = 0.0, max(pL, pR)
    while f(hi) < 0.0:
        hi *= 2.0
    for _ in range(400):
        mid = 0.5 * (lo + hi)
        if f(mid) > 0.0:
            hi = mid
        else:
            lo = mid
        if hi - lo <= tol * hi:
            break
    ps = 0.5 * (lo + hi)
    us = 0.5 * (uL + uR) + 0.5 * (_fK(ps, rR, pR, cR, gamma) - _fK(ps, rL, pL, cL, gamma))
    return ps, us


def riemann_sample(left, right, xi, gamma=1.4):
    """(rho, u, p) at similarity coordinates xi = (x - x_s)/t (array)."""
    g = gamma
    rL, uL, pL = left
    rR, uR, pR = right
    cL, cR = math.sqrt(g * pL / rL), math.sqrt(g * pR / rR)
    ps, us = star_state(left, right, g)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    gm = (g - 1.0) / (g + 1.0)
    for n, S in enumerate(xi.flat):
        if S <= us:  # left of the contact
            if ps > pL:
                SL = uL - cL * math.sqrt((g + 1) / (2 * g) * ps / pL + (g - 1) / (2 * g))
                if S <= SL:
                    w = (rL, uL, pL)
                else:
                    w = (rL * (ps / pL + gm) / (gm * ps / pL + 1.0), us, ps)
            else:
                SHL = uL - cL
                csL = cL * (ps / pL) ** ((g - 1) / (2 * g))
                STL = us - csL
                if S <= SHL:
                    w = (rL, uL, pL)
                elif S >= STL:
                    w = (rL * (ps / pL) ** (1.0 / g), us, ps)
                else:
                    br = 2.0 / (g + 1) + (g - 1) / ((g + 1) * cL) * (uL - S)
                    w = (rL * br ** (2.0 / (g - 1)),
                         2.0 / (g + 1) * (cL + (g - 1) / 2.0 * uL + S),
                         pL * br ** (2.0 * g / (g - 1)))
        else:  # right of the contact
            if ps > pR:
                SR = uR + cR * math.sqrt((g + 1) / (2 * g) * ps / pR + (g - 1) / (2 * g))
                if S >= SR:
                    w = (rR, uR, pR)
                else:
                    w = (rR * (ps / pR + gm) / (gm * ps / pR + 1.0), us, ps)
            else:
                SHR = uR + cR
                csR = cR * (ps / pR) ** ((g - 1) / (2 * g))
                STR = us + csR
                if S >= SHR:
                    w = (rR, uR, pR)
                elif S <= STR:
                    w = (rR * (ps / pR) ** (1.0 / g), us, ps)
                else:
                    br = 2.0 / (g + 1) - (g - 1) / ((g + 1) * cR) * (uR - S)
                    w = (rR * br ** (2.0 / (g - 1)),
                         2.0 / (g + 1) * (-cR + (g - 1) / 2.0 * uR + S),
                         pR * br ** (2.0 * g / (g - 1)))
        rho.flat[n], u.flat[n], p.flat[n] = w
    return rho, u, p


def euler_primitive(U, gamma=1.4):
    """(rho, u, p) from 1D conserved planes (rho, rho u, E)."""
    rho = U[0]
    u = U[1] / rho
    p = (gamma - 1.0) * (U[2] - 0.5 * rho * u * u)
    return rho, u, p


# --------------------------------------------------------------------------
# Shallow water: Ritter's dry-bed dam break
# --------------------------------------------------------------------------

def ritter(x, t, h0, g=9.81):
    """Depth and velocity for h = h0 (x <= 0), dry (x > 0), u = 0 at t = 0."""
    x = np.asarray(x, dtype=np.float64)
    c0 = math.sqrt(g * h0)
    h = np.where(x <= -c0 * t, h0, 0.0)
    u = np.zeros_like(x)
    fan = (x > -c0 * t) & (x < 2.0 * c0 * t)
    xi = x[fan] / t
    h[fan] = (2.0 * c0 - xi) ** 2 / (9.0 * g)
    u[fan] = 2.0 / 3.0 * (c0 + xi)
    return h, u


def total_variation(q):
    return float(np.sum(np.abs(np.diff(q))))
