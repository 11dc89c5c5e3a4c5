"""Exact solution of the 1D Riemann problem for the ideal-gas Euler equations
(Toro, "Riemann Solvers and Numerical Methods for Fluid Dynamics", Ch. 4:
pressure function, Newton iteration for p*, similarity sampling).

Independent of the oracle: used to pin the oracle's shock-tube results and to
check the paper's printed star states (tab:shock_1d).
"""
from __future__ import annotations

import math

import numpy as np


def _fK(p, rho, pK, g):
    a = math.sqrt(g * pK / rho)
    if p > pK:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pK
        f = (p - pK) * math.sqrt(A / (p + B))
        df = math.sqrt(A / (B + p)) * (1.0 - (p - pK) / (2.0 * (B + p)))
    else:  # rarefaction
        f = 2.0 * a / (g - 1.0) * ((p / pK) ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rho * a) * (p / pK) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(L, R, g=1.4, tol=1e-15):
    """(p*, u*) for left/right primitive states (rho, u, p)."""
    rL, uL, pL = L
    rR, uR, pR = R
    aL, aR = math.sqrt(g * pL / rL), math.sqrt(g * pR / rR)
    # two-rarefaction guess
    z = (g - 1.0) / (2.0 * g)
    p = ((aL + aR - 0.5 * (g - 1.0) * (uR - uL)) / (aL / pL ** z + aR / pR ** z)) ** (1.0 / z)
    p = max(p, 1e-12)
    for _ in range(200):
        fL, dL = _fK(p, rL, pL, g)
        fR, dR = _fK(p, rR, pR, g)
        f = fL + fR + (uR - uL)
        pn = max(p - f / (dL + dR), 1e-14)
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fL, _ = _fK(p, rL, pL, g)
    fR, _ = _fK(p, rR, pR, g)
    u = 0.5 * (uL + uR) + 0.5 * (fR - fL)
    return p, u


def star_densities(L, R, p, g=1.4):
    out = []
    for (r, _, pK) in (L, R):
        if p > pK:
            q = p / pK
            gm = (g - 1.0) / (g + 1.0)
            out.append(r * (q + gm) / (gm * q + 1.0))
        else:
            out.append(r * (p / pK) ** (1.0 / g))
    return tuple(out)


def sample(L, R, x, t, x0=0.5, g=1.4):
    """Exact (rho, u, p) at positions x and time t > 0."""
    rL, uL, pL = L
    rR, uR, pR = R
    ps, us = star_state(L, R, g)
    rsL, rsR = star_densities(L, R, ps, g)
    aL, aR = math.sqrt(g * pL / rL), math.sqrt(g * pR / rR)
    s = (np.asarray(x, dtype=np.float64) - x0) / t
    rho, u, p = np.empty_like(s), np.empty_like(s), np.empty_like(s)
    for n, S in enumerate(s):
        if S <= us:  # left of contact
            if ps > pL:
                SL = uL - aL * math.sqrt((g + 1) / (2 * g) * ps / pL + (g - 1) / (2 * g))
                st = (rL, uL, pL) if S <= SL else (rsL, us, ps)
            else:
                asL = aL * (ps / pL) ** ((g - 1) / (2 * g))
                SHL, STL = uL - aL, us - asL
                if S <= SHL:
                    st = (rL, uL, pL)
                elif S >= STL:
                    st = (rsL, us, ps)
                else:
                    c = 2 / (g + 1) + (g - 1) / ((g + 1) * aL) * (uL - S)
                    st = (rL * c ** (2 / (g - 1)), 2 / (g + 1) * (aL + (g - 1) / 2 * uL + S),
                          pL * c ** (2 * g / (g - 1)))
        else:
            if ps > pR:
                SR = uR + aR * math.sqrt((g + 1) / (2 * g) * ps / pR + (g - 1) / (2 * g))
                st = (rR, uR, pR) if S >= SR else (rsR, us, ps)
            else:
                asR = aR * (ps / pR) ** ((g - 1) / (2 * g))
                SHR, STR = uR + aR, us + asR
                if S >= SHR:
                    st = (rR, uR, pR)
                elif S <= STR:
                    st = (rsR, us, ps)
                else:
                    c = 2 / (g + 1) - (g - 1) / ((g + 1) * aR) * (uR - S)
                    st = (rR * c ** (2 / (g - 1)), 2 / (g + 1) * (-aR + (g - 1) / 2 * uR + S),
                          pR * c ** (2 * g / (g - 1)))
        rho[n], u[n], p[n] = st
    return rho, u, p
