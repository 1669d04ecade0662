"""Exact solutions of the 1D shallow-water equations on a flat bed, used to pin
the oracle (independent of it).

Riemann problem: depth function with shock (Hugoniot locus) and rarefaction
(Riemann invariant) branches, root h* by bisection, dry-bed and vacuum
cases; solution sampled at xi = x / t.  Ritter: the dry-bed dam break.
"""
import math

import numpy as np


def _fK(h, hK, g):
    if h <= hK:
        return 2.0 * (math.sqrt(g * h) - math.sqrt(g * hK))
    return (h - hK) * math.sqrt(0.5 * g * (h + hK) / (h * hK))


def star_depth(hL, uL, hR, uR, g=9.81):
    f = lambda h: _fK(h, hL, g) + _fK(h, hR, g) + uR - uL
    lo, hi = 1e-14, max(hL, hR)
    while f(hi) < 0:
        hi *= 2.0
    for _ in range(200):  # plain bisection: slow, obviously convergent
        mid = 0.5 * (lo + hi)
        if f(mid) > 0:
            hi = mid
        else:
            lo = mid
    h = 0.5 * (lo + hi)
    u = 0.5 * (uL + uR) + 0.5 * (_fK(h, hR, g) - _fK(h, hL, g))
    return h, u


def sample(hL, uL, hR, uR, xi, g=9.81):
    """Exact (h, u) at similarity coordinate(s) xi."""
    xi = np.atleast_1d(np.asarray(xi, dtype=np.float64))
    h = np.zeros_like(xi)
    u = np.zeros_like(xi)
    cL = math.sqrt(g * hL)
    cR = math.sqrt(g * hR)
    for n, x in enumerate(xi):
        if hR == 0.0 and hL == 0.0:
            continue
        if hR == 0.0:  # right dry
            if x <= uL - cL:
                h[n], u[n] = hL, uL
            elif x < uL + 2 * cL:
                uu = (uL + 2 * cL + 2 * x) / 3.0
                cc = (uL + 2 * cL - x) / 3.0
                h[n], u[n] = cc * cc / g, uu
            continue
        if hL == 0.0:  # left dry
            if x >= uR + cR:
                h[n], u[n] = hR, uR
            elif x > uR - 2 * cR:
                uu = (uR - 2 * cR + 2 * x) / 3.0
                cc = (-uR + 2 * cR + x) / 3.0
                h[n], u[n] = cc * cc / g, uu
            continue
        if uR - uL >= 2 * (cL + cR):  # vacuum generated in the middle
            if x <= uL - cL:
                h[n], u[n] = hL, uL
            elif x < uL + 2 * cL:
                uu = (uL + 2 * cL + 2 * x) / 3.0
                cc = (uL + 2 * cL - x) / 3.0
                h[n], u[n] = cc * cc / g, uu
            elif x <= uR - 2 * cR:
                pass
            elif x < uR + cR:
                uu = (uR - 2 * cR + 2 * x) / 3.0
                cc = (-uR + 2 * cR + x) / 3.0
                h[n], u[n] = cc * cc / g, uu
            else:
                h[n], u[n] = hR, uR
            continue
        hs, us = star_depth(hL, uL, hR, uR, g)
        cs = math.sqrt(g * hs)
        if x <= us:  # left of the contact
            if hs > hL:
                SL = uL - cL * math.sqrt(0.5 * hs * (hs + hL) / (hL * hL))
                h[n], u[n] = (hL, uL) if x < SL else (hs, us)
            else:
                if x <= uL - cL:
                    h[n], u[n] = hL, uL
                elif x >= us - cs:
                    h[n], u[n] = hs, us
                else:
                    uu = (uL + 2 * cL + 2 * x) / 3.0
                    cc = (uL + 2 * cL - x) / 3.0
                    h[n], u[n] = cc * cc / g, uu
        else:
            if hs > hR:
                SR = uR + cR * math.sqrt(0.5 * hs * (hs + hR) / (hR * hR))
                h[n], u[n] = (hR, uR) if x > SR else (hs, us)
            else:
                if x >= uR + cR:
                    h[n], u[n] = hR, uR
                elif x <= us + cs:
                    h[n], u[n] = hs, us
                else:
                    uu = (uR - 2 * cR + 2 * x) / 3.0
                    cc = (-uR + 2 * cR + x) / 3.0
                    h[n], u[n] = cc * cc / g, uu
    return h, u


def ritter(x, t, x0, h0, g=9.81):
    """Dry-bed dam break: depth h0 for x < x0 at t = 0."""
    c0 = math.sqrt(g * h0)
    xi = (np.asarray(x, dtype=np.float64) - x0) / t
    h = np.where(xi <= -c0, h0, np.where(xi >= 2 * c0, 0.0, (2 * c0 - xi) ** 2 / (9 * g)))
    u = np.where(xi <= -c0, 0.0, np.where(xi >= 2 * c0, 0.0, 2.0 / 3.0 * (xi + c0)))
    return h, u
