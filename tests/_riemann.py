"""Exact solution of the Riemann problem of the 1D Euler equations for an
ideal gas (the textbook construction: the star pressure is the root of the
sum of the two wave functions, shock branch from the Rankine--Hugoniot
conditions, rarefaction branch from the isentropic relations).  Test
infrastructure: an independent reference for the Riemann data of the 1D
examples, shared by neither the oracle nor the library."""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


def _wave(p, rho, pk, g):
    """Velocity jump across the wave that connects state (rho, pk) to
    pressure p, and its sign convention f_K(p)."""
    c = math.sqrt(g * pk / rho)
    if p > pk:
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        return (p - pk) * math.sqrt(A / (p + B))
    return 2.0 * c / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)


def star_state(left, right, g=1.4):
    """(p*, u*) for primitive states left = (rho, u, p), right = (rho, u, p).
    p* = 0 when the data generate vacuum."""
    rl, ul, pl = left
    rr, ur, pr = right
    f = lambda p: _wave(p, rl, pl, g) + _wave(p, rr, pr, g) + (ur - ul)
    if f(0.0) >= 0.0:                      # vacuum (or its threshold) in the middle
        return 0.0, 0.5 * (ul + ur) + 0.5 * (_wave(0.0, rr, pr, g) - _wave(0.0, rl, pl, g))
    hi = max(pl, pr)
    while f(hi) < 0.0:
        hi *= 2.0
    ps = brentq(f, 0.0, hi, xtol=1e-15, rtol=1e-15, maxiter=500)
    us = 0.5 * (ul + ur) + 0.5 * (_wave(ps, rr, pr, g) - _wave(ps, rl, pl, g))
    return ps, us


def sample(left, right, xi, g=1.4):
    """Primitive (rho, u, p) of the self-similar solution at xi = x / t."""
    ps, us = star_state(left, right, g)
    xi = np.asarray(xi, dtype=float)
    out = np.zeros(xi.shape + (3,))
    for idx, s in np.ndenumerate(xi):
        # look from the side of the contact the point is on (mirror the right side)
        if s < us:
            rho, u, p, sgn = left[0], left[1], left[2], 1.0
        else:
            rho, u, p, sgn = right[0], -right[1], right[2], -1.0
            s = -s
        ustar = sgn * us
        c = math.sqrt(g * p / rho)
        if ps > p:                                   # shock
            rstar = rho * ((ps / p + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * ps / p + 1))
            speed = u - c * math.sqrt((g + 1) / (2 * g) * ps / p + (g - 1) / (2 * g))
            st = (rho, u, p) if s < speed else (rstar, ustar, ps)
        else:                                        # rarefaction
            head = u - c
            if s < head:
                st = (rho, u, p)
            else:
                rstar = rho * (ps / p) ** (1.0 / g)
                cstar = math.sqrt(g * ps / rstar) if rstar > 0 else 0.0
                tail = ustar - cstar
                if s > tail:
                    st = (rstar, ustar, ps)
                else:
                    fac = 2.0 / (g + 1) + (g - 1) / ((g + 1) * c) * (u - s)
                    st = (rho * fac ** (2.0 / (g - 1)), 2.0 / (g + 1) * (c + (g - 1) / 2 * u + s),
                          p * fac ** (2.0 * g / (g - 1)))
        out[idx] = (st[0], sgn * st[1], st[2])
    return out


def cell_averages(left, right, x0, edges, t, g=1.4, sub=64):
    """Conservative cell averages of the exact solution at time t on the
    cells between consecutive `edges` (midpoint rule on `sub` sub-cells)."""
    out = np.zeros((len(edges) - 1, 3))
    for i in range(len(edges) - 1):
        xs = edges[i] + (np.arange(sub) + 0.5) * (edges[i + 1] - edges[i]) / sub
        w = sample(left, right, (xs - x0) / t, g)
        rho, u, p = w[:, 0], w[:, 1], w[:, 2]
        out[i] = [rho.mean(), (rho * u).mean(), (p / (g - 1) + 0.5 * rho * u * u).mean()]
    return out
