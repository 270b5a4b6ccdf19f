"""Exact solution of the shallow-water Riemann problem (flat bottom, 1D),
written for the tests from the standard wave analysis: the star depth h*
solves f_L(h*) + f_R(h*) + u_R - u_L = 0 with f_K(h) = 2 (sqrt(g h) -
sqrt(g h_K)) for a rarefaction (h <= h_K) and (h - h_K) sqrt(g (h + h_K) /
(2 h h_K)) for a shock (h > h_K); a dry right state (h_R = 0) gives the
dry-bed fan with its front at u_L + 2 sqrt(g h_L)."""
import math

import numpy as np


def _f(h, hk, g):
    if h <= hk:
        return 2.0 * (math.sqrt(g * h) - math.sqrt(g * hk))
    return (h - hk) * math.sqrt(0.5 * g * (h + hk) / (h * hk))


def star_state(hl, ul, hr, ur, g):
    """(h*, u*) of a wet-wet problem by bisection on the monotone f."""
    F = lambda h: _f(h, hl, g) + _f(h, hr, g) + ur - ul   # noqa: E731
    lo, hi = 1e-14, 10.0 * max(hl, hr) + (ul - ur) ** 2 / g + 1.0
    assert F(lo) < 0.0 < F(hi), "dry star region"
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if F(mid) > 0.0:
            hi = mid
        else:
            lo = mid
    hs = 0.5 * (lo + hi)
    us = 0.5 * (ul + ur) + 0.5 * (_f(hs, hr, g) - _f(hs, hl, g))
    return hs, us


def sample(xi, hl, ul, hr, ur, g):
    """(h, u) at x / t = xi (arrays)."""
    xi = np.asarray(xi, dtype=np.float64)
    al = math.sqrt(g * hl)
    h = np.empty_like(xi)
    u = np.empty_like(xi)
    if hr == 0.0:
        # dry bed: fan between ul - al and the front ul + 2 al
        head, front = ul - al, ul + 2.0 * al
        left, dry = xi <= head, xi >= front
        fan = ~left & ~dry
        h[left], u[left] = hl, ul
        h[dry], u[dry] = 0.0, 0.0
        a = (ul + 2.0 * al - xi[fan]) / 3.0
        h[fan], u[fan] = a * a / g, (ul + 2.0 * al + 2.0 * xi[fan]) / 3.0
        return h, u
    ar = math.sqrt(g * hr)
    hs, us = star_state(hl, ul, hr, ur, g)
    as_ = math.sqrt(g * hs)
    for i, x in enumerate(xi):
        if x <= us:
            if hs > hl:                                    # left shock
                s = ul - al * math.sqrt(0.5 * (hs + hl) * hs / (hl * hl))
                h[i], u[i] = (hl, ul) if x <= s else (hs, us)
            else:                                          # left rarefaction
                if x <= ul - al:
                    h[i], u[i] = hl, ul
                elif x >= us - as_:
                    h[i], u[i] = hs, us
                else:
                    a = (ul + 2.0 * al - x) / 3.0
                    h[i], u[i] = a * a / g, (ul + 2.0 * al + 2.0 * x) / 3.0
        else:
            if hs > hr:                                    # right shock
                s = ur + ar * math.sqrt(0.5 * (hs + hr) * hs / (hr * hr))
                h[i], u[i] = (hr, ur) if x >= s else (hs, us)
            else:                                          # right rarefaction
                if x >= ur + ar:
                    h[i], u[i] = hr, ur
                elif x <= us + as_:
                    h[i], u[i] = hs, us
                else:
                    a = (-ur + 2.0 * ar + x) / 3.0
                    h[i], u[i] = a * a / g, (ur - 2.0 * ar + 2.0 * x) / 3.0
    return h, u


def cell_averages(x_lo, x_hi, n, t, hl, ul, hr, ur, g, sub=64):
    """Cell averages of h and h u over n equal cells at time t (midpoint rule
    on sub points per cell)."""
    dx = (x_hi - x_lo) / n
    xs = x_lo + (np.arange(n * sub) + 0.5) * dx / sub
    h, u = sample(xs / t, hl, ul, hr, ur, g)
    return h.reshape(n, sub).mean(axis=1), (h * u).reshape(n, sub).mean(axis=1)
