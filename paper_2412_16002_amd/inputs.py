"""Seeded synthetic inputs shaped like the paper's test problems.

This module holds initial data and problem parameters only -- none of the
method's arithmetic.  Both the GPU path and the CPU oracle take their inputs
from here: per-cell constant states (evaluated at cell centres), closed-form
initial functions u0(x), or random Legendre-mode perturbations.  Euler states
are returned as conservative variables (rho, m, E) with
E = p / (gamma - 1) + rho |w|^2 / 2, the equation of state of Sec. 2.2.3.

Workloads (all seeded with numpy.random.default_rng(seed)):
  burgers_1d      1D Burgers, periodic [0,1], 256 cells, P^2, 3 stages, CFL 0.1,
                  u0 = 0.5 + 0.4 * (normalised sum of 4 random-phase sines),
                  bounds [min u0, max u0]
  euler_1d_riemann  1D Euler, 4096 cells, P^3, 4 stages, outflow, 16 equal
                  segments with rho = 10^U[-4,0], u = U[-2,2], p = 10^U[-8,0]
  euler_2d_voronoi  2D Euler, 1024^2, Q^2, 3 stages, periodic, 64 Voronoi sites
                  (periodic metric) with rho = 10^U[-3,0], p = 10^U[-6,1],
                  |w| = U[0,3] at a uniform angle
  euler_3d_wave   3D Euler, 128^3, Q^2, 4 stages, periodic, exact density wave
                  rho = 1 + 0.99 sin(2 pi (x+y+z) + phi), w = (1,1,1), p = 1
  euler_3d_blast  3D Euler, 128^3, Q^2, 4 stages, p = 100 inside a random
                  sphere, 1e-4 outside, rho = 1, w = 0
  batched_2d      64 independent 2D Euler instances, N_i ~ U{64..512},
                  P^k with k ~ U{1,2,3}, 3 stages for k <= 2 and 4 for k = 3,
                  16 Voronoi sites each with the states of euler_1d_riemann
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = 1.4


def conservative(rho, w, p, gamma=GAMMA):
    """(rho, w[..., d], p) -> conservative (rho, m, E) stacked on the last axis."""
    rho = np.asarray(rho, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    m = rho[..., None] * w
    E = p / (gamma - 1.0) + 0.5 * rho * np.sum(w * w, axis=-1)
    return np.concatenate([rho[..., None], m, E[..., None]], axis=-1)


@dataclass
class Case:
    """Problem parameters (names as in crkdg_problem) plus the initial data:
    either `cell_states` [Nc, V] (piecewise constant by cell) or `u0` (a
    function of physical points [..., d] returning [..., V])."""
    name: str
    params: dict
    cell_states: np.ndarray | None = None
    u0: object = None
    t_end: float = math.inf
    exact: object = None            # exact solution u(x, t) where one exists
    meta: dict = field(default_factory=dict)


def cell_centres(n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    """Cell centres [Nc, d] in natural order (first index fastest)."""
    d = len(n)
    axes = [lo[j] + (np.arange(n[j]) + 0.5) * (hi[j] - lo[j]) / n[j] for j in range(d)]
    grids = np.meshgrid(*axes, indexing="ij")
    return np.stack([g.transpose(tuple(range(d))[::-1]).reshape(-1) for g in grids], axis=-1)


# ---------------------------------------------------------------------------
def burgers_1d(seed=0, n=256):
    rng = np.random.default_rng(seed)
    amp = rng.uniform(0.0, 1.0, 4)
    amp /= amp.sum()
    ph = rng.uniform(0.0, 2.0 * np.pi, 4)
    j = np.arange(1, 5)

    def u0(x):
        x = np.asarray(x)[..., 0]
        s = np.sum(amp * np.sin(2.0 * np.pi * j * x[..., None] + ph), axis=-1)
        return (0.5 + 0.4 * s)[..., None]

    # global bounds of u0 by dense sampling refined with Newton on u0'
    xs = np.linspace(0.0, 1.0, 20001)
    vals = u0(xs[:, None])[:, 0]
    ext = []
    for idx in (np.argmin(vals), np.argmax(vals)):
        x = xs[idx]
        for _ in range(50):
            d1 = 0.4 * np.sum(amp * 2 * np.pi * j * np.cos(2 * np.pi * j * x + ph))
            d2 = -0.4 * np.sum(amp * (2 * np.pi * j) ** 2 * np.sin(2 * np.pi * j * x + ph))
            x = x - d1 / d2
        ext.append(float(u0(np.array([[x]]))[0, 0]))
    lo_b, hi_b = min(ext[0], vals.min()), max(ext[1], vals.max())
    params = dict(dim=1, n=(n,), system="burgers", k=2, stages=3, cfl=0.1,
                  bc=("periodic",), bound_lo=lo_b, bound_hi=hi_b)
    return Case("burgers_1d", params, u0=u0, t_end=0.5,
                meta=dict(amp=amp, phase=ph))


def euler_1d_riemann(seed=0, n=4096, segments=16):
    rng = np.random.default_rng(seed)
    rho = 10.0 ** rng.uniform(-4.0, 0.0, segments)
    u = rng.uniform(-2.0, 2.0, segments)
    p = 10.0 ** rng.uniform(-8.0, 0.0, segments)
    seg = (np.arange(n) * segments) // n
    states = conservative(rho[seg], u[seg][:, None], p[seg])
    params = dict(dim=1, n=(n,), system="euler", k=3, stages=4, cfl=0.093, eps=1e-13,
                  bc=("outflow",))
    return Case("euler_1d_riemann", params, cell_states=states, t_end=1e-3)


def _voronoi_labels(centres, sites):
    """Index of the nearest site under the periodic unit-box metric (ties to
    the lowest index)."""
    best = np.full(len(centres), np.inf)
    lab = np.zeros(len(centres), dtype=np.int64)
    for i, s in enumerate(sites):
        dlt = np.abs(centres - s)
        dlt = np.minimum(dlt, 1.0 - dlt)
        d2 = np.sum(dlt * dlt, axis=1)
        better = d2 < best
        best[better] = d2[better]
        lab[better] = i
    return lab


def euler_2d_voronoi(seed=0, n=1024, sites=64, precision="mixed"):
    rng = np.random.default_rng(seed)
    pts = rng.uniform(0.0, 1.0, (sites, 2))
    rho = 10.0 ** rng.uniform(-3.0, 0.0, sites)
    p = 10.0 ** rng.uniform(-6.0, 1.0, sites)
    speed = rng.uniform(0.0, 3.0, sites)
    ang = rng.uniform(0.0, 2.0 * np.pi, sites)
    w = np.stack([speed * np.cos(ang), speed * np.sin(ang)], axis=-1)
    lab = _voronoi_labels(cell_centres((n, n)), pts)
    states = conservative(rho[lab], w[lab], p[lab])
    params = dict(dim=2, n=(n, n), system="euler", k=2, space="Q", stages=3, cfl=0.153,
                  eps=1e-8, bc=("periodic", "periodic"), precision=precision)
    return Case("euler_2d_voronoi", params, cell_states=states)


def euler_3d_wave(seed=0, n=128, precision="mixed"):
    rng = np.random.default_rng(seed)
    ph = float(rng.uniform(0.0, 2.0 * np.pi))

    def exact(x, t):
        x = np.asarray(x)
        s = np.sum(x, axis=-1) - 3.0 * t
        rho = 1.0 + 0.99 * np.sin(2.0 * np.pi * s + ph)
        return conservative(rho, np.ones(x.shape[:-1] + (3,)), np.ones(x.shape[:-1]))

    params = dict(dim=3, n=(n, n, n), system="euler", k=2, space="Q", stages=4, cfl=0.153,
                  eps=1e-8, bc=("periodic",) * 3, precision=precision)
    return Case("euler_3d_wave", params, u0=lambda x: exact(x, 0.0), exact=exact,
                meta=dict(phase=ph))


def euler_3d_blast(seed=0, n=128, precision="mixed"):
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.25, 0.75, 3)
    r = float(rng.uniform(0.05, 0.15))
    x = cell_centres((n, n, n))
    inside = np.sum((x - c) ** 2, axis=1) < r * r
    p = np.where(inside, 100.0, 1e-4)
    states = conservative(np.ones(len(x)), np.zeros((len(x), 3)), p)
    params = dict(dim=3, n=(n, n, n), system="euler", k=2, space="Q", stages=4, cfl=0.153,
                  eps=1e-8, bc=("periodic",) * 3, precision=precision)
    return Case("euler_3d_blast", params, cell_states=states, meta=dict(centre=c, radius=r))


def sedov_2d(n=160, k=2, space="Q", precision="fp64", length=1.1, eps=1e-13):
    """The Sedov blast of the 2D examples (Sec. 4.4, Example 4.7): [0, 1.1]^2, rho = 1,
    w = 0, E = 1e-12 except E = 0.244816 / dx^2 in the corner cell; reflective
    walls on the lower sides, outflow on the upper ones (the blast's energy
    makes the shock reach radius 1 at t = 1).  eps below the background
    rho e (reading A6)."""
    dx = length / n
    E = np.full(n * n, 1e-12)
    E[0] = 0.244816 / dx ** 2
    states = np.zeros((n * n, 4))
    states[:, 0] = 1.0
    states[:, 3] = E
    stages = 3 if k <= 2 else 4
    params = dict(dim=2, n=(n, n), system="euler", k=k, space=space, stages=stages,
                  cfl={1: 0.3, 2: 0.153, 3: 0.093}[k], eps=eps, hi=(length, length, 1.0),
                  bc=("reflect", "reflect"), bc_upper=("outflow", "outflow"), precision=precision)
    return Case("sedov_2d", params, cell_states=states, t_end=1.0, meta=dict(dx=dx, shock_radius=1.0))


def euler_wave(dim, n, k, space="Q", stages=None, seed=0, precision="fp64", amp=0.99):
    """Exact smooth Euler solution in d dimensions: rho = 1 + amp sin(2 pi
    (sum x - d t) + phi), w = (1, .., 1), p = 1 (a translating density wave)."""
    rng = np.random.default_rng(seed)
    ph = float(rng.uniform(0.0, 2.0 * np.pi))

    def exact(x, t):
        x = np.asarray(x)
        s = np.sum(x, axis=-1) - dim * t
        rho = 1.0 + amp * np.sin(2.0 * np.pi * s + ph)
        return conservative(rho, np.ones(x.shape[:-1] + (dim,)), np.ones(x.shape[:-1]))

    params = dict(dim=dim, n=tuple(n), system="euler", k=k, space=space,
                  stages=stages or k + 1, cfl=0.05, eps=1e-8, bc=("periodic",) * dim,
                  precision=precision)
    return Case(f"euler_wave_{dim}d", params, u0=lambda x: exact(x, 0.0), exact=exact)


def batched_2d(seed=0, count=64, nmin=64, nmax=512, sites=16, precision="mixed"):
    rng = np.random.default_rng(seed)
    cases = []
    for i in range(count):
        n = int(rng.integers(nmin, nmax + 1))
        k = int(rng.integers(1, 4))
        pts = rng.uniform(0.0, 1.0, (sites, 2))
        rho = 10.0 ** rng.uniform(-4.0, 0.0, sites)
        w = rng.uniform(-2.0, 2.0, (sites, 2))
        p = 10.0 ** rng.uniform(-8.0, 0.0, sites)
        lab = _voronoi_labels(cell_centres((n, n)), pts)
        states = conservative(rho[lab], w[lab], p[lab])
        params = dict(dim=2, n=(n, n), system="euler", k=k, space="P",
                      stages=3 if k <= 2 else 4, cfl={1: 0.30, 2: 0.153, 3: 0.093}[k],
                      eps=1e-13, bc=("periodic", "periodic"), precision=precision)
        cases.append(Case(f"batched_2d[{i}]", params, cell_states=states))
    return cases


def random_legendre(ncell, nvars, nmodes, mode_degree, seed=0, avg=None, rel_amp=0.1):
    """Random Legendre coefficients [Nc, V, M]: averages `avg` [Nc, V] (default
    U[0.5, 1.5]) and higher modes with amplitude rel_amp * |avg| / (1 + degree)^2,
    `mode_degree[m]` the total degree of mode m."""
    rng = np.random.default_rng(seed)
    if avg is None:
        avg = rng.uniform(0.5, 1.5, (ncell, nvars))
    c = np.zeros((ncell, nvars, nmodes))
    c[:, :, 0] = avg
    deg = np.asarray(mode_degree, dtype=np.float64)
    for m in range(1, nmodes):
        c[:, :, m] = rng.uniform(-1.0, 1.0, (ncell, nvars)) * rel_amp * np.abs(avg) / (1.0 + deg[m]) ** 2
    return c


def random_euler_averages(ncell, dim, seed=0, rho=(0.5, 1.5), p=(0.5, 1.5), speed=1.0):
    """Random admissible Euler cell averages [Nc, d+2]."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(*rho, ncell)
    pp = rng.uniform(*p, ncell)
    w = rng.uniform(-speed, speed, (ncell, dim))
    return conservative(r, w, pp)
