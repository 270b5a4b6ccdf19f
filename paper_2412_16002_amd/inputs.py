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


def euler_3d_wave_slab(seed=0, n=128, parts=8, precision="mixed"):
    """One GPU's share of the 3D wave workload when its n^3 mesh is split into
    `parts` slabs along z: n x n x n/parts cells of the same width on
    [0, 1]^2 x [0, 1/parts], periodic in z (the slab's own opposite face
    stands in for the neighbour's traces of the exchange), the wave's z
    frequency raised to `parts` so that the slab holds whole periods."""
    rng = np.random.default_rng(seed)
    ph = float(rng.uniform(0.0, 2.0 * np.pi))

    def exact(x, t):
        x = np.asarray(x)
        s = x[..., 0] + x[..., 1] + parts * x[..., 2] - (2.0 + parts) * t
        rho = 1.0 + 0.99 * np.sin(2.0 * np.pi * s + ph)
        return conservative(rho, np.ones(x.shape[:-1] + (3,)), np.ones(x.shape[:-1]))

    params = dict(dim=3, n=(n, n, n // parts), system="euler", k=2, space="Q", stages=4, cfl=0.153,
                  eps=1e-8, bc=("periodic",) * 3, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0 / parts),
                  precision=precision)
    return Case("euler_3d_wave_slab", params, u0=lambda x: exact(x, 0.0), exact=exact,
                meta=dict(phase=ph, parts=parts))


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


# ---------------------------------------------------------------------------
# Manufactured solution of the 2D Euler accuracy test (Sec. 4.2, Example 4.2,
# scenario I): rho = z sin(2 pi (x+y)) + 2, w = (z cos(2 pi x) sin(2 pi y) + 2,
# z sin(2 pi x) cos(2 pi y) + 2), e = z cos(2 pi (x+y)) / 2 + 1 with
# z = exp(-t), on [0,1]^2 (1-periodic in x and y), end time 0.1024.  Its
# right-hand side s = dU/dt + div f(U) is problem data: it is formed here by
# the chain rule from the closed-form primitives and their derivatives.
# Every term of s is z^p times a function of x (p = 1..4: U is a polynomial
# of degree <= 3 in z, the fluxes of degree <= 4, and dz/dt = -z), so
# s(x, t) = sum_p exp(-p t) S_p(x) exactly.
# ---------------------------------------------------------------------------
MMS_T_END = 0.1024
MMS_RATES = (1.0, 2.0, 3.0, 4.0)


def _mms_fields(X, z, gamma=GAMMA):
    """Primitives (rho, w1, w2, e) of scenario I at X[..., 2] with z = exp(-t)
    (z may be complex), and their derivatives in t, x and y."""
    x, y = X[..., 0], X[..., 1]
    k = 2.0 * np.pi
    S, C = np.sin(k * (x + y)), np.cos(k * (x + y))
    sx, cx, sy, cy = np.sin(k * x), np.cos(k * x), np.sin(k * y), np.cos(k * y)
    f = {
        "rho": (z * S + 2.0, -z * S, k * z * C, k * z * C),
        "w1": (z * cx * sy + 2.0, -z * cx * sy, -k * z * sx * sy, k * z * cx * cy),
        "w2": (z * sx * cy + 2.0, -z * sx * cy, k * z * cx * cy, -k * z * sx * sy),
        "e": (0.5 * z * C + 1.0, -0.5 * z * C, -0.5 * k * z * S, -0.5 * k * z * S),
    }
    return f


def _mms_source_z(X, z, gamma=GAMMA):
    """s = dU/dt + d f_1/dx + d f_2/dy of scenario I at X[..., 2], z = exp(-t)."""
    f = _mms_fields(X, z, gamma)
    r, rt, rx, ry = f["rho"]
    u, ut, ux, uy = f["w1"]
    v, vt, vx, vy = f["w2"]
    e, et, ex, ey = f["e"]
    g1 = gamma - 1.0
    # pressure p = (gamma - 1) rho e and total energy E = rho e + rho |w|^2 / 2
    p = g1 * r * e
    px, py = g1 * (rx * e + r * ex), g1 * (ry * e + r * ey)
    q = 0.5 * (u * u + v * v)
    En = r * e + r * q
    Et = rt * e + r * et + rt * q + r * (u * ut + v * vt)
    Ex = rx * e + r * ex + rx * q + r * (u * ux + v * vx)
    Ey = ry * e + r * ey + ry * q + r * (u * uy + v * vy)
    mass = rt + (rx * u + r * ux) + (ry * v + r * vy)
    mom1 = (rt * u + r * ut) + (rx * u * u + 2.0 * r * u * ux + px) + (ry * u * v + r * uy * v + r * u * vy)
    mom2 = (rt * v + r * vt) + (rx * u * v + r * ux * v + r * u * vx) + (ry * v * v + 2.0 * r * v * vy + py)
    ener = Et + ((Ex + px) * u + (En + p) * ux) + ((Ey + py) * v + (En + p) * vy)
    return np.stack([mass, mom1, mom2, ener], axis=-1)


def mms_euler2d_exact(X, t, gamma=GAMMA):
    """Conservative (rho, m_1, m_2, E) of scenario I at X[..., 2] and time t."""
    X = np.asarray(X, dtype=np.float64)
    f = _mms_fields(X, math.exp(-t), gamma)
    r, u, v, e = f["rho"][0], f["w1"][0], f["w2"][0], f["e"][0]
    return np.stack([r, r * u, r * v, r * e + 0.5 * r * (u * u + v * v)], axis=-1)


def mms_euler2d_source(X, t, gamma=GAMMA):
    """The source s(x, t) of scenario I at X[..., 2] [..., 4]."""
    return _mms_source_z(np.asarray(X, dtype=np.float64), math.exp(-t), gamma)


def mms_euler2d_source_terms(X, gamma=GAMMA):
    """The fields S_p(x), p = 1..4, of s(x, t) = sum_p exp(-p t) S_p(x):
    the coefficients of the degree-4 polynomial z -> s(x, z), read off its
    values at the fifth roots of unity (a discrete Fourier transform, exact
    up to rounding).  Returns [4, ..., 4]; the z^0 coefficient is zero."""
    X = np.asarray(X, dtype=np.float64)
    zs = np.exp(2j * np.pi * np.arange(5) / 5.0)
    vals = np.stack([_mms_source_z(X, z, gamma) for z in zs])          # [5, ..., 4]
    coef = np.tensordot(np.exp(-2j * np.pi * np.outer(np.arange(5), np.arange(5)) / 5.0) / 5.0,
                        vals, axes=(1, 0))
    return np.ascontiguousarray(coef[1:].real)


# step sizes and meshes of the accuracy table (Table 2): dt = 2^(5-l) 1e-5 on
# the l-th mesh 1/2^(l + base[k])
MMS_MESH_BASE = {1: 4, 2: 3, 3: 2}


def mms_euler2d(k, level, space="P", precision="fp64", limiter=True):
    """Example 4.2 scenario I on the level-th mesh of Table 2 (level 0..3)
    for P^k / Q^k with the (k+1)-stage cRKDG scheme, fixed dt, periodic."""
    n = 2 ** (MMS_MESH_BASE[k] + level)
    dt = 2.0 ** (5 - level) * 1e-5
    params = dict(dim=2, n=(n, n), system="euler", k=k, space=space, stages=k + 1, cfl=0.1,
                  eps=1e-8, bc=("periodic", "periodic"), precision=precision, limiter=limiter)
    return Case(f"mms_euler2d_{space}{k}_{n}", params, u0=lambda X: mms_euler2d_exact(X, 0.0),
                t_end=MMS_T_END, exact=mms_euler2d_exact,
                meta=dict(dt=dt, source=mms_euler2d_source, rates=MMS_RATES,
                          source_terms=mms_euler2d_source_terms))


def mms_euler2d_scenario2_exact(X, t, gamma=GAMMA):
    """Example 4.2 scenario II: rho = 0.99 sin(pi (x + y - 2 t)) + 1, w = (1, 1),
    rho e = 1 / (gamma - 1) (p = 1): an exact solution (no source), density
    down to 0.01."""
    X = np.asarray(X, dtype=np.float64)
    rho = 0.99 * np.sin(np.pi * (X[..., 0] + X[..., 1] - 2.0 * t)) + 1.0
    return conservative(rho, np.ones(X.shape[:-1] + (2,)), np.ones(X.shape[:-1]), gamma)


def mms_euler2d_scenario2(k, level, space="P", precision="fp64"):
    """Scenario II on the meshes and steps of Table 3, on the periodic box
    [0, 2]^2 (the solution has period 2 in x and y; the paper's [0, 1]^2 needs
    time-dependent boundary data): the same mesh width 1/2^(level + base[k])
    and dt = 2^(5-level) 1e-5, to t = 0.1024."""
    n = 2 * 2 ** (MMS_MESH_BASE[k] + level)
    dt = 2.0 ** (5 - level) * 1e-5
    params = dict(dim=2, n=(n, n), system="euler", k=k, space=space, stages=k + 1, cfl=0.1, eps=1e-8,
                  hi=(2.0, 2.0, 1.0), bc=("periodic", "periodic"), precision=precision)
    return Case(f"mms_euler2d_s2_{space}{k}_{n}", params, u0=lambda X: mms_euler2d_scenario2_exact(X, 0.0),
                t_end=MMS_T_END, exact=mms_euler2d_scenario2_exact, meta=dict(dt=dt))


def boundary_face_points(params, side):
    """Physical coordinates [n_faces, n_fp, d] of the face Gauss points of
    side `side` (2 d + upper) of a box mesh: faces in natural order of the
    other directions, points the tensor (k+1)-point Gauss points of the
    other directions (both lower direction fastest)."""
    d = params["dim"]
    n = tuple(params["n"])[:d]
    lo = tuple(params.get("lo", (0.0, 0.0, 0.0)))[:d]
    hi = tuple(params.get("hi", (1.0, 1.0, 1.0)))[:d]
    dd, up = side // 2, side % 2
    g, _ = np.polynomial.legendre.leggauss(params["k"] + 1)
    others = [j for j in range(d) if j != dd]
    dx = [(hi[j] - lo[j]) / n[j] for j in range(d)]
    cells = np.array(list(np.ndindex(*[n[j] for j in others][::-1])))[:, ::-1] if others else np.zeros((1, 0), int)
    pts = np.array(list(np.ndindex(*([len(g)] * len(others))[::-1])))[:, ::-1] if others else np.zeros((1, 0), int)
    X = np.zeros((len(cells), len(pts), d))
    X[..., dd] = hi[dd] if up else lo[dd]
    for a, j in enumerate(others):
        X[..., j] = lo[j] + (cells[:, None, a] + 0.5 + 0.5 * g[pts[None, :, a]]) * dx[j]
    return X


def boundary_values(params, side, terms):
    """Boundary data values [n_terms, n_faces, n_fp, V] of time-separable
    Dirichlet data sum_p g_p(t) G_p(x): terms = [G_p(X[..., d]) -> [..., V]]."""
    X = boundary_face_points(params, side)
    return np.ascontiguousarray(np.stack([np.asarray(G(X), dtype=np.float64) for G in terms]))


# the exact data of scenario II as three time-separable terms: rho = 1 + 0.99
# (sin(pi s) cos(2 pi t) - cos(pi s) sin(2 pi t)), s = x + y; U is affine in rho
SCENARIO2_COEF = ((0.0, 0.0, 0.0), (0.0, 2.0 * math.pi, 0.0), (0.0, 2.0 * math.pi, -0.5 * math.pi))


def scenario2_boundary_terms(gamma=GAMMA):
    one = np.array([1.0, 1.0, 1.0, 1.0])
    base = np.array([1.0, 1.0, 1.0, 1.0 / (gamma - 1.0) + 1.0])
    return [lambda X: np.broadcast_to(base, X.shape[:-1] + (4,)),
            lambda X: 0.99 * np.sin(np.pi * (X[..., 0] + X[..., 1]))[..., None] * one,
            lambda X: -0.99 * np.cos(np.pi * (X[..., 0] + X[..., 1]))[..., None] * one]


def mms_euler2d_scenario2_box(k, level, space="P", precision="fp64"):
    """Scenario II on the paper's [0, 1]^2 with the exact solution as
    Dirichlet data on all four sides (Table 3's meshes and steps)."""
    n = 2 ** (MMS_MESH_BASE[k] + level)
    dt = 2.0 ** (5 - level) * 1e-5
    st = [float(v) for v in mms_euler2d_scenario2_exact(np.zeros((1, 2)), 0.0)[0]]
    params = dict(dim=2, n=(n, n), system="euler", k=k, space=space, stages=k + 1, cfl=0.1, eps=1e-8,
                  bc=("dirichlet", "dirichlet"), bc_state={f: st for f in range(4)}, precision=precision)
    return Case(f"mms_euler2d_s2box_{space}{k}_{n}", params, u0=lambda X: mms_euler2d_scenario2_exact(X, 0.0),
                t_end=MMS_T_END, exact=mms_euler2d_scenario2_exact,
                meta=dict(dt=dt, bc_coef=SCENARIO2_COEF, bc_terms=scenario2_boundary_terms()))


def euler_wave_box3d(k, n, space="Q", precision="fp64", amp=0.5, gamma=GAMMA):
    """The 3D density wave rho = 1 + amp sin(2 pi (x + y + z - 3 t)), w = (1,
    1, 1), p = 1 on [0, 1]^3 with its exact values as Dirichlet data on the
    four x and y sides (z periodic).  The data are three time-separable terms
    (U is affine in rho): a constant, sin(2 pi s) cos(6 pi t) and
    cos(2 pi s) cos(6 pi t + pi / 2), s = x + y + z."""
    def exact(X, t):
        X = np.asarray(X)
        rho = 1.0 + amp * np.sin(2.0 * np.pi * (np.sum(X, axis=-1) - 3.0 * t))
        return conservative(rho, np.ones(X.shape[:-1] + (3,)), np.ones(X.shape[:-1]))

    lin = np.array([1.0, 1.0, 1.0, 1.0, 1.5])                   # dU / drho
    base = np.array([1.0, 1.0, 1.0, 1.0, 1.0 / (gamma - 1.0) + 1.5])
    terms = [lambda X: np.broadcast_to(base, X.shape[:-1] + (5,)),
             lambda X: amp * np.sin(2.0 * np.pi * np.sum(X, axis=-1))[..., None] * lin,
             lambda X: amp * np.cos(2.0 * np.pi * np.sum(X, axis=-1))[..., None] * lin]
    coef = ((0.0, 0.0, 0.0), (0.0, 6.0 * math.pi, 0.0), (0.0, 6.0 * math.pi, 0.5 * math.pi))
    st = [float(v) for v in exact(np.zeros((1, 3)), 0.0)[0]]
    params = dict(dim=3, n=tuple(n), system="euler", k=k, space=space, stages=k + 1, cfl=0.1, eps=1e-8,
                  bc=("dirichlet", "dirichlet", "periodic"), bc_state={f: st for f in range(4)},
                  precision=precision)
    return Case(f"euler_wave_box3d_{space}{k}", params, u0=lambda X: exact(X, 0.0), t_end=0.01, exact=exact,
                meta=dict(bc_coef=coef, bc_terms=terms))


def table1_advection(k, level, precision="fp64"):
    """Example 4.1: u_t + u_x = 0 on [0, 1], u = sin(2 pi (x - t)) + 2 in [1, 3],
    the meshes and steps of Table 1 (dt = 2^(4-level) 1e-4, dx = 1/2^(level +
    5 - k)... per k), t = 0.1024, the exact inflow u(0, t) = 2 - sin(2 pi t)
    as Dirichlet data on the left, outflow on the right, limiter on B = [1, 3]."""
    n = 2 ** ({1: 5, 2: 4, 3: 3}[k] + level)
    dt = 2.0 ** (4 - level) * 1e-4

    def exact(X, t):
        return (np.sin(2.0 * np.pi * (np.asarray(X)[..., 0] - t)) + 2.0)[..., None]

    params = dict(dim=1, n=(n,), system="advection", k=k, stages=k + 1, cfl=0.1, vel=(1.0, 0.0, 0.0),
                  bc=("dirichlet",), bc_upper=("outflow",), bc_state={0: [2.0]}, bound_lo=1.0, bound_hi=3.0,
                  precision=precision)
    return Case(f"table1_p{k}_{n}", params, u0=lambda X: exact(X, 0.0), t_end=0.1024, exact=exact,
                meta=dict(dt=dt, bc_coef=((0.0, 0.0, 0.0), (0.0, 2.0 * math.pi, -0.5 * math.pi)),
                          bc_terms=[lambda X: np.full(X.shape[:-1] + (1,), 2.0),
                                    lambda X: np.full(X.shape[:-1] + (1,), -1.0)]))


def mms_advection_1d(k, n, precision="fp64", t_end=0.25, dt_per_dx=0.05):
    """A manufactured solution of u_t + u_x = s on the periodic [0,1]:
    u = exp(-t) sin(2 pi x) + 2, so s = exp(-t) (2 pi cos(2 pi x) - sin(2 pi x))
    (one term of rate 1); P^k with k+1 stages, fixed dt = dt_per_dx dx."""
    def exact(X, t):
        return (math.exp(-t) * np.sin(2.0 * np.pi * np.asarray(X)[..., 0]) + 2.0)[..., None]

    def term(X):
        x = np.asarray(X, dtype=np.float64)[..., 0]
        return (2.0 * np.pi * np.cos(2.0 * np.pi * x) - np.sin(2.0 * np.pi * x))[..., None]

    def source(X, t):
        return math.exp(-t) * term(X)

    params = dict(dim=1, n=(n,), system="advection", k=k, stages=k + 1, cfl=0.1, vel=(1.0, 0.0, 0.0),
                  bc=("periodic",), precision=precision, limiter=False)
    return Case(f"mms_advection_1d_p{k}_{n}", params, u0=lambda X: exact(X, 0.0), t_end=t_end, exact=exact,
                meta=dict(dt=dt_per_dx / n, source=source, rates=(1.0,), source_terms=lambda X: term(X)[None]))


# ---------------------------------------------------------------------------
# Shallow water (flat bottom): U = (h, h w_1, .., h w_d), g = gravity
# ---------------------------------------------------------------------------
def swe_conservative(h, w):
    """(h, w[..., d]) -> (h, h w) stacked on the last axis."""
    h = np.asarray(h, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    return np.concatenate([h[..., None], h[..., None] * w], axis=-1)


def swe_dam_break_1d(n=200, k=2, h_left=2.0, h_right=1.0, gravity=1.0, precision="fp64", eps=1e-12,
                     t_end=0.3):
    """A dam break on [-1, 1], still water on both sides: h = h_left for
    x < 0, h_right for x > 0, the end states held as Dirichlet data (the
    waves stay inside until t_end)."""
    x = cell_centres((n,), lo=(-1.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0))[:, 0]
    h = np.where(x < 0.0, h_left, h_right)
    params = dict(dim=1, n=(n,), system="shallow_water", k=k, stages=k + 1, lo=(-1.0, 0.0, 0.0),
                  hi=(1.0, 1.0, 1.0), bc=("dirichlet",), bc_state={0: [h_left, 0.0], 1: [h_right, 0.0]},
                  gravity=gravity, eps=eps, cfl={1: 0.3, 2: 0.153, 3: 0.093}[k], precision=precision)
    return Case(f"swe_dam_break_{n}", params, cell_states=swe_conservative(h, np.zeros((n, 1))), t_end=t_end,
                meta=dict(h_left=h_left, h_right=h_right))


def _swe_mms_fields(X, z):
    """Primitives (h, w_1..w_d) of the manufactured shallow-water solution
    and their derivatives [value, d/dt, d/dx_1, ..] with z = exp(-t):
    h = z sin(2 pi sum x) + 3, w_j = z cos(2 pi x_j) + 1."""
    d = X.shape[-1]
    k = 2.0 * np.pi
    sx = np.sum(X, axis=-1)
    h = [z * np.sin(k * sx) + 3.0, -z * np.sin(k * sx)] + [k * z * np.cos(k * sx)] * d
    ws = []
    for j in range(d):
        xj = X[..., j]
        wj = [z * np.cos(k * xj) + 1.0, -z * np.cos(k * xj)]
        wj += [(-k * z * np.sin(k * xj)) if i == j else 0.0 * xj for i in range(d)]
        ws.append(wj)
    return h, ws


def _swe_mms_source_z(X, z, gravity):
    """s = dU/dt + sum_i d f_i / dx_i of the manufactured solution."""
    h, ws = _swe_mms_fields(X, z)
    d = X.shape[-1]
    out = []
    # mass: h_t + sum_i (h w_i)_i
    mass = h[1] + sum(h[2 + i] * ws[i][0] + h[0] * ws[i][2 + i] for i in range(d))
    out.append(mass)
    for j in range(d):
        # (h w_j)_t + sum_i (h w_j w_i)_i + (g h^2 / 2)_j
        m = h[1] * ws[j][0] + h[0] * ws[j][1]
        for i in range(d):
            m = m + (h[2 + i] * ws[j][0] * ws[i][0] + h[0] * ws[j][2 + i] * ws[i][0]
                     + h[0] * ws[j][0] * ws[i][2 + i])
        m = m + gravity * h[0] * h[2 + j]
        out.append(m)
    return np.stack(out, axis=-1)


SWE_MMS_RATES = (1.0, 2.0, 3.0)


def swe_mms_exact(X, t):
    X = np.asarray(X, dtype=np.float64)
    h, ws = _swe_mms_fields(X, math.exp(-t))
    return swe_conservative(h[0], np.stack([w[0] for w in ws], axis=-1))


def swe_mms_source(X, t, gravity=1.0):
    return _swe_mms_source_z(np.asarray(X, dtype=np.float64), math.exp(-t), gravity)


def swe_mms_source_terms(X, gravity=1.0):
    """S_p, p = 1..3, of s = sum_p exp(-p t) S_p (s is a cubic in z = exp(-t)
    with no constant term), read off at the fourth roots of unity."""
    X = np.asarray(X, dtype=np.float64)
    zs = np.exp(2j * np.pi * np.arange(4) / 4.0)
    vals = np.stack([_swe_mms_source_z(X, z, gravity) for z in zs])
    coef = np.tensordot(np.exp(-2j * np.pi * np.outer(np.arange(4), np.arange(4)) / 4.0) / 4.0, vals, axes=(1, 0))
    return np.ascontiguousarray(coef[1:].real)


def swe_mms(dim, n, k, space="Q", precision="fp64", t_end=0.1, dt_per_dx=0.01):
    """The manufactured shallow-water solution on the periodic unit box, g = 1,
    k+1 stages, fixed dt = dt_per_dx dx."""
    params = dict(dim=dim, n=tuple([n] * dim), system="shallow_water", k=k, space=space, stages=k + 1,
                  cfl=0.1, eps=1e-8, gravity=1.0, bc=("periodic",) * dim, precision=precision)
    return Case(f"swe_mms_{dim}d_{space}{k}_{n}", params, u0=lambda X: swe_mms_exact(X, 0.0), t_end=t_end,
                exact=swe_mms_exact,
                meta=dict(dt=dt_per_dx / n, source=swe_mms_source, rates=SWE_MMS_RATES,
                          source_terms=swe_mms_source_terms))


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
