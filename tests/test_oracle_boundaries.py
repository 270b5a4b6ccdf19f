"""Pins of the oracle's non-periodic boundaries (reflective walls and
Dirichlet / inflow sides, used by the paper's Sec. 4 examples) against facts
that do not depend on the boundary code itself (no GPU):

* a reflective wall is a mirror plane: the run with walls equals the
  periodic run on the doubled domain with mirrored data, restricted;
* a Dirichlet side whose state equals the (constant) state next to it
  changes nothing against an outflow side, and swapping the two states does;
* inflow into linear advection adds mass at the closed-form rate a (g - u_R)
  per unit time, the Lax--Friedrichs flux with alpha = |a| being upwind."""
import numpy as np
import pytest

from oracle import ADVECTION, DIRICHLET, EULER, OUTFLOW, PERIODIC, REFLECT, CRKDG, Problem
from _helpers import random_state


def _mirror(o, C, dd):
    """Legendre coefficients of the mirror image across a plane normal to
    direction dd: P_e(-x) = (-1)^e P_e(x); the normal momentum changes sign."""
    sign = np.array([(-1.0) ** e[dd] for e in o.legendre_modes()])
    out = C * sign[None, None, :]
    out[:, 1 + dd, :] *= -1.0
    return out


def _cell(n, ijk):
    c, stride = 0, 1
    for j, v in enumerate(ijk):
        c += v * stride
        stride *= n[j]
    return c


@pytest.mark.parametrize("dim,dd,k", [(1, 0, 2), (2, 0, 1), (2, 1, 2)])
def test_reflective_walls_equal_mirrored_periodic_run(dim, dd, k):
    n = (10,) if dim == 1 else (6, 5)
    bc_r = tuple(REFLECT if j == dd else PERIODIC for j in range(dim))
    R = CRKDG(Problem(dim=dim, n=n, system=EULER, k=k, stages=3, bc=bc_r, cfl=0.15))
    n2 = tuple(2 * v if j == dd else v for j, v in enumerate(n))
    hi2 = tuple(2.0 if j == dd else 1.0 for j in range(dim)) + (1.0,) * (3 - dim)
    P = CRKDG(Problem(dim=dim, n=n2, system=EULER, k=k, stages=3, hi=hi2,
                      bc=(PERIODIC,) * dim, cfl=0.15))
    C = random_state(R, seed=5, rel_amp=0.2)
    Cm = _mirror(R, C, dd)
    CP = np.zeros((P.ncell,) + C.shape[1:])
    own, img = [], []
    for c in range(R.ncell):
        ijk = list(R.idx[c])
        own.append(_cell(n2, ijk))
        ijk_m = list(ijk)
        ijk_m[dd] = n2[dd] - 1 - ijk[dd]
        img.append(_cell(n2, ijk_m))
    CP[own] = C
    CP[img] = Cm
    UR, UP = R.from_legendre(C), P.from_legendre(CP)
    dt = 0.6 * R.trial_dt(UR)
    for _ in range(3):
        UR, _ = R.step(UR, dt_fixed=dt)
        UP, _ = P.step(UP, dt_fixed=dt)
    a, b = R.to_legendre(UR), P.to_legendre(UP)[own]
    scale = np.max(np.abs(b), axis=(0, 2))
    assert np.max(np.abs(a - b) / scale[None, :, None]) < 1e-12
    # the doubled run stays a mirror image (the symmetry the wall imposes)
    assert np.max(np.abs(P.to_legendre(UP)[img] - _mirror(R, b, dd)) / scale[None, :, None]) < 1e-12


def _riemann(o, left, right, dd=0):
    avg = np.where((o.cell_centres()[:, dd] < 0.5)[:, None], np.asarray(left)[None, :], np.asarray(right)[None, :])
    C = np.zeros((o.ncell, o.V, o.M))
    C[:, :, 0] = avg
    return o.from_legendre(C)


def _euler_state(rho, w, p, gamma=1.4):
    w = np.asarray(w, dtype=float)
    return [rho] + list(rho * w) + [p / (gamma - 1.0) + 0.5 * rho * float(w @ w)]


@pytest.mark.parametrize("dim", [1, 2])
def test_dirichlet_sides_with_the_adjacent_state_equal_outflow(dim):
    """Sod-like data whose waves stay away from the ends for three steps:
    Dirichlet sides holding the end states give the outflow run; the same
    sides with the two states swapped do not."""
    L = _euler_state(1.0, [0.3] + [0.1] * (dim - 1), 1.0)
    Rs = _euler_state(0.125, [-0.2] + [0.0] * (dim - 1), 0.1)
    n = (40,) if dim == 1 else (40, 3)
    bcs = (OUTFLOW,) + (PERIODIC,) * (dim - 1)
    base = dict(dim=dim, n=n, system=EULER, k=2, stages=3, cfl=0.15, eps=1e-13)
    out = CRKDG(Problem(bc=bcs, **base))
    dbc = (DIRICHLET,) + (PERIODIC,) * (dim - 1)
    dir_ = CRKDG(Problem(bc=dbc, bc_state={0: L, 1: Rs}, **base))
    swp = CRKDG(Problem(bc=dbc, bc_state={0: Rs, 1: L}, **base))
    U0 = _riemann(out, L, Rs)
    dt = 0.5 * out.trial_dt(U0)
    Uo, Ud, Us = U0, U0, U0
    for _ in range(3):
        Uo, _ = out.step(Uo, dt_fixed=dt)
        Ud, _ = dir_.step(Ud, dt_fixed=dt)
        Us, _ = swp.step(Us, dt_fixed=dt)
    a, b, c = out.to_legendre(Uo), dir_.to_legendre(Ud), swp.to_legendre(Us)
    assert np.max(np.abs(a - b)) < 1e-13
    assert np.max(np.abs(a - c)) > 1e-3


@pytest.mark.parametrize("k,stages", [(1, 2), (2, 3), (3, 4)])
def test_inflow_adds_mass_at_the_closed_form_rate(k, stages):
    """Linear advection (a = 1), u0 = 1, Dirichlet inflow u = 2 on the left,
    outflow on the right (the inflow example of Sec. 4.2): while the front is
    away from the right end, every step adds dt a (2 - 1) to the total, and
    the solution stays in [1, 2]."""
    p = Problem(dim=1, n=(30,), system=ADVECTION, k=k, stages=stages, vel=(1.0, 0, 0), bc=(DIRICHLET,),
                bc_upper=(OUTFLOW,), bc_state={0: [2.0]}, bound_lo=1.0, bound_hi=2.0, cfl=0.1)
    o = CRKDG(p)
    U = o.project(lambda x: np.ones(x.shape[:-1] + (1,)))
    t0 = o.totals(U)[0]
    for _ in range(5):
        U1, info = o.step(U)
        assert abs((o.totals(U1)[0] - o.totals(U)[0]) - info["dt"] * 1.0 * (2.0 - 1.0)) < 1e-14
        U = U1
    assert o.totals(U)[0] > t0
    assert o.bound_violations(U) == 0


def test_boundary_validation():
    with pytest.raises(ValueError):
        CRKDG(Problem(dim=1, n=(8,), system=EULER, bc=(PERIODIC,), bc_upper=(OUTFLOW,)))
    with pytest.raises(ValueError):
        CRKDG(Problem(dim=1, n=(8,), system=ADVECTION, bc=(REFLECT,)))
    with pytest.raises(ValueError):
        CRKDG(Problem(dim=1, n=(8,), system=EULER, bc=(DIRICHLET,), bc_state={0: [1.0, 0.0, 2.5]}))
