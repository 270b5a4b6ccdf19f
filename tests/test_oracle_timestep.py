"""Pins of the oracle's wave-speed maximum a0 and trial step (no GPU).

a0_d is the largest wave speed of u~^n in direction d over the limiter
points S_K (Sec. 2.1 definition of a0, read over S_K: A5), and the trial step
of Sec. 4.1 is CFL dx / a0 in 1D, read in d dimensions as
dt = CFL / sum_d (a0_d / dx_d) (A2).  Every expected value below is worked
out by hand from the state's primitive variables (sound speed from the
gamma-law equation of state of Sec. 2.2.3), on anisotropic meshes and with
unequal speeds per direction, so that a maximum taken instead of the sum
over directions, dx in place of 1/dx, a direction mixed up, or a maximum
over the Gauss points only (missing the Lobatto end points of S_K) fails."""
import math

import numpy as np
import pytest

import oracle


def _euler_const(o, rho, w, p, gamma=1.4):
    """Oracle coefficients of the constant Euler state (rho, w, p)."""
    d = o.d
    m = [rho * wj for wj in w]
    E = p / (gamma - 1.0) + 0.5 * rho * sum(wj * wj for wj in w)
    ubar = np.tile(np.array([rho] + m + [E]), (o.ncell, 1))
    assert ubar.shape[1] == d + 2
    return o.constant_state(ubar)


@pytest.mark.parametrize("dim", [2, 3])
def test_trial_dt_constant_euler_anisotropic(dim):
    """Constant Euler state: a0_d = |w_d| + c with c = sqrt(gamma p / rho),
    dt = CFL / sum_d (|w_d| + c) / dx_d on a mesh with a different dx per
    direction."""
    n = (4, 6, 5)[:dim]
    hi = (1.0, 2.0, 0.5)[:dim]
    dx = [hi[j] / n[j] for j in range(dim)]
    rho, p, gamma, cfl = 0.7, 0.4, 1.4, 0.13
    w = (0.3, -1.1, 2.5)[:dim]
    o = oracle.CRKDG(oracle.Problem(dim=dim, n=n, hi=hi + (1.0,) * (3 - dim), system="euler", k=2,
                                    cfl=cfl, gamma=gamma))
    U = _euler_const(o, rho, w, p, gamma)
    c = math.sqrt(gamma * p / rho)
    want_a0 = [abs(wj) + c for wj in w]
    np.testing.assert_allclose(o.a0(U), want_a0, rtol=1e-14)
    rate = sum(want_a0[j] / dx[j] for j in range(dim))
    assert math.isclose(o.trial_dt(U), cfl / rate, rel_tol=1e-14)
    # the step the halving strategy starts from, and its clip to t_end
    _, info = o.step(U, t=0.0)
    assert math.isclose(info["dt"], cfl / rate, rel_tol=1e-14) and info["halvings"] == 0
    _, info = o.step(U, t=0.0, t_end=0.25 * cfl / rate)
    assert math.isclose(info["dt"], 0.25 * cfl / rate, rel_tol=1e-14)
    # a fixed step replaces the CFL rule
    _, info = o.step(U, t=0.0, dt_fixed=1e-5)
    assert info["dt"] == 1e-5


def test_trial_dt_advection_unequal_speeds():
    """Advection with |a_x| != |a_y| on an anisotropic mesh: a0 = (|a_x|,
    |a_y|) whatever the data, dt = CFL / (|a_x| / dx + |a_y| / dy)."""
    ax, ay = 0.5, -2.0
    o = oracle.CRKDG(oracle.Problem(dim=2, n=(5, 3), hi=(1.0, 3.0, 1.0), system="advection", k=1,
                                    vel=(ax, ay, 0.0), cfl=0.2))
    rng = np.random.default_rng(3)
    U = rng.uniform(-1.0, 1.0, (o.ncell, 1, o.M))
    np.testing.assert_array_equal(o.a0(U), [0.5, 2.0])
    assert math.isclose(o.trial_dt(U), 0.2 / (0.5 / 0.2 + 2.0 / 1.0), rel_tol=1e-15)


def test_burgers_a0_at_a_lobatto_end_point():
    """1D Burgers P^2: in a cell with u = a + b xi the largest |u| sits at
    xi = +-1, which S_K holds (Gauss--Lobatto end points) and the Gauss rule
    does not; a0 = |a| + |b| there.  dt = CFL dx / a0 (Sec. 4.1)."""
    o = oracle.CRKDG(oracle.Problem(dim=1, n=(8,), system="burgers", k=2, cfl=0.1))
    C = np.zeros((8, 1, 3))
    C[:, 0, 0] = 0.5
    C[3, 0, :] = [0.4, -0.35, 0.0]      # u = 0.4 - 0.35 xi: |u| <= 0.75 at xi = -1
    U = o.from_legendre(C)
    assert math.isclose(o.a0(U)[0], 0.75, rel_tol=1e-14)
    # the Gauss points alone would give 0.4 + 0.35 sqrt(3/5)
    g = math.sqrt(0.6)
    assert o.a0(U)[0] > 0.4 + 0.35 * g + 0.05
    assert math.isclose(o.trial_dt(U), 0.1 * (1.0 / 8) / 0.75, rel_tol=1e-14)


def test_euler_a0_where_the_density_is_smallest():
    """1D Euler P^1 with rho = r0 + r1 xi, m = 0, E constant: the pressure is
    (gamma - 1) E everywhere, so c = sqrt(gamma (gamma - 1) E / rho) peaks at
    the smallest density, xi = -1 for r1 > 0, a point of S_K (Lobatto)."""
    gamma = 1.4
    o = oracle.CRKDG(oracle.Problem(dim=1, n=(4,), system="euler", k=1, cfl=0.3, gamma=gamma))
    C = np.zeros((4, 3, 2))
    C[:, 0, 0] = 1.0
    C[:, 2, 0] = 2.0
    C[2, 0, :] = [0.6, 0.25]            # rho in [0.35, 0.85]
    U = o.from_legendre(C)
    want = math.sqrt(gamma * (gamma - 1.0) * 2.0 / 0.35)
    assert math.isclose(o.a0(U)[0], want, rel_tol=1e-14)
    assert math.isclose(o.trial_dt(U), 0.3 * 0.25 / want, rel_tol=1e-14)


def test_wave_speed_of_a_state_without_sound_speed():
    """A trace with p < 0 (inadmissible, e.g. from rounding near vacuum) has
    no real sound speed; its speed is the flow speed |w_d|, never NaN, so the
    Lax--Friedrichs alpha of its face still bounds |w_d|."""
    o = oracle.CRKDG(oracle.Problem(dim=2, n=(2, 2), system="euler", k=1))
    rho, mx, my = 0.5, 0.4, -0.9
    E = 0.5 * (mx * mx + my * my) / rho - 0.01          # rho e = -0.01
    u = np.array([[rho, mx, my, E]])
    s = [float(o.wave_speed(u, dd)[0]) for dd in range(2)]
    assert s == [abs(mx / rho), abs(my / rho)]
    # the Lax--Friedrichs flux on a face where one trace lacks a sound speed
    up = np.array([[[1.0, 0.0, 0.0, 2.5]]])              # p = 1 at rest: c = sqrt(1.4)
    um = u[None, :, :]
    f = o.lf_flux(um, up, 1, 1)
    alpha = max(abs(my / rho), math.sqrt(1.4))
    want = 0.5 * (o.flux(um, 1) + o.flux(up, 1)) - 0.5 * alpha * (up - um)
    np.testing.assert_allclose(f, want, rtol=1e-15)
