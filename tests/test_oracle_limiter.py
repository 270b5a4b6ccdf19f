"""Pins of the oracle's scaling limiters (Prop. 2.4 scalar; Sec. 2.2.3 Euler)
and of the adaptive halving of Sec. 4.1 (no GPU)."""
import math

import numpy as np
import pytest

from oracle import ADVECTION, BURGERS, EULER, CRKDG, Problem

from paper_2412_16002_amd import inputs


def _one_cell(system, k=1, dim=1, **kw):
    return CRKDG(Problem(dim=dim, n=(1,) * dim, system=system, k=k, **kw))


def test_scalar_theta_hand_case():
    """P^1 cell with average 0.5 and end values 0.5 -+ 1.0 on B = [0, 1]:
    M_K = 1.5, m_K = -0.5, theta = min(|1-0.5|/|1.5-0.5|, |0-0.5|/|-0.5-0.5|) = 0.5,
    so the limited end values are 0 and 1."""
    o = _one_cell(ADVECTION, bound_lo=0.0, bound_hi=1.0)
    C = np.array([[[0.5, 1.0]]])                         # Legendre: ubar + c1 xi
    out, theta = o.limit(o.from_legendre(C))
    assert abs(theta[0] - 0.5) < 1e-15
    assert np.allclose(o.to_legendre(out), [[[0.5, 0.5]]], atol=1e-15)
    assert np.allclose(o.evaluate(out, np.array([[-1.0], [1.0]]))[0, 0], [0.0, 1.0], atol=1e-15)


def test_scalar_theta_only_violated_bound_acts():
    """Only the violated side enters theta: upper excursion 0.2 above M with
    the average 0.4 below M gives theta = 0.4 / 0.6."""
    o = _one_cell(ADVECTION, k=2, bound_lo=-5.0, bound_hi=1.0)
    # u = 0.6 + 0.6 xi on [-1,1] -> values 0 .. 1.2 at the Lobatto ends
    C = np.array([[[0.6, 0.6, 0.0]]])
    out, theta = o.limit(o.from_legendre(C))
    assert abs(theta[0] - 0.4 / 0.6) < 1e-14


def test_euler_density_step_hand_case():
    """Density step: rho = 1 + 2 xi at the Lobatto ends is -1 .. 3;
    theta_1 = (1 - eps)/(1 - (-1)) = (1 - eps)/2, so the limited minimum is eps."""
    eps = 1e-8
    o = _one_cell(EULER, eps=eps)
    avg = inputs.conservative(1.0, [0.0], 10.0)
    C = np.zeros((1, 3, 2))
    C[0, :, 0] = avg
    C[0, 0, 1] = 2.0
    out, theta = o.limit(o.from_legendre(C))
    Cl = o.to_legendre(out)
    assert abs(Cl[0, 0, 1] - 2.0 * (1 - eps) / 2) < 1e-15
    vals = o.sk_values(out)[0]
    assert abs(vals[:, 0].min() - eps) < 1e-15
    assert np.allclose(Cl[0, :, 0], avg, atol=1e-15)


def test_euler_energy_step_hand_case():
    """Internal-energy step with constant density and momentum: rho e = E - m^2/(2 rho)
    is linear, E = Ebar + c xi; theta_2 = (rhoe_bar - eps) / (rhoe_bar - min rhoe)."""
    eps = 1e-8
    o = _one_cell(EULER, eps=eps)
    rho, m, Eb = 1.0, 1.0, 1.0          # rhoe_bar = 1 - 0.5 = 0.5
    C = np.zeros((1, 3, 2))
    C[0, :, 0] = [rho, m, Eb]
    C[0, 2, 1] = 1.0                    # E from 0 to 2: rhoe from -0.5 to 1.5
    out, theta = o.limit(o.from_legendre(C))
    th2 = (0.5 - eps) / (0.5 - (-0.5))
    assert abs(theta[0] - th2) < 1e-15
    assert abs(o.to_legendre(out)[0, 2, 1] - th2) < 1e-15


@pytest.mark.parametrize("system,dim,k,space", [(BURGERS, 1, 2, "Q"), (EULER, 1, 3, "Q"), (EULER, 2, 2, "Q"),
                                                (EULER, 2, 3, "P"), (ADVECTION, 3, 1, "Q")])
def test_limiter_properties(system, dim, k, space):
    """Averages unchanged, every S_K value inside B / B^eps after limiting,
    idempotent (L(L(u)) = L(u)), identity on admissible data."""
    o = CRKDG(Problem(dim=dim, n=(12,) if dim == 1 else (6,) * dim, system=system, k=k, space=space,
                      bound_lo=0.0, bound_hi=1.0))
    rng = np.random.default_rng(12)
    if system == EULER:
        avg = inputs.random_euler_averages(o.ncell, dim, seed=12, p=(0.01, 0.5))
    else:
        avg = rng.uniform(0.05, 0.95, (o.ncell, 1))
    C = inputs.random_legendre(o.ncell, o.V, o.M, [sum(e) for e in o.legendre_modes()], seed=13, avg=avg,
                               rel_amp=3.0)
    U = o.from_legendre(C)
    L1, th = o.limit(U)
    assert np.mean(th < 1) > 0.15
    assert np.allclose(o.cell_average(L1), o.cell_average(U), atol=1e-14)
    assert o.bound_violations(L1) == 0
    L2, th2 = o.limit(L1)
    assert np.max(np.abs(L2 - L1)) < 1e-12
    assert np.all(th2 > 1 - 1e-9)
    # admissible data are left unchanged
    C_small = inputs.random_legendre(o.ncell, o.V, o.M, [sum(e) for e in o.legendre_modes()], seed=14,
                                     avg=avg, rel_amp=0.01)
    Us = o.from_legendre(C_small)
    assert np.array_equal(o.limit(Us)[0], Us)


def test_forced_rejections_halve_and_recover():
    """Sec. 4.1: a trial step far above the stability limit produces stage
    averages outside B, the step is halved and restarted from u^n until it
    is accepted; the accepted result is inside the bounds."""
    lo_b, hi_b = 0.2, 1.0
    o = CRKDG(Problem(dim=1, n=(40,), system=BURGERS, k=2, stages=3, bound_lo=lo_b, bound_hi=hi_b))
    U = o.limit(o.project(lambda x: (0.6 + 0.39 * np.sign(np.sin(2 * np.pi * x[..., 0])))[..., None]))[0]
    U1, info = o.step(U, dt_fixed=20.0 * o.dx[0])
    assert info["halvings"] >= 3
    assert o.bound_violations(U1) == 0
    assert np.all(o.admissible_average(o.cell_average(U1)))
    assert math.isclose(info["dt"], 20.0 * o.dx[0] / 2 ** info["halvings"], rel_tol=1e-15)


def test_inadmissible_data_underflow():
    """An average outside B can never be repaired by halving: the step ends
    with a time-step underflow after max_halvings."""
    o = CRKDG(Problem(dim=1, n=(8,), system=BURGERS, k=1, stages=2, bound_lo=0.0, bound_hi=1.0,
                      max_halvings=5))
    C = np.zeros((8, 1, 2))
    C[:, 0, 0] = 0.5
    C[3, 0, 0] = 1.5
    with pytest.raises(RuntimeError, match="underflow"):
        o.step(o.from_legendre(C), dt_fixed=0.01)


def test_nonfinite_state_is_rejected():
    o = CRKDG(Problem(dim=1, n=(8,), system=EULER, k=1, stages=2, max_halvings=3))
    avg = inputs.random_euler_averages(8, 1, seed=1)
    C = np.zeros((8, 3, 2))
    C[:, :, 0] = avg
    C[5, 2, 0] = np.nan
    assert not np.all(o.admissible_average(o.cell_average(o.from_legendre(C))))
    with pytest.raises(RuntimeError):
        o.step(o.from_legendre(C), dt_fixed=1e-3)
