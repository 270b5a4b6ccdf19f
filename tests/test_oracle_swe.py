"""Pins of the oracle's shallow-water system (flat bottom; reading A28) on
the CPU, against facts other than the oracle:

* the exact Riemann solver of the tests: Rankine--Hugoniot conditions across
  its shocks, the Riemann invariant u + 2 sqrt(g h) across its rarefactions,
  the closed-form dry-bed fan, and the mass of its solution;
* the flux Jacobian (central differences of the oracle's flux) has the
  eigenvalues w_d +- sqrt(g h) (and w_d in 2D), whose largest magnitude is
  the oracle's wave speed;
* still water stays still, to rounding, in both operators;
* the manufactured solution's source (chain rule) is the residual of the
  oracle's flux, and the scheme converges at order k+1 on it;
* the limiter: averages kept, one factor for every component, min h over
  S_K = eps exactly where it acts;
* dam breaks against the exact solution (depth ratios 2 and 4: relative L1
  of h, no violations).  Nearly dry beds are not run: there the limiter
  holds h at eps at some S_K point while the discharge there stays O(1),
  so the wave-speed maximum over S_K (reading A5) and the trial step
  collapse (a velocity desingularisation would be needed, which the paper
  does not give)."""
import math

import numpy as np
import pytest

import oracle
import _swe_riemann as R
from paper_2412_16002_amd import inputs


def _problem(d, k=2, **kw):
    base = dict(dim=d, n=(6,) * d, system=oracle.SHALLOW_WATER, k=k, gravity=1.3, eps=1e-8)
    base.update(kw)
    return oracle.Problem(**base)


def test_exact_riemann_solver():
    g = 1.3
    for hl, ul, hr, ur in [(2.0, 0.0, 1.0, 0.0), (1.0, 0.5, 1.5, -0.3), (3.0, -0.2, 0.5, 0.4)]:
        hs, us = R.star_state(hl, ul, hr, ur, g)
        for side, (hk, uk) in ((-1, (hl, ul)), (1, (hr, ur))):
            if hs > hk:   # shock: the jump satisfies both Rankine-Hugoniot conditions
                s = uk + side * math.sqrt(g * hk) * math.sqrt(0.5 * (hs + hk) * hs / (hk * hk))
                assert abs(s * (hs - hk) - (hs * us - hk * uk)) < 1e-12
                fk = hk * uk * uk + 0.5 * g * hk * hk
                fs = hs * us * us + 0.5 * g * hs * hs
                assert abs(s * (hs * us - hk * uk) - (fs - fk)) < 1e-11
            else:         # rarefaction: u -+ 2 sqrt(g h) is constant across it
                assert abs((us - side * 2 * math.sqrt(g * hs)) - (uk - side * 2 * math.sqrt(g * hk))) < 1e-12
    # dry bed: the fan h = (u_L + 2 a_L - xi)^2 / (9 g) ends at u_L + 2 a_L
    xi = np.linspace(-2.0, 3.0, 101)
    h, u = R.sample(xi, 2.0, 0.0, 0.0, 0.0, g)
    al = math.sqrt(g * 2.0)
    fan = (xi > -al) & (xi < 2 * al)
    assert np.allclose(h[fan], (2 * al - xi[fan]) ** 2 / (9 * g))
    assert np.all(h[xi >= 2 * al] == 0.0) and np.all(h[xi <= -al] == 2.0)
    # mass of the wet-bed solution on [-1, 1] at t = 0.3 equals the initial mass
    hav, _ = R.cell_averages(-1.0, 1.0, 400, 0.3, 2.0, 0.0, 1.0, 0.0, g, sub=256)
    assert abs(hav.mean() * 2.0 - 3.0) < 1e-6


@pytest.mark.parametrize("d", [1, 2])
def test_flux_jacobian_eigenvalues(d):
    o = oracle.CRKDG(_problem(d))
    rng = np.random.default_rng(4)
    for _ in range(20):
        h = rng.uniform(0.2, 3.0)
        w = rng.uniform(-2.0, 2.0, d)
        u = inputs.swe_conservative(h, w)
        for dd in range(d):
            J = np.empty((d + 1, d + 1))
            for j in range(d + 1):
                e = np.zeros(d + 1)
                e[j] = 1e-6
                J[:, j] = (o.flux(u + e, dd) - o.flux(u - e, dd)) / 2e-6
            ev = np.sort(np.linalg.eigvals(J).real)
            c = math.sqrt(1.3 * h)
            expect = np.sort([w[dd] - c, w[dd] + c] + ([w[dd]] if d == 2 else []))
            assert np.allclose(ev, expect, atol=1e-7)
            assert abs(o.wave_speed(u, dd) - np.max(np.abs(expect))) < 1e-12


@pytest.mark.parametrize("d,k", [(1, 3), (2, 2)])
def test_still_water_stays_still(d, k):
    o = oracle.CRKDG(_problem(d, k))
    U = o.constant_state(np.tile(inputs.swe_conservative(1.7, np.zeros(d)), (o.ncell, 1)))
    assert np.max(np.abs(o.G(U))) < 1e-12 and np.max(np.abs(o.F(U))) < 1e-12


def test_manufactured_source_is_the_residual_of_the_flux():
    for d in (1, 2):
        o = oracle.CRKDG(oracle.Problem(dim=d, n=(2,) * d, system=oracle.SHALLOW_WATER, k=1, gravity=1.0))
        X = np.random.default_rng(5).uniform(0.0, 1.0, (40, d))
        h = 1e-5
        for t in (0.0, 0.2):
            ut = (inputs.swe_mms_exact(X, t + h) - inputs.swe_mms_exact(X, t - h)) / (2 * h)
            div = sum((o.flux(inputs.swe_mms_exact(X + h * np.eye(d)[i], t), i)
                       - o.flux(inputs.swe_mms_exact(X - h * np.eye(d)[i], t), i)) / (2 * h) for i in range(d))
            s = inputs.swe_mms_source(X, t)
            assert np.max(np.abs(ut + div - s)) < 1e-8 * np.max(np.abs(s)) + 1e-6
            T = inputs.swe_mms_source_terms(X)
            sep = sum(math.exp(-r * t) * T[p] for p, r in enumerate(inputs.SWE_MMS_RATES))
            assert np.max(np.abs(sep - s)) < 1e-12 * np.max(np.abs(s))


@pytest.mark.parametrize("k", [1, 2, 3])
def test_manufactured_solution_converges_at_order_k_plus_one(k):
    errs = []
    for n in (8, 16, 32):
        cs = inputs.swe_mms(1, n, k)
        prob = oracle.Problem(dim=1, n=(n,), system=oracle.SHALLOW_WATER, k=k, stages=k + 1, gravity=1.0,
                              source=cs.meta["source"])
        o = oracle.CRKDG(prob)
        U, t, _ = o.run(o.limit(o.project(cs.u0))[0], cs.t_end, dt_fixed=cs.meta["dt"])
        errs.append(float(np.sum(o.l1_norm(U, lambda X: cs.exact(X, t)))))
    rate = math.log2(errs[1] / errs[2])
    assert rate > k + 1 - 0.25, (errs, rate)


def test_limiter_scales_every_component_by_one_factor():
    o = oracle.CRKDG(_problem(2, k=2, n=(7, 5), eps=1e-3))
    rng = np.random.default_rng(6)
    avg = inputs.swe_conservative(rng.uniform(0.01, 0.5, o.ncell), rng.uniform(-1, 1, (o.ncell, 2)))
    C = inputs.random_legendre(o.ncell, o.V, o.M, [sum(e) for e in o.legendre_modes()], seed=7, avg=avg,
                               rel_amp=4.0)
    U = o.from_legendre(C)
    out, theta = o.limit(U)
    Co = o.to_legendre(out)
    assert np.array_equal(Co[:, :, 0], C[:, :, 0]) or np.allclose(Co[:, :, 0], C[:, :, 0], rtol=1e-15, atol=0)
    acted = theta < 1.0
    assert acted.mean() > 0.2
    # every component of a limited cell scaled by theta
    assert np.allclose(Co[:, :, 1:], theta[:, None, None] * C[:, :, 1:], rtol=1e-12, atol=1e-15)
    hs = np.einsum("cm,pm->cp", out[:, 0, :], o.phi_s)
    assert np.all(hs.min(axis=1) >= o.p.eps * (1 - 1e-12))
    assert np.allclose(hs.min(axis=1)[acted], o.p.eps, rtol=1e-9, atol=0)
    assert o.bound_violations(out) == 0


def _dam_break_oracle(case, k):
    pr = case.params
    prob = oracle.Problem(dim=1, n=pr["n"], system=oracle.SHALLOW_WATER, k=k, stages=pr["stages"],
                          lo=pr["lo"], hi=pr["hi"], bc=(oracle.DIRICHLET,), bc_state=pr["bc_state"],
                          gravity=pr["gravity"], eps=pr["eps"], cfl=pr["cfl"])
    o = oracle.CRKDG(prob)
    U = o.limit(o.constant_state(case.cell_states))[0]
    U, t, log = o.run(U, case.t_end)
    return o, U, t, log


def test_dam_break_against_the_exact_solution():
    cs = inputs.swe_dam_break_1d(n=200, k=2, h_left=2.0, h_right=1.0)
    o, U, t, log = _dam_break_oracle(cs, 2)
    hav, _ = R.cell_averages(-1.0, 1.0, 200, t, 2.0, 0.0, 1.0, 0.0, 1.0)
    h = o.cell_average(U)[:, 0]
    l1 = np.sum(np.abs(h - hav)) / np.sum(hav)
    assert l1 < 0.005, l1
    assert o.bound_violations(U) == 0
    # still water held at both ends: no mass crosses them
    assert abs(o.totals(U)[0] - 3.0) < 1e-12


def test_strong_dam_break_against_the_exact_solution():
    """Depth ratio 4 (2 onto 0.5): a stronger shock, same checks."""
    cs = inputs.swe_dam_break_1d(n=200, k=2, h_left=2.0, h_right=0.5, eps=1e-4, t_end=0.2)
    o, U, t, log = _dam_break_oracle(cs, 2)
    assert all(x["halvings"] == 0 for x in log)
    hav, _ = R.cell_averages(-1.0, 1.0, 200, t, 2.0, 0.0, 0.5, 0.0, 1.0)
    h = o.cell_average(U)[:, 0]
    assert np.sum(np.abs(h - hav)) / np.sum(hav) < 0.01
    assert o.bound_violations(U) == 0
