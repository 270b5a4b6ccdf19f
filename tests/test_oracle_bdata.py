"""Pins of time-dependent Dirichlet data in the oracle (reading A29), on the
CPU: data equal to a side's constant state reproduce that state bitwise;
the time-separable boundary terms of the inputs sum back to the exact
solutions; and Example 4.1 with its exact inflow data converges at the
printed rates of Table 1 (k = 2: 3.00), with errors a constant 0.42 of the
printed ones (the norm behind the printed figures is not stated; absolute
values stay unpinned)."""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle.crkdg_oracle import gauss_legendre
from _helpers import oracle_problem, random_state
from paper_2412_16002_amd import inputs


def _g(coef, t):
    return [math.exp(-r * t) * math.cos(w * t + ph) for r, w, ph in coef]


def test_constant_data_equals_the_constant_state():
    params = dict(dim=2, n=(6, 5), system="euler", k=2, stages=3, bc=("dirichlet", "periodic"),
                  bc_state={0: [1.1, 0.2, -0.1, 2.7], 1: [0.9, -0.3, 0.1, 2.2]})
    a = oracle.CRKDG(oracle_problem(params))
    pb = oracle_problem(params)
    pb.bc_function = {0: lambda X, t: np.broadcast_to([1.1, 0.2, -0.1, 2.7], X.shape[:-1] + (4,)),
                      1: lambda X, t: np.broadcast_to([0.9, -0.3, 0.1, 2.2], X.shape[:-1] + (4,))}
    b = oracle.CRKDG(pb)
    U = a.from_legendre(random_state(a, seed=3))
    assert np.array_equal(a.F(U), b.F(U, t=0.7))


def test_separable_terms_reproduce_the_exact_data():
    rng = np.random.default_rng(8)
    X = rng.uniform(0.0, 1.0, (50, 2))
    terms = inputs.scenario2_boundary_terms()
    for t in rng.uniform(0.0, 1.0, 5):
        sep = sum(g * G(X) for g, G in zip(_g(inputs.SCENARIO2_COEF, t), terms))
        assert np.allclose(sep, inputs.mms_euler2d_scenario2_exact(X, t), rtol=1e-14, atol=1e-14)
        cs = inputs.table1_advection(2, 0)
        sep1 = sum(g * G(X[:, :1]) for g, G in zip(_g(cs.meta["bc_coef"], t), cs.meta["bc_terms"]))
        assert np.allclose(sep1, cs.exact(np.zeros((50, 1)), t), rtol=1e-14, atol=1e-14)
        # the 3D density wave with exact data on its x and y sides
        cw = inputs.euler_wave_box3d(2, (4, 4, 4))
        X3 = rng.uniform(0.0, 1.0, (50, 3))
        sep3 = sum(g * G(X3) for g, G in zip(_g(cw.meta["bc_coef"], t), cw.meta["bc_terms"]))
        assert np.allclose(sep3, cw.exact(X3, t), rtol=1e-14, atol=1e-14)


def test_slab_share_input_is_periodic_over_the_slab():
    """The one-GPU share of the 3D wave (a z-slab of the 128^3 mesh with the
    wave's z frequency raised to the number of slabs) is periodic over the
    slab, so the periodic slab stands in for its neighbours without a seam."""
    cs = inputs.euler_3d_wave_slab(seed=0, n=16, parts=8)
    assert tuple(cs.params["n"]) == (16, 16, 2) and cs.params["hi"][2] == 1.0 / 8
    rng = np.random.default_rng(3)
    X = rng.uniform(0.0, 1.0, (40, 3)) * np.array([1.0, 1.0, 1.0 / 8])
    for t in (0.0, 0.3):
        shifted = X + np.array([0.0, 0.0, 1.0 / 8])
        assert np.allclose(cs.exact(X, t), cs.exact(shifted, t), rtol=1e-12, atol=1e-12)


def _l2(o, U, exact, t):
    g, w = gauss_legendre(o.k + 3)
    x = np.array(list(itertools.product(g, repeat=o.d)))[:, ::-1].copy()
    wt = np.array([np.prod(v) for v in itertools.product(w, repeat=o.d)])
    vals = o.evaluate(U, x)
    ex = np.transpose(exact(o.physical_points(x), t), (0, 2, 1))
    return math.sqrt(np.einsum("p,cvp->", wt, (vals - ex) ** 2) * o.vol / 2.0 ** o.d)


TABLE1_P2 = [4.641e-4, 5.822e-5, 7.272e-6]


def test_table1_with_exact_inflow():
    errs = []
    for level in range(3):
        cs = inputs.table1_advection(2, level)
        prob = oracle_problem(cs.params)
        prob.bc_function = {0: lambda X, t, e=cs.exact: e(X, t)}
        o = oracle.CRKDG(prob)
        U, t, _ = o.run(o.limit(o.project(cs.u0))[0], cs.t_end, dt_fixed=cs.meta["dt"])
        assert abs(t - cs.t_end) < 1e-12
        errs.append(_l2(o, U, cs.exact, t))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    ratios = [e / p for e, p in zip(errs, TABLE1_P2)]
    assert all(abs(r - 3.0) < 0.05 for r in rates), rates
    assert max(ratios) / min(ratios) < 1.05, ratios
