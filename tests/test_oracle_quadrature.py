"""Pins of the oracle's one-dimensional rules, bases and the S_K point set
against closed forms (no GPU)."""
import itertools
import math

import numpy as np
import pytest

from oracle import CRKDG, EULER, ADVECTION, Problem, gauss_legendre, gauss_lobatto, legendre_table
from oracle.crkdg_oracle import lagrange_1d


def test_gauss_closed_forms():
    x, w = gauss_legendre(2)
    assert np.allclose(x, [-1 / math.sqrt(3), 1 / math.sqrt(3)], atol=1e-15)
    assert np.allclose(w, [1.0, 1.0], atol=1e-15)
    x, w = gauss_legendre(3)
    assert np.allclose(x, [-math.sqrt(0.6), 0.0, math.sqrt(0.6)], atol=1e-15)
    assert np.allclose(w, [5 / 9, 8 / 9, 5 / 9], atol=1e-15)
    x, w = gauss_legendre(4)
    a = math.sqrt(3 / 7 - 2 / 7 * math.sqrt(6 / 5))
    b = math.sqrt(3 / 7 + 2 / 7 * math.sqrt(6 / 5))
    assert np.allclose(x, [-b, -a, a, b], atol=1e-15)
    wa, wb = (18 + math.sqrt(30)) / 36, (18 - math.sqrt(30)) / 36
    assert np.allclose(w, [wb, wa, wa, wb], atol=1e-15)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_gauss_exactness(n):
    x, w = gauss_legendre(n)
    for deg in range(2 * n):
        exact = 0.0 if deg % 2 else 2.0 / (deg + 1)
        assert abs(np.sum(w * x ** deg) - exact) < 1e-14
    # and not exact one degree higher (degree 2n)
    assert abs(np.sum(w * x ** (2 * n)) - 2.0 / (2 * n + 1)) > 1e-6


def test_lobatto_closed_forms_and_exactness():
    x, w = gauss_lobatto(2)
    assert np.allclose(x, [-1, 1]) and np.allclose(w, [1, 1])
    x, w = gauss_lobatto(3)
    assert np.allclose(x, [-1, 0, 1], atol=1e-15)
    assert np.allclose(w, [1 / 3, 4 / 3, 1 / 3], atol=1e-15)
    for N in (2, 3, 4, 5):
        x, w = gauss_lobatto(N)
        for deg in range(2 * N - 2):
            exact = 0.0 if deg % 2 else 2.0 / (deg + 1)
            assert abs(np.sum(w * x ** deg) - exact) < 1e-13


def test_legendre_closed_forms():
    x = np.linspace(-1, 1, 17)
    P, dP = legendre_table(4, x)
    assert np.allclose(P[2], (3 * x ** 2 - 1) / 2, atol=1e-15)
    assert np.allclose(P[3], (5 * x ** 3 - 3 * x) / 2, atol=1e-15)
    assert np.allclose(P[4], (35 * x ** 4 - 30 * x ** 2 + 3) / 8, atol=1e-14)
    assert np.allclose(dP[3], (15 * x ** 2 - 3) / 2, atol=1e-14)
    assert np.allclose(dP[4], (140 * x ** 3 - 60 * x) / 8, atol=1e-13)
    assert np.allclose(P[:, -1], 1.0) and np.allclose(P[:, 0], [(-1) ** n for n in range(5)])


def test_lagrange_interpolates_and_differentiates():
    nodes, _ = gauss_legendre(4)
    x = np.linspace(-1, 1, 11)
    L, dL = lagrange_1d(nodes, x)
    # reproduces cubic polynomials and their derivatives exactly
    coef = np.array([0.3, -1.2, 0.7, 2.0])
    f = np.polynomial.polynomial.polyval(nodes, coef)
    assert np.allclose(f @ L, np.polynomial.polynomial.polyval(x, coef), atol=1e-13)
    dcoef = np.polynomial.polynomial.polyder(coef)
    assert np.allclose(f @ dL, np.polynomial.polynomial.polyval(x, dcoef), atol=1e-12)


@pytest.mark.parametrize("dim,k,space,nsk", [
    (1, 1, "Q", 2), (1, 2, "Q", 3), (1, 3, "Q", 3),
    (2, 1, "Q", 8), (2, 2, "Q", 17), (2, 3, "Q", 24), (2, 2, "P", 17),
    (3, 2, "Q", 73), (3, 1, "Q", 24),
])
def test_sk_point_count_and_faces(dim, k, space, nsk):
    o = CRKDG(Problem(dim=dim, n=(2,) * dim, system=ADVECTION, k=k, space=space))
    assert len(o.xs) == nsk
    # S_K contains every face quadrature point (Prop. 2.2)
    for f in o.faces:
        for p in f["pts"]:
            assert np.min(np.max(np.abs(o.xs - p), axis=1)) < 1e-14


@pytest.mark.parametrize("dim,k,space", [(1, 2, "Q"), (2, 2, "Q"), (2, 3, "P"), (3, 1, "Q")])
def test_sk_convex_decomposition_of_average(dim, k, space):
    """The tensor Gauss x Lobatto rules of S_K average a polynomial of the
    space exactly (Prop. 2.2); their mean is the convex decomposition."""
    o = CRKDG(Problem(dim=dim, n=(1,) * dim, system=ADVECTION, k=k, space=space))
    g, wg = gauss_legendre(k + 1)
    gl, wl = gauss_lobatto(2 if k == 1 else 3)
    rng = np.random.default_rng(1)
    U = rng.standard_normal((1, 1, o.M))
    avg = o.cell_average(U)[0, 0]
    for d in range(dim):
        axes = [(gl, wl) if j == d else (g, wg) for j in range(dim)]
        pts, wts = [], []
        for combo in itertools.product(*[list(zip(*a)) for a in axes]):
            pts.append([c[0] for c in combo])
            wts.append(np.prod([c[1] for c in combo]) / 2 ** dim)
        vals = o.evaluate(U, np.array(pts))[0, 0]
        assert abs(np.dot(wts, vals) - avg) < 1e-13


@pytest.mark.parametrize("dim,k,space", [(1, 3, "Q"), (2, 2, "Q"), (2, 3, "P"), (3, 2, "Q")])
def test_legendre_roundtrip_and_mode_zero(dim, k, space):
    o = CRKDG(Problem(dim=dim, n=(3,) * dim, system=EULER, k=k, space=space))
    rng = np.random.default_rng(2)
    Cm = rng.standard_normal((o.ncell, o.V, o.M))
    U = o.from_legendre(Cm)
    assert np.allclose(o.to_legendre(U), Cm, atol=1e-13)
    assert np.allclose(o.cell_average(U), Cm[:, :, 0], atol=1e-13)
    # a single Legendre product evaluates to the product of numpy's Legendre series
    modes = o.legendre_modes()
    m = len(modes) - 1
    C1 = np.zeros((1, 1, o.M))
    C1[0, 0, m] = 1.0
    o1 = CRKDG(Problem(dim=dim, n=(1,) * dim, system=ADVECTION, k=k, space=space))
    x = rng.uniform(-1, 1, (7, dim))
    vals = o1.evaluate(o1.from_legendre(C1), x)[0, 0]
    ref = np.ones(7)
    for j in range(dim):
        e = np.zeros(modes[m][j] + 1)
        e[-1] = 1.0
        ref *= np.polynomial.legendre.legval(x[:, j], e)
    assert np.allclose(vals, ref, atol=1e-13)
