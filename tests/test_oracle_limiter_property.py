"""The limiter-property check the GPU parity tests apply to cells whose
density step pins rho at eps (no GPU): the oracle's own limiter output
satisfies it on heavily limited Euler data in 1D, 2D and 3D (eps 1e-8 and
1e-13), and plausible mistakes fail it -- a density factor smaller than
needed, a theta above 1, momentum and energy scaled differently, a changed
average, modes not proportional to the unlimited ones."""
import numpy as np
import pytest

import oracle
from paper_2412_16002_amd import inputs
from _helpers import check_limiter_property, pinned_cells, random_state

CASES = [dict(dim=1, n=(200,), k=3, eps=1e-13), dict(dim=2, n=(9, 8), k=2, eps=1e-8),
         dict(dim=3, n=(4, 3, 3), k=1, eps=1e-8)]


def _limited(case, seed=7):
    o = oracle.CRKDG(oracle.Problem(system="euler", stages=3, **case))
    # low densities and pressures: many cells need the density step
    avg = inputs.random_euler_averages(o.ncell, o.d, seed=seed, rho=(1e-3, 1e-1), p=(1e-3, 1e-1))
    C = random_state(o, seed=seed, rel_amp=6.0, limited=False, avg=avg)
    L = o.to_legendre(o.limit(o.from_legendre(C))[0])
    return o, C, L


@pytest.mark.parametrize("case", CASES, ids=["1d_p3", "2d_q2", "3d_q1"])
def test_the_oracle_limiter_has_the_property(case):
    o, C, L = _limited(case)
    cells = pinned_cells(o, C)
    assert cells.sum() >= 3, "the data must pin some cells at eps"
    check_limiter_property(o, C, L, cells)


@pytest.mark.parametrize("case", CASES, ids=["1d_p3", "2d_q2", "3d_q1"])
def test_planted_mistakes_fail(case):
    o, C, L = _limited(case)
    cells = np.flatnonzero(pinned_cells(o, C))
    # the pinned cell with the largest factor (a flattened one hides changes)
    ratio = np.sum(np.abs(L[cells, -1, 1:]), axis=1) / np.sum(np.abs(C[cells, -1, 1:]), axis=1)
    c = cells[np.argmax(ratio)]

    def fails(G):
        with pytest.raises(AssertionError):
            check_limiter_property(o, C, G, cells)

    dens = np.flatnonzero(pinned_cells(o, C))
    G = L.copy(); G[dens, 0, 1:] *= 0.5; fails(G)                   # density factor smaller than needed
    G = L.copy(); G[c, :, 1:] = 1.5 * C[c, :, 1:]; fails(G)         # theta above 1
    G = L.copy(); G[c, -1, 1:] *= 0.9; fails(G)                     # energy scaled apart from momentum
    G = L.copy(); G[c, 0, 0] *= 1.001; fails(G)                     # average changed
    G = L.copy(); G[c, 1, 1] += 1e-3 * np.max(np.abs(C[:, 1])); fails(G)   # not a multiple
