"""3D P^2, P^3 (total degree) and Q^3 Euler, FP64 and mixed precision,
through the cooperative tensor kernels (P^k held inside Q^k): three
controller steps of the mixed form against the FP64 oracle, and the exact
density wave at three resolutions in both forms, and blast runs with the
limiter at work.  Stage, limiter, step, boundary, alpha and
standard-RKDG parity of the same families run with the other families'
(test_gpu_parity, test_gpu_mixed_parity, test_gpu_boundaries,
test_gpu_alpha, test_gpu_rkdg)."""
import math
import sys

import numpy as np
import pytest

import oracle
from _helpers import gpu_problem, oracle_problem, random_state, rel_err_per_var, round_hi
from paper_2412_16002_amd import inputs
from test_gpu_parity import CASES

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_16002_amd import crkdg
    return crkdg


@pytest.mark.parametrize("name", ["euler3d_p2", "euler3d_p3", "euler3d_q3"])
def test_mixed_step_parity(lib, name):
    """Three accepted steps of the mixed form through the device controller
    against the oracle's FP64 steps (1e-5 of the variable's magnitude),
    totals conserved."""
    params = dict(CASES[name], precision="mixed")
    o, mesh = oracle.CRKDG(oracle_problem(params)), lib.Mesh(gpu_problem(params))
    C0 = round_hi(random_state(o, seed=181, rel_amp=0.1), "mixed")
    slots = mesh.new_slots()
    mesh.set_legendre(slots[0], C0)
    ctl = mesh.new_ctl()
    mesh.start(slots, ctl, t0=0.0)
    T0 = mesh.totals(slots[0]).cpu().numpy().copy()
    U = o.from_legendre(C0)
    t = 0.0
    for n in range(3):
        _say(f"[3D mixed step] {name} step {n}")
        U, info_o = o.step(U, t)
        t = info_o["t"]
        info = mesh.step(slots, ctl)[0]
        assert info["status"] == 0 and info["halvings"] == info_o["halvings"]
        assert math.isclose(info["dt"], info_o["dt"], rel_tol=1e-5)
        got = mesh.get_legendre(slots[info["cur"]])
        err = rel_err_per_var(got, o.to_legendre(U))
        _say(f"   dt {info['dt']:.4e} rel err {err:.2e}")
        assert err < 1e-5
        assert o.bound_violations(o.from_legendre(got)) == 0
    T = mesh.totals(slots[info["cur"]]).cpu().numpy()
    assert np.all(np.abs(T - T0) <= 1e-13 * np.maximum(np.abs(T0), 1.0))


@pytest.mark.parametrize("space,k,meshes,lo", [("P", 2, (8, 16, 32), 2.7), ("P", 3, (8, 16, 32), 3.4),
                                               ("Q", 3, (8, 16, 32), 3.4)])
def test_density_wave_converges(lib, space, k, meshes, lo):
    """The exact 3D density wave (rho = 1 + 0.5 sin(2 pi (x + y + z - 3t)))
    to t = 0.01: the relative L1 error of rho falls at about order k+1 in
    both forms (measured FP64 rates: P^2 2.97, 3.04; P^3 and Q^3 about 4),
    and the mixed form stays at the FP64 error."""
    from test_gpu_convergence import _error
    errs = {}
    for precision in ("fp64", "mixed"):
        errs[precision] = []
        for n in meshes:
            e, steps = _error(lib, 3, n, k, precision, 0.01, space=space)
            errs[precision].append(e)
            _say(f"[wave 3D {space}{k} {precision}] n = {n}: {steps} steps, relative L1 error of rho {e:.3e}")
        rates = [math.log2(a / b) for a, b in zip(errs[precision], errs[precision][1:])]
        _say(f"[wave 3D {space}{k} {precision}] rates {['%.2f' % r for r in rates]}")
        assert rates[-1] > lo
    # the mixed form at the FP64 error, up to its own rounding floor (FP32
    # modes: 3e-8 of relative L1 on 32^3 Q^3, where the FP64 error is 1.5e-7)
    for ef, em in zip(errs["fp64"], errs["mixed"]):
        assert abs(em - ef) <= 0.05 * ef + 1e-7


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("space,k", [("P", 2), ("P", 3), ("Q", 3)])
def test_blast_runs(lib, space, k, precision):
    """A 24^3 blast (p = 100 inside a seeded sphere, 1e-4 outside, rho = 1,
    w = 0) through the cooperative kernels: 20 accepted steps of the device
    controller (halvings allowed), totals conserved to 1e-12 of the largest,
    and no S_K point outside B^eps in any cell (oracle check)."""
    n = 24
    case = inputs.euler_3d_blast(seed=0, n=n, precision=precision)
    params = dict(case.params, precision=precision, k=k, space=space, stages=k + 1,
                  cfl={2: 0.15, 3: 0.09}[k])
    mesh = lib.Mesh(gpu_problem(params))
    slots = mesh.new_slots()
    a, h = mesh.views(slots[0])
    a.copy_(torch.from_numpy(case.cell_states.T.copy()))
    h.zero_()
    ctl = mesh.new_ctl()
    mesh.start(slots, ctl, t0=0.0)
    T0 = mesh.totals(slots[0]).cpu().numpy()
    halvings = 0
    for _ in range(20):
        info = mesh.step(slots, ctl)[0]
        assert info["status"] == 0
        halvings += info["halvings"]
    T1 = mesh.totals(slots[info["cur"]]).cpu().numpy()
    cons = np.abs(T1 - T0) / np.abs(T0).max()
    o = oracle.CRKDG(oracle_problem(params))
    U = o.from_legendre(mesh.get_legendre(slots[info["cur"]]))
    viol = o.bound_violations(U)
    _say(f"[blast 24^3] {space}{k} {precision}: t {info['t']:.3e}, halvings {halvings}, "
         f"totals change {cons.max():.1e}, violations {viol}")
    assert np.all(np.isfinite(U))
    assert np.all(cons <= 1e-12)
    assert viol == 0
