"""3D P^2 (total degree) Euler, built in the mixed form only: every stage and
three controller steps against the FP64 oracle, and the FP64 form refused at
init."""
import math
import sys

import numpy as np
import pytest

import oracle
from _helpers import gpu_problem, oracle_problem, random_state, rel_err_per_var, round_hi

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

PARAMS = dict(dim=3, n=(7, 6, 5), system="euler", k=2, space="P", stages=3, cfl=0.15)


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_16002_amd import crkdg
    return crkdg


def _setup(lib, precision="mixed"):
    params = dict(PARAMS, precision=precision)
    return oracle.CRKDG(oracle_problem(params)), lib.Mesh(gpu_problem(params))


def test_fp64_form_not_built(lib):
    with pytest.raises(lib.CRKDGError) as e:
        _setup(lib, "fp64")
    assert e.value.code == lib.E_UNSUPPORTED


def test_mixed_stage_parity(lib):
    """Each stage from identical (FP32-representable) inputs within 1e-5 of
    the variable's magnitude, averages within 1e-6; limited points in B^eps."""
    o, mesh = _setup(lib)
    s = o.p.stages
    tilde = [round_hi(random_state(o, seed=170 + j, rel_amp=0.1), "mixed") for j in range(s)]
    U = [o.from_legendre(c) for c in tilde]
    dt = 0.8 * o.trial_dt(U[0])
    states = []
    for c in tilde:
        st = mesh.new_state()
        mesh.set_legendre(st, c)
        states.append(st)
    out = mesh.new_state()
    ctl = mesh.new_ctl()
    for i in range(2, s + 2):
        _say(f"[3D P2 mixed stage] stage {i}")
        ref = o.to_legendre(o.limit(o.stage(i, U[0], U, dt))[0])
        mesh.ctl_write(ctl, [{"dt": dt}])
        mesh.stage(i, states, out, ctl)
        got = mesh.get_legendre(out)
        err = rel_err_per_var(got, ref)
        err0 = rel_err_per_var(got[:, :, :1], ref[:, :, :1])
        _say(f"   rel err {err:.2e} (averages {err0:.2e}) flags {mesh.ctl_read(ctl)[0]['flags']}")
        assert err < 1e-5 and err0 < 1e-6
        assert o.bound_violations(o.from_legendre(got)) == 0


def test_mixed_step_parity(lib):
    """Three accepted steps through the device controller against the
    oracle's steps (1e-5 of the variable's magnitude), conserved totals."""
    o, mesh = _setup(lib)
    C0 = round_hi(random_state(o, seed=181, rel_amp=0.1), "mixed")
    slots = mesh.new_slots()
    mesh.set_legendre(slots[0], C0)
    ctl = mesh.new_ctl()
    mesh.start(slots, ctl, t0=0.0)
    T0 = mesh.totals(slots[0]).cpu().numpy().copy()
    U = o.from_legendre(C0)
    t = 0.0
    for n in range(3):
        _say(f"[3D P2 mixed step] step {n}")
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


def test_mixed_density_wave_converges(lib):
    """The exact 3D density wave (rho = 1 + 0.5 sin(2 pi (x + y + z - 3t)))
    at 8^3, 16^3, 32^3 to t = 0.01: the error falls at order k+1 = 3
    (measured rates 2.97, 3.04)."""
    from test_gpu_convergence import _error
    errs = []
    for n in (8, 16, 32):
        e, steps = _error(lib, 3, n, 2, "mixed", 0.01, space="P")
        errs.append(e)
        _say(f"[wave 3D P2 mixed] n = {n}: {steps} steps, relative L1 error of rho {e:.3e}")
    rates = [math.log2(a / b) for a, b in zip(errs, errs[1:])]
    _say(f"[wave 3D P2 mixed] rates {['%.2f' % r for r in rates]}")
    assert rates[-1] > 3 - 0.3
