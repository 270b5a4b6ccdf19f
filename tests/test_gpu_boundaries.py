"""Reflective walls and Dirichlet / inflow sides on the GPU against the
oracle: every stage from random limited states (the sides see states that
differ from the prescribed ones), three adaptive steps through the device
controller, and the mixed form.  Boundaries enter only the final stage (F);
the inner stages (G) use no exterior data.  Sizes span several tiles plus a
ragged tail."""
import math
import sys

import numpy as np
import pytest

import oracle
from _helpers import gpu_problem, oracle_problem, limited_err, random_state, rel_err_per_var, round_hi

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


def _cons(rho, w, p, gamma=1.4):
    w = np.asarray(w, dtype=float)
    return [rho] + list(rho * w) + [p / (gamma - 1.0) + 0.5 * rho * float(w @ w)]


# the Lax data of the 1D Euler example (given as rho, u, p)
LAX_L, LAX_R = _cons(0.445, [0.698], 3.528), _cons(0.5, [0.0], 0.571)

CASES = {
    "euler1d_p3_dirichlet": dict(dim=1, n=(517,), system="euler", k=3, stages=4, cfl=0.09, bc=("dirichlet",),
                                 bc_state={0: LAX_L, 1: LAX_R}),
    "euler1d_p2_walls": dict(dim=1, n=(300,), system="euler", k=2, stages=3, cfl=0.15, bc=("reflect",)),
    "euler2d_q2_quadrant": dict(dim=2, n=(23, 19), system="euler", k=2, stages=3, cfl=0.15,
                                bc=("reflect", "reflect"), bc_upper=("outflow", "outflow")),
    "euler2d_q1_mixed_sides": dict(dim=2, n=(21, 17), system="euler", k=1, stages=2, cfl=0.3,
                                   bc=("outflow", "dirichlet"), bc_upper=("reflect", "outflow"),
                                   bc_state={2: _cons(0.8, [0.2, 0.5], 0.7)}),
    "euler2d_p2_walls": dict(dim=2, n=(19, 17), system="euler", k=2, space="P", stages=3, cfl=0.15,
                             bc=("reflect", "dirichlet"), bc_upper=("reflect", "dirichlet"),
                             bc_state={2: _cons(1.0, [0.1, 0.3], 1.0), 3: _cons(0.2, [0.0, -0.4], 0.3)}),
    "adv1d_inflow": dict(dim=1, n=(301,), system="advection", k=2, stages=3, vel=(1.0, 0, 0), bc=("dirichlet",),
                         bc_upper=("outflow",), bc_state={0: [1.9]}, bound_lo=1.0, bound_hi=2.0, cfl=0.1),
    "adv2d_q2_inflow": dict(dim=2, n=(20, 21), system="advection", k=2, stages=3, vel=(0.7, -1.1, 0),
                            bc=("dirichlet", "outflow"), bc_upper=("outflow", "dirichlet"),
                            bc_state={0: [0.3], 3: [1.7]}, bound_lo=0.0, bound_hi=2.0, cfl=0.15),
    "euler3d_q1_sides": dict(dim=3, n=(9, 7, 8), system="euler", k=1, stages=2, cfl=0.3,
                             bc=("dirichlet", "periodic", "reflect"), bc_upper=("outflow", "periodic", "reflect"),
                             bc_state={0: _cons(0.9, [0.3, 0.0, -0.1], 1.1)}),
    "euler3d_p1_sides": dict(dim=3, n=(9, 7, 8), system="euler", k=1, space="P", stages=2, cfl=0.3,
                             bc=("reflect", "dirichlet", "periodic"), bc_upper=("outflow", "reflect", "periodic"),
                             bc_state={2: _cons(1.1, [0.2, 0.3, 0.0], 0.8)}),
    "euler3d_q2_sides": dict(dim=3, n=(9, 6, 5), system="euler", k=2, stages=4, cfl=0.15,
                             bc=("reflect", "periodic", "dirichlet"), bc_upper=("reflect", "periodic", "outflow"),
                             bc_state={4: _cons(1.2, [0.0, 0.2, 0.4], 0.9)}),
    "euler3d_p2_sides": dict(dim=3, n=(19, 5, 3), system="euler", k=2, space="P", stages=3, cfl=0.15,
                             bc=("dirichlet", "reflect", "periodic"), bc_upper=("reflect", "outflow", "periodic"),
                             bc_state={0: _cons(0.8, [0.4, -0.1, 0.2], 1.0)}),
    "euler3d_p3_sides": dict(dim=3, n=(19, 5, 3), system="euler", k=3, space="P", stages=4, cfl=0.09,
                             bc=("periodic", "reflect", "dirichlet"), bc_upper=("periodic", "reflect", "outflow"),
                             bc_state={4: _cons(1.1, [0.1, 0.0, 0.3], 0.9)}),
    "euler3d_q3_sides": dict(dim=3, n=(19, 5, 3), system="euler", k=3, stages=4, cfl=0.09,
                             bc=("reflect", "dirichlet", "periodic"), bc_upper=("outflow", "reflect", "periodic"),
                             bc_state={2: _cons(0.9, [0.2, 0.1, -0.3], 1.2)}),
    "adv3d_q3_inflow": dict(dim=3, n=(19, 5, 3), system="advection", k=3, stages=4, vel=(1.0, -0.5, 0.3),
                            bc=("dirichlet", "periodic", "outflow"), bc_upper=("outflow", "periodic", "dirichlet"),
                            bc_state={0: [1.6], 5: [0.4]}, bound_lo=0.0, bound_hi=2.0, cfl=0.09),
    "euler2d_q3_walls": dict(dim=2, n=(13, 11), system="euler", k=3, stages=4, cfl=0.09,
                             bc=("reflect", "dirichlet"), bc_upper=("outflow", "reflect"),
                             bc_state={2: _cons(0.7, [0.1, 0.2], 0.6)}),
}
FP64_TOL = 1e-12


def _setup(lib, name, precision="fp64"):
    params = dict(CASES[name], precision=precision)
    return params, oracle.CRKDG(oracle_problem(params)), lib.Mesh(gpu_problem(params))


def _states(mesh, coeffs):
    out = []
    for c in coeffs:
        st = mesh.new_state()
        mesh.set_legendre(st, c)
        out.append(st)
    return out


@pytest.mark.parametrize("name", list(CASES))
def test_boundary_stage_parity(lib, name):
    params, o, mesh = _setup(lib, name)
    s = o.p.stages
    tilde = [random_state(o, seed=120 + j, rel_amp=0.1) for j in range(s)]
    U = [o.from_legendre(c) for c in tilde]
    dt = 0.8 * o.trial_dt(U[0])
    states = _states(mesh, tilde)
    out = mesh.new_state()
    ctl = mesh.new_ctl()
    for i in range(2, s + 2):
        _say(f"[bc stage] {name} stage {i}")
        ref_u = o.stage(i, U[0], U, dt)
        ok_ref = bool(np.all(o.admissible_average(o.cell_average(ref_u))))
        ref = o.to_legendre(o.limit(ref_u)[0])
        mesh.ctl_write(ctl, [{"dt": dt}])
        mesh.stage(i, states, out, ctl)
        got = mesh.get_legendre(out)
        c = mesh.ctl_read(ctl)[0]
        err = limited_err(o, o.to_legendre(ref_u), got, ref, FP64_TOL)
        _say(f"   error/tolerance {err:.2e} flags {c['flags']} oracle-admissible {ok_ref}")
        assert (c["flags"] == 0) == ok_ref
        assert err < 1.0


@pytest.mark.parametrize("name", list(CASES))
def test_boundary_step_parity(lib, name):
    """Three accepted steps (adaptive dt, limiter, device controller)."""
    params, o, mesh = _setup(lib, name)
    C0 = random_state(o, seed=131, rel_amp=0.1)
    slots = mesh.new_slots()
    mesh.set_legendre(slots[0], C0)
    ctl = mesh.new_ctl()
    mesh.start(slots, ctl, t0=0.0)
    U = o.from_legendre(C0)
    t = 0.0
    for n in range(3):
        _say(f"[bc step] {name} step {n}")
        U, info_o = o.step(U, t)
        t = info_o["t"]
        info = mesh.step(slots, ctl)[0]
        assert info["status"] == 0 and info["halvings"] == info_o["halvings"]
        assert math.isclose(info["dt"], info_o["dt"], rel_tol=1e-12)
        got = mesh.get_legendre(slots[info["cur"]])
        err = rel_err_per_var(got, o.to_legendre(U))
        _say(f"   dt {info['dt']:.4e} rel err {err:.2e}")
        assert err < 10 * FP64_TOL
        assert o.bound_violations(o.from_legendre(got)) == 0


@pytest.mark.parametrize("name", ["euler1d_p3_dirichlet", "euler2d_q2_quadrant", "adv2d_q2_inflow",
                                  "euler3d_q2_sides", "euler2d_q3_walls"])
def test_boundary_mixed_stage_parity(lib, name):
    params, o, mesh = _setup(lib, name, precision="mixed")
    s = o.p.stages
    tilde = [round_hi(random_state(o, seed=140 + j, rel_amp=0.1), "mixed") for j in range(s)]
    U = [o.from_legendre(c) for c in tilde]
    dt = 0.8 * o.trial_dt(U[0])
    states = _states(mesh, tilde)
    out = mesh.new_state()
    ctl = mesh.new_ctl()
    for i in range(2, s + 2):
        _say(f"[bc mixed stage] {name} stage {i}")
        ref = o.to_legendre(o.limit(o.stage(i, U[0], U, dt))[0])
        mesh.ctl_write(ctl, [{"dt": dt}])
        mesh.stage(i, states, out, ctl)
        got = mesh.get_legendre(out)
        err, err0 = rel_err_per_var(got, ref), rel_err_per_var(got[:, :, :1], ref[:, :, :1])
        _say(f"   rel err {err:.2e} (averages {err0:.2e})")
        assert err < 1e-5 and err0 < 1e-6
        assert o.bound_violations(o.from_legendre(got)) == 0


def test_inflow_mass_rate_on_gpu(lib):
    """Advection inflow on the GPU: every accepted step adds dt a (g - u_R)
    to the total (u0 = 1, inflow 2, a = 1), in FP64 and in the mixed form
    (FP64 averages and mode-0 face sums)."""
    for precision in ("fp64", "mixed"):
        params = dict(dim=1, n=(300,), system="advection", k=2, stages=3, vel=(1.0, 0, 0), bc=("dirichlet",),
                      bc_upper=("outflow",), bc_state={0: [2.0]}, bound_lo=1.0, bound_hi=2.0, cfl=0.1,
                      precision=precision)
        mesh = lib.Mesh(gpu_problem(params))
        slots = mesh.new_slots()
        a, h = mesh.views(slots[0])
        a.fill_(1.0)
        h.zero_()
        ctl = mesh.new_ctl()
        mesh.start(slots, ctl)
        tot = float(mesh.totals(slots[0]).cpu()[0])
        for _ in range(20):
            info = mesh.step(slots, ctl)[0]
            new = float(mesh.totals(slots[info["cur"]]).cpu()[0])
            _say(f"[inflow {precision}] dt {info['dt']:.4e} mass gain {new - tot:.17g}")
            assert abs((new - tot) - info["dt"]) < 1e-14
            tot = new
