"""The shallow-water system (flat bottom; reading A28) on the GPU against the
oracle: stage parity on 1D and 2D families with periodic, outflow, wall and
Dirichlet sides, FP64 and mixed; the depth limiter under heavy limiting;
controller steps; the dam breaks of the oracle pins against the exact
Riemann solution; and order k+1 on the manufactured solution (through the
source-term hook)."""
import math
import sys

import numpy as np
import pytest

import oracle
import _swe_riemann as R
from _helpers import gpu_problem, oracle_problem, random_state, rel_err_per_var, round_hi
from paper_2412_16002_amd import inputs

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


SW = dict(system="shallow_water", gravity=1.3, eps=1e-6)
CASES = {
    "swe1d_p2": dict(dim=1, n=(20,), k=2, stages=3, cfl=0.15, **SW),
    "swe1d_p3_outflow": dict(dim=1, n=(17,), k=3, stages=4, cfl=0.09, bc=("outflow",), **SW),
    "swe2d_q1": dict(dim=2, n=(11, 9), k=1, stages=2, cfl=0.3, **SW),
    "swe2d_q2_walls": dict(dim=2, n=(9, 7), k=2, stages=3, cfl=0.15, bc=("reflect", "dirichlet"),
                           bc_upper=("outflow", "reflect"), bc_state={2: [1.2, 0.1, 0.3]}, **SW),
    "swe2d_q3": dict(dim=2, n=(6, 5), k=3, stages=4, cfl=0.09, **SW),
    "swe2d_p2": dict(dim=2, n=(8, 7), k=2, space="P", stages=3, cfl=0.15, **SW),
    "swe2d_p3_walls": dict(dim=2, n=(7, 6), k=3, space="P", stages=4, cfl=0.09, bc=("dirichlet", "reflect"),
                           bc_upper=("reflect", "outflow"), bc_state={0: [0.9, 0.2, -0.1]}, **SW),
}


def _setup(lib, name, precision):
    params = dict(CASES[name], precision=precision)
    return params, oracle.CRKDG(oracle_problem(params)), lib.Mesh(gpu_problem(params))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", list(CASES))
def test_swe_stage_parity(lib, name, precision):
    params, o, mesh = _setup(lib, name, precision)
    s = o.p.stages
    tilde = [round_hi(random_state(o, seed=600 + j, rel_amp=0.1), precision) for j in range(s)]
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
        ref = o.to_legendre(o.limit(o.stage(i, U[0], U, dt))[0])
        mesh.ctl_write(ctl, [{"dt": dt}])
        mesh.stage(i, states, out, ctl)
        got = mesh.get_legendre(out)
        err, err0 = rel_err_per_var(got, ref), rel_err_per_var(got[:, :, :1], ref[:, :, :1])
        _say(f"[swe stage] {name} {precision} stage {i}: rel err {err:.2e} (averages {err0:.2e})")
        if precision == "fp64":
            assert err < 1e-12
        else:
            assert err < 1e-5 and err0 < 1e-6
        assert o.bound_violations(o.from_legendre(got)) == 0
        assert mesh.ctl_read(ctl)[0]["flags"] == 0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["swe1d_p2", "swe2d_q2_walls", "swe2d_p3_walls", "swe2d_q3"])
def test_swe_limit_parity(lib, name, precision):
    """Heavily perturbed states around low depths: the limiter acts in many
    cells; one factor per cell, equal to the oracle's (FP64: 1e-12; mixed:
    the FP32 modes within the A16 re-verification, 2^-17 relative)."""
    params, o, mesh = _setup(lib, name, precision)
    rng = np.random.default_rng(31)
    avg = inputs.swe_conservative(rng.uniform(0.01, 0.3, o.ncell), rng.uniform(-1.0, 1.0, (o.ncell, o.d)))
    C = round_hi(random_state(o, seed=32, rel_amp=8.0, limited=False, avg=avg), precision)
    ref, theta = o.limit(o.from_legendre(C))
    ref = o.to_legendre(ref)
    u = mesh.new_state()
    mesh.set_legendre(u, C)
    ctl = mesh.new_ctl()
    mesh.ctl_write(ctl, [{}])
    mesh.limit(u, ctl)
    got = mesh.get_legendre(u)
    acted = theta < 1.0
    _say(f"[swe limit] {name} {precision}: limited {acted.mean():.2f}")
    assert acted.mean() > 0.1
    assert np.array_equal(got[:, :, 0], C[:, :, 0])
    if precision == "fp64":
        tol = 1e-12 * np.abs(ref) + 1e-15
    else:
        tol = 2.0 ** -17 * np.abs(ref) + 2.0 ** -23 * np.abs(C) + 1e-300
    assert np.all(np.abs(got - ref) <= tol)
    assert o.bound_violations(o.from_legendre(got)) == 0
    assert mesh.ctl_read(ctl)[0]["flags"] == 0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_swe_steps(lib, precision):
    params, o, mesh = _setup(lib, "swe2d_q2_walls", precision)
    C0 = round_hi(random_state(o, seed=41, rel_amp=0.05), precision)
    slots = mesh.new_slots()
    mesh.set_legendre(slots[0], C0)
    ctl = mesh.new_ctl()
    mesh.start(slots, ctl)
    U = o.from_legendre(C0)
    t = 0.0
    for n in range(4):
        U, io = o.step(U, t)
        t = io["t"]
        info = mesh.step(slots, ctl)[0]
        assert info["status"] == 0 and info["halvings"] == io["halvings"]
        assert math.isclose(info["dt"], io["dt"], rel_tol=1e-12 if precision == "fp64" else 1e-5)
        err = rel_err_per_var(mesh.get_legendre(slots[info["cur"]]), o.to_legendre(U))
        _say(f"[swe step] {precision} step {n}: dt {info['dt']:.3e} rel err {err:.2e}")
        assert err < (1e-11 if precision == "fp64" else 1e-5)


@pytest.mark.parametrize("h_right", [1.0, 0.5])
@pytest.mark.parametrize("k,precision", [(2, "fp64"), (2, "mixed"), (3, "fp64")])
def test_swe_dam_break(lib, h_right, k, precision):
    cs = inputs.swe_dam_break_1d(n=200, k=k, h_left=2.0, h_right=h_right, eps=1e-4, precision=precision,
                                 t_end=0.2)
    params = cs.params
    o = oracle.CRKDG(oracle_problem(params))
    U = o.limit(o.constant_state(cs.cell_states))[0]
    mesh = lib.Mesh(gpu_problem(params))
    slots = mesh.new_slots()
    mesh.set_legendre(slots[0], o.to_legendre(U))
    ctl = mesh.new_ctl()
    mesh.start(slots, ctl, t0=0.0, t_end=cs.t_end)
    m0 = float(mesh.totals(slots[0]).cpu()[0])
    t = 0.0
    for n in range(10):                       # lockstep with the oracle
        U, io = o.step(U, t, cs.t_end)
        t = io["t"]
        info = mesh.step(slots, ctl)[0]
        err = rel_err_per_var(mesh.get_legendre(slots[info["cur"]]), o.to_legendre(U))
        assert err < (1e-10 if precision == "fp64" else 1e-5), (n, err)
    for _ in range(5000):
        if mesh.ctl_read(ctl)[0]["status"] == lib.S_DONE:
            break
        mesh.step(slots, ctl)
    c = mesh.ctl_read(ctl)[0]
    assert c["status"] == lib.S_DONE and c["rejected"] == 0
    C = mesh.get_legendre(slots[c["cur"]])
    hav, _ = R.cell_averages(-1.0, 1.0, 200, c["t"], 2.0, 0.0, h_right, 0.0, 1.0)
    l1 = float(np.sum(np.abs(C[:, 0, 0] - hav)) / np.sum(hav))
    dm = float(mesh.totals(slots[c["cur"]]).cpu()[0]) - m0
    _say(f"[swe dam break] h_R {h_right} P{k} {precision}: {c['accepted']} steps, rel L1 of h {l1:.4f}, "
         f"mass change {dm:.1e}")
    assert l1 < 0.01
    # still water held at both ends: no mass crosses them, up to the FP32
    # rounding of the discharge traces in the mixed form
    assert abs(dm) < (1e-12 if precision == "fp64" else 1e-7)
    assert o.bound_violations(o.from_legendre(C)) == 0


def _project_on_gpu(mesh, o, fn):
    xq = mesh.points(0, 0)[:, :o.d]
    vals = np.asarray(fn(o.physical_points(xq)), dtype=np.float64)
    samples = torch.from_numpy(np.ascontiguousarray(np.transpose(vals, (2, 0, 1)))).cuda()
    st = mesh.new_state()
    mesh.project(samples.reshape(-1), st)
    return st


@pytest.mark.parametrize("space,k", [("Q", 1), ("Q", 2), ("P", 2), ("Q", 3)])
def test_swe_manufactured_convergence(lib, space, k):
    errs = []
    ns = (8, 16, 32) if k == 3 else (16, 32, 64)
    for n in ns:
        cs = inputs.swe_mms(2, n, k, space=space)
        o = oracle.CRKDG(oracle_problem(cs.params))
        mesh = lib.Mesh(gpu_problem(cs.params))
        sts = [_project_on_gpu(mesh, o, lambda X, p=p: inputs.swe_mms_source_terms(X)[p]) for p in range(3)]
        mesh.set_source(sts, [(r, 0.0, 0.0) for r in inputs.SWE_MMS_RATES])
        slots = mesh.new_slots()
        slots[0].copy_(_project_on_gpu(mesh, o, cs.u0))
        mesh.limit(slots[0])
        ctl = mesh.new_ctl()
        mesh.start(slots, ctl, t_end=cs.t_end, dt_fixed=cs.meta["dt"])
        steps = int(math.ceil(cs.t_end / cs.meta["dt"]))
        for _ in range(steps + 2):
            mesh.step(slots, ctl, sync=False)
        rec = mesh.ctl_read(ctl)[0]
        assert rec["status"] == lib.S_DONE and rec["rejected"] == 0
        got = o.from_legendre(mesh.get_legendre(slots[rec["cur"]]))
        errs.append(float(np.sum(o.l1_norm(got, lambda X: cs.exact(X, rec["t"])))))
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    _say(f"[swe mms] {space}{k}: L1 errors {', '.join(f'{e:.3e}' for e in errs)}, rates {rates}")
    assert rates[-1] > k + 1 - 0.25
