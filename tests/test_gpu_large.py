"""A mesh whose state arrays pass 2^31 elements: 3D Euler Q2, 256^3 cells,
mixed form (the hi array holds 5 x 26 x 256^3 = 2.18e9 FP32 values, so every
energy mode >= 1 sits beyond element 2^31).  One accepted step from the
projected smooth wave (conservation), then every stage of the next step on
sampled cells, the last cells of the mesh included, against the oracle
evaluated on exactly those cells from the GPU's own stage inputs."""
import sys

import numpy as np
import pytest

import oracle
from _helpers import gpu_problem, oracle_problem, limited_err
from paper_2412_16002_amd import inputs
from test_gpu_euler3d import RK4, _cells_legendre, _project_on_device, _sparse_U, _with_neighbours

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


def test_state_arrays_beyond_2_31_elements(lib):
    n = 256
    case = inputs.euler_3d_wave(seed=1, n=n, precision="mixed")
    params = dict(case.params, precision="mixed")
    mesh = lib.Mesh(gpu_problem(params))
    L = mesh.inst[0]
    hi_elems = L["n_vars"] * (L["n_modes"] - 1) * L["n_cells"]
    _say(f"[large] 256^3 Q2 mixed: {hi_elems:.3e} hi elements per state")
    assert hi_elems > 2 ** 31
    u0 = _project_on_device(mesh, case, n)
    slots = mesh.new_slots()
    a0, h0 = mesh.views(u0)
    a, h = mesh.views(slots[0])
    a.copy_(a0)
    h.copy_(h0)
    del u0, a0, h0
    ctl = mesh.new_ctl()
    mesh.limit(slots[0], ctl)
    mesh.start(slots, ctl, t0=0.0)
    T0 = mesh.totals(slots[0]).cpu().numpy()
    info = mesh.step(slots, ctl)[0]
    assert info["status"] == 0 and info["accepted"] == 1
    T1 = mesh.totals(slots[info["cur"]]).cpu().numpy()
    cons = float(np.max(np.abs(T1 - T0) / np.abs(T0)))
    _say(f"[large] one step: dt {info['dt']:.3e}, conservation {cons:.1e}")
    assert cons <= 1e-12

    o = oracle.CRKDG(oracle_problem(params))
    c = mesh.ctl_read(ctl)[0]
    dt, cur = c["dt"], c["cur"]
    rng = np.random.default_rng(7)
    cells = np.unique(np.concatenate([rng.integers(0, o.ncell, 300), np.arange(o.ncell - 40, o.ncell)]))
    need = _with_neighbours(o, cells)
    base = slots[cur]
    states = [base]
    outs = [mesh.new_state() for _ in range(4)]
    Ub = _sparse_U(o, mesh, base, need)
    tilde = [Ub]
    for i in (2, 3, 4):
        mesh.ctl_write(ctl, [{"dt": dt}])
        mesh.stage(i, states, outs[i - 2], ctl)
        u = Ub[cells] + dt * RK4["a"][i - 2] * o.G(tilde[-1], cells)
        ref = o.to_legendre(o.limit(u)[0])
        got = _cells_legendre(mesh, outs[i - 2], cells)
        err = limited_err(o, o.to_legendre(u), got, ref, 1e-5, mixed=True)
        _say(f"[large] stage {i}: sampled error/tolerance {err:.2e}")
        assert err < 1.0
        states.append(outs[i - 2])
        tilde.append(_sparse_U(o, mesh, outs[i - 2], need))
    mesh.ctl_write(ctl, [{"dt": dt}])
    mesh.stage(5, states, outs[3], ctl)
    u = Ub[cells] + dt * sum(b * o.F(tj, cells) for b, tj in zip(RK4["b"], tilde))
    ref = o.to_legendre(o.limit(u)[0])
    got = _cells_legendre(mesh, outs[3], cells)
    err = limited_err(o, o.to_legendre(u), got, ref, 1e-5, mixed=True)
    _say(f"[large] final stage: sampled error/tolerance {err:.2e}")
    assert err < 1.0
    assert mesh.ctl_read(ctl)[0]["flags"] == 0
