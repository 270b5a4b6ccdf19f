"""The device step controller (Sec. 4.1 algorithm) on the GPU: forced
halvings against the oracle, time-step underflow, the final-time clip, a
non-finite state, and the independence of the instances of a batch.  Every
failure is forced from the host through the data; every kernel exits
normally."""
import math
import sys

import numpy as np
import pytest

import oracle
from _helpers import gpu_problem, oracle_problem, rel_err_per_var

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


BURGERS = dict(dim=1, n=(40,), system="burgers", k=2, stages=3, bound_lo=0.2, bound_hi=1.0, cfl=0.1)


def _square_wave(o):
    return o.limit(o.project(lambda x: (0.6 + 0.39 * np.sign(np.sin(2 * np.pi * x[..., 0])))[..., None]))[0]


def test_forced_halvings_match_oracle(lib):
    """A trial step of 20 dx is rejected and halved until the stage averages
    stay in B; the GPU takes the oracle's number of halvings, the same dt and
    the same accepted state."""
    params = dict(BURGERS, precision="fp64")
    o = oracle.CRKDG(oracle_problem(params))
    U = _square_wave(o)
    dt0 = 20.0 * o.dx[0]
    U1, io = o.step(U, 0.0, dt_fixed=dt0)
    mesh = lib.Mesh(gpu_problem(params))
    slots = mesh.new_slots()
    mesh.set_legendre(slots[0], o.to_legendre(U))
    ctl = mesh.new_ctl()
    mesh.start(slots, ctl, dt_fixed=dt0)
    info = mesh.step(slots, ctl)[0]
    _say(f"[controller] halvings oracle {io['halvings']} gpu {info['halvings']}, rejected {info['rejected']}")
    assert io["halvings"] >= 3
    assert info["status"] == 0 and info["halvings"] == io["halvings"] and info["rejected"] == io["halvings"]
    assert math.isclose(info["dt"], dt0 / 2 ** io["halvings"], rel_tol=1e-15)
    got = mesh.get_legendre(slots[info["cur"]])
    assert rel_err_per_var(got, o.to_legendre(U1)) < 1e-11
    assert o.bound_violations(o.from_legendre(got)) == 0


def test_underflow_status(lib):
    """An average outside B cannot be repaired by halving: after
    max_halvings + 1 rejected attempts the instance stops with
    CRKDG_S_DT_UNDERFLOW (the oracle raises), and the state is untouched."""
    params = dict(dim=1, n=(8,), system="burgers", k=1, stages=2, bound_lo=0.0, bound_hi=1.0, cfl=0.1,
                  max_halvings=5, precision="fp64")
    o = oracle.CRKDG(oracle_problem(params))
    C = np.zeros((8, 1, 2))
    C[:, 0, 0] = 0.5
    C[3, 0, 0] = 1.5
    with pytest.raises(RuntimeError):
        o.step(o.from_legendre(C), dt_fixed=0.01)
    mesh = lib.Mesh(gpu_problem(params))
    slots = mesh.new_slots()
    mesh.set_legendre(slots[0], C)
    ctl = mesh.new_ctl()
    mesh.start(slots, ctl, dt_fixed=0.01)
    info = mesh.step(slots, ctl)[0]
    _say(f"[controller] underflow: status {info['status']} rc {info['rc']} rejected {info['rejected']}")
    assert info["status"] == lib.S_DT_UNDERFLOW and info["rc"] == lib.S_DT_UNDERFLOW
    assert info["rejected"] == 6 and info["accepted"] == 0
    assert np.array_equal(mesh.get_legendre(slots[0]), C)
    # a stopped instance stays stopped
    again = mesh.step(slots, ctl)[0]
    assert again["status"] == lib.S_DT_UNDERFLOW and again["rejected"] == 6


def test_final_time_clip(lib):
    """With t_end = 2.5 trial steps the third step is clipped to end exactly
    at t_end; the oracle does the same; afterwards the instance is done and
    further calls change nothing."""
    params = dict(dim=1, n=(64,), system="advection", k=2, stages=3, vel=(1.0, 0, 0), bound_lo=0.0,
                  bound_hi=2.0, cfl=0.15, precision="fp64")
    o = oracle.CRKDG(oracle_problem(params))
    U = o.limit(o.project(lambda x: (1.0 + 0.5 * np.sin(2 * np.pi * x[..., 0]))[..., None]))[0]
    t_end = 2.5 * o.trial_dt(U)
    mesh = lib.Mesh(gpu_problem(params))
    slots = mesh.new_slots()
    mesh.set_legendre(slots[0], o.to_legendre(U))
    ctl = mesh.new_ctl()
    mesh.start(slots, ctl, t_end=t_end)
    t = 0.0
    steps = 0
    while t < t_end and steps < 5:
        U, io = o.step(U, t, t_end)
        t = io["t"]
        info = mesh.step(slots, ctl)[0]
        steps += 1
        assert math.isclose(info["t"], t, rel_tol=1e-14)
    _say(f"[controller] t_end {t_end:.17g}: {steps} steps, t {info['t']:.17g}")
    assert steps == 3 and math.isclose(info["t"], t_end, rel_tol=1e-15)
    c = mesh.ctl_read(ctl)[0]
    assert c["status"] == lib.S_DONE and c["accepted"] == 3
    got = mesh.get_legendre(slots[info["cur"]])
    assert rel_err_per_var(got, o.to_legendre(U)) < 1e-11
    again = mesh.step(slots, ctl)[0]
    assert again["accepted"] == 3 and again["status"] == 0
    assert mesh.ctl_read(ctl)[0]["status"] == lib.S_DONE


def test_nonfinite_state_stops(lib):
    """A NaN in a cell average raises the flags of every attempt: the
    instance stops (non-zero status) instead of accepting a step."""
    params = dict(dim=1, n=(8,), system="euler", k=1, stages=2, cfl=0.3, max_halvings=3, precision="fp64")
    from paper_2412_16002_amd import inputs
    avg = inputs.random_euler_averages(8, 1, seed=1)
    C = np.zeros((8, 3, 2))
    C[:, :, 0] = avg
    mesh = lib.Mesh(gpu_problem(params))
    slots = mesh.new_slots()
    mesh.set_legendre(slots[0], C)
    ctl = mesh.new_ctl()
    mesh.start(slots, ctl, dt_fixed=1e-3)
    a, _ = mesh.views(slots[0])
    a[2, 5] = float("nan")
    info = mesh.step(slots, ctl)[0]
    _say(f"[controller] NaN: status {info['status']} rejected {info['rejected']}")
    assert info["status"] in (lib.S_DT_UNDERFLOW, lib.S_NONFINITE)
    assert info["accepted"] == 0


def test_batch_instances_are_independent(lib):
    """A batch of an underflowing instance and a regular one: the regular
    instance's step is bitwise the step it takes alone."""
    bad = dict(dim=1, n=(8,), system="burgers", k=1, stages=2, bound_lo=0.0, bound_hi=1.0, cfl=0.1,
               max_halvings=5, precision="fp64")
    good = dict(BURGERS, precision="fp64")
    ob = oracle.CRKDG(oracle_problem(good))
    Ug = ob.to_legendre(_square_wave(ob))
    Cb = np.zeros((8, 1, 2))
    Cb[:, 0, 0] = 0.5
    Cb[3, 0, 0] = 1.5

    solo = lib.Mesh(gpu_problem(good))
    ss = solo.new_slots()
    solo.set_legendre(ss[0], Ug)
    cs = solo.new_ctl()
    solo.start(ss, cs)
    i_solo = solo.step(ss, cs)[0]

    both = lib.Mesh([gpu_problem(bad), gpu_problem(good)])
    sb = both.new_slots()
    both.set_legendre(sb[0], Cb, inst=0)
    both.set_legendre(sb[0], Ug, inst=1)
    cb = both.new_ctl()
    both.start(sb, cb, dt_fixed=[0.01, 0.0])
    infos = both.step(sb, cb)
    assert infos[0]["status"] == lib.S_DT_UNDERFLOW
    assert infos[1]["status"] == 0 and infos[1]["accepted"] == 1
    assert infos[1]["dt"] == i_solo["dt"] and infos[1]["halvings"] == i_solo["halvings"]
    assert np.array_equal(both.get_legendre(sb[infos[1]["cur"]], inst=1), solo.get_legendre(ss[i_solo["cur"]]))
