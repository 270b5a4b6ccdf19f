"""Batched form on the GPU: launch shapes of the stage kernels (tile shape,
workgroup size, persistent grids), the autotuner, and step graphs.

A launch shape only decides which thread handles which cell, so every shape
must give bitwise the same states and controllers as the default one; a step
graph replayed n times must give bitwise what n eager attempts give, with
eager work between the replays."""
import sys

import numpy as np
import pytest

from _helpers import gpu_problem
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


def _cases(precision):
    cases = inputs.batched_2d(seed=7, count=5, nmin=20, nmax=70, precision=precision)
    probs = [gpu_problem(dict(c.params, precision=precision)) for c in cases]
    states = [c.cell_states for c in cases]
    b = inputs.burgers_1d(seed=1, n=300)
    probs.append(gpu_problem(dict(b.params, precision=precision)))
    states.append(None)
    return probs, states, b


def _build(lib, precision):
    probs, states, b = _cases(precision)
    mesh = lib.Mesh(probs)
    slots = mesh.new_slots()
    for i, st in enumerate(states):
        a, h = mesh.views(slots[0], inst=i)
        h.zero_()
        if st is not None:
            a.copy_(torch.from_numpy(st.T.copy()))
        else:
            x = (np.arange(a.shape[1]) + 0.5) / a.shape[1]
            a.copy_(torch.from_numpy(b.u0(x[:, None])[:, 0][None, :].copy()))
    ctl = mesh.new_ctl()
    mesh.limit(slots[0], ctl)
    return mesh, slots, ctl


def _snapshot(mesh, slots, ctl):
    c = mesh.ctl_read(ctl)
    out = []
    for i, ci in enumerate(c):
        a, h = mesh.views(slots[ci["cur"]], inst=i)
        out.append((a.cpu().numpy().copy(), h.cpu().numpy().copy(),
                    {k: ci[k] for k in ("t", "dt", "cur", "accepted", "rejected", "stages_run", "status")}))
    return out


def _same(sa, sb):
    for (a1, h1, c1), (a2, h2, c2) in zip(sa, sb):
        assert c1 == c2
        assert np.array_equal(a1, a2) and np.array_equal(h1, h2)


def _run(lib, precision, shape=None, steps=3):
    mesh, slots, ctl = _build(lib, precision)
    if shape is not None:
        for g in range(mesh.group_count()):
            th, tx, grid = shape
            tx = th if mesh.get_tuning(g)["dim"] == 1 else tx
            mesh.set_tuning(g, th, tx, grid)
    mesh.start(slots, ctl)
    for _ in range(steps):
        mesh.step(slots, ctl)
    return mesh, slots, ctl, _snapshot(mesh, slots, ctl)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_launch_shapes_bitwise(lib, precision):
    """Three accepted steps of a batched mesh (five 2D Euler instances of
    random size and degree plus a 1D Burgers instance) under several launch
    shapes, persistent grids included, against the default shape."""
    _say(f"[shapes] {precision} default")
    mesh, _, _, ref = _run(lib, precision)
    assert mesh.group_count() >= 2
    for shape in [(64, 8, 0), (128, 16, 0), (256, 64, 0), (128, 32, 1024), (256, 32, 8), (64, 64, 16)]:
        _say(f"[shapes] {precision} threads/tile/grid {shape}")
        _, _, _, got = _run(lib, precision, shape)
        _same(ref, got)


def test_bad_shapes_rejected(lib):
    mesh, slots, ctl = _build(lib, "mixed")
    for shape in [(96, 32, 0), (256, 4, 0), (256, 512, 0), (128, 32, 12), (64, 24, 0)]:
        with pytest.raises(lib.CRKDGError):
            mesh.set_tuning(0, *shape)


def test_autotune_keeps_results(lib):
    """The autotuner leaves u~^n, the controllers and the step results
    untouched and picks valid shapes."""
    _, _, _, ref = _run(lib, "mixed")
    mesh, slots, ctl = _build(lib, "mixed")
    mesh.start(slots, ctl)
    before = _snapshot(mesh, slots, ctl)
    tunes = mesh.autotune(slots, ctl, reps=1)
    _same(before, _snapshot(mesh, slots, ctl))
    for t in tunes:
        _say(f"[autotune] dim {t['dim']} k {t['k']} s {t['stages']} cells {t['n_cells']}: "
             f"threads {t['threads']} tile_x {t['tile_x']} grid {t['grid']} {t['ms']:.3f} ms")
        assert t["threads"] in (64, 128, 256) and t["ms"] > 0
    for _ in range(3):
        mesh.step(slots, ctl)
    _same(ref, _snapshot(mesh, slots, ctl))


def test_graph_replays_match_eager(lib):
    """A graph of two attempts, replayed four times with host reads and eager
    kernels (a limiter call on a scratch state) between the replays, equals
    eight eager attempts after every replay; shapes are locked while it
    exists."""
    mesh_e, slots_e, ctl_e = _build(lib, "mixed")
    mesh_g, slots_g, ctl_g = _build(lib, "mixed")
    for g in range(mesh_g.group_count()):
        if mesh_g.get_tuning(g)["dim"] > 1:
            mesh_g.set_tuning(g, 128, 16, 1024)
    mesh_e.start(slots_e, ctl_e)
    mesh_g.start(slots_g, ctl_g)
    graph = mesh_g.graph(slots_g, ctl_g, attempts=2)
    with pytest.raises(lib.CRKDGError):
        mesh_g.set_tuning(0, 64, 8, 0)
    scratch = mesh_g.new_state()
    for r in range(4):
        for _ in range(2):
            mesh_e.step(slots_e, ctl_e, sync=False)
        graph.launch()
        mesh_g.limit(scratch)               # eager work between replays
        torch.cuda.synchronize()
        se, sg = _snapshot(mesh_e, slots_e, ctl_e), _snapshot(mesh_g, slots_g, ctl_g)
        _say(f"[graph] replay {r}: accepted {[x[2]['accepted'] for x in sg]}")
        _same(se, sg)
    graph.close()
    mesh_g.set_tuning(0, 64, 8, 0)           # unlocked again
