"""The C ABI used from plain C: tests/c/step_demo.c (hipMalloc'd buffers, the
default stream, no Python) runs five accepted steps of a 2D Euler Q^2 mesh;
the same problem through the Python binding (torch buffers, torch's stream)
gives bitwise the same cell averages and time."""
import subprocess
import sys
from pathlib import Path

import numpy as np
import pytest

from _helpers import gpu_problem
from paper_2412_16002_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

DEMO = Path(__file__).resolve().parents[1] / "paper_2412_16002_amd" / "_lib" / "step_demo"


def test_plain_c_caller_matches_binding(tmp_path):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not DEMO.exists():
        pytest.skip("C caller not built (python -m paper_2412_16002_amd.build)")
    from paper_2412_16002_amd import crkdg
    n0, n1, steps = 48, 40, 5
    x = inputs.cell_centres((n0, n1))
    rho = 1.0 + 0.5 * np.sin(2 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 1])
    w = np.stack([0.3 + 0.0 * rho, -0.2 + 0.0 * rho], axis=-1)
    pr = 1.0 + 0.2 * np.cos(2 * np.pi * x[:, 0])
    avg = inputs.conservative(rho, w, pr).T.copy()               # [V, Nc]
    src = tmp_path / "avg_in.bin"
    dst = tmp_path / "avg_out.bin"
    avg.astype(np.float64).tofile(src)
    r = subprocess.run([str(DEMO), str(src), str(dst), str(steps)], capture_output=True, text=True, timeout=120)
    print(r.stdout.strip(), r.stderr.strip(), file=sys.stderr, flush=True)
    assert r.returncode == 0
    out = np.fromfile(dst, dtype=np.float64)
    c_avg, c_t = out[:-1].reshape(4, n0 * n1), out[-1]

    params = dict(dim=2, n=(n0, n1), system="euler", k=2, stages=3, cfl=0.15, precision="fp64")
    mesh = crkdg.Mesh(gpu_problem(params))
    slots = mesh.new_slots()
    a, h = mesh.views(slots[0])
    a.copy_(torch.from_numpy(avg))
    h.zero_()
    ctl = mesh.new_ctl()
    mesh.limit(slots[0], ctl)
    mesh.start(slots, ctl, t0=0.0)
    for _ in range(steps):
        info = mesh.step(slots, ctl)[0]
    p_avg = mesh.views(slots[info["cur"]])[0].cpu().numpy()
    assert info["t"] == c_t
    assert np.array_equal(p_avg, c_avg)
