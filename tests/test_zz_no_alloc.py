"""crkdg_cell_avg_noalloc, the entry point for callers that cannot allocate:
through the C ABI, its averages and totals equal crkdg_cell_avg's bitwise
(the same fixed-order reduction, partial sums in the library's static device
array instead of the mesh's buffer), on two calls in a row on meshes of
different sizes (the second smaller, so it reads none of the first call's
leftovers), with several instances of different variable counts, and a mesh
above the array's limit is refused before any device work."""
import sys

import numpy as np
import pytest

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


def _mesh_with_data(lib, problems, seed):
    mesh = lib.Mesh(problems)
    u = mesh.new_state()
    g = torch.Generator(device="cpu").manual_seed(seed)
    u.avg.copy_(torch.rand(u.avg.shape, generator=g, dtype=torch.float64) * 2.0 + 0.5)
    return mesh, u


def _both(mesh, u):
    nv = sum(L["n_vars"] for L in mesh.inst)
    out = {}
    for name, fn in (("alloc", mesh.cell_avg), ("noalloc", mesh.cell_avg_noalloc)):
        avg = torch.full_like(u.avg, float("nan"))
        tot = torch.full((nv,), float("nan"), dtype=torch.float64, device=u.avg.device)
        fn(u, avg=avg, totals=tot)
        torch.cuda.synchronize()
        out[name] = (avg.cpu().numpy(), tot.cpu().numpy())
    return out


def test_noalloc_totals_equal_the_allocating_entry_point(lib):
    big = [lib.Problem(dim=3, n=(40, 36, 30), system=lib.SYS_EULER, k=2, stages=4),
           lib.Problem(dim=2, n=(300, 170, 1), system=lib.SYS_EULER, k=2, stages=3)]
    small = [lib.Problem(dim=2, n=(33, 17, 1), system=lib.SYS_ADVECTION, k=1, stages=2),
             lib.Problem(dim=1, n=(700, 1, 1), system=lib.SYS_EULER, k=3, stages=4)]
    for label, probs, seed in (("first, larger", big, 1), ("second, smaller", small, 2)):
        mesh, u = _mesh_with_data(lib, probs, seed)
        r = _both(mesh, u)
        _say(f"[noalloc] {label}: totals {r['noalloc'][1]}")
        assert np.array_equal(r["alloc"][0], r["noalloc"][0])
        assert np.array_equal(r["alloc"][1], r["noalloc"][1])
        assert np.all(np.isfinite(r["noalloc"][1]))
        # the totals are the volume-weighted sums of the averages (to rounding)
        off = 0
        for i, L in enumerate(mesh.inst):
            a, _ = mesh.views(u, inst=i)
            p = mesh.problems[i]
            vol = np.prod([(p.hi[d] - p.lo[d]) / p.n[d] for d in range(p.dim)])
            ref = vol * a.double().sum(dim=1).cpu().numpy()
            assert np.allclose(r["noalloc"][1][off:off + L["n_vars"]], ref, rtol=1e-12)
            off += L["n_vars"]
        mesh.close()


def test_noalloc_refuses_a_mesh_above_its_limit(lib):
    """6.7 million cells is the limit (26214 blocks of 256 cells); a larger
    mesh is refused with CRKDG_E_ARG and a message, before any device work
    (the state passed here is never read)."""
    mesh = lib.Mesh(lib.Problem(dim=2, n=(4096, 2048, 1), system=lib.SYS_ADVECTION, k=1, stages=2))
    tiny = lib.State(torch.zeros(8, dtype=torch.float64, device="cuda"),
                     torch.zeros(8, dtype=torch.float64, device="cuda"))
    with pytest.raises(lib.CRKDGError) as e:
        mesh.cell_avg_noalloc(tiny, totals=torch.zeros(1, dtype=torch.float64, device="cuda"))
    assert e.value.code == lib.E_ARG and "static scratch" in str(e.value)
    mesh.close()
