"""The C-ABI library loads and exports every entry point that include/crkdg.h
declares (no GPU and no compute calls)."""
import ctypes
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
LIB = ROOT / "paper_2412_16002_amd" / "_lib" / "libcrkdg.so"


def declared_symbols():
    text = (ROOT / "include" / "crkdg.h").read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(crkdg_[a-z_]+)\s*\(", text)))


def test_header_declares_the_entry_points():
    names = declared_symbols()
    for must in ("crkdg_init_mesh", "crkdg_stage", "crkdg_step", "crkdg_limit", "crkdg_cell_avg"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not LIB.exists():
        pytest.skip("libcrkdg.so not built (python -m paper_2412_16002_amd.build)")
    lib = ctypes.CDLL(str(LIB))
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, f"missing exports: {missing}"


def test_binding_covers_every_declared_symbol():
    if not LIB.exists():
        pytest.skip("libcrkdg.so not built")
    from paper_2412_16002_amd import crkdg
    assert set(declared_symbols()) <= set(crkdg.EXPORTED)


def test_struct_layouts_match_header(tmp_path):
    """ctypes mirrors of the ABI structs have the sizes and field offsets that
    a C compiler gives the declarations of include/crkdg.h."""
    import shutil
    import subprocess
    if not LIB.exists():
        pytest.skip("libcrkdg.so not built")
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    from paper_2412_16002_amd import crkdg
    mirrors = {"crkdg_problem": crkdg.CProblem, "crkdg_layout": crkdg.CLayout,
               "crkdg_instance_layout": crkdg.CInstLayout, "crkdg_state": crkdg.CState,
               "crkdg_ctl": crkdg.CCtl, "crkdg_step_info": crkdg.CStepInfo,
               "crkdg_tuning": crkdg.CTuning}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "crkdg.h"', "int main(void) {"]
    for cname, py in mirrors.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "abi.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "abi"
    subprocess.run([cc, f"-I{ROOT / 'include'}", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for line in out:
        if line.strip():
            a, b, c = line.split()
            got[(a, b)] = int(c)
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_init_rejects_bad_problems_without_gpu():
    """Validation happens before any device call: a bad problem returns
    CRKDG_E_ARG with a message."""
    if not LIB.exists():
        pytest.skip("libcrkdg.so not built")
    from paper_2412_16002_amd import crkdg
    bad = crkdg.Problem(dim=4, n=(4,)).to_c()
    h = ctypes.c_void_p()
    lay = crkdg.CLayout()
    rc = crkdg.LIB.crkdg_init_mesh(ctypes.byref(bad), 1, ctypes.byref(h), ctypes.byref(lay))
    assert rc == crkdg.E_ARG
    assert b"dim" in crkdg.LIB.crkdg_last_error()
    p = crkdg.Problem(dim=1, n=(4,), k=5).to_c()
    assert crkdg.LIB.crkdg_init_mesh(ctypes.byref(p), 1, ctypes.byref(h), ctypes.byref(lay)) == crkdg.E_ARG
    p = crkdg.Problem(dim=1, n=(4,), scheme=7).to_c()
    assert crkdg.LIB.crkdg_init_mesh(ctypes.byref(p), 1, ctypes.byref(h), ctypes.byref(lay)) == crkdg.E_ARG
    assert b"scheme" in crkdg.LIB.crkdg_last_error()
    p = crkdg.Problem(dim=1, n=(4,), alpha=3).to_c()
    assert crkdg.LIB.crkdg_init_mesh(ctypes.byref(p), 1, ctypes.byref(h), ctypes.byref(lay)) == crkdg.E_ARG
    assert b"alpha" in crkdg.LIB.crkdg_last_error()


def test_boundary_validation_without_gpu():
    """Boundary sides are checked before any device call: periodic on one
    side only, a reflective wall for a scalar law and a Dirichlet state
    outside the admissible set are CRKDG_E_ARG."""
    if not LIB.exists():
        pytest.skip("libcrkdg.so not built")
    from paper_2412_16002_amd import crkdg
    h = ctypes.c_void_p()
    lay = crkdg.CLayout()
    bad = [
        (crkdg.Problem(dim=1, n=(8,), bc=(crkdg.BC_PERIODIC,) * 3, bc_upper=(crkdg.BC_OUTFLOW, 0, 0)), b"periodic"),
        (crkdg.Problem(dim=1, n=(8,), system=crkdg.SYS_ADVECTION, bc=(crkdg.BC_REFLECT, 0, 0)), b"reflective"),
        (crkdg.Problem(dim=1, n=(8,), bc=(crkdg.BC_DIRICHLET, 0, 0), bc_state={0: [1.0, 0.0, -1.0], 1: [1, 0, 2.5]}),
         b"Dirichlet"),
        (crkdg.Problem(dim=1, n=(8,), bc=(crkdg.BC_OUTFLOW, 0, 0), bc_upper=(7, 0, 0)), b"bc_upper"),
    ]
    for p, word in bad:
        c = p.to_c()
        assert crkdg.LIB.crkdg_init_mesh(ctypes.byref(c), 1, ctypes.byref(h), ctypes.byref(lay)) == crkdg.E_ARG
        assert word in crkdg.LIB.crkdg_last_error(), crkdg.LIB.crkdg_last_error()


def test_size_limits_without_gpu():
    """A mesh of more than 2^31 - 1 cells in one instance is refused before
    any device call (cell indices of one instance are 32-bit in the tile
    maps)."""
    if not LIB.exists():
        pytest.skip("libcrkdg.so not built")
    from paper_2412_16002_amd import crkdg
    h = ctypes.c_void_p()
    lay = crkdg.CLayout()
    p = crkdg.Problem(dim=2, n=(65536, 65536, 1)).to_c()
    assert crkdg.LIB.crkdg_init_mesh(ctypes.byref(p), 1, ctypes.byref(h), ctypes.byref(lay)) == crkdg.E_ARG
    assert b"2^31" in crkdg.LIB.crkdg_last_error()
    p = crkdg.Problem(dim=1, n=(0, 1, 1)).to_c()
    assert crkdg.LIB.crkdg_init_mesh(ctypes.byref(p), 1, ctypes.byref(h), ctypes.byref(lay)) == crkdg.E_ARG
