"""Build the HIP library libcrkdg.so for gfx950, in-tree.

Every translation unit under csrc/ is compiled by hipcc in parallel and linked
into paper_2412_16002_amd/_lib/libcrkdg.so.  Run as a module:
    python -m paper_2412_16002_amd.build
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys
import time
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
CSRC = PKG / "csrc"
OUT_DIR = PKG / "_lib"
LIB = OUT_DIR / "libcrkdg.so"
OBJ_DIR = ROOT / "_build"

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", shutil.which("hipcc") or "/opt/rocm/bin/hipcc")
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    f"-I{ROOT / 'include'}", f"-I{CSRC}",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # the compile-time basis tables of the largest spaces (3D Q^3)
    "-fconstexpr-steps=200000000",
]


def _compile(src: Path) -> Path:
    obj = OBJ_DIR / (src.stem + ".o")
    cmd = [HIPCC, *FLAGS, "-c", str(src), "-o", str(obj)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src.name}:\n{r.stderr[-8000:]}")
    return obj


def build(verbose: bool = True) -> Path:
    OBJ_DIR.mkdir(exist_ok=True)
    OUT_DIR.mkdir(exist_ok=True)
    srcs = sorted(CSRC.glob("*.hip"))
    t0 = time.time()
    jobs = min(len(srcs), max(1, min(16, os.cpu_count() or 1)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB.with_suffix(".so.tmp")
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *map(str, objs), "-o", str(tmp)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-8000:]}")
    os.replace(tmp, LIB)
    _build_c_demo()
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources in {time.time() - t0:.1f}s", flush=True)
    return LIB


# a plain C caller of the library (tests/c/step_demo.c), run by the GPU tests
C_DEMO_SRC = ROOT / "tests" / "c" / "step_demo.c"
C_DEMO = OUT_DIR / "step_demo"


def _build_c_demo():
    if not C_DEMO_SRC.exists():
        return
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        return
    rocm = Path(os.environ.get("ROCM_PATH", "/opt/rocm"))
    cmd = [cc, "-O2", "-std=c11", "-Wall", f"-I{ROOT / 'include'}", f"-I{rocm / 'include'}",
           "-D__HIP_PLATFORM_AMD__", str(C_DEMO_SRC), f"-L{OUT_DIR}", "-lcrkdg", f"-L{rocm / 'lib'}",
           "-lamdhip64", "-Wl,-rpath,$ORIGIN", f"-Wl,-rpath,{rocm / 'lib'}", "-o", str(C_DEMO)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"building the C caller failed:\n{r.stderr[-4000:]}")


if __name__ == "__main__":
    build()
    sys.exit(0)
