"""Benchmark of the cRKDG hot path on one MI355X.

Headline workload (the largest single-GPU configuration): 3D compressible
Euler on a periodic 128^3 mesh, tensor Q^2 modal DG (27 modes x 5
variables), four-stage cRKDG (classical RK4) with the scaling limiter after
every stage, seeded smooth translating density wave (rho = 1 + 0.99 sin,
w = (1, 1, 1), p = 1).  One step = all stages (inner stages with G, the
final stage with F and Lax--Friedrichs fluxes, the scaling limiter after
each, the fused CFL wave-speed maximum) plus the device step controller,
for the whole mesh.

The headline `value` is the mixed-precision form (FP32 modes >= 1, FP64
averages / checks / limiter theta / average update); the plain FP64 form is
timed on the same workload and reported beside it, with the relative L1
difference of their averages after the same steps taken with the same dt
sequence (the FP64 run's steps replayed in the mixed form).

More workloads are measured in the same run and reported under
"workloads" (a failure there is reported, never fatal to the headline):
  euler2d       2D Euler, 1024^2 periodic, Q^2 (9 modes x 4 variables),
                Heun3 cRKDG, seeded 64-site Voronoi states
                (rho in [1e-3, 1], p in [1e-6, 10], |w| <= 3);
  batched       64 independent 2D Euler instances in one mesh,
                N_i ~ U{64..512}, P^1-P^3, 3 or 4 stages, 16-site Voronoi
                states, per-instance dt;
  euler2d_rkdg  the 2D workload under the standard RKDG scheme (F in every
                stage, same Butcher table and limiter), with the
                cRKDG-over-RKDG step-time ratio;
  euler3d_share8  one GPU's share of the headline mesh split into 8 z-slabs
                (128 x 128 x 16 cells of the same width, periodic in z: the
                slab's own opposite face stands in for the neighbour traces
                of the one exchange per step; the wave's z frequency raised
                to 8), throughput of that one GPU.

Metric: DOF-stage updates/s = sum over instances of Nc M V x executed stages
/ wall time, with the state resident in HBM before the timed region starts.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
import traceback

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E

# states the final stage reads besides writing one: u~^n plus every u~^(j),
# j >= 2, with b_j != 0 (Heun3: b_2 = 0; RK2: b_1 = 0 but u~^n is the base)
FINAL_READS = {2: 2, 3: 2, 4: 4}
# algorithmic state transfers per step (Scheme 1L): reads + writes of all stages
STEP_STATES = {2: 5, 3: 8, 4: 13}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1024, help="cells per direction of the 2D workloads")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparison run")
    ap.add_argument("--workloads", default="euler2d,batched,euler2d_rkdg,euler3d_share8",
                    help="extra workloads to measure (comma list of euler2d, batched, euler2d_rkdg, "
                         "euler3d_share8; empty for none)")
    ap.add_argument("--only", choices=["euler3d", "euler2d", "batched", "euler2d_rkdg", "euler3d_share8"],
                    default=None,
                    help="run only this workload (mixed and FP64) and print its results (for profiling)")
    ap.add_argument("--alpha", choices=["face", "point", "global"], default="face",
                    help="Lax-Friedrichs alpha of every workload: per face (default), per face point, "
                         "or the global a0")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--cpu-budget", type=float, default=10.0,
                    help="seconds of oracle work per CPU-baseline leg (all threads, then one thread)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (to scale HBM byte counters)")
    return ap.parse_args()


def state_bytes(nvars, nmodes, mixed):
    return nvars * (8 + (4 if mixed else 8) * (nmodes - 1))


# ---------------------------------------------------------------------------
# workload set-up (synthetic, seeded; state resident on the device)
# ---------------------------------------------------------------------------
def wave3d_state(mesh, state, case, n, torch, nz=None, zfreq=1.0):
    """Samples of the smooth 3D wave at every volume Gauss point, made on the
    device, projected by the library (n x n x nz cells of width 1/n; the
    wave's z frequency zfreq)."""
    nz = n if nz is None else nz
    xq = torch.from_numpy(mesh.points(0, 0)[:, :3]).cuda()
    Q = xq.shape[0]
    c = (torch.arange(n, device="cuda", dtype=torch.float64) + 0.5) / n
    cz = (torch.arange(nz, device="cuda", dtype=torch.float64) + 0.5) / n
    h = 0.5 / n
    X = c.view(1, 1, n, 1) + h * xq[:, 0].view(1, 1, 1, Q)
    Y = c.view(1, n, 1, 1) + h * xq[:, 1].view(1, 1, 1, Q)
    Z = cz.view(nz, 1, 1, 1) + h * xq[:, 2].view(1, 1, 1, Q)
    rho = 1.0 + 0.99 * torch.sin(2.0 * math.pi * (X + Y + zfreq * Z).reshape(-1, Q) + case.meta["phase"])
    smp = torch.empty((5, n * n * nz, Q), dtype=torch.float64, device="cuda")
    for v in range(1, 4):
        smp[v] = rho
    smp[0] = rho
    smp[4] = 2.5 + 1.5 * rho          # p = 1, gamma = 1.4, w = (1, 1, 1)
    mesh.project(smp.reshape(-1), state)


def setup(name, precision, crkdg, inputs, torch, n2d, alpha="face"):
    scheme = "crkdg"
    extra = {"alpha": alpha}
    if name in ("euler2d", "euler2d_rkdg"):
        cases = [inputs.euler_2d_voronoi(seed=0, n=n2d)]
        if name == "euler2d_rkdg":
            scheme = "rkdg"     # same workload, standard RKDG (F in every stage)
    elif name == "euler3d":
        cases = [inputs.euler_3d_wave(seed=0, n=128)]
    elif name == "euler3d_share8":
        # one GPU's share of the headline mesh split into 8 z-slabs
        cases = [inputs.euler_3d_wave_slab(seed=0, n=128, parts=8)]
    else:
        cases = inputs.batched_2d(seed=0)
    probs = [crkdg.problem_from_params(dict(c.params, precision=precision, scheme=scheme, **extra))
             for c in cases]
    mesh = crkdg.Mesh(probs)
    slots = mesh.new_slots()
    if name == "euler3d":
        wave3d_state(mesh, slots[0], cases[0], 128, torch)
    elif name == "euler3d_share8":
        wave3d_state(mesh, slots[0], cases[0], 128, torch, nz=16, zfreq=8.0)
    else:
        for i, c in enumerate(cases):
            a, h = mesh.views(slots[0], inst=i)
            a.copy_(torch.from_numpy(c.cell_states.T.copy()))
            h.zero_()
    ctl = mesh.new_ctl()
    mesh.limit(slots[0], ctl)
    mesh.start(slots, ctl)
    torch.cuda.synchronize()
    return cases, mesh, slots, ctl


def run_steps(mesh, slots, ctl, k, torch, stream):
    """k asynchronous attempts (one crkdg_step each); returns elapsed ms from
    HIP events on the stream the kernels run on."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(k):
        mesh.step(slots, ctl, sync=False)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def time_kernels(mesh, slots, ctl, reps, torch, stream):
    """Average duration (ms) of each stage (its kernel plus the deferred
    limiter kernel that completes it), launched alone through crkdg_stage on
    the same buffers, timed with HIP events on its stream (one instance)."""
    s = mesh.problems[0].stages
    c = mesh.ctl_read(ctl)[0]
    cur = c["cur"]
    n = len(slots)
    states = [slots[(cur + j) % n] for j in range(s)]
    out = slots[(cur + s) % n]
    mesh.ctl_write(ctl, [{"dt": c["dt"], "cur": 0}])
    res = {}
    for i in range(2, s + 2):
        o = out if i == s + 1 else slots[(cur + i - 1) % n]
        mesh.stage(i, states, o, ctl)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            mesh.stage(i, states, o, ctl)
        e1.record(stream)
        torch.cuda.synchronize()
        res[i] = e0.elapsed_time(e1) / reps
    return res


def run_graph(graph, torch, stream):
    """One launch of a step graph; elapsed ms from HIP events on the stream."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    graph.launch()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1)


def measure(name, precision, args, crkdg, inputs, torch, stream, kernels=True, batched=False):
    """Autotune the launch shapes, then time the steps (batched: warm-up and
    timed steps as two captured step graphs, one launch each)."""
    cases, mesh, slots, ctl = setup(name, precision, crkdg, inputs, torch, args.n, args.alpha)
    # launch shapes from the library's autotuner (results do not depend on them)
    tuning = mesh.autotune(slots, ctl, reps=1 if name.startswith("euler3d") else 2)
    if batched:
        gw = mesh.graph(slots, ctl, attempts=args.warmup)
        gt = mesh.graph(slots, ctl, attempts=args.steps)
        run_graph(gw, torch, stream)
        c0 = mesh.ctl_read(ctl)
        ms = run_graph(gt, torch, stream)
        c1 = mesh.ctl_read(ctl)
        gw.close()
        gt.close()
    else:
        run_steps(mesh, slots, ctl, args.warmup, torch, stream)
        c0 = mesh.ctl_read(ctl)
        ms = run_steps(mesh, slots, ctl, args.steps, torch, stream)
        c1 = mesh.ctl_read(ctl)
    mixed = precision == "mixed"
    dof_stages = 0
    step_bytes = 0
    for i, L in enumerate(mesh.inst):
        dof = L["n_cells"] * L["n_modes"] * L["n_vars"]
        dof_stages += dof * (c1[i]["stages_run"] - c0[i]["stages_run"])
        S = state_bytes(L["n_vars"], L["n_modes"], mixed)
        step_bytes += STEP_STATES[L["n_stages"]] * S * L["n_cells"] * (c1[i]["accepted"] - c0[i]["accepted"]
                                                                      + c1[i]["rejected"] - c0[i]["rejected"])
    r = dict(ms=ms, value=dof_stages / (ms / 1e3),
             accepted=sum(c1[i]["accepted"] - c0[i]["accepted"] for i in range(len(c1))),
             rejected=sum(c1[i]["rejected"] - c0[i]["rejected"] for i in range(len(c1))),
             step_hbm_fraction=step_bytes / (ms / 1e3) / 1e9 / HBM_PEAK_GBS,
             t=[c["t"] for c in c1], cur=[c["cur"] for c in c1])
    if tuning is not None:
        r["tuning"] = [{k: t[k] for k in ("dim", "k", "stages", "n_inst", "n_cells", "threads", "tile_x",
                                          "grid", "ms")} for t in tuning]
        # per kernel group: its stage kernels' pass (the tuner's time of the
        # chosen shape) against the HBM roofline of the group's step bytes
        for t in r["tuning"]:
            L = next(L for L, p in zip(mesh.inst, mesh.problems) if p.k == t["k"] and p.dim == t["dim"]
                     and L["n_stages"] == t["stages"])
            gb = STEP_STATES[t["stages"]] * state_bytes(L["n_vars"], L["n_modes"], mixed) * t["n_cells"]
            t["hbm_fraction"] = gb / (t["ms"] / 1e3) / 1e9 / HBM_PEAK_GBS
    if kernels and len(mesh.inst) == 1:
        r["kern"] = time_kernels(mesh, slots, ctl, args.kernel_reps, torch, stream)
        L = mesh.inst[0]
        s = L["n_stages"]
        S = state_bytes(L["n_vars"], L["n_modes"], mixed)
        alg = (FINAL_READS[s] + 1) * S * L["n_cells"]
        kfin = r["kern"][s + 1]
        r["final"] = dict(alg_bytes=alg, kernel_ms=kfin, achieved=alg / (kfin / 1e3) / 1e9)
    return r, mesh, slots


def l1_diff(mesh_a, slots_a, cur_a, mesh_b, slots_b, cur_b, torch):
    """max over instances and variables of sum |avg_a - avg_b| / sum |avg_b|."""
    worst = 0.0
    for i in range(len(mesh_a.inst)):
        a, _ = mesh_a.views(slots_a[cur_a[i]], inst=i)
        b, _ = mesh_b.views(slots_b[cur_b[i]], inst=i)
        d = (a - b).abs().sum(dim=1) / b.abs().sum(dim=1)
        worst = max(worst, float(d.max()))
    return worst


# ---------------------------------------------------------------------------
# committed rocprofv3 counter summaries (they describe a kernel only as long as
# its sources are unchanged: each summary carries the hash of those sources)
# ---------------------------------------------------------------------------
# the sources the headline final-stage kernel and its launch are built from
# (the 3D Q^2 Euler instantiation, the cooperative and shared device code,
# tables, launchers, the host code that maps tiles to workgroups, the header)
HEADLINE_SOURCES = ("include/crkdg.h", "paper_2412_16002_amd/csrc/device.hpp",
                    "paper_2412_16002_amd/csrc/coop.hpp",
                    "paper_2412_16002_amd/csrc/tables.hpp", "paper_2412_16002_amd/csrc/variants.hpp",
                    "paper_2412_16002_amd/csrc/variants_v3d_q2_euler.hip",
                    "paper_2412_16002_amd/csrc/host.hip")
HEADLINE_COUNTERS = "profiles/counters_final_stage_euler3d_q2_128_mixed.json"


def kernel_source_hash(sources=HEADLINE_SOURCES):
    """Hash of the sources of a kernel, to tell whether committed counter data
    still describe the kernel that runs."""
    import hashlib
    from pathlib import Path
    h = hashlib.sha256()
    for name in sources:
        h.update(name.encode())
        h.update((Path(ROOT) / name).read_bytes())
    return h.hexdigest()[:16]


def _committed_counters(path=HEADLINE_COUNTERS, sources=HEADLINE_SOURCES):
    """The committed counter summary of a kernel, or None when its sources
    changed since the counters were taken."""
    from pathlib import Path
    f = Path(ROOT) / path
    if not f.exists():
        return None
    d = json.loads(f.read_text())
    return d if d.get("source_hash") == kernel_source_hash(sources) else None


def measured_traffic():
    """HBM bytes per launch of the headline final-stage kernel (FETCH_SIZE +
    WRITE_SIZE, scaled by what the same counters read for a plain copy), or
    None."""
    d = _committed_counters()
    return d.get("traffic_bytes_per_launch") if d else None


# VALU issue: a wave64 VALU instruction occupies a 16-lane SIMD for 4 cycles
# (full-rate FP32 and FP64 ops; transcendentals take longer), 4 SIMDs per CU
VALU_CYCLES_PER_INSTR = 4
SIMDS = 256 * 4
CLOCK_HZ = 2.4e9


def valu_issue(kernel_ms):
    """The final stage's VALU instruction-issue floor from the committed
    SQ_INSTS_VALU / SQ_WAVES counts, and the fraction of the measured time it
    accounts for (None without counters for these sources)."""
    d = _committed_counters()
    if not d or "valu_instr_per_wave" not in d:
        return None
    instr, waves = d["valu_instr_per_wave"], d["waves_per_launch"]
    floor_ms = instr * VALU_CYCLES_PER_INSTR * waves / SIMDS / CLOCK_HZ * 1e3
    return {"instr_per_wave": instr, "waves_per_launch": waves, "issue_floor_ms": floor_ms,
            "frac": floor_ms / kernel_ms}


# ---------------------------------------------------------------------------
# CPU baseline: the oracle as it stands, on independent sub-meshes of the
# headline workload, one numpy thread per process
# ---------------------------------------------------------------------------
CPU_SAMPLE_N = 12


def _cpu_worker(job):
    seed, n, budget = job
    from threadpoolctl import threadpool_limits

    import oracle
    from paper_2412_16002_amd import inputs
    from tests._helpers import oracle_problem

    case = inputs.euler_3d_wave(seed=seed, n=n)
    with threadpool_limits(limits=1):
        o = oracle.CRKDG(oracle_problem(case.params))
        U = o.limit(o.project(case.u0))[0]
        t0 = time.perf_counter()
        steps = stages = 0
        t = 0.0
        while time.perf_counter() - t0 < budget or steps == 0:
            U, info = o.step(U, t)
            t = info["t"]
            steps += 1
            stages += o.p.stages * (info["halvings"] + 1)
        el = time.perf_counter() - t0
    return o.ncell * o.M * o.V * stages / el, steps, el


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(budget_s=10.0):
    """The oracle (FP64 numpy, unmodified) on periodic 12^3 sub-meshes of the
    headline 3D workload: one process per host thread (at most 16, the CPU
    share of one GPU), each on its own seeded sub-mesh, for ~budget_s, then
    one process alone.  DOF-stage updates/s summed over the processes."""
    import multiprocessing as mp
    procs = max(1, min(16, os.cpu_count() or 1))
    ctx = mp.get_context("spawn")
    with ctx.Pool(procs) as pool:
        res = pool.map(_cpu_worker, [(s, CPU_SAMPLE_N, budget_s) for s in range(procs)])
    with ctx.Pool(1) as pool:
        one = pool.map(_cpu_worker, [(0, CPU_SAMPLE_N, budget_s)])[0]
    value = sum(r[0] for r in res)
    steps = sum(r[1] for r in res)
    n = CPU_SAMPLE_N
    return {"value": value, "unit": "DOF-stage updates/s", "cores": procs, "kind": "oracle",
            "value_1thread": one[0], "cpu_model": _cpu_model(), "host_threads": os.cpu_count(),
            "sample": f"{procs} processes (one numpy thread each), each on its own seeded periodic "
                      f"{n}^3 sub-mesh of the 3D Euler Q2 RK4 density-wave workload, {steps} full steps "
                      f"in ~{budget_s:.0f} s; then one process alone ({one[1]} steps): "
                      f"FP64 oracle as it stands"}


# ---------------------------------------------------------------------------
# mixed vs FP64 at the same dt sequence
# ---------------------------------------------------------------------------
def equal_dt_l1(name, args, crkdg, inputs, torch, steps=10):
    """Steps of the FP64 form with its own CFL steps, the same steps (dt
    replayed per step) in the mixed form, from the same point samples;
    relative L1 of the cell averages (max over variables) after each."""
    runs = {}
    dts = []
    for prec in ("fp64", "mixed"):
        _, mesh, slots, ctl = setup(name, prec, crkdg, inputs, torch, args.n, args.alpha)
        for n in range(steps):
            if prec == "mixed":
                rec = mesh.ctl_read(ctl)[0]
                rec["dt"] = rec["dt_fixed"] = dts[n]
                mesh.ctl_write(ctl, [rec])
            info = mesh.step(slots, ctl)[0]
            if info["status"] != 0:
                raise RuntimeError(f"{name} {prec}: status {info['status']} at step {n}")
            if prec == "fp64":
                dts.append(info["dt"])
            elif info["dt"] != dts[n]:
                raise RuntimeError(f"{name}: the mixed step {n} took dt {info['dt']}, not {dts[n]}")
        runs[prec] = (mesh, slots, [c["cur"] for c in mesh.ctl_read(ctl)])
    mf, sf, cf = runs["fp64"]
    mm, sm, cm = runs["mixed"]
    return {"steps": steps, "l1_rel_avg": l1_diff(mm, sm, cm, mf, sf, cf, torch), "t": sum(dts)}


def summarise(name, r, args, mixed):
    """JSON entry of one measured form of a workload."""
    e = {"value": r["value"], "ms_per_step": r["ms"] / args.steps, "accepted_steps": r["accepted"],
         "rejected_attempts": r["rejected"], "step_hbm_fraction": r["step_hbm_fraction"],
         "tuning": r["tuning"]}
    if name == "batched":
        e["launch"] = "autotuned shapes; warm-up and timed attempts as two captured step graphs"
    if "kern" in r:
        e["kernel_ms"] = {f"stage{i}": v for i, v in r["kern"].items()}
        f = r["final"]
        e["final_stage_roofline"] = {"bound": "hbm", "achieved": f["achieved"], "peak": HBM_PEAK_GBS,
                                     "unit": "GB/s", "frac": f["achieved"] / HBM_PEAK_GBS,
                                     "alg_bytes_per_launch": f["alg_bytes"], "kernel_ms": f["kernel_ms"]}
    return e


def _progress(msg):
    """A progress line on stderr (stdout carries only the result line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def workload(name, args, crkdg, inputs, torch, stream):
    """Mixed and FP64 runs of one workload (step throughput, final-stage
    roofline for single-instance meshes, mixed vs FP64 difference)."""
    out = {}
    finals = {}
    for prec in ("mixed",) + (() if args.no_fp64 else ("fp64",)):
        r, mesh, slots = measure(name, prec, args, crkdg, inputs, torch, stream, batched=(name == "batched"))
        _progress(f"{name} {prec}: {r['ms'] / args.steps:.3f} ms per step")
        finals[prec] = (mesh, slots, r["cur"])
        out[prec] = summarise(name, r, args, prec == "mixed")
        out[prec]["_raw"] = r
    if "fp64" in out:
        out["speedup_mixed_vs_fp64"] = out["mixed"]["value"] / out["fp64"]["value"]
        mm, sm, cm = finals["mixed"]
        mf, sf, cf = finals["fp64"]
        # after the same number of steps, each form with its own trial steps
        out["l1_rel_avg_mixed_vs_fp64_own_dt"] = l1_diff(mm, sm, cm, mf, sf, cf, torch)
    del finals
    torch.cuda.empty_cache()
    if "fp64" in out and name != "batched":
        out["mixed_vs_fp64_equal_dt"] = equal_dt_l1(name, args, crkdg, inputs, torch)
        torch.cuda.empty_cache()
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only: sharding over several GPUs "
                                   "(instances of a batch, or slabs of one mesh with one halo exchange "
                                   "per step) is not implemented",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    # the CPU baseline first, before anything touches the GPU (its worker
    # processes start from a process without GPU state)
    cpu = None
    if not args.no_cpu and not args.only and not args.copy_calibration:
        cpu = cpu_baseline(args.cpu_budget)
        _progress(f"CPU baseline: {cpu['value']:.3e} {cpu['unit']} on {cpu['cores']} threads")
    import torch

    from paper_2412_16002_amd import crkdg, inputs

    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": n * 4, "launches": 3}), flush=True)
        return
    stream = torch.cuda.current_stream()
    if args.only:
        res = workload(args.only, args, crkdg, inputs, torch, stream)
        for p in ("mixed", "fp64"):
            if p in res:
                res[p].pop("_raw")
        print(json.dumps({args.only: res}), flush=True)
        return

    head = workload("euler3d", args, crkdg, inputs, torch, stream)
    mixed = head["mixed"].pop("_raw")
    fin = mixed["final"]
    L = {"cells": 128 ** 3, "modes": 27, "vars": 5, "stages": 4}
    dof = L["cells"] * L["modes"] * L["vars"]
    S = state_bytes(L["vars"], L["modes"], True)
    line = {
        "metric": "DOF-stage updates/s (mixed vs FP64, same L1 error); % HBM roofline",
        "value": mixed["value"],
        "unit": "DOF-stage updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": mixed["ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic (seeded smooth density wave, projected on the device)",
        "config": {"workload": "3D Euler Q2 modal DG, 128^3 periodic, 4-stage cRKDG (RK4) + scaling "
                               "limiter, mixed precision, smooth density wave rho = 1 + 0.99 sin",
                   "dof": dof, "lf_alpha": args.alpha, **L},
        "accepted_steps": mixed["accepted"],
        "rejected_attempts": mixed["rejected"],
        "kernel_ms": {f"stage{i}": v for i, v in mixed["kern"].items()},
        "step_hbm_fraction": mixed["step_hbm_fraction"],
        # the whole step against the HBM roofline: 13 state transfers of
        # Scheme 1L with RK4 (2S + 3S + 3S + 5S)
        "step_roofline": {"bound": "hbm", "alg_bytes_per_step": STEP_STATES[4] * S * L["cells"],
                          "achieved": STEP_STATES[4] * S * L["cells"] / (mixed["ms"] / args.steps / 1e3) / 1e9,
                          "peak": HBM_PEAK_GBS, "unit": "GB/s"},
        "tuning": mixed["tuning"],
        # dominant kernel: the final stage (reads u~^n, u~^(2), u~^(3),
        # u~^(4), writes u~^{n+1}: 5 S per cell); its event time covers the
        # stage kernel and the deferred-limiter kernel that completes it
        "roofline": {"bound": "hbm", "achieved": fin["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": fin["achieved"] / HBM_PEAK_GBS,
                     "traffic": measured_traffic() if args.alpha == "face" else None,
                     "kernel": "k_coop_stage<3,2,Euler,float,16,2,2,final> + k_limit_queue<...,final>",
                     "alg_bytes_per_launch": fin["alg_bytes"], "kernel_ms": fin["kernel_ms"]},
        # the same launch against its VALU instruction-issue floor
        "valu": valu_issue(fin["kernel_ms"]) if args.alpha == "face" else None,
    }
    line["step_roofline"]["frac"] = line["step_roofline"]["achieved"] / HBM_PEAK_GBS
    if "fp64" in head:
        f = head["fp64"]
        f.pop("_raw", None)
        line["fp64"] = f
        line["speedup_mixed_vs_fp64"] = head["speedup_mixed_vs_fp64"]
        line["l1_rel_avg_mixed_vs_fp64_own_dt"] = head["l1_rel_avg_mixed_vs_fp64_own_dt"]
        line["mixed_vs_fp64_equal_dt"] = head.get("mixed_vs_fp64_equal_dt")
    torch.cuda.empty_cache()
    extra = {}
    for name in [w for w in args.workloads.split(",") if w]:
        try:
            extra[name] = workload(name, args, crkdg, inputs, torch, stream)
            for p in ("mixed", "fp64"):
                if p in extra[name]:
                    extra[name][p].pop("_raw", None)
        except Exception as e:  # reported, never fatal to the headline line
            extra[name] = {"error": f"{type(e).__name__}: {e}", "trace": traceback.format_exc()[-600:]}
        torch.cuda.empty_cache()
    rk, e2 = extra.get("euler2d_rkdg"), extra.get("euler2d")
    if rk and e2 and "error" not in rk and "error" not in e2:
        # what compactness buys: cRKDG step time against standard RKDG's on
        # the same 2D workload, kernels and launch-shape tuning
        rk["crkdg_speedup_over_rkdg"] = {p: rk[p]["ms_per_step"] / e2[p]["ms_per_step"]
                                         for p in ("mixed", "fp64") if p in rk and p in e2}
    if extra:
        line["workloads"] = extra
    if cpu is not None:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
