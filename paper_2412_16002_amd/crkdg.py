"""ctypes binding of libcrkdg.so (the C ABI of include/crkdg.h).

Argument marshalling only: torch provides device memory and the current HIP
stream; every step of the method runs in the library's HIP kernels.  There is
no fallback: if the library is missing or fails to load, importing this module
raises.
"""
from __future__ import annotations

import ctypes as C
import math
import weakref
from dataclasses import dataclass, field
from pathlib import Path

import numpy as np

_LIB_PATH = Path(__file__).resolve().parent / "_lib" / "libcrkdg.so"

BC_PERIODIC, BC_OUTFLOW, BC_REFLECT, BC_DIRICHLET = 0, 1, 2, 3
SYS_ADVECTION, SYS_BURGERS, SYS_EULER, SYS_SHALLOW_WATER = 0, 1, 2, 3
SPACE_Q, SPACE_P = 0, 1
FP64, MIXED = 0, 1
SCHEME_CRKDG, SCHEME_RKDG = 0, 1
ALPHA_FACE, ALPHA_POINT, ALPHA_GLOBAL = 0, 1, 2
E_ARG, E_HIP, E_UNSUPPORTED, E_LAYOUT = -1, -2, -3, -4
S_REJECTED, S_DT_UNDERFLOW, S_NONFINITE, S_DONE = 1, 2, 3, 4
F_AVERAGE, F_NONFINITE = 1, 2
INT64_MAX = 2 ** 63 - 1


class CProblem(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("n", C.c_int32 * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("bc", C.c_int32 * 3), ("system", C.c_int32), ("vel", C.c_double * 3), ("gamma", C.c_double),
        ("bound_lo", C.c_double), ("bound_hi", C.c_double), ("eps", C.c_double),
        ("k", C.c_int32), ("space", C.c_int32), ("stages", C.c_int32), ("precision", C.c_int32),
        ("limiter", C.c_int32), ("cfl", C.c_double), ("max_halvings", C.c_int32),
        ("scheme", C.c_int32), ("bc_upper", C.c_int32 * 3), ("alpha", C.c_int32),
        ("bc_state", (C.c_double * 5) * 6), ("gravity", C.c_double),
    ]


class CLayout(C.Structure):
    _fields_ = [("n_inst", C.c_int32), ("hi_bytes", C.c_int32), ("n_slots", C.c_int32),
                ("ctl_bytes", C.c_int32), ("avg_elems", C.c_int64), ("hi_elems", C.c_int64)]


class CInstLayout(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_modes", C.c_int32), ("n_vars", C.c_int32),
                ("n_stages", C.c_int32), ("n_vol_pts", C.c_int32), ("n_sk_pts", C.c_int32),
                ("pad", C.c_int32), ("avg_offset", C.c_int64), ("hi_offset", C.c_int64),
                ("sample_offset", C.c_int64)]


class CState(C.Structure):
    _fields_ = [("avg", C.c_void_p), ("hi", C.c_void_p)]


class CCtl(C.Structure):
    _fields_ = [
        ("t", C.c_double), ("t_end", C.c_double), ("dt", C.c_double), ("dt_fixed", C.c_double),
        ("a0", C.c_double * 3), ("a0_next", C.c_uint64 * 3), ("flags", C.c_uint32),
        ("cur", C.c_int32), ("halvings", C.c_int32), ("status", C.c_int32),
        ("accepted", C.c_int64), ("rejected", C.c_int64), ("goal", C.c_int64),
        ("stages_run", C.c_int64), ("dt_last", C.c_double), ("halvings_last", C.c_int32),
        ("pad", C.c_int32),
    ]


class CStepInfo(C.Structure):
    _fields_ = [("t", C.c_double), ("dt", C.c_double), ("halvings", C.c_int32), ("status", C.c_int32),
                ("cur", C.c_int32), ("pad", C.c_int32), ("accepted", C.c_int64), ("rejected", C.c_int64)]


class CTuning(C.Structure):
    _fields_ = [("threads", C.c_int32), ("tile_x", C.c_int32), ("grid", C.c_int32), ("dim", C.c_int32),
                ("k", C.c_int32), ("space", C.c_int32), ("stages", C.c_int32), ("n_inst", C.c_int32),
                ("n_items", C.c_int32), ("scheme", C.c_int32), ("n_cells", C.c_int64), ("ms", C.c_double)]


def _load():
    if not _LIB_PATH.exists():
        raise ImportError(f"{_LIB_PATH} is not built: run `python -m paper_2412_16002_amd.build`")
    lib = C.CDLL(str(_LIB_PATH))
    P = C.POINTER
    sig = {
        "crkdg_last_error": (C.c_char_p, []),
        "crkdg_init_mesh": (C.c_int, [P(CProblem), C.c_int32, P(C.c_void_p), P(CLayout)]),
        "crkdg_free_mesh": (C.c_int, [C.c_void_p]),
        "crkdg_instance_query": (C.c_int, [C.c_void_p, C.c_int32, P(CInstLayout)]),
        "crkdg_points": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, P(C.c_double), C.c_int32,
                                   P(C.c_int32)]),
        "crkdg_project": (C.c_int, [C.c_void_p, C.c_void_p, CState, C.c_void_p]),
        "crkdg_limit": (C.c_int, [C.c_void_p, CState, C.c_void_p, C.c_void_p]),
        "crkdg_set_source": (C.c_int, [C.c_void_p, C.c_int32, P(CState), P(C.c_double)]),
        "crkdg_set_boundary_data": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, P(C.c_double),
                                              C.c_void_p]),
        "crkdg_cell_avg": (C.c_int, [C.c_void_p, CState, C.c_void_p, C.c_void_p, C.c_void_p]),
        "crkdg_cell_avg_noalloc": (C.c_int, [C.c_void_p, CState, C.c_void_p, C.c_void_p, C.c_void_p]),
        "crkdg_cfl": (C.c_int, [C.c_void_p, CState, C.c_void_p, C.c_void_p]),
        "crkdg_start": (C.c_int, [C.c_void_p, P(CState), C.c_int32, C.c_void_p, P(C.c_double),
                                  P(C.c_double), P(C.c_double), C.c_void_p]),
        "crkdg_stage": (C.c_int, [C.c_void_p, C.c_int32, P(CState), C.c_int32, CState, C.c_void_p,
                                  C.c_void_p]),
        "crkdg_step": (C.c_int, [C.c_void_p, P(CState), C.c_int32, C.c_void_p, P(CStepInfo),
                                 C.c_void_p]),
        "crkdg_group_count": (C.c_int, [C.c_void_p, P(C.c_int32)]),
        "crkdg_get_tuning": (C.c_int, [C.c_void_p, C.c_int32, P(CTuning)]),
        "crkdg_set_tuning": (C.c_int, [C.c_void_p, C.c_int32, P(CTuning)]),
        "crkdg_autotune": (C.c_int, [C.c_void_p, P(CState), C.c_int32, C.c_void_p, C.c_int32, C.c_void_p]),
        "crkdg_graph_create": (C.c_int, [C.c_void_p, P(CState), C.c_int32, C.c_void_p, C.c_int32,
                                         P(C.c_void_p)]),
        "crkdg_graph_launch": (C.c_int, [C.c_void_p, C.c_void_p]),
        "crkdg_graph_destroy": (C.c_int, [C.c_void_p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


LIB = _load()
EXPORTED = ("crkdg_last_error", "crkdg_init_mesh", "crkdg_free_mesh", "crkdg_instance_query",
            "crkdg_points", "crkdg_project", "crkdg_limit", "crkdg_set_source", "crkdg_set_boundary_data",
            "crkdg_cell_avg",
            "crkdg_cell_avg_noalloc",
            "crkdg_cfl",
            "crkdg_start", "crkdg_stage", "crkdg_step", "crkdg_group_count", "crkdg_get_tuning",
            "crkdg_set_tuning", "crkdg_autotune", "crkdg_graph_create", "crkdg_graph_launch",
            "crkdg_graph_destroy")


class CRKDGError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = LIB.crkdg_last_error().decode(errors="replace")
        super().__init__(f"{where} failed with {code}: {msg}")


def _check(code, where):
    if code < 0:
        raise CRKDGError(code, where)
    return code


@dataclass
class Problem:
    """Mirror of crkdg_problem (field meanings in include/crkdg.h)."""
    dim: int
    n: tuple
    system: int = SYS_EULER
    k: int = 2
    space: int = SPACE_Q
    stages: int = 3
    precision: int = FP64
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    bc: tuple = (BC_PERIODIC, BC_PERIODIC, BC_PERIODIC)
    vel: tuple = (1.0, 1.0, 1.0)
    gamma: float = 1.4
    bound_lo: float = -math.inf
    bound_hi: float = math.inf
    eps: float = 1e-8
    limiter: int = 1
    cfl: float = 0.1
    max_halvings: int = 40
    scheme: int = SCHEME_CRKDG
    bc_upper: tuple = (0, 0, 0)   # upper side per direction; 0: as bc
    bc_state: dict = field(default_factory=dict)  # side 2 d + upper -> Dirichlet state
    alpha: int = ALPHA_FACE
    gravity: float = 1.0

    def to_c(self) -> CProblem:
        p = CProblem()
        p.dim = self.dim
        for i in range(3):
            p.n[i] = int(self.n[i]) if i < len(self.n) else 1
            p.lo[i] = float(self.lo[i])
            p.hi[i] = float(self.hi[i])
            p.bc[i] = int(self.bc[i])
            p.vel[i] = float(self.vel[i])
        p.system, p.k, p.space, p.stages = self.system, self.k, self.space, self.stages
        p.precision, p.limiter, p.max_halvings = self.precision, int(self.limiter), self.max_halvings
        p.gamma, p.bound_lo, p.bound_hi = self.gamma, self.bound_lo, self.bound_hi
        p.eps, p.cfl, p.scheme, p.alpha = self.eps, self.cfl, self.scheme, self.alpha
        p.gravity = self.gravity
        for i in range(3):
            p.bc_upper[i] = int(self.bc_upper[i]) if i < len(self.bc_upper) else 0
        for side, vals in self.bc_state.items():
            for v, x in enumerate(vals):
                p.bc_state[int(side)][v] = float(x)
        return p


_SYS_NAMES = {"advection": SYS_ADVECTION, "burgers": SYS_BURGERS, "euler": SYS_EULER,
              "shallow_water": SYS_SHALLOW_WATER}
_BC_NAMES = {"periodic": BC_PERIODIC, "outflow": BC_OUTFLOW, "reflect": BC_REFLECT, "dirichlet": BC_DIRICHLET}
_SCHEME_NAMES = {"crkdg": SCHEME_CRKDG, "rkdg": SCHEME_RKDG}


def problem_from_params(params: dict) -> Problem:
    """Problem from a workload parameter dict (names as in crkdg_problem,
    enumerations spelled as words: system 'euler', space 'Q', bc 'periodic',
    precision 'fp64' / 'mixed', scheme 'crkdg' / 'rkdg'; bc_upper per direction,
    bc_state {side 2 d + upper: state}; alpha 'face' / 'point' / 'global')."""
    d = params["dim"]
    bc = tuple(_BC_NAMES[b] for b in params.get("bc", ("periodic",) * d)) + (BC_PERIODIC,) * (3 - d)
    n = tuple(params["n"]) + (1,) * (3 - d)
    return Problem(
        dim=d, n=n, system=_SYS_NAMES[params["system"]], k=params["k"],
        space=SPACE_Q if params.get("space", "Q") == "Q" else SPACE_P, stages=params["stages"],
        precision=FP64 if params.get("precision", "fp64") == "fp64" else MIXED,
        lo=tuple(params.get("lo", (0.0, 0.0, 0.0))), hi=tuple(params.get("hi", (1.0, 1.0, 1.0))),
        bc=bc, vel=tuple(params.get("vel", (1.0, 1.0, 1.0))), gamma=params.get("gamma", 1.4),
        bound_lo=params.get("bound_lo", -math.inf), bound_hi=params.get("bound_hi", math.inf),
        eps=params.get("eps", 1e-8), limiter=int(params.get("limiter", True)),
        cfl=params.get("cfl", 0.1), max_halvings=params.get("max_halvings", 40),
        scheme=_SCHEME_NAMES[params.get("scheme", "crkdg")],
        bc_upper=tuple(_BC_NAMES[b] for b in params["bc_upper"]) if params.get("bc_upper") else (0, 0, 0),
        bc_state=dict(params.get("bc_state", {})),
        alpha={"face": ALPHA_FACE, "point": ALPHA_POINT, "global": ALPHA_GLOBAL}[params.get("alpha", "face")],
        gravity=params.get("gravity", 1.0))


class State:
    """A state: avg (FP64) and hi (FP64 or FP32) flat device tensors."""

    def __init__(self, avg, hi):
        self.avg = avg
        self.hi = hi

    def c(self) -> CState:
        return CState(self.avg.data_ptr(), self.hi.data_ptr())

    def clone(self):
        return State(self.avg.clone(), self.hi.clone())

    def copy_(self, other):
        self.avg.copy_(other.avg)
        self.hi.copy_(other.hi)
        return self


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Mesh:
    """One crkdg_mesh handle over one or more instances."""

    def __init__(self, problems, device="cuda"):
        import torch
        if isinstance(problems, Problem):
            problems = [problems]
        self.problems = list(problems)
        self.device = torch.device(device)
        arr = (CProblem * len(self.problems))(*[p.to_c() for p in self.problems])
        handle = C.c_void_p()
        lay = CLayout()
        with torch.cuda.device(self.device):
            _check(LIB.crkdg_init_mesh(arr, len(self.problems), C.byref(handle), C.byref(lay)),
                   "crkdg_init_mesh")
        self.h = handle
        self.layout = lay
        self.inst = []
        for i in range(len(self.problems)):
            il = CInstLayout()
            _check(LIB.crkdg_instance_query(self.h, i, C.byref(il)), "crkdg_instance_query")
            self.inst.append({f: getattr(il, f) for f, _ in CInstLayout._fields_})
        self.hi_dtype = torch.float64 if lay.hi_bytes == 8 else torch.float32
        assert lay.ctl_bytes == C.sizeof(CCtl), "crkdg_ctl size mismatch between header and binding"

    def close(self):
        for g in list(getattr(self, "_graphs", ())):
            g.close()
        if self.h:
            LIB.crkdg_free_mesh(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------- buffers ----------------
    def new_state(self) -> State:
        import torch
        avg = torch.zeros(self.layout.avg_elems, dtype=torch.float64, device=self.device)
        hi = torch.zeros(self.layout.hi_elems, dtype=self.hi_dtype, device=self.device)
        return State(avg, hi)

    def new_slots(self):
        return [self.new_state() for _ in range(self.layout.n_slots)]

    def new_ctl(self):
        import torch
        return torch.zeros(len(self.problems) * self.layout.ctl_bytes, dtype=torch.uint8,
                           device=self.device)

    def views(self, state: State, inst: int = 0):
        """(avg [V, Nc], hi [V, M-1, Nc]) views of one instance."""
        L = self.inst[inst]
        V, M, Nc = L["n_vars"], L["n_modes"], L["n_cells"]
        a = state.avg[L["avg_offset"]: L["avg_offset"] + V * Nc].view(V, Nc)
        h = state.hi[L["hi_offset"]: L["hi_offset"] + V * (M - 1) * Nc].view(V, M - 1, Nc)
        return a, h

    def set_legendre(self, state: State, coeffs, inst: int = 0):
        """Write host Legendre coefficients coeffs[Nc, V, M] (FP64 numpy) into a state."""
        import torch
        a, h = self.views(state, inst)
        c = np.ascontiguousarray(np.transpose(np.asarray(coeffs, dtype=np.float64), (1, 2, 0)))
        a.copy_(torch.from_numpy(c[:, 0, :]))
        h.copy_(torch.from_numpy(c[:, 1:, :]).to(self.hi_dtype))

    def get_legendre(self, state: State, inst: int = 0):
        """Host Legendre coefficients [Nc, V, M] (FP64) of a state."""
        a, h = self.views(state, inst)
        av = a.double().cpu().numpy()
        hv = h.double().cpu().numpy()
        out = np.concatenate([av[:, None, :], hv], axis=1)
        return np.ascontiguousarray(np.transpose(out, (2, 0, 1)))

    # ---------------- controller ----------------
    def ctl_read(self, ctl):
        import torch
        torch.cuda.synchronize(self.device)
        raw = ctl.cpu().numpy().tobytes()
        n = self.layout.ctl_bytes
        out = []
        for i in range(len(self.problems)):
            c = CCtl.from_buffer_copy(raw[i * n:(i + 1) * n])
            out.append({f: (list(getattr(c, f)) if f in ("a0", "a0_next") else getattr(c, f))
                        for f, _ in CCtl._fields_})
        return out

    def ctl_write(self, ctl, entries):
        import torch
        n = self.layout.ctl_bytes
        buf = bytearray(n * len(entries))
        for i, e in enumerate(entries):
            c = CCtl()
            c.goal = INT64_MAX
            c.t_end = math.inf
            for k, v in e.items():
                if k in ("a0", "a0_next"):
                    for j, x in enumerate(v):
                        getattr(c, k)[j] = x
                else:
                    setattr(c, k, v)
            buf[i * n:(i + 1) * n] = bytes(c)
        ctl.copy_(torch.frombuffer(buf, dtype=torch.uint8).to(self.device))

    def set_dt(self, ctl, dt):
        dts = dt if isinstance(dt, (list, tuple)) else [dt] * len(self.problems)
        self.ctl_write(ctl, [{"dt": float(d)} for d in dts])

    # ---------------- entry points ----------------
    def points(self, inst=0, which=0):
        cnt = C.c_int32()
        _check(LIB.crkdg_points(self.h, inst, which, None, 0, C.byref(cnt)), "crkdg_points")
        buf = (C.c_double * (3 * cnt.value))()
        _check(LIB.crkdg_points(self.h, inst, which, buf, cnt.value, C.byref(cnt)), "crkdg_points")
        return np.array(buf, dtype=np.float64).reshape(cnt.value, 3)

    def project(self, samples, out: State):
        _check(LIB.crkdg_project(self.h, C.c_void_p(samples.data_ptr()), out.c(), _stream()),
               "crkdg_project")

    def set_source(self, terms, coef):
        """crkdg_set_source: s(x, t) = sum_p exp(-rate_p t) cos(omega_p t +
        phase_p) S_p(x) with S_p the states `terms` and coef a list of
        (rate, omega, phase) triples; the states stay referenced by the mesh
        (kept alive here too).  Empty lists remove the source."""
        n = len(terms)
        flat = [float(x) for c in coef for x in c]
        if len(flat) != 3 * n:
            raise ValueError("one (rate, omega, phase) triple per term")
        cs = (CState * max(n, 1))(*[t.c() for t in terms])
        cf = (C.c_double * max(3 * n, 1))(*flat)
        _check(LIB.crkdg_set_source(self.h, n, cs, cf), "crkdg_set_source")
        self._source_terms = list(terms)

    def set_boundary_data(self, inst, side, coef, values):
        """crkdg_set_boundary_data: `values` a device float64 tensor
        [n_terms, n_faces, n_fp, V] (kept alive here), coef a list of (rate,
        omega, phase) triples; empty lists return the side to its constant
        state."""
        n = len(coef)
        flat = [float(x) for c in coef for x in c]
        cf = (C.c_double * max(3 * n, 1))(*flat)
        ptr = C.c_void_p(values.data_ptr()) if n else None
        _check(LIB.crkdg_set_boundary_data(self.h, inst, side, n, cf, ptr), "crkdg_set_boundary_data")
        if not hasattr(self, "_bdata"):
            self._bdata = {}
        self._bdata[(inst, side)] = values

    def limit(self, u: State, ctl=None):
        _check(LIB.crkdg_limit(self.h, u.c(), None if ctl is None else C.c_void_p(ctl.data_ptr()),
                               _stream()), "crkdg_limit")

    def cell_avg(self, u: State, avg=None, totals=None):
        _check(LIB.crkdg_cell_avg(self.h, u.c(), None if avg is None else C.c_void_p(avg.data_ptr()),
                                  None if totals is None else C.c_void_p(totals.data_ptr()), _stream()),
               "crkdg_cell_avg")

    def cell_avg_noalloc(self, u: State, avg=None, totals=None):
        """crkdg_cell_avg_noalloc: the same results, partial sums in the
        library's static device array (no allocation)."""
        _check(LIB.crkdg_cell_avg_noalloc(self.h, u.c(), None if avg is None else C.c_void_p(avg.data_ptr()),
                                          None if totals is None else C.c_void_p(totals.data_ptr()), _stream()),
               "crkdg_cell_avg_noalloc")

    def totals(self, u: State):
        import torch
        nv = sum(L["n_vars"] for L in self.inst)
        t = torch.empty(nv, dtype=torch.float64, device=self.device)
        self.cell_avg(u, totals=t)
        return t

    def cfl(self, u: State, ctl):
        _check(LIB.crkdg_cfl(self.h, u.c(), C.c_void_p(ctl.data_ptr()), _stream()), "crkdg_cfl")

    def start(self, slots, ctl, t0=0.0, t_end=math.inf, dt_fixed=0.0, cur=0):
        n = len(self.problems)

        def arr(x):
            vals = x if isinstance(x, (list, tuple)) else [x] * n
            return (C.c_double * n)(*[float(v) for v in vals])
        cs = (CState * len(slots))(*[s.c() for s in slots])
        _check(LIB.crkdg_start(self.h, cs, cur, C.c_void_p(ctl.data_ptr()), arr(t0), arr(t_end),
                               arr(dt_fixed), _stream()), "crkdg_start")

    def stage(self, i, states, out: State, ctl):
        cs = (CState * len(states))(*[s.c() for s in states])
        _check(LIB.crkdg_stage(self.h, i, cs, len(states), out.c(), C.c_void_p(ctl.data_ptr()),
                               _stream()), "crkdg_stage")

    def step(self, slots, ctl, sync=True):
        """One step (sync=True: accepted, returns per-instance info dicts) or
        one asynchronous attempt (sync=False)."""
        cs = (CState * len(slots))(*[s.c() for s in slots])
        if not sync:
            _check(LIB.crkdg_step(self.h, cs, len(slots), C.c_void_p(ctl.data_ptr()), None, _stream()),
                   "crkdg_step")
            return None
        info = (CStepInfo * len(self.problems))()
        rc = _check(LIB.crkdg_step(self.h, cs, len(slots), C.c_void_p(ctl.data_ptr()), info, _stream()),
                    "crkdg_step")
        out = [{f: getattr(x, f) for f, _ in CStepInfo._fields_} for x in info]
        for o in out:
            o["rc"] = rc
        return out

    # ---------------- launch shapes, autotuning, step graphs ----------------
    def group_count(self):
        n = C.c_int32()
        _check(LIB.crkdg_group_count(self.h, C.byref(n)), "crkdg_group_count")
        return n.value

    def get_tuning(self, group=0):
        t = CTuning()
        _check(LIB.crkdg_get_tuning(self.h, group, C.byref(t)), "crkdg_get_tuning")
        return {f: getattr(t, f) for f, _ in CTuning._fields_}

    def set_tuning(self, group, threads, tile_x, grid=0):
        t = CTuning()
        t.threads, t.tile_x, t.grid = threads, tile_x, grid
        _check(LIB.crkdg_set_tuning(self.h, group, C.byref(t)), "crkdg_set_tuning")

    def autotune(self, slots, ctl, reps=3):
        cs = (CState * len(slots))(*[s.c() for s in slots])
        _check(LIB.crkdg_autotune(self.h, cs, len(slots), C.c_void_p(ctl.data_ptr()), reps, _stream()),
               "crkdg_autotune")
        return [self.get_tuning(g) for g in range(self.group_count())]

    def graph(self, slots, ctl, attempts=1):
        """A StepGraph of `attempts` asynchronous step attempts on these buffers."""
        return StepGraph(self, slots, ctl, attempts)


class StepGraph:
    """crkdg_graph handle: launch() enqueues the captured attempts on the
    current stream.  Keeps the mesh and buffers alive; close() before the
    mesh is freed."""

    def __init__(self, mesh, slots, ctl, attempts):
        self.mesh, self.slots, self.ctl = mesh, list(slots), ctl
        cs = (CState * len(self.slots))(*[s.c() for s in self.slots])
        h = C.c_void_p()
        _check(LIB.crkdg_graph_create(mesh.h, cs, len(self.slots), C.c_void_p(ctl.data_ptr()), attempts,
                                      C.byref(h)), "crkdg_graph_create")
        self.h = h
        self.attempts = attempts
        if not hasattr(mesh, "_graphs"):
            mesh._graphs = weakref.WeakSet()
        mesh._graphs.add(self)

    def launch(self):
        _check(LIB.crkdg_graph_launch(self.h, _stream()), "crkdg_graph_launch")

    def close(self):
        if self.h:
            LIB.crkdg_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
