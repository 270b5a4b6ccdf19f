"""Shared helpers of the test suite: translate a workload's parameters into
the oracle's Problem and into the library's Problem, and move states between
the two (the oracle converts its own basis to Legendre coefficients)."""
from __future__ import annotations

import math

import numpy as np

import oracle
from paper_2412_16002_amd import inputs

def oracle_problem(params: dict) -> oracle.Problem:
    d = params["dim"]
    bc = tuple(params.get("bc", ("periodic",) * d)) + ("periodic",) * (3 - d)
    return oracle.Problem(
        dim=d, n=tuple(params["n"]), system=params["system"], k=params["k"],
        space=params.get("space", "Q"), stages=params["stages"],
        lo=tuple(params.get("lo", (0.0, 0.0, 0.0))), hi=tuple(params.get("hi", (1.0, 1.0, 1.0))),
        bc=bc, vel=tuple(params.get("vel", (1.0, 1.0, 1.0))), gamma=params.get("gamma", 1.4),
        bound_lo=params.get("bound_lo", -math.inf), bound_hi=params.get("bound_hi", math.inf),
        eps=params.get("eps", 1e-8), cfl=params.get("cfl", 0.1),
        max_halvings=params.get("max_halvings", 40), limiter=bool(params.get("limiter", True)),
        bc_upper=tuple(params["bc_upper"]) if params.get("bc_upper") else None,
        bc_state=dict(params.get("bc_state", {})), alpha=params.get("alpha", "face"))


def gpu_problem(params: dict):
    from paper_2412_16002_amd import crkdg
    return crkdg.problem_from_params(params)


def mode_degrees(o: oracle.CRKDG):
    return [sum(e) for e in o.legendre_modes()]


def random_state(o: oracle.CRKDG, seed, rel_amp=0.05, limited=True, avg=None):
    """Random Legendre state [Nc, V, M] around admissible averages; limited by
    the oracle's limiter if `limited`."""
    if avg is None:
        if o.p.system == oracle.EULER:
            avg = inputs.random_euler_averages(o.ncell, o.d, seed=seed)
        else:
            lo, hi = o.p.bound_lo, o.p.bound_hi
            rng = np.random.default_rng(seed)
            if np.isfinite(lo) and np.isfinite(hi):
                avg = rng.uniform(lo + 0.1 * (hi - lo), hi - 0.1 * (hi - lo), (o.ncell, 1))
            else:
                avg = rng.uniform(0.5, 1.5, (o.ncell, 1))
    C = inputs.random_legendre(o.ncell, o.V, o.M, mode_degrees(o), seed=seed + 1000, avg=avg,
                               rel_amp=rel_amp)
    if limited:
        C = o.to_legendre(o.limit(o.from_legendre(C))[0])
    return C


def round_hi(C, precision):
    """Round modes >= 1 to FP32 when the library stores them in FP32."""
    if precision == "fp64":
        return C
    out = C.copy()
    out[:, :, 1:] = C[:, :, 1:].astype(np.float32).astype(np.float64)
    return out


def rel_err(a, b, scale=None):
    a = np.asarray(a)
    b = np.asarray(b)
    s = np.max(np.abs(b)) if scale is None else scale
    return float(np.max(np.abs(a - b)) / max(s, 1e-300))


def rel_err_per_var(a, b):
    """max over variables of max|a-b| / max|b| (states [Nc, V, M])."""
    out = 0.0
    for v in range(b.shape[1]):
        s = max(np.max(np.abs(b[:, v, :])), 1e-300)
        out = max(out, float(np.max(np.abs(a[:, v, :] - b[:, v, :])) / s))
    return out


def l1_rel(o: oracle.CRKDG, Ca, Cb):
    """Relative L1 distance of two Legendre states (reading A18): per variable
    ||a - b||_1 / ||b||_1 with a (k+2)^d Gauss rule, max over variables."""
    Ua, Ub = o.from_legendre(Ca), o.from_legendre(Cb)
    num = o.l1_norm(Ua - Ub)
    den = o.l1_norm(Ub)
    return float(np.max(num / np.maximum(den, 1e-300)))


def parity_tolerance(o: oracle.CRKDG, unlimited, ref, rtol=1e-12):
    """Elementwise tolerance for comparing a limited state with the oracle's.

    rtol times the variable's magnitude everywhere; in Euler cells whose
    density step drives rho to eps at a point of S_K (min rho < eps before
    limiting), theta_2 depends on 1/rho_hat at that point and inherits a
    relative error of ulp(rho_bar)/eps, so the modes >= 1 of those cells get
    that relative slack (64 ulp)."""
    scale = np.max(np.abs(ref), axis=(0, 2))[None, :, None]
    tol = rtol * scale * np.ones_like(ref)
    if o.p.system == oracle.EULER:
        rho_min = o.sk_values(o.from_legendre(unlimited))[..., 0].min(axis=1)
        kappa = np.where(rho_min < o.p.eps, 64 * 2.0 ** -52 * np.abs(unlimited[:, 0, 0]) / o.p.eps, 0.0)
        tol[:, :, 1:] += kappa[:, None, None] * np.abs(ref[:, :, 1:])
    return tol
