"""Plain FP64 CPU oracle of the bound-preserving compact-stencil RKDG (cRKDG)
method of Liu, Sun and Zhang, "A bound-preserving Runge--Kutta discontinuous
Galerkin method with compact stencils for hyperbolic conservation laws"
(arXiv 2412.16002).

TEST INFRASTRUCTURE ONLY.  This module is the slow, obviously-correct reference
that the HIP library is checked against.  Only the test suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the library never
does, and it imports nothing from the library.  Everything is FP64 numpy with
one library primitive per step (einsum / solve), no blocking and no fusion.

What is computed, and where the paper defines it
-------------------------------------------------
* DG space (Sec. 2, definition of V_h): P^k or Q^k per cell, m components.
  The oracle uses its OWN bases, chosen to differ from the library's modal
  Legendre basis: nodal Lagrange on the tensor Gauss grid for 1D and Q^k, and
  monomials xi^a eta^b (a+b <= k) for P^k.  Same space and same quadrature give
  the same discrete solution, so the basis choice is invisible in the results.
* DG operator F = -div^DG f with the Lax--Friedrichs flux (Sec. 2.1, the
  weak form defining div^DG and the Lax--Friedrichs flux that follows it).
* Local operator G = -div^loc f, same weak form with the interior trace
  f(u^int).nu on every face (Sec. 2.1, definition of div^loc).
* Edge quadrature with weights summing to one (Sec. 2.2.1, Prop. 2.1) and the
  point set S_K of the convex decomposition (Sec. 2.2.1, Prop. 2.2 and Fig. 1):
  Gauss x Gauss--Lobatto tensor points, used only by the limiter and by the
  wave-speed maximum.
* Scalar scaling limiter (Sec. 2.2.2, Prop. 2.4) and the two-step Euler
  positivity limiter (Sec. 2.2.3, density then internal energy).
* cRKDG stages in Butcher form with the limiter after every stage, in the
  "Scheme 1L" form the paper recommends (Appendix B, the limited scheme):
  inner stages use G, the final stage uses F, every stage starts from the
  limited u^n.  Butcher tables of Sec. 3.3 (explicit midpoint, Heun's
  third-order, classical fourth-order).
* Adaptive time marching (Sec. 4.1): trial step CFL/a0 * dx, halve and restart
  the whole step whenever a stage cell average leaves the admissible set.

Readings of the paper where it is silent or ambiguous (also listed in the
design notes of the repository):
  A1  LF alpha is taken per face: max over that face's quadrature points and
      both traces of |w.nu| + c (symmetric between the two cells of a face).
      Optional (Problem.alpha = "point"): alpha at each face quadrature point
      from its two traces alone (local LF); Prop. 2.1's bound argument holds
      pointwise, since each point's alpha still bounds the wave speed of both
      of its traces.  A trace with p < 0 has no real sound speed: its speed
      is the flow speed |w_d| (c^2 clamped at zero; only inadmissible traces,
      e.g. FP32 cancellation near vacuum, reach this), and a point whose
      speeds are undefined (zero density) takes the face alpha.  Optional (Problem.alpha = "global"): one alpha for every
      face of every stage of a step, the a0 of Sec. 2.1 taken as the maximum
      over directions of a0_d(u~^n) (A5); stage values whose wave speeds
      exceed it are caught by the average check and halving (A10).
  A2  multi-D trial step: dt = CFL / sum_d (a0_d / dx_d)  (1D: CFL dx / a0).
  A4  S_K = union over d of (Gauss^{k+1} in the other directions x
      Gauss--Lobatto^N in direction d), N = 2 for k = 1, N = 3 for k = 2, 3.
  A5  a0_d is the maximum over the S_K points of u^n.
  A6  Euler admissibility: rho >= eps and rho*e = E - |m|^2/(2 rho) >= eps,
      the quantities the limiter itself enforces.
  A7  theta_2 minimises rho*e over the density-limited polynomial.
  A8  a limiter factor only acts where its bound is violated at some point of
      S_K; theta is clamped to [0, 1].
  A10 a failed check restarts the whole step from u^n with dt/2.
  A13 outflow boundary: exterior trace = interior trace.
  A21 reflective wall (Euler): exterior trace = the interior trace with the
      momentum component normal to the wall negated (mirror state).
  A22 Dirichlet / inflow boundary: exterior trace = the prescribed state of
      that side (conservative variables), the same at every face point.
  A24 the scalar cell-average check accepts averages within 2^-40 max(1,
      |m|, |M|) of B (round-off at a bound the data attain); the limiter then
      flattens such a cell to its average.  Euler checks are exact (B^eps
      already keeps a margin to positivity).
  A25 a source term s(x, t) (the manufactured solutions of Sec. 4.2) enters
      both operators as its L2 projection (the volume Gauss rule) at the time
      of the stage value it is paired with: G(u, t) = -div^loc f(u) + P s(t),
      F likewise, with u~^(j) at t^n + c_j dt, c_j = sum_k a_jk.
  A28 shallow-water equations (named by the paper as a system the method
      extends to; the limiter it points to is that of positivity-preserving
      DG for shallow water): the invariant region is h >= eps, and one factor
      theta = (hbar - eps) / (hbar - min_{S_K} h), taken where the minimum is
      below eps and clamped to [0, 1], scales every component (depth and
      discharge alike, so the velocity of the limited polynomial stays that
      of a convex combination); reflective walls mirror the normal discharge.
  A29 boundary data that depend on time (the exact-solution boundary data of
      the accuracy tests, Sec. 4.2) are taken at the face quadrature points
      at the time of the stage value the operator acts on, t^n + c_j dt.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

ADVECTION, BURGERS, EULER = "advection", "burgers", "euler"
SHALLOW_WATER = "shallow_water"
PERIODIC, OUTFLOW, REFLECT, DIRICHLET = "periodic", "outflow", "reflect", "dirichlet"

# Butcher tables of the three cRKDG schemes (Sec. 3.3): explicit midpoint
# (second order), Heun's third-order method, the classical fourth-order method.
BUTCHER = {
    2: (np.array([[0.0, 0.0], [0.5, 0.0]]), np.array([0.0, 1.0])),
    3: (np.array([[0.0, 0.0, 0.0], [1.0 / 3.0, 0.0, 0.0], [0.0, 2.0 / 3.0, 0.0]]),
        np.array([0.25, 0.0, 0.75])),
    4: (np.array([[0.0, 0.0, 0.0, 0.0], [0.5, 0.0, 0.0, 0.0],
                  [0.0, 0.5, 0.0, 0.0], [0.0, 0.0, 1.0, 0.0]]),
        np.array([1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0])),
}


# --------------------------------------------------------------------------
# One-dimensional rules
# --------------------------------------------------------------------------
def legendre_table(n, x):
    """Legendre polynomials P_0..P_n and their derivatives at x (Bonnet's
    recurrence; derivative recurrence P'_{j+1} = P'_{j-1} + (2j+1) P_j)."""
    x = np.asarray(x, dtype=np.float64)
    P = np.zeros((n + 1,) + x.shape)
    dP = np.zeros((n + 1,) + x.shape)
    P[0] = 1.0
    if n >= 1:
        P[1] = x
        dP[1] = 1.0
    for j in range(1, n):
        P[j + 1] = ((2 * j + 1) * x * P[j] - j * P[j - 1]) / (j + 1)
        dP[j + 1] = dP[j - 1] + (2 * j + 1) * P[j]
    return P, dP


def gauss_legendre(n):
    """n-point Gauss--Legendre rule on [-1, 1] (nodes ascending, weights sum 2).
    Newton iteration on P_n from the Chebyshev-like initial guesses."""
    i = np.arange(n)
    x = -np.cos(np.pi * (i + 0.75) / (n + 0.5))
    for _ in range(100):
        P, dP = legendre_table(n, x)
        dx = P[n] / dP[n]
        x = x - dx
        if np.max(np.abs(dx)) < 1e-16:
            break
    P, dP = legendre_table(n, x)
    w = 2.0 / ((1.0 - x * x) * dP[n] ** 2)
    return x, w


def gauss_lobatto(N):
    """N-point Gauss--Lobatto rule on [-1, 1]: endpoints plus the roots of
    P'_{N-1}; weights 2 / (N (N-1) P_{N-1}(x)^2)."""
    if N < 2:
        raise ValueError("Gauss-Lobatto needs N >= 2")
    n = N - 1
    x = -np.cos(np.pi * np.arange(N) / n)
    inner = x[1:-1].copy()
    for _ in range(100):
        if inner.size == 0:
            break
        P, dP = legendre_table(n, inner)
        # P'' from Legendre's equation (1-x^2) P'' - 2x P' + n(n+1) P = 0
        d2P = (2.0 * inner * dP[n] - n * (n + 1) * P[n]) / (1.0 - inner * inner)
        step = dP[n] / d2P
        inner = inner - step
        if np.max(np.abs(step)) < 1e-16:
            break
    x = np.concatenate([[-1.0], inner, [1.0]])
    P, _ = legendre_table(n, x)
    w = 2.0 / (N * (N - 1) * P[n] ** 2)
    return x, w


def lobatto_points_for(k):
    """Gauss--Lobatto size used in S_K: 2N-3 >= k (reading A4)."""
    return 2 if k == 1 else 3


def lagrange_1d(nodes, x):
    """Values and derivatives of the Lagrange polynomials through `nodes` at x.
    Returns (L[j, ...], dL[j, ...])."""
    x = np.asarray(x, dtype=np.float64)
    n = len(nodes)
    L = np.ones((n,) + x.shape)
    dL = np.zeros((n,) + x.shape)
    for j in range(n):
        for m in range(n):
            if m != j:
                L[j] = L[j] * (x - nodes[m]) / (nodes[j] - nodes[m])
        for i in range(n):
            if i == j:
                continue
            term = np.full(x.shape, 1.0 / (nodes[j] - nodes[i]))
            for m in range(n):
                if m != j and m != i:
                    term = term * (x - nodes[m]) / (nodes[j] - nodes[m])
            dL[j] = dL[j] + term
    return L, dL


# --------------------------------------------------------------------------
# Problem description
# --------------------------------------------------------------------------
@dataclass
class Problem:
    """A conservation law on a box with a Cartesian mesh (Sec. 1 problem
    statement, Sec. 2 mesh and space), plus the time-marching parameters of
    Sec. 4.1."""
    dim: int
    n: tuple
    system: str = EULER
    k: int = 2
    space: str = "Q"            # "Q" tensor degree <= k per variable, "P" total degree <= k
    stages: int = 3
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    bc: tuple = (PERIODIC, PERIODIC, PERIODIC)   # per direction (both sides)
    bc_upper: tuple = None        # per direction, upper side; None: as `bc`
    bc_state: dict = field(default_factory=dict)  # side 2 d + (upper) -> Dirichlet state [V]
    bc_function: dict = field(default_factory=dict)  # side -> g(X[..., d], t) -> [..., V] (A29)
    vel: tuple = (1.0, 1.0, 1.0)  # advection velocity
    gamma: float = 1.4
    bound_lo: float = -math.inf   # scalar invariant region B = [m, M]
    bound_hi: float = math.inf
    eps: float = 1e-8             # Euler admissible set B^eps
    cfl: float = 0.1
    max_halvings: int = 40
    limiter: bool = True
    alpha: str = "face"           # LF alpha per face (A1), per face point, or global
    gravity: float = 1.0          # g of the shallow-water equations
    source: object = None         # s(X[..., d], t) -> [..., V]: right-hand side (A25)

    @property
    def nvars(self):
        if self.system == EULER:
            return self.dim + 2
        return self.dim + 1 if self.system == SHALLOW_WATER else 1

    def side_bc(self, dd, side):
        """Boundary kind of the lower (side < 0) or upper side of direction dd."""
        if side > 0 and self.bc_upper is not None:
            return self.bc_upper[dd]
        return self.bc[dd]


# --------------------------------------------------------------------------
# The discretisation
# --------------------------------------------------------------------------
class CRKDG:
    """Reference cRKDG discretisation of one Problem.

    State layout: U[cell, var, basis] in the oracle's own basis, cells in
    natural order (first index fastest).
    """

    def __init__(self, prob: Problem):
        self.p = prob
        d = prob.dim
        self.d = d
        self.k = prob.k
        self.V = prob.nvars
        self.n = tuple(int(v) for v in prob.n[:d])
        self.ncell = int(np.prod(self.n))
        self.dx = np.array([(prob.hi[i] - prob.lo[i]) / self.n[i] for i in range(d)])
        self.vol = float(np.prod(self.dx))
        if prob.space not in ("P", "Q"):
            raise ValueError("space must be P or Q")
        if prob.alpha not in ("face", "point", "global"):
            raise ValueError("alpha must be face, point or global")
        self.space = "Q" if d == 1 else prob.space
        for dd in range(d):
            kinds = (prob.side_bc(dd, -1), prob.side_bc(dd, 1))
            if (PERIODIC in kinds) and kinds != (PERIODIC, PERIODIC):
                raise ValueError("a periodic direction is periodic on both sides")
            for j, kind in enumerate(kinds):
                if kind not in (PERIODIC, OUTFLOW, REFLECT, DIRICHLET):
                    raise ValueError(f"unknown boundary kind {kind}")
                if kind == REFLECT and prob.system not in (EULER, SHALLOW_WATER):
                    raise ValueError("reflective walls are defined for the Euler and shallow-water equations")
                if (kind == DIRICHLET and 2 * dd + j not in prob.bc_function
                        and len(prob.bc_state.get(2 * dd + j, ())) != self.V):
                    raise ValueError("a Dirichlet side needs a state of V values")

        # (k+1)-point Gauss rule, tensor volume rule (weights sum to 2^d)
        g, wg = gauss_legendre(self.k + 1)
        self.g1, self.wg1 = g, wg
        self.xq = np.array(list(itertools.product(g, repeat=d)))[:, ::-1].copy()
        self.wq = np.array([np.prod(w) for w in itertools.product(wg, repeat=d)])

        # basis exponents / node indices
        if self.space == "Q":
            self.modes = [tuple(e[::-1]) for e in itertools.product(range(self.k + 1), repeat=d)]
        else:
            self.modes = [e[::-1] for e in itertools.product(range(self.k + 1), repeat=d)
                          if sum(e) <= self.k]
            self.modes = sorted(self.modes, key=lambda e: (sum(e), [-v for v in e]))
        self.M = len(self.modes)

        # reference mass matrix by Gauss quadrature (exact for both bases)
        phi_q, _ = self.basis(self.xq)
        self.mass_ref = np.einsum("q,qm,qn->mn", self.wq, phi_q, phi_q)
        self.mass = self.mass_ref * self.vol / 2.0 ** d
        self.one = np.linalg.solve(self.mass_ref, np.einsum("q,qm->m", self.wq, phi_q))

        # volume tables
        self.phi_q, self.dphi_q = self.basis(self.xq)

        # faces: (direction, side) with side = -1 / +1; tangential Gauss points
        self.faces = []
        for dd in range(d):
            for side in (-1, 1):
                if d == 1:
                    tang = np.zeros((1, 0))
                    wb = np.array([1.0])
                else:
                    tang = np.array(list(itertools.product(g, repeat=d - 1)))[:, ::-1]
                    wb = np.array([np.prod(w) for w in itertools.product(wg, repeat=d - 1)])
                    wb = wb / wb.sum()                 # Prop. 2.1: weights sum to one
                pts = np.zeros((len(wb), d))
                others = [o for o in range(d) if o != dd]
                for j, o in enumerate(others):
                    pts[:, o] = tang[:, j]
                pts[:, dd] = side
                phi_f, _ = self.basis(pts)
                area = self.vol / self.dx[dd]          # |e|; equals 1 in 1D (Sec. 2.1 convention)
                self.faces.append(dict(dim=dd, side=side, pts=pts, wb=wb, phi=phi_f, area=area))

        # S_K (reading A4): union over directions of Gauss x Lobatto products
        gl, _ = gauss_lobatto(lobatto_points_for(self.k))
        self.gl1 = gl
        pts = []
        for dd in range(d):
            axes = [gl if o == dd else g for o in range(d)]
            for tup in itertools.product(*axes[::-1]):
                pts.append(tup[::-1])
        sk = np.unique(np.round(np.array(pts), 15), axis=0)
        self.xs = sk
        self.phi_s, _ = self.basis(self.xs)

        # neighbours
        self.idx = np.array(list(itertools.product(*[range(v) for v in self.n[::-1]])))[:, ::-1]

    # ---------------- basis ----------------
    def basis(self, x):
        """Values [P, M] and reference gradients [P, M, d] of the oracle basis
        at reference points x[P, d] in [-1, 1]^d."""
        x = np.atleast_2d(np.asarray(x, dtype=np.float64))
        P = x.shape[0]
        val = np.ones((P, self.M))
        grad = np.ones((P, self.M, self.d))
        if self.space == "Q":
            L = [lagrange_1d(self.g1, x[:, j]) for j in range(self.d)]
            for m, e in enumerate(self.modes):
                for j in range(self.d):
                    val[:, m] *= L[j][0][e[j]]
                    for jj in range(self.d):
                        grad[:, m, jj] *= L[j][1][e[j]] if jj == j else L[j][0][e[j]]
        else:
            for m, e in enumerate(self.modes):
                for j in range(self.d):
                    val[:, m] *= x[:, j] ** e[j]
                    for jj in range(self.d):
                        if jj == j:
                            grad[:, m, jj] *= e[j] * x[:, j] ** (e[j] - 1) if e[j] > 0 else 0.0
                        else:
                            grad[:, m, jj] *= x[:, j] ** e[j]
        return val, grad

    def evaluate(self, U, x):
        """Point values u(x) [ncell, V, P] of the DG function at reference points."""
        phi, _ = self.basis(x)
        return np.einsum("cvm,pm->cvp", U, phi)

    def project_point_values(self, vals):
        """Discrete L2 projection of values at the volume Gauss points
        vals[ncell, V, Q] onto the space (Gauss-quadrature inner product)."""
        rhs = np.einsum("q,qm,cvq->cvm", self.wq, self.phi_q, vals)
        return np.linalg.solve(self.mass_ref, rhs.reshape(-1, self.M).T).T.reshape(rhs.shape)

    def cell_centres(self):
        lo = np.array(self.p.lo[: self.d])
        return lo + (self.idx + 0.5) * self.dx

    def physical_points(self, xref, cells=None):
        c = self.cell_centres() if cells is None else self.cell_centres()[cells]
        return c[:, None, :] + 0.5 * xref[None, :, :] * self.dx

    def project(self, u0):
        """L2 projection of u0(x[..., d]) -> [..., V] with the (k+1)^d Gauss rule."""
        X = self.physical_points(self.xq)                       # [C, Q, d]
        vals = np.asarray(u0(X), dtype=np.float64)              # [C, Q, V]
        return self.project_point_values(np.transpose(vals, (0, 2, 1)))

    def cell_average(self, U):
        """Cell averages [ncell, V] by the volume Gauss rule (exact)."""
        return np.einsum("q,qm,cvm->cv", self.wq, self.phi_q, U) / 2.0 ** self.d

    def constant_state(self, ubar):
        """Coefficients of the cell-wise constant function ubar[ncell, V]."""
        return ubar[:, :, None] * self.one[None, None, :]

    # ---------------- Legendre interface ----------------
    def legendre_modes(self):
        """Exponent tuples of the Legendre layout of the library: 1D and Q^k with
        the first variable fastest; P^k by total degree, then decreasing first
        exponent."""
        if self.space == "Q":
            return [tuple(e[::-1]) for e in itertools.product(range(self.k + 1), repeat=self.d)]
        out = []
        for tot in range(self.k + 1):
            for e in itertools.product(range(tot + 1), repeat=self.d):
                if sum(e) == tot:
                    out.append(tuple(e))
        return sorted(out, key=lambda e: (sum(e), [-v for v in e]))

    def _legendre_at(self, x):
        x = np.atleast_2d(x)
        tabs = [legendre_table(self.k, x[:, j])[0] for j in range(self.d)]
        modes = self.legendre_modes()
        L = np.ones((x.shape[0], len(modes)))
        for m, e in enumerate(modes):
            for j in range(self.d):
                L[:, m] *= tabs[j][e[j]]
        return L

    def to_legendre(self, U):
        """Legendre coefficients c[cell, V, M] of the DG function (mode 0 is the
        cell average).  Exact projection by the Gauss rule."""
        L = self._legendre_at(self.xq)
        vals = np.einsum("qm,cvm->cvq", self.phi_q, U)
        num = np.einsum("q,qe,cvq->cve", self.wq, L, vals)
        den = np.einsum("q,qe,qe->e", self.wq, L, L)
        return num / den

    def from_legendre(self, C):
        """Inverse of to_legendre: oracle coefficients of sum_e C[., ., e] L_e."""
        L = self._legendre_at(self.xq)
        vals = np.einsum("qe,cve->cvq", L, C)
        return self.project_point_values(vals)

    # ---------------- physics (Sec. 2.2.3 for Euler) ----------------
    def flux(self, u, dd):
        """f_dd(u) for states u[..., V]."""
        p = self.p
        if p.system == ADVECTION:
            return p.vel[dd] * u
        if p.system == BURGERS:
            return 0.5 * u * u
        if p.system == SHALLOW_WATER:
            # (h w_dd, h w_j w_dd + g h^2 / 2 delta_j,dd)
            h = u[..., 0]
            mom = u[..., 1:1 + self.d]
            w = mom[..., dd] / h
            f = np.empty_like(u)
            f[..., 0] = mom[..., dd]
            for j in range(self.d):
                f[..., 1 + j] = mom[..., j] * w + (0.5 * p.gravity * h * h if j == dd else 0.0)
            return f
        rho = u[..., 0]
        mom = u[..., 1:1 + self.d]
        E = u[..., 1 + self.d]
        w = mom[..., dd] / rho
        pres = (p.gamma - 1.0) * (E - 0.5 * np.sum(mom * mom, axis=-1) / rho)
        f = np.empty_like(u)
        f[..., 0] = mom[..., dd]
        for j in range(self.d):
            f[..., 1 + j] = mom[..., j] * w + (pres if j == dd else 0.0)
        f[..., 1 + self.d] = (E + pres) * w
        return f

    def wave_speed(self, u, dd):
        """max |eig(df_dd/du)| at states u[..., V]: |a_dd|, |u|, |w_dd| + c."""
        p = self.p
        if p.system == ADVECTION:
            return np.full(u.shape[:-1], abs(p.vel[dd]))
        if p.system == BURGERS:
            return np.abs(u[..., 0])
        if p.system == SHALLOW_WATER:
            # |w_dd| + sqrt(g h); a negative depth (not admissible) counts as dry
            h = u[..., 0]
            return np.abs(u[..., 1 + dd] / h) + np.sqrt(p.gravity * np.fmax(h, 0.0))
        rho = u[..., 0]
        mom = u[..., 1:1 + self.d]
        E = u[..., 1 + self.d]
        pres = (p.gamma - 1.0) * (E - 0.5 * np.sum(mom * mom, axis=-1) / rho)
        # a state with p < 0 (not admissible: FP32 cancellation near vacuum)
        # has no real sound speed; its speed is |w_dd| (c^2 clamped at zero),
        # so the flow speed still bounds the alpha of its face
        c2 = np.fmax(p.gamma * pres / rho, 0.0)
        return np.abs(mom[..., dd] / rho) + np.sqrt(c2)

    # ---------------- mesh connectivity ----------------
    def neighbour(self, cells, dd, side):
        """Neighbour cell across face (dd, side), or -1 on a non-periodic
        boundary."""
        ijk = self.idx[cells].copy()
        ijk[:, dd] += side
        nd = self.n[dd]
        out = np.zeros(len(cells), dtype=np.int64)
        bnd = (ijk[:, dd] < 0) | (ijk[:, dd] >= nd)
        if self.p.side_bc(dd, side) == PERIODIC:
            ijk[:, dd] %= nd
            bnd[:] = False
        ijk[bnd, dd] = 0
        stride = 1
        for j in range(self.d):
            out += ijk[:, j] * stride
            stride *= self.n[j]
        out[bnd] = -1
        return out

    # ---------------- operators (Sec. 2.1) ----------------
    def _volume_residual(self, Uc):
        """int_K f(u_h) : grad(phi_m) dx by the volume Gauss rule -> [c, V, M]."""
        uq = np.einsum("cvm,qm->cqv", Uc, self.phi_q)
        r = np.zeros(Uc.shape)
        jac = self.vol / 2.0 ** self.d
        for dd in range(self.d):
            fd = self.flux(uq, dd)                                   # [c, q, V]
            r += jac * (2.0 / self.dx[dd]) * np.einsum(
                "q,cqv,qm->cvm", self.wq, fd, self.dphi_q[:, :, dd])
        return r

    def _face_residual(self, face, fn):
        """|e| sum_beta wB_beta fn_beta phi_m(x_beta) -> [c, V, M]."""
        return face["area"] * np.einsum("b,cbv,bm->cvm", face["wb"], fn, face["phi"])

    def G(self, U, cells=None):
        """Local operator G = -div^loc f (Sec. 2.1): the DG weak form with the
        interior flux f(u^int).nu on every face; needs no neighbour data."""
        cells = np.arange(self.ncell) if cells is None else np.asarray(cells)
        Uc = U[cells]
        r = self._volume_residual(Uc)
        for face in self.faces:
            uf = np.einsum("cvm,bm->cbv", Uc, face["phi"])
            r -= self._face_residual(face, face["side"] * self.flux(uf, face["dim"]))
        return np.linalg.solve(self.mass, r.reshape(-1, self.M).T).T.reshape(r.shape)

    def lf_flux(self, um, up, dd, side, a_glob=None):
        """Lax--Friedrichs flux f^.nu on a face with outward normal side*e_dd
        (Sec. 2.1); um/up [c, b, V] interior/exterior traces.  alpha per face
        (reading A1), per face point (alpha = "point"), or the given a_glob
        (alpha = "global")."""
        with np.errstate(invalid="ignore"):
            a = np.fmax(self.wave_speed(um, dd), self.wave_speed(up, dd))    # [c, b]
        a_face = np.max(np.where(np.isnan(a), 0.0, a), axis=1)     # over the defined speeds
        if self.p.alpha == "face":
            a = np.broadcast_to(a_face[:, None], a.shape)
        elif self.p.alpha == "point":
            # a point whose two speeds are undefined (zero density) takes the
            # face's alpha
            a = np.where(np.isnan(a), a_face[:, None], a)
        elif self.p.alpha == "global":
            if a_glob is None:
                raise ValueError("the global alpha needs a_glob")
            a = np.full(a.shape, float(a_glob))
        return (0.5 * side * (self.flux(um, dd) + self.flux(up, dd))
                - 0.5 * a[:, :, None] * (up - um))

    def face_traces(self, U, cells, face, t=0.0):
        """Interior and exterior traces on `face` of `cells` -> ([c,b,V], [c,b,V]);
        t is the time of the state U (for boundary data that depend on it)."""
        Uc = U[cells]
        um = np.einsum("cvm,bm->cbv", Uc, face["phi"])
        nb = self.neighbour(cells, face["dim"], face["side"])
        opp = [f for f in self.faces if f["dim"] == face["dim"] and f["side"] == -face["side"]][0]
        up = um.copy()                                      # outflow: u^ext = u^int (A13)
        kind = self.p.side_bc(face["dim"], face["side"])
        if kind == REFLECT:                                 # mirror state (A21)
            up[..., 1 + face["dim"]] *= -1.0
        elif kind == DIRICHLET:                             # prescribed state (A22)
            j = 2 * face["dim"] + (1 if face["side"] > 0 else 0)
            if j in self.p.bc_function:                     # data g(x, t) at the face points (A29)
                X = self.physical_points(face["pts"], cells)
                up[...] = np.asarray(self.p.bc_function[j](X, t), dtype=np.float64)
            else:
                up[...] = np.asarray(self.p.bc_state[j], dtype=np.float64)
        inner = nb >= 0
        if np.any(inner):
            up[inner] = np.einsum("cvm,bm->cbv", U[nb[inner]], opp["phi"])
        return um, up

    def F(self, U, cells=None, a_glob=None, t=0.0):
        """DG operator F = -div^DG f with the Lax--Friedrichs flux (Sec. 2.1);
        a_glob is the alpha of every face when Problem.alpha is "global"; t
        is the time of U (boundary data that depend on time)."""
        cells = np.arange(self.ncell) if cells is None else np.asarray(cells)
        r = self._volume_residual(U[cells])
        for face in self.faces:
            um, up = self.face_traces(U, cells, face, t)
            r -= self._face_residual(face, self.lf_flux(um, up, face["dim"], face["side"], a_glob))
        return np.linalg.solve(self.mass, r.reshape(-1, self.M).T).T.reshape(r.shape)

    # ---------------- admissibility and limiter (Sec. 2.2) ----------------
    def rho_e(self, u):
        """rho*e = E - |m|^2 / (2 rho) of Euler states u[..., V]."""
        mom = u[..., 1:1 + self.d]
        return u[..., 1 + self.d] - 0.5 * np.sum(mom * mom, axis=-1) / u[..., 0]

    def admissible_average(self, avg):
        """Cell averages avg[c, V] inside B (scalar) or B^eps (Euler, A6)."""
        p = self.p
        ok = np.all(np.isfinite(avg), axis=1)
        if p.system == EULER:
            with np.errstate(invalid="ignore", divide="ignore"):
                ok &= avg[:, 0] >= p.eps
                ok &= self.rho_e(avg) >= p.eps
        elif p.system == SHALLOW_WATER:
            ok &= avg[:, 0] >= p.eps
        else:
            tau = self.average_slack()
            ok &= (avg[:, 0] >= p.bound_lo - tau) & (avg[:, 0] <= p.bound_hi + tau)
        return ok

    def average_slack(self):
        """Round-off margin of the scalar average check (A24): 2^-40 times the
        largest finite bound magnitude (at least 1).  Data that attain a bound
        exactly (an inflow state equal to M) leave averages a few ulp outside
        B through rounding alone, and no halving of dt removes that."""
        p = self.p
        mags = [1.0] + [abs(b) for b in (p.bound_lo, p.bound_hi) if math.isfinite(b)]
        return math.ldexp(max(mags), -40)

    def limit(self, U):
        """Scaling limiter on S_K (Prop. 2.4 for scalars; Sec. 2.2.3 density
        then internal-energy steps for Euler).  Cell averages are unchanged.
        Returns (limited U, theta[c])."""
        p = self.p
        if not p.limiter:
            return U.copy(), np.ones(U.shape[0])
        avg = self.cell_average(U)
        one = self.one[None, None, :]
        with np.errstate(invalid="ignore", divide="ignore"):
            if p.system == SHALLOW_WATER:
                # one factor from the depth, applied to every component (A28)
                hs = np.einsum("cm,pm->cp", U[:, 0, :], self.phi_s)
                hmin = hs.min(axis=1)
                hb = avg[:, 0]
                theta = np.ones(U.shape[0])
                bad = hmin < p.eps
                theta[bad] = (hb[bad] - p.eps) / (hb[bad] - hmin[bad])
                theta = np.clip(np.where(np.isnan(theta), 0.0, theta), 0.0, 1.0)
                out = theta[:, None, None] * (U - avg[:, :, None] * one) + avg[:, :, None] * one
                return out, theta
            if p.system != EULER:
                vals = np.einsum("cvm,pm->cvp", U, self.phi_s)[:, 0, :]
                ub = avg[:, 0]
                theta = np.ones(U.shape[0])
                Mk = vals.max(axis=1)
                mk = vals.min(axis=1)
                hi = Mk > p.bound_hi
                theta[hi] = np.minimum(theta[hi], (p.bound_hi - ub[hi]) / (Mk[hi] - ub[hi]))
                lo = mk < p.bound_lo
                theta[lo] = np.minimum(theta[lo], (p.bound_lo - ub[lo]) / (mk[lo] - ub[lo]))
                theta = np.clip(np.where(np.isnan(theta), 0.0, theta), 0.0, 1.0)
                out = theta[:, None, None] * (U - avg[:, :, None] * one) + avg[:, :, None] * one
                return out, theta
            eps = p.eps
            # step 1: density
            rho_s = np.einsum("cm,pm->cp", U[:, 0, :], self.phi_s)
            rmin = rho_s.min(axis=1)
            rb = avg[:, 0]
            th1 = np.ones(U.shape[0])
            bad = rmin < eps
            th1[bad] = (rb[bad] - eps) / (rb[bad] - rmin[bad])
            th1 = np.clip(np.where(np.isnan(th1), 0.0, th1), 0.0, 1.0)
            Uh = U.copy()
            Uh[:, 0, :] = th1[:, None] * (U[:, 0, :] - rb[:, None] * self.one) + rb[:, None] * self.one
            # step 2: internal energy of the density-limited polynomial (A7)
            us = np.einsum("cvm,pm->cpv", Uh, self.phi_s)
            emin = self.rho_e(us).min(axis=1)
            eb = self.rho_e(avg)
            th2 = np.ones(U.shape[0])
            bad = emin < eps
            th2[bad] = (eb[bad] - eps) / (eb[bad] - emin[bad])
            th2 = np.clip(np.where(np.isnan(th2), 0.0, th2), 0.0, 1.0)
            out = th2[:, None, None] * (Uh - avg[:, :, None] * one) + avg[:, :, None] * one
            return out, th1 * th2

    # ---------------- time stepping (Sec. 3.3, Sec. 4.1, Appendix B) ----------------
    def a0(self, U):
        """Per-direction maximum wave speed over the S_K points of U (A5)."""
        us = np.einsum("cvm,pm->cpv", U, self.phi_s)
        return np.array([np.max(self.wave_speed(us, dd)) for dd in range(self.d)])

    def trial_dt(self, U):
        """Trial step of Sec. 4.1, generalised to d dimensions by reading A2."""
        a = self.a0(U)
        return self.p.cfl / np.sum(a / self.dx)

    def source_term(self, t):
        """P s(t): the L2 projection of the source at time t (A25), or None."""
        if self.p.source is None:
            return None
        return self.project(lambda X: self.p.source(X, t))

    def stage(self, i, Un, tilde, dt, op=None, t=0.0):
        """Un-limited stage i (2..s) or the final stage (i = s+1) of Scheme 1L:
        u^(i) = u~^n + dt sum_j a_ij G(u~^(j)),  u^{n+1} = u~^n + dt sum_i b_i F(u~^(i)).
        `tilde` is the list [u~^(1) = u~^n, u~^(2), ...].  `op` overrides the
        operator of the inner stages (standard RKDG uses F everywhere).  With
        a source, each operator value gains P s at its stage time (A25); t is
        the time of u~^n."""
        A, b = BUTCHER[self.p.stages]
        c = A.sum(axis=1)
        s = self.p.stages
        out = Un.copy()
        ag = float(np.max(self.a0(Un))) if self.p.alpha == "global" else None   # a0 of u~^n (A1 option)

        def F(V, tj):
            return self.F(V, a_glob=ag, t=tj)

        def G(V, tj):
            return self.G(V)

        def with_source(value, j):
            src = self.source_term(t + c[j - 1] * dt)
            return value if src is None else value + src

        if i <= s:
            inner = G if op is None else (F if op == self.F else (lambda V, tj: op(V)))
            for j in range(1, i):
                if A[i - 1, j - 1] != 0.0:
                    out = out + dt * A[i - 1, j - 1] * with_source(inner(tilde[j - 1], t + c[j - 1] * dt), j)
        else:
            for j in range(1, s + 1):
                if b[j - 1] != 0.0:
                    out = out + dt * b[j - 1] * with_source(F(tilde[j - 1], t + c[j - 1] * dt), j)
        return out

    def attempt(self, Un, dt, op=None, t=0.0):
        """One step attempt from the limited u~^n at time t.  Returns
        (u~^{n+1}, ok)."""
        s = self.p.stages
        tilde = [Un]
        for i in range(2, s + 2):
            u = self.stage(i, Un, tilde, dt, op, t)
            if not np.all(self.admissible_average(self.cell_average(u))):
                return None, False
            tilde.append(self.limit(u)[0])
        return tilde[-1], True

    def step(self, Un, t=0.0, t_end=math.inf, dt_fixed=None, op=None):
        """One accepted step with the halving strategy of Sec. 4.1 (A10).
        Returns (u~^{n+1}, info dict)."""
        dt = dt_fixed if dt_fixed else self.trial_dt(Un)
        dt = min(dt, t_end - t)
        halvings = 0
        while True:
            out, ok = self.attempt(Un, dt, op, t)
            if ok:
                return out, dict(dt=dt, halvings=halvings, t=t + dt)
            halvings += 1
            if halvings > self.p.max_halvings:
                raise RuntimeError("time step underflow: max halvings exceeded")
            dt *= 0.5

    def run(self, U, t_end, dt_fixed=None, max_steps=10 ** 9):
        t = 0.0
        log = []
        steps = 0
        while t < t_end and steps < max_steps:
            U, info = self.step(U, t, t_end, dt_fixed)
            t = info["t"]
            log.append(info)
            steps += 1
        return U, t, log

    # ---------------- diagnostics ----------------
    def totals(self, U):
        """sum_K |K| ubar_K per variable (math.fsum)."""
        avg = self.cell_average(U)
        return np.array([math.fsum(self.vol * avg[:, v]) for v in range(self.V)])

    def sk_values(self, U):
        """u at the S_K points: [c, P, V]."""
        return np.einsum("cvm,pm->cpv", U, self.phi_s)

    def bound_violations(self, U):
        """Number of cells with an S_K value outside B (B^eps for Euler), a
        non-positive density, or a non-finite value.

        The values are taken from the Legendre coefficients C of U (every
        Legendre product satisfies |L_m| <= 1 on the cell).  A point counts
        as outside only beyond the FP64 rounding of its value: the coefficient
        conversion and the evaluation are sums of at most M + Q products, so
        tol_v = 8 (M + Q) 2^-53 sum_m |C_v,m|; for Euler the check is
        q = E rho - |m|^2 / 2 >= eps rho (rho e >= eps times rho > 0) with
        those errors carried through the products.  Scalar bounds also allow
        the round-off margin of the average check (A24).  Internal energy
        must be strictly positive wherever FP64 resolves eps rho (its
        tolerance is below eps rho)."""
        C = self.to_legendre(U)
        L = self._legendre_at(self.xs)                                 # [P, M]
        us = np.einsum("cvm,pm->cpv", C, L)
        u53 = 2.0 ** -53
        tol = 8.0 * (self.M + len(self.wq)) * u53 * np.sum(np.abs(C), axis=2)     # [c, V]
        p = self.p
        bad = ~np.all(np.isfinite(us), axis=(1, 2))
        with np.errstate(invalid="ignore", divide="ignore"):
            if p.system == EULER:
                d = self.d
                rho, mom, E = us[..., 0], us[..., 1:1 + d], us[..., 1 + d]
                tr, tm, tE = tol[:, None, 0], tol[:, None, 1:1 + d], tol[:, None, 1 + d]
                q = E * rho - 0.5 * np.sum(mom * mom, axis=-1)
                tol_q = (tE * np.abs(rho) + tr * np.abs(E) + np.sum(tm * np.abs(mom), axis=-1)
                         + 4.0 * u53 * (np.abs(E * rho) + 0.5 * np.sum(mom * mom, axis=-1)))
                bad |= np.any(rho <= 0.0, axis=1)
                bad |= np.any(rho < p.eps - tr, axis=1)
                bad |= np.any(q < p.eps * rho - tol_q, axis=1)
                bad |= np.any((q <= 0.0) & (tol_q < p.eps * rho), axis=1)
            elif p.system == SHALLOW_WATER:
                h, th = us[..., 0], tol[:, None, 0]
                bad |= np.any(h <= 0.0, axis=1)
                bad |= np.any(h < p.eps - th, axis=1)
            else:
                t = tol[:, None, 0] + self.average_slack()
                bad |= np.any(us[..., 0] > p.bound_hi + t, axis=1)
                bad |= np.any(us[..., 0] < p.bound_lo - t, axis=1)
        return int(np.sum(bad))

    def l1_norm(self, U, ref_fn=None, npts=None):
        """L1 norm per variable of U (minus ref_fn(x) if given) by a (k+2)^d
        Gauss rule per cell (reading A18)."""
        q = self.k + 2 if npts is None else npts
        g, w = gauss_legendre(q)
        x = np.array(list(itertools.product(g, repeat=self.d)))[:, ::-1].copy()
        wt = np.array([np.prod(v) for v in itertools.product(w, repeat=self.d)])
        vals = self.evaluate(U, x)                           # [c, V, P]
        if ref_fn is not None:
            X = self.physical_points(x)
            vals = vals - np.transpose(np.asarray(ref_fn(X)), (0, 2, 1))
        return np.einsum("p,cvp->v", wt, np.abs(vals)) * self.vol / 2.0 ** self.d


def make(prob: Problem) -> CRKDG:
    return CRKDG(prob)
