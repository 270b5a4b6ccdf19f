/*
 * crkdg.h -- C ABI of the MI355X (gfx950) library for the per-stage hot path
 * of the bound-preserving compact-stencil Runge--Kutta discontinuous Galerkin
 * method (cRKDG) of Liu, Sun and Zhang, arXiv 2412.16002.
 *
 * The library advances   d/dt u + div f(u) = 0   (Sec. 1, the conservation
 * law) on boxes with uniform Cartesian meshes, for one or many independent
 * instances ("problems") at once.  One time step is the Butcher-form cRKDG
 * scheme with the scaling limiter after every stage, in the limited form the
 * paper recommends (Appendix B, "Scheme 1L"):
 *     u^(i)   = u~^n + dt * a_{i,i-1} * G(u~^(i-1)),   u~^(i)   = L(u^(i)),   i = 2..s
 *     u^{n+1} = u~^n + dt * sum_i b_i F(u~^(i)),       u~^{n+1} = L(u^{n+1})
 * with G = -div^loc f (interior traces only, no neighbour data; Sec. 2.1) and
 * F = -div^DG f with the Lax--Friedrichs flux (Sec. 2.1), the Butcher tables of
 * Sec. 3.3, the scaling limiters of Sec. 2.2.2 (scalar, Prop. 2.4) and
 * Sec. 2.2.3 (Euler, density then internal energy), and the adaptive halving
 * strategy of Sec. 4.1.  Options of each problem: the standard RKDG scheme
 * of Sec. 2.1 instead (F in every stage, scheme = CRKDG_SCHEME_RKDG),
 * periodic, outflow, reflective or Dirichlet / inflow sides, and the
 * Lax--Friedrichs alpha per face, per face point or global (CRKDG_ALPHA_*).
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 * - All pointers whose name starts with d_ or that live inside crkdg_state are
 *   DEVICE pointers owned by the caller; the library never frees or allocates
 *   them.  The library's own device memory is allocated by crkdg_init_mesh
 *   (basis tables, tile maps, and the deferred-limiter queue: room for one
 *   record per cell, about one state's size) and freed by crkdg_free_mesh;
 *   crkdg_set_tuning may grow a tile map and crkdg_graph_create builds a
 *   graph.  The stepping entry points allocate nothing.
 * - `stream` is a hipStream_t (NULL = the default stream).  Work is enqueued
 *   asynchronously unless an entry point says it synchronises.
 * - Return value: 0 on success; negative = usage or runtime error
 *   (CRKDG_E_*), with a message from crkdg_last_error(); positive = numerical
 *   status (CRKDG_S_*).  Nothing throws, exits or aborts across the ABI.
 *   Asynchronous HIP faults surface at the next synchronising call.
 * - Results are deterministic: no floating-point atomics are used for sums.
 *
 * State layout (modal Legendre coefficients, structure of arrays)
 * ---------------------------------------------------------------
 * Per cell K the DG function of variable v is
 *     u_v(x) = sum_m c[v][m] * phi_m(xi),  xi = 2 (x - x_K) / dx in [-1, 1]^d,
 * phi_m(xi) = prod_j P_{e_j(m)}(xi_j) with Legendre polynomials P_n
 * (P_n(1) = 1, unnormalised), so c[v][0] is the cell average.  Mode order:
 *   1D and Q^k: e_0 fastest (m = e_0 + (k+1) e_1 + (k+1)^2 e_2);
 *   P^k (2D/3D total degree <= k): by total degree, then by decreasing e_0,
 *   then by decreasing e_1, e.g. 2D P^2: (0,0),(1,0),(0,1),(2,0),(1,1),(0,2).
 * Cells are numbered naturally, x fastest: K = i + n0 (j + n1 l).
 * A state holds two arrays:
 *   avg[v][K]        FP64, the cell averages c[v][0];
 *   hi [v][m-1][K]   modes m >= 1: double (CRKDG_FP64) or float (CRKDG_MIXED).
 * Several instances are packed one after the other; crkdg_instance_query gives
 * each instance's element offsets inside avg and hi.
 * Euler variables are (rho, m_1..m_d, E); gamma-law gas (Sec. 2.2.3).
 */
#ifndef CRKDG_H
#define CRKDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- enumerations ---------------------------------------------------- */
#define CRKDG_BC_PERIODIC 0
#define CRKDG_BC_OUTFLOW 1   /* exterior trace = interior trace */
#define CRKDG_BC_REFLECT 2   /* Euler wall: exterior trace = interior trace with the normal
                                momentum negated (mirror state; reflective sides of Sec. 4) */
#define CRKDG_BC_DIRICHLET 3 /* exterior trace = the prescribed state bc_state of the side
                                (Dirichlet and inflow sides of Sec. 4) */
/* Reflective and Dirichlet sides enter only the final stage (the inner stages
 * use no exterior data); every compiled family has them. */

#define CRKDG_SYS_ADVECTION 0 /* f(u) = a u, scalar */
#define CRKDG_SYS_BURGERS 1   /* f_d(u) = u^2 / 2, scalar */
#define CRKDG_SYS_EULER 2     /* compressible Euler, d + 2 variables */
#define CRKDG_SYS_SHALLOW_WATER 3 /* shallow water (h, h w_1..h w_d), d + 1 variables, flat
                                     bottom; the paper's Remark on other systems (Sec. 3.2) */

#define CRKDG_SPACE_Q 0 /* degree <= k in each variable (1D: P^k) */
#define CRKDG_SPACE_P 1 /* total degree <= k */

#define CRKDG_SCHEME_CRKDG 0 /* inner stages with the local operator G (Sec. 3.1, Scheme 1L of App. B) */
#define CRKDG_SCHEME_RKDG 1  /* standard RKDG (Sec. 2.1): F in every stage, same Butcher table,
                                limiter and check after every stage */

#define CRKDG_ALPHA_FACE 0  /* Lax-Friedrichs alpha per face: largest wave speed over the face's
                               quadrature points and both traces (the reading of Sec. 2.1 used
                               throughout); a trace without a real sound speed (pressure < 0,
                               e.g. FP32 rounding near vacuum) counts with its flow speed |w_d| */
#define CRKDG_ALPHA_POINT 1 /* alpha at each face quadrature point from its two traces (local
                               Lax-Friedrichs / Rusanov); a point whose speeds are undefined (a
                               zero or non-finite density) takes the face alpha */
#define CRKDG_ALPHA_GLOBAL 2 /* one alpha for every face: the wave-speed maximum a0 of Sec. 2.1,
                               max over d of crkdg_ctl.a0[d] (that of u~^n over S_K, which the
                               controller holds during a step; a caller of crkdg_stage sets it).
                               Neither option is built for 2D P^3 Euler FP64:
                               its init call returns CRKDG_E_UNSUPPORTED */

#define CRKDG_FP64 0  /* every mode and all arithmetic in FP64 */
#define CRKDG_MIXED 1 /* modes >= 1 and transforms/fluxes in FP32; averages,
                         admissibility checks, limiter theta and the
                         conservative average update in FP64 */

/* ---- status codes ---------------------------------------------------- */
#define CRKDG_OK 0
#define CRKDG_E_ARG (-1)         /* invalid argument */
#define CRKDG_E_HIP (-2)         /* HIP runtime error */
#define CRKDG_E_UNSUPPORTED (-3) /* valid problem, combination not built */
#define CRKDG_E_LAYOUT (-4)      /* buffer sizes / pointers inconsistent */
#define CRKDG_S_REJECTED 1       /* a stage cell average left the admissible set */
#define CRKDG_S_DT_UNDERFLOW 2   /* more than max_halvings halvings in one step */
#define CRKDG_S_NONFINITE 3      /* non-finite values met */
#define CRKDG_S_DONE 4           /* the instance reached t_end */

/* flag bits written into crkdg_ctl.flags by the stage kernels */
#define CRKDG_F_AVERAGE 1u   /* a cell average left B (scalar) / B^eps (Euler) */
#define CRKDG_F_NONFINITE 2u /* a non-finite cell average */

/* ---- problem description -------------------------------------------- */
typedef struct crkdg_problem {
  int32_t dim;       /* 1, 2 or 3 */
  int32_t n[3];      /* cells per direction (entries >= dim ignored) */
  double lo[3];      /* box corner */
  double hi[3];      /* opposite corner */
  int32_t bc[3];     /* CRKDG_BC_* per direction: the lower side, and the upper side
                        unless bc_upper overrides it; periodic means both sides */
  int32_t system;    /* CRKDG_SYS_* */
  double vel[3];     /* advection velocity (CRKDG_SYS_ADVECTION) */
  double gamma;      /* ratio of specific heats (Euler) */
  double bound_lo;   /* scalar invariant region B = [bound_lo, bound_hi] (Sec. 2.2.2); */
  double bound_hi;   /*   +-INFINITY disables that side.  The stage check accepts cell
                        averages within 2^-40 max(1, |bound_lo|, |bound_hi|) of B (finite
                        bounds only): round-off where the data attain a bound */
  double eps;        /* Euler admissible set: rho >= eps and rho e >= eps (Sec. 2.2.3) */
  int32_t k;         /* polynomial degree, 1..3 */
  int32_t space;     /* CRKDG_SPACE_* */
  int32_t stages;    /* 2, 3 or 4: the cRKDG schemes of Sec. 3.3 */
  int32_t precision; /* CRKDG_FP64 or CRKDG_MIXED */
  int32_t limiter;   /* 1: scaling limiter after every stage; 0: off */
  double cfl;        /* trial step dt = cfl / sum_d (a0_d / dx_d)   (Sec. 4.1) */
  int32_t max_halvings; /* bound on halvings within one step (Sec. 4.1) */
  int32_t scheme;    /* CRKDG_SCHEME_* (0, the cRKDG scheme, in a zeroed struct) */
  int32_t bc_upper[3]; /* upper side of direction d: 0 = as bc[d]; else CRKDG_BC_OUTFLOW,
                          _REFLECT or _DIRICHLET (a periodic direction takes 0) */
  int32_t alpha;     /* CRKDG_ALPHA_* (0, per face, in a zeroed struct) */
  double bc_state[6][5]; /* Dirichlet state of side 2 d + (upper side), conservative
                            variables (rho, m_1..m_dim, E; shallow water h, h w_1..h w_dim;
                            scalars use [0]); it must lie in the admissible set (B, or
                            B^eps for Euler and shallow water) */
  double gravity;    /* g of the shallow-water equations (> 0); their admissible set is
                        h >= eps */
} crkdg_problem;

typedef struct crkdg_mesh crkdg_mesh; /* opaque handle */

typedef struct crkdg_layout {
  int32_t n_inst;
  int32_t hi_bytes;   /* bytes of one hi element: 8 (FP64) or 4 (MIXED), same for all instances */
  int32_t n_slots;    /* state buffers one step needs: max over instances of stages + 1 */
  int32_t ctl_bytes;  /* bytes of one crkdg_ctl */
  int64_t avg_elems;  /* doubles in one state's avg array (all instances) */
  int64_t hi_elems;   /* elements in one state's hi array (all instances) */
} crkdg_layout;

typedef struct crkdg_instance_layout {
  int64_t n_cells;
  int32_t n_modes;    /* M */
  int32_t n_vars;     /* V */
  int32_t n_stages;   /* s */
  int32_t n_vol_pts;  /* (k+1)^d volume Gauss points */
  int32_t n_sk_pts;   /* points of the limiter set S_K */
  int32_t pad;
  int64_t avg_offset; /* element offset of this instance in avg */
  int64_t hi_offset;  /* element offset of this instance in hi */
  int64_t sample_offset; /* element offset of this instance's block in crkdg_project's samples:
                            the blocks ([v][K][q], n_vars x n_cells x n_vol_pts elements) are
                            packed in instance order */
} crkdg_instance_layout;

/* One state: device pointers to the two arrays described above. */
typedef struct crkdg_state {
  double *avg;
  void *hi;
} crkdg_state;

/* Per-instance time-step controller, in caller-owned DEVICE memory
 * (n_inst entries of layout.ctl_bytes = sizeof(crkdg_ctl)).  The stage
 * kernels read dt and the slot index from it and write flags and wave
 * speeds into it; the controller kernel of crkdg_step updates it.
 * crkdg_start initialises it; a caller that fills it by hand must set
 * status = 0 and goal = INT64_MAX, else every kernel skips the instance. */
typedef struct crkdg_ctl {
  double t;              /* time of u~^n */
  double t_end;          /* final time (INFINITY: none) */
  double dt;             /* trial step of the current attempt */
  double dt_fixed;       /* > 0: use this step instead of the CFL rule */
  double a0[3];          /* max wave speed of u~^n per direction over S_K */
  uint64_t a0_next[3];   /* same for the candidate u~^{n+1}: bits of non-negative doubles */
  uint32_t flags;        /* CRKDG_F_* raised during the current attempt */
  int32_t cur;           /* slot holding u~^n (crkdg_step) */
  int32_t halvings;      /* halvings in the current step */
  int32_t status;        /* 0 running, else CRKDG_S_DONE / _DT_UNDERFLOW / _NONFINITE */
  int64_t accepted;      /* accepted steps */
  int64_t rejected;      /* rejected attempts */
  int64_t goal;          /* kernels skip the instance once accepted >= goal */
  int64_t stages_run;    /* executed stages, accepted or not */
  double dt_last;        /* step size of the last accepted step */
  int32_t halvings_last; /* halvings the last accepted step needed */
  int32_t pad;
} crkdg_ctl;

typedef struct crkdg_step_info {
  double t;         /* time after the step */
  double dt;        /* step size taken */
  int32_t halvings; /* halvings needed in this step */
  int32_t status;   /* 0 or CRKDG_S_* */
  int32_t cur;      /* slot that now holds u~^{n+1} */
  int32_t pad;
  int64_t accepted, rejected;
} crkdg_step_info;

/* ---- entry points ----------------------------------------------------- */

/* Thread-local message of the last error (never NULL). */
const char *crkdg_last_error(void);

/* Validate `n_inst` problems, build the quadrature / basis / S_K tables in
 * FP64 (Gauss rule of k+1 points per direction, edge weights summing to one,
 * Prop. 2.1; S_K = Gauss x Gauss--Lobatto points, Prop. 2.2 and Fig. 1),
 * upload them, and fill *layout.  Synchronous.  Errors: CRKDG_E_ARG for an
 * invalid problem, CRKDG_E_UNSUPPORTED for a combination not compiled,
 * CRKDG_E_HIP.  Compiled, each in FP64 and mixed form: 1D P^1-P^3 (all
 * systems); 2D Q^1-Q^3 and P^1-P^3 (advection, Euler); 3D Q^1-Q^3 and
 * P^1-P^3 (advection, Euler).  Burgers is 1D only.  Shallow water: 1D P^1-P^3 and 2D Q^1-Q^3, P^1-P^3,
 * FP64 and mixed. */
int crkdg_init_mesh(const crkdg_problem *problems, int32_t n_inst, crkdg_mesh **out,
                    crkdg_layout *layout);

/* Free the handle and its device tables (NULL is accepted).  Synchronous. */
int crkdg_free_mesh(crkdg_mesh *mesh);

/* Sizes and offsets of instance `inst`. */
int crkdg_instance_query(const crkdg_mesh *mesh, int32_t inst, crkdg_instance_layout *out);

/* Reference coordinates in [-1,1]^3 (unused coordinates 0) of the points of
 * instance `inst`: which = 0 volume Gauss points (order used by
 * crkdg_project, first coordinate fastest), 1 the S_K points.  Writes at most
 * `cap` points into the host array xyz[cap][3] and their number to *count. */
int crkdg_points(const crkdg_mesh *mesh, int32_t inst, int32_t which, double *xyz, int32_t cap,
                 int32_t *count);

/* Discrete L2 projection with the volume Gauss rule (the initial-data
 * projection): d_samples holds u at the volume Gauss points of every cell,
 * layout [v][K][q] per instance, instance blocks packed one after another
 * (element offset sample_offset of crkdg_instance_query).  Writes the modal state `out`.  The result is not
 * limited: call crkdg_limit afterwards (the bound-preservation theorem,
 * Thm. 3.5, assumes a limited u^0). */
int crkdg_project(crkdg_mesh *mesh, const double *d_samples, crkdg_state out, void *stream);

/* Source term (right-hand side) of every instance, for the manufactured
 * solutions of the accuracy tests (Sec. 4.2, Example 4.2 scenario I):
 *   s(x, t) = sum_{p < n_terms} exp(-rate_p t) cos(omega_p t + phase_p) S_p(x),
 * with coef[3 p + 0..2] = (rate_p, omega_p, phase_p) (host array) and S_p
 * given as the modal state terms[p] (the mesh's layout and precision, e.g.
 * the crkdg_project of S_p's volume Gauss-point values; an instance without
 * a source holds zeros there).  Each operator value of a stage gains the
 * source at the time of the stage value it is applied to, t^n + c_j dt with
 * c_j the Butcher table's stage times: dt a_{i,i-1} g(t^n + c_{i-1} dt) S in
 * inner stage i, dt sum_j b_j g(t^n + c_j dt) S in the final stage.  The
 * mesh keeps the pointers (caller-owned device memory that must stay valid
 * while the mesh steps); n_terms = 0 removes the source.  At most
 * CRKDG_MAX_SOURCE_TERMS terms; refused (CRKDG_E_ARG) while step graphs of
 * the mesh exist, since they hold the previous source.  A source breaks
 * conservation by design, and the bound-preservation theorem does not cover
 * it: the halving of Sec. 4.1 still guards every stage average. */
#define CRKDG_MAX_SOURCE_TERMS 4
int crkdg_set_source(crkdg_mesh *mesh, int32_t n_terms, const crkdg_state *terms, const double *coef);

/* Time-dependent Dirichlet data on side `side` (2 d + upper) of instance
 * `inst`, e.g. the exact-solution boundary data of the accuracy tests
 * (Sec. 4.2): the exterior state at face point b of boundary face c is
 *   sum_{p < n_terms} exp(-rate_p t) cos(omega_p t + phase_p) values[p][c][b][v]
 * with coef[3 p + 0..2] = (rate_p, omega_p, phase_p) (host array) and
 * `values` a caller-owned DEVICE array of FP64 [n_terms][n_faces][n_fp][V]:
 * boundary faces c in natural order of the other directions (lower
 * direction fastest, n_faces their product), face points b the tensor
 * (k+1)-point Gauss points of the other directions (lower direction
 * fastest, ascending; the 1D nodes are the first coordinates of the first
 * k+1 volume points of crkdg_points), n_fp = (k+1)^(dim-1).  t is the time
 * of the stage value the operator F acts on, t^n + c_j dt (the inner stages
 * of the cRKDG scheme use no boundary data).  The side must be Dirichlet;
 * its bc_state still serves the admissibility check at mesh creation.  The
 * mesh keeps the pointer; n_terms = 0 returns the side to its constant
 * state.  Refused while step graphs of the mesh exist (CRKDG_E_ARG).
 * Synchronous. */
int crkdg_set_boundary_data(crkdg_mesh *mesh, int32_t inst, int32_t side, int32_t n_terms, const double *coef,
                            const double *values);

/* Scaling limiter in place (Prop. 2.4 scalar; Sec. 2.2.3 Euler).  Cell
 * averages are unchanged.  Cells whose average is outside B / B^eps raise
 * CRKDG_F_AVERAGE in d_ctl[inst].flags (theta is then clamped to [0,1]).
 * d_ctl may be NULL (no flags).  Asynchronous. */
int crkdg_limit(crkdg_mesh *mesh, crkdg_state u, crkdg_ctl *d_ctl, void *stream);

/* Cell averages (mode 0 of the Legendre basis is the average of u over K,
 * Sec. 2.1) in natural cell order, d_avg[v][K] per instance (same packing as
 * a state's avg array; may be NULL), and d_totals[inst][v] = sum_K |K| ubar_K
 * by a fixed-order tree reduction (may be NULL): the conserved totals, which
 * a periodic cRKDG step keeps unchanged (the local conservation remark at the
 * end of Sec. 3.2).  Deterministic: the same state gives bitwise the same
 * totals.  Uses a mesh-owned partial-sum buffer, so two calls on one mesh
 * must not overlap on different streams.  Asynchronous. */
int crkdg_cell_avg(crkdg_mesh *mesh, crkdg_state u, double *d_avg, double *d_totals,
                   void *stream);

/* crkdg_cell_avg for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same averages and bitwise the same totals, with the per-block partial
 * sums in a static device array of the library (1 MiB per GPU, held until
 * the process ends) instead of the mesh's buffer.  Allocates nothing, frees
 * nothing; the array's address is looked up once per device when a mesh is
 * created on it.  Limit: meshes of at most 26214 blocks of 256 cells (about
 * 6.7 million cells); larger ones are refused with CRKDG_E_ARG before any
 * device work.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (different streams, host threads or meshes) race.
 * Asynchronous. */
int crkdg_cell_avg_noalloc(crkdg_mesh *mesh, crkdg_state u, double *d_avg, double *d_totals,
                           void *stream);

/* CFL wave-speed reduction (Sec. 2.1 definition of a0; Sec. 4.1 trial step):
 * d_ctl[inst].a0[d] = max over cells and S_K points of the largest |eigenvalue|
 * of df_d/du at u, and d_ctl[inst].dt = the trial step (or dt_fixed), clipped
 * to t_end - t.  Asynchronous. */
int crkdg_cfl(crkdg_mesh *mesh, crkdg_state u, crkdg_ctl *d_ctl, void *stream);

/* Initialise the controllers (host arrays t0, t_end, dt_fixed of n_inst
 * entries; t_end may be NULL = no end, dt_fixed may be NULL = CFL rule), mark
 * `slots[cur]` as u~^n, compute a0 and the first trial step from it. The
 * state must already be limited.  Asynchronous (the host arrays are copied
 * before return). */
int crkdg_start(crkdg_mesh *mesh, const crkdg_state *slots, int32_t cur, crkdg_ctl *d_ctl,
                const double *t0, const double *t_end, const double *dt_fixed, void *stream);

/* One stage from explicit buffers, for stage-level checks.
 *   stage = 2..s    : out = L(u~^n + dt a_{stage,stage-1} G(u~^(stage-1)))
 *   stage = s+1     : out = L(u~^n + dt sum_j b_j F(u~^(j)))
 * states[0] = u~^n, states[j-1] = u~^(j) (j = 2..s); entries the stage does
 * not read may be anything.  dt = d_ctl[inst].dt.  Sets CRKDG_F_* flags in
 * d_ctl when an (unlimited) stage average is not admissible (the adaptive
 * strategy of Sec. 4.1 then rejects the step); on stage s+1 also stores the
 * wave speeds of the result in d_ctl[inst].a0_next (atomic max).  `out` must
 * not alias any state the stage reads. Asynchronous. */
int crkdg_stage(crkdg_mesh *mesh, int32_t stage, const crkdg_state *states, int32_t n_states,
                crkdg_state out, crkdg_ctl *d_ctl, void *stream);

/* One time step on the slot ring slots[0..layout.n_slots-1] (all instances).
 * The slot of u~^n is d_ctl[inst].cur; stage j lives in slot (cur + j - 1)
 * mod (s + 1); on acceptance cur advances by s.  Every step is checked as in
 * Sec. 4.1: a stage average outside the admissible set rejects the attempt,
 * halves dt and restarts from the untouched u~^n.
 *   info == NULL: enqueue ONE attempt for every running instance and return
 *     without synchronising (graph-capturable; the device controller
 *     accepts or rejects and computes the next trial dt).
 *   info != NULL: attempt until every running instance has accepted one step
 *     (or stopped), synchronising after each attempt; info[inst] receives
 *     the outcome.  Returns CRKDG_S_DT_UNDERFLOW / CRKDG_S_NONFINITE if any
 *     instance stopped on that, else 0. */
int crkdg_step(crkdg_mesh *mesh, const crkdg_state *slots, int32_t n_slots, crkdg_ctl *d_ctl,
               crkdg_step_info *info, void *stream);

/* ---- launch shapes, autotuning and step graphs ------------------------
 * The instances of a mesh fall into kernel groups: one group per compiled
 * variant (dim, k, space, system, precision) and stage count.  The stage
 * kernels of a group (crkdg_stage, crkdg_step) run with one launch shape:
 * workgroups of `threads` threads, each tile of `tile_x` x (threads / tile_x)
 * cells of one x-y plane (1D: `threads` consecutive cells), walked in an
 * XCD-ordered map either by one workgroup per tile (grid = 0) or by a
 * persistent grid of `grid` workgroups.  The shape changes which thread
 * handles which cell, never the arithmetic: results are bitwise identical
 * for every shape. */
typedef struct crkdg_tuning {
  int32_t threads;   /* 64, 128 or 256 */
  int32_t tile_x;    /* 2D/3D: power of two in [8, threads]; 1D: = threads */
  int32_t grid;      /* 0: one workgroup per tile; else a multiple of 8 */
  int32_t dim, k, space, stages, n_inst; /* read only: the group */
  int32_t n_items;   /* read only: tiles in the group's map */
  int32_t scheme;    /* read only: CRKDG_SCHEME_* of the group */
  int64_t n_cells;   /* read only: cells of the group */
  double ms;         /* read only: stage time of one attempt measured by crkdg_autotune */
} crkdg_tuning;

/* Number of kernel groups of the mesh. */
int crkdg_group_count(const crkdg_mesh *mesh, int32_t *n_groups);

/* Current launch shape of group `group` (default: 256 threads, 32-wide
 * tiles, one workgroup per tile). */
int crkdg_get_tuning(const crkdg_mesh *mesh, int32_t group, crkdg_tuning *out);

/* Set the launch shape of group `group` from threads, tile_x and grid
 * (CRKDG_E_ARG when out of range).  Synchronous (uploads the tile map). */
int crkdg_set_tuning(crkdg_mesh *mesh, int32_t group, const crkdg_tuning *t);

/* Autotuner: for every group, time `reps` passes of its stage kernels over
 * the slot ring (as crkdg_step would run them, without the controller) for
 * each candidate shape (threads 64/128/256, tile widths 8..64, one workgroup
 * per tile or persistent grids of 1024 and 2048) and keep the fastest.  Call
 * after crkdg_start: the passes read u~^n = slots[d_ctl.cur] and write only
 * the other slots; d_ctl and the internal queues are restored afterwards, so
 * the next crkdg_step proceeds exactly as without tuning.  Synchronous. */
int crkdg_autotune(crkdg_mesh *mesh, const crkdg_state *slots, int32_t n_slots, crkdg_ctl *d_ctl,
                   int32_t reps, void *stream);

/* A HIP graph of `attempts` consecutive crkdg_step attempts (info == NULL
 * form) on these slots and controllers, with the current launch shapes.
 * Launching it is equivalent to calling crkdg_step(..., NULL, stream)
 * `attempts` times; instances that finished skip the remaining attempts on
 * the device.  The buffers must outlive the graph, and the graph must be
 * destroyed before the mesh; while a graph of the mesh exists,
 * crkdg_set_tuning and crkdg_autotune fail with CRKDG_E_ARG (the graph uses
 * the mesh's tile maps). */
typedef struct crkdg_graph crkdg_graph;
int crkdg_graph_create(crkdg_mesh *mesh, const crkdg_state *slots, int32_t n_slots, crkdg_ctl *d_ctl,
                       int32_t attempts, crkdg_graph **out);
int crkdg_graph_launch(crkdg_graph *graph, void *stream);
int crkdg_graph_destroy(crkdg_graph *graph);

#ifdef __cplusplus
}
#endif

#endif /* CRKDG_H */
