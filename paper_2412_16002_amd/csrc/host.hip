// Host side of the C ABI declared in include/crkdg.h: validation, layout,
// variant dispatch, the device step controller and the deterministic totals.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "crkdg.h"
#include "variants.hpp"

using namespace crkdg;

namespace {

using Registry = int (*)(const VariantOps**);
const Registry kRegistries[] = {&variants_v1d, &variants_v2d_q_adv, &variants_v2d_p_adv, &variants_v2d_q12_euler, &variants_v2d_q3_euler, &variants_v2d_p_euler, &variants_v3d_q1, &variants_v3d_q2_adv, &variants_v3d_q2_euler, &variants_v3d_p, &variants_v3d_p2_euler, &variants_v3d_p3_euler, &variants_v3d_q3_euler, &variants_v3d_k3_adv, &variants_swe_1d_q, &variants_swe_2d_p};

thread_local std::string g_err = "";

// Partial sums of crkdg_cell_avg_noalloc (5 doubles per logical block of the
// default tile map): file-scope device memory, one copy per GPU the library
// runs on, held until the process ends.  Host code never uses the array's
// name as an address: the device address comes from hipGetSymbolAddress,
// once per device (in crkdg_init_mesh, with that device current).
constexpr int64_t kScratchDoubles = int64_t(1) << 17;   // 1 MiB
static __device__ __align__(256) double scratch[kScratchDoubles];
std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_ptr;   // device -> address of its scratch

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(CRKDG_E_HIP, std::string(#expr ": ") + hipGetErrorString(e_));  \
  } while (0)

// Butcher tables of the cRKDG schemes (Sec. 3.3): only the subdiagonal of A
// is non-zero for the three schemes.
struct Butcher {
  double a[5];  // a[i] = a_{i,i-1}, i = 2..s
  double b[4];
};
Butcher butcher(int s) {
  Butcher t{};
  if (s == 2) {
    t.a[2] = 0.5;
    t.b[0] = 0.0; t.b[1] = 1.0;
  } else if (s == 3) {
    t.a[2] = 1.0 / 3.0; t.a[3] = 2.0 / 3.0;
    t.b[0] = 0.25; t.b[1] = 0.0; t.b[2] = 0.75;
  } else {
    t.a[2] = 0.5; t.a[3] = 0.5; t.a[4] = 1.0;
    t.b[0] = 1.0 / 6.0; t.b[1] = 1.0 / 3.0; t.b[2] = 1.0 / 3.0; t.b[3] = 1.0 / 6.0;
  }
  return t;
}

const VariantOps* find_ops(int dim, int k, int space, int system, int precision) {
  const int sp = (dim == 1) ? SP_Q : space;
  for (Registry r : kRegistries) {
    const VariantOps* tab = nullptr;
    const int n = r(&tab);
    for (int i = 0; i < n; ++i) {
      const VariantOps& o = tab[i];
      if (o.dim == dim && o.k == k && o.space == sp && o.system == system && o.precision == precision)
        return &o;
    }
  }
  return nullptr;
}

// Launch shape of the stage kernels of one group (see crkdg_tuning).
struct Tune {
  int threads = BLOCK;          // workgroup size
  int tile_x = TILE_X;          // tile width (2D/3D); 1D: = threads
  int grid = 0;                 // 0: one workgroup per tile; else persistent grid
  double ms = 0.0;              // measured by the autotuner
};

struct Group {
  const VariantOps* ops;
  int stages;
  int scheme;                   // CRKDG_SCHEME_*: operator of the inner stages
  int dim;
  std::vector<int> insts;
  int nblocks = 0;              // default map: grid size (a multiple of 8, padded)
  BlockItem* d_bmap = nullptr;  // default map (256 threads, 32 x 8 tiles): all but the stage kernels
  Tune tune;                    // stage kernels
  int n_items = 0;              // entries of the stage map
  int smap_cap = 0;             // allocated entries of the stage map
  BlockItem* d_smap = nullptr;  // stage map (tiles of the tuned shape, XCD order)
  int64_t ncells = 0;           // cells of all instances of the group
  int64_t queue_off = 0;        // byte offset of the group's deferred-limiter queue
  unsigned qcap = 0;            // its record capacity
};

constexpr int QSTAGES = 8;      // queue counters per group, indexed by stage number

}  // namespace

struct crkdg_mesh {
  std::vector<crkdg_problem> probs;
  std::vector<crkdg_instance_layout> lay;
  crkdg_layout layout{};
  std::vector<InstDev> inst;
  std::vector<Group> groups;
  InstDev* d_inst = nullptr;
  double* d_partial = nullptr;  // [total logical blocks][5]
  char* d_queue = nullptr;      // deferred-limiter queue records, one region per group
  unsigned* d_qcount = nullptr; // [groups][QSTAGES] deferred-limiter queue lengths
  int total_lblocks = 0;
  int max_stages = 0;
  int device = 0;
  int live_graphs = 0;          // step graphs holding this mesh's stage maps
  Src src{};                    // source term (crkdg_set_source)
  double* d_srcw = nullptr;     // its per-stage weights [instance][SRC_STAGES][MAX_SRC]
  // with several kernel groups, one stream per group so that their stage
  // chains of an attempt overlap (fork and join through events)
  std::vector<hipStream_t> gstreams;
  std::vector<hipEvent_t> gjoin;
  hipEvent_t gfork = nullptr;
  // time-dependent Dirichlet data (crkdg_set_boundary_data)
  std::vector<BSide> bsides;    // [instance][6]
  BSide* d_bside = nullptr;
  double* d_bw = nullptr;       // [instance][6][BW_STAGES][MAX_SRC] time factors
  bool has_bdata = false;
};

namespace {

// Logical blocks of a group in instance-major, cell-ascending order, placed so
// that hardware dispatch (round-robin over the 8 XCDs) hands each XCD one
// contiguous run of logical blocks: neighbouring rows of the final stage then
// meet in the same L2.
std::vector<BlockItem> xcd_block_map(const std::vector<BlockItem>& logical) {
  const int nl = static_cast<int>(logical.size());
  const int nx = 8;
  const int chunk = (nl + nx - 1) / nx;
  BlockItem pad{};
  pad.inst = -1;
  pad.lblock = -1;
  std::vector<BlockItem> phys(static_cast<size_t>(chunk) * nx, pad);
  for (int b = 0; b < chunk * nx; ++b) {
    const int x = b % nx, j = b / nx;
    const int l = x * chunk + j;
    if (l < nl) phys[b] = logical[l];
  }
  return phys;
}

// Logical tiles of one instance for workgroups of `threads` threads and tiles
// `tile_x` cells wide (2D/3D), z-plane by z-plane, rows of tiles x fastest.
void instance_tiles(const crkdg_problem& p, int inst, int threads, int tile_x, int& lblock,
                    std::vector<BlockItem>& out) {
  int64_t nc = 1;
  for (int d = 0; d < p.dim; ++d) nc *= p.n[d];
  const int tx_cells = (p.dim == 1) ? threads : tile_x;
  const int ty_cells = (p.dim == 1) ? 1 : threads / tile_x;
  const int64_t tx = (p.dim == 1) ? (nc + threads - 1) / threads : (p.n[0] + tx_cells - 1) / tx_cells;
  const int64_t ty = (p.dim == 1) ? 1 : (p.n[1] + ty_cells - 1) / ty_cells;
  const int64_t tz = (p.dim == 3) ? p.n[2] : 1;
  for (int64_t z = 0; z < tz; ++z)
    for (int64_t y = 0; y < ty; ++y)
      for (int64_t x = 0; x < tx; ++x) {
        BlockItem it{};
        it.inst = inst;
        it.lblock = lblock++;
        it.x0 = static_cast<int32_t>(x * tx_cells);
        it.y0 = static_cast<int32_t>(y * ty_cells);
        it.z = static_cast<int32_t>(z);
        out.push_back(it);
      }
}

// Tiles of tx x ty x tz cells (cooperative stage kernels), x fastest.
void instance_tiles_3d(const crkdg_problem& p, int inst, const int* tile, int& lblock,
                       std::vector<BlockItem>& out) {
  const int n2 = (p.dim == 3) ? p.n[2] : 1;
  for (int z = 0; z < n2; z += tile[2])
    for (int y = 0; y < p.n[1]; y += tile[1])
      for (int x = 0; x < p.n[0]; x += tile[0]) {
        BlockItem it{};
        it.inst = inst;
        it.lblock = lblock++;
        it.x0 = x;
        it.y0 = y;
        it.z = z;
        out.push_back(it);
      }
}

int64_t instance_tile_count(const crkdg_problem& p, int threads, int tile_x) {
  int64_t nc = 1;
  for (int d = 0; d < p.dim; ++d) nc *= p.n[d];
  if (p.dim == 1) return (nc + threads - 1) / threads;
  const int ty_cells = threads / tile_x;
  return ((p.n[0] + tile_x - 1) / tile_x) * ((p.n[1] + ty_cells - 1) / ty_cells) * (p.dim == 3 ? p.n[2] : 1);
}

// boundary kind of side `up` (0 lower, 1 upper) of direction d
int side_bc(const crkdg_problem& p, int d, int up) {
  return (up && p.bc_upper[d] != 0) ? p.bc_upper[d] : p.bc[d];
}

int n_vars_of(int system, int dim) {
  if (system == CRKDG_SYS_EULER) return dim + 2;
  return system == CRKDG_SYS_SHALLOW_WATER ? dim + 1 : 1;
}

// a prescribed boundary state inside B (scalar) or B^eps (Euler, shallow water)
bool admissible_state(const crkdg_problem& p, const double* u) {
  const int V = n_vars_of(p.system, p.dim);
  for (int v = 0; v < V; ++v)
    if (!std::isfinite(u[v])) return false;
  if (p.system == CRKDG_SYS_SHALLOW_WATER) return u[0] >= p.eps;
  if (p.system != CRKDG_SYS_EULER) return u[0] >= p.bound_lo && u[0] <= p.bound_hi;
  double m2 = 0.0;
  for (int d = 0; d < p.dim; ++d) m2 += u[1 + d] * u[1 + d];
  return u[0] >= p.eps && u[p.dim + 1] - 0.5 * m2 / u[0] >= p.eps;
}

int validate(const crkdg_problem& p, int idx) {
  auto bad = [&](const char* what) {
    return fail(CRKDG_E_ARG, "problem " + std::to_string(idx) + ": " + what);
  };
  if (p.dim < 1 || p.dim > 3) return bad("dim must be 1, 2 or 3");
  for (int d = 0; d < p.dim; ++d) {
    if (p.n[d] < 1) return bad("n must be >= 1");
    if (!(p.hi[d] > p.lo[d])) return bad("hi must exceed lo");
    if (p.bc[d] < CRKDG_BC_PERIODIC || p.bc[d] > CRKDG_BC_DIRICHLET) return bad("unknown bc");
    if (p.bc_upper[d] < 0 || p.bc_upper[d] > CRKDG_BC_DIRICHLET) return bad("unknown bc_upper");
    if (p.bc[d] == CRKDG_BC_PERIODIC && p.bc_upper[d] != 0)
      return bad("a periodic direction is periodic on both sides (bc_upper must be 0)");
    for (int up = 0; up < 2; ++up) {
      const int kind = side_bc(p, d, up);
      if (kind == CRKDG_BC_REFLECT && p.system != CRKDG_SYS_EULER && p.system != CRKDG_SYS_SHALLOW_WATER)
        return bad("reflective walls are defined for the Euler and shallow-water equations");
      if (kind == CRKDG_BC_DIRICHLET && !admissible_state(p, p.bc_state[2 * d + up]))
        return bad("Dirichlet state not finite or outside the admissible set");
    }
  }
  if (p.system < 0 || p.system > 3) return bad("unknown system");
  if (p.k < 1 || p.k > 3) return bad("k must be 1..3");
  if (p.space != CRKDG_SPACE_Q && p.space != CRKDG_SPACE_P) return bad("unknown space");
  if (p.stages < 2 || p.stages > 4) return bad("stages must be 2, 3 or 4");
  if (p.precision != CRKDG_FP64 && p.precision != CRKDG_MIXED) return bad("unknown precision");
  if (p.system == CRKDG_SYS_EULER && !(p.gamma > 1.0)) return bad("gamma must exceed 1");
  if ((p.system == CRKDG_SYS_EULER || p.system == CRKDG_SYS_SHALLOW_WATER) && !(p.eps > 0.0))
    return bad("eps must be positive");
  if (p.system == CRKDG_SYS_SHALLOW_WATER && !(p.gravity > 0.0)) return bad("gravity must be positive");
  if (p.system != CRKDG_SYS_EULER && p.system != CRKDG_SYS_SHALLOW_WATER && !(p.bound_lo <= p.bound_hi))
    return bad("bound_lo > bound_hi");
  if (!(p.cfl > 0.0)) return bad("cfl must be positive");
  if (p.max_halvings < 0) return bad("max_halvings must be >= 0");
  if (p.scheme != CRKDG_SCHEME_CRKDG && p.scheme != CRKDG_SCHEME_RKDG) return bad("unknown scheme");
  if (p.alpha != CRKDG_ALPHA_FACE && p.alpha != CRKDG_ALPHA_POINT && p.alpha != CRKDG_ALPHA_GLOBAL)
    return bad("unknown alpha");
  int64_t nc = 1;
  for (int d = 0; d < p.dim; ++d) nc *= p.n[d];
  if (nc > INT32_MAX) return bad("more than 2^31 - 1 cells in one instance");
  return CRKDG_OK;
}

__global__ void k_zero_u32(unsigned* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// Weights of the source terms in stage `stage` of every instance with
// `stages` stages, from its controller's t^n and dt: dt a_{i,i-1} g_p(t^n +
// c_{i-1} dt) in an inner stage i, dt sum_j b_j g_p(t^n + c_j dt) in the final
// stage, g_p(t) = exp(-rate_p t) cos(omega_p t + phase_p).  One thread per
// instance; idle instances are skipped as the stage kernels skip them.
struct StageCoef {
  double a;      // a_{stage, stage-1}
  double b[4];
  double c[4];   // stage times c_1..c_s
};
__global__ void k_source_weights(const InstDev* inst, const crkdg_ctl* ctl, int n, int group, int stages,
                                 int stage, StageCoef sc, Src src) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || inst[i].group != group || instance_idle(ctl + i)) return;
  const double t = ctl[i].t, dt = ctl[i].dt;
  double* w = src.w + (static_cast<int64_t>(i) * SRC_STAGES + stage) * MAX_SRC;
  for (int p = 0; p < src.n; ++p) {
    auto g = [&](double cj) {
      const double tj = t + cj * dt;
      return exp(-src.rate[p] * tj) * cos(fma(src.omega[p], tj, src.phase[p]));
    };
    double k = 0.0;
    if (stage > stages) {
      for (int j = 0; j < stages; ++j)
        if (sc.b[j] != 0.0) k += sc.b[j] * g(sc.c[j]);
    } else {
      k = sc.a * g(sc.c[stage - 2]);
    }
    w[p] = dt * k;
  }
}

// Time factors g_p(t^n + c_j dt), j = 0..s-1, of the time-dependent boundary
// data of every instance of `group` (one thread per instance and side).
__global__ void k_boundary_weights(const InstDev* inst, const crkdg_ctl* ctl, const BSide* bside, double* bw,
                                   int n, int group, int stages, StageCoef sc) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = e / 6, f = e % 6;
  if (i >= n || inst[i].group != group || !(inst[i].bdyn & (1u << f)) || instance_idle(ctl + i)) return;
  const BSide& bs = bside[e];
  const double t = ctl[i].t, dt = ctl[i].dt;
  double* w = bw + static_cast<int64_t>(e) * BW_STAGES * MAX_SRC;
  for (int j = 0; j < stages && j < BW_STAGES; ++j) {
    const double tj = t + sc.c[j] * dt;
    for (int p = 0; p < bs.n_terms; ++p)
      w[j * MAX_SRC + p] = exp(-bs.coef[p][0] * tj) * cos(fma(bs.coef[p][1], tj, bs.coef[p][2]));
  }
}

__global__ void k_controller(crkdg_ctl* ctl, const InstDev* inst, int n, unsigned* qcount, int nq) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  // every deferred-limiter queue of this attempt has been drained
  for (int k = i; k < nq; k += gridDim.x * blockDim.x) qcount[k] = 0u;
  if (i >= n) return;
  crkdg_ctl& c = ctl[i];
  const InstDev& I = inst[i];
  if (c.status != 0 || c.accepted >= c.goal) return;
  c.stages_run += I.stages;
  if (c.flags != 0u) {
    // Sec. 4.1: restart the step from u~^n with half the step size
    c.rejected += 1;
    c.halvings += 1;
    c.flags = 0u;
    for (int d = 0; d < 3; ++d) c.a0_next[d] = 0ull;
    if (c.halvings > I.max_halvings) c.status = CRKDG_S_DT_UNDERFLOW;
    else c.dt *= 0.5;
    return;
  }
  c.accepted += 1;
  c.dt_last = c.dt;
  c.halvings_last = c.halvings;
  c.halvings = 0;
  c.t = c.t + c.dt;
  c.cur = (c.cur + I.stages) % (I.stages + 1);
  double rate = 0.0;
  bool finite = true;
  for (int d = 0; d < 3; ++d) {
    const double a = __longlong_as_double(static_cast<long long>(c.a0_next[d]));
    c.a0[d] = a;
    c.a0_next[d] = 0ull;
    finite = finite && isfinite(a);
    rate += a * I.rdx[d];
  }
  if (!finite) { c.status = CRKDG_S_NONFINITE; return; }
  if (!(c.t < c.t_end)) { c.status = CRKDG_S_DONE; return; }
  double dt = (c.dt_fixed > 0.0) ? c.dt_fixed : I.cfl / rate;
  c.dt = fmin(dt, c.t_end - c.t);
}

// a0 = a0_next, a0_next = 0, trial dt (Sec. 4.1, reading A2 in several dimensions)
__global__ void k_a0_finish(crkdg_ctl* ctl, const InstDev* inst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  crkdg_ctl& c = ctl[i];
  const InstDev& I = inst[i];
  double rate = 0.0;
  for (int d = 0; d < 3; ++d) {
    const double a = __longlong_as_double(static_cast<long long>(c.a0_next[d]));
    c.a0[d] = a;
    c.a0_next[d] = 0ull;
    rate += a * I.rdx[d];
  }
  const double dt = (c.dt_fixed > 0.0) ? c.dt_fixed : I.cfl / rate;
  c.dt = fmin(dt, c.t_end - c.t);
}

__global__ void k_clear_a0(crkdg_ctl* ctl, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int d = 0; d < 3; ++d) ctl[i].a0_next[d] = 0ull;
}

__global__ void k_arm(crkdg_ctl* ctl, int n, int disarm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  ctl[i].goal = disarm ? INT64_MAX : ctl[i].accepted + 1;
}

// per-block sums of |K| * ubar in a fixed tree order
__global__ __launch_bounds__(BLOCK) void k_totals_partial(const InstDev* inst, const BlockItem* bmap,
                                                          const double* avg, double* partial, int V) {
  const BlockItem bi = bmap[blockIdx.x];
  if (bi.inst < 0) return;
  const InstDev& I = inst[bi.inst];
  __shared__ double sh[BLOCK];
  bool active;
  const int64_t c = tile_cell(bi, I.dim, I.n, I.ncell, TILE_SHIFT, active);
  for (int v = 0; v < V; ++v) {
    sh[threadIdx.x] = active ? I.vol * avg[I.avg_off + v * I.ncell + c] : 0.0;
    __syncthreads();
    for (int s = BLOCK / 2; s > 0; s >>= 1) {
      if (static_cast<int>(threadIdx.x) < s) sh[threadIdx.x] += sh[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[static_cast<int64_t>(bi.lblock) * 5 + v] = sh[0];
    __syncthreads();
  }
}

__global__ __launch_bounds__(BLOCK) void k_totals_final(const InstDev* inst, const double* partial,
                                                        double* totals, int V) {
  const InstDev& I = inst[blockIdx.x];
  __shared__ double sh[BLOCK];
  for (int v = 0; v < V; ++v) {
    double s = 0.0;
    for (int b = threadIdx.x; b < I.n_blocks; b += BLOCK)
      s += partial[static_cast<int64_t>(I.first_block + b) * 5 + v];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int k = BLOCK / 2; k > 0; k >>= 1) {
      if (static_cast<int>(threadIdx.x) < k) sh[threadIdx.x] += sh[threadIdx.x + k];
      __syncthreads();
    }
    if (threadIdx.x == 0) totals[blockIdx.x * V + v] = sh[0];
    __syncthreads();
  }
}

// The device address of `scratch` on the current device `dev` (looked up
// once per device; later calls return the stored address).
int scratch_address(int dev, double** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) {
    *out = it->second;
    return CRKDG_OK;
  }
  double* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(reinterpret_cast<void**>(&p), HIP_SYMBOL(scratch));
  if (e != hipSuccess || p == nullptr)
    return fail(CRKDG_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch_ptr[dev] = p;
  *out = p;
  return CRKDG_OK;
}

int check_mesh(const crkdg_mesh* m) {
  if (!m) return fail(CRKDG_E_ARG, "mesh is NULL");
  return CRKDG_OK;
}

int check_state(const crkdg_state& s, const char* what) {
  if (!s.avg || !s.hi) return fail(CRKDG_E_ARG, std::string(what) + ": NULL state array");
  return CRKDG_OK;
}

KArgs base_args(const crkdg_mesh* m, const Group& g, crkdg_ctl* ctl) {
  KArgs a{};
  a.inst = m->d_inst;
  a.bmap = g.d_bmap;
  a.n_items = g.nblocks;
  a.tile_shift = TILE_SHIFT;
  a.ctl = ctl;
  a.src = m->src;
  a.bside = m->has_bdata ? m->d_bside : nullptr;
  a.bw = m->d_bw;
  // stage times c_j = a_{j,j-1} (c_1 = 0): the tables are subdiagonal
  const Butcher bt = butcher(g.stages);
  for (int j = 1; j < 4; ++j) a.c[j] = (j < g.stages) ? bt.a[j + 1] : 0.0;
  return a;
}

int ilog2(int x) {
  int r = 0;
  while ((1 << r) < x) ++r;
  return r;
}

// Check a launch shape for a group: workgroups of 64, 128 or 256 threads;
// 2D/3D tiles a power of two between 8 and the workgroup size wide; a
// persistent grid a positive multiple of 8.
int check_tune(const Group& g, const Tune& t) {
  if (g.ops->coop) {
    // one workgroup (one wavefront per variable) per tile of the variant's shape
    if (t.threads != g.ops->coop || t.tile_x != g.ops->coop_tile[0] || t.grid != 0)
      return fail(CRKDG_E_ARG, "this variant runs cooperative stage kernels: threads must be " +
                                   std::to_string(g.ops->coop) + ", tile_x " +
                                   std::to_string(g.ops->coop_tile[0]) + " and grid 0");
    return CRKDG_OK;
  }
  if (t.threads != 64 && t.threads != 128 && t.threads != 256)
    return fail(CRKDG_E_ARG, "threads must be 64, 128 or 256");
  if (g.dim == 1) {
    if (t.tile_x != t.threads) return fail(CRKDG_E_ARG, "1D: tile_x must equal threads");
  } else if (t.tile_x < 8 || t.tile_x > t.threads || (t.tile_x & (t.tile_x - 1)) != 0) {
    return fail(CRKDG_E_ARG, "tile_x must be a power of two in [8, threads]");
  }
  if (t.grid < 0 || t.grid % 8 != 0) return fail(CRKDG_E_ARG, "grid must be 0 or a positive multiple of 8");
  return CRKDG_OK;
}

// Build and upload the stage map of group gi for launch shape t (synchronous).
int apply_tune(crkdg_mesh* m, int gi, const Tune& t) {
  Group& g = m->groups[gi];
  if (int rc = check_tune(g, t)) return rc;
  if (m->live_graphs > 0)
    return fail(CRKDG_E_ARG, "launch shapes are fixed while a step graph of the mesh exists");
  std::vector<BlockItem> logical;
  int lb = 0;
  for (int i : g.insts) {
    if (g.ops->coop) instance_tiles_3d(m->probs[i], i, g.ops->coop_tile, lb, logical);
    else instance_tiles(m->probs[i], i, t.threads, t.tile_x, lb, logical);
  }
  std::vector<BlockItem> phys = xcd_block_map(logical);
  const int n = static_cast<int>(phys.size());
  if (n > g.smap_cap) {
    if (g.d_smap) HIP_TRY(hipFree(g.d_smap));
    g.d_smap = nullptr;
    g.smap_cap = 0;
    HIP_TRY(hipMalloc(&g.d_smap, sizeof(BlockItem) * n));
    g.smap_cap = n;
  }
  HIP_TRY(hipMemcpy(g.d_smap, phys.data(), sizeof(BlockItem) * n, hipMemcpyHostToDevice));
  g.n_items = n;
  g.tune = t;
  return CRKDG_OK;
}

// Grid of the stage kernels: one workgroup per tile, or the persistent grid
// (never more workgroups than tiles).
int stage_grid(const Group& g) {
  return (g.tune.grid > 0) ? std::min(g.tune.grid, g.n_items) : g.n_items;
}


int set_device(const crkdg_mesh* m) {
  HIP_TRY(hipSetDevice(m->device));
  return CRKDG_OK;
}

}  // namespace

extern "C" {

const char* crkdg_last_error(void) { return g_err.c_str(); }

int crkdg_init_mesh(const crkdg_problem* problems, int32_t n_inst, crkdg_mesh** out,
                    crkdg_layout* layout) {
  if (!problems || n_inst < 1 || !out || !layout) return fail(CRKDG_E_ARG, "bad arguments");
  *out = nullptr;
  for (int i = 0; i < n_inst; ++i) {
    const int rc = validate(problems[i], i);
    if (rc) return rc;
  }
  const int prec = problems[0].precision;
  for (int i = 1; i < n_inst; ++i)
    if (problems[i].precision != prec)
      return fail(CRKDG_E_ARG, "all instances of a mesh must share one precision");

  auto* m = new crkdg_mesh();
  m->probs.assign(problems, problems + n_inst);
  if (hipGetDevice(&m->device) != hipSuccess) {
    delete m;
    return fail(CRKDG_E_HIP, "hipGetDevice failed");
  }
  {
    // set-up of the allocation-free totals: this device's scratch address
    double* sp = nullptr;
    if (int rc = scratch_address(m->device, &sp)) {
      delete m;
      return rc;
    }
  }
  std::map<std::tuple<const VariantOps*, int, int>, int> gidx;
  int64_t avg_off = 0, hi_off = 0, smp_off = 0;
  m->inst.resize(n_inst);
  m->lay.resize(n_inst);
  std::vector<std::vector<BlockItem>> logical;
  int lblock = 0;
  for (int i = 0; i < n_inst; ++i) {
    const crkdg_problem& p = problems[i];
    const VariantOps* ops = find_ops(p.dim, p.k, p.space, p.system, p.precision);
    if (!ops) {
      delete m;
      return fail(CRKDG_E_UNSUPPORTED, "problem " + std::to_string(i) +
                                           ": no compiled kernel for this dim/k/space/system/precision");
    }
    if (!ops->walls)
      for (int d = 0; d < p.dim; ++d)
        for (int up = 0; up < 2; ++up)
          if (side_bc(p, d, up) == CRKDG_BC_REFLECT || side_bc(p, d, up) == CRKDG_BC_DIRICHLET) {
            delete m;
            return fail(CRKDG_E_UNSUPPORTED, "problem " + std::to_string(i) +
                                                 ": reflective and Dirichlet sides are not built for this "
                                                 "dim/k/space/system/precision");
          }
    if (!ops->alpha_modes && p.alpha != CRKDG_ALPHA_FACE) {
      delete m;
      return fail(CRKDG_E_UNSUPPORTED, "problem " + std::to_string(i) +
                                           ": the per-point and global Lax-Friedrichs alpha are not built "
                                           "for this dim/k/space/system/precision (2D P^3 Euler FP64)");
    }
    int64_t nc = 1;
    for (int d = 0; d < p.dim; ++d) nc *= p.n[d];
    if (ops->coop && nc >= (int64_t(1) << 29)) {
      // the cooperative kernels address a cell's row entries with 32-bit
      // byte offsets (such a mesh would not fit in device memory anyway)
      delete m;
      return fail(CRKDG_E_UNSUPPORTED, "problem " + std::to_string(i) +
                                           ": this variant takes fewer than 2^29 cells per instance");
    }
    crkdg_instance_layout& L = m->lay[i];
    L.n_cells = nc;
    L.n_modes = ops->M;
    L.n_vars = ops->V;
    L.n_stages = p.stages;
    L.n_vol_pts = ops->NQ;
    L.n_sk_pts = ops->NS;
    L.avg_offset = avg_off;
    L.hi_offset = hi_off;
    L.sample_offset = smp_off;
    avg_off += static_cast<int64_t>(ops->V) * nc;
    hi_off += static_cast<int64_t>(ops->V) * (ops->M - 1) * nc;
    smp_off += static_cast<int64_t>(ops->V) * ops->NQ * nc;

    InstDev& I = m->inst[i];
    std::memset(&I, 0, sizeof(I));
    I.ncell = nc;
    I.avg_off = L.avg_offset;
    I.hi_off = L.hi_offset;
    I.smp_off = L.sample_offset;
    double vol = 1.0;
    for (int d = 0; d < 3; ++d) {
      if (d < p.dim) {
        const double dx = (p.hi[d] - p.lo[d]) / p.n[d];
        I.n[d] = p.n[d];
        for (int up = 0; up < 2; ++up) {
          I.bc[2 * d + up] = side_bc(p, d, up);
          for (int v = 0; v < 5; ++v) I.bcs[2 * d + up][v] = p.bc_state[2 * d + up][v];
        }
        I.rdx[d] = 1.0 / dx;
        I.r2dx[d] = 2.0 / dx;
        I.vel[d] = p.vel[d];
        vol *= dx;
      } else {
        I.n[d] = 1;
        I.bc[2 * d] = I.bc[2 * d + 1] = CRKDG_BC_PERIODIC;
      }
    }
    I.vol = vol;
    I.dim = p.dim;
    I.stages = p.stages;
    I.limiter = p.limiter;
    I.alpha_mode = p.alpha;
    I.max_halvings = p.max_halvings;
    I.gamma = p.gamma;
    I.grav = p.gravity;
    I.blo = p.bound_lo;
    I.bhi = p.bound_hi;
    {
      // averages within 2^-40 max(1, |m|, |M|) of B pass the check: data
      // that attain a bound leave averages a few ulp outside it by rounding
      double mag = 1.0;
      if (std::isfinite(p.bound_lo)) mag = std::max(mag, std::fabs(p.bound_lo));
      if (std::isfinite(p.bound_hi)) mag = std::max(mag, std::fabs(p.bound_hi));
      const double tau = std::ldexp(mag, -40);
      I.blo_chk = p.bound_lo - tau;
      I.bhi_chk = p.bound_hi + tau;
    }
    I.eps = p.eps;
    I.cfl = p.cfl;
    m->max_stages = std::max(m->max_stages, p.stages);

    auto key = std::make_tuple(ops, p.stages, p.scheme);
    auto it = gidx.find(key);
    int g;
    if (it == gidx.end()) {
      g = static_cast<int>(m->groups.size());
      gidx[key] = g;
      Group G;
      G.ops = ops;
      G.stages = p.stages;
      G.scheme = p.scheme;
      m->groups.push_back(G);
      logical.emplace_back();
    } else {
      g = it->second;
    }
    m->groups[g].insts.push_back(i);
    m->groups[g].dim = p.dim;
    I.group = g;
    // the smallest tiles any tuning may use (64 threads) must stay countable
    const int64_t nb = instance_tile_count(p, BLOCK, TILE_X);
    if (nb + lblock > (int64_t(1) << 30) || instance_tile_count(p, 64, 8) > (int64_t(1) << 30)) {
      delete m;
      return fail(CRKDG_E_ARG, "too many cells in total");
    }
    I.first_block = lblock;
    I.n_blocks = static_cast<int>(nb);
    instance_tiles(p, i, BLOCK, TILE_X, lblock, logical[g]);
  }
  m->total_lblocks = lblock;

  auto cleanup = [&](const char* what, hipError_t e) {
    crkdg_free_mesh(m);
    return fail(CRKDG_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  };
  hipError_t e;
  if ((e = hipMalloc(&m->d_inst, sizeof(InstDev) * n_inst)) != hipSuccess) return cleanup("hipMalloc", e);
  if ((e = hipMemcpy(m->d_inst, m->inst.data(), sizeof(InstDev) * n_inst, hipMemcpyHostToDevice)) != hipSuccess)
    return cleanup("hipMemcpy", e);
  if ((e = hipMalloc(&m->d_partial, sizeof(double) * 5 * std::max(1, lblock))) != hipSuccess)
    return cleanup("hipMalloc", e);
  for (size_t g = 0; g < m->groups.size(); ++g) {
    std::vector<BlockItem> phys = xcd_block_map(logical[g]);
    Group& G = m->groups[g];
    G.nblocks = static_cast<int>(phys.size());
    if ((e = hipMalloc(&G.d_bmap, sizeof(BlockItem) * phys.size())) != hipSuccess) return cleanup("hipMalloc", e);
    if ((e = hipMemcpy(G.d_bmap, phys.data(), sizeof(BlockItem) * phys.size(), hipMemcpyHostToDevice)) != hipSuccess)
      return cleanup("hipMemcpy", e);
  }

  for (size_t g = 0; g < m->groups.size(); ++g) {
    Tune t;
    if (m->groups[g].dim == 1) t.tile_x = t.threads;
    if (m->groups[g].ops->coop) {
      t.threads = m->groups[g].ops->coop;
      t.tile_x = m->groups[g].ops->coop_tile[0];
    }
    if (int rc = apply_tune(m, static_cast<int>(g), t)) {
      crkdg_free_mesh(m);
      return rc;
    }
  }

  // deferred-limiter queue: one record per cell of the group, so a stage
  // can queue every cell (allocated once, with the mesh)
  int64_t qtotal = 0;
  for (Group& G : m->groups) {
    G.ncells = 0;
    for (int i : G.insts) G.ncells += m->lay[i].n_cells;
    if (G.ncells > UINT32_MAX) {
      crkdg_free_mesh(m);
      return fail(CRKDG_E_ARG, "more than 2^32 - 1 cells share one kernel variant");
    }
    G.qcap = static_cast<unsigned>(G.ncells);
    G.queue_off = qtotal;
    qtotal += static_cast<int64_t>(G.qcap) * G.ops->rec_bytes;
    qtotal = (qtotal + 255) / 256 * 256;
  }
  if ((e = hipMalloc(&m->d_queue, std::max<int64_t>(256, qtotal))) != hipSuccess)
    return cleanup("hipMalloc", e);
  const int nq = static_cast<int>(m->groups.size()) * QSTAGES;
  if ((e = hipMalloc(&m->d_qcount, sizeof(unsigned) * nq)) != hipSuccess) return cleanup("hipMalloc", e);
  if ((e = hipMemset(m->d_qcount, 0, sizeof(unsigned) * nq)) != hipSuccess) return cleanup("hipMemset", e);
  if (m->groups.size() > 1) {
    // streams (default priority) and events for the overlapped group chains
    if ((e = hipEventCreateWithFlags(&m->gfork, hipEventDisableTiming)) != hipSuccess)
      return cleanup("hipEventCreateWithFlags", e);
    for (size_t gi = 0; gi < m->groups.size(); ++gi) {
      hipStream_t st = nullptr;
      hipEvent_t ev = nullptr;
      if ((e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking)) != hipSuccess)
        return cleanup("hipStreamCreateWithFlags", e);
      m->gstreams.push_back(st);
      if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess)
        return cleanup("hipEventCreateWithFlags", e);
      m->gjoin.push_back(ev);
    }
  }

  crkdg_layout& lo = m->layout;
  lo.n_inst = n_inst;
  lo.hi_bytes = (prec == CRKDG_FP64) ? 8 : 4;
  lo.n_slots = m->max_stages + 1;
  lo.ctl_bytes = static_cast<int32_t>(sizeof(crkdg_ctl));
  lo.avg_elems = avg_off;
  lo.hi_elems = hi_off;
  *layout = lo;
  *out = m;
  return CRKDG_OK;
}

int crkdg_free_mesh(crkdg_mesh* m) {
  if (!m) return CRKDG_OK;
  hipSetDevice(m->device);
  for (Group& g : m->groups) {
    if (g.d_bmap) hipFree(g.d_bmap);
    if (g.d_smap) hipFree(g.d_smap);
  }
  if (m->d_inst) hipFree(m->d_inst);
  if (m->d_partial) hipFree(m->d_partial);
  if (m->d_queue) hipFree(m->d_queue);
  if (m->d_qcount) hipFree(m->d_qcount);
  if (m->d_srcw) hipFree(m->d_srcw);
  if (m->d_bside) hipFree(m->d_bside);
  if (m->d_bw) hipFree(m->d_bw);
  for (hipStream_t st : m->gstreams) hipStreamDestroy(st);
  for (hipEvent_t ev : m->gjoin) hipEventDestroy(ev);
  if (m->gfork) hipEventDestroy(m->gfork);
  delete m;
  return CRKDG_OK;
}

int crkdg_instance_query(const crkdg_mesh* m, int32_t inst, crkdg_instance_layout* out) {
  if (check_mesh(m)) return CRKDG_E_ARG;
  if (inst < 0 || inst >= m->layout.n_inst || !out) return fail(CRKDG_E_ARG, "bad instance index");
  *out = m->lay[inst];
  return CRKDG_OK;
}

int crkdg_points(const crkdg_mesh* m, int32_t inst, int32_t which, double* xyz, int32_t cap,
                 int32_t* count) {
  if (check_mesh(m)) return CRKDG_E_ARG;
  if (inst < 0 || inst >= m->layout.n_inst || !count) return fail(CRKDG_E_ARG, "bad arguments");
  const crkdg_problem& p = m->probs[inst];
  // reproduce the table order of tables.hpp
  static const double g2[] = {-0.57735026918962576451, 0.57735026918962576451};
  static const double g3[] = {-0.77459666924148337704, 0.0, 0.77459666924148337704};
  static const double g4[] = {-0.86113631159405257522, -0.33998104358485626480,
                              0.33998104358485626480, 0.86113631159405257522};
  static const double l2[] = {-1.0, 1.0};
  static const double l3[] = {-1.0, 0.0, 1.0};
  const int ng = p.k + 1;
  const double* g = (ng == 2) ? g2 : (ng == 3) ? g3 : g4;
  const int nl = (p.k == 1) ? 2 : 3;
  const double* l = (nl == 2) ? l2 : l3;
  std::vector<double> pts;
  if (which == 0) {
    int nq = 1;
    for (int d = 0; d < p.dim; ++d) nq *= ng;
    for (int q = 0; q < nq; ++q) {
      int r = q;
      for (int j = 0; j < 3; ++j) {
        if (j < p.dim) { pts.push_back(g[r % ng]); r /= ng; }
        else pts.push_back(0.0);
      }
    }
  } else if (which == 1) {
    int per = nl;
    for (int d = 0; d < p.dim - 1; ++d) per *= ng;
    for (int d = 0; d < p.dim; ++d) {
      for (int c = 0; c < per; ++c) {
        int r = c;
        double x[3] = {0.0, 0.0, 0.0};
        for (int j = 0; j < p.dim; ++j) {
          if (j == d) { x[j] = l[r % nl]; r /= nl; }
          else { x[j] = g[r % ng]; r /= ng; }
        }
        bool dup = false;
        for (size_t o = 0; o < pts.size(); o += 3)
          if (pts[o] == x[0] && pts[o + 1] == x[1] && pts[o + 2] == x[2]) dup = true;
        if (!dup) pts.insert(pts.end(), x, x + 3);
      }
    }
  } else {
    return fail(CRKDG_E_ARG, "which must be 0 or 1");
  }
  const int n = static_cast<int>(pts.size() / 3);
  *count = n;
  if (xyz) {
    if (cap < n) return fail(CRKDG_E_ARG, "capacity too small");
    std::memcpy(xyz, pts.data(), sizeof(double) * pts.size());
  }
  return CRKDG_OK;
}

int crkdg_project(crkdg_mesh* m, const double* d_samples, crkdg_state out, void* stream) {
  if (check_mesh(m)) return CRKDG_E_ARG;
  if (!d_samples) return fail(CRKDG_E_ARG, "samples is NULL");
  if (int rc = check_state(out, "out")) return rc;
  if (int rc = set_device(m)) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (const Group& g : m->groups) {
    KArgs a = base_args(m, g, nullptr);
    a.slots.avg[0] = out.avg;
    a.slots.hi[0] = out.hi;
    a.samples = d_samples;
    g.ops->project(a, g.nblocks, BLOCK, s);
  }
  HIP_TRY(hipGetLastError());
  return CRKDG_OK;
}

int crkdg_set_source(crkdg_mesh* m, int32_t n_terms, const crkdg_state* terms, const double* coef) {
  if (check_mesh(m)) return CRKDG_E_ARG;
  if (n_terms < 0 || n_terms > CRKDG_MAX_SOURCE_TERMS)
    return fail(CRKDG_E_ARG, "n_terms must lie in 0.." + std::to_string(CRKDG_MAX_SOURCE_TERMS));
  if (n_terms > 0 && (!terms || !coef)) return fail(CRKDG_E_ARG, "NULL terms or coef");
  if (m->live_graphs > 0)
    return fail(CRKDG_E_ARG, "step graphs of this mesh are alive: they hold the previous source");
  Src src{};
  for (int p = 0; p < n_terms; ++p) {
    if (int rc = check_state(terms[p], "terms[p]")) return rc;
    for (int j = 0; j < 3; ++j)
      if (!std::isfinite(coef[3 * p + j])) return fail(CRKDG_E_ARG, "non-finite source coefficient");
    src.avg[p] = terms[p].avg;
    src.hi[p] = terms[p].hi;
    src.rate[p] = coef[3 * p];
    src.omega[p] = coef[3 * p + 1];
    src.phase[p] = coef[3 * p + 2];
  }
  src.n = n_terms;
  if (n_terms > 0 && !m->d_srcw) {
    if (int rc = set_device(m)) return rc;
    const size_t bytes = sizeof(double) * static_cast<size_t>(m->layout.n_inst) * SRC_STAGES * MAX_SRC;
    HIP_TRY(hipMalloc(&m->d_srcw, bytes));
    HIP_TRY(hipMemset(m->d_srcw, 0, bytes));
  }
  src.w = m->d_srcw;
  m->src = src;
  return CRKDG_OK;
}

int crkdg_set_boundary_data(crkdg_mesh* m, int32_t inst, int32_t side, int32_t n_terms, const double* coef,
                            const double* d_values) {
  if (check_mesh(m)) return CRKDG_E_ARG;
  if (inst < 0 || inst >= m->layout.n_inst) return fail(CRKDG_E_ARG, "instance out of range");
  const crkdg_problem& p = m->probs[inst];
  if (side < 0 || side >= 2 * p.dim) return fail(CRKDG_E_ARG, "side out of range");
  if (side_bc(p, side / 2, side % 2) != CRKDG_BC_DIRICHLET) return fail(CRKDG_E_ARG, "the side is not Dirichlet");
  if (n_terms < 0 || n_terms > CRKDG_MAX_SOURCE_TERMS)
    return fail(CRKDG_E_ARG, "n_terms must lie in 0.." + std::to_string(CRKDG_MAX_SOURCE_TERMS));
  if (n_terms > 0 && (!coef || !d_values)) return fail(CRKDG_E_ARG, "NULL coef or values");
  if (m->live_graphs > 0)
    return fail(CRKDG_E_ARG, "step graphs of this mesh are alive: they hold the previous boundary data");
  for (int j = 0; j < 3 * n_terms; ++j)
    if (!std::isfinite(coef[j])) return fail(CRKDG_E_ARG, "non-finite coefficient");
  if (int rc = set_device(m)) return rc;
  const int n = m->layout.n_inst;
  if (m->bsides.empty()) m->bsides.assign(static_cast<size_t>(n) * 6, BSide{});
  if (!m->d_bside) {
    HIP_TRY(hipMalloc(&m->d_bside, sizeof(BSide) * n * 6));
    const size_t wb = sizeof(double) * static_cast<size_t>(n) * 6 * BW_STAGES * MAX_SRC;
    HIP_TRY(hipMalloc(&m->d_bw, wb));
    HIP_TRY(hipMemset(m->d_bw, 0, wb));
  }
  BSide bs{};
  int64_t nf = 1;
  for (int d = 0; d < p.dim; ++d)
    if (d != side / 2) nf *= p.n[d];
  bs.val = n_terms > 0 ? d_values : nullptr;
  bs.n_terms = n_terms;
  bs.n_faces = static_cast<int32_t>(nf);
  for (int q = 0; q < n_terms; ++q)
    for (int j = 0; j < 3; ++j) bs.coef[q][j] = coef[3 * q + j];
  m->bsides[static_cast<size_t>(inst) * 6 + side] = bs;
  InstDev& I = m->inst[inst];
  if (n_terms > 0) I.bdyn |= 1u << side;
  else I.bdyn &= ~(1u << side);
  HIP_TRY(hipMemcpy(m->d_bside, m->bsides.data(), sizeof(BSide) * n * 6, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(m->d_inst + inst, &I, sizeof(InstDev), hipMemcpyHostToDevice));
  m->has_bdata = false;
  for (const InstDev& J : m->inst) m->has_bdata = m->has_bdata || J.bdyn != 0;
  return CRKDG_OK;
}

int crkdg_limit(crkdg_mesh* m, crkdg_state u, crkdg_ctl* d_ctl, void* stream) {
  if (check_mesh(m)) return CRKDG_E_ARG;
  if (int rc = check_state(u, "u")) return rc;
  if (int rc = set_device(m)) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (const Group& g : m->groups) {
    KArgs a = base_args(m, g, d_ctl);
    a.slots.avg[0] = u.avg;
    a.slots.hi[0] = u.hi;
    g.ops->limit(a, g.nblocks, BLOCK, s);
  }
  HIP_TRY(hipGetLastError());
  return CRKDG_OK;
}

// averages and totals with the per-block partial sums in `partial`
static int cell_avg_into(crkdg_mesh* m, crkdg_state u, double* d_avg, double* d_totals, double* partial,
                         hipStream_t s) {
  if (d_avg)
    HIP_TRY(hipMemcpyAsync(d_avg, u.avg, sizeof(double) * m->layout.avg_elems, hipMemcpyDeviceToDevice, s));
  if (d_totals) {
    // instances of different variable counts are reduced per group
    for (const Group& g : m->groups) {
      const int V = g.ops->V;
      hipLaunchKernelGGL(k_totals_partial, dim3(g.nblocks), dim3(BLOCK), 0, s, m->d_inst, g.d_bmap,
                         u.avg, partial, V);
    }
    HIP_TRY(hipGetLastError());
    // totals are packed per instance with that instance's V
    int64_t off = 0;
    for (int i = 0; i < m->layout.n_inst; ++i) {
      hipLaunchKernelGGL(k_totals_final, dim3(1), dim3(BLOCK), 0, s, m->d_inst + i, partial,
                         d_totals + off, m->lay[i].n_vars);
      off += m->lay[i].n_vars;
    }
    HIP_TRY(hipGetLastError());
  }
  return CRKDG_OK;
}

int crkdg_cell_avg(crkdg_mesh* m, crkdg_state u, double* d_avg, double* d_totals, void* stream) {
  if (check_mesh(m)) return CRKDG_E_ARG;
  if (!u.avg) return fail(CRKDG_E_ARG, "u.avg is NULL");
  if (int rc = set_device(m)) return rc;
  return cell_avg_into(m, u, d_avg, d_totals, m->d_partial, static_cast<hipStream_t>(stream));
}

int crkdg_cell_avg_noalloc(crkdg_mesh* m, crkdg_state u, double* d_avg, double* d_totals, void* stream) {
  if (check_mesh(m)) return CRKDG_E_ARG;
  if (!u.avg) return fail(CRKDG_E_ARG, "u.avg is NULL");
  if (static_cast<int64_t>(m->total_lblocks) * 5 > kScratchDoubles)
    return fail(CRKDG_E_ARG, "crkdg_cell_avg_noalloc: the mesh has " + std::to_string(m->total_lblocks) +
                                 " blocks of 256 cells; the static scratch holds partial sums of at most " +
                                 std::to_string(kScratchDoubles / 5) + " (use crkdg_cell_avg)");
  if (int rc = set_device(m)) return rc;
  double* sp = nullptr;
  if (int rc = scratch_address(m->device, &sp)) return rc;   // stored at mesh creation: no runtime call
  return cell_avg_into(m, u, d_avg, d_totals, sp, static_cast<hipStream_t>(stream));
}

static int launch_cfl(crkdg_mesh* m, const crkdg_state* slots, int nslots, int rotate, crkdg_ctl* d_ctl,
                      hipStream_t s) {
  const int n = m->layout.n_inst;
  hipLaunchKernelGGL(k_clear_a0, dim3((n + 63) / 64), dim3(64), 0, s, d_ctl, n);
  for (const Group& g : m->groups) {
    KArgs a = base_args(m, g, d_ctl);
    for (int j = 0; j < nslots && j < MAX_SLOTS; ++j) {
      a.slots.avg[j] = slots[j].avg;
      a.slots.hi[j] = slots[j].hi;
    }
    a.slots.n = nslots;
    a.slots.rotate = rotate;
    g.ops->cfl(a, g.nblocks, BLOCK, s);
  }
  hipLaunchKernelGGL(k_a0_finish, dim3((n + 63) / 64), dim3(64), 0, s, d_ctl, m->d_inst, n);
  HIP_TRY(hipGetLastError());
  return CRKDG_OK;
}

int crkdg_cfl(crkdg_mesh* m, crkdg_state u, crkdg_ctl* d_ctl, void* stream) {
  if (check_mesh(m)) return CRKDG_E_ARG;
  if (int rc = check_state(u, "u")) return rc;
  if (!d_ctl) return fail(CRKDG_E_ARG, "d_ctl is NULL");
  if (int rc = set_device(m)) return rc;
  return launch_cfl(m, &u, 1, 0, d_ctl, static_cast<hipStream_t>(stream));
}

int crkdg_start(crkdg_mesh* m, const crkdg_state* slots, int32_t cur, crkdg_ctl* d_ctl, const double* t0,
                const double* t_end, const double* dt_fixed, void* stream) {
  if (check_mesh(m)) return CRKDG_E_ARG;
  if (!slots || !d_ctl || !t0) return fail(CRKDG_E_ARG, "NULL argument");
  const int ns = m->layout.n_slots;
  if (cur < 0 || cur >= ns) return fail(CRKDG_E_ARG, "cur out of range");
  for (int j = 0; j < ns; ++j)
    if (int rc = check_state(slots[j], "slot")) return rc;
  if (int rc = set_device(m)) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = m->layout.n_inst;
  std::vector<crkdg_ctl> h(n);
  for (int i = 0; i < n; ++i) {
    std::memset(&h[i], 0, sizeof(crkdg_ctl));
    h[i].t = t0[i];
    h[i].t_end = t_end ? t_end[i] : INFINITY;
    h[i].dt_fixed = dt_fixed ? dt_fixed[i] : 0.0;
    h[i].cur = cur;
    h[i].goal = INT64_MAX;
    if (!(h[i].t < h[i].t_end)) h[i].status = CRKDG_S_DONE;
  }
  HIP_TRY(hipMemcpyAsync(d_ctl, h.data(), sizeof(crkdg_ctl) * n, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int nq = static_cast<int>(m->groups.size()) * QSTAGES;
  hipLaunchKernelGGL(k_zero_u32, dim3((nq + 63) / 64), dim3(64), 0, s, m->d_qcount, nq);
  return launch_cfl(m, slots, ns, 1, d_ctl, s);
}

static int launch_stage(crkdg_mesh* m, int gi, int stage, const Slots& slots, crkdg_ctl* d_ctl,
                        hipStream_t s) {
  const Group& g = m->groups[gi];
  if (stage < 2 || stage >= QSTAGES || stage > g.stages + 1)
    return fail(CRKDG_E_ARG, "stage index out of range");
  const Butcher bt = butcher(g.stages);
  KArgs a = base_args(m, g, d_ctl);
  a.bmap = g.d_smap;
  a.n_items = g.n_items;
  a.tile_shift = ilog2(g.tune.tile_x);
  a.slots = slots;
  a.stage = stage;
  a.queue = m->d_queue + g.queue_off;
  a.qcap = g.qcap;
  a.qcount = m->d_qcount + gi * QSTAGES + stage;
  // every counter is cleared by the controller at the end of an attempt
  // (crkdg_stage clears its own after the stage)
  // the queue holds a few percent of the cells: up to 256 workgroups drain it
  const int qblocks = static_cast<int>(std::min<int64_t>(256, (g.ncells + BLOCK - 1) / BLOCK));
  const int grid = stage_grid(g);
  const bool persistent = grid < g.n_items;
  if (m->has_bdata && (stage > g.stages || g.scheme == CRKDG_SCHEME_RKDG)) {
    // the stage evaluates F: time factors of the boundary data
    StageCoef sc{};
    for (int j = 0; j < 4; ++j) sc.c[j] = a.c[j];
    const int n = m->layout.n_inst;
    hipLaunchKernelGGL(k_boundary_weights, dim3((6 * n + 63) / 64), dim3(64), 0, s, m->d_inst, d_ctl,
                       m->d_bside, m->d_bw, n, gi, g.stages, sc);
  }
  if (m->src.n > 0) {
    StageCoef sc{};
    sc.a = (stage <= g.stages) ? bt.a[stage] : 0.0;
    for (int j = 0; j < 4; ++j) {
      sc.b[j] = bt.b[j];
      sc.c[j] = a.c[j];
    }
    const int n = m->layout.n_inst;
    hipLaunchKernelGGL(k_source_weights, dim3((n + 63) / 64), dim3(64), 0, s, m->d_inst, d_ctl, n, gi,
                       g.stages, stage, sc, m->src);
  }
  if (g.ops->coop) {
    // meshes with time-dependent boundary data take the kernel forms that read it
    const bool bdy = a.bside != nullptr;
    if (stage <= g.stages) {
      a.a = bt.a[stage];
      (g.scheme != CRKDG_SCHEME_RKDG ? g.ops->coop_local
                                     : bdy ? g.ops->coop_inner_dg_bd : g.ops->coop_inner_dg)(a, g.n_items,
                                                                                             g.ops->coop, s);
      g.ops->queue_local(a, qblocks, BLOCK, s);
    } else {
      for (int j = 0; j < 4; ++j) a.b[j] = bt.b[j];
      (bdy ? g.ops->coop_final_bd : g.ops->coop_final)(a, g.n_items, g.ops->coop, s);
      g.ops->queue_final(a, qblocks, BLOCK, s);
    }
    return CRKDG_OK;
  }
  if (stage <= g.stages) {
    a.a = bt.a[stage];
    if (g.scheme == CRKDG_SCHEME_RKDG)
      (persistent ? g.ops->stage_inner_dg_p : g.ops->stage_inner_dg)(a, grid, g.tune.threads, s);
    else
      (persistent ? g.ops->stage_local_p : g.ops->stage_local)(a, grid, g.tune.threads, s);
    g.ops->queue_local(a, qblocks, BLOCK, s);
  } else {
    for (int j = 0; j < 4; ++j) a.b[j] = bt.b[j];
    (persistent ? g.ops->stage_final_p : g.ops->stage_final)(a, grid, g.tune.threads, s);
    g.ops->queue_final(a, qblocks, BLOCK, s);
  }
  return CRKDG_OK;
}

int crkdg_stage(crkdg_mesh* m, int32_t stage, const crkdg_state* states, int32_t n_states, crkdg_state out,
                crkdg_ctl* d_ctl, void* stream) {
  if (check_mesh(m)) return CRKDG_E_ARG;
  if (!states || !d_ctl) return fail(CRKDG_E_ARG, "NULL argument");
  if (int rc = check_state(out, "out")) return rc;
  if (int rc = set_device(m)) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  bool any = false;
  if (stage < 2 || stage >= QSTAGES) return fail(CRKDG_E_ARG, "stage index out of range");
  for (int gi = 0; gi < static_cast<int>(m->groups.size()); ++gi) {
    const Group& g = m->groups[gi];
    if (stage > g.stages + 1) continue;
    // stage 2..s reads u~^(stage-1); the final stage reads u~^(j), b_j != 0
    const int need = (stage <= g.stages) ? stage - 1 : g.stages;
    if (n_states < need) return fail(CRKDG_E_ARG, "too few states for this stage");
    Slots sl{};
    for (int j = 0; j < need; ++j) {
      if (int rc = check_state(states[j], "states[j]")) return rc;
      sl.avg[j] = states[j].avg;
      sl.hi[j] = states[j].hi;
      if (states[j].avg == out.avg || states[j].hi == out.hi)
        return fail(CRKDG_E_ARG, "out aliases an input state");
    }
    const int oslot = (stage <= g.stages) ? stage - 1 : g.stages;
    sl.avg[oslot] = out.avg;
    sl.hi[oslot] = out.hi;
    sl.n = g.stages + 1;
    sl.rotate = 0;
    if (int rc = launch_stage(m, gi, stage, sl, d_ctl, s)) return rc;
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, m->d_qcount + gi * QSTAGES + stage, 1);
    any = true;
  }
  if (!any) return fail(CRKDG_E_ARG, "stage index out of range for every instance");
  HIP_TRY(hipGetLastError());
  return CRKDG_OK;
}

// One attempt of every running instance: the stage chain of each kernel
// group, then the controller.  The groups touch disjoint instances, queue
// regions and counters, so with several groups each chain runs on its own
// stream (forked from s and joined back through events; under stream
// capture this records parallel branches of the step graph): a group's
// small or tail-heavy launches overlap the others'.
static int enqueue_attempt(crkdg_mesh* m, const Slots& sl, crkdg_ctl* d_ctl, hipStream_t s) {
  const int ng = static_cast<int>(m->groups.size());
  const bool fork = ng > 1 && static_cast<int>(m->gstreams.size()) == ng;
  if (fork) HIP_TRY(hipEventRecord(m->gfork, s));
  for (int gi = 0; gi < ng; ++gi) {
    hipStream_t gs = fork ? m->gstreams[gi] : s;
    if (fork) HIP_TRY(hipStreamWaitEvent(gs, m->gfork, 0));
    for (int stage = 2; stage <= m->groups[gi].stages + 1; ++stage)
      if (int rc = launch_stage(m, gi, stage, sl, d_ctl, gs)) return rc;
    if (fork) {
      HIP_TRY(hipEventRecord(m->gjoin[gi], gs));
      HIP_TRY(hipStreamWaitEvent(s, m->gjoin[gi], 0));
    }
  }
  const int n = m->layout.n_inst;
  const int nq = static_cast<int>(m->groups.size()) * QSTAGES;
  hipLaunchKernelGGL(k_controller, dim3((std::max(n, nq) + 63) / 64), dim3(64), 0, s, d_ctl, m->d_inst, n,
                     m->d_qcount, nq);
  HIP_TRY(hipGetLastError());
  return CRKDG_OK;
}

int crkdg_step(crkdg_mesh* m, const crkdg_state* slots, int32_t n_slots, crkdg_ctl* d_ctl,
               crkdg_step_info* info, void* stream) {
  if (check_mesh(m)) return CRKDG_E_ARG;
  if (!slots || !d_ctl) return fail(CRKDG_E_ARG, "NULL argument");
  if (n_slots < m->layout.n_slots || n_slots > MAX_SLOTS)
    return fail(CRKDG_E_LAYOUT, "n_slots must be layout.n_slots");
  Slots sl{};
  for (int j = 0; j < n_slots; ++j) {
    if (int rc = check_state(slots[j], "slot")) return rc;
    sl.avg[j] = slots[j].avg;
    sl.hi[j] = slots[j].hi;
  }
  sl.n = n_slots;
  sl.rotate = 1;
  if (int rc = set_device(m)) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = m->layout.n_inst;
  if (!info) return enqueue_attempt(m, sl, d_ctl, s);

  hipLaunchKernelGGL(k_arm, dim3((n + 63) / 64), dim3(64), 0, s, d_ctl, n, 0);
  std::vector<crkdg_ctl> h(n);
  int max_attempts = 2;
  for (const crkdg_problem& p : m->probs) max_attempts = std::max(max_attempts, p.max_halvings + 2);
  bool done = false;
  for (int att = 0; att < max_attempts && !done; ++att) {
    if (int rc = enqueue_attempt(m, sl, d_ctl, s)) return rc;
    HIP_TRY(hipMemcpyAsync(h.data(), d_ctl, sizeof(crkdg_ctl) * n, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    done = true;
    for (int i = 0; i < n; ++i)
      if (h[i].status == 0 && h[i].accepted < h[i].goal) done = false;
  }
  hipLaunchKernelGGL(k_arm, dim3((n + 63) / 64), dim3(64), 0, s, d_ctl, n, 1);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  int ret = CRKDG_OK;
  for (int i = 0; i < n; ++i) {
    crkdg_step_info& o = info[i];
    std::memset(&o, 0, sizeof(o));
    o.t = h[i].t;
    o.dt = h[i].dt_last;
    o.halvings = h[i].halvings_last;
    o.status = h[i].status == CRKDG_S_DONE ? 0 : h[i].status;
    o.cur = h[i].cur;
    o.accepted = h[i].accepted;
    o.rejected = h[i].rejected;
    if (h[i].status == CRKDG_S_DT_UNDERFLOW || h[i].status == CRKDG_S_NONFINITE) ret = h[i].status;
  }
  return ret;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// launch shapes of the stage kernels, the autotuner, and step graphs
// ---------------------------------------------------------------------------
namespace {

void tune_out(const Group& g, crkdg_tuning* o) {
  std::memset(o, 0, sizeof(*o));
  o->threads = g.tune.threads;
  o->tile_x = g.tune.tile_x;
  o->grid = g.tune.grid;
  o->dim = g.dim;
  o->k = g.ops->k;
  o->space = g.ops->space;
  o->stages = g.stages;
  o->scheme = g.scheme;
  o->n_inst = static_cast<int32_t>(g.insts.size());
  o->n_items = g.n_items;
  o->n_cells = g.ncells;
  o->ms = g.tune.ms;
}

// the stage kernels of one group for one attempt, without the controller;
// the group's deferred-limiter counters are cleared afterwards
int group_pass(crkdg_mesh* m, int gi, const Slots& sl, crkdg_ctl* d_ctl, hipStream_t s) {
  const Group& g = m->groups[gi];
  for (int stage = 2; stage <= g.stages + 1; ++stage)
    if (int rc = launch_stage(m, gi, stage, sl, d_ctl, s)) return rc;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, s, m->d_qcount + gi * QSTAGES, QSTAGES);
  HIP_TRY(hipGetLastError());
  return CRKDG_OK;
}

std::vector<Tune> candidates(const Group& g) {
  std::vector<Tune> out;
  if (g.ops->coop) {
    // the cooperative kernels have one launch shape per variant
    Tune t;
    t.threads = g.ops->coop;
    t.tile_x = g.ops->coop_tile[0];
    out.push_back(t);
    return out;
  }
  const int grids[] = {0, 1024, 2048};
  for (int th : {256, 128, 64}) {
    std::vector<int> widths;
    if (g.dim == 1) widths.push_back(th);
    else
      for (int w = 8; w <= std::min(th, 64); w *= 2) widths.push_back(w);
    for (int w : widths)
      for (int gr : grids) {
        Tune t;
        t.threads = th;
        t.tile_x = w;
        t.grid = gr;
        out.push_back(t);
      }
  }
  return out;
}

int slots_from(const crkdg_mesh* m, const crkdg_state* slots, int32_t n_slots, Slots& sl) {
  if (!slots) return fail(CRKDG_E_ARG, "slots is NULL");
  if (n_slots < m->layout.n_slots || n_slots > MAX_SLOTS)
    return fail(CRKDG_E_LAYOUT, "n_slots must be layout.n_slots");
  sl = Slots{};
  for (int j = 0; j < n_slots; ++j) {
    if (int rc = check_state(slots[j], "slot")) return rc;
    sl.avg[j] = slots[j].avg;
    sl.hi[j] = slots[j].hi;
  }
  sl.n = n_slots;
  sl.rotate = 1;
  return CRKDG_OK;
}

}  // namespace

struct crkdg_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  crkdg_mesh* mesh = nullptr;
  int device = 0;
};

extern "C" {

int crkdg_group_count(const crkdg_mesh* m, int32_t* n_groups) {
  if (check_mesh(m)) return CRKDG_E_ARG;
  if (!n_groups) return fail(CRKDG_E_ARG, "n_groups is NULL");
  *n_groups = static_cast<int32_t>(m->groups.size());
  return CRKDG_OK;
}

int crkdg_get_tuning(const crkdg_mesh* m, int32_t group, crkdg_tuning* out) {
  if (check_mesh(m)) return CRKDG_E_ARG;
  if (group < 0 || group >= static_cast<int>(m->groups.size()) || !out)
    return fail(CRKDG_E_ARG, "bad group index");
  tune_out(m->groups[group], out);
  return CRKDG_OK;
}

int crkdg_set_tuning(crkdg_mesh* m, int32_t group, const crkdg_tuning* t) {
  if (check_mesh(m)) return CRKDG_E_ARG;
  if (group < 0 || group >= static_cast<int>(m->groups.size()) || !t)
    return fail(CRKDG_E_ARG, "bad group index");
  if (int rc = set_device(m)) return rc;
  Tune u;
  u.threads = t->threads;
  u.tile_x = t->tile_x;
  u.grid = t->grid;
  return apply_tune(m, group, u);
}

int crkdg_autotune(crkdg_mesh* m, const crkdg_state* slots, int32_t n_slots, crkdg_ctl* d_ctl,
                   int32_t reps, void* stream) {
  if (check_mesh(m)) return CRKDG_E_ARG;
  if (!d_ctl) return fail(CRKDG_E_ARG, "d_ctl is NULL");
  if (reps < 1 || reps > 1000) return fail(CRKDG_E_ARG, "reps must be 1..1000");
  Slots sl;
  if (int rc = slots_from(m, slots, n_slots, sl)) return rc;
  if (int rc = set_device(m)) return rc;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int n = m->layout.n_inst;
  std::vector<crkdg_ctl> saved(n);
  HIP_TRY(hipMemcpyAsync(saved.data(), d_ctl, sizeof(crkdg_ctl) * n, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  int rc = CRKDG_OK;
  for (int gi = 0; gi < static_cast<int>(m->groups.size()) && rc == CRKDG_OK; ++gi) {
    Tune best = m->groups[gi].tune;
    double best_ms = INFINITY;
    for (const Tune& t : candidates(m->groups[gi])) {
      if ((rc = apply_tune(m, gi, t))) break;
      if ((rc = group_pass(m, gi, sl, d_ctl, s))) break;   // warm-up
      if (hipEventRecord(e0, s) != hipSuccess) { rc = fail(CRKDG_E_HIP, "hipEventRecord"); break; }
      for (int r = 0; r < reps && rc == CRKDG_OK; ++r) rc = group_pass(m, gi, sl, d_ctl, s);
      if (rc) break;
      float ms = 0.0f;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        rc = fail(CRKDG_E_HIP, "event timing failed");
        break;
      }
      if (ms / reps < best_ms) {
        best_ms = ms / reps;
        best = t;
      }
    }
    if (rc == CRKDG_OK) {
      best.ms = best_ms;
      rc = apply_tune(m, gi, best);
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  // the tuning passes wrote only stage slots, never slot cur; the
  // controllers and the queue counters go back to their state before
  HIP_TRY(hipMemcpyAsync(d_ctl, saved.data(), sizeof(crkdg_ctl) * n, hipMemcpyHostToDevice, s));
  const int nq = static_cast<int>(m->groups.size()) * QSTAGES;
  hipLaunchKernelGGL(k_zero_u32, dim3((nq + 63) / 64), dim3(64), 0, s, m->d_qcount, nq);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s));
  return rc;
}

int crkdg_graph_create(crkdg_mesh* m, const crkdg_state* slots, int32_t n_slots, crkdg_ctl* d_ctl,
                       int32_t attempts, crkdg_graph** out) {
  if (check_mesh(m)) return CRKDG_E_ARG;
  if (!d_ctl || !out) return fail(CRKDG_E_ARG, "NULL argument");
  if (attempts < 1 || attempts > 4096) return fail(CRKDG_E_ARG, "attempts must be 1..4096");
  *out = nullptr;
  Slots sl;
  if (int rc = slots_from(m, slots, n_slots, sl)) return rc;
  if (int rc = set_device(m)) return rc;
  hipStream_t cs;
  HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  auto* g = new crkdg_graph();
  g->device = m->device;
  int rc = CRKDG_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    rc = fail(CRKDG_E_HIP, "hipStreamBeginCapture failed");
  } else {
    for (int a = 0; a < attempts && rc == CRKDG_OK; ++a) rc = enqueue_attempt(m, sl, d_ctl, cs);
    const hipError_t e = hipStreamEndCapture(cs, &g->graph);
    if (rc == CRKDG_OK && e != hipSuccess) rc = fail(CRKDG_E_HIP, "hipStreamEndCapture failed");
  }
  if (rc == CRKDG_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
    rc = fail(CRKDG_E_HIP, "hipGraphInstantiate failed");
  hipStreamDestroy(cs);
  if (rc != CRKDG_OK) {
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    delete g;
    return rc;
  }
  g->mesh = m;
  ++m->live_graphs;
  *out = g;
  return CRKDG_OK;
}

int crkdg_graph_launch(crkdg_graph* g, void* stream) {
  if (!g) return fail(CRKDG_E_ARG, "graph is NULL");
  HIP_TRY(hipSetDevice(g->device));
  HIP_TRY(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
  return CRKDG_OK;
}

int crkdg_graph_destroy(crkdg_graph* g) {
  if (!g) return CRKDG_OK;
  hipSetDevice(g->device);
  if (g->exec) hipGraphExecDestroy(g->exec);
  if (g->graph) hipGraphDestroy(g->graph);
  if (g->mesh) --g->mesh->live_graphs;
  delete g;
  return CRKDG_OK;
}

}  // extern "C"
