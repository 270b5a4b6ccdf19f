// Device code of the cRKDG hot path: physics, the element operators G and F,
// the scaling limiters, and the stage / limiter / CFL / projection kernels.
//
// One thread owns one cell.  A cell's modal coefficients are read with fully
// coalesced loads (cell index fastest in HBM), every contraction is unrolled
// against the compile-time tables of tables.hpp, and the result is written
// once.  Inner stages read no neighbour (the compactness of G, Sec. 2.1 and
// the compactness remark of Sec. 3.2); the final stage reads the face traces
// of the 2d face neighbours.
#pragma once

#include <hip/hip_runtime.h>

#include <cfloat>
#include <cmath>
#include <cstdint>
#include <utility>

#include "crkdg.h"
#include "tables.hpp"

namespace crkdg {

constexpr int SYS_ADV = CRKDG_SYS_ADVECTION;
constexpr int SYS_BURG = CRKDG_SYS_BURGERS;
constexpr int SYS_EULER = CRKDG_SYS_EULER;
constexpr int SYS_SWE = CRKDG_SYS_SHALLOW_WATER;
constexpr int BLOCK = 256;
constexpr int MAX_SLOTS = 5;

// Per-instance constants, resident in device memory.
struct InstDev {
  int64_t ncell;
  int64_t avg_off;   // element offset inside a state's avg array
  int64_t hi_off;    // element offset inside a state's hi array
  int64_t smp_off;   // element offset of the instance's point samples (crkdg_project)
  int32_t n[3];
  int32_t bc[6];     // CRKDG_BC_* per side 2 d + (upper side)
  int32_t stages;
  int32_t limiter;
  int32_t max_halvings;
  int32_t first_block;  // logical block range of this instance
  int32_t n_blocks;
  int32_t dim;
  int32_t alpha_mode;   // CRKDG_ALPHA_*: Lax-Friedrichs alpha per face, per point, global
  double rdx[3];     // 1 / dx_d
  double r2dx[3];    // 2 / dx_d
  double vel[3];
  double gamma, blo, bhi, eps, cfl, vol;
  double blo_chk, bhi_chk;  // scalar average check: B widened by a round-off margin
  double bcs[6][5];  // Dirichlet states per side
  double grav;       // g (shallow water)
  int32_t group;     // kernel group of the instance
  uint32_t bdyn;     // bit f: side f takes time-dependent Dirichlet data (BSide)
};

// One work item = one tile of cells of one instance: blockDim.x consecutive
// cells in 1D, a tile_x x (blockDim.x / tile_x) tile of one x-y plane in
// 2D/3D.  The default 32 x 8 tile of a 256-thread workgroup gives every
// wavefront 32 x 2 cells: full 128-byte row segments of the FP32 arrays, both
// face neighbours close, and fewer wavefronts crossed by a discontinuity than
// with 64-cell row segments.  The stage kernels take their tile shape,
// workgroup size and grid from the group's tuning (crkdg_autotune).
struct BlockItem {
  int32_t inst;
  int32_t lblock;    // logical block number (fixed order for reductions)
  int32_t x0, y0;    // tile origin (1D: first cell)
  int32_t z, pad;
};
constexpr int TILE_X = 32;
constexpr int TILE_SHIFT = 5;   // log2 TILE_X

// a thread's cell: natural index and coordinates
struct CellPos {
  int64_t c;
  int32_t x, y, z;
};

__device__ __forceinline__ int64_t tile_cell(const BlockItem& bi, int dim, const int32_t* n,
                                             int64_t ncell, int shift, bool& active, CellPos* pos = nullptr) {
  if (dim == 1) {
    const int64_t c = static_cast<int64_t>(bi.x0) + threadIdx.x;
    active = c < ncell;
    if (pos) *pos = CellPos{c, static_cast<int32_t>(c), 0, 0};
    return c;
  }
  const int x = bi.x0 + static_cast<int>(threadIdx.x & ((1u << shift) - 1u));
  const int y = bi.y0 + static_cast<int>(threadIdx.x >> shift);
  active = x < n[0] && y < n[1];
  const int64_t c = x + static_cast<int64_t>(n[0]) * (y + static_cast<int64_t>(n[1]) * bi.z);
  if (pos) *pos = CellPos{c, x, y, bi.z};
  return c;
}

struct Slots {
  double* avg[MAX_SLOTS];
  void* hi[MAX_SLOTS];
  int32_t n;
  int32_t rotate;    // 1: slot of u~^n is ctl->cur (step ring); 0: slot 0
};

// A source term s(x, t) = sum_p g_p(t) S_p(x) with g_p(t) = exp(-rate_p t)
// cos(omega_p t + phase_p): the S_p as modal states (their L2 projections,
// the mesh's layout and precision).  The manufactured solutions of the
// accuracy tests (Sec. 4.2) have sources of this form.
constexpr int MAX_SRC = CRKDG_MAX_SOURCE_TERMS;
constexpr int SRC_STAGES = 8;   // weight rows per instance, indexed by stage number
struct Src {
  const double* avg[MAX_SRC];
  const void* hi[MAX_SRC];
  double rate[MAX_SRC], omega[MAX_SRC], phase[MAX_SRC];
  double* w;         // [instance][SRC_STAGES][MAX_SRC] weights of the terms per stage
  int32_t n;         // 0: no source
  int32_t pad;
};

// Time-dependent Dirichlet data of one side of one instance: the exterior
// state at face point b of boundary face c (tangential cell index, the lower
// tangential direction fastest) is sum_p g_p(t) val[((p n_faces + c) NFP +
// b) V + v], g_p(t) = exp(-coef[p][0] t) cos(coef[p][1] t + coef[p][2]),
// taken at the time of the stage value the operator acts on.
struct BSide {
  const double* val;
  int32_t n_terms;
  int32_t n_faces;
  double coef[CRKDG_MAX_SOURCE_TERMS][3];
};
constexpr int BW_STAGES = 4;   // stage values per step with boundary weights

struct KArgs {
  const InstDev* inst;
  const BlockItem* bmap;
  crkdg_ctl* ctl;      // may be null for limit without flags
  Slots slots;
  int32_t stage;       // 2..s+1
  int32_t pad;
  double a;            // a_{stage, stage-1}
  double b[4];         // b_1..b_s (final stage)
  const double* samples;
  double* out;         // totals partials / other outputs
  void* queue;         // records of the cells whose limiter is deferred
  unsigned* qcount;    // number of queued cells of this stage
  unsigned qcap;       // record capacity of the queue (cells of the group)
  int32_t n_items;     // entries of bmap
  int32_t tile_shift;  // log2 of the tile width (2D/3D)
  double c[4];         // stage times c_1..c_s of the Butcher table (fractions of dt)
  Src src;
  const BSide* bside;  // [instance][6] time-dependent boundary data (sides with I.bdyn set)
  const double* bw;    // [instance][6][BW_STAGES][MAX_SRC] their time factors per stage value
};

// the time-dependent boundary data of one instance for stage value j
// (0-based), or none
struct BData {
  const BSide* side;   // [6], null when the mesh has no such data
  const double* w;     // [6][BW_STAGES][MAX_SRC] offset to stage value j
};
__device__ __forceinline__ BData bdata(const KArgs& a, int inst, int j) {
  if (!a.bside) return BData{nullptr, nullptr};
  return BData{a.bside + static_cast<int64_t>(inst) * 6,
               a.bw + static_cast<int64_t>(inst) * 6 * BW_STAGES * MAX_SRC + j * MAX_SRC};
}

// The time-dependent exterior state (FP64) of variable v at face point b of
// boundary face fc of side f (nfp points per face, nv variables).  Not
// inlined: only boundary cells of sides with such data call it, and inlined
// its index arithmetic and term loop took the 2D Q^2 Euler final stage from
// 244 to 272 registers (one wavefront per SIMD instead of two) although
// periodic meshes never run it.
__device__ __attribute__((noinline)) inline double boundary_value(const BData& bd, int f, int64_t fc, int nfp,
                                                                  int nv, int b, int v) {
  const BSide& bs = bd.side[f];
  const double* w = bd.w + f * (BW_STAGES * MAX_SRC);
  double x = 0.0;
  for (int q = 0; q < bs.n_terms; ++q)
    x = fma(w[q], bs.val[((static_cast<int64_t>(q) * bs.n_faces + fc) * nfp + b) * nv + v], x);
  return x;
}

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T cmad(double c, T x, T acc) {
  if (c == 0.0) return acc;
  if (c == 1.0) return acc + x;
  if (c == -1.0) return acc - x;
  return fma(T(c), x, acc);
}

__device__ __forceinline__ double* sel_avg(const Slots& s, int i) {
  double* p = s.avg[0];
#pragma unroll
  for (int k = 1; k < MAX_SLOTS; ++k)
    if (i == k) p = s.avg[k];
  return p;
}
__device__ __forceinline__ void* sel_hi(const Slots& s, int i) {
  void* p = s.hi[0];
#pragma unroll
  for (int k = 1; k < MAX_SLOTS; ++k)
    if (i == k) p = s.hi[k];
  return p;
}

// The weight of each source term in a stage (the source paired with the
// stage values as the operators are, Sec. 4.2): dt a_{i,i-1} g_p(t^n +
// c_{i-1} dt) in inner stage i, dt sum_j b_j g_p(t^n + c_j dt) in the final
// stage; written per instance by a one-thread-per-instance kernel before the
// stage (the stage kernels only read them: the transcendental calls stay out
// of their register budget).
__device__ __forceinline__ const double* source_weights(const KArgs& a, int inst) {
  return a.src.w + (static_cast<int64_t>(inst) * SRC_STAGES + a.stage) * MAX_SRC;
}

__device__ __forceinline__ bool instance_idle(const crkdg_ctl* c) {
  return c != nullptr && (c->status != 0 || c->accepted >= c->goal);
}

// raise `bits` in *flags once per wavefront if any lane has `bad`
__device__ __forceinline__ void raise_flag(uint32_t* flags, bool bad, uint32_t bits) {
  const unsigned long long m = __ballot(bad);
  if (m != 0ull && flags != nullptr) {
    const int lane = threadIdx.x & 63;
    if (lane == __ffsll(static_cast<long long>(m)) - 1) atomicOr(flags, bits);
  }
}

// 1/x: FP32 uses the hardware reciprocal (1 ulp); FP64 refines the hardware
// estimate with two Newton--Raphson steps r <- r (2 - x r).  Deterministic,
// so both cells of a face still compute bitwise the same flux.
__device__ __forceinline__ float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = r * fma(-x, r, 2.0);
  r = r * fma(-x, r, 2.0);
  return r;
}
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// fn(std::integral_constant<int, i>) for i = 0 .. N-1, expanded at compile
// time whatever the size of the body (a plain unrolled loop may stay a loop
// when its body is large)
template <class Fn, int... I>
__device__ __forceinline__ void static_for_impl(Fn&& fn, std::integer_sequence<int, I...>) {
  (fn(std::integral_constant<int, I>{}), ...);
}
template <int N, class Fn>
__device__ __forceinline__ void static_for(Fn&& fn) {
  static_for_impl(fn, std::make_integer_sequence<int, N>{});
}

// ---------------------------------------------------------------------------
// physics (Sec. 2.2.3 for Euler)
// ---------------------------------------------------------------------------
template <int D, int SYS> struct Phys {
  static constexpr int V = (SYS == SYS_EULER) ? D + 2 : (SYS == SYS_SWE) ? D + 1 : 1;

  // auxiliary quantities of one state shared by all directions
  template <typename T> struct Aux {
    T ir;      // 1 / rho
    T w[D];    // velocity
    T p;       // pressure
  };

  // The flux, the auxiliary quantities and the wave speed are evaluated by
  // both cells of a face on the same trace values; floating-point
  // contraction is switched off here (explicit fma only) so that both
  // evaluations are bitwise identical whatever code they are inlined into.
  template <typename T>
  __device__ __forceinline__ static Aux<T> aux(const T* u, const InstDev& I) {
#pragma clang fp contract(off)
    Aux<T> a{};
    if constexpr (SYS == SYS_EULER) {
      a.ir = recip(u[0]);
      T ke = T(0);
#pragma unroll
      for (int j = 0; j < D; ++j) {
        a.w[j] = u[1 + j] * a.ir;
        ke = fma(u[1 + j], a.w[j], ke);
      }
      a.p = T(I.gamma - 1.0) * (u[D + 1] - T(0.5) * ke);
    } else if constexpr (SYS == SYS_SWE) {
      // velocity and the hydrostatic term g h^2 / 2 (held in p)
      a.ir = recip(u[0]);
#pragma unroll
      for (int j = 0; j < D; ++j) a.w[j] = u[1 + j] * a.ir;
      a.p = T(0.5 * I.grav) * (u[0] * u[0]);
    }
    return a;
  }

  template <typename T>
  __device__ __forceinline__ static void flux(const T* u, const Aux<T>& a, int d, const InstDev& I,
                                              T* f) {
#pragma clang fp contract(off)
    if constexpr (SYS == SYS_ADV) {
      f[0] = T(I.vel[d]) * u[0];
    } else if constexpr (SYS == SYS_BURG) {
      f[0] = T(0.5) * u[0] * u[0];
    } else if constexpr (SYS == SYS_SWE) {
      f[0] = u[1 + d];
#pragma unroll
      for (int j = 0; j < D; ++j) f[1 + j] = u[1 + j] * a.w[d] + (j == d ? a.p : T(0));
    } else {
      f[0] = u[1 + d];
#pragma unroll
      for (int j = 0; j < D; ++j) f[1 + j] = u[1 + j] * a.w[d] + (j == d ? a.p : T(0));
      f[D + 1] = (u[D + 1] + a.p) * a.w[d];
    }
  }

  // largest |eigenvalue| of df_d/du; a state with p < 0 (not admissible:
  // FP32 cancellation near vacuum) has no real sound speed, and its speed is
  // the flow speed |w_d| (c^2 clamped at zero), which still bounds alpha
  template <typename T>
  __device__ __forceinline__ static T speed(const T* u, const Aux<T>& a, int d, const InstDev& I) {
#pragma clang fp contract(off)
    if constexpr (SYS == SYS_ADV) {
      return T(fabs(I.vel[d]));
    } else if constexpr (SYS == SYS_BURG) {
      return fabs(u[0]);
    } else if constexpr (SYS == SYS_SWE) {
      // |w_d| + sqrt(g h); a negative depth (not admissible) counts as dry
      return fabs(a.w[d]) + fsqrt(fmax(T(I.grav) * u[0], T(0)));
    } else {
      return fabs(a.w[d]) + fsqrt(fmax(T(I.gamma) * a.p * a.ir, T(0)));
    }
  }
};

// ---------------------------------------------------------------------------
// Basis tables in the arithmetic type, for the spaces whose point loops stay
// rolled (see Cell::BIG): a row is picked by a loop counter that is uniform
// across the wavefront, so it arrives through scalar loads.
// ---------------------------------------------------------------------------
template <int D, int K, int SP, typename T> struct RtTab {
  using S = Space<D, K, SP>;
  static constexpr int TM = S::TM;
  T phi_v[S::NQ][S::M];
  T cvol[S::NQ][S::M][D];
  T phi_s[S::NS_RAW][S::M];
  T cface[S::NF][S::NFP][S::M];
  T ftan[S::NFP][TM];    // tangential Legendre products at the face points
  constexpr RtTab() : phi_v{}, cvol{}, phi_s{}, cface{}, ftan{} {
    for (int f = 0; f < S::NF; ++f)
      for (int b = 0; b < S::NFP; ++b)
        for (int m = 0; m < S::M; ++m) cface[f][b][m] = static_cast<T>(S::tab.cface[f][b][m]);
    for (int q = 0; q < S::NQ; ++q)
      for (int m = 0; m < S::M; ++m) {
        phi_v[q][m] = static_cast<T>(S::tab.phi_v[q][m]);
        for (int d = 0; d < D; ++d) cvol[q][m][d] = static_cast<T>(S::tab.cvol[q][m][d]);
      }
    for (int p = 0; p < S::NS; ++p)
      for (int m = 0; m < S::M; ++m) phi_s[p][m] = static_cast<T>(S::tab.phi_s[p][m]);
    for (int b = 0; b < S::NFP; ++b)
      for (int t = 0; t < TM; ++t) {
        ftan[b][t] = static_cast<T>(S::tab.ftan[b][t]);
      }
  }
};
template <int D, int K, int SP, typename T> struct Rt {
  static constexpr RtTab<D, K, SP, T> tab{};
};

// ---------------------------------------------------------------------------
// the cell kernels of one variant
// ---------------------------------------------------------------------------
template <int D, int K, int SP, int SYS, typename T> struct Cell {
  using S = Space<D, K, SP>;
  using P = Phys<D, SYS>;
  static constexpr int V = P::V;
  static constexpr int M = S::M;
  static constexpr int MH = M - 1;
  static constexpr int NS = S::NS;
  static constexpr bool MIXED = sizeof(T) == 4;

  // Large spaces (3D Q^2 and P^3 Euler: 27 or 20 modes x 5 variables; 3D
  // Q^3: 64 modes) keep their point loops rolled.  The work of one point is
  // still unrolled over modes and variables, with table rows from Rt (scalar
  // loads); the face traces go through the tangential coefficients of the
  // face (face_modes).  This bounds code size, compile time and live
  // registers.
  static constexpr bool BIG = (M * V >= 100) || M >= 64;
  static constexpr int UQ = BIG ? 1 : S::NQ;    // unroll of volume-point loops
  static constexpr int US = BIG ? 1 : NS;       // unroll of S_K loops
  static constexpr int TM = S::TM;
  using RT = Rt<D, K, SP, T>;
  // Reflective and Dirichlet sides.  Not built into one-thread-per-cell 2D
  // Q^3 Euler FP64 stage kernels (64 FP64 values per state: 256 VGPRs, 256
  // AGPRs and scratch), whose final stage computed wrong values with the
  // boundary code in it although that code is never reached on periodic
  // meshes.  That family now runs the cooperative stage kernels (coop.hpp),
  // which have every boundary kind; these kernels are no longer built for it.
  static constexpr bool WALLS = BIG || MIXED || M * V <= 60;
  // The per-point and global Lax-Friedrichs alpha: not in the BIG face loop,
  // whose per-point pass runs at the register limit, nor in the 2D P^3 Euler
  // FP64 kernels, where the option code alone makes them spill.
  static constexpr bool ALPHA_MODES = !BIG && (MIXED || !(D == 2 && SP == CRKDG_SPACE_P && K == 3 && SYS == SYS_EULER));

  struct State {
    double ub[V];     // cell averages (FP64)
    T ch[V][MH];      // modes >= 1
  };

  __device__ __forceinline__ static void load(const double* avg, const T* hi, int64_t nc, int64_t c,
                                              State& s) {
#pragma unroll
    for (int v = 0; v < V; ++v) s.ub[v] = avg[v * nc + c];
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
      for (int m = 0; m < MH; ++m) s.ch[v][m] = hi[(static_cast<int64_t>(v) * MH + m) * nc + c];
  }

  __device__ __forceinline__ static void store(double* avg, T* hi, int64_t nc, int64_t c,
                                               const State& s) {
#pragma unroll
    for (int v = 0; v < V; ++v) avg[v * nc + c] = s.ub[v];
#pragma unroll
    for (int v = 0; v < V; ++v)
#pragma unroll
      for (int m = 0; m < MH; ++m) hi[(static_cast<int64_t>(v) * MH + m) * nc + c] = s.ch[v][m];
  }

  // u at a volume point / face point / S_K point (T arithmetic)
  __device__ __forceinline__ static void at_vol(const State& s, int q, T* u) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      T a = T(s.ub[v]);
#pragma unroll
      for (int m = 1; m < M; ++m) {
        if constexpr (BIG) a = fma(RT::tab.phi_v[q][m], s.ch[v][m - 1], a);
        else a = cmad(S::tab.phi_v[q][m], s.ch[v][m - 1], a);
      }
      u[v] = a;
    }
  }
  __device__ __forceinline__ static void at_face(const State& s, int f, int b, T* u) {
#pragma clang fp contract(off)
#pragma unroll
    for (int v = 0; v < V; ++v) {
      T a = T(s.ub[v]);
#pragma unroll
      for (int m = 1; m < M; ++m) a = cmad(S::tab.phi_f[f][b][m], s.ch[v][m - 1], a);
      u[v] = a;
    }
  }
  // Face traces of 2D spaces by sum factorisation: the restriction to the
  // face, R_t = sum_a (+-1)^a c(a, t) (P_a(+-1) = (+-1)^a; total-degree
  // spaces sum over the modes they have), then the 1D Legendre series at the
  // Gauss points of the tangential direction, whose nodes come in pairs +-y
  // (even and odd parts shared).  The same operations serve a cell's own
  // trace and its neighbour's; floating-point contraction is off here (as in
  // Phys), so that the two inlined copies -- the cell's own trace and the
  // neighbour's view of it -- round alike and the face flux is bitwise the
  // same in both cells (without it a lone product added to the even part
  // was fused in one copy only: 2D P^1 mixed lost conservation at 1e-10).
  static constexpr bool SF = (D == 2) && !BIG;
  static constexpr int mode_of(int a, int b) {
    for (int m = 0; m < M; ++m)
      if (S::modes.e[m][0] == a && S::modes.e[m][1] == b) return m;
    return -1;
  }
  struct Leg1D {
    double p[K + 1][K + 1];   // p[j][b] = P_b(y_j) at the Gauss nodes
    constexpr Leg1D() : p{} {
      for (int j = 0; j <= K; ++j)
        for (int b = 0; b <= K; ++b) p[j][b] = leg(b, S::gx(j));
    }
  };
  static constexpr Leg1D leg1d{};
  __device__ __forceinline__ static T coef(const State& s, int v, int m) {
    return m == 0 ? T(s.ub[v]) : s.ch[v][m - 1];
  }
  __device__ __forceinline__ static void face_traces(const State& s, int f, T (&u)[S::NFP][V]) {
#pragma clang fp contract(off)
    if constexpr (SF) {
      const int d = f / 2;
      const bool up = (f & 1) != 0;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        T R[K + 1];
#pragma unroll
        for (int t = 0; t <= K; ++t) {
          T acc = coef(s, v, d == 0 ? mode_of(0, t) : mode_of(t, 0));
#pragma unroll
          for (int a = 1; a <= K; ++a) {
            const int m = d == 0 ? mode_of(a, t) : mode_of(t, a);
            if (m < 0) continue;
            const T c = coef(s, v, m);
            acc = (up || (a % 2 == 0)) ? acc + c : acc - c;
          }
          R[t] = acc;
        }
#pragma unroll
        for (int j = 0; j < (K + 2) / 2; ++j) {
          const int jp = K - j;
          T E = R[0];
#pragma unroll
          for (int b = 2; b <= K; b += 2) E = fma(T(leg1d.p[jp][b]), R[b], E);
          if (jp == j) {
            u[jp][v] = E;
          } else {
            T O = T(leg1d.p[jp][1]) * R[1];
#pragma unroll
            for (int b = 3; b <= K; b += 2) O = fma(T(leg1d.p[jp][b]), R[b], O);
            u[jp][v] = E + O;
            u[j][v] = E - O;
          }
        }
      }
    } else {
#pragma unroll
      for (int b = 0; b < S::NFP; ++b) at_face(s, f, b, u[b]);
    }
  }

  // Point values of the S_K set of 2D spaces by sum factorisation: the set is
  // (Lobatto in x) x (Gauss in y) and (Gauss in x) x (Lobatto in y); each
  // family is evaluated row by row (the series in y at the row's node, then
  // in x), with the symmetric nodes +-y and +-x paired.  fn(u) is called for
  // every point (the centre twice when both rules contain 0, which the
  // order-free min/max checks do not notice).  Every value is reached through
  // at most 2K + 3 roundings of partial sums bounded by |ubar| + sum |c_m|.
  struct LegL {
    double p[S::NL][K + 1];   // p[l][b] = P_b(x_l) at the Gauss--Lobatto nodes
    constexpr LegL() : p{} {
      for (int l = 0; l < S::NL; ++l)
        for (int b = 0; b <= K; ++b) p[l][b] = leg(b, S::lx(l));
    }
  };
  static constexpr LegL legl{};
  template <typename Fn>
  __device__ __forceinline__ static void sk_points_sf(const State& s, Fn&& fn) {
    static_for<2>([&](auto FAM) {
      constexpr int fam = decltype(FAM)::value;
      constexpr int NR = (fam == 0) ? K + 1 : S::NL;   // rows (y nodes)
      constexpr int NX = (fam == 0) ? S::NL : K + 1;   // points of a row (x nodes)
#pragma unroll
      for (int r = 0; r < (NR + 1) / 2; ++r) {
        const int rp = NR - 1 - r;                      // y_rp >= 0, y_r = -y_rp
        T tp[V][K + 1], tm[V][K + 1];
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
          for (int a = 0; a <= K; ++a) {
            T E = coef(s, v, mode_of(a, 0)), O = T(0);
            bool odd = false;
#pragma unroll
            for (int b = 1; b <= K; ++b) {
              const int m = mode_of(a, b);
              if (m < 0) continue;
              const double pb = (fam == 0) ? leg1d.p[rp][b] : legl.p[rp][b];
              if (b % 2 == 0) {
                E = cmad(pb, coef(s, v, m), E);
              } else if (pb != 0.0) {
                O = odd ? cmad(pb, coef(s, v, m), O) : T(pb) * coef(s, v, m);
                odd = true;
              }
            }
            tp[v][a] = odd ? E + O : E;
            tm[v][a] = odd ? E - O : E;
          }
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          if (side == 1 && rp == r) continue;           // the row at y = 0 once
          const auto& t = side == 0 ? tp : tm;
#pragma unroll
          for (int c = 0; c < (NX + 1) / 2; ++c) {
            const int cp = NX - 1 - c;                  // x_cp >= 0
            T up[V], um[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
              T E = t[v][0], O = T(0);
              bool odd = false;
#pragma unroll
              for (int a = 1; a <= K; ++a) {
                const double pa = (fam == 0) ? legl.p[cp][a] : leg1d.p[cp][a];
                if (a % 2 == 0) {
                  E = cmad(pa, t[v][a], E);
                } else if (pa != 0.0) {
                  O = odd ? cmad(pa, t[v][a], O) : T(pa) * t[v][a];
                  odd = true;
                }
              }
              up[v] = odd ? E + O : E;
              um[v] = odd ? E - O : E;
            }
            fn(up);
            if (cp != c) fn(um);
          }
        }
      }
    });
  }

  // S_K values in FP64 (limiter decisions are taken in FP64)
  __device__ __forceinline__ static double sk_var(const State& s, int p, int v) {
    double a = 0.0;
#pragma unroll
    for (int m = 1; m < M; ++m) {
      if constexpr (BIG) a = fma(S::tab.phi_s[p][m], static_cast<double>(s.ch[v][m - 1]), a);
      else a = cmad(S::tab.phi_s[p][m], static_cast<double>(s.ch[v][m - 1]), a);
    }
    return s.ub[v] + a;
  }

  struct Acc {
    double a0[V];     // mode 0 (FP64)
    T ah[V][MH];      // modes >= 1
  };
  __device__ __forceinline__ static void zero(Acc& r) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      r.a0[v] = 0.0;
#pragma unroll
      for (int m = 0; m < MH; ++m) r.ah[v][m] = T(0);
    }
  }

  // r += scale * [ sum_q sum_d (2/dx_d) wq f_d(u_q) dphi_m/dxi_d ] * prod(2e+1)
  // (the volume part of the weak form, Sec. 2.1); the mode-0 row is zero.
  __device__ __forceinline__ static void volume(const State& s, const InstDev& I, double scale,
                                                Acc& r) {
    T sd[D];
#pragma unroll
    for (int d = 0; d < D; ++d) sd[d] = T(scale * I.r2dx[d]);
    // 2D spaces: the series along y at the rows of the Gauss grid
    // first (t[v][j][a] = sum_b c(a, b) P_b(y_j), nodes in +-y pairs), then
    // along x at each point
    T trow[SF ? V : 1][SF ? K + 1 : 1][SF ? K + 1 : 1];
    if constexpr (SF) {
#pragma unroll
      for (int v = 0; v < V; ++v)
#pragma unroll
        for (int a = 0; a <= K; ++a)
#pragma unroll
          for (int j = 0; j < (K + 2) / 2; ++j) {
            const int jp = K - j;
            T E = coef(s, v, mode_of(a, 0));
#pragma unroll
            for (int b = 2; b <= K; b += 2)
              if (mode_of(a, b) >= 0) E = fma(T(leg1d.p[jp][b]), coef(s, v, mode_of(a, b)), E);
            if (jp == j || mode_of(a, 1) < 0) {
              // middle node, or no odd y-mode in this column (total degree)
              trow[v][jp][a] = E;
              trow[v][j][a] = E;
            } else {
              T O = T(leg1d.p[jp][1]) * coef(s, v, mode_of(a, 1));
#pragma unroll
              for (int b = 3; b <= K; b += 2)
                if (mode_of(a, b) >= 0) O = fma(T(leg1d.p[jp][b]), coef(s, v, mode_of(a, b)), O);
              trow[v][jp][a] = E + O;
              trow[v][j][a] = E - O;
            }
          }
    }
#pragma unroll UQ
    for (int q = 0; q < S::NQ; ++q) {
      T u[V];
      if constexpr (SF) {
        const int i = q % (K + 1), j = q / (K + 1);
        const bool low = i < K - i;              // x_i < 0: odd part enters negated
        const int ip = low ? K - i : i;
#pragma unroll
        for (int v = 0; v < V; ++v) {
          T E = trow[v][j][0];
#pragma unroll
          for (int a = 2; a <= K; a += 2) E = fma(T(leg1d.p[ip][a]), trow[v][j][a], E);
          if (2 * i == K) {
            u[v] = E;
          } else {
            T O = T(leg1d.p[ip][1]) * trow[v][j][1];
#pragma unroll
            for (int a = 3; a <= K; a += 2) O = fma(T(leg1d.p[ip][a]), trow[v][j][a], O);
            u[v] = low ? E - O : E + O;
          }
        }
      } else {
        at_vol(s, q, u);
      }
      const auto a = P::aux(u, I);
#pragma unroll
      for (int d = 0; d < D; ++d) {
        T f[V];
        P::flux(u, a, d, I, f);
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const T g = sd[d] * f[v];
#pragma unroll
          for (int m = 1; m < M; ++m) {
            if constexpr (BIG) {
              // d phi_m / d xi_d vanishes identically when e_d(m) = 0
              if (S::modes.e[m][d] != 0) r.ah[v][m - 1] = fma(RT::tab.cvol[q][m][d], g, r.ah[v][m - 1]);
            } else {
              r.ah[v][m - 1] = cmad(S::tab.cvol[q][m][d], g, r.ah[v][m - 1]);
            }
          }
        }
      }
    }
  }

  // r -= scale / dx_d * sum_b cface[f][b][m] * fn_b  for one face, fn = flux
  // through the face along +e_d (the sign of the outward normal is in cface).
  // With H0, mode 0 takes the FP64 fluxes fn0[b] (scalar laws in the mixed
  // form, see SPLIT0) instead of the FP32 ones.
  template <bool H0 = false>
  __device__ __forceinline__ static void face_accum(int f, const T (&fn)[S::NFP][V], const InstDev& I,
                                                    double scale, Acc& r, const double* fn0 = nullptr) {
    const int d = f / 2;
    const double sc = scale * I.rdx[d];
    const T sct = T(sc);
    if constexpr (SF) {
      // sum factorised: h_t = sum_b wb_b P_t(y_b) g_b over the face points
      // (pairs +-y share their sum and difference), then every mode m with
      // normal degree a and tangential degree t takes pfac(m) side^(a+1) h_t
      const bool up = (f & 1) != 0;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        // mode 0 in FP64, in the same order in both cells of the face
#pragma unroll
        for (int b = 0; b < S::NFP; ++b)
          r.a0[v] = cmad(-S::tab.cface[f][b][0], sc * (H0 ? fn0[b] : static_cast<double>(fn[b][v])), r.a0[v]);
        T sum[(K + 2) / 2], dif[(K + 2) / 2];
#pragma unroll
        for (int j = 0; j < (K + 2) / 2; ++j) {
          const int jp = K - j;
          const T gp = sct * fn[jp][v];
          if (jp == j) {
            sum[j] = gp;
            dif[j] = T(0);
          } else {
            const T gm = sct * fn[j][v];
            sum[j] = gp + gm;
            dif[j] = gp - gm;
          }
        }
        T h[K + 1];
#pragma unroll
        for (int t = 0; t <= K; ++t) {
          T acc = T(0);
#pragma unroll
          for (int j = 0; j < (K + 2) / 2; ++j) {
            const int jp = K - j;
            const double w = S::tab.wb[jp] * leg1d.p[jp][t];
            if (jp == j && (t % 2) == 1) continue;   // P_t(0) = 0 for odd t
            acc = fma(T(w), (t % 2 == 0) ? sum[j] : dif[j], acc);
          }
          h[t] = acc;
        }
#pragma unroll
        for (int m = 1; m < M; ++m) {
          const int a = S::modes.e[m][d];
          const int t = S::modes.e[m][1 - d];
          const double kf = S::pfac(m) * ((up || ((a + 1) % 2 == 0)) ? 1.0 : -1.0);
          r.ah[v][m - 1] = cmad(-kf, h[t], r.ah[v][m - 1]);
        }
      }
    } else {
#pragma unroll
      for (int b = 0; b < S::NFP; ++b)
#pragma unroll
        for (int v = 0; v < V; ++v) {
          r.a0[v] = cmad(-S::tab.cface[f][b][0], sc * (H0 ? fn0[b] : static_cast<double>(fn[b][v])), r.a0[v]);
          const T g = sct * fn[b][v];
#pragma unroll
          for (int m = 1; m < M; ++m) r.ah[v][m - 1] = cmad(-S::tab.cface[f][b][m], g, r.ah[v][m - 1]);
        }
    }
  }

  // --- faces of the large spaces (BIG), tensor spaces only -----------------
  // tangential mode of mode m on a face normal to direction d
  static constexpr int tmode(int m, int d) {
    int t = 0, mul = 1;
    for (int j = 0; j < D; ++j)
      if (j != d) {
        t += mul * S::modes.e[m][j];
        mul *= K + 1;
      }
    return t;
  }

  // Coefficients of the trace of a cell on its face f in the tangential
  // Legendre products: R[v][t] = sum over e_d of P_{e_d}(+-1) c_v(e_d, t),
  // with P_e(+-1) = (+-1)^e.  get(v, m) returns coefficient m >= 1 and avg(v)
  // the average.  The operations depend only on the cell's coefficients and
  // on f, so a cell and its neighbour obtain bitwise the same trace of the
  // shared face.
  template <class GetAvg, class GetHi>
  __device__ __forceinline__ static void face_modes(GetAvg avg, GetHi get, int f, T (&R)[V][TM]) {
#pragma clang fp contract(off)
    static_assert(S::TENSOR, "face_modes needs a tensor-product space");
    const int d = f / 2;
    const bool up = (f & 1) != 0;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      R[v][0] = T(avg(v));
#pragma unroll
      for (int m = 1; m < M; ++m) {
        const int t = tmode(m, d);
        const int e = S::modes.e[m][d];
        const T x = get(v, m);
        // modes with e_d = 0 come first for every t (ascending mode order)
        if (e == 0) R[v][t] = x;
        else if (up || (e % 2) == 0) R[v][t] = R[v][t] + x;
        else R[v][t] = R[v][t] - x;
      }
    }
  }
  __device__ __forceinline__ static void face_modes_state(const State& s, int f, T (&R)[V][TM]) {
    face_modes([&](int v) { return s.ub[v]; }, [&](int v, int m) { return s.ch[v][m - 1]; }, f, R);
  }
  __device__ __forceinline__ static void face_modes_mem(const double* avg, const T* hi, int64_t nc,
                                                        int64_t c, int f, T (&R)[V][TM]) {
    face_modes([&](int v) { return avg[v * nc + c]; },
               [&](int v, int m) { return hi[(static_cast<int64_t>(v) * MH + m - 1) * nc + c]; }, f, R);
  }
  // trace value at face point b from the tangential coefficients
  __device__ __forceinline__ static void face_eval(const T (&R)[V][TM], int b, T* u) {
#pragma clang fp contract(off)
#pragma unroll
    for (int v = 0; v < V; ++v) {
      T a = R[v][0];
#pragma unroll
      for (int t = 1; t < TM; ++t) a = fma(RT::tab.ftan[b][t], R[v][t], a);
      u[v] = a;
    }
  }
  // r -= scale / dx_d * cface[f][b][m] fn(b) for one face point b of face f
  __device__ __forceinline__ static void face_point_scatter(int f, int b, const T* fn, const InstDev& I,
                                                            double scale, Acc& r) {
    const double sc = scale * I.rdx[f / 2];
    const double w = sc * S::tab.cface[f][b][0];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      r.a0[v] = fma(-w, static_cast<double>(fn[v]), r.a0[v]);
      const T g = T(-sc) * fn[v];
#pragma unroll
      for (int m = 1; m < M; ++m) r.ah[v][m - 1] = fma(RT::tab.cface[f][b][m], g, r.ah[v][m - 1]);
    }
  }
  __device__ __forceinline__ static void op_local_big(const State& s, const InstDev& I, double scale,
                                                      Acc& r) {
    volume(s, I, scale, r);
    static_for<S::NF>([&](auto F) {
      constexpr int f = decltype(F)::value;
      T R[V][TM];
      face_modes_state(s, f, R);
#pragma unroll 1
      for (int b = 0; b < S::NFP; ++b) {
        T u[V], fn[V];
        face_eval(R, b, u);
        const auto a = P::aux(u, I);
        P::flux(u, a, f / 2, I, fn);
        face_point_scatter(f, b, fn, I, scale, r);
      }
    });
  }

  __device__ __forceinline__ static void op_dg_big(const State& s, const double* avg, const T* hi,
                                                   const CellPos& p, const InstDev& I, double scale, Acc& r) {
    const int64_t c = p.c;
    volume(s, I, scale, r);
    static_for<S::NF>([&](auto F) {
      constexpr int f = decltype(F)::value;
      constexpr int d = f / 2;
      constexpr bool upper = (f & 1) != 0;   // this cell is the lower cell of the face
      const int64_t nb = neighbour(p, f, I);
      T Ri[V][TM], Re[V][TM];
      face_modes_state(s, f, Ri);
      if (nb >= 0) {
        face_modes_mem(avg, hi, I.ncell, nb, f ^ 1, Re);
      } else {
        // the exterior trace of ghost() in tangential modes (it is linear in
        // the interior trace, or constant)
        const int kind = I.bc[f];
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
          for (int t = 0; t < TM; ++t) {
            T x = Ri[v][t];
            if (kind == CRKDG_BC_REFLECT && v == 1 + d) x = -x;
            if (kind == CRKDG_BC_DIRICHLET) x = (t == 0) ? T(I.bcs[f][v]) : T(0);
            Re[v][t] = x;
          }
      }
      // alpha: largest wave speed over the face points and both traces
      T alpha = T(0);
#pragma unroll 1
      for (int b = 0; b < S::NFP; ++b) {
        T ui[V], ue[V];
        face_eval(Ri, b, ui);
        face_eval(Re, b, ue);
        const T* uL = upper ? ui : ue;
        const T* uR = upper ? ue : ui;
        const auto aL = P::aux(uL, I);
        const auto aR = P::aux(uR, I);
        alpha = fmax(alpha, fmax(P::speed(uL, aL, d, I), P::speed(uR, aR, d, I)));
      }
#pragma unroll 1
      for (int b = 0; b < S::NFP; ++b) {
        T ui[V], ue[V];
        face_eval(Ri, b, ui);
        face_eval(Re, b, ue);
        const T* uL = upper ? ui : ue;
        const T* uR = upper ? ue : ui;
        const auto aL = P::aux(uL, I);
        const auto aR = P::aux(uR, I);
        T fL[V], fR[V], fn[V];
        P::flux(uL, aL, d, I, fL);
        P::flux(uR, aR, d, I, fR);
        {
#pragma clang fp contract(off)
          const T ha = T(0.5) * alpha;
#pragma unroll
          for (int v = 0; v < V; ++v) fn[v] = fma(-ha, uR[v] - uL[v], T(0.5) * (fL[v] + fR[v]));
        }
        face_point_scatter(f, b, fn, I, scale, r);
      }
    });
  }

  // Mixed form of a scalar law: the fluxes that update the average (mode 0)
  // are formed in FP64 from the traces ubar + delta_b, the FP64 average plus
  // the FP32 trace of the higher modes, so that the average of a cell at a
  // bound the data attain (the cells behind an inflow carrying the end of B)
  // gets no FP32 rounding of ubar in its update; the higher modes keep the
  // FP32 fluxes.  Both cells of a face form delta_b with the same operations
  // (face_traces), so the FP64 face flux is still bitwise shared.
  static constexpr bool SPLIT0 = (V == 1) && (sizeof(T) == 4);
  __device__ __forceinline__ static void traces64(const State& s, int f, double (&u)[S::NFP]) {
    State s0 = s;
    s0.ub[0] = 0.0;
    T dv[S::NFP][V];
    face_traces(s0, f, dv);
#pragma unroll
    for (int b = 0; b < S::NFP; ++b) u[b] = s.ub[0] + static_cast<double>(dv[b][0]);
  }

  // G = -div^loc f: interior trace flux on every face (Sec. 2.1).
  __device__ __forceinline__ static void op_local(const State& s, const InstDev& I, double scale,
                                                  Acc& r) {
    if constexpr (BIG) {
      op_local_big(s, I, scale, r);
      return;
    }
    volume(s, I, scale, r);
#pragma unroll
    for (int f = 0; f < S::NF; ++f) {
      T fn[S::NFP][V];
      T tr[S::NFP][V];
      face_traces(s, f, tr);
#pragma unroll
      for (int b = 0; b < S::NFP; ++b) {
        const auto a = P::aux(tr[b], I);
        P::flux(tr[b], a, f / 2, I, fn[b]);
      }
      if constexpr (SPLIT0) {
        double u64[S::NFP], fn0[S::NFP];
        traces64(s, f, u64);
#pragma unroll
        for (int b = 0; b < S::NFP; ++b) P::flux(&u64[b], P::aux(&u64[b], I), f / 2, I, &fn0[b]);
        face_accum<true>(f, fn, I, scale, r, fn0);
      } else {
        face_accum(f, fn, I, scale, r);
      }
    }
  }

  // neighbour across face f of the cell at p (-1 on an outflow boundary);
  // from the coordinates, without integer division
  __device__ __forceinline__ static int64_t neighbour(const CellPos& p, int f, const InstDev& I) {
    const int d = f / 2;
    const int q = (d == 0) ? p.x : (d == 1) ? p.y : p.z;
    const int64_t stride = (d == 0) ? 1 : (d == 1) ? static_cast<int64_t>(I.n[0])
                                                   : static_cast<int64_t>(I.n[0]) * I.n[1];
    const int nd = I.n[d];
    const bool periodic = I.bc[f] == CRKDG_BC_PERIODIC;
    if ((f & 1) == 0) {
      if (q > 0) return p.c - stride;
      return periodic ? p.c + (nd - 1) * stride : -1;
    }
    if (q < nd - 1) return p.c + stride;
    return periodic ? p.c - (nd - 1) * stride : -1;
  }


  // Exterior trace on a non-periodic side f = 2 d + upper (no neighbour):
  // outflow, the interior trace; reflective wall, the mirror state (normal
  // momentum negated); Dirichlet / inflow, the prescribed state.
  __device__ __forceinline__ static void ghost(int f, const InstDev& I, const T* ui, T* ue) {
    const int kind = I.bc[f];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      T x = ui[v];
      if (kind == CRKDG_BC_REFLECT && v == 1 + f / 2) x = -x;
      if (kind == CRKDG_BC_DIRICHLET) x = T(I.bcs[f][v]);
      ue[v] = x;
    }
  }

  // F = -div^DG f with the Lax--Friedrichs flux (Sec. 2.1).  Each face flux is
  // formed in the canonical (lower cell, upper cell) orientation with the same
  // operation order in both cells, so the two cells of a face see bitwise the
  // same value and the averages are updated conservatively.
  // The global Lax-Friedrichs alpha: the wave-speed maximum a0 of u~^n over
  // S_K and all directions (Sec. 2.1), as the controller holds it in a step.
  __device__ __forceinline__ static double global_alpha(const crkdg_ctl* ctl) {
    double a = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) a = fmax(a, ctl->a0[d]);
    return a;
  }

  // `ag` is the global alpha (used when I.alpha_mode is CRKDG_ALPHA_GLOBAL).
  // `bd` locates the time-dependent boundary data of the instance for the
  // stage value the operator acts on (null: none).
  __device__ __forceinline__ static void op_dg(const State& s, const double* avg, const T* hi,
                                               const CellPos& p, const InstDev& I, double scale, Acc& r,
                                               double ag, const BData& bd) {
    if constexpr (BIG) {
      op_dg_big(s, avg, hi, p, I, scale, r);
    } else {
      op_dg_from(s, p, I, scale, r, ag, bd,
                 [&](int, int64_t nb, State& sn) { load(avg, hi, I.ncell, nb, sn); });
    }
  }

  // the time-dependent exterior state (FP64) of variable v at face point b
  // of side f of the cell at p
  __device__ __forceinline__ static double bvalue(int f, const CellPos& p, const InstDev& I, const BData& bd,
                                                  int b, int v) {
    const int d = f / 2;
    const int64_t fc = (d == 0) ? p.y + static_cast<int64_t>(I.n[1]) * p.z
                     : (d == 1) ? p.x + static_cast<int64_t>(I.n[0]) * p.z
                                : p.x + static_cast<int64_t>(I.n[0]) * p.y;
    return boundary_value(bd, f, fc, S::NFP, V, b, v);
  }
  // exterior traces of side f from its time-dependent data
  __device__ __forceinline__ static void boundary_data(int f, const CellPos& p, const InstDev& I,
                                                       const BData& bd, T (&ue)[S::NFP][V]) {
    for (int b = 0; b < S::NFP; ++b)
      for (int v = 0; v < V; ++v) ue[b][v] = T(bvalue(f, p, I, bd, b, v));
  }

  // F with the neighbour states read by getnb(f, nb, state)
  template <class GetNb>
  __device__ __forceinline__ static void op_dg_from(const State& s, const CellPos& p, const InstDev& I,
                                                    double scale, Acc& r, double ag, const BData& bd,
                                                    GetNb getnb) {
    volume(s, I, scale, r);
#pragma unroll
    for (int f = 0; f < S::NF; ++f) {
      const int d = f / 2;
      const bool upper = (f & 1) != 0;   // this cell is the lower cell of the face
      const int64_t nb = neighbour(p, f, I);
      T ui[S::NFP][V], ue[S::NFP][V];
      face_traces(s, f, ui);
      State sn;
      if (nb >= 0) {
        getnb(f, nb, sn);
        face_traces(sn, f ^ 1, ue);
      } else if constexpr (WALLS) {
        if (bd.side && (I.bdyn & (1u << f))) {
          boundary_data(f, p, I, bd, ue);
        } else {
#pragma unroll
          for (int b = 0; b < S::NFP; ++b) ghost(f, I, ui[b], ue[b]);
        }
      } else {
#pragma unroll
        for (int b = 0; b < S::NFP; ++b)
#pragma unroll
          for (int v = 0; v < V; ++v) ue[b][v] = ui[b][v];
      }
      // canonical orientation: L = lower cell, R = upper cell
      T fL[S::NFP][V], fR[S::NFP][V];
      T alpha = T(0);
#pragma unroll
      for (int b = 0; b < S::NFP; ++b) {
        const T* uL = upper ? ui[b] : ue[b];
        const T* uR = upper ? ue[b] : ui[b];
        const auto aL = P::aux(uL, I);
        const auto aR = P::aux(uR, I);
        P::flux(uL, aL, d, I, fL[b]);
        P::flux(uR, aR, d, I, fR[b]);
        alpha = fmax(alpha, fmax(P::speed(uL, aL, d, I), P::speed(uR, aR, d, I)));
      }
      if constexpr (ALPHA_MODES)
        if (I.alpha_mode == CRKDG_ALPHA_GLOBAL) alpha = static_cast<T>(ag);
      T fn[S::NFP][V];
      {
        // same operations, in the same order, in both cells of the face
#pragma clang fp contract(off)
#pragma unroll
        for (int b = 0; b < S::NFP; ++b) {
          const T* uL = upper ? ui[b] : ue[b];
          const T* uR = upper ? ue[b] : ui[b];
          T ab = alpha;
          if (ALPHA_MODES && I.alpha_mode == CRKDG_ALPHA_POINT) {
            // the point's own speed, recomputed so that the per-face form
            // keeps no per-point values alive (bitwise the value the face
            // maximum saw, so the fmin is exact); a NaN speed (a zero or
            // non-finite density) falls back to the face alpha
            ab = fmin(fmax(P::speed(uL, P::aux(uL, I), d, I), P::speed(uR, P::aux(uR, I), d, I)), alpha);
          }
          const T ha = T(0.5) * ab;
#pragma unroll
          for (int v = 0; v < V; ++v)
            fn[b][v] = fma(-ha, uR[v] - uL[v], T(0.5) * (fL[b][v] + fR[b][v]));
        }
      }
      if constexpr (SPLIT0) {
        // the same Lax--Friedrichs flux in FP64 for the average update
        double di[S::NFP], de[S::NFP], fn0[S::NFP];
        traces64(s, f, di);
        if (nb >= 0) {
          traces64(sn, f ^ 1, de);
        } else {
#pragma unroll
          for (int b = 0; b < S::NFP; ++b)
            de[b] = !(WALLS && I.bc[f] == CRKDG_BC_DIRICHLET) ? di[b]
                    : (bd.side && (I.bdyn & (1u << f))) ? bvalue(f, p, I, bd, b, 0) : I.bcs[f][0];
        }
        double a64 = 0.0;
#pragma unroll
        for (int b = 0; b < S::NFP; ++b) {
          const double* uL = upper ? &di[b] : &de[b];
          const double* uR = upper ? &de[b] : &di[b];
          a64 = fmax(a64, fmax(P::speed(uL, P::aux(uL, I), d, I), P::speed(uR, P::aux(uR, I), d, I)));
        }
        if constexpr (ALPHA_MODES)
          if (I.alpha_mode == CRKDG_ALPHA_GLOBAL) a64 = ag;
        {
#pragma clang fp contract(off)
#pragma unroll
          for (int b = 0; b < S::NFP; ++b) {
            const double* uL = upper ? &di[b] : &de[b];
            const double* uR = upper ? &de[b] : &di[b];
            double ab = a64;
            if (ALPHA_MODES && I.alpha_mode == CRKDG_ALPHA_POINT)
              ab = fmin(fmax(P::speed(uL, P::aux(uL, I), d, I), P::speed(uR, P::aux(uR, I), d, I)), a64);
            double fl, fr;
            P::flux(uL, P::aux(uL, I), d, I, &fl);
            P::flux(uR, P::aux(uR, I), d, I, &fr);
            fn0[b] = fma(-0.5 * ab, *uR - *uL, 0.5 * (fl + fr));
          }
        }
        face_accum<true>(f, fn, I, scale, r, fn0);
      } else {
        face_accum(f, fn, I, scale, r);
      }
    }
  }

  // u_out = base + r
  __device__ __forceinline__ static void combine(const State& base, const Acc& r, State& out) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      out.ub[v] = base.ub[v] + r.a0[v];
#pragma unroll
      for (int m = 0; m < MH; ++m) out.ch[v][m] = base.ch[v][m] + r.ah[v][m];
    }
  }

  // out += sum_p kap_p S_p (mode 0 in FP64, the other modes in T)
  __device__ __forceinline__ static void add_source(const KArgs& a, const InstDev& I, int64_t c,
                                                    const double* kap, State& out) {
    const int64_t nc = I.ncell;
    for (int p = 0; p < a.src.n; ++p) {
      const double* sa = a.src.avg[p] + I.avg_off;
      const T* sh = static_cast<const T*>(a.src.hi[p]) + I.hi_off;
      const T kt = T(kap[p]);
#pragma unroll
      for (int v = 0; v < V; ++v) {
        out.ub[v] = fma(kap[p], sa[v * nc + c], out.ub[v]);
#pragma unroll
        for (int m = 0; m < MH; ++m)
          out.ch[v][m] = fma(kt, sh[(static_cast<int64_t>(v) * MH + m) * nc + c], out.ch[v][m]);
      }
    }
  }

  // admissibility of the cell average (Sec. 4.1 algorithm; B^eps by reading A6)
  __device__ __forceinline__ static bool average_ok(const State& s, const InstDev& I) {
    if constexpr (SYS == SYS_EULER) {
      double ke = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) ke = fma(s.ub[1 + j], s.ub[1 + j], ke);
      const double rhoe = s.ub[D + 1] - 0.5 * ke / s.ub[0];
      return (s.ub[0] >= I.eps) && (rhoe >= I.eps);
    } else if constexpr (SYS == SYS_SWE) {
      return s.ub[0] >= I.eps;
    } else {
      return (s.ub[0] >= I.blo_chk) && (s.ub[0] <= I.bhi_chk);
    }
  }
  __device__ __forceinline__ static bool average_finite(const State& s) {
    bool ok = true;
#pragma unroll
    for (int v = 0; v < V; ++v) ok = ok && isfinite(s.ub[v]);
    return ok;
  }

  __device__ __forceinline__ static void scale_modes(State& s, double th_first, double th_rest) {
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const double th = (v == 0) ? th_first : th_rest;
#pragma unroll
      for (int m = 0; m < MH; ++m) s.ch[v][m] = T(th * static_cast<double>(s.ch[v][m]));
    }
  }

  // every S_K point inside B (scalar) / B^eps (Euler); FP64 evaluation
  __device__ __forceinline__ static bool points_ok(const State& s, const InstDev& I) {
    bool ok = true;
#pragma unroll US
    for (int p = 0; p < NS; ++p) {
      if constexpr (SYS == SYS_EULER) {
        const double rho = sk_var(s, p, 0);
        double ke = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
          const double mj = sk_var(s, p, 1 + j);
          ke = fma(mj, mj, ke);
        }
        const double E = sk_var(s, p, D + 1);
        ok = ok && (rho >= I.eps) && (fma(E, rho, -0.5 * ke) >= I.eps * rho);
      } else if constexpr (SYS == SYS_SWE) {
        ok = ok && (sk_var(s, p, 0) >= I.eps);
      } else {
        const double u = sk_var(s, p, 0);
        ok = ok && (u >= I.blo) && (u <= I.bhi);
      }
    }
    return ok;
  }

  // One pass over S_K for the common case.  Returns true when every S_K
  // point is inside B (scalar) / B^eps (Euler) -- then the limiter is the
  // identity, exactly as the FP64 algorithm decides -- and, with A0, folds the
  // wave speeds of the points into a0[].  FP64: the exact tests of the
  // limiter.  Mixed: FP32 evaluation with a rigorous bound on its rounding
  // error (each value is a sum of at most M terms bounded by
  // B = |ubar| + sum |c_m|, since |phi_m| <= 1 on the cell; the sum-factorised
  // 2D evaluation takes at most 2K + 3 <= M + 1 roundings of partial sums
  // bounded by B), so "pass" in FP32 implies "pass" in FP64; near the bounds
  // the FP64 limiter decides.
  template <bool A0>
  __device__ __forceinline__ static bool sk_pass(const State& s, const InstDev& I, double* a0) {
    T ub[V], err[V], bnd[V];
    // wave speeds are maximised in T and widened once (exact and monotone)
    T am[D];
#pragma unroll
    for (int d = 0; d < D; ++d) am[d] = T(0);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      ub[v] = T(s.ub[v]);
      if constexpr (MIXED) {
        T b = fabs(ub[v]);
#pragma unroll
        for (int m = 0; m < MH; ++m) b += fabs(s.ch[v][m]);
        bnd[v] = b;
        err[v] = T(2.0 * (M + 1) * 0x1p-24) * b;
      } else {
        bnd[v] = T(0);
        err[v] = T(0);
      }
    }
    bool ok = true;
    if constexpr (SYS == SYS_EULER) {
      T thr_rho = T(I.eps) + T(2) * err[0];
      T marg = T(0);
      if constexpr (MIXED) {
        T mm = bnd[D + 1] * err[0] + bnd[0] * err[D + 1];
        T bb = bnd[D + 1] * bnd[0];
#pragma unroll
        for (int j = 0; j < D; ++j) {
          mm += bnd[1 + j] * err[1 + j];
          bb += bnd[1 + j] * bnd[1 + j];
        }
        marg = T(2) * (mm + T(4 * 0x1p-24) * bb) + T(2 * I.eps) * err[0];
        thr_rho *= T(1 + 0x1p-20);
      }
      const T eps = T(I.eps);
      auto check = [&](const T* u) {
        T ke = T(0);
#pragma unroll
        for (int j = 0; j < D; ++j) ke = fma(u[1 + j], u[1 + j], ke);
        const T q = fma(u[D + 1], u[0], T(-0.5) * ke);
        T rhs = fma(eps, u[0], marg);
        if constexpr (MIXED) rhs *= T(1 + 0x1p-20);
        ok = ok && (u[0] >= thr_rho) && (q >= rhs);
        if constexpr (A0) {
          const auto ax = P::aux(u, I);
#pragma unroll
          for (int d = 0; d < D; ++d) am[d] = fmax(am[d], P::speed(u, ax, d, I));
        }
      };
      if constexpr (SF) {
        sk_points_sf(s, check);
      } else {
#pragma unroll US
        for (int p = 0; p < NS; ++p) {
          T u[V];
#pragma unroll
          for (int v = 0; v < V; ++v) {
            T a = ub[v];
#pragma unroll
            for (int m = 1; m < M; ++m) {
              if constexpr (BIG) a = fma(RT::tab.phi_s[p][m], s.ch[v][m - 1], a);
              else a = cmad(S::tab.phi_s[p][m], s.ch[v][m - 1], a);
            }
            u[v] = a;
          }
          check(u);
        }
      }
    } else if constexpr (SYS == SYS_SWE) {
      // depth >= eps with the rounding bound of the FP32 evaluation
      T thr = T(I.eps) + T(2) * err[0];
      if constexpr (MIXED) thr *= T(1 + 0x1p-20);
      auto check = [&](const T* u) {
        ok = ok && (u[0] >= thr);
        if constexpr (A0) {
          const auto ax = P::aux(u, I);
#pragma unroll
          for (int d = 0; d < D; ++d) am[d] = fmax(am[d], P::speed(u, ax, d, I));
        }
      };
      if constexpr (SF) {
        sk_points_sf(s, check);
      } else {
#pragma unroll US
        for (int p = 0; p < NS; ++p) {
          T u[V];
#pragma unroll
          for (int v = 0; v < V; ++v) {
            T a = ub[v];
#pragma unroll
            for (int m = 1; m < M; ++m) {
              if constexpr (BIG) a = fma(RT::tab.phi_s[p][m], s.ch[v][m - 1], a);
              else a = cmad(S::tab.phi_s[p][m], s.ch[v][m - 1], a);
            }
            u[v] = a;
          }
          check(u);
        }
      }
    } else {
      const double lo = I.blo, hi = I.bhi;
      auto check = [&](const T* pa) {
        const T a = pa[0];
        const double u = static_cast<double>(a);
        const double e = static_cast<double>(err[0]);
        ok = ok && (u - e >= lo) && (u + e <= hi);
        if constexpr (A0) {
          const auto ax = P::aux(&a, I);
#pragma unroll
          for (int d = 0; d < D; ++d) am[d] = fmax(am[d], P::speed(&a, ax, d, I));
        }
      };
      if constexpr (SF) {
        sk_points_sf(s, check);
      } else {
#pragma unroll US
        for (int p = 0; p < NS; ++p) {
          T a = ub[0];
#pragma unroll
          for (int m = 1; m < M; ++m) {
            if constexpr (BIG) a = fma(RT::tab.phi_s[p][m], s.ch[0][m - 1], a);
            else a = cmad(S::tab.phi_s[p][m], s.ch[0][m - 1], a);
          }
          check(&a);
        }
      }
    }
    if constexpr (A0) {
#pragma unroll
      for (int d = 0; d < D; ++d) a0[d] = fmax(a0[d], static_cast<double>(am[d]));
    }
    return ok;
  }

  // Cheaper sufficient test without point evaluation: every Legendre product
  // satisfies |phi_m| <= 1 on the cell, so u_v lies in [ubar_v - R_v, ubar_v
  // + R_v] with R_v = sum_{m>=1} |c_vm| everywhere on K.  For Euler,
  // rho e >= eps follows from E rho - |m|^2 / 2 >= eps rho, bounded below by
  // (Ebar - R_E)(rhobar - R_rho) - sum_j (|mbar_j| + R_mj)^2 / 2 when both
  // factors are positive.  A pass proves the limiter is the identity.
  __device__ __forceinline__ static bool interval_pass(const State& s, const InstDev& I) {
    double R[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      T r = T(0);
#pragma unroll
      for (int m = 0; m < MH; ++m) r += fabs(s.ch[v][m]);
      // covers the rounding of the sum (at most MH terms)
      R[v] = static_cast<double>(r) * (1.0 + (MH + 2) * (MIXED ? 0x1p-23 : 0x1p-52));
    }
    if constexpr (SYS == SYS_EULER) {
      const double rlo = s.ub[0] - R[0];
      const double elo = s.ub[D + 1] - R[D + 1];
      if (!(rlo >= I.eps) || !(elo > 0.0)) return false;
      double mm = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const double mh = fabs(s.ub[1 + j]) + R[1 + j];
        mm = fma(mh, mh, mm);
      }
      const double qlo = fma(elo, rlo, -0.5 * mm);
      return qlo * (1.0 - 0x1p-40) >= I.eps * (s.ub[0] + R[0]);
    } else if constexpr (SYS == SYS_SWE) {
      return s.ub[0] - R[0] >= I.eps;
    } else {
      return (s.ub[0] - R[0] >= I.blo) && (s.ub[0] + R[0] <= I.bhi);
    }
  }

  // Scaling limiter on S_K, FP64 decisions.  Scalar: Prop. 2.4; Euler:
  // density step then internal-energy step on the density-limited polynomial
  // (Sec. 2.2.3); shallow water: one depth factor for every component.  A factor only acts where its bound is violated; it is
  // clamped to [0, 1].
  __device__ __forceinline__ static void limit_full(State& s, const InstDev& I) {
    double th_first = 1.0, th_rest = 1.0;
    if constexpr (SYS == SYS_EULER) {
      const double eps = I.eps;
      const double rb = s.ub[0];
      double rmin = INFINITY;
#pragma unroll US
      for (int p = 0; p < NS; ++p) rmin = fmin(rmin, sk_var(s, p, 0));
      double th1 = 1.0;
      if (!(rmin >= eps)) {
        th1 = (rb - eps) / (rb - rmin);
        th1 = (th1 >= 0.0) ? fmin(th1, 1.0) : 0.0;
      }
      // internal energy of the density-limited polynomial: cheap test first
      bool low = false;
#pragma unroll US
      for (int p = 0; p < NS; ++p) {
        const double r0 = sk_var(s, p, 0);
        const double rho = (th1 == 1.0) ? r0 : rb + th1 * (r0 - rb);
        double ke = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
          const double mj = sk_var(s, p, 1 + j);
          ke = fma(mj, mj, ke);
        }
        const double E = sk_var(s, p, D + 1);
        low = low || !(fma(E, rho, -0.5 * ke) >= eps * rho);
      }
      double th2 = 1.0;
      if (low) {
        double emin = INFINITY;
        for (int p = 0; p < NS; ++p) {
          const double r0 = sk_var(s, p, 0);
          const double rho = (th1 == 1.0) ? r0 : rb + th1 * (r0 - rb);
          double ke = 0.0;
          for (int j = 0; j < D; ++j) {
            const double mj = sk_var(s, p, 1 + j);
            ke = fma(mj, mj, ke);
          }
          emin = fmin(emin, sk_var(s, p, D + 1) - 0.5 * ke / rho);
        }
        double kb = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) kb = fma(s.ub[1 + j], s.ub[1 + j], kb);
        const double eb = s.ub[D + 1] - 0.5 * kb / rb;
        th2 = (eb - eps) / (eb - emin);
        th2 = (th2 >= 0.0) ? fmin(th2, 1.0) : 0.0;
        if (!(emin < eps)) th2 = 1.0;
      }
      th_first = th1 * th2;
      th_rest = th2;
    } else if constexpr (SYS == SYS_SWE) {
      // one depth factor scales every component (reading A28)
      const double hb = s.ub[0];
      double hmin = INFINITY;
#pragma unroll US
      for (int p = 0; p < NS; ++p) hmin = fmin(hmin, sk_var(s, p, 0));
      double th = 1.0;
      if (!(hmin >= I.eps)) {
        th = (hb - I.eps) / (hb - hmin);
        th = (th >= 0.0) ? fmin(th, 1.0) : 0.0;
      }
      th_first = th_rest = th;
    } else {
      const double ub = s.ub[0];
      double mx = -INFINITY, mn = INFINITY;
#pragma unroll US
      for (int p = 0; p < NS; ++p) {
        const double u = sk_var(s, p, 0);
        mx = fmax(mx, u);
        mn = fmin(mn, u);
      }
      double th = 1.0;
      if (mx > I.bhi) th = fmin(th, (I.bhi - ub) / (mx - ub));
      if (mn < I.blo) th = fmin(th, (I.blo - ub) / (mn - ub));
      th = (th >= 0.0) ? th : 0.0;
      th_first = th_rest = th;
    }
    if (th_first < 1.0 || th_rest < 1.0) {
      if constexpr (MIXED) {
        // FP32 rounding of the scaled modes can leave a point a few ulp
        // outside the bound: re-verify in FP64 and shrink theta by 2^-22,
        // 2^-18, 2^-14, 2^-10 in turn, finally theta = 0 (exact: the FP64
        // average is admissible).
        State orig = s;
        double f1 = th_first, f2 = th_rest;
        for (int attempt = 0; attempt < 6; ++attempt) {
          s = orig;
          if (attempt == 5) { f1 = 0.0; f2 = 0.0; }
          scale_modes(s, f1, f2);
          if (attempt == 5 || points_ok(s, I)) break;
          const double shrink = 1.0 - ldexp(1.0, -22 + 4 * attempt);
          f1 *= shrink;
          f2 *= shrink;
        }
      } else {
        scale_modes(s, th_first, th_rest);
      }
    }
  }

  // limiter (when enabled) and, with A0, the wave-speed maxima of the result
  template <bool A0>
  __device__ __forceinline__ static void limit_and_speeds(State& s, const InstDev& I, double* a0) {
    const bool pass = sk_pass<A0>(s, I, a0);
    if (!pass && I.limiter) {
      limit_full(s, I);
      if constexpr (A0) {
#pragma unroll
        for (int d = 0; d < D; ++d) a0[d] = 0.0;
        sk_pass<true>(s, I, a0);
      }
    }
  }

  __device__ __forceinline__ static void limit(State& s, const InstDev& I) {
    limit_and_speeds<false>(s, I, nullptr);
  }

  // Cells whose S_K test fails are not limited in the stage kernel: their
  // unlimited state goes, as one contiguous record, into a queue that a
  // small kernel drains right after the stage (the FP64 limiter then runs
  // at full lane occupancy instead of stalling the wavefronts that contain
  // such a cell; they are a few percent of the cells, near discontinuities).
  struct Record {
    int32_t inst;
    int32_t cell;
    double ub[V];
    T ch[V][MH];
  };
  // the queue holds a record for every cell of the group, so it never
  // overflows; the bound check only guards memory against a stale counter
  __device__ __forceinline__ static void enqueue(const KArgs& a, int inst, int64_t c, const State& s) {
    const unsigned idx = atomicAdd(a.qcount, 1u);
    if (idx >= a.qcap) return;
    Record* r = static_cast<Record*>(a.queue) + idx;
    r->inst = inst;
    r->cell = static_cast<int32_t>(c);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      r->ub[v] = s.ub[v];
#pragma unroll
      for (int m = 0; m < MH; ++m) r->ch[v][m] = s.ch[v][m];
    }
  }

  // max over S_K of the wave speed per direction
  __device__ __forceinline__ static void wave_speeds(const State& s, const InstDev& I, double* a0) {
#pragma unroll
    for (int d = 0; d < D; ++d) a0[d] = 0.0;
    sk_pass<true>(s, I, a0);
  }
};

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T* hi_ptr(void* p, int64_t off) {
  return static_cast<T*>(p) + off;
}

// Inner stage i = 2..s (Scheme 1L): out = L(base + dt a G(in)); flags on a
// non-admissible unlimited average.  With DG the operator is F instead of G:
// the inner stage of the standard RKDG scheme (Sec. 2.1) with the same
// Butcher table, limiter and check, which needs the neighbours' traces.
template <int D, int K, int SP, int SYS, typename T, bool DG = false>
__device__ __forceinline__ void stage_local_item(const KArgs& a, const BlockItem& bi) {
  using C = Cell<D, K, SP, SYS, T>;
  if (bi.inst < 0) return;  // padding entry of the XCD-ordered block map
  const InstDev& I = a.inst[bi.inst];
  crkdg_ctl* ctl = a.ctl + bi.inst;
  if (instance_idle(ctl)) return;
  const int s = I.stages;
  const int cur = a.slots.rotate ? ctl->cur : 0;
  const int nsl = s + 1;
  const int sl_in = (cur + a.stage - 2) % nsl;
  const int sl_out = (cur + a.stage - 1) % nsl;
  const double* in_avg = sel_avg(a.slots, sl_in) + I.avg_off;
  const T* in_hi = hi_ptr<T>(sel_hi(a.slots, sl_in), I.hi_off);
  const double* b_avg = sel_avg(a.slots, cur) + I.avg_off;
  const T* b_hi = hi_ptr<T>(sel_hi(a.slots, cur), I.hi_off);
  double* o_avg = sel_avg(a.slots, sl_out) + I.avg_off;
  T* o_hi = hi_ptr<T>(sel_hi(a.slots, sl_out), I.hi_off);
  const double dt = ctl->dt;

  bool active;
  CellPos pos;
  const int64_t c = tile_cell(bi, D, I.n, I.ncell, a.tile_shift, active, DG ? &pos : nullptr);
  bool bad = false, nonfin = false;
  if (active) {
    typename C::State u;
    C::load(in_avg, in_hi, I.ncell, c, u);
    typename C::Acc r;
    C::zero(r);
    if constexpr (DG)
      C::op_dg(u, in_avg, in_hi, pos, I, dt * a.a, r, C::global_alpha(ctl), bdata(a, bi.inst, a.stage - 2));
    else
      C::op_local(u, I, dt * a.a, r);
    typename C::State base, out;
    C::load(b_avg, b_hi, I.ncell, c, base);
    C::combine(base, r, out);
    if (a.src.n > 0) C::add_source(a, I, c, source_weights(a, bi.inst), out);
    bad = !C::average_ok(out, I);
    nonfin = !C::average_finite(out);
    const bool pass = !I.limiter || C::interval_pass(out, I) || C::template sk_pass<false>(out, I, nullptr);
    if (pass) C::store(o_avg, o_hi, I.ncell, c, out);
    else C::enqueue(a, bi.inst, c, out);
  }
  raise_flag(&ctl->flags, bad, CRKDG_F_AVERAGE);
  raise_flag(&ctl->flags, nonfin, CRKDG_F_NONFINITE);
}

// Each stage kernel comes in two forms: one workgroup per tile of the block
// map, and a persistent grid (a multiple of 8, so that a workgroup stays on
// one XCD's run of tiles) walking the map with a grid stride.  The loop of
// the persistent form costs registers and scheduling freedom (measured: the
// 2D Q^2 final stage runs 2x slower as a loop even with one tile per
// workgroup), so the one-tile form serves grids of one workgroup per tile.
template <int D, int K, int SP, int SYS, typename T>
__global__ __launch_bounds__(BLOCK) void k_stage_local(KArgs a) {
  if (static_cast<int>(blockIdx.x) < a.n_items) stage_local_item<D, K, SP, SYS, T>(a, a.bmap[blockIdx.x]);
}
template <int D, int K, int SP, int SYS, typename T>
__global__ __launch_bounds__(BLOCK) void k_stage_local_p(KArgs a) {
  for (int it = blockIdx.x; it < a.n_items; it += gridDim.x) stage_local_item<D, K, SP, SYS, T>(a, a.bmap[it]);
}
// inner stage of the standard RKDG scheme (operator F)
template <int D, int K, int SP, int SYS, typename T>
__global__ __launch_bounds__(BLOCK) void k_stage_inner_dg(KArgs a) {
  if (static_cast<int>(blockIdx.x) < a.n_items) stage_local_item<D, K, SP, SYS, T, true>(a, a.bmap[blockIdx.x]);
}
template <int D, int K, int SP, int SYS, typename T>
__global__ __launch_bounds__(BLOCK) void k_stage_inner_dg_p(KArgs a) {
  for (int it = blockIdx.x; it < a.n_items; it += gridDim.x) stage_local_item<D, K, SP, SYS, T, true>(a, a.bmap[it]);
}

// Final stage (Scheme 1L): out = L(base + dt sum_j b_j F(u~^(j))); also the
// wave speeds of the limited result for the next trial step.
template <int D, int K, int SP, int SYS, typename T>
__device__ __forceinline__ void stage_final_item(const KArgs& a, const BlockItem& bi) {
  using C = Cell<D, K, SP, SYS, T>;
  if (bi.inst < 0) return;  // padding entry of the XCD-ordered block map
  const InstDev& I = a.inst[bi.inst];
  crkdg_ctl* ctl = a.ctl + bi.inst;
  if (instance_idle(ctl)) return;
  const int s = I.stages;
  const int cur = a.slots.rotate ? ctl->cur : 0;
  const int nsl = s + 1;
  const int sl_out = (cur + s) % nsl;
  const double dt = ctl->dt;
  const double* b_avg = sel_avg(a.slots, cur) + I.avg_off;
  const T* b_hi = hi_ptr<T>(sel_hi(a.slots, cur), I.hi_off);
  double* o_avg = sel_avg(a.slots, sl_out) + I.avg_off;
  T* o_hi = hi_ptr<T>(sel_hi(a.slots, sl_out), I.hi_off);

  bool active;
  CellPos pos;
  const int64_t c = tile_cell(bi, D, I.n, I.ncell, a.tile_shift, active, &pos);
  bool bad = false, nonfin = false;
  double a0[D];
#pragma unroll
  for (int d = 0; d < D; ++d) a0[d] = 0.0;
  if (active) {
    typename C::Acc r;
    C::zero(r);
    // one inlined copy of F, applied to every stage with b_j != 0
#pragma unroll 1
    for (int j = 1; j <= s; ++j) {
      if (a.b[j - 1] == 0.0) continue;
      const int sl = (cur + j - 1) % nsl;
      const double* j_avg = sel_avg(a.slots, sl) + I.avg_off;
      const T* j_hi = hi_ptr<T>(sel_hi(a.slots, sl), I.hi_off);
      typename C::State uj;
      C::load(j_avg, j_hi, I.ncell, c, uj);
      C::op_dg(uj, j_avg, j_hi, pos, I, dt * a.b[j - 1], r, C::global_alpha(ctl), bdata(a, bi.inst, j - 1));
    }
    typename C::State base;
    C::load(b_avg, b_hi, I.ncell, c, base);
    typename C::State out;
    C::combine(base, r, out);
    if (a.src.n > 0) C::add_source(a, I, c, source_weights(a, bi.inst), out);
    bad = !C::average_ok(out, I);
    nonfin = !C::average_finite(out);
    double sp[D];
#pragma unroll
    for (int d = 0; d < D; ++d) sp[d] = 0.0;
    const bool pass = C::template sk_pass<true>(out, I, sp);
    if (!pass && I.limiter) {
      // limited (and its speeds taken) by the queue kernel
      C::enqueue(a, bi.inst, c, out);
    } else {
#pragma unroll
      for (int d = 0; d < D; ++d) a0[d] = sp[d];
      C::store(o_avg, o_hi, I.ncell, c, out);
    }
  }
  if (bad || nonfin) {
#pragma unroll
    for (int d = 0; d < D; ++d) a0[d] = 0.0;
  }
  raise_flag(&ctl->flags, bad, CRKDG_F_AVERAGE);
  raise_flag(&ctl->flags, nonfin, CRKDG_F_NONFINITE);
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const double m = wave_max(a0[d]);
    if ((threadIdx.x & 63) == 0 && m > 0.0)
      atomicMax(reinterpret_cast<unsigned long long*>(&ctl->a0_next[d]),
                static_cast<unsigned long long>(__double_as_longlong(m)));
  }
}

// Wavefronts per SIMD the register allocation of the one-thread final stage
// aims at: in the mixed 2D kernels at least two (at most 256 registers; the
// 2D P^3 Euler final stage took 272 and ran one wavefront per SIMD: 0.80 ms
// against 0.61 ms at two with a few spills); in FP64 unconstrained (there
// the limit spilled heavily: 1.13 -> 2.53 ms for the same stage), and in 3D
// too (3D Q^1 Euler spilled 240 B per lane under it).
template <int D, typename T>
constexpr int final_waves_per_eu() {
  return (sizeof(T) == 4 && D == 2) ? 2 : 1;
}

template <int D, int K, int SP, int SYS, typename T>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(final_waves_per_eu<D, T>()))) void
k_stage_final(KArgs a) {
  if (static_cast<int>(blockIdx.x) < a.n_items) stage_final_item<D, K, SP, SYS, T>(a, a.bmap[blockIdx.x]);
}
template <int D, int K, int SP, int SYS, typename T>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(final_waves_per_eu<D, T>()))) void
k_stage_final_p(KArgs a) {
  for (int it = blockIdx.x; it < a.n_items; it += gridDim.x) stage_final_item<D, K, SP, SYS, T>(a, a.bmap[it]);
}

// Limiter of the cells a stage kernel queued (same slot rotation as the
// stage); on the final stage also their wave speeds.
template <int D, int K, int SP, int SYS, typename T, bool FINAL>
__global__ __launch_bounds__(BLOCK) void k_limit_queue(KArgs a) {
  using C = Cell<D, K, SP, SYS, T>;
  const unsigned n0 = *a.qcount;
  const unsigned n = n0 < a.qcap ? n0 : a.qcap;
  const typename C::Record* rec = static_cast<const typename C::Record*>(a.queue);
  for (unsigned e = blockIdx.x * BLOCK + threadIdx.x; e < n; e += gridDim.x * BLOCK) {
    const typename C::Record& r = rec[e];
    const InstDev& I = a.inst[r.inst];
    crkdg_ctl* ctl = a.ctl + r.inst;
    const int s = I.stages;
    const int cur = a.slots.rotate ? ctl->cur : 0;
    const int sl_out = FINAL ? (cur + s) % (s + 1) : (cur + a.stage - 1) % (s + 1);
    double* avg = sel_avg(a.slots, sl_out) + I.avg_off;
    T* hi = hi_ptr<T>(sel_hi(a.slots, sl_out), I.hi_off);
    typename C::State u;
#pragma unroll
    for (int v = 0; v < C::V; ++v) {
      u.ub[v] = r.ub[v];
#pragma unroll
      for (int m = 0; m < C::MH; ++m) u.ch[v][m] = r.ch[v][m];
    }
    C::limit_full(u, I);
    C::store(avg, hi, I.ncell, r.cell, u);
    if constexpr (FINAL) {
      double a0[D];
      C::wave_speeds(u, I, a0);
      // the stage kernel already holds the maximum of the other cells: only
      // a larger speed needs the (contended) atomic; a stale read only costs
      // an unneeded atomic, never a lost update, as the value only grows
#pragma unroll
      for (int d = 0; d < D; ++d) {
        const unsigned long long bits = static_cast<unsigned long long>(__double_as_longlong(a0[d]));
        unsigned long long* dst = reinterpret_cast<unsigned long long*>(&ctl->a0_next[d]);
        if (bits > __atomic_load_n(dst, __ATOMIC_RELAXED)) atomicMax(dst, bits);
      }
    }
  }
}

// Standalone limiter in place, slot 0.
template <int D, int K, int SP, int SYS, typename T>
__global__ __launch_bounds__(BLOCK) void k_limit(KArgs a) {
  using C = Cell<D, K, SP, SYS, T>;
  const BlockItem bi = a.bmap[blockIdx.x];
  if (bi.inst < 0) return;  // padding entry of the XCD-ordered block map
  const InstDev& I = a.inst[bi.inst];
  crkdg_ctl* ctl = a.ctl ? a.ctl + bi.inst : nullptr;
  double* avg = a.slots.avg[0] + I.avg_off;
  T* hi = hi_ptr<T>(a.slots.hi[0], I.hi_off);
  bool active;
  const int64_t c = tile_cell(bi, D, I.n, I.ncell, a.tile_shift, active);
  bool bad = false;
  if (active) {
    typename C::State u;
    C::load(avg, hi, I.ncell, c, u);
    bad = !C::average_ok(u, I);
    if (I.limiter) {
      C::limit(u, I);
      C::store(avg, hi, I.ncell, c, u);
    }
  }
  if (ctl) raise_flag(&ctl->flags, bad, CRKDG_F_AVERAGE);
}

// a0 of slot 0 (or of slot ctl->cur when rotate) into ctl->a0_next (atomic max of bits).
template <int D, int K, int SP, int SYS, typename T>
__global__ __launch_bounds__(BLOCK) void k_cfl(KArgs a) {
  using C = Cell<D, K, SP, SYS, T>;
  const BlockItem bi = a.bmap[blockIdx.x];
  if (bi.inst < 0) return;  // padding entry of the XCD-ordered block map
  const InstDev& I = a.inst[bi.inst];
  crkdg_ctl* ctl = a.ctl + bi.inst;
  const int cur = a.slots.rotate ? ctl->cur : 0;
  const double* avg = sel_avg(a.slots, cur) + I.avg_off;
  const T* hi = hi_ptr<T>(sel_hi(a.slots, cur), I.hi_off);
  bool active;
  const int64_t c = tile_cell(bi, D, I.n, I.ncell, a.tile_shift, active);
  double a0[D];
#pragma unroll
  for (int d = 0; d < D; ++d) a0[d] = 0.0;
  if (active) {
    typename C::State u;
    C::load(avg, hi, I.ncell, c, u);
    C::wave_speeds(u, I, a0);
  }
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const double m = wave_max(a0[d]);
    if ((threadIdx.x & 63) == 0 && m > 0.0)
      atomicMax(reinterpret_cast<unsigned long long*>(&ctl->a0_next[d]),
                static_cast<unsigned long long>(__double_as_longlong(m)));
  }
}

// Discrete L2 projection of point samples at the volume Gauss points.
template <int D, int K, int SP, int SYS, typename T>
__global__ __launch_bounds__(BLOCK) void k_project(KArgs a) {
  using C = Cell<D, K, SP, SYS, T>;
  using S = typename C::S;
  const BlockItem bi = a.bmap[blockIdx.x];
  if (bi.inst < 0) return;  // padding entry of the XCD-ordered block map
  const InstDev& I = a.inst[bi.inst];
  double* avg = a.slots.avg[0] + I.avg_off;
  T* hi = hi_ptr<T>(a.slots.hi[0], I.hi_off);
  const double* smp = a.samples + I.smp_off;
  bool active;
  const int64_t c = tile_cell(bi, D, I.n, I.ncell, a.tile_shift, active);
  if (!active) return;
  typename C::State u;
#pragma unroll
  for (int v = 0; v < C::V; ++v) {
    double acc[C::M];
#pragma unroll
    for (int m = 0; m < C::M; ++m) acc[m] = 0.0;
#pragma unroll C::UQ
    for (int q = 0; q < S::NQ; ++q) {
      const double x = smp[(v * I.ncell + c) * S::NQ + q];
#pragma unroll
      for (int m = 0; m < C::M; ++m)
        acc[m] = fma(S::pfac(m) * S::tab.wq[q] * S::tab.phi_v[q][m], x, acc[m]);
    }
    u.ub[v] = acc[0];
#pragma unroll
    for (int m = 1; m < C::M; ++m) u.ch[v][m - 1] = T(acc[m]);
  }
  C::store(avg, hi, I.ncell, c, u);
}

}  // namespace crkdg
