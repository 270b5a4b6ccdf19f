// Cooperative stage kernels for the tensor-product spaces Q^k in 2D and 3D,
// and for the total-degree spaces P^k as subspaces of Q^k.
//
// One workgroup owns a tile of 64 cells (TX x TY x TZ) and has one wavefront
// per conserved variable: lane l of wavefront v holds the modes of variable v
// of cell l.  Everything linear in the modes runs per variable, by sum
// factorisation over the 1D Legendre series at the k+1 Gauss points (and the
// Lobatto points of S_K), with the few 1D values as immediates:
//   * point values at the volume Gauss points, the face traces (restriction to
//     the face, then the tangential series), the S_K point values;
//   * the volume residual sum_q sum_d (2/dx_d) w_q f_d(u_q) d phi_m/d xi_d and
//     the face residuals (Sec. 2.1 weak form), as transposed 1D passes.
// Everything nonlinear needs all variables at a point, so point values go
// through LDS: the fluxes at the volume points, and the Lax--Friedrichs
// fluxes at the face points.  Each face of the tile has one slot holding the
// traces of its two cells; its flux is formed once, in the canonical (lower,
// upper) orientation, and both cells read it.  Faces on the tile boundary get
// the outside cell's trace from that cell's modes in memory (a halo), with the
// same operations as an own trace, so the two tiles sharing such a face form
// bitwise the same flux and the averages stay conservative.
//
// P^k (Sec. 2, the spaces of the DG method) runs through the same arithmetic:
// its Legendre modes are the Q^k modes of total degree <= k, the quadrature
// rules are the same tensor rules, and the modes are orthogonal under them,
// so the P^k residual of a P^k state is the Q^k residual of the same state
// (zero in the other modes) restricted to the P^k modes.  Those other modes
// are compile-time zeros on input and never stored.
//
// The stage semantics are those of stage_local_item / stage_final_item
// (Scheme 1L of Appendix B, the checks of Sec. 4.1, the limiter of Sec. 2.2
// through the deferred queue, the wave speeds of Sec. 2.1 for the next trial
// step); only the arithmetic order differs.
#pragma once

#include <type_traits>

#include "device.hpp"

namespace crkdg {

// 1D tables of the Legendre basis at the k+1 Gauss nodes
template <int K> struct Leg1 {
  static constexpr int N = K + 1;
  double P[N][N];    // P[i][a] = P_a(g_i)
  double W[N][N];    // W[a][i] = (2a+1) (w_i/2) P_a(g_i): projection onto mode a
  double Dv[N][N];   // Dv[a][i] = (2a+1) (w_i/2) P_a'(g_i): derivative rows of the weak form
  double P0[N];      // P_a(0)
  constexpr Leg1() : P{}, W{}, Dv{}, P0{} {
    for (int i = 0; i < N; ++i)
      for (int a = 0; a < N; ++a) {
        const double wh = 0.5 * Gauss<N>::w[i];
        P[i][a] = leg(a, Gauss<N>::x[i]);
        W[a][i] = (2.0 * a + 1.0) * wh * leg(a, Gauss<N>::x[i]);
        Dv[a][i] = (2.0 * a + 1.0) * wh * dleg(a, Gauss<N>::x[i]);
      }
    for (int a = 0; a < N; ++a) P0[a] = leg(a, 0.0);
  }
};

// 1D operators on N = k+1 values.  The Gauss nodes come in pairs +-g (and 0
// when N is odd): P_a(-x) = (-1)^a P_a(x) splits every series into an even
// and an odd part that the two nodes of a pair share.
template <int K, typename T> struct Op1 {
  static constexpr int N = K + 1;
  static constexpr int H = (K + 2) / 2;        // node pairs (the middle node counts once)
  static constexpr int NL = (K == 1) ? 2 : 3;  // Lobatto nodes of S_K
  static constexpr Leg1<K> L{};

  // u_i = sum_a P_a(g_i) c_a.  Floating-point contraction is off in these
  // operators: a cell's trace and the same cell's trace as a halo of another
  // tile must be bitwise equal wherever they are inlined.
  __device__ __forceinline__ static void eval(const T (&c)[N], T (&u)[N]) {
#pragma clang fp contract(off)
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const int i = K - j;
      T E = c[0];
#pragma unroll
      for (int a = 2; a <= K; a += 2) E = fma(T(L.P[i][a]), c[a], E);
      if (i == j) {
        u[i] = E;
      } else {
        T O = T(L.P[i][1]) * c[1];
#pragma unroll
        for (int a = 3; a <= K; a += 2) O = fma(T(L.P[i][a]), c[a], O);
        u[i] = E + O;
        u[j] = E - O;
      }
    }
  }
  // values at the faces xi = -1 (lo) and +1 (up): P_a(+-1) = (+-1)^a
  __device__ __forceinline__ static void ends(const T (&c)[N], T& lo, T& up) {
#pragma clang fp contract(off)
    T E = c[0];
#pragma unroll
    for (int a = 2; a <= K; a += 2) E = E + c[a];
    T O = c[1];
#pragma unroll
    for (int a = 3; a <= K; a += 2) O = O + c[a];
    up = E + O;
    lo = E - O;
  }
  // values at the Lobatto nodes (-1, [0,] 1)
  __device__ __forceinline__ static void eval_l(const T (&c)[N], T (&u)[NL]) {
#pragma clang fp contract(off)
    ends(c, u[0], u[NL - 1]);
    if constexpr (NL == 3) {
      T Z = c[0];
#pragma unroll
      for (int a = 2; a <= K; a += 2) Z = fma(T(L.P0[a]), c[a], Z);
      u[1] = Z;
    }
  }
  // sums and differences of the node pairs
  __device__ __forceinline__ static void pairs(const T (&f)[N], T (&S)[H], T (&Df)[H]) {
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const int i = K - j;
      if (i == j) {
        S[j] = f[i];
        Df[j] = T(0);
      } else {
        S[j] = f[i] + f[j];
        Df[j] = f[i] - f[j];
      }
    }
  }
  // r_a = sum_i W[a][i] f_i
  __device__ __forceinline__ static void proj(const T (&f)[N], T (&r)[N]) {
    T S[H], Df[H];
    pairs(f, S, Df);
#pragma unroll
    for (int a = 0; a <= K; ++a) {
      T acc = T(0);
      bool first = true;
#pragma unroll
      for (int j = 0; j < H; ++j) {
        const int i = K - j;
        if (i == j && (a & 1)) continue;            // P_a(0) = 0 for odd a
        const T x = (a & 1) ? Df[j] : S[j];
        const T w = T(L.W[a][i]);
        acc = first ? w * x : fma(w, x, acc);
        first = false;
      }
      r[a] = acc;
    }
  }
  // r_a = sum_i Dv[a][i] f_i  (r_0 = 0: P_0' = 0)
  __device__ __forceinline__ static void projd(const T (&f)[N], T (&r)[N]) {
    T S[H], Df[H];
    pairs(f, S, Df);
    r[0] = T(0);
#pragma unroll
    for (int a = 1; a <= K; ++a) {
      T acc = T(0);
      bool first = true;
#pragma unroll
      for (int j = 0; j < H; ++j) {
        const int i = K - j;
        if (i == j && !(a & 1)) continue;           // P_a'(0) = 0 for even a
        const T x = (a & 1) ? S[j] : Df[j];         // P_a'(-x) = (-1)^(a+1) P_a'(x)
        const T w = T(L.Dv[a][i]);
        acc = first ? w * x : fma(w, x, acc);
        first = false;
      }
      r[a] = acc;
    }
  }
};

// y = op(x) along axis AX of an N^ND array (index i_0 + N i_1 + N^2 i_2)
template <int N, int ND, int AX, typename T, class Op>
__device__ __forceinline__ void along(const T (&x)[ipow(N, ND)], T (&y)[ipow(N, ND)], Op op) {
  constexpr int st = ipow(N, AX);
  static_for<ipow(N, ND - 1)>([&](auto LN) {
    constexpr int l = decltype(LN)::value;
    constexpr int base = (l % st) + (l / st) * st * N;
    T in[N], out[N];
#pragma unroll
    for (int i = 0; i < N; ++i) in[i] = x[base + i * st];
    op(in, out);
#pragma unroll
    for (int i = 0; i < N; ++i) y[base + i * st] = out[i];
  });
}
// y = op1(x1) + op2(x2) along axis AX
template <int N, int ND, int AX, typename T, class Op1_, class Op2_>
__device__ __forceinline__ void along2(const T (&x1)[ipow(N, ND)], const T (&x2)[ipow(N, ND)],
                                       T (&y)[ipow(N, ND)], Op1_ op1, Op2_ op2) {
  constexpr int st = ipow(N, AX);
  static_for<ipow(N, ND - 1)>([&](auto LN) {
    constexpr int l = decltype(LN)::value;
    constexpr int base = (l % st) + (l / st) * st * N;
    T a1[N], a2[N], b1[N], b2[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      a1[i] = x1[base + i * st];
      a2[i] = x2[base + i * st];
    }
    op1(a1, b1);
    op2(a2, b2);
#pragma unroll
    for (int i = 0; i < N; ++i) y[base + i * st] = b1[i] + b2[i];
  });
}

// KL = 1: the LDS layout of the inner stage with G (KIND 0), which shares no
// face values between cells: per-cell face slots (64 cells instead of the
// tile's faces), and where the volume goes through LDS by slabs (Q^3 in 3D)
// the S_K values one Lobatto node at a time.
template <int D, int K, int SP, int SYS, typename T, int TX, int TY, int TZ, int KL = 0>
struct Coop {
  using S = Space<D, K, SP_Q>;    // the tensor space the arithmetic runs in
  using SS = Space<D, K, SP>;     // the stored space (Q^k, or P^k inside it)
  using P = Phys<D, SYS>;
  using O1 = Op1<K, T>;
  using CellT = Cell<D, K, SP, SYS, T>;
  using Rec = typename CellT::Record;
  static constexpr int V = P::V;
  static constexpr int N = K + 1;
  static constexpr int M = S::M;       // tensor modes per variable (registers)
  static constexpr int MH = SS::M - 1; // stored modes >= 1 per variable (memory)
  static constexpr int NQ = S::NQ;
  static constexpr int NFP = S::NFP;
  static constexpr int NL = O1::NL;
  static constexpr int NPF = NL * ipow(N, D - 1);  // S_K points of one family
  static constexpr int NT = 64 * V;
  static constexpr bool MIXED = sizeof(T) == 4;
  static_assert(TX * TY * TZ == 64, "a tile holds one cell per lane");
  static_assert(D == 3 || TZ == 1, "2D tiles are flat");

  static constexpr int tdim(int d) { return d == 0 ? TX : d == 1 ? TY : TZ; }
  // the directions tangential to faces normal to d (ascending)
  static constexpr int oax1(int d) { return d == 0 ? 1 : 0; }
  static constexpr int oax2(int d) { return d == 2 ? 1 : 2; }
  static constexpr int tsz1(int d) { return tdim(oax1(d)); }
  static constexpr int tsz2(int d) { return D == 3 ? tdim(oax2(d)) : 1; }
  // face slots of the tile normal to d: (T_d + 1) positions x tangential cells
  static constexpr int nfd(int d) { return (tdim(d) + 1) * tsz1(d) * tsz2(d); }
  static constexpr int cmax(int a, int b) { return a > b ? a : b; }
  static constexpr int NF_MAX = cmax(cmax(nfd(0), nfd(1)), D == 3 ? nfd(2) : 0);
  static constexpr bool LOCAL = KL == 1;
  // the volume point values of all variables go through LDS at once, or
  // (when that would exceed 120 KiB: FP64 Q^3 in 3D) one slab of the last
  // direction at a time.  (For mixed Q^3, 80 KiB at once, the slabs only
  // added barriers: the face slots keep it at one workgroup per CU either
  // way; 19.3 against 18.8 ms per step on 96^3.)  (Slabs for the 3D Q^2 G stage, with the S_K values
  // by Lobatto node, took its LDS from 40 to 28 KB, room for four workgroups
  // per CU instead of two or three, but the stage ran 9% slower: the slabs'
  // barriers and the x-y values kept live cost more than the occupancy gave;
  // two passes with the modes loaded again for the second ran 18% slower.)
  static constexpr bool SLAB = D == 3 && V * NQ * 64 * sizeof(T) > 120 * 1024;
  static constexpr int NQL = SLAB ? NQ / N : NQ;    // volume points per LDS pass
  static constexpr int NLC = (LOCAL && SLAB) ? 1 : NL;  // Lobatto nodes of S_K per LDS pass
  static constexpr int NPC = NLC * ipow(N, D - 1);  // S_K points per LDS pass
  static constexpr int LDS_T = LOCAL ? cmax(cmax(V * NQL * 64, V * NFP * 2 * 64), V * NPC * 64)
                                     : cmax(cmax(V * NQL * 64, V * NFP * 2 * NF_MAX), V * NPC * 64);

  // stored index of tensor mode m (exponents m % N, (m / N) % N, m / N^2),
  // -1 for a mode outside the stored space
  struct SMap {
    int s[M];
    constexpr SMap() : s{} {
      for (int m = 0; m < M; ++m) s[m] = -1;
      for (int p = 0; p < SS::M; ++p) s[SS::modes.e[p][0] + N * (SS::modes.e[p][1] + N * SS::modes.e[p][2])] = p;
    }
  };
  static constexpr SMap smap{};
  // face quadrature weights (tensor Gauss, summing to one; Prop. 2.1)
  struct FaceW {
    double w[NFP];
    constexpr FaceW() : w{} {
      for (int b = 0; b < NFP; ++b) {
        double x = 1.0;
        for (int j = 0, r = b; j < D - 1; ++j, r /= N) x *= 0.5 * Gauss<N>::w[r % N];
        w[b] = x;
      }
    }
  };
  static constexpr FaceW fw{};
  // a mode >= 1 of the stored space: one whose residual is formed
  static constexpr bool live(int m) { return smap.s[m] > 0; }

  // non-negative T values ordered by their bits: LDS max of wave speeds
  using AB = typename std::conditional<MIXED, unsigned, unsigned long long>::type;
  __device__ __forceinline__ static AB bits_of(T x) {
    if constexpr (MIXED) return __float_as_uint(x);
    else return static_cast<unsigned long long>(__double_as_longlong(x));
  }
  __device__ __forceinline__ static T of_bits(AB b) {
    if constexpr (MIXED) return __uint_as_float(b);
    else return __longlong_as_double(static_cast<long long>(b));
  }

  // the LDS word type: indices into it stay 32-bit
  using LT = __attribute__((address_space(3))) T;
  struct Smem {
    T buf[LDS_T];
    double avg[V][64];     // output averages of the tile's cells
    T rsum[V][64];         // sum_{m >= 1} |c_vm| of the output
    AB spd[D][64];         // per cell: largest wave speed over S_K (bits)
    unsigned fail[64];     // per cell: an S_K point failed the test
    unsigned qidx[64];     // per cell: record index in the queue
    int flag;
  };

  // Element c of the row that starts at `row` (a wave-uniform address): the
  // byte offset is 32-bit (meshes of these variants hold fewer than 2^29
  // cells, checked at mesh creation), so the access is a scalar base plus
  // one vector offset register.  Stores go through the global address space
  // (vector memory instructions, not flat ones); loads stay generic, since
  // global-space loads let the scheduler hoist the halo loads far ahead of
  // their use and spill
  template <typename U>
  __device__ __forceinline__ static U ld(const U* row, uint32_t c) {
    return *reinterpret_cast<const U*>(reinterpret_cast<const char*>(row) + c * static_cast<uint32_t>(sizeof(U)));
  }
  template <typename U>
  __device__ __forceinline__ static void st(U* row, uint32_t c, U x) {
    using G = __attribute__((address_space(1))) char;
    using GU = __attribute__((address_space(1))) U;
    *(GU*)((G*)row + c * static_cast<uint32_t>(sizeof(U))) = x;
  }
  // modes of variable v (wave-uniform) of cell c in memory (mode 0 rounded to T)
  __device__ __forceinline__ static void load_var(const double* avg, const T* hi, int64_t nc, uint32_t c, int v,
                                                  T (&cm)[M], double& c0) {
    c0 = ld(avg + v * nc, c);
    cm[0] = T(c0);
    const T* h = hi + static_cast<int64_t>(v) * MH * nc;
    static_for<M - 1>([&](auto MM) {
      constexpr int m = decltype(MM)::value + 1;
      constexpr int p = smap.s[m];
      if constexpr (p > 0) cm[m] = ld(h + (p - 1) * nc, c);
      else cm[m] = T(0);
    });
  }

  // trace values of a cell on its two faces normal to d (tangential index
  // b = b1 + N b2 over the tangential directions, ascending)
  template <int d>
  __device__ __forceinline__ static void traces(const T (&cm)[M], T (&lo)[NFP], T (&up)[NFP]) {
    constexpr int sd = ipow(N, d);
    constexpr int s1 = ipow(N, oax1(d));
    constexpr int s2 = (D == 3) ? ipow(N, oax2(d)) : 0;
    T Rl[NFP], Ru[NFP];
#pragma unroll
    for (int t = 0; t < NFP; ++t) {
      const int t1 = t % N, t2 = t / N;
      const int base = t1 * s1 + t2 * s2;
      T line[N];
#pragma unroll
      for (int a = 0; a < N; ++a) line[a] = cm[base + a * sd];
      O1::ends(line, Rl[t], Ru[t]);
    }
    auto ev = [](const T (&x)[N], T (&y)[N]) { O1::eval(x, y); };
    if constexpr (D == 2) {
      O1::eval(Rl, lo);
      O1::eval(Ru, up);
    } else {
      T tl[NFP], tu[NFP];
      along<N, 2, 0>(Rl, tl, ev);
      along<N, 2, 1>(tl, lo, ev);
      along<N, 2, 0>(Ru, tu, ev);
      along<N, 2, 1>(tu, up, ev);
    }
  }

  __device__ __forceinline__ static LT* lds(Smem& sm) { return (LT*)(sm.buf); }
  __device__ __forceinline__ static const LT* lds(const Smem& sm) { return (const LT*)(sm.buf); }

  // tile geometry of the calling thread
  struct Geo {
    int v, lane;
    int l[3];       // local cell coordinates
    int o[3];       // tile origin
    int A[3];       // active extent of the tile per direction
    bool active;
    uint32_t c;     // cell index (0 when inactive)
  };
  __device__ __forceinline__ static Geo geo(const BlockItem& bi, const InstDev& I, int tid) {
    Geo g;
    // the variable is uniform across the wavefront: keep it (and every
    // per-variable address) in scalar registers
    g.v = __builtin_amdgcn_readfirstlane(tid >> 6);
    g.lane = tid & 63;
    g.l[0] = g.lane % TX;
    g.l[1] = (g.lane / TX) % TY;
    g.l[2] = g.lane / (TX * TY);
    g.o[0] = bi.x0;
    g.o[1] = bi.y0;
    g.o[2] = (D == 3) ? bi.z : 0;
    g.active = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      g.A[d] = (d < D) ? min(tdim(d), I.n[d] - g.o[d]) : 1;
      g.active = g.active && g.l[d] < g.A[d];
    }
    g.c = g.active ? static_cast<uint32_t>((g.o[0] + g.l[0]) +
                                           I.n[0] * ((g.o[1] + g.l[1]) + I.n[1] * (g.o[2] + g.l[2])))
                   : 0u;
    return g;
  }

  // face slot of position p along d and tangential cell coordinates (q1, q2)
  template <int d>
  __device__ __forceinline__ static int slot(int p, int q1, int q2) {
    return p + (tdim(d) + 1) * (q1 + tsz1(d) * q2);
  }
  // LDS index of a face value: [v][side][slot][b] (the points of a face
  // contiguous: the lanes of a face group read consecutive words)
  template <int d>
  __device__ __forceinline__ static int fidx(int v, int b, int side, int fi) {
    return ((v * 2 + side) * nfd(d) + fi) * NFP + b;
  }
  // G (no value shared between cells): the traces of each cell's own lower
  // (side 0) and upper (side 1) face, [v][side][b][lane]
  __device__ __forceinline__ static int cidx(int v, int b, int side, int lane) {
    return ((v * 2 + side) * NFP + b) * 64 + lane;
  }

  // ---- volume part of the weak form (Sec. 2.1): r += scale * volume residual
  // of the state (avg, hi) of this thread's cell and variable
  __device__ __forceinline__ static void volume(const Geo& g, const double* avg, const T* hi, const InstDev& I,
                                                double scale, T (&r)[M], Smem& sm) {
    auto ev = [](const T (&x)[N], T (&y)[N]) { O1::eval(x, y); };
    T t2[M];   // with slabs: the x and y passes, kept for the z node of each slab
    {
      T cm[M], t1[M];
      double c0;
      if (g.active) load_var(avg, hi, I.ncell, g.c, g.v, cm, c0);
      else
#pragma unroll
        for (int m = 0; m < M; ++m) cm[m] = T(0);
      along<N, D, 0>(cm, t1, ev);
      along<N, D, 1>(t1, t2, ev);
      if constexpr (D == 2) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) lds(sm)[(g.v * NQ + q) * 64 + g.lane] = t2[q];
      } else if constexpr (!SLAB) {
        along<N, D, 2>(t2, t1, ev);
#pragma unroll
        for (int q = 0; q < NQ; ++q) lds(sm)[(g.v * NQ + q) * 64 + g.lane] = t1[q];
      }
    }
    if constexpr (!SLAB) __syncthreads();
    // this variable's flux components, scaled by scale * 2 / dx_d; the
    // transposed passes sum_d (Dv along d) x (W along the others), slab by
    // slab of the last direction so that few partial sums are live
    T sd[D];
#pragma unroll
    for (int d = 0; d < D; ++d) sd[d] = T(scale * I.r2dx[d]);
    static_for<N>([&](auto KK) {
      constexpr int k = decltype(KK)::value;      // z node (3D) / y node (2D)
      if constexpr (D == 2) {
        T fx[N], fy[N], gx[N], gy[N];
#pragma unroll
        for (int i = 0; i < N; ++i) {
          T fd[D];
          flux_at(g, i + N * k, I, sd, fd, sm);
          fx[i] = fd[0];
          fy[i] = fd[1];
        }
        O1::projd(fx, gx);
        O1::proj(fy, gy);
#pragma unroll
        for (int a = 0; a < N; ++a)
#pragma unroll
          for (int b = 0; b < N; ++b) {
            const int m = a + N * b;
            if (!live(m)) continue;
            if (O1::L.W[b][k] != 0.0) r[m] = fma(T(O1::L.W[b][k]), gx[a], r[m]);
            if (O1::L.Dv[b][k] != 0.0) r[m] = fma(T(O1::L.Dv[b][k]), gy[a], r[m]);
          }
      } else {
        if constexpr (SLAB) {
          // the point values of z node k: one slab of every variable in LDS
#pragma unroll
          for (int q = 0; q < N * N; ++q) {
            T u = T(O1::L.P[k][0]) * t2[q];
#pragma unroll
            for (int c = 1; c < N; ++c) u = fma(T(O1::L.P[k][c]), t2[q + N * N * c], u);
            lds(sm)[(g.v * NQL + q) * 64 + g.lane] = u;
          }
          __syncthreads();
        }
        constexpr int qk = SLAB ? 0 : N * N * k;   // first point of the slab in LDS
        // x pass of the three components on every x line of the slab
        T gx[N][N], gy[N][N], gz[N][N];   // [y node][x mode]
#pragma unroll
        for (int j = 0; j < N; ++j) {
          T fx[N], fy[N], fz[N];
#pragma unroll
          for (int i = 0; i < N; ++i) {
            T fd[D];
            flux_at(g, i + N * j + qk, I, sd, fd, sm);
            fx[i] = fd[0];
            fy[i] = fd[1];
            fz[i] = fd[2];
          }
          O1::projd(fx, gx[j]);
          O1::proj(fy, gy[j]);
          O1::proj(fz, gz[j]);
        }
        // y pass: A = W_y gx + Dv_y gy (both take W_z next), B = W_y gz (takes Dv_z)
#pragma unroll
        for (int a = 0; a < N; ++a) {
          T lx[N], ly[N], lz[N], A1[N], A2[N], B[N];
#pragma unroll
          for (int j = 0; j < N; ++j) {
            lx[j] = gx[j][a];
            ly[j] = gy[j][a];
            lz[j] = gz[j][a];
          }
          O1::proj(lx, A1);
          O1::projd(ly, A2);
          O1::proj(lz, B);
          // z: r(a, b, c) += W_z[c][k] A(a, b) + Dv_z[c][k] B(a, b)
#pragma unroll
          for (int b = 0; b < N; ++b) {
            const T A = A1[b] + A2[b];
#pragma unroll
            for (int c = 0; c < N; ++c) {
              const int m = a + N * b + N * N * c;
              if (!live(m)) continue;
              if (O1::L.W[c][k] != 0.0) r[m] = fma(T(O1::L.W[c][k]), A, r[m]);
              if (O1::L.Dv[c][k] != 0.0) r[m] = fma(T(O1::L.Dv[c][k]), B[b], r[m]);
            }
          }
        }
        if constexpr (SLAB) __syncthreads();   // the slab is read before the next one is written
      }
    });
    if constexpr (!SLAB) __syncthreads();
  }

  // this variable's flux components (all directions, scaled by sd) at
  // volume point q, from the point values of every variable in LDS; the
  // variable is uniform across the wavefront, so each wavefront takes one
  // branch and forms only its own components
  __device__ __forceinline__ static void flux_at(const Geo& g, int q, const InstDev& I, const T (&sd)[D],
                                                 T (&fd)[D], const Smem& sm) {
    T u[V];
#pragma unroll
    for (int w = 0; w < V; ++w) u[w] = lds(sm)[(w * NQL + q) * 64 + g.lane];
    if constexpr (SYS == SYS_EULER) {
      if (g.v == 0) {
        // mass flux m_d
#pragma unroll
        for (int d = 0; d < D; ++d) fd[d] = sd[d] * u[1 + d];
        return;
      }
      const auto ax = P::aux(u, I);
      if (g.v == D + 1) {
        // energy flux (E + p) w_d
        const T ep = u[D + 1] + ax.p;
#pragma unroll
        for (int d = 0; d < D; ++d) fd[d] = sd[d] * (ep * ax.w[d]);
        return;
      }
      // momentum flux m_j w_d + p delta_jd, j = v - 1
      static_for<D>([&](auto JJ) {
        constexpr int j = decltype(JJ)::value;
        if (g.v == 1 + j) {
#pragma unroll
          for (int d = 0; d < D; ++d) {
            const T x = u[1 + j] * ax.w[d];
            fd[d] = sd[d] * ((j == d) ? x + ax.p : x);
          }
        }
      });
    } else {
#pragma unroll
      for (int d = 0; d < D; ++d) {
        T f[V];
        P::flux(u, P::aux(u, I), d, I, f);
        fd[d] = sd[d] * f[0];
      }
    }
  }

  // ---- faces normal to d: traces into the slots; the flux (F: Lax--Friedrichs
  // with neighbours and halos; G: each cell's interior trace) back into the
  // slots; then the face residuals of both faces of the cell
  template <int d, bool DG>
  __device__ __forceinline__ static void faces(const Geo& g, const double* avg, const T* hi, const InstDev& I,
                                               double scale, double ag, T (&r)[M], double& r0, Smem& sm,
                                               const BData& bd) {
    constexpr int NFD = nfd(d);
    constexpr int T1 = tsz1(d), T2 = tsz2(d);
    const int q1 = g.l[oax1(d)];
    const int q2 = (D == 3) ? g.l[oax2(d)] : 0;
    const int fi_lo = slot<d>(g.l[d], q1, q2);
    const int fi_up = slot<d>(g.l[d] + 1, q1, q2);
    // (0) the halo cell of this lane (the tile shapes used have at most 64
    // halo cells per direction: one per lane; periodic wrap included, while
    // a non-periodic mesh side has none: its ghost is formed in the flux
    // pass): its modes are loaded before the own traces are formed, so that
    // the loads' latency overlaps that work
    static_assert(2 * T1 * T2 <= 64, "one halo cell per lane");
    T hm[M];
    double h0 = 0.0;
    bool hv = false;
    int hside = 0, hfi = 0;
    if constexpr (DG) {
      const int j = g.lane;
      if (j < 2 * T1 * T2) {
        const int side = j / (T1 * T2);
        const int qq = j % (T1 * T2);
        const int h1 = qq % T1, h2 = qq / T1;
        hv = h1 < g.A[oax1(d)] && (D == 2 || h2 < g.A[oax2(d)]);
        int x = g.o[d] + (side ? g.A[d] : -1);
        if (hv && (x < 0 || x >= I.n[d])) {
          hv = I.bc[2 * d + side] == CRKDG_BC_PERIODIC;
          x = (x < 0) ? x + I.n[d] : x - I.n[d];
        }
        if (hv) {
          int hc[3] = {0, 0, 0};
          hc[oax1(d)] = g.o[oax1(d)] + h1;
          if (D == 3) hc[oax2(d)] = g.o[oax2(d)] + h2;
          hc[d] = x;
          const uint32_t hcell = static_cast<uint32_t>(hc[0] + I.n[0] * (hc[1] + I.n[1] * hc[2]));
          load_var(avg, hi, I.ncell, hcell, g.v, hm, h0);
          hside = side;
          hfi = slot<d>(side ? g.A[d] : 0, h1, h2);
        }
      }
    }
    // (1) own traces: this cell is the upper cell of its lower face (side 1)
    // and the lower cell of its upper face (side 0)
    if (g.active) {
      T cm[M], lo[NFP], up[NFP];
      double c0;
      load_var(avg, hi, I.ncell, g.c, g.v, cm, c0);
      traces<d>(cm, lo, up);
#pragma unroll
      for (int b = 0; b < NFP; ++b) {
        if constexpr (DG) {
          lds(sm)[fidx<d>(g.v, b, 1, fi_lo)] = lo[b];
          lds(sm)[fidx<d>(g.v, b, 0, fi_up)] = up[b];
        } else {
          lds(sm)[cidx(g.v, b, 0, g.lane)] = lo[b];
          lds(sm)[cidx(g.v, b, 1, g.lane)] = up[b];
        }
      }
    }
    if constexpr (DG) {
      if (hv) {
        T lo[NFP], up[NFP];
        traces<d>(hm, lo, up);
        // the halo cell below the tile shows its upper trace, the one above its lower trace
#pragma unroll
        for (int b = 0; b < NFP; ++b) lds(sm)[fidx<d>(g.v, b, hside, hfi)] = hside ? lo[b] : up[b];
      }
      // time-dependent Dirichlet data of a mesh side the tile touches: the
      // exterior values go into the ghost side of its boundary slots (side 0
      // below the mesh, side 1 above it), where the flux pass reads them.
      // Boundary face index: tangential cell coordinates, lower direction
      // fastest.  Kept out of the flux pass: there the call would hold its
      // registers across the whole pass.
      if (bd.side) {
#pragma unroll 1
        for (int up = 0; up < 2; ++up) {
          const int f = 2 * d + up;
          const bool edge = up ? (g.o[d] + g.A[d] == I.n[d]) : (g.o[d] == 0);
          if (!edge || I.bc[f] != CRKDG_BC_DIRICHLET || !(I.bdyn & (1u << f))) continue;
          const int p = up ? g.A[d] : 0;
#pragma unroll 1
          for (int j = g.lane; j < T1 * T2 * NFP; j += 64) {
            const int b = j % NFP, qq = j / NFP;
            const int h1 = qq % T1, h2 = qq / T1;
            if (h1 >= g.A[oax1(d)] || (D == 3 && h2 >= g.A[oax2(d)])) continue;
            int64_t fc = g.o[oax1(d)] + h1;
            if constexpr (D == 3) fc += static_cast<int64_t>(I.n[oax1(d)]) * (g.o[oax2(d)] + h2);
            lds(sm)[fidx<d>(g.v, b, up, slot<d>(p, h1, h2))] = T(boundary_value(bd, f, fc, NFP, V, b, g.v));
          }
        }
      }
    }
    __syncthreads();
    if constexpr (DG) {
      // (2) Lax--Friedrichs flux along +e_d at every face point.  The NFP
      // points of a face sit in NFP consecutive lanes (GPW faces per
      // wavefront), so the face alpha -- the largest wave speed over its
      // points and both traces -- is a maximum across those lanes, and the
      // flux is formed in the same pass from the same values.
      constexpr int GPW = 64 / NFP;
      constexpr int PASSES = (NFD + V * GPW - 1) / (V * GPW);
      const int grp = g.lane / NFP;
      const int b = g.lane - grp * NFP;
      const int base = grp * NFP;
#pragma unroll 1
      for (int pass = 0; pass < PASSES; ++pass) {
        const int fi = (pass * V + g.v) * GPW + grp;
        T uL[V], uR[V];
        const bool use = grp < GPW && fi < NFD && face_pair<d>(g, I, fi, b, uL, uR, sm, bd);
        if (!use)
#pragma unroll
          for (int w = 0; w < V; ++w) uL[w] = uR[w] = T(1);
        const auto aL = P::aux(uL, I);
        const auto aR = P::aux(uR, I);
        const T sp = fmax(P::speed(uL, aL, d, I), P::speed(uR, aR, d, I));
        T ab = (use && sp == sp) ? sp : T(0);
        if (I.alpha_mode != CRKDG_ALPHA_GLOBAL) {
          // maximum over the group's lanes by rotations within the group
          T m = ab;
#pragma unroll
          for (int st = 1; st < NFP; st *= 2) {
            const int src = base + ((b + st) % NFP);
            m = fmax(m, __shfl(m, src, 64));
          }
          // per point: the point's own speed, an undefined one (zero
          // density) the face alpha; per face: the face alpha
          ab = (I.alpha_mode == CRKDG_ALPHA_POINT) ? fmin(sp, m) : m;
        } else {
          ab = static_cast<T>(ag);
        }
        if (use) {
#pragma clang fp contract(off)
          T fL[V], fR[V];
          P::flux(uL, aL, d, I, fL);
          P::flux(uR, aR, d, I, fR);
          const T ha = T(0.5) * ab;
#pragma unroll
          for (int w = 0; w < V; ++w)
            lds(sm)[fidx<d>(w, b, 0, fi)] = fma(-ha, uR[w] - uL[w], T(0.5) * (fL[w] + fR[w]));
        }
      }
    } else {
      // (3) interior flux f_d(u) of each cell's own traces, in place
#pragma unroll 1
      for (int it = threadIdx.x; it < 2 * NFP * 64; it += NT) {
        const int cl = it & 63;
        const int sb = it >> 6;
        const int side = sb & 1, b = sb >> 1;     // side 0: the cell's lower face
        const int cx = cl % TX, cy = (cl / TX) % TY, cz = cl / (TX * TY);
        const int lc[3] = {cx, cy, cz};
        if (lc[0] >= g.A[0] || lc[1] >= g.A[1] || lc[2] >= g.A[2]) continue;
        T u[V];
#pragma unroll
        for (int w = 0; w < V; ++w) u[w] = lds(sm)[cidx(w, b, side, cl)];
        T fu[V];
        P::flux(u, P::aux(u, I), d, I, fu);
#pragma unroll
        for (int w = 0; w < V; ++w) lds(sm)[cidx(w, b, side, cl)] = fu[w];
      }
    }
    __syncthreads();
    // (4) face residuals: r -= scale/dx_d * (2a+1) side^(a+1) (W x W) fn
    if (g.active) {
      T flo[NFP], fup[NFP];
#pragma unroll
      for (int b = 0; b < NFP; ++b) {
        // F: the face's flux (side 0 of the slot); G: the cell's own trace flux
        flo[b] = DG ? lds(sm)[fidx<d>(g.v, b, 0, fi_lo)] : lds(sm)[cidx(g.v, b, 0, g.lane)];
        fup[b] = DG ? lds(sm)[fidx<d>(g.v, b, 0, fi_up)] : lds(sm)[cidx(g.v, b, 1, g.lane)];
      }
      const double sc = scale * I.rdx[d];
      // mode 0 in FP64, face by face in point order (the same sum in both cells)
      double slo = 0.0, sup = 0.0;
#pragma unroll
      for (int b = 0; b < NFP; ++b) {
        const double wb = fw.w[b];
        slo = fma(wb, static_cast<double>(flo[b]), slo);
        sup = fma(wb, static_cast<double>(fup[b]), sup);
      }
      r0 = r0 - sc * sup;
      r0 = r0 + sc * slo;
      T hlo[NFP], hup[NFP];
      auto pw = [](const T (&x)[N], T (&y)[N]) { O1::proj(x, y); };
      if constexpr (D == 2) {
        O1::proj(flo, hlo);
        O1::proj(fup, hup);
      } else {
        T t[NFP];
        along<N, 2, 0>(flo, t, pw);
        along<N, 2, 1>(t, hlo, pw);
        along<N, 2, 0>(fup, t, pw);
        along<N, 2, 1>(t, hup, pw);
      }
      const T sct = T(sc);
      constexpr int sdd = ipow(N, d);
      constexpr int s1 = ipow(N, oax1(d));
      constexpr int s2 = (D == 3) ? ipow(N, oax2(d)) : 0;
#pragma unroll
      for (int t = 0; t < NFP; ++t) {
        const T Sx = hup[t] + hlo[t];
        const T Dx = hup[t] - hlo[t];
        const int base = (t % N) * s1 + (t / N) * s2;
#pragma unroll
        for (int a = 0; a < N; ++a) {
          const int m = base + a * sdd;
          if (!live(m)) continue;
          const T k = T(-(2.0 * a + 1.0)) * sct;
          r[m] = fma(k, (a & 1) ? Sx : Dx, r[m]);
        }
      }
    }
    __syncthreads();
  }

  // the two traces of face point b of slot fi (lower cell, upper cell), with
  // ghosts on non-periodic mesh sides; false when the slot is not used
  template <int d>
  __device__ __forceinline__ static bool face_pair(const Geo& g, const InstDev& I, int fi, int b, T (&uL)[V],
                                                   T (&uR)[V], Smem& sm, const BData& bd) {
    constexpr int T1 = tsz1(d);
    const int p = fi % (tdim(d) + 1);
    const int qq = fi / (tdim(d) + 1);
    const int q1 = qq % T1, q2 = qq / T1;
    if (p > g.A[d] || q1 >= g.A[oax1(d)] || (D == 3 && q2 >= g.A[oax2(d)])) return false;
    const bool ghost_lo = (p == 0) && (g.o[d] == 0) && I.bc[2 * d] != CRKDG_BC_PERIODIC;
    const bool ghost_up = (p == g.A[d]) && (g.o[d] + p == I.n[d]) && I.bc[2 * d + 1] != CRKDG_BC_PERIODIC;
    // both sides read unconditionally (a ghost side's slot holds stale
    // words, overwritten below, or the side's time-dependent data)
#pragma unroll
    for (int w = 0; w < V; ++w) {
      uL[w] = lds(sm)[fidx<d>(w, b, 0, fi)];
      uR[w] = lds(sm)[fidx<d>(w, b, 1, fi)];
    }
    // a side with time-dependent data has its exterior values in the slot
    // already (written with the halos)
    const bool dyn_lo = bd.side && (I.bdyn & (1u << (2 * d)));
    const bool dyn_up = bd.side && (I.bdyn & (1u << (2 * d + 1)));
    if (ghost_lo && !dyn_lo) ghost(2 * d, I, uR, uL);
    if (ghost_up && !dyn_up) ghost(2 * d + 1, I, uL, uR);
    return true;
  }

  // exterior trace on the non-periodic side f (outflow, reflective wall,
  // Dirichlet / inflow): the same readings as Cell::ghost
  __device__ __forceinline__ static void ghost(int f, const InstDev& I, const T* ui, T* ue) {
    const int kind = I.bc[f];
#pragma unroll
    for (int w = 0; w < V; ++w) {
      T x = ui[w];
      if (kind == CRKDG_BC_REFLECT && w == 1 + f / 2) x = -x;
      if (kind == CRKDG_BC_DIRICHLET) x = T(I.bcs[f][w]);
      ue[w] = x;
    }
  }

  // the operator (F with DG, else G) of the state held in cm / memory,
  // accumulated into r, r0 with `scale`
  template <bool DG>
  __device__ __forceinline__ static void op(const Geo& g, const double* avg, const T* hi, const InstDev& I,
                                            double scale, double ag, T (&r)[M], double& r0, Smem& sm,
                                            const BData& bd) {
    volume(g, avg, hi, I, scale, r, sm);
    faces<0, DG>(g, avg, hi, I, scale, ag, r, r0, sm, bd);
    faces<1, DG>(g, avg, hi, I, scale, ag, r, r0, sm, bd);
    if constexpr (D == 3) faces<2, DG>(g, avg, hi, I, scale, ag, r, r0, sm, bd);
  }

  // ---- S_K values of one family (Lobatto nodes along fam, Gauss nodes
  // along the others) of the output modes, into LDS: the Lobatto nodes
  // L0 .. L0 + NLC - 1 of the family
  template <int fam, int L0>
  __device__ __forceinline__ static void sk_family(const Geo& g, const T (&oc)[M], Smem& sm) {
    auto ev = [](const T (&x)[N], T (&y)[N]) { O1::eval(x, y); };
    // Gauss nodes along the other directions first (N^D values), then the
    // Lobatto nodes along fam: point p = (Lobatto index - L0) + NLC *
    // (tangential point b, b over the other directions ascending)
    T t[M], u[M];
    if constexpr (D == 2) {
      along<N, 2, 1 - fam>(oc, t, ev);
#pragma unroll
      for (int b = 0; b < N; ++b) {
        T line[N], lv[NL];
#pragma unroll
        for (int a = 0; a < N; ++a) line[a] = t[fam == 0 ? a + N * b : b + N * a];
        O1::eval_l(line, lv);
#pragma unroll
        for (int l = 0; l < NLC; ++l) lds(sm)[(g.v * NPC + l + NLC * b) * 64 + g.lane] = lv[L0 + l];
      }
      (void)u;
    } else {
      along<N, 3, oax1(fam)>(oc, t, ev);
      along<N, 3, oax2(fam)>(t, u, ev);
      constexpr int sf = ipow(N, fam), s1 = ipow(N, oax1(fam)), s2 = ipow(N, oax2(fam));
#pragma unroll
      for (int b = 0; b < N * N; ++b) {
        T line[N], lv[NL];
#pragma unroll
        for (int a = 0; a < N; ++a) line[a] = u[(b % N) * s1 + (b / N) * s2 + a * sf];
        O1::eval_l(line, lv);
#pragma unroll
        for (int l = 0; l < NLC; ++l) lds(sm)[(g.v * NPC + l + NLC * b) * 64 + g.lane] = lv[L0 + l];
      }
    }
  }

  // ---- a stage: inner (KIND 0: G, KIND 1: F) or final (KIND 2)
  // r0, r += sum_p kap_p S_p for this thread's variable and cell
  __device__ __forceinline__ static void add_source(const KArgs& a, const BlockItem& bi, const InstDev& I,
                                                    const Geo& g, T (&r)[M], double& r0) {
    const double* kap = source_weights(a, bi.inst);
    const int64_t nc = I.ncell;
#pragma unroll 1
    for (int p = 0; p < a.src.n; ++p) {
      r0 = fma(kap[p], ld(a.src.avg[p] + I.avg_off + g.v * nc, g.c), r0);
      const T kt = T(kap[p]);
      const T* h = static_cast<const T*>(a.src.hi[p]) + I.hi_off + static_cast<int64_t>(g.v) * MH * nc;
      static_for<M - 1>([&](auto MM) {
        constexpr int m = decltype(MM)::value + 1;
        if constexpr (live(m)) r[m] = fma(kt, ld(h + (smap.s[m] - 1) * nc, g.c), r[m]);
      });
    }
  }

  // BDY: the kernel form that reads time-dependent boundary data (launched
  // for meshes that have some; without it the exterior states are the
  // constant ones and no boundary-data code is compiled in)
  template <int KIND, bool BDY>
  __device__ __forceinline__ static void run(const KArgs& a, const BlockItem& bi, const InstDev& I, crkdg_ctl* ctl,
                                             Smem& sm) {
    const Geo g = geo(bi, I, threadIdx.x);
    const int s = I.stages;
    // the controller's fields this kernel reads, none of which it writes:
    // scalar loads (constant address space)
    using CC = const __attribute__((address_space(4))) crkdg_ctl;
    const CC* cc = (const CC*)ctl;
    const int cur = a.slots.rotate ? cc->cur : 0;
    const int nsl = s + 1;
    const int64_t nc = I.ncell;
    const double dt = cc->dt;
    double ag = 0.0;
#pragma unroll
    for (int d = 0; d < D; ++d) ag = fmax(ag, cc->a0[d]);   // the global alpha (Sec. 2.1 a0)
    T r[M];
#pragma unroll
    for (int m = 0; m < M; ++m) r[m] = T(0);
    double r0 = 0.0;
    // the stage's source terms sum_p kap_p S_p: in the final stage they seed
    // the accumulator (before the four F, while nothing else holds
    // registers), in an inner stage they join it after the operator (a
    // seeded accumulator stays live through the operator and spills there)
    if constexpr (KIND == 2) {
      if (a.src.n > 0 && g.active) add_source(a, bi, I, g, r, r0);
    }
    int sl_out;
    if constexpr (KIND == 2) {
      sl_out = (cur + s) % nsl;
      // unrolled over the stages: as a loop, values hoisted out of it hold
      // registers through every F and halve the workgroups per CU
      static_for<4>([&](auto JJ) {
        constexpr int j = decltype(JJ)::value + 1;
        if (j > s || a.b[j - 1] == 0.0) return;
        const int sl = (cur + j - 1) % nsl;
        const double* j_avg = sel_avg(a.slots, sl) + I.avg_off;
        const T* j_hi = hi_ptr<T>(sel_hi(a.slots, sl), I.hi_off);
        // the thread geometry and everything addressed by it recomputed per
        // stage rather than kept live from one F to the next
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const Geo gj = geo(bi, I, tid);
        op<true>(gj, j_avg, j_hi, I, dt * a.b[j - 1], ag, r, r0, sm,
                 BDY ? bdata(a, bi.inst, j - 1) : BData{nullptr, nullptr});
      });
    } else {
      const int sl_in = (cur + a.stage - 2) % nsl;
      sl_out = (cur + a.stage - 1) % nsl;
      const double* in_avg = sel_avg(a.slots, sl_in) + I.avg_off;
      const T* in_hi = hi_ptr<T>(sel_hi(a.slots, sl_in), I.hi_off);
      op<KIND == 1>(g, in_avg, in_hi, I, dt * a.a, ag, r, r0, sm,
                    (BDY && KIND == 1) ? bdata(a, bi.inst, a.stage - 2) : BData{nullptr, nullptr});
    }
    if constexpr (KIND != 2) {
      if (a.src.n > 0 && g.active) add_source(a, bi, I, g, r, r0);
    }
    // out = u~^n + r
    const double* b_avg = sel_avg(a.slots, cur) + I.avg_off;
    const T* b_hi = hi_ptr<T>(sel_hi(a.slots, cur), I.hi_off);
    T oc[M];
    double o0 = 0.0;
    if (g.active) {
      load_var(b_avg, b_hi, nc, g.c, g.v, oc, o0);
      o0 = o0 + r0;
      oc[0] = T(o0);
#pragma unroll
      for (int m = 1; m < M; ++m) oc[m] = live(m) ? oc[m] + r[m] : T(0);
    } else {
#pragma unroll
      for (int m = 0; m < M; ++m) oc[m] = T(0);
      o0 = 1.0;
    }
    finish<KIND == 2>(a, bi, I, ctl, g, oc, o0, sl_out, sm);
  }

  // checks, the one-pass S_K test (with wave speeds on the final stage),
  // store or queue, flags
  template <bool A0>
  __device__ __forceinline__ static void finish(const KArgs& a, const BlockItem& bi, const InstDev& I,
                                                crkdg_ctl* ctl, const Geo& g, const T (&oc)[M], double o0,
                                                int sl_out, Smem& sm) {
    // per-variable magnitudes for the rounding bound of the FP32 test and
    // the interval test
    {
      T rs = T(0);
#pragma unroll
      for (int m = 1; m < M; ++m)
        if (live(m)) rs += fabs(oc[m]);
      sm.avg[g.v][g.lane] = o0;
      sm.rsum[g.v][g.lane] = rs;
    }
    if (g.v == 0) {
      sm.fail[g.lane] = 0u;
#pragma unroll
      for (int d = 0; d < D; ++d) sm.spd[d][g.lane] = 0;
    }
    if (threadIdx.x == 0) sm.flag = 0;
    __syncthreads();
    typename CellT::State cs;   // the cell's averages (modes unused here)
#pragma unroll
    for (int w = 0; w < V; ++w) cs.ub[w] = sm.avg[w][g.lane];
    const bool bad = g.active && !CellT::average_ok(cs, I);
    const bool nonfin = g.active && !CellT::average_finite(cs);
    // cheap interval test (every |phi_m| <= 1): a pass proves the limiter is
    // the identity; without wave speeds to take, a tile that passes skips S_K
    bool ipass = !g.active || !I.limiter;
    if (!ipass) ipass = interval_pass(cs, sm, g.lane, I);
    if (!A0 && !ipass) sm.flag = 1;   // benign race: every writer stores 1
    __syncthreads();
    bool ok = true;
    T am[D];
#pragma unroll
    for (int d = 0; d < D; ++d) am[d] = T(0);
    if (A0 || sm.flag) {
      // thresholds of the FP32 test of this cell (mixed): rigorous rounding
      // bound err_v = 2 (M + 1) 2^-24 (|ubar_v| + sum |c_vm|); each value
      // takes at most 3 D + 1 roundings of partial sums bounded by that sum
      T ub[V], bnd[V], err[V];
      (void)ub;
#pragma unroll
      for (int w = 0; w < V; ++w) {
        ub[w] = T(cs.ub[w]);
        bnd[w] = fabs(ub[w]) + sm.rsum[w][g.lane];
        err[w] = MIXED ? T(2.0 * (M + 1) * 0x1p-24) * bnd[w] : T(0);
      }
      T thr_rho = T(I.eps) + T(2) * err[0];
      T marg = T(0);
      if constexpr (SYS == SYS_EULER && MIXED) {
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
      auto check = [&](const T* u) {
        if constexpr (SYS == SYS_EULER) {
          T ke = T(0);
#pragma unroll
          for (int j = 0; j < D; ++j) ke = fma(u[1 + j], u[1 + j], ke);
          const T q = fma(u[D + 1], u[0], T(-0.5) * ke);
          T rhs = fma(T(I.eps), u[0], marg);
          if constexpr (MIXED) rhs *= T(1 + 0x1p-20);
          ok = ok && (u[0] >= thr_rho) && (q >= rhs);
        } else {
          const double uu = static_cast<double>(u[0]);
          const double e = static_cast<double>(err[0]);
          ok = ok && (uu - e >= I.blo) && (uu + e <= I.bhi);
        }
        if constexpr (A0) {
          const auto ax = P::aux(u, I);
#pragma unroll
          for (int d = 0; d < D; ++d) am[d] = fmax(am[d], P::speed(u, ax, d, I));
        }
      };
      static_for<D * (NL / NLC)>([&](auto FL) {
        constexpr int fam = decltype(FL)::value / (NL / NLC);
        constexpr int l0 = (decltype(FL)::value % (NL / NLC)) * NLC;
        sk_family<fam, l0>(g, oc, sm);
        __syncthreads();
        if (g.active) {
          for (int p = g.v; p < NPC; p += V) {
            T u[V];
#pragma unroll
            for (int w = 0; w < V; ++w) u[w] = lds(sm)[(w * NPC + p) * 64 + g.lane];
            check(u);
          }
        }
        __syncthreads();
      });
    }
    if (!ok) atomicOr(&sm.fail[g.lane], 1u);
    if constexpr (A0) {
#pragma unroll
      for (int d = 0; d < D; ++d) atomicMax(&sm.spd[d][g.lane], bits_of(am[d]));
    }
    __syncthreads();
    const bool pass = (sm.fail[g.lane] == 0u) || ipass;
    const bool queue = g.active && !pass && I.limiter;
    double* o_avg = sel_avg(a.slots, sl_out) + I.avg_off;
    T* o_hi = hi_ptr<T>(sel_hi(a.slots, sl_out), I.hi_off);
    const int64_t nc = I.ncell;
    if (g.active && !queue) {
      st(o_avg + g.v * nc, g.c, o0);
      T* h = o_hi + static_cast<int64_t>(g.v) * MH * nc;
      static_for<M - 1>([&](auto MM) {
        constexpr int m = decltype(MM)::value + 1;
        if constexpr (live(m)) st(h + (smap.s[m] - 1) * nc, g.c, oc[m]);
      });
    }
    // queued cells: one record each, limited by the queue kernel
    if (g.v == 0 && queue) sm.qidx[g.lane] = atomicAdd(a.qcount, 1u);
    __syncthreads();
    if (queue) {
      const unsigned idx = sm.qidx[g.lane];
      if (idx < a.qcap) {
        Rec* rec = static_cast<Rec*>(a.queue) + idx;
        if (g.v == 0) {
          rec->inst = bi.inst;
          rec->cell = static_cast<int32_t>(g.c);
        }
        rec->ub[g.v] = o0;
        static_for<M - 1>([&](auto MM) {
          constexpr int m = decltype(MM)::value + 1;
          if constexpr (live(m)) rec->ch[g.v][smap.s[m] - 1] = oc[m];
        });
      }
    }
    if (g.v == 0) {
      raise_flag(&ctl->flags, bad, CRKDG_F_AVERAGE);
      raise_flag(&ctl->flags, nonfin, CRKDG_F_NONFINITE);
      if constexpr (A0) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
          const T mx = of_bits(sm.spd[d][g.lane]);
          double sp = (g.active && !queue && !bad && !nonfin) ? static_cast<double>(mx) : 0.0;
          const double wm = wave_max(sp);
          if (g.lane == 0 && wm > 0.0)
            atomicMax(reinterpret_cast<unsigned long long*>(&ctl->a0_next[d]),
                      static_cast<unsigned long long>(__double_as_longlong(wm)));
        }
      }
    }
  }

  // the interval test of Cell::interval_pass from the per-variable sums
  __device__ __forceinline__ static bool interval_pass(const typename CellT::State& cs, const Smem& sm, int lane,
                                                       const InstDev& I) {
    double R[V];
#pragma unroll
    for (int w = 0; w < V; ++w)
      R[w] = static_cast<double>(sm.rsum[w][lane]) * (1.0 + (MH + 2) * (MIXED ? 0x1p-23 : 0x1p-52));
    if constexpr (SYS == SYS_EULER) {
      const double rlo = cs.ub[0] - R[0];
      const double elo = cs.ub[D + 1] - R[D + 1];
      if (!(rlo >= I.eps) || !(elo > 0.0)) return false;
      double mm = 0.0;
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const double mh = fabs(cs.ub[1 + j]) + R[1 + j];
        mm = fma(mh, mh, mm);
      }
      const double qlo = fma(elo, rlo, -0.5 * mm);
      return qlo * (1.0 - 0x1p-40) >= I.eps * (cs.ub[0] + R[0]);
    } else {
      return (cs.ub[0] - R[0] >= I.blo) && (cs.ub[0] + R[0] <= I.bhi);
    }
  }
};

// Wavefronts per SIMD the register allocation of a stage kernel aims at
// (measured on the 3D Q^2 Euler workload): the mixed final stage at 4 (128
// VGPRs, a few spilled: three workgroups per CU) runs 20% faster than
// unconstrained, the mixed inner stages at 5 (96 VGPRs: four workgroups per
// CU) 13% faster than at 4; the inner stage with F (standard RKDG) needs the
// final stage's budget (at 96 VGPRs its Lax--Friedrichs pass spills
// kilobytes per lane); the FP64 kernels stay unconstrained (their LDS limits
// them to two workgroups per CU).
template <typename T, int KIND>
constexpr int coop_waves_per_eu() {
  return (sizeof(T) == 4) ? (KIND == 0 ? 5 : 4) : 1;
}

// One workgroup (one wavefront per variable) per tile of the stage map.
// KIND 0: inner stage with G; 1: inner stage with F (standard RKDG); 2: final
// stage.  BDY: with time-dependent boundary data (KIND 1 and 2).
template <int D, int K, int SP, int SYS, typename T, int TX, int TY, int TZ, int KIND, bool BDY = false>
__global__ __launch_bounds__((64 * Phys<D, SYS>::V)) __attribute__((amdgpu_waves_per_eu(
    coop_waves_per_eu<T, KIND>()))) void k_coop_stage(KArgs a) {
  using C = Coop<D, K, SP, SYS, T, TX, TY, TZ, KIND == 0 ? 1 : 0>;
  __shared__ typename C::Smem sm;
  if (static_cast<int>(blockIdx.x) >= a.n_items) return;
  // the tile, the instance's constants and the controller's state are
  // uniform and read-only here: scalar loads (constant address space)
  using CB = const __attribute__((address_space(4))) BlockItem;
  using CI = const __attribute__((address_space(4))) InstDev;
  using CC = const __attribute__((address_space(4))) crkdg_ctl;
  const CB* pb = (const CB*)a.bmap + blockIdx.x;
  BlockItem bi;
  bi.inst = pb->inst;
  bi.lblock = pb->lblock;
  bi.x0 = pb->x0;
  bi.y0 = pb->y0;
  bi.z = pb->z;
  bi.pad = 0;
  if (bi.inst < 0) return;  // padding entry of the XCD-ordered block map
  // the instance's constants, read where used through the constant address
  // space (scalar loads)
  const InstDev& I = *(const InstDev*)((const CI*)a.inst + bi.inst);
  crkdg_ctl* ctl = a.ctl + bi.inst;
  const CC* cc = (const CC*)ctl;
  if (cc->status != 0 || cc->accepted >= cc->goal) return;   // instance idle
  C::template run<KIND, BDY>(a, bi, I, ctl, sm);
}

}  // namespace crkdg
