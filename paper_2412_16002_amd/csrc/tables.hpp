// Compile-time quadrature and modal-basis tables for one DG space.
//
// Everything here is evaluated by the C++ compiler (constexpr) so that, after
// the stage kernels unroll their point and mode loops, every table entry is an
// immediate operand and entries equal to 0 or +-1 fold away.
//
//  * Gauss--Legendre rules of k+1 points per direction (closed forms), used
//    for volume integrals and, with weights normalised to sum one, for face
//    integrals (Sec. 2.2.1, Prop. 2.1).
//  * Gauss--Lobatto rules of N = 2 (k = 1) or 3 (k = 2, 3) points; the
//    limiter set S_K is the union over directions d of the tensor products
//    with Lobatto points in direction d and Gauss points in the others
//    (Sec. 2.2.1, Prop. 2.2 and Fig. 1), duplicates removed.
//  * Legendre products phi_m = prod_j P_{e_j}, P_n(1) = 1; inverse reference
//    mass prod_j (2 e_j + 1) (the basis is L2-orthogonal).
#pragma once

#include <cstdint>

namespace crkdg {

constexpr int SP_Q = 0;
constexpr int SP_P = 1;

constexpr int ipow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// Legendre polynomial P_n(x) by Bonnet's recurrence
constexpr double leg(int n, double x) {
  if (n == 0) return 1.0;
  double p0 = 1.0, p1 = x;
  for (int j = 1; j < n; ++j) {
    const double p2 = ((2.0 * j + 1.0) * x * p1 - j * p0) / (j + 1.0);
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

// P_n'(x) = sum over j = n-1, n-3, ... >= 0 of (2j+1) P_j(x)
constexpr double dleg(int n, double x) {
  double s = 0.0;
  for (int j = n - 1; j >= 0; j -= 2) s += (2.0 * j + 1.0) * leg(j, x);
  return s;
}

// Gauss--Legendre rules, closed forms (nodes ascending, weights sum 2)
template <int N> struct Gauss;
template <> struct Gauss<2> {
  static constexpr double x[2] = {-0.57735026918962576451, 0.57735026918962576451};
  static constexpr double w[2] = {1.0, 1.0};
};
template <> struct Gauss<3> {
  static constexpr double x[3] = {-0.77459666924148337704, 0.0, 0.77459666924148337704};
  static constexpr double w[3] = {5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0};
};
template <> struct Gauss<4> {
  static constexpr double a = 0.33998104358485626480;  // sqrt(3/7 - 2/7 sqrt(6/5))
  static constexpr double b = 0.86113631159405257522;  // sqrt(3/7 + 2/7 sqrt(6/5))
  static constexpr double x[4] = {-b, -a, a, b};
  static constexpr double wa = 0.65214515486254614263;  // (18 + sqrt 30) / 36
  static constexpr double wb = 0.34785484513745385737;  // (18 - sqrt 30) / 36
  static constexpr double w[4] = {wb, wa, wa, wb};
};

template <int N> struct Lobatto;
template <> struct Lobatto<2> {
  static constexpr double x[2] = {-1.0, 1.0};
};
template <> struct Lobatto<3> {
  static constexpr double x[3] = {-1.0, 0.0, 1.0};
};

// ---------------------------------------------------------------------------
// One DG space: dimension D, degree K, tensor (Q) or total-degree (P) space.
// ---------------------------------------------------------------------------
template <int D, int K, int SP> struct Space {
  static constexpr int NG = K + 1;                   // Gauss points per direction
  static constexpr int NQ = ipow(NG, D);             // volume points
  static constexpr bool TENSOR = (D == 1 || SP == SP_Q);
  static constexpr int M = TENSOR ? ipow(K + 1, D)
                                  : (D == 2 ? (K + 1) * (K + 2) / 2 : (K + 1) * (K + 2) * (K + 3) / 6);
  static constexpr int NF = 2 * D;                   // faces
  static constexpr int NFP = (D == 1) ? 1 : ipow(NG, D - 1);  // points per face
  static constexpr int NL = (K == 1) ? 2 : 3;        // Lobatto points in S_K
  static constexpr int NS_RAW = D * ipow(NG, D - 1) * NL;
  static constexpr int TM = ipow(K + 1, D - 1);      // tangential modes of a face

  static constexpr double gx(int i) { return Gauss<NG>::x[i]; }
  static constexpr double gw(int i) { return Gauss<NG>::w[i]; }
  static constexpr double lx(int i) { return Lobatto<NL>::x[i]; }

  struct Modes {
    int e[M][3];
    constexpr Modes() : e{} {
      int m = 0;
      if (TENSOR) {
        for (int c = 0; c < ipow(K + 1, D); ++c) {
          int r = c;
          for (int j = 0; j < 3; ++j) {
            e[m][j] = (j < D) ? r % (K + 1) : 0;
            if (j < D) r /= (K + 1);
          }
          ++m;
        }
      } else {
        // total degree, then decreasing e0, then decreasing e1
        for (int tot = 0; tot <= K; ++tot)
          for (int e0 = tot; e0 >= 0; --e0) {
            if (D == 2) {
              e[m][0] = e0; e[m][1] = tot - e0; e[m][2] = 0; ++m;
            } else {
              for (int e1 = tot - e0; e1 >= 0; --e1) {
                e[m][0] = e0; e[m][1] = e1; e[m][2] = tot - e0 - e1; ++m;
              }
            }
          }
      }
    }
  };
  static constexpr Modes modes{};

  static constexpr double phi(int m, const double* x) {
    double v = 1.0;
    for (int j = 0; j < D; ++j) v *= leg(modes.e[m][j], x[j]);
    return v;
  }
  static constexpr double dphi(int m, int d, const double* x) {
    double v = 1.0;
    for (int j = 0; j < D; ++j) v *= (j == d) ? dleg(modes.e[m][j], x[j]) : leg(modes.e[m][j], x[j]);
    return v;
  }
  // inverse reference mass of mode m times 2^D / |[-1,1]^D| factor: prod (2e+1)
  static constexpr double pfac(int m) {
    double v = 1.0;
    for (int j = 0; j < D; ++j) v *= 2.0 * modes.e[m][j] + 1.0;
    return v;
  }

  struct Tables {
    double xq[NQ][3];       // volume points (first coordinate fastest)
    double wq[NQ];          // product weights / 2^D (sum 1)
    double phi_v[NQ][M];
    double cvol[NQ][M][D];  // pfac * wq * dphi: volume residual coefficients
    double xf[NF][NFP][3];  // face f = 2 d + (side > 0): points
    double phi_f[NF][NFP][M];
    double cface[NF][NFP][M];  // pfac * side * wb * phi: face residual coefficients
    double wb[NFP];         // face weights (sum 1)
    double ftan[NFP][TM];   // tangential Legendre products at the face points
    double xs[NS_RAW][3];   // S_K points (first NS entries valid)
    double phi_s[NS_RAW][M];
    int ns;
    constexpr Tables()
        : xq{}, wq{}, phi_v{}, cvol{}, xf{}, phi_f{}, cface{}, wb{}, ftan{}, xs{}, phi_s{}, ns(0) {
      for (int q = 0; q < NQ; ++q) {
        int r = q;
        double w = 1.0;
        for (int j = 0; j < 3; ++j) {
          if (j < D) {
            xq[q][j] = gx(r % NG);
            w *= 0.5 * gw(r % NG);
            r /= NG;
          } else {
            xq[q][j] = 0.0;
          }
        }
        wq[q] = w;
        for (int m = 0; m < M; ++m) {
          phi_v[q][m] = phi(m, xq[q]);
          for (int d = 0; d < D; ++d) cvol[q][m][d] = pfac(m) * w * dphi(m, d, xq[q]);
        }
      }
      for (int b = 0; b < NFP; ++b) {
        int r = b;
        double w = 1.0;
        for (int j = 0; j < D - 1; ++j) {
          w *= 0.5 * gw(r % NG);
          r /= NG;
        }
        wb[b] = w;
        // face point b and tangential mode t: indices over the directions
        // other than the normal, lower direction fastest
        for (int t = 0; t < TM; ++t) {
          double v = 1.0;
          int rb = b, rt = t;
          for (int j = 0; j < D - 1; ++j) {
            v *= leg(rt % (K + 1), gx(rb % NG));
            rb /= NG;
            rt /= (K + 1);
          }
          ftan[b][t] = v;
        }
      }
      for (int f = 0; f < NF; ++f) {
        const int d = f / 2;
        const double side = (f % 2) ? 1.0 : -1.0;
        for (int b = 0; b < NFP; ++b) {
          int r = b;
          int t = 0;
          for (int j = 0; j < 3; ++j) {
            if (j == d) {
              xf[f][b][j] = side;
            } else if (j < D) {
              xf[f][b][j] = gx(r % NG);
              r /= NG;
              ++t;
            } else {
              xf[f][b][j] = 0.0;
            }
          }
          for (int m = 0; m < M; ++m) {
            phi_f[f][b][m] = phi(m, xf[f][b]);
            cface[f][b][m] = pfac(m) * side * wb[b] * phi_f[f][b][m];
          }
        }
      }
      // S_K: union over directions d of (Lobatto in d) x (Gauss elsewhere)
      int n = 0;
      for (int d = 0; d < D; ++d) {
        for (int c = 0; c < ipow(NG, D - 1) * NL; ++c) {
          int r = c;
          double p[3] = {0.0, 0.0, 0.0};
          for (int j = 0; j < D; ++j) {
            if (j == d) {
              p[j] = lx(r % NL);
              r /= NL;
            } else {
              p[j] = gx(r % NG);
              r /= NG;
            }
          }
          bool dup = false;
          for (int o = 0; o < n; ++o)
            if (xs[o][0] == p[0] && xs[o][1] == p[1] && xs[o][2] == p[2]) dup = true;
          if (!dup) {
            for (int j = 0; j < 3; ++j) xs[n][j] = p[j];
            for (int m = 0; m < M; ++m) phi_s[n][m] = phi(m, p);
            ++n;
          }
        }
      }
      ns = n;
    }
  };
  static constexpr Tables tab{};
  static constexpr int NS = tab.ns;
};

}  // namespace crkdg
