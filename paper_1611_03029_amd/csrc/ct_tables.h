// Compile-time one-dimensional rules and even-odd matrices for the operator kernels.
//
// The kernels apply four 1D matrices along every line of a cell (Sec. 3: sum
// factorization; Sec. 2.1: GLL-Lagrange basis; k+1 Gauss points):
//   M, K : reference [0,1] mass and stiffness of the GLL basis (exact Gauss integrals),
//   S    : GLL basis at the Gauss points,
//   D    : collocation derivative of the Gauss-point Lagrange basis at the Gauss points.
// Computing them here as constexpr values makes every coefficient an immediate in the
// instruction stream, so the compiler rematerializes coefficients instead of holding them
// in scalar registers for the whole kernel.  The host library computes the same rules
// (tables.hip) for the setup kernels and for the oracle-independent consistency check.
#pragma once

#include "mfl_internal.h"

namespace mfl {
namespace ct {

constexpr double kPi = 3.14159265358979323846264338327950288;

// cos by its Taylor series (|x| <= pi: 40 terms are far past double precision)
constexpr double cos_series(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 40; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}

constexpr double abs_(double x) { return x < 0 ? -x : x; }

// Legendre P_m(x) and P_m'(x)
struct LegVal {
  double P, dP;
};
constexpr LegVal legendre(int m, double x) {
  if (m == 0) return {1.0, 0.0};
  double p0 = 1.0, p1 = x;
  for (int j = 2; j <= m; ++j) {
    const double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
    p0 = p1;
    p1 = p2;
  }
  return {p1, m * (x * p1 - p0) / (x * x - 1.0)};
}

template <int N>
struct Rules {
  double xg[N], wg[N];   // Gauss-Legendre on [0,1]
  double xl[N];          // Gauss-Lobatto-Legendre on [0,1]
};

template <int N>
constexpr Rules<N> rules() {
  Rules<N> r{};
  for (int j = 0; j < N; ++j) {   // Gauss: Newton on P_N
    double t = -cos_series(kPi * (j + 0.75) / (N + 0.5));
    for (int it = 0; it < 100; ++it) {
      const LegVal v = legendre(N, t);
      const double dt = v.P / v.dP;
      t -= dt;
      if (abs_(dt) < 1e-17) break;
    }
    const LegVal v = legendre(N, t);
    r.xg[j] = 0.5 * (t + 1.0);
    r.wg[j] = 1.0 / ((1.0 - t * t) * v.dP * v.dP);
  }
  const int k = N - 1;
  for (int j = 0; j < N; ++j) {   // Gauss-Lobatto: end points and roots of P_k'
    double t = j == 0 ? -1.0 : (j == k ? 1.0 : -cos_series(kPi * j / k));
    if (j > 0 && j < k) {
      for (int it = 0; it < 100; ++it) {
        const LegVal v = legendre(k, t);
        const double d2P = (2.0 * t * v.dP - k * (k + 1.0) * v.P) / (1.0 - t * t);
        const double dt = v.dP / d2P;
        t -= dt;
        if (abs_(dt) < 1e-17) break;
      }
    }
    r.xl[j] = 0.5 * (t + 1.0);
  }
  return r;
}

// value and derivative of the Lagrange polynomial i of `nodes` at x
template <int N>
constexpr LegVal lagrange(const double (&nodes)[N], int i, double x) {
  double v = 1.0;
  for (int j = 0; j < N; ++j)
    if (j != i) v *= (x - nodes[j]) / (nodes[i] - nodes[j]);
  double d = 0.0;
  for (int m = 0; m < N; ++m) {
    if (m == i) continue;
    double t = 1.0 / (nodes[i] - nodes[m]);
    for (int j = 0; j < N; ++j)
      if (j != i && j != m) t *= (x - nodes[j]) / (nodes[i] - nodes[j]);
    d += t;
  }
  return {v, d};
}

template <int N>
struct Dense {
  double M[N * N], K[N * N], S[N * N], D[N * N];
};

template <int N>
constexpr Dense<N> dense() {
  const Rules<N> r = rules<N>();
  Dense<N> o{};
  double S[N * N] = {}, Sd[N * N] = {};
  for (int q = 0; q < N; ++q)
    for (int i = 0; i < N; ++i) {
      const LegVal v = lagrange<N>(r.xl, i, r.xg[q]);
      S[q * N + i] = v.P;
      Sd[q * N + i] = v.dP;
      o.D[q * N + i] = lagrange<N>(r.xg, i, r.xg[q]).dP;
    }
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      double m = 0.0, s = 0.0;
      for (int q = 0; q < N; ++q) {
        m += r.wg[q] * S[q * N + i] * S[q * N + j];
        s += r.wg[q] * Sd[q * N + i] * Sd[q * N + j];
      }
      o.M[i * N + j] = m;
      o.K[i * N + j] = s;
    }
  for (int i = 0; i < N * N; ++i) o.S[i] = S[i];
  return o;
}

template <int N, typename T>
constexpr EO<N, T> to_eo(const double (&A)[N * N]) {
  EO<N, T> e{};
  constexpr int H = N / 2;
  for (int q = 0; q < H; ++q) {
    for (int i = 0; i < H; ++i) {
      e.ep[q * H + i] = T(0.5 * (A[q * N + i] + A[q * N + N - 1 - i]));
      e.op[q * H + i] = T(0.5 * (A[q * N + i] - A[q * N + N - 1 - i]));
    }
    e.ec[q] = (N % 2) ? T(A[q * N + H]) : T(0);
  }
  for (int i = 0; i <= H; ++i) e.mid[i] = (N % 2) ? T(A[H * N + i]) : T(0);
  return e;
}

template <int N, typename T>
constexpr EOTab<N, T> eotab() {
  const Dense<N> d = dense<N>();
  EOTab<N, T> e{};
  e.M = to_eo<N, T>(d.M);
  e.K = to_eo<N, T>(d.K);
  e.S = to_eo<N, T>(d.S);
  e.D = to_eo<N, T>(d.D);
  return e;
}

template <int N, typename T>
struct Tables {
  static constexpr EOTab<N, T> eo = eotab<N, T>();
};

// DG basis (Lagrange in the N Gauss points of [0,1]): Gauss points xg and weights w,
// reference stiffness Kg[i][j] = sum_q w_q psi_i'(x_q) psi_j'(x_q) in even-odd form and its
// diagonal kgd, and the basis values and derivatives at the end points: fv0[i] = psi_i(0),
// fd0[i] = psi_i'(0).  By the symmetry of the points, psi_i(1) = fv0[N-1-i] and
// psi_i'(1) = -fd0[N-1-i].  Even and odd halves of the end-point rows for i < N/2:
// fe = (fv0[i] + fv0[N-1-i]) / 2, fo = (fv0[i] - fv0[N-1-i]) / 2, and de, dd alike from fd0.
template <int N, typename T>
struct DGTab {
  T xg[N], w[N];
  T fv0[N], fd0[N];
  T kgd[N];
  T fe[N / 2 + 1], fo[N / 2 + 1], de[N / 2 + 1], dd[N / 2 + 1];
  EO<N, T> Kg;
};

template <int N, typename T>
constexpr DGTab<N, T> dgtab() {
  const Rules<N> r = rules<N>();
  DGTab<N, T> t{};
  double D[N * N] = {}, Kg[N * N] = {};
  for (int q = 0; q < N; ++q)
    for (int i = 0; i < N; ++i) D[q * N + i] = lagrange<N>(r.xg, i, r.xg[q]).dP;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      double s = 0.0;
      for (int q = 0; q < N; ++q) s += r.wg[q] * D[q * N + i] * D[q * N + j];
      Kg[i * N + j] = s;
    }
  for (int i = 0; i < N; ++i) {
    t.xg[i] = T(r.xg[i]);
    t.w[i] = T(r.wg[i]);
    t.kgd[i] = T(Kg[i * N + i]);
    const LegVal v = lagrange<N>(r.xg, i, 0.0);
    t.fv0[i] = T(v.P);
    t.fd0[i] = T(v.dP);
  }
  for (int i = 0; i < N / 2; ++i) {
    const LegVal a = lagrange<N>(r.xg, i, 0.0), b = lagrange<N>(r.xg, N - 1 - i, 0.0);
    t.fe[i] = T(0.5 * (a.P + b.P));
    t.fo[i] = T(0.5 * (a.P - b.P));
    t.de[i] = T(0.5 * (a.dP + b.dP));
    t.dd[i] = T(0.5 * (a.dP - b.dP));
  }
  t.Kg = to_eo<N, T>(Kg);
  return t;
}

template <int N, typename T>
struct DGTables {
  static constexpr DGTab<N, T> tab = dgtab<N, T>();
};

// For the Jacobi smoother of the GLL-Lagrange basis on DG cells: the diagonals of the GLL
// mass and stiffness matrices (k+1 Gauss quadrature, reference [0,1]) and the derivative of
// the first GLL Lagrange polynomial at 0 (by symmetry the last one has -d0 at 1).
template <int N, typename T>
struct GLLDiag {
  T m[N], k[N];
  T d0;
};

template <int N, typename T>
constexpr GLLDiag<N, T> glldiag() {
  const Dense<N> d = dense<N>();
  const Rules<N> r = rules<N>();
  GLLDiag<N, T> g{};
  for (int i = 0; i < N; ++i) {
    g.m[i] = T(d.M[i * N + i]);
    g.k[i] = T(d.K[i * N + i]);
  }
  g.d0 = T(lagrange<N>(r.xl, 0, 0.0).dP);
  return g;
}

template <int N, typename T>
struct GLLDiagTables {
  static constexpr GLLDiag<N, T> tab = glldiag<N, T>();
};

}  // namespace ct
}  // namespace mfl
