// Host-side one-dimensional rules and basis tables.
//
// Sec. 2.1: the continuous basis is Lagrange in the k+1 Gauss-Lobatto-Legendre nodes.
// Sec. 3 (eq. mf_eval): integrals use k+1 Gauss-Legendre points per direction; on
// Cartesian cells this quadrature is exact, so the 1D mass and stiffness matrices below
// are exact integrals.  The DG basis is Lagrange in the Gauss points.
#include <cmath>

#include "mfl_internal.h"

namespace mfl {

namespace {

// Legendre P_m and P_m' at x by the three-term recurrence.
void legendre(int m, double x, double &P, double &dP) {
  double p0 = 1.0, p1 = x;
  if (m == 0) {
    P = 1.0;
    dP = 0.0;
    return;
  }
  for (int j = 2; j <= m; ++j) {
    double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
    p0 = p1;
    p1 = p2;
  }
  P = p1;
  dP = m * (x * p1 - p0) / (x * x - 1.0);
}

}  // namespace

void gauss_legendre(int n, double *x, double *w) {
  for (int j = 0; j < n; ++j) {
    double t = -std::cos(M_PI * (j + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(n, t, P, dP);
      double dt = P / dP;
      t -= dt;
      if (std::fabs(dt) < 1e-17) break;
    }
    double P, dP;
    legendre(n, t, P, dP);
    x[j] = 0.5 * (t + 1.0);
    w[j] = 1.0 / ((1.0 - t * t) * dP * dP);   // 2/((1-t^2) P'^2) on [-1,1], halved
  }
}

void gauss_lobatto(int n, double *x, double *w) {
  const int k = n - 1;
  for (int j = 0; j < n; ++j) {
    double t;
    if (j == 0) {
      t = -1.0;
    } else if (j == k) {
      t = 1.0;
    } else {
      t = -std::cos(M_PI * j / k);
      // Newton on P_k'(t); P_k'' from the Legendre equation
      for (int it = 0; it < 100; ++it) {
        double P, dP;
        legendre(k, t, P, dP);
        double d2P = (2.0 * t * dP - k * (k + 1.0) * P) / (1.0 - t * t);
        double dt = dP / d2P;
        t -= dt;
        if (std::fabs(dt) < 1e-17) break;
      }
    }
    double P, dP;
    legendre(k, t, P, dP);
    x[j] = 0.5 * (t + 1.0);
    w[j] = 1.0 / (k * (k + 1.0) * P * P);     // 2/(k(k+1) P_k^2) on [-1,1], halved
  }
}

void lagrange_eval(int n, const double *nodes, double x, double *val, double *der) {
  for (int i = 0; i < n; ++i) {
    double v = 1.0;
    for (int j = 0; j < n; ++j)
      if (j != i) v *= (x - nodes[j]) / (nodes[i] - nodes[j]);
    val[i] = v;
    double d = 0.0;
    for (int m = 0; m < n; ++m) {
      if (m == i) continue;
      double t = 1.0 / (nodes[i] - nodes[m]);
      for (int j = 0; j < n; ++j)
        if (j != i && j != m) t *= (x - nodes[j]) / (nodes[i] - nodes[j]);
      d += t;
    }
    der[i] = d;
  }
}

void build_tables(int k, Tab<kMaxN, double> &t, Tab<kMaxN, float> &t32, TransferTab &tt) {
  const int n = k + 1;
  double xq[kMaxN], wq[kMaxN], xl[kMaxN], wl[kMaxN], v[kMaxN], d[kMaxN];
  gauss_legendre(n, xq, wq);
  gauss_lobatto(n, xl, wl);
  t = Tab<kMaxN, double>{};
  // tables are stored densely with row length n (not kMaxN)
  for (int q = 0; q < n; ++q) {
    lagrange_eval(n, xl, xq[q], v, d);
    for (int i = 0; i < n; ++i) {
      t.S[q * n + i] = v[i];
      t.Sd[q * n + i] = d[i];
    }
    lagrange_eval(n, xq, xq[q], v, d);
    for (int p = 0; p < n; ++p) t.D[q * n + p] = d[p];
    t.w[q] = wq[q];
    t.gll[q] = xl[q];
    t.xg[q] = xq[q];
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double m = 0.0, s = 0.0;
      for (int q = 0; q < n; ++q) {
        m += wq[q] * t.S[q * n + i] * t.S[q * n + j];
        s += wq[q] * t.Sd[q * n + i] * t.Sd[q * n + j];
      }
      t.M[i * n + j] = m;
      t.K[i * n + j] = s;
    }
  for (int e = 0; e < 2; ++e) {
    lagrange_eval(n, xq, double(e), v, d);
    for (int p = 0; p < n; ++p) {
      t.Fv[e * n + p] = v[p];
      t.Fd[e * n + p] = d[p];
    }
  }
  const double *src = reinterpret_cast<const double *>(&t);
  float *dst = reinterpret_cast<float *>(&t32);
  const int count = sizeof(t) / sizeof(double);
  static_assert(sizeof(Tab<kMaxN, double>) == 2 * sizeof(Tab<kMaxN, float>), "table layout");
  for (int i = 0; i < count; ++i) dst[i] = float(src[i]);
  // embedding of the coarse cell's basis at its 2k+1 fine points per direction
  tt = TransferTab{};
  for (int f = 0; f <= 2 * k; ++f) {
    int j = f / k < 1 ? f / k : 1;
    double xi = 0.5 * (j + xl[f - j * k]);
    lagrange_eval(n, xl, xi, v, d);
    for (int i = 0; i < n; ++i) tt.P[f * n + i] = v[i];
  }
  for (int s = 0; s < 2; ++s)
    for (int f = 0; f < n; ++f) {
      lagrange_eval(n, xq, 0.5 * (s + xq[f]), v, d);
      for (int c = 0; c < n; ++c) tt.E[(s * n + f) * n + c] = v[c];
    }
}

}  // namespace mfl
