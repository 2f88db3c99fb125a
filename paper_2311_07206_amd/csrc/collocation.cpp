// Collocation data on Radau-IIA nodes (paper Sec. 3.1, eq. "SDC Integration"
// and eq. (SDC)), computed on the host once per context.
//
//  tau  right Radau points on [0,1]: x = 2*tau - 1 solves P_M(x) = P_{M-1}(x);
//       x = 1 is always a root, the others are bracketed on a grid and
//       refined by bisection and Newton steps on the Legendre recurrence.
//  Q    Q[m][j] = integral_0^{tau_m} l_j(s) ds by an M-point Gauss-Legendre
//       rule on [0, tau_m] (exact: l_j has degree M-1).
//  QI   lower-triangular U^T from the Doolittle factorisation Q^T = L U
//       (the "LU trick" the paper uses for S-hat).
//  QE   forward Euler between consecutive nodes: QE[m][j] = tau_{j+1}-tau_j, j<m.
#include "internal.hpp"

#include <cmath>

namespace sdc {

namespace {

// P_n(x) and P_n'(x) by the three-term recurrence.
void legendre(int n, double x, double* p, double* dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { *p = 1.0; *dp = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double pk = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = pk;
  }
  *p = p1;
  // (x^2 - 1) P_n'(x) = n (x P_n - P_{n-1})
  *dp = (std::fabs(x * x - 1.0) > 1e-300) ? n * (x * p1 - p0) / (x * x - 1.0) : 0.0;
}

// All roots of f on (lo, hi) by sign changes on a grid, bisection and Newton.
template <class F>
int roots(F f, double lo, double hi, double* out, int max_out) {
  const int G = 20000;
  int found = 0;
  double xa = lo, fa = f(xa, nullptr);
  for (int g = 1; g <= G && found < max_out; ++g) {
    double xb = lo + (hi - lo) * g / G;
    double fb = f(xb, nullptr);
    if (fa == 0.0) {
      out[found++] = xa;
    } else if (fa * fb < 0.0) {
      double a = xa, b = xb, fa2 = fa;
      for (int it = 0; it < 200 && b - a > 1e-15; ++it) {
        double c = 0.5 * (a + b), fc = f(c, nullptr);
        if (fa2 * fc <= 0.0) b = c; else { a = c; fa2 = fc; }
      }
      double x = 0.5 * (a + b);
      for (int it = 0; it < 3; ++it) {
        double d;
        double fx = f(x, &d);
        if (d != 0.0) {
          double xn = x - fx / d;
          if (xn > xa && xn < xb) x = xn;
        }
      }
      out[found++] = x;
    }
    xa = xb;
    fa = fb;
  }
  return found;
}

}  // namespace

int collocation(int M, Collocation* c) {
  if (M < 1 || M > kMaxNodes) return -1;
  c->M = M;
  // Radau right points
  if (M == 1) {
    c->tau[0] = 1.0;
  } else {
    auto f = [M](double x, double* d) {
      double pm, dpm, pm1, dpm1;
      legendre(M, x, &pm, &dpm);
      legendre(M - 1, x, &pm1, &dpm1);
      if (d) *d = dpm - dpm1;
      return pm - pm1;
    };
    double x[kMaxNodes];
    int n = roots(f, -1.0, 1.0 - 1e-9, x, M - 1);
    if (n != M - 1) return -2;
    for (int i = 0; i < M - 1; ++i) c->tau[i] = 0.5 * (x[i] + 1.0);
    c->tau[M - 1] = 1.0;
  }
  // Gauss-Legendre rule with M points on [-1, 1]
  double gx[kMaxNodes], gw[kMaxNodes];
  {
    auto f = [M](double x, double* d) {
      double p, dp;
      legendre(M, x, &p, &dp);
      if (d) *d = dp;
      return p;
    };
    int n = roots(f, -1.0, 1.0, gx, M);
    if (n != M) return -3;
    for (int i = 0; i < M; ++i) {
      double p, dp;
      legendre(M, gx[i], &p, &dp);
      gw[i] = 2.0 / ((1.0 - gx[i] * gx[i]) * dp * dp);
    }
  }
  // Q[m][j] = int_0^{tau_m} l_j
  for (int m = 0; m < M; ++m) {
    for (int j = 0; j < M; ++j) {
      double s = 0.0;
      for (int g = 0; g < M; ++g) {
        double t = 0.5 * c->tau[m] * (gx[g] + 1.0);
        double l = 1.0;
        for (int q = 0; q < M; ++q)
          if (q != j) l *= (t - c->tau[q]) / (c->tau[j] - c->tau[q]);
        s += gw[g] * l;
      }
      c->Q[m][j] = 0.5 * c->tau[m] * s;
    }
  }
  // Doolittle: Q^T = L U, QI = U^T
  double U[kMaxNodes][kMaxNodes] = {}, L[kMaxNodes][kMaxNodes] = {};
  for (int i = 0; i < M; ++i) {
    L[i][i] = 1.0;
    for (int k = i; k < M; ++k) {
      double s = c->Q[k][i];  // (Q^T)[i][k]
      for (int q = 0; q < i; ++q) s -= L[i][q] * U[q][k];
      U[i][k] = s;
    }
    for (int k = i + 1; k < M; ++k) {
      double s = c->Q[i][k];  // (Q^T)[k][i]
      for (int q = 0; q < i; ++q) s -= L[k][q] * U[q][i];
      L[k][i] = s / U[i][i];
    }
  }
  for (int m = 0; m < kMaxNodes; ++m)
    for (int j = 0; j < kMaxNodes; ++j) {
      c->QI[m][j] = (m < M && j < M && j <= m) ? U[j][m] : 0.0;
      c->QE[m][j] = (m < M && j < m) ? c->tau[j + 1] - c->tau[j] : 0.0;
      if (m >= M || j >= M) c->Q[m][j] = 0.0;
    }
  return 0;
}

}  // namespace sdc
