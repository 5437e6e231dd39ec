// One-dimensional finite-element tables for the tensor-product Taylor-Hood
// cell operators (host code).
//
// Sec. 2: velocity Q_k and pressure Q_{k-1} are tensor products of 1D
// Lagrange bases on (0,1).  Node positions: Gauss-Lobatto-Legendre points
// (k+1 for velocity, k for pressure).  Quadrature: Gauss-Legendre with k+1
// points, exact for every integrand of the forms a and b on affine cells.
//
// On an axis-aligned box cell of width h the Jacobian is the constant
// diagonal matrix diag(h_x, h_y, h_z), so the reference-cell quadrature of
// Sec. 3.1 factors into 1D integrals: the cell matrix of a(.,.) is the
// Kronecker sum  mu (K_x (x) M_y (x) M_z + M_x (x) K_y (x) M_z + ...) +
// gamma rho M_x (x) M_y (x) M_z, and that of b(.,.) the Kronecker products of
// the mixed 1D matrices below.  The tables are those 1D integrals, each
// evaluated with the same (k+1)-point Gauss rule.
#pragma once
#include <cmath>
#include <vector>

namespace smg {

// Legendre polynomial P_n and its derivative at x in [-1,1] (three-term recurrence).
inline void legendre(int n, double x, double &p, double &dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { p = 1.0; dp = 0.0; return; }
  for (int j = 2; j <= n; ++j) {
    double pj = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
    p0 = p1;
    p1 = pj;
  }
  p = p1;
  dp = (std::fabs(x) < 1.0) ? n * (x * p1 - p0) / (x * x - 1.0) : 0.5 * n * (n + 1) * (x > 0 ? 1.0 : (n % 2 ? 1.0 : -1.0));
}

// Gauss-Legendre points/weights on (0,1): Newton on P_n from Chebyshev guesses.
inline void gauss_points(int n, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(n, z, p, dp);
      double dz = p / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p, dp;
    legendre(n, z, p, dp);
    // map from [-1,1] to [0,1]; points ascending
    x[n - 1 - i] = 0.5 * (z + 1.0);
    w[n - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);  // = 0.5 * 2/((1-z^2) P'^2)
  }
}

// Gauss-Lobatto-Legendre points on [0,1]: end points plus the roots of P'_{n-1}.
inline std::vector<double> gll_points(int n) {
  std::vector<double> x(n);
  x[0] = 0.0;
  x[n - 1] = 1.0;
  int m = n - 1;  // roots of P'_m, m-1 of them
  for (int i = 1; i < m; ++i) {
    double z = -std::cos(M_PI * i / m);
    for (int it = 0; it < 100; ++it) {
      // q(z) = P'_m(z); q'(z) from the Legendre ODE: (1-z^2) P'' = 2 z P' - m(m+1) P
      double p, dp;
      legendre(m, z, p, dp);
      double ddp = (2.0 * z * dp - m * (m + 1.0) * p) / (1.0 - z * z);
      double dz = dp / ddp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = 0.5 * (z + 1.0);
  }
  return x;
}

// Lagrange polynomial l_i through nodes z, and its derivative, at t.
inline double lagrange(const std::vector<double> &z, int i, double t) {
  double v = 1.0;
  for (size_t j = 0; j < z.size(); ++j)
    if ((int)j != i) v *= (t - z[j]) / (z[i] - z[j]);
  return v;
}
inline double lagrange_deriv(const std::vector<double> &z, int i, double t) {
  double s = 0.0;
  for (size_t m = 0; m < z.size(); ++m) {
    if ((int)m == i) continue;
    double term = 1.0 / (z[i] - z[m]);
    for (size_t j = 0; j < z.size(); ++j)
      if ((int)j != i && j != m) term *= (t - z[j]) / (z[i] - z[j]);
    s += term;
  }
  return s;
}

// 1D reference tables for degree k, unit cell:
//   Kv[i][j] = int l_i' l_j',  Mv[i][j] = int l_i l_j        (velocity, (k+1)^2)
//   G[i][j]  = int psi_i l_j', N[i][j]  = int psi_i l_j      (pressure x velocity, k x (k+1))
//   Mp[i][j] = int psi_i psi_j                               (pressure, k^2)
//   Vq[q][i] = l_i(x_q), Dq[q][i] = l_i'(x_q), Pq[q][i] = psi_i(x_q), wq[q]  (quadrature)
struct Ref1D {
  int k;
  std::vector<double> zv, zp, xq, wq;
  std::vector<double> Kv, Mv, G, N, Mp, Vq, Dq, Pq;
};

inline Ref1D make_ref1d(int k) {
  Ref1D r;
  r.k = k;
  const int nv = k + 1, np = k, nq = k + 1;
  r.zv = gll_points(nv);
  r.zp = gll_points(np);
  gauss_points(nq, r.xq, r.wq);
  r.Kv.assign(nv * nv, 0.0);
  r.Mv.assign(nv * nv, 0.0);
  r.G.assign(np * nv, 0.0);
  r.N.assign(np * nv, 0.0);
  r.Mp.assign(np * np, 0.0);
  r.Vq.assign(nq * nv, 0.0);
  r.Dq.assign(nq * nv, 0.0);
  r.Pq.assign(nq * np, 0.0);
  for (int q = 0; q < nq; ++q) {
    for (int i = 0; i < nv; ++i) {
      r.Vq[q * nv + i] = lagrange(r.zv, i, r.xq[q]);
      r.Dq[q * nv + i] = lagrange_deriv(r.zv, i, r.xq[q]);
    }
    for (int i = 0; i < np; ++i) r.Pq[q * np + i] = lagrange(r.zp, i, r.xq[q]);
  }
  for (int q = 0; q < nq; ++q) {
    const double w = r.wq[q];
    for (int i = 0; i < nv; ++i)
      for (int j = 0; j < nv; ++j) {
        r.Kv[i * nv + j] += w * r.Dq[q * nv + i] * r.Dq[q * nv + j];
        r.Mv[i * nv + j] += w * r.Vq[q * nv + i] * r.Vq[q * nv + j];
      }
    for (int i = 0; i < np; ++i) {
      for (int j = 0; j < nv; ++j) {
        r.G[i * nv + j] += w * r.Pq[q * np + i] * r.Dq[q * nv + j];
        r.N[i * nv + j] += w * r.Pq[q * np + i] * r.Vq[q * nv + j];
      }
      for (int j = 0; j < np; ++j) r.Mp[i * np + j] += w * r.Pq[q * np + i] * r.Pq[q * np + j];
    }
  }
  return r;
}

// Prolongation weights of the canonical injection (Sec. 3.2) in 1D: the
// coarse cell (0,1) is split into two fine cells; W[f][j] = l_j(t_f) for the
// 2k+1 fine nodes t_f of the coarse cell (fine node f lies in fine cell f/k
// at local node f%k, the last one at t = 1).
inline std::vector<double> prolongation_weights(const std::vector<double> &z) {
  const int deg = (int)z.size() - 1;
  const int nf = 2 * deg + 1;
  std::vector<double> W(nf * (deg + 1));
  for (int f = 0; f < nf; ++f) {
    int cf = f / deg;
    double tf = (cf < 2) ? z[f - cf * deg] : 1.0;
    if (cf == 2) cf = 1, tf = 1.0;
    double t = 0.5 * (cf + tf);
    for (int j = 0; j <= deg; ++j) W[f * (deg + 1) + j] = lagrange(z, j, t);
  }
  return W;
}

}  // namespace smg
