// Compile-time 1D reference tables of the Taylor-Hood cell operators on the
// unit interval (Sec. 2: velocity Q_k on the k+1 Gauss-Lobatto-Legendre
// points, pressure Q_{k-1} on k of them, Gauss-Legendre quadrature with k+1
// points).  The device kernels read these as literals, so matrix entries cost
// neither registers nor loads; the cell width enters through a few scalars:
// on a box cell of widths h_a the velocity stiffness is Kr / h_a, the masses
// Mr h_a, Mpr h_a, the mixed matrices Gr (unscaled) and Nr h_a.
//
// The values are computed here by the same steps as the host tables
// (Legendre three-term recurrence, Newton iteration for the Gauss and GLL
// points, products of Lagrange values summed over the quadrature points); the
// solver set-up checks that both agree.
#pragma once

namespace smg {
namespace cfe {

constexpr double kPi = 3.14159265358979323846;

constexpr double cabs(double x) { return x < 0 ? -x : x; }

// cos by range reduction to [-pi, pi] and its Taylor series
constexpr double ccos(double x) {
  while (x > kPi) x -= 2 * kPi;
  while (x < -kPi) x += 2 * kPi;
  double term = 1.0, sum = 1.0;
  for (int n = 1; n < 40; ++n) {
    term *= -x * x / ((2.0 * n - 1) * (2.0 * n));
    sum += term;
  }
  return sum;
}

struct PD {
  double p, dp;
};

// Legendre P_n and P_n' at x in (-1, 1)
constexpr PD legendre(int n, double x) {
  if (n == 0) return PD{1.0, 0.0};
  double p0 = 1.0, p1 = x;
  for (int j = 2; j <= n; ++j) {
    const double pj = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
    p0 = p1;
    p1 = pj;
  }
  return PD{p1, n * (x * p1 - p0) / (x * x - 1.0)};
}

template <int N>
struct Rule {
  double x[N];
  double w[N];
};

// N-point Gauss-Legendre rule on (0, 1), points ascending
template <int N>
constexpr Rule<N> gauss() {
  Rule<N> r{};
  for (int i = 0; i < N; ++i) {
    double z = ccos(kPi * (i + 0.75) / (N + 0.5));
    for (int it = 0; it < 100; ++it) {
      const PD v = legendre(N, z);
      const double dz = v.p / v.dp;
      z -= dz;
      if (cabs(dz) < 1e-16) break;
    }
    const PD v = legendre(N, z);
    r.x[N - 1 - i] = 0.5 * (z + 1.0);
    r.w[N - 1 - i] = 1.0 / ((1.0 - z * z) * v.dp * v.dp);
  }
  return r;
}

// N Gauss-Lobatto-Legendre points on [0, 1]
template <int N>
struct Pts {
  double z[N];
};
template <int N>
constexpr Pts<N> gll() {
  Pts<N> r{};
  r.z[0] = 0.0;
  r.z[N - 1] = 1.0;
  const int m = N - 1;
  for (int i = 1; i < m; ++i) {
    double z = -ccos(kPi * i / m);
    for (int it = 0; it < 100; ++it) {
      const PD v = legendre(m, z);
      const double ddp = (2.0 * z * v.dp - m * (m + 1.0) * v.p) / (1.0 - z * z);
      const double dz = v.dp / ddp;
      z -= dz;
      if (cabs(dz) < 1e-16) break;
    }
    r.z[i] = 0.5 * (z + 1.0);
  }
  return r;
}

template <int N>
constexpr double lagrange(const Pts<N> &z, int i, double t) {
  double v = 1.0;
  for (int j = 0; j < N; ++j)
    if (j != i) v *= (t - z.z[j]) / (z.z[i] - z.z[j]);
  return v;
}
template <int N>
constexpr double lagrange_deriv(const Pts<N> &z, int i, double t) {
  double s = 0.0;
  for (int m = 0; m < N; ++m) {
    if (m == i) continue;
    double term = 1.0 / (z.z[i] - z.z[m]);
    for (int j = 0; j < N; ++j)
      if (j != i && j != m) term *= (t - z.z[j]) / (z.z[i] - z.z[j]);
    s += term;
  }
  return s;
}

// Kr = int l_i' l_j', Mr = int l_i l_j, Gr = int psi_i l_j', Nr = int psi_i l_j,
// Mpr = int psi_i psi_j on (0, 1)
template <int K>
struct Tab {
  double Kr[K + 1][K + 1];
  double Mr[K + 1][K + 1];
  double Gr[K][K + 1];
  double Nr[K][K + 1];
  double Mpr[K][K];
};

template <int K>
constexpr Tab<K> make_tab() {
  constexpr int NV = K + 1, NP = K, NQ = K + 1;
  Tab<K> t{};
  const Pts<NV> zv = gll<NV>();
  const Pts<NP> zp = gll<NP>();
  const Rule<NQ> q = gauss<NQ>();
  for (int k = 0; k < NQ; ++k) {
    double V[NV] = {}, D[NV] = {}, P[NP] = {};
    for (int i = 0; i < NV; ++i) {
      V[i] = lagrange(zv, i, q.x[k]);
      D[i] = lagrange_deriv(zv, i, q.x[k]);
    }
    for (int i = 0; i < NP; ++i) P[i] = lagrange(zp, i, q.x[k]);
    const double w = q.w[k];
    for (int i = 0; i < NV; ++i)
      for (int j = 0; j < NV; ++j) {
        t.Kr[i][j] += w * D[i] * D[j];
        t.Mr[i][j] += w * V[i] * V[j];
      }
    for (int i = 0; i < NP; ++i) {
      for (int j = 0; j < NV; ++j) {
        t.Gr[i][j] += w * P[i] * D[j];
        t.Nr[i][j] += w * P[i] * V[j];
      }
      for (int j = 0; j < NP; ++j) t.Mpr[i][j] += w * P[i] * P[j];
    }
  }
  return t;
}

// the tables in the arithmetic type of a kernel
template <int K, typename T>
struct TabT {
  T Kr[K + 1][K + 1];
  T Mr[K + 1][K + 1];
  T Gr[K][K + 1];
  T Nr[K][K + 1];
  T Mpr[K][K];
};

template <int K, typename T>
constexpr TabT<K, T> make_tab_t() {
  const Tab<K> d = make_tab<K>();
  TabT<K, T> t{};
  for (int i = 0; i <= K; ++i)
    for (int j = 0; j <= K; ++j) {
      t.Kr[i][j] = (T)d.Kr[i][j];
      t.Mr[i][j] = (T)d.Mr[i][j];
    }
  for (int i = 0; i < K; ++i) {
    for (int j = 0; j <= K; ++j) {
      t.Gr[i][j] = (T)d.Gr[i][j];
      t.Nr[i][j] = (T)d.Nr[i][j];
    }
    for (int j = 0; j < K; ++j) t.Mpr[i][j] = (T)d.Mpr[i][j];
  }
  return t;
}

template <int K, typename T = double>
struct Ref {
  static constexpr TabT<K, T> t = make_tab_t<K, T>();
};

// Quadrature-point tables for general (multilinear) cells: the k+1 Gauss
// points x_q and weights w_q on (0, 1); V[q][i] = l_i(x_q) (velocity GLL
// basis), Vp[q][i] = psi_i(x_q) (pressure basis), and the collocation
// derivative D[q][j] = lg_j'(x_q) of the Lagrange basis lg on the Gauss points
// (exact for the degree-k restrictions of Q_k fields to coordinate lines).
template <int K, typename T>
struct QTab {
  T x[K + 1], w[K + 1];
  T V[K + 1][K + 1];
  T D[K + 1][K + 1];
  T Vp[K + 1][K];
};

template <int K, typename T>
constexpr QTab<K, T> make_qtab() {
  constexpr int NQ = K + 1;
  QTab<K, T> t{};
  const Rule<NQ> q = gauss<NQ>();
  const Pts<K + 1> zv = gll<K + 1>();
  const Pts<K> zp = gll<K>();
  Pts<NQ> zq{};
  for (int i = 0; i < NQ; ++i) zq.z[i] = q.x[i];
  for (int a = 0; a < NQ; ++a) {
    t.x[a] = (T)q.x[a];
    t.w[a] = (T)q.w[a];
    for (int i = 0; i <= K; ++i) t.V[a][i] = (T)lagrange(zv, i, q.x[a]);
    for (int j = 0; j < NQ; ++j) t.D[a][j] = (T)lagrange_deriv(zq, j, q.x[a]);
    for (int i = 0; i < K; ++i) t.Vp[a][i] = (T)lagrange(zp, i, q.x[a]);
  }
  return t;
}

}  // namespace cfe
}  // namespace smg
