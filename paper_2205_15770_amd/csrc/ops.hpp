// Epilogue functors of the tile kernel: what is read into the DoF patch and
// what is written for each owned node.  Each fuses the vector algebra that
// follows an operator application in the solver into the same memory pass.
#pragma once
#include "common.hpp"

namespace smg {

// y = (block of K) x
template <typename T>
struct OpApply {
  static constexpr bool ZERO_BC = true;
  const T *xu, *xp;
  T *yu, *yp;
  __device__ T load_u(i64 i) const { return xu[i]; }
  __device__ T load_p(i64 i) const { return xp[i]; }
  __device__ void store_u(i64 i, T t, T, bool) const { yu[i] = t; }
  __device__ void store_p(i64 i, T t, T) const { yp[i] = t; }
};

// r = b - (block of K) x
template <typename T>
struct OpResidual {
  static constexpr bool ZERO_BC = true;
  const T *xu, *xp, *bu, *bp;
  T *ru, *rp;
  __device__ T load_u(i64 i) const { return xu[i]; }
  __device__ T load_p(i64 i) const { return xp[i]; }
  __device__ void store_u(i64 i, T t, T, bool) const { ru[i] = bu[i] - t; }
  __device__ void store_p(i64 i, T t, T) const { rp[i] = bp[i] - t; }
};

// y = M_v f on every node, 0 on Dirichlet rows (load vector of a nodal field)
template <typename T>
struct OpMass {
  static constexpr bool ZERO_BC = false;
  const T *f;
  T *y;
  __device__ T load_u(i64 i) const { return f[i]; }
  __device__ T load_p(i64) const { return 0; }
  __device__ void store_u(i64 i, T t, T, bool bc) const { y[i] = bc ? T(0) : t; }
  __device__ void store_p(i64, T, T) const {}
};

// One step of the Chebyshev-acceleration recurrence for A (velocity vectors),
// Sec. 3.3.1 (Cheb(A, D_A, k)), with t = A d_i:
//   r_{i+1} = r_i - t,  x_{i+1} = x_i + d_i,  d_{i+1} = c1 d_i + c2 D^-1 r_{i+1}
// FIRST: d_0 = D^-1 r_0 / theta is formed while loading (r_0 = rin, x_0 = 0).
// LAST:  out = base + s (x_{k} + d_{k}) instead of storing r, x, d.
template <typename T, bool FIRST, bool LAST>
struct OpChebA {
  static constexpr bool ZERO_BC = true;
  const T *rin;      // r_0 (FIRST) or r_i
  const T *dinv;     // D_A^-1
  const T *d;        // d_i (not FIRST)
  const T *x;        // x_i (not FIRST)
  T *r_out, *x_out, *d_out;  // (not LAST)
  const T *base;     // LAST: optional base vector (nullptr = 0)
  T *out;            // LAST
  T inv_theta, c1, c2, s;
  __device__ T load_u(i64 i) const {
    if constexpr (FIRST) return dinv[i] * rin[i] * inv_theta;
    else return d[i];
  }
  __device__ T load_p(i64) const { return 0; }
  __device__ void store_u(i64 i, T t, T v, bool) const {
    const T rn = rin[i] - t;
    const T xn = FIRST ? v : x[i] + v;
    const T dn = c1 * v + c2 * dinv[i] * rn;
    if constexpr (LAST) {
      out[i] = (base ? base[i] : T(0)) + s * (xn + dn);
    } else {
      r_out[i] = rn;
      x_out[i] = xn;
      d_out[i] = dn;
    }
  }
  __device__ void store_p(i64, T, T) const {}
};

// q = B^T d with d = D_S^-1 r / theta formed while loading (FIRST) or d given.
template <typename T, bool FIRST>
struct OpGrad {
  static constexpr bool ZERO_BC = true;
  const T *rp, *dinv_s, *d;
  T inv_theta;
  T *q;
  __device__ T load_u(i64) const { return 0; }
  __device__ T load_p(i64 i) const {
    if constexpr (FIRST) return dinv_s[i] * rp[i] * inv_theta;
    else return d[i];
  }
  __device__ void store_u(i64 i, T t, T, bool) const { q[i] = t; }
  __device__ void store_p(i64, T, T) const {}
};

// Chebyshev step for S~ = B A_hat^-1 B^T + C (pressure vectors): the kernel
// computes t = B w + C d_i from w = A_hat^-1 B^T d_i and the pressure patch d_i.
// LAST: dp = tau (x_k + d_k) is stored and added to the pressure iterate.
template <typename T, bool FIRST, bool LAST>
struct OpChebS {
  static constexpr bool ZERO_BC = true;
  const T *w;        // velocity input
  const T *rin;      // r_0 (FIRST) or r_i
  const T *dinv_s;
  const T *d;        // d_i (not FIRST)
  const T *x;        // x_i (not FIRST)
  T *r_out, *x_out, *d_out;
  T *p, *dp;         // LAST
  T inv_theta, c1, c2, tau;
  __device__ T load_u(i64 i) const { return w[i]; }
  __device__ T load_p(i64 i) const {
    if constexpr (FIRST) return dinv_s[i] * rin[i] * inv_theta;
    else return d[i];
  }
  __device__ void store_u(i64, T, T, bool) const {}
  __device__ void store_p(i64 i, T t, T) const {
    const T di = FIRST ? dinv_s[i] * rin[i] * inv_theta : d[i];
    const T rn = rin[i] - t;
    const T xn = FIRST ? di : x[i] + di;
    const T dn = c1 * di + c2 * dinv_s[i] * rn;
    if constexpr (LAST) {
      const T delta = tau * (xn + dn);
      dp[i] = delta;
      if (p) p[i] += delta;
    } else {
      r_out[i] = rn;
      x_out[i] = xn;
      d_out[i] = dn;
    }
  }
};

// r_p = B u - C p - g, the argument of the second Uzawa update.
template <typename T>
struct OpDivResidual {
  static constexpr bool ZERO_BC = true;
  const T *u, *p_in, *g;
  T *rp;
  __device__ T load_u(i64 i) const { return u[i]; }
  __device__ T load_p(i64 i) const { return p_in[i]; }
  __device__ void store_u(i64, T, T, bool) const {}
  __device__ void store_p(i64 i, T t, T) const { rp[i] = t - (g ? g[i] : T(0)); }
};

}  // namespace smg
