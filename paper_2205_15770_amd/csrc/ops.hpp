// Epilogue functors of the tile kernel: what is read into the DoF patch and
// what is written for each owned node.  Each fuses the vector algebra that
// follows an operator application in the solver into the same memory pass.
#pragma once
#include "common.hpp"

namespace smg {

// y = (block of K) x
template <typename T>
struct OpApply {
  static constexpr const char *NAME = "apply";
  static constexpr int VARIANT = 0;
  static constexpr bool ZERO_BC = true;
  const T *xu, *xp;
  T *yu, *yp;
  struct Pre {};
  template <class I>
  __device__ T load_u(I i) const { return at(xu, i); }
  template <class I>
  __device__ T load_p(I i) const { return at(xp, i); }
  template <class I>
  __device__ Pre fetch_u(I) const { return Pre{}; }
  template <class I>
  __device__ Pre fetch_p(I) const { return Pre{}; }
  template <class I>
  __device__ void store_u(I i, T t, T, bool, const Pre &) const { at(yu, i) = t; }
  template <class I>
  __device__ void store_p(I i, T t, T, const Pre &) const { at(yp, i) = t; }
  // algorithmic HBM bytes of one launch: every vector read or written once
  double algo_bytes(bool need_u, bool need_p, bool out_u, bool out_p, double nu, double np) const {
    return sizeof(T) * ((need_u ? nu : 0) + (need_p ? np : 0) + (out_u ? nu : 0) + (out_p ? np : 0));
  }
};

// r = b - (block of K) x
template <typename T>
struct OpResidual {
  static constexpr const char *NAME = "residual";
  static constexpr int VARIANT = 0;
  static constexpr bool ZERO_BC = true;
  const T *xu, *xp, *bu, *bp;
  T *ru, *rp;
  struct Pre {
    T b;
  };
  template <class I>
  __device__ T load_u(I i) const { return at(xu, i); }
  template <class I>
  __device__ T load_p(I i) const { return at(xp, i); }
  template <class I>
  __device__ Pre fetch_u(I i) const { return Pre{at(bu, i)}; }
  template <class I>
  __device__ Pre fetch_p(I i) const { return Pre{at(bp, i)}; }
  template <class I>
  __device__ void store_u(I i, T t, T, bool, const Pre &q) const { at(ru, i) = q.b - t; }
  template <class I>
  __device__ void store_p(I i, T t, T, const Pre &q) const { at(rp, i) = q.b - t; }
  double algo_bytes(bool need_u, bool need_p, bool out_u, bool out_p, double nu, double np) const {
    return sizeof(T) * ((need_u ? nu : 0) + (need_p ? np : 0) + (out_u ? 2 * nu : 0) + (out_p ? 2 * np : 0));
  }
};

// y = M_v f on every node, 0 on Dirichlet rows (load vector of a nodal field)
template <typename T>
struct OpMass {
  static constexpr const char *NAME = "mass";
  static constexpr int VARIANT = 0;
  static constexpr bool ZERO_BC = false;
  const T *f;
  T *y;
  struct Pre {};
  template <class I>
  __device__ T load_u(I i) const { return at(f, i); }
  template <class I>
  __device__ T load_p(I) const { return 0; }
  template <class I>
  __device__ Pre fetch_u(I) const { return Pre{}; }
  template <class I>
  __device__ Pre fetch_p(I) const { return Pre{}; }
  template <class I>
  __device__ void store_u(I i, T t, T, bool bc, const Pre &) const { at(y, i) = bc ? T(0) : t; }
  template <class I>
  __device__ void store_p(I, T, T, const Pre &) const {}
  double algo_bytes(bool, bool, bool, bool, double nu, double) const { return sizeof(T) * 2 * nu; }
};

// One step of the Chebyshev-acceleration recurrence for A (velocity vectors),
// Sec. 3.3.1 (Cheb(A, D_A, k)), with t = A d_i:
//   r_{i+1} = r_i - t,  x_{i+1} = x_i + d_i,  d_{i+1} = c1 d_i + c2 D^-1 r_{i+1}
// FIRST: d_0 = D^-1 r_0 / theta is formed while loading (r_0 = rin, x_0 = 0).
// LAST:  out = base + s (x_{k} + d_{k}) instead of storing r, x, d.
template <typename T, bool FIRST, bool LAST>
struct OpChebA {
  static constexpr const char *NAME = "cheb_A";
  static constexpr int VARIANT = (FIRST ? 1 : 0) + (LAST ? 2 : 0);
  static constexpr bool ZERO_BC = true;
  const T *rin;      // r_0 (FIRST) or r_i
  const T *dinv;     // D_A^-1
  const T *d;        // d_i (not FIRST)
  const T *x;        // x_i (not FIRST)
  T *r_out, *x_out, *d_out;  // (not LAST)
  const T *base;     // LAST: optional base vector (nullptr = 0)
  T *out;            // LAST
  T inv_theta, c1, c2, s;
  struct Pre {
    T r, x, dinv, base;
  };
  template <class I>
  __device__ T load_u(I i) const {
    if constexpr (FIRST) return at(dinv, i) * at(rin, i) * inv_theta;
    else return at(d, i);
  }
  template <class I>
  __device__ T load_p(I) const { return 0; }
  template <class I>
  __device__ Pre fetch_u(I i) const {
    Pre q;
    q.r = at(rin, i);
    q.x = FIRST ? T(0) : at(x, i);
    q.dinv = at(dinv, i);
    q.base = (LAST && base) ? at(base, i) : T(0);
    return q;
  }
  template <class I>
  __device__ Pre fetch_p(I) const { return Pre{}; }
  template <class I>
  __device__ void store_u(I i, T t, T v, bool, const Pre &q) const {
    const T rn = q.r - t;
    const T xn = q.x + v;
    const T dn = c1 * v + c2 * q.dinv * rn;
    if constexpr (LAST) {
      at(out, i) = q.base + s * (xn + dn);
    } else {
      at(r_out, i) = rn;
      at(x_out, i) = xn;
      at(d_out, i) = dn;
    }
  }
  template <class I>
  __device__ void store_p(I, T, T, const Pre &) const {}
  double algo_bytes(bool, bool, bool, bool, double nu, double) const {
    const double reads = FIRST ? 2 : 4, writes = LAST ? (base ? 2 : 1) : 3;
    return sizeof(T) * nu * (reads + writes);
  }
};

// q = B^T d with d = D_S^-1 r / theta formed while loading (FIRST) or d given.
template <typename T, bool FIRST>
struct OpGrad {
  static constexpr const char *NAME = "grad";
  static constexpr int VARIANT = FIRST ? 1 : 0;
  static constexpr bool ZERO_BC = true;
  const T *rp, *dinv_s, *d;
  T inv_theta;
  T *q;
  template <class I>
  __device__ T load_u(I) const { return 0; }
  template <class I>
  __device__ T load_p(I i) const {
    if constexpr (FIRST) return at(dinv_s, i) * at(rp, i) * inv_theta;
    else return at(d, i);
  }
  struct Pre {};
  template <class I>
  __device__ Pre fetch_u(I) const { return Pre{}; }
  template <class I>
  __device__ Pre fetch_p(I) const { return Pre{}; }
  template <class I>
  __device__ void store_u(I i, T t, T, bool, const Pre &) const { at(q, i) = t; }
  template <class I>
  __device__ void store_p(I, T, T, const Pre &) const {}
  double algo_bytes(bool, bool, bool, bool, double nu, double np) const {
    return sizeof(T) * ((FIRST ? 2 : 1) * np + nu);
  }
};

// Chebyshev step for S~ = B A_hat^-1 B^T + C (pressure vectors): the kernel
// computes t = B w + C d_i from w = A_hat^-1 B^T d_i and the pressure patch d_i.
// LAST: dp = tau (x_k + d_k) is stored and added to the pressure iterate.
template <typename T, bool FIRST, bool LAST>
struct OpChebS {
  static constexpr const char *NAME = "cheb_S";
  static constexpr int VARIANT = (FIRST ? 1 : 0) + (LAST ? 2 : 0);
  static constexpr bool ZERO_BC = true;
  const T *w;        // velocity input
  const T *rin;      // r_0 (FIRST) or r_i
  const T *dinv_s;
  const T *d;        // d_i (not FIRST)
  const T *x;        // x_i (not FIRST)
  T *r_out, *x_out, *d_out;
  T *p, *dp;         // LAST
  T inv_theta, c1, c2, tau;
  template <class I>
  __device__ T load_u(I i) const { return at(w, i); }
  template <class I>
  __device__ T load_p(I i) const {
    if constexpr (FIRST) return at(dinv_s, i) * at(rin, i) * inv_theta;
    else return at(d, i);
  }
  struct Pre {
    T r, x, d, dinv, p;
  };
  template <class I>
  __device__ Pre fetch_u(I) const { return Pre{}; }
  template <class I>
  __device__ Pre fetch_p(I i) const {
    Pre q;
    q.r = at(rin, i);
    q.dinv = at(dinv_s, i);
    q.x = FIRST ? T(0) : at(x, i);
    q.d = FIRST ? q.dinv * q.r * inv_theta : at(d, i);
    q.p = (LAST && p) ? at(p, i) : T(0);
    return q;
  }
  template <class I>
  __device__ void store_u(I, T, T, bool, const Pre &) const {}
  template <class I>
  __device__ void store_p(I i, T t, T, const Pre &q) const {
    const T di = q.d;
    const T rn = q.r - t;
    const T xn = q.x + di;
    const T dn = c1 * di + c2 * q.dinv * rn;
    if constexpr (LAST) {
      const T delta = tau * (xn + dn);
      at(dp, i) = delta;
      if (p) at(p, i) = q.p + delta;
    } else {
      at(r_out, i) = rn;
      at(x_out, i) = xn;
      at(d_out, i) = dn;
    }
  }
  double algo_bytes(bool, bool, bool, bool, double nu, double np) const {
    const double reads = FIRST ? 2 : 4, writes = LAST ? (p ? 3 : 1) : 3;
    return sizeof(T) * (nu + np * (reads + writes));
  }
};

// Lifting of non-homogeneous Dirichlet data: with t = K u~ for the operator
// with its Dirichlet columns kept (ZERO_BC off) and u~ the Dirichlet values
// extended by zero,
//   b_u <- b_u - t_u on free rows and 0 on Dirichlet rows,  b_p <- b_p - t_p.
// b may be updated in place (each entry is read and written by one lane).
template <typename T>
struct OpLift {
  static constexpr const char *NAME = "lift";
  static constexpr int VARIANT = 0;
  static constexpr bool ZERO_BC = false;
  const T *ud;          // u~ (zero off the Dirichlet nodes)
  const T *bu, *bp;
  T *yu, *yp;
  struct Pre {
    T b;
  };
  template <class I>
  __device__ T load_u(I i) const { return at(ud, i); }
  template <class I>
  __device__ T load_p(I) const { return 0; }
  template <class I>
  __device__ Pre fetch_u(I i) const { return Pre{at(bu, i)}; }
  template <class I>
  __device__ Pre fetch_p(I i) const { return Pre{at(bp, i)}; }
  template <class I>
  __device__ void store_u(I i, T t, T, bool bc, const Pre &q) const { at(yu, i) = bc ? T(0) : q.b - t; }
  template <class I>
  __device__ void store_p(I i, T t, T, const Pre &q) const { at(yp, i) = q.b - t; }
  double algo_bytes(bool, bool, bool, bool, double nu, double np) const { return sizeof(T) * (3 * nu + 2 * np); }
};

// r_p = B u - C p - g, the argument of the second Uzawa update.
template <typename T>
struct OpDivResidual {
  static constexpr const char *NAME = "div_residual";
  static constexpr int VARIANT = 0;
  static constexpr bool ZERO_BC = true;
  const T *u, *p_in, *g;
  T *rp;
  template <class I>
  __device__ T load_u(I i) const { return at(u, i); }
  template <class I>
  __device__ T load_p(I i) const { return at(p_in, i); }
  struct Pre {
    T g;
  };
  template <class I>
  __device__ Pre fetch_u(I) const { return Pre{}; }
  template <class I>
  __device__ Pre fetch_p(I i) const { return Pre{g ? at(g, i) : T(0)}; }
  template <class I>
  __device__ void store_u(I, T, T, bool, const Pre &) const {}
  template <class I>
  __device__ void store_p(I i, T t, T, const Pre &q) const { at(rp, i) = t - q.g; }
  double algo_bytes(bool, bool need_p, bool, bool, double nu, double np) const {
    return sizeof(T) * (nu + (need_p ? np : 0) + (g ? np : 0) + np);
  }
};

}  // namespace smg
