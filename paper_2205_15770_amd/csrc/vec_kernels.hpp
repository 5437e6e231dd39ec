// Element-wise, reduction, transfer, diagonal and coarse-solve kernels.
#pragma once
#include "common.hpp"

namespace smg {

constexpr int VB = 256;  // threads per block of the element-wise kernels

inline unsigned grid_for(i64 n, int per_block = VB) {
  i64 g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > 1048576) g = 1048576;
  return (unsigned)g;
}

template <typename T>
__global__ void k_set(T *y, T v, i64 n) { SMG_GRID_LOOP(i, n) y[i] = v; }

template <typename TO, typename TI>
__global__ void k_copy(TO *y, const TI *x, i64 n) { SMG_GRID_LOOP(i, n) y[i] = (TO)x[i]; }

// y += a x
template <typename T>
__global__ void k_axpy(T *y, T a, const T *x, i64 n) { SMG_GRID_LOOP(i, n) y[i] += a * x[i]; }

// y = x + a z (TO output, any input types)
template <typename TO, typename TI>
__global__ void k_add_scaled(TO *y, const TI *x, TO a, const TO *z, i64 n) {
  SMG_GRID_LOOP(i, n) y[i] = (TO)x[i] + a * z[i];
}

// out = base + s * dinv * r   (Chebyshev of degree 0: damped Jacobi)
template <typename T>
__global__ void k_jacobi(T *out, const T *base, T s, const T *dinv, const T *r, i64 n) {
  SMG_GRID_LOOP(i, n) out[i] = (base ? base[i] : T(0)) + s * dinv[i] * r[i];
}

// p += dp, dp = s * dinv * r
template <typename T>
__global__ void k_jacobi_update(T *p, T *dp, T s, const T *dinv, const T *r, i64 n) {
  SMG_GRID_LOOP(i, n) {
    const T d = s * dinv[i] * r[i];
    dp[i] = d;
    p[i] += d;
  }
}

template <typename TO>
__global__ void k_reciprocal(TO *y, const double *x, i64 n) { SMG_GRID_LOOP(i, n) y[i] = (TO)(1.0 / x[i]); }

// ---------------------------------------------------------------------------
// deterministic reductions: fixed partition into RB blocks, per-block tree
// sums (wave64 shuffles, then LDS), then one block sums the partials in order.
// ---------------------------------------------------------------------------
constexpr int RB = 512;   // number of partial sums

template <typename T>
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double sm[VB / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sm[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < VB / 64; ++w) s += sm[w];
  }
  __syncthreads();
  return s;
}

// partial[b * nv + j] = sum over the chunk of block b of V_j[i] * w[i]
// (V_j = V + j * ldv), for j < nv; FP64 accumulation.
template <typename T>
__global__ void __launch_bounds__(VB) k_multidot_partial(const T *V, i64 ldv, int nv, const T *w, i64 n, double *partial) {
  const i64 chunk = (n + gridDim.x - 1) / gridDim.x;
  const i64 lo = (i64)blockIdx.x * chunk;
  const i64 hi = lo + chunk < n ? lo + chunk : n;
  for (int j = 0; j < nv; ++j) {
    const T *v = V + (i64)j * ldv;
    double s = 0.0;
    for (i64 i = lo + threadIdx.x; i < hi; i += VB) s += (double)v[i] * (double)w[i];
    s = block_sum<T>(s);
    if (threadIdx.x == 0) partial[(i64)blockIdx.x * nv + j] = s;
  }
}

// out[j] = sum_b partial[b * nv + j]: one block per j, fixed-order tree sum.
static __global__ void __launch_bounds__(VB) k_partial_finish(const double *partial, int nblocks, int nv, double *out) {
  const int j = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += VB) s += partial[(i64)b * nv + j];
  s = block_sum<double>(s);
  if (threadIdx.x == 0) out[j] = s;
}

// w *= 1 / sqrt(s2[0])  (normalisation by a norm that stays on the device)
template <typename T>
__global__ void k_scale_inv_sqrt(T *w, const double *s2, i64 n) {
  const double v = s2[0];
  const double f = v > 0.0 ? 1.0 / sqrt(v) : 0.0;
  SMG_GRID_LOOP(i, n) w[i] = (T)((double)w[i] * f);
}

// w -= sum_j h[j] V_j  (h on the device)
template <typename T>
__global__ void k_multi_axpy(T *w, const T *V, i64 ldv, int nv, const double *h, double sign, i64 n) {
  SMG_GRID_LOOP(i, n) {
    double s = 0.0;
    for (int j = 0; j < nv; ++j) s += h[j] * (double)V[(i64)j * ldv + i];
    w[i] = (T)((double)w[i] + sign * s);
  }
}

// The same reductions and updates as launch functors (packed launches over
// many problems, see packed.hpp); identical arithmetic and summation order.
template <typename T>
struct LMultidotPartial {
  static constexpr int THREADS = VB;
  const T *V;
  i64 ldv;
  int nv;
  const T *w;
  i64 n;
  double *partial;
  __device__ void run(int b, int nb) const {
    const i64 chunk = (n + nb - 1) / nb;
    const i64 lo = (i64)b * chunk;
    const i64 hi = lo + chunk < n ? lo + chunk : n;
    for (int j = 0; j < nv; ++j) {
      const T *v = V + (i64)j * ldv;
      double s = 0.0;
      for (i64 i = lo + threadIdx.x; i < hi; i += VB) s += (double)v[i] * (double)w[i];
      s = block_sum<T>(s);
      if (threadIdx.x == 0) partial[(i64)b * nv + j] = s;
    }
  }
};

struct LPartialFinish {
  static constexpr int THREADS = VB;
  const double *partial;
  int nblocks, nv;
  double *out;
  __device__ void run(int j, int) const {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += VB) s += partial[(i64)b * nv + j];
    s = block_sum<double>(s);
    if (threadIdx.x == 0) out[j] = s;
  }
};

template <typename T>
struct LMultiAxpy {
  static constexpr int THREADS = VB;
  T *w;
  const T *V;
  i64 ldv;
  int nv;
  const double *h;
  double sign;
  i64 n;
  __device__ void run(int b, int nb) const {
    for (i64 i = (i64)b * VB + threadIdx.x; i < n; i += (i64)nb * VB) {
      double s = 0.0;
      for (int j = 0; j < nv; ++j) s += h[j] * (double)V[(i64)j * ldv + i];
      w[i] = (T)((double)w[i] + sign * s);
    }
  }
};

template <typename T>
struct LScaleInvSqrt {
  static constexpr int THREADS = VB;
  T *w;
  const double *s2;
  i64 n;
  __device__ void run(int b, int nb) const {
    const double v = s2[0];
    const double f = v > 0.0 ? 1.0 / sqrt(v) : 0.0;
    for (i64 i = (i64)b * VB + threadIdx.x; i < n; i += (i64)nb * VB) w[i] = (T)((double)w[i] * f);
  }
};

// x0 = Kinv[0:N0, 0:N0] b0 (coarse solve), one wave per row
template <typename T>
struct LCoarseGemv {
  static constexpr int THREADS = VB;
  const double *Kinv;
  i64 ld;
  int n0;
  const T *b;
  T *x;
  __device__ void run(int blk, int) const {
    const int row = blk * (VB / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (row >= n0) return;
    double s = 0.0;
    for (int c = lane; c < n0; c += 64) s += Kinv[(i64)row * ld + c] * (double)b[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
    if (lane == 0) x[row] = (T)s;
  }
};

// ---------------------------------------------------------------------------
// transfers (Sec. 3.2): canonical injection P per field, R = P^T
// ---------------------------------------------------------------------------
// 1D prolongation weights of both fields (host tables, see transfer kernels)
struct TransferTables {
  double W[2][7 * 4];   // W[field][f * (deg+1) + j], f = 0..2deg; field 0 = velocity, 1 = pressure
};

// ---------------------------------------------------------------------------
// coarse solve: x0 = Kinv[0:N0, 0:N0] b0 (border column multiplies zero),
// FP64 arithmetic for any T; one wave per row.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(VB) k_coarse_gemv(const double *Kinv, i64 ld, int n0, const T *b, T *x) {
  const int row = blockIdx.x * (VB / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n0) return;
  double s = 0.0;
  for (int c = lane; c < n0; c += 64) s += Kinv[(i64)row * ld + c] * (double)b[c];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) x[row] = (T)s;
}

// p -= (w . p) / (w . 1) with w = M_p 1 given, for pressure mean removal
static __global__ void k_subtract_scalar(double *p, const double *scal, double denom, i64 n) {
  const double m = scal[0] / denom;
  SMG_GRID_LOOP(i, n) p[i] -= m;
}

// g -= w (1 . g) / (w . 1): the transpose of the mean removal above
static __global__ void k_subtract_weighted(double *g, const double *w, const double *scal, double denom, i64 n) {
  const double m = scal[0] / denom;
  SMG_GRID_LOOP(i, n) g[i] -= w[i] * m;
}

}  // namespace smg
