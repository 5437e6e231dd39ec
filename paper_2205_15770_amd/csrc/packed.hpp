// Launch functors and packed launches.
//
// A launch functor L holds the arguments of one kernel launch and the body:
//   static constexpr int THREADS;                 threads per block
//   __device__ void run(int b, int nb) const;     block b of nb
// k_one<L> runs one functor over its grid (the ordinary launch).  k_packed<L>
// runs many functors of the same type in one launch, e.g. the same operator
// stage of many independent problems: a table of functors, the first block of
// each (a multiple of 8, so that block b of a functor runs on the XCD that
// b % 8 names, as in a launch of its own) and its block count; block B runs
// block B - first[e] of functor e with first[e] <= B < first[e + 1].
#pragma once
#include "common.hpp"

namespace smg {

template <class L>
__global__ void __launch_bounds__(L::THREADS) k_one(const L l) {
  l.run((int)blockIdx.x, (int)gridDim.x);
}

template <class L>
__global__ void __launch_bounds__(L::THREADS)
k_packed(const L *__restrict__ ls, const uint32_t *__restrict__ first, const uint32_t *__restrict__ count, int n) {
  const uint32_t B = blockIdx.x;
  int lo = 0, hi = n - 1;
  while (lo < hi) {   // last entry with first[e] <= B (wave-uniform)
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= B) lo = mid;
    else hi = mid - 1;
  }
  const int b = (int)(B - first[lo]);
  const int nb = (int)count[lo];
  if (b >= nb) return;   // alignment padding
  const L l = ls[lo];
  l.run(b, nb);
}

// ------------------------------------------------- element-wise functors
template <typename T>
struct LSet {
  static constexpr int THREADS = 256;
  T *y;
  T v;
  i64 n;
  __device__ void run(int b, int nb) const {
    for (i64 i = (i64)b * THREADS + threadIdx.x; i < n; i += (i64)nb * THREADS) y[i] = v;
  }
};

template <typename TO, typename TI>
struct LCopy {
  static constexpr int THREADS = 256;
  TO *y;
  const TI *x;
  i64 n;
  __device__ void run(int b, int nb) const {
    for (i64 i = (i64)b * THREADS + threadIdx.x; i < n; i += (i64)nb * THREADS) y[i] = (TO)x[i];
  }
};

// out = base + s * dinv * r
template <typename T>
struct LJacobi {
  static constexpr int THREADS = 256;
  T *out;
  const T *base;
  T s;
  const T *dinv, *r;
  i64 n;
  __device__ void run(int b, int nb) const {
    for (i64 i = (i64)b * THREADS + threadIdx.x; i < n; i += (i64)nb * THREADS)
      out[i] = (base ? base[i] : T(0)) + s * dinv[i] * r[i];
  }
};

// p += dp, dp = s * dinv * r
template <typename T>
struct LJacobiUpdate {
  static constexpr int THREADS = 256;
  T *p, *dp;
  T s;
  const T *dinv, *r;
  i64 n;
  __device__ void run(int b, int nb) const {
    for (i64 i = (i64)b * THREADS + threadIdx.x; i < n; i += (i64)nb * THREADS) {
      const T d = s * dinv[i] * r[i];
      dp[i] = d;
      p[i] += d;
    }
  }
};

inline unsigned grid_for_n(i64 n, int per_block = 256) {
  i64 g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > 1048576) g = 1048576;
  return (unsigned)g;
}

}  // namespace smg
