// Building blocks shared by the wave-tile operator kernels (Sec. 3.1: K x =
// sum_tau P_tau K_tau P_tau^T x by cell-wise sum factorisation): the operator
// block flags, the XCD-aware block-to-tile map and the lane hand-over of the
// contributions to nodes shared with the neighbouring cells.
#pragma once
#include "common.hpp"

namespace smg {

enum : int { BLK_A = 1, BLK_MASS = 2, BLK_BT = 4, BLK_B = 8, BLK_C = 16, BLK_CPLUS = 32 };

// Bijection blockIdx -> tile such that the blocks of one XCD (b % 8 == k) take
// the contiguous tile range [prefix_k, prefix_k + count_k).
__host__ __device__ __forceinline__ int xcd_contiguous_tile(int b, int nb) {
  constexpr int NXCD = 8;
  const int k = b % NXCD;
  int prefix = 0;
  for (int j = 0; j < k; ++j) prefix += (nb - j + NXCD - 1) / NXCD;
  return prefix + b / NXCD;
}

// Hand the x = N-1 and y = N-1 faces of a cell array to the neighbouring lanes
// (x: lane + 1 within a row of TX lanes, y: lane + TX) and add what arrives
// from the other side to the x = 0 / y = 0 faces.  Faces that were handed
// over are cleared unless they lie on the domain's high boundary.
template <int TX, typename T, int NZ, int N>
__device__ __forceinline__ void hand_over_xy(T (&y)[NZ][N][N], int lcx, int lcy, bool last_x, bool last_y) {
#pragma unroll
  for (int z = 0; z < NZ; ++z)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      // x neighbour: lane - 1 (its value is used only where lcx > 0, i.e. by
      // lanes whose lane - 1 is in the same row of TX lanes)
      const T r = __shfl_up(y[z][j][N - 1], 1, (TX & (TX - 1)) == 0 ? TX : 64);
      if (lcx > 0) y[z][j][0] += r;
      if (!last_x) y[z][j][N - 1] = 0;
    }
#pragma unroll
  for (int z = 0; z < NZ; ++z)
#pragma unroll
    for (int i = 0; i < N; ++i) {
      const T r = __shfl_up(y[z][N - 1][i], TX, 64);
      if (lcy > 0) y[z][0][i] += r;
      if (!last_y) y[z][N - 1][i] = 0;
    }
}

}  // namespace smg
