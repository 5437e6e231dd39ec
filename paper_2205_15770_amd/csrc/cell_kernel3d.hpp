// Column-sweep application of the Taylor-Hood saddle-point operator
// K = [A B^T; B -C] on axis-aligned box cells in 3D (Sec. 3.1: K x =
// sum_tau P_tau K_tau P_tau^T x, cell matrices by sum factorisation).
//
// Work decomposition (gfx950): one wave64 per (tile of 8 x 8 cell columns,
// z chunk, output field).  Lane l holds the cell column (l % 8, l / 8) of the
// tile and sweeps the cells of its column through the chunk in z.  A tile
// owns 7 x 7 columns; lane column 0 and lane row 0 are halo columns, and the
// cell layer below a chunk is a halo layer: their cell results are computed
// only to hand them over.  No LDS, no barriers, no atomics; every output
// entry is written once, from complete cell sums.
//
//   velocity wave (field c < 3):  y_c = (A u)_c + (B^T p)_c
//   pressure wave (field 3):      y_p = B u -/+ C p
//
// Cell results on nodes shared with the neighbours are handed over in three
// steps: the x = K face to lane + 1 and the y = K face to lane + 8 by lane
// shuffles, the z = K face to the next cell of the column in registers.  After
// that a cell holds the complete sums of its nodes with local indices [0, K)
// in every direction (plus the domain high faces), which it writes through the
// epilogue functor.  The DoFs of the next cell layer are requested before the
// current layer is computed; the z = 0 plane of a layer is the z = K plane of
// the layer below and is not read again.
#pragma once
#include "cell_kernel.hpp"

namespace smg {

template <int K, typename T>
struct Column3D {
  static constexpr int NV = K + 1, NP = K;
  const LevelGeom<T, 3, K> &g;
  int gcx, gcy;      // cell column
  bool active;       // column inside the mesh
  bool bx, by;       // column's low node on the x / y boundary (per node below)
  __device__ i64 vidx(int c, int gx, int gy, int gz) const {
    return (i64)c * g.Nv + gx + (i64)g.vd[0] * (gy + (i64)g.vd[1] * gz);
  }
  __device__ i64 pidx(int gx, int gy, int gz) const {
    return gx + (i64)g.pd[0] * (gy + (i64)g.pd[1] * gz);
  }
  __device__ bool vbc(int gx, int gy, int gz) const {
    return on_box_boundary(gx, g.vd[0]) || on_box_boundary(gy, g.vd[1]) || on_box_boundary(gz, g.vd[2]);
  }
  // planes [Z0, NV) of velocity component c of cell layer cz into dst[z - Z0]
  template <int Z0, class Op, int NZ>
  __device__ void load_u(const Op &op, int c, int cz, T (&dst)[NZ][NV][NV]) const {
    static_assert(NZ == NV - Z0, "plane count");
#pragma unroll
    for (int z = Z0; z < NV; ++z)
#pragma unroll
      for (int y = 0; y < NV; ++y)
#pragma unroll
        for (int x = 0; x < NV; ++x) {
          T v = 0;
          const int gx = K * gcx + x, gy = K * gcy + y, gz = K * cz + z;
          if (active && !(Op::ZERO_BC && vbc(gx, gy, gz))) v = op.load_u(vidx(c, gx, gy, gz));
          dst[z - Z0][y][x] = v;
        }
  }
  template <int Z0, class Op, int NZ>
  __device__ void load_p(const Op &op, int cz, T (&dst)[NZ][NP][NP]) const {
    static_assert(NZ == NP - Z0, "plane count");
#pragma unroll
    for (int z = Z0; z < NP; ++z)
#pragma unroll
      for (int y = 0; y < NP; ++y)
#pragma unroll
        for (int x = 0; x < NP; ++x) {
          T v = 0;
          if (active) v = op.load_p(pidx((K - 1) * gcx + x, (K - 1) * gcy + y, (K - 1) * cz + z));
          dst[z - Z0][y][x] = v;
        }
  }
};

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
      const T r = __shfl_up(y[z][j][N - 1], 1, TX);
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

template <int K, typename T, int BLK, class Op, int TX, int TY>
__global__ void __launch_bounds__(64)
tile3d_kernel(const LevelGeom<T, 3, K> g, const Op op) {
  constexpr int NV = K + 1, NP = K;
  static_assert(TX * TY == 64, "one wave per tile");
  constexpr bool OUT_U = (BLK & (BLK_A | BLK_MASS | BLK_BT)) != 0;
  constexpr bool OUT_P = (BLK & (BLK_B | BLK_C)) != 0;
  constexpr int NFIELD = (OUT_U ? 3 : 0) + (OUT_P ? 1 : 0);
  constexpr bool V_NEED_U = (BLK & (BLK_A | BLK_MASS)) != 0;
  constexpr bool V_NEED_P = (BLK & BLK_BT) != 0;
  constexpr bool P_NEED_U = (BLK & BLK_B) != 0;
  constexpr bool P_NEED_P = (BLK & BLK_C) != 0;

  // block -> (field, x tile, z chunk, y tile); the fields of one tile and
  // chunk run on the same XCD and share its L2.
  const int b = xcd_contiguous_tile(blockIdx.x, gridDim.x);
  const int field = b % NFIELD;
  int rest = b / NFIELD;
  const int tx = rest % g.tiles[0];
  rest /= g.tiles[0];
  const int zc = rest % g.tiles[2];
  const int ty = rest / g.tiles[2];
  const int zlen = (g.n[2] + g.tiles[2] - 1) / g.tiles[2];
  const int z_lo = zc * zlen;
  const int z_hi = z_lo + zlen < g.n[2] ? z_lo + zlen : g.n[2];
  if (z_lo >= z_hi) return;  // whole wave: empty chunk
  const int z_start = z_lo > 0 ? z_lo - 1 : 0;

  const int lane = threadIdx.x;
  const int lcx = lane % TX, lcy = lane / TX;
  Column3D<K, T> col{g, tx * (TX - 1) - 1 + lcx, ty * (TY - 1) - 1 + lcy, false, false, false};
  col.active = col.gcx >= 0 && col.gcx < g.n[0] && col.gcy >= 0 && col.gcy < g.n[1];
  const bool col_owner = col.active && lcx > 0 && lcy > 0;
  const bool last_x = col.gcx == g.n[0] - 1, last_y = col.gcy == g.n[1] - 1;
  const Coef1D<T, K> &cx = g.c[0];
  const Coef1D<T, K> &cy = g.c[1];
  const Coef1D<T, K> &cz = g.c[2];

  if (OUT_U && field < 3) {
    // ------------------------------------------------------ velocity wave
    const int comp = field;
    T u[NV][NV][NV], un[K][NV][NV];
    T p[NP][NP][NP], pn[NP - 1][NP][NP];
    T carry[NV][NV];
#pragma unroll
    for (int j = 0; j < NV; ++j)
#pragma unroll
      for (int i = 0; i < NV; ++i) carry[j][i] = 0;
    if constexpr (V_NEED_U) {
      col.template load_u<0>(op, comp, z_start, u);
    } else {
#pragma unroll
      for (int z = 0; z < NV; ++z)
#pragma unroll
        for (int j = 0; j < NV; ++j)
#pragma unroll
          for (int i = 0; i < NV; ++i) u[z][j][i] = 0;
    }
    if constexpr (V_NEED_P) col.template load_p<0>(op, z_start, p);
    // B_c^T = -(N^T or G^T per direction): G in direction comp
    const auto &Bx = comp == 0 ? cx.G : cx.N;
    const auto &By = comp == 1 ? cy.G : cy.N;
    const auto &Bz = comp == 2 ? cz.G : cz.N;

    for (int cl = z_start; cl < z_hi; ++cl) {
      const bool more = cl + 1 < z_hi;
      if (more) {
        if constexpr (V_NEED_U) col.template load_u<1>(op, comp, cl + 1, un);
        if constexpr (V_NEED_P) col.template load_p<1>(op, cl + 1, pn);
      }
      const bool owner = col_owner && cl >= z_lo;
      const bool last_z = cl == g.n[2] - 1;
      // epilogue inputs of the owned nodes [0,K)^3
      typename Op::Pre pre[K][K][K];
      T raw[K][K][K];
      if (owner) {
#pragma unroll
        for (int z = 0; z < K; ++z)
#pragma unroll
          for (int y = 0; y < K; ++y)
#pragma unroll
            for (int x = 0; x < K; ++x) {
              const int gx = K * col.gcx + x, gy = K * col.gcy + y, gz = K * cl + z;
              const i64 gi = col.vidx(comp, gx, gy, gz);
              pre[z][y][x] = op.fetch_u(gi);
              raw[z][y][x] = 0;
              if constexpr ((BLK & BLK_A) != 0)
                if (gx == 0 || gy == 0 || gz == 0) raw[z][y][x] = op.load_u(gi);
            }
      }
      T mu = g.mu;
      if (g.mu_cell != nullptr && col.active) mu = g.mu_cell[col.gcx + (i64)g.n[0] * (col.gcy + (i64)g.n[1] * cl)];

      T y[NV][NV][NV];
      if constexpr ((BLK & BLK_A) != 0) {
        T X[NV][NV];
#pragma unroll
        for (int i = 0; i < NV; ++i)
#pragma unroll
          for (int j = 0; j < NV; ++j) X[i][j] = mu * cx.Kv[i][j] + g.gr * cx.Mv[i][j];
        T a[NV][NV][NV], t[NV][NV][NV];
        pass_z<false, false>(cz.Mv, u, a, T(1));
        pass_y<false, false>(cy.Mv, a, t, T(1));
        pass_x<false, false>(X, t, y, T(1));
        pass_y<false, false>(cy.Kv, a, t, mu);
        pass_z<false, false>(cz.Kv, u, a, mu);
        pass_y<false, true>(cy.Mv, a, t, T(1));
        pass_x<false, true>(cx.Mv, t, y, T(1));
      } else if constexpr ((BLK & BLK_MASS) != 0) {
        T a[NV][NV][NV], t[NV][NV][NV];
        pass_z<false, false>(cz.Mv, u, a, T(1));
        pass_y<false, false>(cy.Mv, a, t, T(1));
        pass_x<false, false>(cx.Mv, t, y, T(1));
      }
      if constexpr ((BLK & BLK_BT) != 0) {
        constexpr bool ACC = (BLK & (BLK_A | BLK_MASS)) != 0;
        T s1[NV][NP][NP], s2[NV][NV][NP];
        pass_z<true, false>(Bz, p, s1, T(1));
        pass_y<true, false>(By, s1, s2, T(1));
        pass_x<true, ACC>(Bx, s2, y, T(-1));
      }
      hand_over_xy<TX>(y, lcx, lcy, last_x, last_y);
#pragma unroll
      for (int j = 0; j < NV; ++j)
#pragma unroll
        for (int i = 0; i < NV; ++i) {
          y[0][j][i] += carry[j][i];
          carry[j][i] = y[K][j][i];
        }
      if (owner) {
#pragma unroll
        for (int z = 0; z < K; ++z)
#pragma unroll
          for (int yy = 0; yy < K; ++yy)
#pragma unroll
            for (int x = 0; x < K; ++x) {
              const int gx = K * col.gcx + x, gy = K * col.gcy + yy, gz = K * cl + z;
              const i64 gi = col.vidx(comp, gx, gy, gz);
              if (gx == 0 || gy == 0 || gz == 0) op.store_u(gi, raw[z][yy][x], raw[z][yy][x], true, pre[z][yy][x]);
              else op.store_u(gi, y[z][yy][x], u[z][yy][x], false, pre[z][yy][x]);
            }
        if (last_x || last_y || last_z) {
          // nodes on the domain's high faces: Dirichlet rows
#pragma unroll
          for (int z = 0; z < NV; ++z)
#pragma unroll
            for (int yy = 0; yy < NV; ++yy)
#pragma unroll
              for (int x = 0; x < NV; ++x) {
                if (x < K && yy < K && z < K) continue;
                if ((x == K && !last_x) || (yy == K && !last_y) || (z == K && !last_z)) continue;
                const i64 gi = col.vidx(comp, K * col.gcx + x, K * col.gcy + yy, K * cl + z);
                T rw = 0;
                if constexpr ((BLK & BLK_A) != 0) rw = op.load_u(gi);
                op.store_u(gi, rw, rw, true, op.fetch_u(gi));
              }
        }
      }
      if (more) {
#pragma unroll
        for (int j = 0; j < NV; ++j)
#pragma unroll
          for (int i = 0; i < NV; ++i) u[0][j][i] = u[K][j][i];
#pragma unroll
        for (int z = 1; z < NV; ++z)
#pragma unroll
          for (int j = 0; j < NV; ++j)
#pragma unroll
            for (int i = 0; i < NV; ++i) u[z][j][i] = un[z - 1][j][i];
        if constexpr (V_NEED_P) {
#pragma unroll
          for (int j = 0; j < NP; ++j)
#pragma unroll
            for (int i = 0; i < NP; ++i) p[0][j][i] = p[NP - 1][j][i];
#pragma unroll
          for (int z = 1; z < NP; ++z)
#pragma unroll
            for (int j = 0; j < NP; ++j)
#pragma unroll
              for (int i = 0; i < NP; ++i) p[z][j][i] = pn[z - 1][j][i];
        }
      }
    }
  } else if constexpr (OUT_P) {
    // ------------------------------------------------------ pressure wave
    T carry[NP][NP];
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
      for (int i = 0; i < NP; ++i) carry[j][i] = 0;
    T p[NP][NP][NP];
#pragma unroll
    for (int z = 0; z < NP; ++z)
#pragma unroll
      for (int j = 0; j < NP; ++j)
#pragma unroll
        for (int i = 0; i < NP; ++i) p[z][j][i] = 0;
    for (int cl = z_start; cl < z_hi; ++cl) {
      const bool owner = col_owner && cl >= z_lo;
      const bool last_z = cl == g.n[2] - 1;
      typename Op::Pre pre[K - 1][K - 1][K - 1];
      if (owner) {
#pragma unroll
        for (int z = 0; z < K - 1; ++z)
#pragma unroll
          for (int yy = 0; yy < K - 1; ++yy)
#pragma unroll
            for (int x = 0; x < K - 1; ++x)
              pre[z][yy][x] = op.fetch_p(col.pidx((K - 1) * col.gcx + x, (K - 1) * col.gcy + yy, (K - 1) * cl + z));
      }
      if constexpr (P_NEED_P) col.template load_p<0>(op, cl, p);
      T yp[NP][NP][NP];
#pragma unroll
      for (int z = 0; z < NP; ++z)
#pragma unroll
        for (int j = 0; j < NP; ++j)
#pragma unroll
          for (int i = 0; i < NP; ++i) yp[z][j][i] = 0;
      if constexpr (P_NEED_U) {
        // B u = -sum_c (G or N per direction) u_c, one component at a time
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          T u[NV][NV][NV];
          col.template load_u<0>(op, c, cl, u);
          T w1[NV][NV][NP], w2[NV][NP][NP];
          pass_x<false, false>(c == 0 ? cx.G : cx.N, u, w1, T(1));
          pass_y<false, false>(c == 1 ? cy.G : cy.N, w1, w2, T(1));
          pass_z<false, true>(c == 2 ? cz.G : cz.N, w2, yp, T(-1));
        }
      }
      if constexpr (P_NEED_P) {
        const T sc = (BLK & BLK_CPLUS) ? g.cp : -g.cp;
        T q1[NP][NP][NP], q2[NP][NP][NP];
        pass_x<false, false>(cx.Mp, p, q1, T(1));
        pass_y<false, false>(cy.Mp, q1, q2, T(1));
        pass_z<false, true>(cz.Mp, q2, yp, sc);
      }
      hand_over_xy<TX>(yp, lcx, lcy, last_x, last_y);
#pragma unroll
      for (int j = 0; j < NP; ++j)
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          yp[0][j][i] += carry[j][i];
          carry[j][i] = yp[NP - 1][j][i];
        }
      if (owner) {
#pragma unroll
        for (int z = 0; z < NP; ++z)
#pragma unroll
          for (int yy = 0; yy < NP; ++yy)
#pragma unroll
            for (int x = 0; x < NP; ++x) {
              const bool main = x < K - 1 && yy < K - 1 && z < K - 1;
              if (!main && ((x == K - 1 && !last_x) || (yy == K - 1 && !last_y) || (z == K - 1 && !last_z))) continue;
              const i64 gi = col.pidx((K - 1) * col.gcx + x, (K - 1) * col.gcy + yy, (K - 1) * cl + z);
              if (main) op.store_p(gi, yp[z][yy][x], p[z][yy][x], pre[main ? z : 0][main ? yy : 0][main ? x : 0]);
              else op.store_p(gi, yp[z][yy][x], p[z][yy][x], op.fetch_p(gi));
            }
      }
    }
  }
}

}  // namespace smg
