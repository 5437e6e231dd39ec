// Tiled, cell-wise sum-factorised application of the Taylor-Hood saddle-point
// operator K = [A B^T; B -C] on axis-aligned box cells (Sec. 3.1: K x =
// sum_tau P_tau K_tau P_tau^T x; Sec. 2: the forms a and b).
//
// Work decomposition (gfx950): one workgroup per tile of (TX-1) x (TY-1)
// [x (TZ-1)] owned cells plus one halo layer of cells on the low side of each
// direction, one cell per thread.  A tile owns the DoF lattice nodes of its
// cells except those on its high faces (they belong to the next tile), so
// every output entry is produced by exactly one workgroup from complete cell
// sums: no atomics, no second pass, bit-reproducible results.  The halo cells
// supply the contributions of the neighbouring tile to the owned low-face
// nodes.
//
//   1. the DoF patch of the tile is read from HBM with x-contiguous
//      (coalesced) loads into LDS; Dirichlet inputs are zeroed;
//   2. each thread gathers its cell's values from LDS and applies the cell
//      matrices by sum factorisation (1D passes in registers);
//   3. cell results are added into an LDS output patch in 2^d colour phases
//      (cells of equal index parity share no node);
//   4. the owned nodes are written through an epilogue functor, which fuses
//      the vector algebra of the caller (residual, Chebyshev recurrence,
//      Uzawa updates) into the same pass over memory.
#pragma once
#include "common.hpp"

namespace smg {

enum : int { BLK_A = 1, BLK_MASS = 2, BLK_BT = 4, BLK_B = 8, BLK_C = 16, BLK_CPLUS = 32 };

template <int DIM, int K>
struct Shape {
  static constexpr int NV = K + 1, NP = K;
  static constexpr int VZ = DIM == 3 ? NV : 1, PZ = DIM == 3 ? NP : 1;
};

// Cell matrices applied to one cell's DoFs (registers).
//   yu_c = mu (Kx Mx... Kronecker sum) u_c + gr M u_c - B_c^T p      (BLK_A, BLK_BT)
//   yp   = sum_c B_c u_c -/+ cp M_p p                                (BLK_B, BLK_C)
// with B_c = - N (x) ... (x) G (direction c) (x) ... N.
template <int DIM, int K, typename T, int BLK>
__device__ __forceinline__ void cell_apply(const LevelGeom<T, DIM, K> &g, T mu,
                                           const T (&u)[DIM][Shape<DIM, K>::VZ][K + 1][K + 1],
                                           const T (&p)[Shape<DIM, K>::PZ][K][K],
                                           T (&yu)[DIM][Shape<DIM, K>::VZ][K + 1][K + 1],
                                           T (&yp)[Shape<DIM, K>::PZ][K][K]) {
  constexpr int NV = K + 1, NP = K, VZ = Shape<DIM, K>::VZ, PZ = Shape<DIM, K>::PZ;
  const Coef1D<T, K> &cx = g.c[0];
  const Coef1D<T, K> &cy = g.c[1];
  if constexpr (BLK & BLK_A) {
    T X[NV][NV];
#pragma unroll
    for (int i = 0; i < NV; ++i)
#pragma unroll
      for (int j = 0; j < NV; ++j) X[i][j] = mu * cx.Kv[i][j] + g.gr * cx.Mv[i][j];
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      T b[VZ][NV][NV], b2[VZ][NV][NV];
      if constexpr (DIM == 2) {
        pass_y<false, false>(cy.Mv, u[c], b, T(1));
        pass_y<false, false>(cy.Kv, u[c], b2, T(1));
      } else {
        const Coef1D<T, K> &cz = g.c[DIM - 1];
        T a[VZ][NV][NV];
        pass_z<false, false>(cz.Mv, u[c], a, T(1));
        pass_y<false, false>(cy.Mv, a, b, T(1));
        pass_y<false, false>(cy.Kv, a, b2, T(1));
        pass_z<false, false>(cz.Kv, u[c], a, T(1));
        pass_y<false, true>(cy.Mv, a, b2, T(1));
      }
      pass_x<false, false>(X, b, yu[c], T(1));
      pass_x<false, true>(cx.Mv, b2, yu[c], mu);
    }
  } else if constexpr (BLK & BLK_MASS) {
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      T b[VZ][NV][NV];
      if constexpr (DIM == 2) {
        pass_y<false, false>(cy.Mv, u[c], b, T(1));
      } else {
        const Coef1D<T, K> &cz = g.c[DIM - 1];
        T a[VZ][NV][NV];
        pass_z<false, false>(cz.Mv, u[c], a, T(1));
        pass_y<false, false>(cy.Mv, a, b, T(1));
      }
      pass_x<false, false>(cx.Mv, b, yu[c], T(1));
    }
  }
  if constexpr (BLK & BLK_BT) {
    constexpr bool ACC = (BLK & (BLK_A | BLK_MASS)) != 0;
    if constexpr (DIM == 2) {
      T s[1][NV][NP];
      pass_y<true, false>(cy.N, p, s, T(1));
      pass_x<true, ACC>(cx.G, s, yu[0], T(-1));
      T s2[1][NP][NV];
      pass_x<true, false>(cx.N, p, s2, T(1));
      pass_y<true, ACC>(cy.G, s2, yu[1], T(-1));
    } else {
      const Coef1D<T, K> &cz = g.c[DIM - 1];
      T s1[NV][NP][NP];
      pass_z<true, false>(cz.N, p, s1, T(1));
      T s2[NV][NV][NP];
      pass_y<true, false>(cy.N, s1, s2, T(1));
      pass_x<true, ACC>(cx.G, s2, yu[0], T(-1));
      pass_y<true, false>(cy.G, s1, s2, T(1));
      pass_x<true, ACC>(cx.N, s2, yu[1], T(-1));
      pass_z<true, false>(cz.G, p, s1, T(1));
      pass_y<true, false>(cy.N, s1, s2, T(1));
      pass_x<true, ACC>(cx.N, s2, yu[2], T(-1));
    }
  }
  if constexpr (BLK & BLK_B) {
    if constexpr (DIM == 2) {
      T w[1][NV][NP];
      pass_x<false, false>(cx.G, u[0], w, T(1));
      pass_y<false, false>(cy.N, w, yp, T(-1));
      pass_x<false, false>(cx.N, u[1], w, T(1));
      pass_y<false, true>(cy.G, w, yp, T(-1));
    } else {
      const Coef1D<T, K> &cz = g.c[DIM - 1];
      T w1[NV][NV][NP];
      T w2[NV][NP][NP];
      pass_x<false, false>(cx.G, u[0], w1, T(1));
      pass_y<false, false>(cy.N, w1, w2, T(1));
      pass_z<false, false>(cz.N, w2, yp, T(-1));
      pass_x<false, false>(cx.N, u[1], w1, T(1));
      pass_y<false, false>(cy.G, w1, w2, T(1));
      pass_z<false, true>(cz.N, w2, yp, T(-1));
      pass_x<false, false>(cx.N, u[2], w1, T(1));
      pass_y<false, false>(cy.N, w1, w2, T(1));
      pass_z<false, true>(cz.G, w2, yp, T(-1));
    }
  }
  if constexpr (BLK & BLK_C) {
    constexpr bool ACC = (BLK & BLK_B) != 0;
    const T sc = (BLK & BLK_CPLUS) ? g.cp : -g.cp;
    T q1[PZ][NP][NP];
    T q2[PZ][NP][NP];
    pass_x<false, false>(cx.Mp, p, q1, T(1));
    if constexpr (DIM == 2) {
      pass_y<false, ACC>(cy.Mp, q1, yp, sc);
    } else {
      const Coef1D<T, K> &cz = g.c[DIM - 1];
      pass_y<false, false>(cy.Mp, q1, q2, T(1));
      pass_z<false, ACC>(cz.Mp, q2, yp, sc);
    }
  }
}

// Bijection blockIdx -> tile such that the blocks of one XCD (b % 8 == k) take
// the contiguous tile range [prefix_k, prefix_k + count_k).
__device__ __forceinline__ int xcd_contiguous_tile(int b, int nb) {
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

// Per-direction tile geometry helper.
struct TileAxis {
  int cell0;   // first cell of the patch (halo cell, may be -1)
  int node0;   // first lattice node of the patch (may be negative)
  int own_lo;  // owned lattice node range [own_lo, own_hi)
  int own_hi;
};

__device__ __forceinline__ TileAxis tile_axis(int t, int ntiles, int owned_cells, int deg, int extent) {
  TileAxis a;
  a.cell0 = t * owned_cells - 1;
  a.node0 = a.cell0 * deg;
  a.own_lo = t * owned_cells * deg;
  a.own_hi = (t == ntiles - 1) ? extent : (t + 1) * owned_cells * deg;
  if (a.own_hi > extent) a.own_hi = extent;
  return a;
}

template <int DIM, int K, typename T, int BLK, class Op, int TX, int TY, int TZ>
__global__ void __launch_bounds__(TX * TY * TZ)
tile_apply_kernel(const LevelGeom<T, DIM, K> g, const Op op) {
  constexpr int NT = TX * TY * TZ;
  constexpr int NV = K + 1, NP = K, VZ = Shape<DIM, K>::VZ, PZ = Shape<DIM, K>::PZ;
  constexpr int PVX = TX * K + 1, PVY = TY * K + 1, PVZ = DIM == 3 ? TZ * K + 1 : 1;
  constexpr int PPX = TX * (K - 1) + 1, PPY = TY * (K - 1) + 1, PPZ = DIM == 3 ? TZ * (K - 1) + 1 : 1;
  constexpr int PV = PVX * PVY * PVZ, PP = PPX * PPY * PPZ;
  constexpr bool NEED_U = (BLK & (BLK_A | BLK_MASS | BLK_B)) != 0;
  constexpr bool NEED_P = (BLK & (BLK_BT | BLK_C)) != 0;
  constexpr bool OUT_U = (BLK & (BLK_A | BLK_MASS | BLK_BT)) != 0;
  constexpr bool OUT_P = (BLK & (BLK_B | BLK_C)) != 0;
  constexpr int OWN_X = TX - 1, OWN_Y = TY - 1, OWN_Z = DIM == 3 ? TZ - 1 : 1;

  __shared__ T s_u[NEED_U ? DIM * PV : 1];
  __shared__ T s_p[NEED_P ? PP : 1];
  __shared__ T o_u[OUT_U ? DIM * PV : 1];
  __shared__ T o_p[OUT_P ? PP : 1];

  // Workgroups are dispatched to the 8 XCDs round-robin (XCD = blockIdx % 8);
  // give each XCD a contiguous run of tiles so that neighbouring tiles, which
  // share patch rows, meet in the same L2.
  const int bid = xcd_contiguous_tile(blockIdx.x, gridDim.x);
  const int tx = bid % g.tiles[0];
  const int ty = (bid / g.tiles[0]) % g.tiles[1];
  const int tz = DIM == 3 ? bid / (g.tiles[0] * g.tiles[1]) : 0;
  const TileAxis ax = tile_axis(tx, g.tiles[0], OWN_X, K, g.vd[0]);
  const TileAxis ay = tile_axis(ty, g.tiles[1], OWN_Y, K, g.vd[1]);
  const TileAxis az = DIM == 3 ? tile_axis(tz, g.tiles[2], OWN_Z, K, g.vd[2]) : TileAxis{0, 0, 0, 1};
  const TileAxis px = tile_axis(tx, g.tiles[0], OWN_X, K - 1, g.pd[0]);
  const TileAxis py = tile_axis(ty, g.tiles[1], OWN_Y, K - 1, g.pd[1]);
  const TileAxis pz = DIM == 3 ? tile_axis(tz, g.tiles[2], OWN_Z, K - 1, g.pd[2]) : TileAxis{0, 0, 0, 1};
  const int vdz = DIM == 3 ? g.vd[2] : 1;
  const int pdz = DIM == 3 ? g.pd[2] : 1;

  // 0. everything the epilogue reads for the owned nodes is requested first,
  //    so that those loads share one memory round trip with the patch loads.
  constexpr int ITU = OUT_U ? (DIM * (OWN_X * K + 1) * (OWN_Y * K + 1) * (DIM == 3 ? OWN_Z * K + 1 : 1) + NT - 1) / NT : 1;
  constexpr int ITP = OUT_P ? ((OWN_X * (K - 1) + 1) * (OWN_Y * (K - 1) + 1) * (DIM == 3 ? OWN_Z * (K - 1) + 1 : 1) + NT - 1) / NT : 1;
  typename Op::Pre pre_u[ITU];
  T raw_u[ITU];
  i64 gidx_u[ITU];
  int lidx_u[ITU];
  bool bc_u[ITU];
  typename Op::Pre pre_p[ITP];
  i64 gidx_p[ITP];
  int lidx_p[ITP];
  if constexpr (OUT_U) {
    const int ox = ax.own_hi - ax.own_lo, oy = ay.own_hi - ay.own_lo, oz = az.own_hi - az.own_lo;
    const int per = ox * oy * oz;
#pragma unroll
    for (int it = 0; it < ITU; ++it) {
      const int i = threadIdx.x + it * NT;
      gidx_u[it] = -1;
      raw_u[it] = 0;
      if (i < DIM * per) {
        const int c = i / per;
        const int r = i - c * per;
        const int gx = ax.own_lo + r % ox, gy = ay.own_lo + (r / ox) % oy, gz = az.own_lo + r / (ox * oy);
        lidx_u[it] = c * PV + (gx - ax.node0) + PVX * ((gy - ay.node0) + PVY * (gz - az.node0));
        gidx_u[it] = (i64)c * g.Nv + gx + (i64)g.vd[0] * (gy + (i64)g.vd[1] * gz);
        bc_u[it] = on_box_boundary(gx, g.vd[0]) || on_box_boundary(gy, g.vd[1]) ||
                   (DIM == 3 && on_box_boundary(gz, vdz));
        pre_u[it] = op.fetch_u(gidx_u[it]);
        // constrained row: identity for A (and K), zero for B^T and the mass load
        if constexpr ((BLK & BLK_A) != 0)
          if (bc_u[it]) raw_u[it] = op.load_u(gidx_u[it]);
      }
    }
  }
  if constexpr (OUT_P) {
    const int ox = px.own_hi - px.own_lo, oy = py.own_hi - py.own_lo, oz = pz.own_hi - pz.own_lo;
    const int per = ox * oy * oz;
#pragma unroll
    for (int it = 0; it < ITP; ++it) {
      const int i = threadIdx.x + it * NT;
      gidx_p[it] = -1;
      if (i < per) {
        const int gx = px.own_lo + i % ox, gy = py.own_lo + (i / ox) % oy, gz = pz.own_lo + i / (ox * oy);
        lidx_p[it] = (gx - px.node0) + PPX * ((gy - py.node0) + PPY * (gz - pz.node0));
        gidx_p[it] = gx + (i64)g.pd[0] * (gy + (i64)g.pd[1] * gz);
        pre_p[it] = op.fetch_p(gidx_p[it]);
      }
    }
  }

  // 1. patch loads (x fastest -> coalesced rows).  All global loads of a
  //    thread are issued before the first LDS store so that their latencies
  //    overlap instead of adding up.
  if constexpr (NEED_U || OUT_U) {
    constexpr int IT = (DIM * PV + NT - 1) / NT;
    T vals[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int i = threadIdx.x + it * NT;
      vals[it] = 0;
      if constexpr (NEED_U) {
        if (i < DIM * PV) {
          const int c = i / PV;
          const int r = i - c * PV;
          const int lx = r % PVX, ly = (r / PVX) % PVY, lz = r / (PVX * PVY);
          const int gx = ax.node0 + lx, gy = ay.node0 + ly, gz = az.node0 + lz;
          if (gx >= 0 && gx < g.vd[0] && gy >= 0 && gy < g.vd[1] && gz >= 0 && gz < vdz) {
            const bool bc = on_box_boundary(gx, g.vd[0]) || on_box_boundary(gy, g.vd[1]) ||
                            (DIM == 3 && on_box_boundary(gz, vdz));
            if (!(bc && Op::ZERO_BC))
              vals[it] = op.load_u((i64)c * g.Nv + gx + (i64)g.vd[0] * (gy + (i64)g.vd[1] * gz));
          }
        }
      }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int i = threadIdx.x + it * NT;
      if (i < DIM * PV) {
        if constexpr (NEED_U) s_u[i] = vals[it];
        if constexpr (OUT_U) o_u[i] = 0;
      }
    }
  }
  if constexpr (NEED_P || OUT_P) {
    constexpr int IT = (PP + NT - 1) / NT;
    T vals[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int i = threadIdx.x + it * NT;
      vals[it] = 0;
      if constexpr (NEED_P) {
        if (i < PP) {
          const int lx = i % PPX, ly = (i / PPX) % PPY, lz = i / (PPX * PPY);
          const int gx = px.node0 + lx, gy = py.node0 + ly, gz = pz.node0 + lz;
          if (gx >= 0 && gx < g.pd[0] && gy >= 0 && gy < g.pd[1] && gz >= 0 && gz < pdz)
            vals[it] = op.load_p(gx + (i64)g.pd[0] * (gy + (i64)g.pd[1] * gz));
        }
      }
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int i = threadIdx.x + it * NT;
      if (i < PP) {
        if constexpr (NEED_P) s_p[i] = vals[it];
        if constexpr (OUT_P) o_p[i] = 0;
      }
    }
  }
  __syncthreads();

  // 2. one cell per thread
  const int lcx = threadIdx.x % TX;
  const int lcy = (threadIdx.x / TX) % TY;
  const int lcz = DIM == 3 ? threadIdx.x / (TX * TY) : 0;
  const int gcx = ax.cell0 + lcx, gcy = ay.cell0 + lcy, gcz = DIM == 3 ? az.cell0 + lcz : 0;
  const bool active = gcx >= 0 && gcx < g.n[0] && gcy >= 0 && gcy < g.n[1] &&
                      (DIM == 2 || (gcz >= 0 && gcz < g.n[2]));
  T yu[DIM][VZ][NV][NV];
  T yp[PZ][NP][NP];
  if (active) {
    T u[DIM][VZ][NV][NV];
    T p[PZ][NP][NP];
    if constexpr (NEED_U) {
#pragma unroll
      for (int c = 0; c < DIM; ++c)
#pragma unroll
        for (int z = 0; z < VZ; ++z)
#pragma unroll
          for (int y = 0; y < NV; ++y)
#pragma unroll
            for (int x = 0; x < NV; ++x)
              u[c][z][y][x] = s_u[c * PV + (lcx * K + x) + PVX * ((lcy * K + y) + PVY * (lcz * K + z))];
    }
    if constexpr (NEED_P) {
#pragma unroll
      for (int z = 0; z < PZ; ++z)
#pragma unroll
        for (int y = 0; y < NP; ++y)
#pragma unroll
          for (int x = 0; x < NP; ++x)
            p[z][y][x] = s_p[(lcx * (K - 1) + x) + PPX * ((lcy * (K - 1) + y) + PPY * (lcz * (K - 1) + z))];
    }
    T mu = g.mu;
    if (g.mu_cell != nullptr) mu = g.mu_cell[gcx + (i64)g.n[0] * (gcy + (i64)g.n[1] * gcz)];
    cell_apply<DIM, K, T, BLK>(g, mu, u, p, yu, yp);
  }

  // 3. colour-phased accumulation into the LDS output patch
  const int colour = (gcx & 1) | ((gcy & 1) << 1) | ((gcz & 1) << 2);
  constexpr int NCOL = 1 << DIM;
#pragma unroll 1
  for (int col = 0; col < NCOL; ++col) {
    if (active && colour == col) {
      if constexpr (OUT_U) {
#pragma unroll
        for (int c = 0; c < DIM; ++c)
#pragma unroll
          for (int z = 0; z < VZ; ++z)
#pragma unroll
            for (int y = 0; y < NV; ++y)
#pragma unroll
              for (int x = 0; x < NV; ++x)
                o_u[c * PV + (lcx * K + x) + PVX * ((lcy * K + y) + PVY * (lcz * K + z))] += yu[c][z][y][x];
      }
      if constexpr (OUT_P) {
#pragma unroll
        for (int z = 0; z < PZ; ++z)
#pragma unroll
          for (int y = 0; y < NP; ++y)
#pragma unroll
            for (int x = 0; x < NP; ++x)
              o_p[(lcx * (K - 1) + x) + PPX * ((lcy * (K - 1) + y) + PPY * (lcz * (K - 1) + z))] += yp[z][y][x];
      }
    }
    __syncthreads();
  }

  // 4. owned nodes through the epilogue (inputs fetched in step 0)
  if constexpr (OUT_U) {
#pragma unroll
    for (int it = 0; it < ITU; ++it) {
      if (gidx_u[it] < 0) continue;
      if (bc_u[it]) {
        op.store_u(gidx_u[it], raw_u[it], raw_u[it], true, pre_u[it]);
      } else {
        T v = 0;
        if constexpr (NEED_U) v = s_u[lidx_u[it]];
        op.store_u(gidx_u[it], o_u[lidx_u[it]], v, false, pre_u[it]);
      }
    }
  }
  if constexpr (OUT_P) {
#pragma unroll
    for (int it = 0; it < ITP; ++it) {
      if (gidx_p[it] < 0) continue;
      T v = 0;
      if constexpr (NEED_P) v = s_p[lidx_p[it]];
      op.store_p(gidx_p[it], o_p[lidx_p[it]], v, pre_p[it]);
    }
  }
}

}  // namespace smg
