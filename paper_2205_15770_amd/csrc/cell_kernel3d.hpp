// Column-sweep application of the Taylor-Hood saddle-point operator
// K = [A B^T; B -C] on axis-aligned box cells in 3D (Sec. 3.1: K x =
// sum_tau P_tau K_tau P_tau^T x, cell matrices by sum factorisation).
//
// Work decomposition (gfx950): one wave64 per (tile of TX x TY cell columns,
// z chunk, output field); the library uses 9 x 7 (lane 63 idle).  Lane l
// holds the cell column (l % TX, l / TX) of the tile and sweeps the cells of
// its column through the chunk in z.  A tile owns (TX - 1) x (TY - 1)
// columns; lane column 0 and lane row 0 are halo columns, and the cell layer
// below a chunk is a halo layer: their cell results are computed only to
// hand them over.  No LDS, no barriers, no atomics; every output
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
// epilogue functor.  The DoFs of the next cell (velocity waves: the next
// layer; pressure waves: the next velocity component) are requested before
// the current one is computed.
//
// Cell matrices: the 1D reference matrices are compile-time literals; on a
// box cell of widths (h_x, h_y, h_z)
//   A_cell = mu [sKx Kr(x)Mr(x)Mr + sKy Mr(x)Kr(x)Mr + sKz Mr(x)Mr(x)Kr]
//            + gamma rho sM Mr(x)Mr(x)Mr,
//   B_c    = -sB_c (Gr in direction c, Nr in the others),  C = cp sM Mpr^(x)3,
// with sKx = h_y h_z / h_x (cyclic), sM = h_x h_y h_z, sB_c = prod_{a != c} h_a.
#pragma once
#include <type_traits>
#include "cell_kernel.hpp"
#include "fe1d_const.hpp"
#include "ops.hpp"

namespace smg {

// Kernel parameters of one level (3D column sweep).
template <typename T>
struct Geo3 {
  int n[3];       // cells per direction
  int vd[3];      // velocity lattice extent per direction
  int pd[3];      // pressure lattice extent per direction
  int tiles[3];   // 8x8 column tiles in x, y; z chunks
  uint32_t nv_bytes;  // bytes of one velocity component vector
  T mu, gr, cp;   // viscosity (if mu_cell == nullptr), gamma rho, C = cp M_p
  const T *mu_cell;
  T sKx, sKy;     // h_y h_z / h_x, h_x h_z / h_y
  T rz;           // sKz / sKy = h_y^2 / h_z^2
  T sM;           // h_x h_y h_z
  T sB[3];        // h_y h_z, h_x h_z, h_x h_y
};

template <int K, typename T>
struct Column3D {
  static constexpr int NV = K + 1, NP = K;
  static constexpr uint32_t ST = sizeof(T);
  const Geo3<T> &g;
  int gcx, gcy;        // cell column (may lie outside the mesh for halo lanes)
  bool active;         // column inside the mesh
  bool bxl, bxh, byl, byh;  // column touches the low / high x, y boundary
  uint32_t base_u;     // byte offset of the column's first velocity node
  uint32_t base_p;     // byte offset of the column's first pressure node
  uint32_t suy, suz, spy, spz;  // byte strides of the velocity / pressure lattices
  uint32_t cell0, cell_sz;      // cell index of the column's first cell, cells per layer
  __host__ __device__ Column3D(const Geo3<T> &g_, int cx, int cy) : g(g_), gcx(cx), gcy(cy) {
    active = cx >= 0 && cx < g.n[0] && cy >= 0 && cy < g.n[1];
    bxl = cx == 0;
    bxh = cx == g.n[0] - 1;
    byl = cy == 0;
    byh = cy == g.n[1] - 1;
    // halo lanes outside the mesh read a valid column and discard the values
    const int ax = cx < 0 ? 0 : (cx >= g.n[0] ? g.n[0] - 1 : cx);
    const int ay = cy < 0 ? 0 : (cy >= g.n[1] ? g.n[1] - 1 : cy);
    suy = ST * (uint32_t)g.vd[0];
    suz = suy * (uint32_t)g.vd[1];
    spy = ST * (uint32_t)g.pd[0];
    spz = spy * (uint32_t)g.pd[1];
    base_u = ST * (uint32_t)(K * ax) + suy * (uint32_t)(K * ay);
    base_p = ST * (uint32_t)((K - 1) * ax) + spy * (uint32_t)((K - 1) * ay);
    cell0 = (uint32_t)ax + (uint32_t)g.n[0] * (uint32_t)ay;
    cell_sz = (uint32_t)g.n[0] * (uint32_t)g.n[1];
  }
  __host__ __device__ uint32_t mu_index(int cz) const { return cell0 + cell_sz * (uint32_t)cz; }
  __device__ T mu_at(int cz) const {
    if (g.mu_cell != nullptr) return g.mu_cell[mu_index(cz)];
    return g.mu;
  }
  // node (x, y, z) of cell layer cz, velocity component c
  __host__ __device__ BOff u_at(int c, int cz, int x, int y, int z) const {
    return BOff{(uint32_t)c * g.nv_bytes + base_u + suz * (uint32_t)(K * cz + z) + suy * (uint32_t)y,
                ST * (uint32_t)x};
  }
  __host__ __device__ BOff p_at(int cz, int x, int y, int z) const {
    return BOff{base_p + spz * (uint32_t)((K - 1) * cz + z) + spy * (uint32_t)y, ST * (uint32_t)x};
  }
  // Dirichlet test of local velocity node (x, y, z) of layer cz (bitwise
  // forms: no short-circuit branches on lane-varying flags)
  __host__ __device__ bool vbc(int cz, int x, int y, int z) const {
    return ((x == 0) & bxl) | ((x == K) & bxh) | ((y == 0) & byl) | ((y == K) & byh) |
           ((z == 0) & (cz == 0)) | ((z == K) & (cz == g.n[2] - 1));
  }
  // raw loads: planes [Z0, Z0 + NZ) of velocity component c of layer cz
  template <int Z0, class Op, int NZ>
  __device__ void load_u(const Op &op, int c, int cz, T (&dst)[NZ][NV][NV]) const {
#pragma unroll
    for (int z = 0; z < NZ; ++z)
#pragma unroll
      for (int y = 0; y < NV; ++y)
#pragma unroll
        for (int x = 0; x < NV; ++x) dst[z][y][x] = op.load_u(u_at(c, cz, x, y, Z0 + z));
  }
  template <int Z0, class Op, int NZ>
  __device__ void load_p(const Op &op, int cz, T (&dst)[NZ][NP][NP]) const {
#pragma unroll
    for (int z = 0; z < NZ; ++z)
#pragma unroll
      for (int y = 0; y < NP; ++y)
#pragma unroll
        for (int x = 0; x < NP; ++x) dst[z][y][x] = op.load_p(p_at(cz, x, y, Z0 + z));
  }
  // zero what must not enter the cell operator: inactive columns and (ZERO_BC)
  // Dirichlet nodes.  Applied where the loaded values are first used, not
  // next to the loads, so the loads stay unconditional and early.
  template <bool ZERO_BC, int Z0, int NZ>
  __device__ void mask_u(int cz, T (&a)[NZ][NV][NV]) const {
#pragma unroll
    for (int z = 0; z < NZ; ++z)
#pragma unroll
      for (int y = 0; y < NV; ++y)
#pragma unroll
        for (int x = 0; x < NV; ++x) {
          const bool keep = active & !(ZERO_BC & vbc(cz, x, y, Z0 + z));
          a[z][y][x] = keep ? a[z][y][x] : T(0);
        }
  }
  template <int NZ>
  __device__ void mask_p(T (&a)[NZ][NP][NP]) const {
#pragma unroll
    for (int z = 0; z < NZ; ++z)
#pragma unroll
      for (int y = 0; y < NP; ++y)
#pragma unroll
        for (int x = 0; x < NP; ++x) a[z][y][x] = active ? a[z][y][x] : T(0);
  }
};

// Sweep geometry shared by the wave roles.
struct Sweep {
  int lcx, lcy;     // lane position in the tile
  int z_lo, z_hi;   // owned cell layers [z_lo, z_hi)
  int z_start;      // first computed layer (halo layer below z_lo if any)
  bool col_owner;   // column owned by the tile
  bool last_x, last_y;
};

// Column-sweep tile used by the library: 9 x 7 lanes (63 of the 64) owning
// 8 x 6 cell columns.  On the power-of-two levels of a box hierarchy 8 owned
// columns divide the level in x; 8 x 8 lanes owning 7 x 7 divide nothing
// (64^2: 10 x 10 tiles, 6400 computed columns for 4096, against 8 x 11
// tiles, 5632).
constexpr int SW_TX = 9, SW_TY = 7;

// Launch shape of the column sweep (host): TX x TY column tiles owning
// (TX - 1) x (TY - 1) columns, NF output fields, the z extent cut into
// chunks of >= 2 cells so that the launch has about `waves` waves when the
// level is large enough.  Sets g.tiles and returns the number of blocks (one
// wave each).
template <int TX, int TY, typename T>
inline int sweep3d_chunks(Geo3<T> &g, int NF, int waves) {
  g.tiles[0] = (g.n[0] + TX - 2) / (TX - 1);
  g.tiles[1] = (g.n[1] + TY - 2) / (TY - 1);
  const int cols = g.tiles[0] * g.tiles[1] * NF;
  int nzc = (waves + cols - 1) / cols;
  const int zmax = (g.n[2] + 1) / 2;
  nzc = nzc < 1 ? 1 : (nzc > zmax ? zmax : nzc);
  const int zlen = (g.n[2] + nzc - 1) / nzc;
  g.tiles[2] = (g.n[2] + zlen - 1) / zlen;
  return cols * g.tiles[2];
}

// Block b (after the XCD map) and lane -> output field, z chunk, lane cell
// column (cx, cy) of the sweep; false for an empty chunk (the whole wave
// returns).  Blocks run (field, x tile, z chunk, y tile), fastest first, so
// the fields of one tile and chunk run on the same XCD.
template <int TX, int TY, typename T>
__host__ __device__ inline bool sweep3d_decode(const Geo3<T> &g, int NF, int b, int lane, int &field, Sweep &s,
                                               int &cx, int &cy) {
  field = b % NF;
  int rest = b / NF;
  const int tx = rest % g.tiles[0];
  rest /= g.tiles[0];
  const int zc = rest % g.tiles[2];
  const int ty = rest / g.tiles[2];
  const int zlen = (g.n[2] + g.tiles[2] - 1) / g.tiles[2];
  s.z_lo = zc * zlen;
  s.z_hi = s.z_lo + zlen < g.n[2] ? s.z_lo + zlen : g.n[2];
  if (s.z_lo >= s.z_hi) return false;
  s.z_start = s.z_lo > 0 ? s.z_lo - 1 : 0;
  s.lcx = lane % TX;
  s.lcy = lane / TX;
  cx = tx * (TX - 1) - 1 + s.lcx;
  cy = ty * (TY - 1) - 1 + s.lcy;
  // (lanes past TX * TY, if any, compute a column outside the tile and own
  // nothing)
  s.col_owner = cx >= 0 && cx < g.n[0] && cy >= 0 && cy < g.n[1] && s.lcx > 0 && s.lcy > 0 && s.lcy < TY;
  s.last_x = cx == g.n[0] - 1;
  s.last_y = cy == g.n[1] - 1;
  return true;
}

// Cell matrices of one velocity component on one box cell:
//   y = (A u)_COMP (BLK_A) or (M u)_COMP (BLK_MASS), plus (B^T p)_COMP (BLK_BT).
template <int K, typename T, int BLK, int COMP>
__device__ __forceinline__ void vel_cell(const Geo3<T> &g, T mu, const T (&u)[K + 1][K + 1][K + 1],
                                         const T (&p)[K][K][K], T (&y)[K + 1][K + 1][K + 1]) {
  constexpr int NV = K + 1, NP = K;
  constexpr cfe::TabT<K, T> R = cfe::make_tab_t<K, T>();
  // B_c^T: Gr^T in direction COMP, Nr^T in the others
  const T(&Bx)[K][K + 1] = COMP == 0 ? R.Gr : R.Nr;
  const T(&By)[K][K + 1] = COMP == 1 ? R.Gr : R.Nr;
  const T(&Bz)[K][K + 1] = COMP == 2 ? R.Gr : R.Nr;
  if constexpr ((BLK & BLK_A) != 0) {
    // plane by plane in z (fewer live values than whole-cell passes):
    //   y[oz] = sum_iz Mz[oz][iz] ((ax Kx + bx Mx) My + cy Mx Ky) u[iz]
    //                + Kz[oz][iz] cz Mx My u[iz]
    // with ax = mu sKx, bx = gamma rho sM, cy = mu sKy, cz = mu sKz
    T X[NV][NV];
    const T ax = mu * g.sKx, bx = g.gr * g.sM, cy = mu * g.sKy, cz = cy * g.rz;
#pragma unroll
    for (int i = 0; i < NV; ++i)
#pragma unroll
      for (int j = 0; j < NV; ++j) X[i][j] = ax * R.Kr[i][j] + bx * R.Mr[i][j];
#pragma unroll
    for (int iz = 0; iz < NV; ++iz) {
      T t1[NV][NV], t2[NV][NV], v1[NV][NV], v2[NV][NV];
      // t1 = My u, t2 = cy Ky u on the plane ([y][x])
#pragma unroll
      for (int x = 0; x < NV; ++x)
#pragma unroll
        for (int o = 0; o < NV; ++o) {
          T s1 = 0, s2 = 0;
#pragma unroll
          for (int i = 0; i < NV; ++i) {
            s1 += R.Mr[o][i] * u[iz][i][x];
            s2 += R.Kr[o][i] * u[iz][i][x];
          }
          t1[o][x] = s1;
          t2[o][x] = cy * s2;
        }
      // v1 = X t1 + Mx t2, v2 = cz Mx t1 along x
#pragma unroll
      for (int yy = 0; yy < NV; ++yy)
#pragma unroll
        for (int o = 0; o < NV; ++o) {
          T s1 = 0, s2 = 0;
#pragma unroll
          for (int i = 0; i < NV; ++i) {
            s1 += X[o][i] * t1[yy][i] + R.Mr[o][i] * t2[yy][i];
            s2 += R.Mr[o][i] * t1[yy][i];
          }
          v1[yy][o] = s1;
          v2[yy][o] = cz * s2;
        }
      // y[oz] (+)= Mz[oz][iz] v1 + Kz[oz][iz] v2
#pragma unroll
      for (int oz = 0; oz < NV; ++oz)
#pragma unroll
        for (int yy = 0; yy < NV; ++yy)
#pragma unroll
          for (int xx = 0; xx < NV; ++xx) {
            const T c = R.Mr[oz][iz] * v1[yy][xx] + R.Kr[oz][iz] * v2[yy][xx];
            y[oz][yy][xx] = iz == 0 ? c : y[oz][yy][xx] + c;
          }
    }
  } else if constexpr ((BLK & BLK_MASS) != 0) {
    T a[NV][NV][NV], t[NV][NV][NV];
    pass_z<false, false>(R.Mr, u, a, T(1));
    pass_y<false, false>(R.Mr, a, t, T(1));
    pass_x<false, false>(R.Mr, t, y, g.sM);
  }
  if constexpr ((BLK & BLK_BT) != 0) {
    constexpr bool ACC = (BLK & (BLK_A | BLK_MASS)) != 0;
    T s1[NV][NP][NP], s2[NV][NV][NP];
    pass_z<true, false>(Bz, p, s1, T(1));
    pass_y<true, false>(By, s1, s2, T(1));
    pass_x<true, ACC>(Bx, s2, y, -g.sB[COMP]);
  } else if constexpr ((BLK & (BLK_A | BLK_MASS)) == 0) {
#pragma unroll
    for (int z = 0; z < NV; ++z)
#pragma unroll
      for (int j = 0; j < NV; ++j)
#pragma unroll
        for (int i = 0; i < NV; ++i) y[z][j][i] = 0;
  }
}

// ------------------------------------------------------------ velocity wave
template <int K, typename T, int BLK, class Op, int COMP, int TX>
__device__ __forceinline__ void vel_wave(const Geo3<T> &g, const Op &op, const Column3D<K, T> &col, const Sweep &s) {
  constexpr int NV = K + 1, NP = K;
  constexpr bool NEED_U = (BLK & (BLK_A | BLK_MASS)) != 0;
  constexpr bool NEED_P = (BLK & BLK_BT) != 0;
  T u[NV][NV][NV], un[K][NV][NV];
  T p[NP][NP][NP], pn[NP - 1][NP][NP];
  T carry[NV][NV];
#pragma unroll
  for (int j = 0; j < NV; ++j)
#pragma unroll
    for (int i = 0; i < NV; ++i) carry[j][i] = 0;
  if constexpr (NEED_U) {
    col.template load_u<0>(op, COMP, s.z_start, u);
    col.template mask_u<Op::ZERO_BC, 0>(s.z_start, u);
  } else {
#pragma unroll
    for (int z = 0; z < NV; ++z)
#pragma unroll
      for (int j = 0; j < NV; ++j)
#pragma unroll
        for (int i = 0; i < NV; ++i) u[z][j][i] = 0;
  }
  if constexpr (NEED_P) {
    col.template load_p<0>(op, s.z_start, p);
    col.mask_p(p);
  }
  T mu = 0, mu_n = 0;
  if constexpr ((BLK & BLK_A) != 0) mu = col.mu_at(s.z_start);

  for (int cl = s.z_start; cl < s.z_hi; ++cl) {
    const bool more = cl + 1 < s.z_hi;
    if (more) {  // next layer: planes 1..K (plane 0 is this layer's plane K)
      if constexpr ((BLK & BLK_A) != 0) mu_n = col.mu_at(cl + 1);
      if constexpr (NEED_U) col.template load_u<1>(op, COMP, cl + 1, un);
      if constexpr (NEED_P) col.template load_p<1>(op, cl + 1, pn);
    }
    const bool owner = s.col_owner && cl >= s.z_lo;
    const bool last_z = cl == g.n[2] - 1;
    T y[NV][NV][NV];
    vel_cell<K, T, BLK, COMP>(g, mu, u, p, y);
    // epilogue inputs of the owned nodes [0,K)^3, requested after the cell
    // product (not live across it) and before the hand-over shuffles
    typename Op::Pre pre[K][K][K];
    if (owner) {
#pragma unroll
      for (int z = 0; z < K; ++z)
#pragma unroll
        for (int yy = 0; yy < K; ++yy)
#pragma unroll
          for (int x = 0; x < K; ++x) pre[z][yy][x] = op.fetch_u(col.u_at(COMP, cl, x, yy, z));
    }
    hand_over_xy<TX>(y, s.lcx, s.lcy, s.last_x, s.last_y);
#pragma unroll
    for (int j = 0; j < NV; ++j)
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        y[0][j][i] += carry[j][i];
        carry[j][i] = y[K][j][i];
      }
    if (owner) {
      // every owned node from the cell sums; the Dirichlet rows among them are
      // rewritten below (same lane, program order)
#pragma unroll
      for (int z = 0; z < K; ++z)
#pragma unroll
        for (int yy = 0; yy < K; ++yy)
#pragma unroll
          for (int x = 0; x < K; ++x)
            op.store_u(col.u_at(COMP, cl, x, yy, z), y[z][yy][x], u[z][yy][x], false, pre[z][yy][x]);
      if (col.bxl | col.byl | (cl == 0)) {
        // Dirichlet rows on the low faces: identity (A) or zero
#pragma unroll
        for (int z = 0; z < K; ++z)
#pragma unroll
          for (int yy = 0; yy < K; ++yy)
#pragma unroll
            for (int x = 0; x < K; ++x) {
              if (!col.vbc(cl, x, yy, z)) continue;
              const BOff gi = col.u_at(COMP, cl, x, yy, z);
              T rw = 0;
              if constexpr ((BLK & BLK_A) != 0) rw = op.load_u(gi);
              op.store_u(gi, rw, rw, true, pre[z][yy][x]);
            }
      }
      if (s.last_x | s.last_y | last_z) {
        // nodes on the domain's high faces: Dirichlet rows
#pragma unroll
        for (int z = 0; z < NV; ++z)
#pragma unroll
          for (int yy = 0; yy < NV; ++yy)
#pragma unroll
            for (int x = 0; x < NV; ++x) {
              if (x < K && yy < K && z < K) continue;
              if ((x == K && !s.last_x) || (yy == K && !s.last_y) || (z == K && !last_z)) continue;
              const BOff gi = col.u_at(COMP, cl, x, yy, z);
              T rw = 0;
              if constexpr ((BLK & BLK_A) != 0) rw = op.load_u(gi);
              op.store_u(gi, rw, rw, true, op.fetch_u(gi));
            }
      }
    }
    if (more) {
      mu = mu_n;
      if constexpr (NEED_U) {
        col.template mask_u<Op::ZERO_BC, 1>(cl + 1, un);
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
      }
      if constexpr (NEED_P) {
        col.mask_p(pn);
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
}

// ------------------------------------------------------------ pressure wave
template <int K, typename T, int BLK, class Op, int TX>
__device__ __forceinline__ void pres_wave(const Geo3<T> &g, const Op &op, const Column3D<K, T> &col, const Sweep &s) {
  constexpr int NV = K + 1, NP = K;
  constexpr cfe::TabT<K, T> R = cfe::make_tab_t<K, T>();
  constexpr bool NEED_U = (BLK & BLK_B) != 0;
  constexpr bool NEED_P = (BLK & BLK_C) != 0;
  T carry[NP][NP];
#pragma unroll
  for (int j = 0; j < NP; ++j)
#pragma unroll
    for (int i = 0; i < NP; ++i) carry[j][i] = 0;
  // velocity component layers are streamed one component at a time with one
  // request ahead: (layer, component) = (cl, 0), (cl, 1), (cl, 2), (cl + 1, 0)...
  T ub[NV][NV][NV];
  T p[NP][NP][NP];
  if constexpr (NEED_U) col.template load_u<0>(op, 0, s.z_start, ub);
  if constexpr (NEED_P) col.template load_p<0>(op, s.z_start, p);
  for (int cl = s.z_start; cl < s.z_hi; ++cl) {
    const bool more = cl + 1 < s.z_hi;
    const bool owner = s.col_owner && cl >= s.z_lo;
    const bool last_z = cl == g.n[2] - 1;
    typename Op::Pre pre[K - 1][K - 1][K - 1];
    if (owner) {
#pragma unroll
      for (int z = 0; z < K - 1; ++z)
#pragma unroll
        for (int yy = 0; yy < K - 1; ++yy)
#pragma unroll
          for (int x = 0; x < K - 1; ++x) pre[z][yy][x] = op.fetch_p(col.p_at(cl, x, yy, z));
    }
    T pn[NP][NP][NP];
    if constexpr (NEED_P) {
      if (more) col.template load_p<0>(op, cl + 1, pn);
      col.mask_p(p);
    }
    T yp[NP][NP][NP];
#pragma unroll
    for (int z = 0; z < NP; ++z)
#pragma unroll
      for (int j = 0; j < NP; ++j)
#pragma unroll
        for (int i = 0; i < NP; ++i) yp[z][j][i] = 0;
    if constexpr (NEED_U) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        T un[NV][NV][NV];
        if (c < 2) col.template load_u<0>(op, c + 1, cl, un);
        else if (more) col.template load_u<0>(op, 0, cl + 1, un);
        col.template mask_u<Op::ZERO_BC, 0>(cl, ub);
        // B u = -sum_c sB_c (Gr in direction c, Nr in the others) u_c
        T w1[NV][NV][NP], w2[NV][NP][NP];
        pass_x<false, false>(c == 0 ? R.Gr : R.Nr, ub, w1, T(1));
        pass_y<false, false>(c == 1 ? R.Gr : R.Nr, w1, w2, T(1));
        pass_z<false, true>(c == 2 ? R.Gr : R.Nr, w2, yp, -g.sB[c]);
#pragma unroll
        for (int z = 0; z < NV; ++z)
#pragma unroll
          for (int j = 0; j < NV; ++j)
#pragma unroll
            for (int i = 0; i < NV; ++i) ub[z][j][i] = un[z][j][i];
      }
    }
    if constexpr (NEED_P) {
      const T sc = ((BLK & BLK_CPLUS) ? g.cp : -g.cp) * g.sM;
      T q1[NP][NP][NP], q2[NP][NP][NP];
      pass_x<false, false>(R.Mpr, p, q1, T(1));
      pass_y<false, false>(R.Mpr, q1, q2, T(1));
      pass_z<false, true>(R.Mpr, q2, yp, sc);
    }
    hand_over_xy<TX>(yp, s.lcx, s.lcy, s.last_x, s.last_y);
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
            if (main) {
              op.store_p(col.p_at(cl, x, yy, z), yp[z][yy][x], p[z][yy][x], pre[main ? z : 0][main ? yy : 0][main ? x : 0]);
            } else if (((x < K - 1) | s.last_x) & ((yy < K - 1) | s.last_y) & ((z < K - 1) | last_z)) {
              const BOff gi = col.p_at(cl, x, yy, z);
              op.store_p(gi, yp[z][yy][x], p[z][yy][x], op.fetch_p(gi));
            }
          }
    }
    if constexpr (NEED_P) {
      if (more) {
#pragma unroll
        for (int z = 0; z < NP; ++z)
#pragma unroll
          for (int j = 0; j < NP; ++j)
#pragma unroll
            for (int i = 0; i < NP; ++i) p[z][j][i] = pn[z][j][i];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Small levels: one wave per 4 x 4 x 4 cells (lane = x + 4 y + 16 z) and
// output field, one cell per lane, no sweep; the tile owns 3 x 3 x 3 cells
// (lane coordinate 0 is halo in each direction) and the z = K face moves to
// lane + 16 by a shuffle like the x and y faces.  A wave's critical path is
// one cell instead of a column, which is what the latency-bound small levels
// need.
// ---------------------------------------------------------------------------
struct Block3D {
  int lx, ly, lz;
  int cz;             // cell layer (clamped into the mesh for addressing)
  bool active, owner;
  bool last_x, last_y, last_z;
};

// Launch shape of the cell-block kernels (host): blocks of 4 x 4 x 4 cells
// owning 3 x 3 x 3, NF output fields; sets g.tiles, returns the block count.
template <typename T>
inline int block3d_tiles(Geo3<T> &g, int NF) {
  for (int a = 0; a < 3; ++a) g.tiles[a] = (g.n[a] + 2) / 3;
  return g.tiles[0] * g.tiles[1] * g.tiles[2] * NF;
}

// Block b (after the XCD map) and lane (0..63) -> output field, the lane's
// cell (s, clamped layer s.cz) and its cell column (cx, cy).
template <typename T>
__host__ __device__ inline void block3d_decode(const Geo3<T> &g, int NF, int b, int lane, int &field, Block3D &s,
                                               int &cx, int &cy) {
  field = b % NF;
  int rest = b / NF;
  const int tx = rest % g.tiles[0];
  rest /= g.tiles[0];
  const int ty = rest % g.tiles[1];
  const int tz = rest / g.tiles[1];
  s.lx = lane % 4;
  s.ly = (lane / 4) % 4;
  s.lz = lane / 16;
  cx = tx * 3 - 1 + s.lx;
  cy = ty * 3 - 1 + s.ly;
  const int cz = tz * 3 - 1 + s.lz;
  s.cz = cz < 0 ? 0 : (cz >= g.n[2] ? g.n[2] - 1 : cz);
  s.active = cx >= 0 && cx < g.n[0] && cy >= 0 && cy < g.n[1] && cz >= 0 && cz < g.n[2];
  s.owner = s.active && s.lx > 0 && s.ly > 0 && s.lz > 0;
  s.last_x = cx == g.n[0] - 1;
  s.last_y = cy == g.n[1] - 1;
  s.last_z = cz == g.n[2] - 1;
}

template <int K, typename T, int BLK, class Op, int COMP>
__device__ __forceinline__ void block_vel(const Geo3<T> &g, const Op &op, const Column3D<K, T> &col,
                                          const Block3D &s) {
  constexpr int NV = K + 1, NP = K;
  constexpr bool NEED_U = (BLK & (BLK_A | BLK_MASS)) != 0;
  constexpr bool NEED_P = (BLK & BLK_BT) != 0;
  T u[NV][NV][NV], p[NP][NP][NP];
  if constexpr (NEED_U) col.template load_u<0>(op, COMP, s.cz, u);
  if constexpr (NEED_P) col.template load_p<0>(op, s.cz, p);
  T mu = 0;
  if constexpr ((BLK & BLK_A) != 0) mu = col.mu_at(s.cz);
  typename Op::Pre pre[K][K][K];
  if (s.owner) {
#pragma unroll
    for (int z = 0; z < K; ++z)
#pragma unroll
      for (int y = 0; y < K; ++y)
#pragma unroll
        for (int x = 0; x < K; ++x) pre[z][y][x] = op.fetch_u(col.u_at(COMP, s.cz, x, y, z));
  }
  // keep the requests above unconditional (see the 2D wave kernel)
  __asm__ volatile("" ::: "memory");
#pragma unroll
  for (int z = 0; z < NV; ++z)
#pragma unroll
    for (int j = 0; j < NV; ++j)
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        if constexpr (NEED_U) {
          const bool keep = s.active & !(Op::ZERO_BC & col.vbc(s.cz, i, j, z));
          u[z][j][i] = keep ? u[z][j][i] : T(0);
        } else {
          u[z][j][i] = 0;
        }
      }
  if constexpr (NEED_P) {
#pragma unroll
    for (int z = 0; z < NP; ++z)
#pragma unroll
      for (int j = 0; j < NP; ++j)
#pragma unroll
        for (int i = 0; i < NP; ++i) p[z][j][i] = s.active ? p[z][j][i] : T(0);
  }
  T y[NV][NV][NV];
  vel_cell<K, T, BLK, COMP>(g, mu, u, p, y);
  hand_over_xy<4>(y, s.lx, s.ly, s.last_x, s.last_y);
#pragma unroll
  for (int j = 0; j < NV; ++j)
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const T r = __shfl_up(y[K][j][i], 16, 64);
      if (s.lz > 0) y[0][j][i] += r;
      if (!s.last_z) y[K][j][i] = 0;
    }
  if (!s.owner) return;
#pragma unroll
  for (int z = 0; z < K; ++z)
#pragma unroll
    for (int yy = 0; yy < K; ++yy)
#pragma unroll
      for (int x = 0; x < K; ++x)
        op.store_u(col.u_at(COMP, s.cz, x, yy, z), y[z][yy][x], u[z][yy][x], false, pre[z][yy][x]);
  if (col.bxl | col.byl | (s.cz == 0)) {
#pragma unroll
    for (int z = 0; z < K; ++z)
#pragma unroll
      for (int yy = 0; yy < K; ++yy)
#pragma unroll
        for (int x = 0; x < K; ++x) {
          if (!col.vbc(s.cz, x, yy, z)) continue;
          const BOff gi = col.u_at(COMP, s.cz, x, yy, z);
          T rw = 0;
          if constexpr ((BLK & BLK_A) != 0) rw = op.load_u(gi);
          op.store_u(gi, rw, rw, true, pre[z][yy][x]);
        }
  }
  if (s.last_x | s.last_y | s.last_z) {
#pragma unroll
    for (int z = 0; z < NV; ++z)
#pragma unroll
      for (int yy = 0; yy < NV; ++yy)
#pragma unroll
        for (int x = 0; x < NV; ++x) {
          if (x < K && yy < K && z < K) continue;
          if ((x == K && !s.last_x) || (yy == K && !s.last_y) || (z == K && !s.last_z)) continue;
          const BOff gi = col.u_at(COMP, s.cz, x, yy, z);
          T rw = 0;
          if constexpr ((BLK & BLK_A) != 0) rw = op.load_u(gi);
          op.store_u(gi, rw, rw, true, op.fetch_u(gi));
        }
  }
}

template <int K, typename T, int BLK, class Op>
__device__ __forceinline__ void block_pres(const Geo3<T> &g, const Op &op, const Column3D<K, T> &col,
                                           const Block3D &s) {
  constexpr int NV = K + 1, NP = K;
  constexpr cfe::TabT<K, T> R = cfe::make_tab_t<K, T>();
  constexpr bool NEED_U = (BLK & BLK_B) != 0;
  constexpr bool NEED_P = (BLK & BLK_C) != 0;
  T ub[3][NV][NV][NV], p[NP][NP][NP];
  if constexpr (NEED_U) {
#pragma unroll
    for (int c = 0; c < 3; ++c) col.template load_u<0>(op, c, s.cz, ub[c]);
  }
  if constexpr (NEED_P) col.template load_p<0>(op, s.cz, p);
  typename Op::Pre pre[K - 1][K - 1][K - 1];
  if (s.owner) {
#pragma unroll
    for (int z = 0; z < K - 1; ++z)
#pragma unroll
      for (int yy = 0; yy < K - 1; ++yy)
#pragma unroll
        for (int x = 0; x < K - 1; ++x) pre[z][yy][x] = op.fetch_p(col.p_at(s.cz, x, yy, z));
  }
  __asm__ volatile("" ::: "memory");
  T yp[NP][NP][NP];
#pragma unroll
  for (int z = 0; z < NP; ++z)
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
      for (int i = 0; i < NP; ++i) yp[z][j][i] = 0;
  if constexpr (NEED_U) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int z = 0; z < NV; ++z)
#pragma unroll
        for (int j = 0; j < NV; ++j)
#pragma unroll
          for (int i = 0; i < NV; ++i) {
            const bool keep = s.active & !(Op::ZERO_BC & col.vbc(s.cz, i, j, z));
            ub[c][z][j][i] = keep ? ub[c][z][j][i] : T(0);
          }
      T w1[NV][NV][NP], w2[NV][NP][NP];
      pass_x<false, false>(c == 0 ? R.Gr : R.Nr, ub[c], w1, T(1));
      pass_y<false, false>(c == 1 ? R.Gr : R.Nr, w1, w2, T(1));
      pass_z<false, true>(c == 2 ? R.Gr : R.Nr, w2, yp, -g.sB[c]);
    }
  }
  if constexpr (NEED_P) {
#pragma unroll
    for (int z = 0; z < NP; ++z)
#pragma unroll
      for (int j = 0; j < NP; ++j)
#pragma unroll
        for (int i = 0; i < NP; ++i) p[z][j][i] = s.active ? p[z][j][i] : T(0);
    const T sc = ((BLK & BLK_CPLUS) ? g.cp : -g.cp) * g.sM;
    T q1[NP][NP][NP], q2[NP][NP][NP];
    pass_x<false, false>(R.Mpr, p, q1, T(1));
    pass_y<false, false>(R.Mpr, q1, q2, T(1));
    pass_z<false, true>(R.Mpr, q2, yp, sc);
  } else {
#pragma unroll
    for (int z = 0; z < NP; ++z)
#pragma unroll
      for (int j = 0; j < NP; ++j)
#pragma unroll
        for (int i = 0; i < NP; ++i) p[z][j][i] = 0;
  }
  hand_over_xy<4>(yp, s.lx, s.ly, s.last_x, s.last_y);
#pragma unroll
  for (int j = 0; j < NP; ++j)
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const T r = __shfl_up(yp[NP - 1][j][i], 16, 64);
      if (s.lz > 0) yp[0][j][i] += r;
      if (!s.last_z) yp[NP - 1][j][i] = 0;
    }
  if (!s.owner) return;
#pragma unroll
  for (int z = 0; z < NP; ++z)
#pragma unroll
    for (int yy = 0; yy < NP; ++yy)
#pragma unroll
      for (int x = 0; x < NP; ++x) {
        const bool main = x < K - 1 && yy < K - 1 && z < K - 1;
        if (main) {
          op.store_p(col.p_at(s.cz, x, yy, z), yp[z][yy][x], p[z][yy][x], pre[main ? z : 0][main ? yy : 0][main ? x : 0]);
        } else if (((x < K - 1) | s.last_x) & ((yy < K - 1) | s.last_y) & ((z < K - 1) | s.last_z)) {
          const BOff gi = col.p_at(s.cz, x, yy, z);
          op.store_p(gi, yp[z][yy][x], p[z][yy][x], op.fetch_p(gi));
        }
      }
}

template <int K, typename T, int BLK, class Op>
__global__ void __launch_bounds__(64)
block3d_kernel(const Geo3<T> g, const Op op) {
  constexpr bool OUT_U = (BLK & (BLK_A | BLK_MASS | BLK_BT)) != 0;
  constexpr bool OUT_P = (BLK & (BLK_B | BLK_C)) != 0;
  constexpr int NFIELD = (OUT_U ? 3 : 0) + (OUT_P ? 1 : 0);
  const int b = xcd_contiguous_tile(blockIdx.x, gridDim.x);
  int field, cx, cy;
  Block3D s;
  block3d_decode(g, NFIELD, b, (int)threadIdx.x, field, s, cx, cy);
  const Column3D<K, T> col(g, cx, cy);
  if constexpr (OUT_U) {
    switch (field) {
      case 0: block_vel<K, T, BLK, Op, 0>(g, op, col, s); return;
      case 1: block_vel<K, T, BLK, Op, 1>(g, op, col, s); return;
      case 2: block_vel<K, T, BLK, Op, 2>(g, op, col, s); return;
      default: break;
    }
  }
  if constexpr (OUT_P) block_pres<K, T, BLK, Op>(g, op, col, s);
}

// ---------------------------------------------------------------------------
// Smallest levels: the cell block of block3d_kernel with one wave per output
// z-plane of the cell (three waves per block and output field for the
// velocity, two for the pressure).  Each wave reads the whole cell but
// contracts in z only for its own plane, so its instruction chain -- the run
// time of a launch with a few dozen waves -- is about a third.  The z = k
// plane moves to the cell above through LDS (the x and y faces still by
// shuffles within the plane's wave).
// ---------------------------------------------------------------------------
// out = sum_z m[O][z] in[z] (TR: m[z][O]) for one output plane O
template <int O, bool TR, int NI, int NY, int NX, typename T, int R, int C>
__device__ __forceinline__ void plane_z(const T (&m)[R][C], const T (&in)[NI][NY][NX], T (&out)[1][NY][NX]) {
#pragma unroll
  for (int y = 0; y < NY; ++y)
#pragma unroll
    for (int x = 0; x < NX; ++x) {
      T acc = 0;
#pragma unroll
      for (int i = 0; i < NI; ++i) acc += (TR ? m[i][O] : m[O][i]) * in[i][y][x];
      out[0][y][x] = acc;
    }
}

// plane O of (A u + B^T p)_COMP (or M u), as vel_cell
template <int K, typename T, int BLK, int COMP, int O>
__device__ __forceinline__ void vel_plane(const Geo3<T> &g, T mu, const T (&u)[K + 1][K + 1][K + 1],
                                          const T (&p)[K][K][K], T (&y)[1][K + 1][K + 1]) {
  constexpr int NV = K + 1, NP = K;
  constexpr cfe::TabT<K, T> R = cfe::make_tab_t<K, T>();
  const T(&Bx)[K][K + 1] = COMP == 0 ? R.Gr : R.Nr;
  const T(&By)[K][K + 1] = COMP == 1 ? R.Gr : R.Nr;
  const T(&Bz)[K][K + 1] = COMP == 2 ? R.Gr : R.Nr;
  if constexpr ((BLK & BLK_A) != 0) {
    T X[NV][NV];
    const T ax = mu * g.sKx, bx = g.gr * g.sM;
#pragma unroll
    for (int i = 0; i < NV; ++i)
#pragma unroll
      for (int j = 0; j < NV; ++j) X[i][j] = ax * R.Kr[i][j] + bx * R.Mr[i][j];
    T a[1][NV][NV], b[1][NV][NV], t[1][NV][NV];
    plane_z<O, false>(R.Mr, u, a);
    plane_z<O, false>(R.Kr, u, b);
    pass_y<false, false>(R.Mr, a, t, T(1));
    pass_x<false, false>(X, t, y, T(1));
    pass_y<false, false>(R.Kr, a, t, T(1));
    pass_y<false, true>(R.Mr, b, t, g.rz);
    pass_x<false, true>(R.Mr, t, y, mu * g.sKy);
  } else if constexpr ((BLK & BLK_MASS) != 0) {
    T a[1][NV][NV], t[1][NV][NV];
    plane_z<O, false>(R.Mr, u, a);
    pass_y<false, false>(R.Mr, a, t, T(1));
    pass_x<false, false>(R.Mr, t, y, g.sM);
  }
  if constexpr ((BLK & BLK_BT) != 0) {
    constexpr bool ACC = (BLK & (BLK_A | BLK_MASS)) != 0;
    T s1[1][NP][NP], s2[1][NV][NP];
    plane_z<O, true>(Bz, p, s1);
    pass_y<true, false>(By, s1, s2, T(1));
    pass_x<true, ACC>(Bx, s2, y, -g.sB[COMP]);
  } else if constexpr ((BLK & (BLK_A | BLK_MASS)) == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j)
#pragma unroll
      for (int i = 0; i < NV; ++i) y[0][j][i] = 0;
  }
}

// plane O (< K) of B u -/+ C p
template <int K, typename T, int BLK, int O>
__device__ __forceinline__ void pres_plane(const Geo3<T> &g, const T (&ub)[3][K + 1][K + 1][K + 1],
                                           const T (&p)[K][K][K], T (&yp)[1][K][K]) {
  constexpr int NV = K + 1, NP = K;
  constexpr cfe::TabT<K, T> R = cfe::make_tab_t<K, T>();
#pragma unroll
  for (int j = 0; j < NP; ++j)
#pragma unroll
    for (int i = 0; i < NP; ++i) yp[0][j][i] = 0;
  if constexpr ((BLK & BLK_B) != 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T w1[1][NV][NV], w2[1][NP][NV];
      plane_z<O, false>(c == 2 ? R.Gr : R.Nr, ub[c], w1);
      pass_y<false, false>(c == 1 ? R.Gr : R.Nr, w1, w2, T(1));
      pass_x<false, true>(c == 0 ? R.Gr : R.Nr, w2, yp, -g.sB[c]);
    }
  }
  if constexpr ((BLK & BLK_C) != 0) {
    const T sc = ((BLK & BLK_CPLUS) ? g.cp : -g.cp) * g.sM;
    T q1[1][NP][NP], q2[1][NP][NP];
    plane_z<O, false>(R.Mpr, p, q1);
    pass_y<false, false>(R.Mpr, q1, q2, T(1));
    pass_x<false, true>(R.Mpr, q2, yp, sc);
  }
}

template <int K, typename T, int BLK, class Op, int COMP>
__device__ __forceinline__ void block_vel_planes(const Geo3<T> &g, const Op &op, const Column3D<K, T> &col,
                                                 const Block3D &s, int o, T (*lds)[K + 1][K + 1]) {
  constexpr int NV = K + 1, NP = K;
  constexpr bool NEED_U = (BLK & (BLK_A | BLK_MASS)) != 0;
  constexpr bool NEED_P = (BLK & BLK_BT) != 0;
  T u[NV][NV][NV], p[NP][NP][NP];
  if constexpr (NEED_U) col.template load_u<0>(op, COMP, s.cz, u);
  if constexpr (NEED_P) col.template load_p<0>(op, s.cz, p);
  T mu = 0;
  if constexpr ((BLK & BLK_A) != 0) mu = col.mu_at(s.cz);
  typename Op::Pre pre[K][K];
  if (s.owner && o < K) {
#pragma unroll
    for (int yy = 0; yy < K; ++yy)
#pragma unroll
      for (int x = 0; x < K; ++x) pre[yy][x] = op.fetch_u(col.u_at(COMP, s.cz, x, yy, o));
  }
  __asm__ volatile("" ::: "memory");
#pragma unroll
  for (int z = 0; z < NV; ++z)
#pragma unroll
    for (int j = 0; j < NV; ++j)
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        if constexpr (NEED_U) {
          const bool keep = s.active & !(Op::ZERO_BC & col.vbc(s.cz, i, j, z));
          u[z][j][i] = keep ? u[z][j][i] : T(0);
        } else {
          u[z][j][i] = 0;
        }
      }
  if constexpr (NEED_P) {
#pragma unroll
    for (int z = 0; z < NP; ++z)
#pragma unroll
      for (int j = 0; j < NP; ++j)
#pragma unroll
        for (int i = 0; i < NP; ++i) p[z][j][i] = s.active ? p[z][j][i] : T(0);
  }
  T y[1][NV][NV];
  switch (o) {
    case 0: vel_plane<K, T, BLK, COMP, 0>(g, mu, u, p, y); break;
    case 1: vel_plane<K, T, BLK, COMP, 1>(g, mu, u, p, y); break;
    default: vel_plane<K, T, BLK, COMP, 2>(g, mu, u, p, y); break;
  }
  hand_over_xy<4>(y, s.lx, s.ly, s.last_x, s.last_y);
  // the z = K plane goes to plane 0 of the cell above (lane + 16)
  if (o == K) {
#pragma unroll
    for (int j = 0; j < NV; ++j)
#pragma unroll
      for (int i = 0; i < NV; ++i) lds[threadIdx.x % 64][j][i] = y[0][j][i];
  }
  __syncthreads();
  if (o == 0 && s.lz > 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j)
#pragma unroll
      for (int i = 0; i < NV; ++i) y[0][j][i] += lds[threadIdx.x % 64 - 16][j][i];
  }
  if (!s.owner) return;
  if (o < K) {
#pragma unroll
    for (int yy = 0; yy < K; ++yy)
#pragma unroll
      for (int x = 0; x < K; ++x) {
        // u[o] without a dynamic index into registers (o is wave-uniform)
        T uo = u[0][yy][x];
#pragma unroll
        for (int z = 1; z < K; ++z) uo = o == z ? u[z][yy][x] : uo;
        op.store_u(col.u_at(COMP, s.cz, x, yy, o), y[0][yy][x], uo, false, pre[yy][x]);
      }
    if (col.bxl | col.byl | ((s.cz == 0) & (o == 0))) {
#pragma unroll
      for (int yy = 0; yy < K; ++yy)
#pragma unroll
        for (int x = 0; x < K; ++x) {
          if (!col.vbc(s.cz, x, yy, o)) continue;
          const BOff gi = col.u_at(COMP, s.cz, x, yy, o);
          T rw = 0;
          if constexpr ((BLK & BLK_A) != 0) rw = op.load_u(gi);
          op.store_u(gi, rw, rw, true, pre[yy][x]);
        }
    }
  }
  // nodes on the domain's high faces in this plane: Dirichlet rows
  if (s.last_x | s.last_y | ((o == K) & s.last_z)) {
#pragma unroll
    for (int yy = 0; yy < NV; ++yy)
#pragma unroll
      for (int x = 0; x < NV; ++x) {
        if (x < K && yy < K && o < K) continue;
        if ((x == K && !s.last_x) || (yy == K && !s.last_y) || (o == K && !s.last_z)) continue;
        const BOff gi = col.u_at(COMP, s.cz, x, yy, o);
        T rw = 0;
        if constexpr ((BLK & BLK_A) != 0) rw = op.load_u(gi);
        op.store_u(gi, rw, rw, true, op.fetch_u(gi));
      }
  }
}

template <int K, typename T, int BLK, class Op>
__device__ __forceinline__ void block_pres_planes(const Geo3<T> &g, const Op &op, const Column3D<K, T> &col,
                                                  const Block3D &s, int o, T (*lds)[K + 1][K + 1]) {
  constexpr int NV = K + 1, NP = K;
  constexpr bool NEED_U = (BLK & BLK_B) != 0;
  constexpr bool NEED_P = (BLK & BLK_C) != 0;
  const bool act = o < NP;   // the pressure has K planes; the last wave only joins the barrier
  T ub[3][NV][NV][NV], p[NP][NP][NP];
  if constexpr (NEED_U) {
#pragma unroll
    for (int c = 0; c < 3; ++c) col.template load_u<0>(op, c, s.cz, ub[c]);
  }
  if constexpr (NEED_P) col.template load_p<0>(op, s.cz, p);
  typename Op::Pre pre[K - 1][K - 1];
  if (s.owner && o < K - 1) {
#pragma unroll
    for (int yy = 0; yy < K - 1; ++yy)
#pragma unroll
      for (int x = 0; x < K - 1; ++x) pre[yy][x] = op.fetch_p(col.p_at(s.cz, x, yy, o));
  }
  __asm__ volatile("" ::: "memory");
  if constexpr (NEED_U) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int z = 0; z < NV; ++z)
#pragma unroll
        for (int j = 0; j < NV; ++j)
#pragma unroll
          for (int i = 0; i < NV; ++i) {
            const bool keep = s.active & !(Op::ZERO_BC & col.vbc(s.cz, i, j, z));
            ub[c][z][j][i] = keep ? ub[c][z][j][i] : T(0);
          }
  }
#pragma unroll
  for (int z = 0; z < NP; ++z)
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
      for (int i = 0; i < NP; ++i) p[z][j][i] = (NEED_P && s.active) ? p[z][j][i] : T(0);
  T yp[1][NP][NP];
  switch (o) {
    case 0: pres_plane<K, T, BLK, 0>(g, ub, p, yp); break;
    default: pres_plane<K, T, BLK, K - 1>(g, ub, p, yp); break;
  }
  hand_over_xy<4>(yp, s.lx, s.ly, s.last_x, s.last_y);
  if (o == NP - 1) {
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
      for (int i = 0; i < NP; ++i) lds[threadIdx.x % 64][j][i] = yp[0][j][i];
  }
  __syncthreads();
  if (o == 0 && s.lz > 0) {
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
      for (int i = 0; i < NP; ++i) yp[0][j][i] += lds[threadIdx.x % 64 - 16][j][i];
  }
  if (!s.owner || !act) return;
  // plane o: nodes [0, K-1)^2 owned; the high faces as in the column sweep
#pragma unroll
  for (int yy = 0; yy < NP; ++yy)
#pragma unroll
    for (int x = 0; x < NP; ++x) {
      T po = p[0][yy][x];
#pragma unroll
      for (int z = 1; z < NP; ++z) po = o == z ? p[z][yy][x] : po;
      const bool main = x < K - 1 && yy < K - 1 && o < K - 1;
      if (main) {
        op.store_p(col.p_at(s.cz, x, yy, o), yp[0][yy][x], po, pre[main ? yy : 0][main ? x : 0]);
      } else if (((x < K - 1) | s.last_x) & ((yy < K - 1) | s.last_y) & ((o < K - 1) | s.last_z)) {
        const BOff gi = col.p_at(s.cz, x, yy, o);
        op.store_p(gi, yp[0][yy][x], po, op.fetch_p(gi));
      }
    }
}

template <int K, typename T, int BLK, class Op>
__global__ void __launch_bounds__(64 * (K + 1))
block3d_plane_kernel(const Geo3<T> g, const Op op) {
  static_assert(K == 2, "the plane switches below cover the K + 1 = 3 velocity planes of Q2");
  constexpr bool OUT_U = (BLK & (BLK_A | BLK_MASS | BLK_BT)) != 0;
  constexpr bool OUT_P = (BLK & (BLK_B | BLK_C)) != 0;
  constexpr int NFIELD = (OUT_U ? 3 : 0) + (OUT_P ? 1 : 0);
  __shared__ T lds[64][K + 1][K + 1];
  const int b = xcd_contiguous_tile(blockIdx.x, gridDim.x);
  const int o = __builtin_amdgcn_readfirstlane((int)threadIdx.x / 64);
  int field, cx, cy;
  Block3D s;
  block3d_decode(g, NFIELD, b, (int)threadIdx.x % 64, field, s, cx, cy);
  const Column3D<K, T> col(g, cx, cy);
  if constexpr (OUT_U) {
    switch (field) {
      case 0: block_vel_planes<K, T, BLK, Op, 0>(g, op, col, s, o, lds); return;
      case 1: block_vel_planes<K, T, BLK, Op, 1>(g, op, col, s, o, lds); return;
      case 2: block_vel_planes<K, T, BLK, Op, 2>(g, op, col, s, o, lds); return;
      default: break;
    }
  }
  if constexpr (OUT_P) block_pres_planes<K, T, BLK, Op>(g, op, col, s, o, lds);
}

// FP32 operator applications (OpApply) of the sweep ask for three waves per
// SIMD (168 VGPRs): measured faster than two although a few registers spill;
// the other epilogues spill inside the sweep at that limit and keep the
// default.
template <class Op, typename T>
constexpr int tile3d_waves_per_eu() {
  return (sizeof(T) == 4 && std::is_same<Op, OpApply<T>>::value) ? 3 : 1;
}

template <int K, typename T, int BLK, class Op, int TX, int TY>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(tile3d_waves_per_eu<Op, T>())))
tile3d_kernel(const Geo3<T> g, const Op op) {
  static_assert(TX * TY <= 64, "one wave per tile");
  constexpr bool OUT_U = (BLK & (BLK_A | BLK_MASS | BLK_BT)) != 0;
  constexpr bool OUT_P = (BLK & (BLK_B | BLK_C)) != 0;
  constexpr int NFIELD = (OUT_U ? 3 : 0) + (OUT_P ? 1 : 0);

  // block -> (field, x tile, z chunk, y tile); the fields of one tile and
  // chunk run on the same XCD and share its L2.
  const int b = xcd_contiguous_tile(blockIdx.x, gridDim.x);
  int field, cx, cy;
  Sweep s;
  if (!sweep3d_decode<TX, TY>(g, NFIELD, b, (int)threadIdx.x, field, s, cx, cy)) return;  // whole wave: empty chunk
  const Column3D<K, T> col(g, cx, cy);

  if constexpr (OUT_U) {
    switch (field) {
      case 0: vel_wave<K, T, BLK, Op, 0, TX>(g, op, col, s); return;
      case 1: vel_wave<K, T, BLK, Op, 1, TX>(g, op, col, s); return;
      case 2: vel_wave<K, T, BLK, Op, 2, TX>(g, op, col, s); return;
      default: break;
    }
  }
  if constexpr (OUT_P) pres_wave<K, T, BLK, Op, TX>(g, op, col, s);
}

}  // namespace smg
