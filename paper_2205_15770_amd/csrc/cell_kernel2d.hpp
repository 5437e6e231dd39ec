// Wave-tile application of the Taylor-Hood saddle-point operator
// K = [A B^T; B -C] on axis-aligned box cells in 2D (Sec. 3.1: K x =
// sum_tau P_tau K_tau P_tau^T x, cell matrices by sum factorisation).
//
// Work decomposition (gfx950): one wave64 per tile of 8 x 8 cells, one cell
// per lane (lane = x + 8 y).  The tile owns 7 x 7 cells; lane column 0 and
// lane row 0 are halo cells whose results are computed only to be handed
// over.  A lane applies both velocity blocks and the pressure block of its
// cell.  Contributions to nodes shared with the right / upper neighbour go to
// lane + 1 / lane + 8 by lane shuffles; afterwards each cell holds the
// complete sums of its nodes with local indices [0, K) (plus the domain high
// faces) and writes them through the epilogue functor.  No LDS, no barriers,
// no atomics; every output entry is written once.
//
// Cell matrices: compile-time 1D reference matrices and per-direction
// scalars; on a cell of widths (h_x, h_y)
//   A_cell = mu [sKx Kr(x)Mr + sKy Mr(x)Kr] + gamma rho sM Mr(x)Mr,
//   B_c    = -sB_c (Gr in direction c, Nr in the other),  C = cp sM Mpr(x)Mpr,
// with sKx = h_y / h_x, sKy = h_x / h_y, sM = h_x h_y, sB_x = h_y, sB_y = h_x.
#pragma once
#include <type_traits>

#include "cell_kernel.hpp"
#include "fe1d_const.hpp"
#include "ops.hpp"

namespace smg {

template <typename T>
struct Geo2 {
  int n[2];        // cells per direction
  int vd[2];       // velocity lattice extent per direction
  int pd[2];       // pressure lattice extent per direction
  int tiles[2];    // 8x8 wave tiles per direction
  uint32_t nv_bytes;  // bytes of one velocity component vector
  T mu, gr, cp;
  const T *mu_cell;
  T sKx, sKy, sM;
  T sB[2];
};

// The cell products of one cell (lane): yu_c = (A u_c | M u_c) + B_c^T p for
// the velocity fields selected by FIELD, yp = B u (+/- C p) for the pressure
// (FIELD -1: every output field of the block, 0 / 1: velocity component
// 0 / 1 only, 2: pressure only).  Inputs are masked already.
template <int K, typename T, int BLK, int FIELD>
__device__ __forceinline__ void cell2d_products(const Geo2<T> &g, const T mu, const T (&u)[2][1][K + 1][K + 1],
                                                const T (&p)[1][K][K], T (&yu)[2][1][K + 1][K + 1],
                                                T (&yp)[1][K][K]) {
  constexpr int NV = K + 1, NP = K;
  constexpr cfe::TabT<K, T> R = cfe::make_tab_t<K, T>();
  constexpr bool ALL_U = (BLK & (BLK_A | BLK_MASS | BLK_BT)) != 0;
  constexpr bool OUT_P = (BLK & (BLK_B | BLK_C)) != 0 && (FIELD == -1 || FIELD == 2);
  constexpr bool DU[2] = {ALL_U && (FIELD == -1 || FIELD == 0), ALL_U && (FIELD == -1 || FIELD == 1)};
  if constexpr ((BLK & BLK_A) != 0) {
    T X[NV][NV];
    const T axk = mu * g.sKx, bxm = g.gr * g.sM;
#pragma unroll
    for (int i = 0; i < NV; ++i)
#pragma unroll
      for (int j = 0; j < NV; ++j) X[i][j] = axk * R.Kr[i][j] + bxm * R.Mr[i][j];
    const T sy = mu * g.sKy;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (!DU[c]) continue;
      T t[1][NV][NV];
      pass_y<false, false>(R.Mr, u[c], t, T(1));
      pass_x<false, false>(X, t, yu[c], T(1));
      pass_y<false, false>(R.Kr, u[c], t, T(1));
      pass_x<false, true>(R.Mr, t, yu[c], sy);
    }
  } else if constexpr ((BLK & BLK_MASS) != 0) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (!DU[c]) continue;
      T t[1][NV][NV];
      pass_y<false, false>(R.Mr, u[c], t, T(1));
      pass_x<false, false>(R.Mr, t, yu[c], g.sM);
    }
  }
  if constexpr ((BLK & BLK_BT) != 0) {
    constexpr bool ACC = (BLK & (BLK_A | BLK_MASS)) != 0;
    if constexpr (DU[0]) {
      T s[1][NV][NP];
      pass_y<true, false>(R.Nr, p, s, T(1));
      pass_x<true, ACC>(R.Gr, s, yu[0], -g.sB[0]);
    }
    if constexpr (DU[1]) {
      T s2[1][NP][NV];
      pass_x<true, false>(R.Nr, p, s2, T(1));
      pass_y<true, ACC>(R.Gr, s2, yu[1], -g.sB[1]);
    }
  } else if constexpr (!ALL_U) {
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int y = 0; y < NV; ++y)
#pragma unroll
        for (int x = 0; x < NV; ++x) yu[c][0][y][x] = 0;
  }
  if constexpr (OUT_P) {
    if constexpr ((BLK & BLK_B) != 0) {
      T w[1][NV][NP];
      pass_x<false, false>(R.Gr, u[0], w, T(1));
      pass_y<false, false>(R.Nr, w, yp, -g.sB[0]);
      pass_x<false, false>(R.Nr, u[1], w, T(1));
      pass_y<false, true>(R.Gr, w, yp, -g.sB[1]);
    }
    if constexpr ((BLK & BLK_C) != 0) {
      constexpr bool ACC = (BLK & BLK_B) != 0;
      const T sc = ((BLK & BLK_CPLUS) ? g.cp : -g.cp) * g.sM;
      T q[1][NP][NP];
      pass_x<false, false>(R.Mpr, p, q, T(1));
      pass_y<false, ACC>(R.Mpr, q, yp, sc);
    }
  }

}

// One tile; FIELD = -1: every output field of the block, 0 / 1: velocity
// component 0 / 1 only, 2: pressure only (the split form for small levels,
// where a wave's instruction count is its latency).
template <int K, typename T, int BLK, class Op, int FIELD>
__device__ __forceinline__ void wave2d_tile(const Geo2<T> &g, const Op &op, int b) {
  constexpr int NV = K + 1, NP = K, TX = 8;
  constexpr uint32_t ST = sizeof(T);
  constexpr cfe::TabT<K, T> R = cfe::make_tab_t<K, T>();
  constexpr bool ALL_U = (BLK & (BLK_A | BLK_MASS | BLK_BT)) != 0;
  constexpr bool OUT_P = (BLK & (BLK_B | BLK_C)) != 0 && (FIELD == -1 || FIELD == 2);
  // per velocity component: computed here?
  constexpr bool DU[2] = {ALL_U && (FIELD == -1 || FIELD == 0), ALL_U && (FIELD == -1 || FIELD == 1)};
  constexpr bool OUT_U = DU[0] || DU[1];
  // inputs: u_c for A / M of component c and for B; p for B^T and C
  constexpr bool LU[2] = {(DU[0] && (BLK & (BLK_A | BLK_MASS)) != 0) || (OUT_P && (BLK & BLK_B) != 0),
                          (DU[1] && (BLK & (BLK_A | BLK_MASS)) != 0) || (OUT_P && (BLK & BLK_B) != 0)};
  constexpr bool NEED_P = (OUT_U && (BLK & BLK_BT) != 0) || (OUT_P && (BLK & BLK_C) != 0);

  const int tx = b % g.tiles[0], ty = b / g.tiles[0];
  const int lcx = threadIdx.x % TX, lcy = threadIdx.x / TX;
  const int gcx = tx * (TX - 1) - 1 + lcx, gcy = ty * (TX - 1) - 1 + lcy;
  const bool active = gcx >= 0 && gcx < g.n[0] && gcy >= 0 && gcy < g.n[1];
  const bool owner = active && lcx > 0 && lcy > 0;
  const bool bxl = gcx == 0, bxh = gcx == g.n[0] - 1, byl = gcy == 0, byh = gcy == g.n[1] - 1;
  // halo lanes outside the mesh read a valid cell and discard the values
  const int ax = gcx < 0 ? 0 : (gcx >= g.n[0] ? g.n[0] - 1 : gcx);
  const int ay = gcy < 0 ? 0 : (gcy >= g.n[1] ? g.n[1] - 1 : gcy);
  const uint32_t suy = ST * (uint32_t)g.vd[0], spy = ST * (uint32_t)g.pd[0];
  const uint32_t base_u = ST * (uint32_t)(K * ax) + suy * (uint32_t)(K * ay);
  const uint32_t base_p = ST * (uint32_t)((K - 1) * ax) + spy * (uint32_t)((K - 1) * ay);
  auto u_at = [&](int c, int x, int y) { return BOff{(uint32_t)c * g.nv_bytes + base_u + suy * (uint32_t)y, ST * (uint32_t)x}; };
  auto p_at = [&](int x, int y) { return BOff{base_p + spy * (uint32_t)y, ST * (uint32_t)x}; };
  auto vbc = [&](int x, int y) { return ((x == 0) & bxl) | ((x == K) & bxh) | ((y == 0) & byl) | ((y == K) & byh); };

  // 1. requests: cell DoFs, viscosity, epilogue inputs of the owned nodes
  T u[2][1][NV][NV], p[1][NP][NP];
#pragma unroll
  for (int c = 0; c < 2; ++c) {
    if (!LU[c]) continue;
#pragma unroll
    for (int y = 0; y < NV; ++y)
#pragma unroll
      for (int x = 0; x < NV; ++x) u[c][0][y][x] = op.load_u(u_at(c, x, y));
  }
  if constexpr (NEED_P) {
#pragma unroll
    for (int y = 0; y < NP; ++y)
#pragma unroll
      for (int x = 0; x < NP; ++x) p[0][y][x] = op.load_p(p_at(x, y));
  }
  T mu = g.mu;
  if constexpr ((BLK & BLK_A) != 0)
    if (g.mu_cell != nullptr) mu = g.mu_cell[(uint32_t)ax + (uint32_t)g.n[0] * (uint32_t)ay];
  typename Op::Pre pre_u[2][K][K];
  typename Op::Pre pre_p[K - 1][K - 1];
  if (owner) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (!DU[c]) continue;
#pragma unroll
      for (int y = 0; y < K; ++y)
#pragma unroll
        for (int x = 0; x < K; ++x) pre_u[c][y][x] = op.fetch_u(u_at(c, x, y));
    }
    if constexpr (OUT_P) {
#pragma unroll
      for (int y = 0; y < K - 1; ++y)
#pragma unroll
        for (int x = 0; x < K - 1; ++x) pre_p[y][x] = op.fetch_p(p_at(x, y));
    }
  }
  // keep the requests above unconditional: no load below this point may be
  // moved into a branch by the select that follows
  __asm__ volatile("" ::: "memory");

  // 2. mask: inactive cells, Dirichlet inputs (ZERO_BC)
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int y = 0; y < NV; ++y)
#pragma unroll
      for (int x = 0; x < NV; ++x) {
        const bool keep = LU[c] & active & !(Op::ZERO_BC & vbc(x, y));
        u[c][0][y][x] = keep ? u[c][0][y][x] : T(0);
      }
  if constexpr (NEED_P) {
#pragma unroll
    for (int y = 0; y < NP; ++y)
#pragma unroll
      for (int x = 0; x < NP; ++x) p[0][y][x] = active ? p[0][y][x] : T(0);
  } else {
#pragma unroll
    for (int y = 0; y < NP; ++y)
#pragma unroll
      for (int x = 0; x < NP; ++x) p[0][y][x] = 0;
  }

  // 3. cell matrices
  T yu[2][1][NV][NV], yp[1][NP][NP];
  cell2d_products<K, T, BLK, FIELD>(g, mu, u, p, yu, yp);

  // 4. hand-over to the right (lane + 1) and upper (lane + 8) neighbours
#pragma unroll
  for (int c = 0; c < 2; ++c)
    if (DU[c]) hand_over_xy<TX>(yu[c], lcx, lcy, bxh, byh);
  if constexpr (OUT_P) hand_over_xy<TX>(yp, lcx, lcy, bxh, byh);

  // 5. owned nodes
  if (!owner) return;
  if constexpr (OUT_U) {
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      if (!DU[c]) continue;
#pragma unroll
      for (int y = 0; y < K; ++y)
#pragma unroll
        for (int x = 0; x < K; ++x) op.store_u(u_at(c, x, y), yu[c][0][y][x], u[c][0][y][x], false, pre_u[c][y][x]);
    }
    if (bxl | byl) {
      // Dirichlet rows on the low faces (rewritten: same lane, program order)
#pragma unroll
      for (int c = 0; c < 2; ++c)
        if (DU[c])
#pragma unroll
        for (int y = 0; y < K; ++y)
#pragma unroll
          for (int x = 0; x < K; ++x) {
            if (!vbc(x, y)) continue;
            const BOff gi = u_at(c, x, y);
            T rw = 0;
            if constexpr ((BLK & BLK_A) != 0) rw = op.load_u(gi);
            op.store_u(gi, rw, rw, true, pre_u[c][y][x]);
          }
    }
    if (bxh | byh) {
      // nodes on the domain's high faces: Dirichlet rows
#pragma unroll
      for (int c = 0; c < 2; ++c)
        if (DU[c])
#pragma unroll
        for (int y = 0; y < NV; ++y)
#pragma unroll
          for (int x = 0; x < NV; ++x) {
            if (x < K && y < K) continue;
            if ((x == K && !bxh) || (y == K && !byh)) continue;
            const BOff gi = u_at(c, x, y);
            T rw = 0;
            if constexpr ((BLK & BLK_A) != 0) rw = op.load_u(gi);
            op.store_u(gi, rw, rw, true, op.fetch_u(gi));
          }
    }
  }
  if constexpr (OUT_P) {
#pragma unroll
    for (int y = 0; y < NP; ++y)
#pragma unroll
      for (int x = 0; x < NP; ++x) {
        const bool main = x < K - 1 && y < K - 1;
        if (main) {
          op.store_p(p_at(x, y), yp[0][y][x], p[0][y][x], pre_p[main ? y : 0][main ? x : 0]);
        } else if (((x < K - 1) | bxh) & ((y < K - 1) | byh)) {
          const BOff gi = p_at(x, y);
          op.store_p(gi, yp[0][y][x], p[0][y][x], op.fetch_p(gi));
        }
      }
  }
}

template <int K, typename T, int BLK, class Op>
__global__ void __launch_bounds__(64)
wave2d_kernel(const Geo2<T> g, const Op op) {
  wave2d_tile<K, T, BLK, Op, -1>(g, op, xcd_contiguous_tile(blockIdx.x, gridDim.x));
}

// Split form: one wave per (tile, output field); the fields of a tile are
// consecutive blocks (same XCD).
template <int K, typename T, int BLK, class Op>
__global__ void __launch_bounds__(64)
wave2d_split_kernel(const Geo2<T> g, const Op op) {
  constexpr bool OUT_U = (BLK & (BLK_A | BLK_MASS | BLK_BT)) != 0;
  constexpr bool OUT_P = (BLK & (BLK_B | BLK_C)) != 0;
  constexpr int NF = (OUT_U ? 2 : 0) + (OUT_P ? 1 : 0);
  const int bb = xcd_contiguous_tile(blockIdx.x, gridDim.x);
  const int f = bb % NF, b = bb / NF;
  if constexpr (OUT_U) {
    if (f == 0) { wave2d_tile<K, T, BLK, Op, 0>(g, op, b); return; }
    if (f == 1) { wave2d_tile<K, T, BLK, Op, 1>(g, op, b); return; }
  }
  if constexpr (OUT_P) wave2d_tile<K, T, BLK, Op, 2>(g, op, b);
}


// ---------------------------------------------------------------------------
// After hand_over_xy a lane holds the complete sums of its cell's nodes with
// local indices [0, N-1) in both directions (and of the faces on the
// domain's high boundary).  This fills the faces x = N-1 / y = N-1 and their
// corner from the lanes that hold them completely: the right cell (lane + 1),
// the upper cell (lane + TX) and the upper-right cell (lane + TX + 1).  On the
// domain's high faces the local values are kept.  The result is the whole
// cell on every lane whose right, upper and upper-right neighbours hold
// complete sums.
template <int TX, typename T, int N>
__device__ __forceinline__ void gather_high_faces(T (&v)[N][N], bool bxh, bool byh) {
  constexpr int E = N - 1;
  T colE[E], rowE[E];
#pragma unroll
  for (int j = 0; j < E; ++j) colE[j] = __shfl_down(v[j][0], 1, 64);
#pragma unroll
  for (int i = 0; i < E; ++i) rowE[i] = __shfl_down(v[0][i], TX, 64);
  const T c9 = __shfl_down(v[0][0], TX + 1, 64);   // (0, 0) of the upper-right cell
  const T c8 = __shfl_down(v[0][E], TX, 64);       // (E, 0) of the upper cell (its right face is local)
  const T c1 = __shfl_down(v[E][0], 1, 64);        // (0, E) of the right cell (its upper face is local)
  if (!bxh) {
#pragma unroll
    for (int j = 0; j < E; ++j) v[j][E] = colE[j];
  }
  if (!byh) {
#pragma unroll
    for (int i = 0; i < E; ++i) v[E][i] = rowE[i];
  }
  if (!bxh && !byh) v[E][E] = c9;
  else if (bxh && !byh) v[E][E] = c8;
  else if (!bxh && byh) v[E][E] = c1;
}

// ---------------------------------------------------------------------------
// Two operator applications in one launch (small levels, where a launch costs
// more than its arithmetic): a velocity field v is formed by a first
// application -- q = B^T d (OpGrad) or the residual r = f - A u - B^T p
// (OpResidual) -- and fed directly into the first step of the Chebyshev
// recurrence for A (OpChebA with FIRST).  v never goes to memory.  After the
// first hand-over, lanes 1..7 hold the complete sums of their owned nodes;
// the values on a cell's right / upper faces and corner come back from lanes
// + 1, + 8, + 9 (or stay local on the domain's high faces), so lanes 1..6 in
// each direction hold v on their whole cell.  The second application runs on
// those lanes only; after its hand-over, lanes 2..6 hold complete sums: the
// tile owns 5 x 5 cells (halo: two cell rings below, one above).  Dirichlet
// rows of v take the values the separate launches would store (r = f - u for
// the residual, 0 for q), so the result equals the two-launch sequence.
// One wave per (tile, velocity component).
// ---------------------------------------------------------------------------
// Workgroups of WX x WY waves, each an 8 x 8 block of cells (one per lane),
// the blocks side by side without overlap.  The two helpers below do what
// hand_over_xy and gather_high_faces do inside a wave, across the whole
// workgroup: values that cross a wave boundary go through LDS.  Every wave of
// the workgroup calls them (they hold barriers).
template <int WX, int WY, int N, typename T>
struct WgFaces {
  T x[WX * WY * 8 * N];    // x step of a hand-over
  T y[WX * WY * 8 * N];    // y step of a hand-over
  T gx[WX * WY * 8 * N];   // published left columns (gather)
  T gy[WX * WY * 8 * N];   // published bottom rows (gather)
};

template <int WX, int WY, typename T, int N>
__device__ __forceinline__ void wg_hand_over(T (&y)[1][N][N], int lcx, int lcy, int wx, int wy, bool last_x,
                                             bool last_y, WgFaces<WX, WY, N, T> &sh) {
  constexpr int TX = 8;
  const int w = wx + WX * wy;
  T r[N];
#pragma unroll
  for (int j = 0; j < N; ++j) r[j] = __shfl_up(y[0][j][N - 1], 1, TX);
  if (lcx == TX - 1 && wx < WX - 1) {
#pragma unroll
    for (int j = 0; j < N; ++j) sh.x[(w * TX + lcy) * N + j] = y[0][j][N - 1];
  }
  __syncthreads();
  if (lcx == 0 && wx > 0) {
#pragma unroll
    for (int j = 0; j < N; ++j) r[j] = sh.x[((w - 1) * TX + lcy) * N + j];
  }
  const bool from_left = lcx > 0 || wx > 0;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    if (from_left) y[0][j][0] += r[j];
    if (!last_x) y[0][j][N - 1] = 0;
  }
#pragma unroll
  for (int i = 0; i < N; ++i) r[i] = __shfl_up(y[0][N - 1][i], TX, 64);
  if (lcy == TX - 1 && wy < WY - 1) {
#pragma unroll
    for (int i = 0; i < N; ++i) sh.y[(w * TX + lcx) * N + i] = y[0][N - 1][i];
  }
  __syncthreads();
  if (lcy == 0 && wy > 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) r[i] = sh.y[((w - WX) * TX + lcx) * N + i];
  }
  const bool from_below = lcy > 0 || wy > 0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    if (from_below) y[0][0][i] += r[i];
    if (!last_y) y[0][N - 1][i] = 0;
  }
}

template <int WX, int WY, typename T, int N>
__device__ __forceinline__ void wg_gather_high_faces(T (&v)[N][N], int lcx, int lcy, int wx, int wy, bool bxh,
                                                     bool byh, WgFaces<WX, WY, N, T> &sh) {
  constexpr int E = N - 1, TX = 8;
  const int w = wx + WX * wy;
  // publish the left column of the lanes at lcx = 0 and the bottom row of the
  // lanes at lcy = 0
  if (lcx == 0) {
#pragma unroll
    for (int j = 0; j < N; ++j) sh.gx[(w * TX + lcy) * N + j] = v[j][0];
  }
  if (lcy == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) sh.gy[(w * TX + lcx) * N + i] = v[0][i];
  }
  T colE[E], rowE[E];
#pragma unroll
  for (int j = 0; j < E; ++j) colE[j] = __shfl_down(v[j][0], 1, 64);
#pragma unroll
  for (int i = 0; i < E; ++i) rowE[i] = __shfl_down(v[0][i], TX, 64);
  T c9 = __shfl_down(v[0][0], TX + 1, 64);   // (0, 0) of the upper-right cell
  T c8 = __shfl_down(v[0][E], TX, 64);       // (E, 0) of the upper cell
  T c1 = __shfl_down(v[E][0], 1, 64);        // (0, E) of the right cell
  __syncthreads();
  const bool rx = lcx == TX - 1 && wx < WX - 1, ry = lcy == TX - 1 && wy < WY - 1;
  const int wr = w + 1, wu = w + WX;
  if (rx) {
#pragma unroll
    for (int j = 0; j < E; ++j) colE[j] = sh.gx[(wr * TX + lcy) * N + j];
    c1 = sh.gx[(wr * TX + lcy) * N + E];
  }
  if (ry) {
#pragma unroll
    for (int i = 0; i < E; ++i) rowE[i] = sh.gy[(wu * TX + lcx) * N + i];
    c8 = sh.gy[(wu * TX + lcx) * N + E];
  }
  if (lcx == TX - 1 && lcy < TX - 1 && rx) c9 = sh.gx[(wr * TX + lcy + 1) * N];
  else if (lcy == TX - 1 && lcx < TX - 1 && ry) c9 = sh.gy[(wu * TX + lcx + 1) * N];
  else if (lcx == TX - 1 && lcy == TX - 1 && rx && ry) c9 = sh.gx[((wu + 1) * TX) * N];
  if (!bxh) {
#pragma unroll
    for (int j = 0; j < E; ++j) v[j][E] = colE[j];
  }
  if (!byh) {
#pragma unroll
    for (int i = 0; i < E; ++i) v[E][i] = rowE[i];
  }
  if (!bxh && !byh) v[E][E] = c9;
  else if (bxh && !byh) v[E][E] = c8;
  else if (!bxh && byh) v[E][E] = c1;
}

template <class Op>
struct is_residual_op : std::false_type {};
template <typename T>
struct is_residual_op<OpResidual<T>> : std::true_type {};

template <int K, typename T, class Op1, bool LAST, int WX = 1, int WY = 1>
__device__ __forceinline__ void wave2d_fused_body(const Geo2<T> &g, const Op1 &op1, const OpChebA<T, true, LAST> &op2,
                                                  const int bb, WgFaces<WX, WY, K + 1, T> *sh = nullptr) {
  constexpr int NV = K + 1, NP = K, TX = 8;
  constexpr int CXW = TX * WX, CYW = TX * WY;       // cells of the tile
  constexpr int OWNX = CXW - 3, OWNY = CYW - 3;     // owned cells
  constexpr bool WG = WX * WY > 1;
  constexpr uint32_t ST = sizeof(T);
  constexpr cfe::TabT<K, T> R = cfe::make_tab_t<K, T>();
  constexpr bool RESID = is_residual_op<Op1>::value;

  const int c = bb % 2, b = bb / 2;
  const int tx = b % g.tiles[0], ty = b / g.tiles[0];
  const int lane = threadIdx.x % 64;
  const int wv = WG ? __builtin_amdgcn_readfirstlane((int)threadIdx.x / 64) : 0;
  const int wx = wv % WX, wy = wv / WX;
  const int lcx = lane % TX, lcy = lane / TX;
  const int lx = TX * wx + lcx, ly = TX * wy + lcy;   // cell of the tile
  const int gcx = tx * OWNX - 2 + lx, gcy = ty * OWNY - 2 + ly;
  const bool active = gcx >= 0 && gcx < g.n[0] && gcy >= 0 && gcy < g.n[1];
  const bool valid2 = active && lx >= 1 && lx <= CXW - 2 && ly >= 1 && ly <= CYW - 2;
  const bool owner = active && lx >= 2 && lx <= CXW - 2 && ly >= 2 && ly <= CYW - 2;
  const bool bxl = gcx == 0, bxh = gcx == g.n[0] - 1, byl = gcy == 0, byh = gcy == g.n[1] - 1;
  const int ax = gcx < 0 ? 0 : (gcx >= g.n[0] ? g.n[0] - 1 : gcx);
  const int ay = gcy < 0 ? 0 : (gcy >= g.n[1] ? g.n[1] - 1 : gcy);
  const uint32_t suy = ST * (uint32_t)g.vd[0], spy = ST * (uint32_t)g.pd[0];
  const uint32_t base_u = (uint32_t)c * g.nv_bytes + ST * (uint32_t)(K * ax) + suy * (uint32_t)(K * ay);
  const uint32_t base_p = ST * (uint32_t)((K - 1) * ax) + spy * (uint32_t)((K - 1) * ay);
  auto u_at = [&](int x, int y) { return BOff{base_u + suy * (uint32_t)y, ST * (uint32_t)x}; };
  auto p_at = [&](int x, int y) { return BOff{base_p + spy * (uint32_t)y, ST * (uint32_t)x}; };
  auto vbc = [&](int x, int y) { return ((x == 0) & bxl) | ((x == K) & bxh) | ((y == 0) & byl) | ((y == K) & byh); };

  // 1. requests: first-stage inputs, the second stage's D^-1 on the whole
  //    cell, its base vector on the owned nodes
  T u[1][NV][NV], f[NV][NV], p[1][NP][NP], dv[NV][NV], bs[K][K];
  if constexpr (RESID) {
#pragma unroll
    for (int y = 0; y < NV; ++y)
#pragma unroll
      for (int x = 0; x < NV; ++x) {
        u[0][y][x] = op1.load_u(u_at(x, y));
        f[y][x] = op1.fetch_u(u_at(x, y)).b;
      }
  }
#pragma unroll
  for (int y = 0; y < NP; ++y)
#pragma unroll
    for (int x = 0; x < NP; ++x) p[0][y][x] = op1.load_p(p_at(x, y));
#pragma unroll
  for (int y = 0; y < NV; ++y)
#pragma unroll
    for (int x = 0; x < NV; ++x) dv[y][x] = at(op2.dinv, u_at(x, y));
  T mu = g.mu;
  if constexpr (RESID)
    if (g.mu_cell != nullptr) mu = g.mu_cell[(uint32_t)ax + (uint32_t)g.n[0] * (uint32_t)ay];
  if (owner) {
#pragma unroll
    for (int y = 0; y < K; ++y)
#pragma unroll
      for (int x = 0; x < K; ++x) bs[y][x] = (LAST && op2.base) ? at(op2.base, u_at(x, y)) : T(0);
  }
  if constexpr (!RESID) {
    if (g.mu_cell != nullptr) mu = g.mu_cell[(uint32_t)ax + (uint32_t)g.n[0] * (uint32_t)ay];
  }
  __asm__ volatile("" ::: "memory");

  const T axk = mu * g.sKx, bxm = g.gr * g.sM, sy = mu * g.sKy;
  T X[NV][NV];
#pragma unroll
  for (int i = 0; i < NV; ++i)
#pragma unroll
    for (int j = 0; j < NV; ++j) X[i][j] = axk * R.Kr[i][j] + bxm * R.Mr[i][j];
  // A of one component on this cell: out = A in
  auto apply_A = [&](const T (&in)[1][NV][NV], T (&out)[1][NV][NV]) {
    T t[1][NV][NV];
    pass_y<false, false>(R.Mr, in, t, T(1));
    pass_x<false, false>(X, t, out, T(1));
    pass_y<false, false>(R.Kr, in, t, T(1));
    pass_x<false, true>(R.Mr, t, out, sy);
  };

  // 2. first stage
  T um[1][NV][NV], t1[1][NV][NV];
#pragma unroll
  for (int y = 0; y < NV; ++y)
#pragma unroll
    for (int x = 0; x < NV; ++x) um[0][y][x] = (RESID && active && !vbc(x, y)) ? u[0][y][x] : T(0);
#pragma unroll
  for (int y = 0; y < NP; ++y)
#pragma unroll
    for (int x = 0; x < NP; ++x) p[0][y][x] = active ? p[0][y][x] : T(0);
  if constexpr (RESID) apply_A(um, t1);
  {
    // B^T_c p
    constexpr bool ACC = RESID;
    if (c == 0) {
      T s1[1][NV][NP];
      pass_y<true, false>(R.Nr, p, s1, T(1));
      pass_x<true, ACC>(R.Gr, s1, t1, -g.sB[0]);
    } else {
      T s2[1][NP][NV];
      pass_x<true, false>(R.Nr, p, s2, T(1));
      pass_y<true, ACC>(R.Gr, s2, t1, -g.sB[1]);
    }
  }
  if constexpr (WG) wg_hand_over<WX, WY>(t1, lcx, lcy, wx, wy, bxh, byh, *sh);
  else hand_over_xy<TX>(t1, lcx, lcy, bxh, byh);
  // v on the nodes this lane holds completely
  T v[NV][NV];
#pragma unroll
  for (int y = 0; y < NV; ++y)
#pragma unroll
    for (int x = 0; x < NV; ++x) {
      const T free_v = RESID ? f[y][x] - t1[0][y][x] : t1[0][y][x];
      const T bc_v = RESID ? f[y][x] - u[0][y][x] : T(0);
      v[y][x] = vbc(x, y) ? bc_v : free_v;
    }
  // 3. right / upper faces and corner from the owners (lane + 1, + 8, + 9)
  if constexpr (WG) wg_gather_high_faces<WX, WY>(v, lcx, lcy, wx, wy, bxh, byh, *sh);
  else gather_high_faces<TX>(v, bxh, byh);
  // 4. second stage: t2 = A d0, d0 = D^-1 v / theta (inputs of the valid lanes only)
  T d0[1][NV][NV], t2[1][NV][NV];
#pragma unroll
  for (int y = 0; y < NV; ++y)
#pragma unroll
    for (int x = 0; x < NV; ++x) {
      const T d = dv[y][x] * v[y][x] * op2.inv_theta;
      d0[0][y][x] = (valid2 && !vbc(x, y)) ? d : T(0);
    }
  apply_A(d0, t2);
  if constexpr (WG) wg_hand_over<WX, WY>(t2, lcx, lcy, wx, wy, bxh, byh, *sh);
  else hand_over_xy<TX>(t2, lcx, lcy, bxh, byh);

  // 5. owned nodes through the Chebyshev epilogue
  if (!owner) return;
  using Pre2 = typename OpChebA<T, true, LAST>::Pre;
  auto pre_at = [&](int x, int y, T base) {
    Pre2 q;
    q.r = v[y][x];
    q.x = T(0);
    q.dinv = dv[y][x];
    q.base = base;
    return q;
  };
#pragma unroll
  for (int y = 0; y < K; ++y)
#pragma unroll
    for (int x = 0; x < K; ++x) op2.store_u(u_at(x, y), t2[0][y][x], d0[0][y][x], false, pre_at(x, y, bs[y][x]));
  if (bxl | byl) {
#pragma unroll
    for (int y = 0; y < K; ++y)
#pragma unroll
      for (int x = 0; x < K; ++x) {
        if (!vbc(x, y)) continue;
        const T rw = dv[y][x] * v[y][x] * op2.inv_theta;
        op2.store_u(u_at(x, y), rw, rw, true, pre_at(x, y, bs[y][x]));
      }
  }
  if (bxh | byh) {
#pragma unroll
    for (int y = 0; y < NV; ++y)
#pragma unroll
      for (int x = 0; x < NV; ++x) {
        if (x < K && y < K) continue;
        if ((x == K && !bxh) || (y == K && !byh)) continue;
        const BOff gi = u_at(x, y);
        const T rw = dv[y][x] * v[y][x] * op2.inv_theta;
        op2.store_u(gi, rw, rw, true, pre_at(x, y, (LAST && op2.base) ? at(op2.base, gi) : T(0)));
      }
  }
}

// ---------------------------------------------------------------------------
// Three operator applications in one launch (small levels, k_S = 1): a
// pressure stage in front of the fused pair above.  Stage 0 applies B (and
// C) to the pressure patch of every lane and turns the sums into a pressure
// vector z; stage 1 forms q_c = B_c^T z; stage 2 is the first Chebyshev step
// for A on q_c.  Each stage shrinks the region of complete sums by one cell
// ring: the 8 x 8 tile owns 3 x 3 cells (halo: three rings below, two
// above).  Stage 0 is one of
//   F3_DIVRES: r_p = B u - C p - g (stored by the owners), z = D~_S^-1 r_p / theta_S,
//              the Uzawa pressure residual and the first S~ direction;
//   F3_CHEBS:  the only step of Cheb(S~, D~_S, 1): d_0 = D~_S^-1 r_0 / theta_S,
//              t = B w + C d_0, z = tau (d_0 + c1 d_0 + c2 D~_S^-1 (r_0 - t)),
//              p += z by the owners; z is the pressure update dp.
// Both velocity components of u (w) are read by every wave; one wave per
// (tile, velocity component), and the component-0 wave stores the pressure
// output.  The arithmetic is that of the separate launches.
enum : int { F3_DIVRES = 0, F3_CHEBS = 1 };

template <typename T>
struct Fuse3P {
  const T *u;        // velocity input of B: u_hat (F3_DIVRES) or w (F3_CHEBS)
  const T *p0;       // F3_DIVRES: pressure iterate of the C term
  const T *g;        // F3_DIVRES: pressure right-hand side (nullable)
  T *rp;             // F3_DIVRES: r_p
  const T *rin;      // F3_CHEBS: r_0
  const T *dinv_s;   // D~_S^-1
  T *p;              // F3_CHEBS: pressure iterate, += dp (nullable)
  T inv_theta, c1, c2, tau;  // of the S~ Chebyshev step
};

template <int K, typename T, int MODE, bool LAST>
__device__ __forceinline__ void wave2d_fused3_body(const Geo2<T> &g, const Fuse3P<T> &P,
                                                   const OpChebA<T, true, LAST> &op2, const int bb) {
  constexpr int NV = K + 1, NP = K, TX = 8, OWN = TX - 5;
  constexpr uint32_t ST = sizeof(T);
  constexpr cfe::TabT<K, T> R = cfe::make_tab_t<K, T>();

  const int c = bb % 2, b = bb / 2;
  const int tx = b % g.tiles[0], ty = b / g.tiles[0];
  const int lcx = threadIdx.x % TX, lcy = threadIdx.x / TX;
  const int gcx = tx * OWN - 3 + lcx, gcy = ty * OWN - 3 + lcy;
  const bool active = gcx >= 0 && gcx < g.n[0] && gcy >= 0 && gcy < g.n[1];
  const bool valid1 = active && lcx >= 1 && lcx <= TX - 2 && lcy >= 1 && lcy <= TX - 2;
  const bool valid2 = active && lcx >= 2 && lcx <= TX - 3 && lcy >= 2 && lcy <= TX - 3;
  const bool owner = active && lcx >= 3 && lcx <= TX - 3 && lcy >= 3 && lcy <= TX - 3;
  const bool bxl = gcx == 0, bxh = gcx == g.n[0] - 1, byl = gcy == 0, byh = gcy == g.n[1] - 1;
  const int ax = gcx < 0 ? 0 : (gcx >= g.n[0] ? g.n[0] - 1 : gcx);
  const int ay = gcy < 0 ? 0 : (gcy >= g.n[1] ? g.n[1] - 1 : gcy);
  const uint32_t suy = ST * (uint32_t)g.vd[0], spy = ST * (uint32_t)g.pd[0];
  const uint32_t base_u0 = ST * (uint32_t)(K * ax) + suy * (uint32_t)(K * ay);
  const uint32_t base_p = ST * (uint32_t)((K - 1) * ax) + spy * (uint32_t)((K - 1) * ay);
  auto uc_at = [&](int cc, int x, int y) { return BOff{(uint32_t)cc * g.nv_bytes + base_u0 + suy * (uint32_t)y, ST * (uint32_t)x}; };
  auto u_at = [&](int x, int y) { return uc_at(c, x, y); };
  auto p_at = [&](int x, int y) { return BOff{base_p + spy * (uint32_t)y, ST * (uint32_t)x}; };
  auto vbc = [&](int x, int y) { return ((x == 0) & bxl) | ((x == K) & bxh) | ((y == 0) & byl) | ((y == K) & byh); };
  const bool has_c = g.cp != T(0);

  // 1. requests: both velocity components and the pressure data of stage 0
  //    on the whole cell, D_A^-1 of this component, the base vector
  T uu[2][1][NV][NV], pa[NP][NP], ds[NP][NP], pc[1][NP][NP], dv[NV][NV], bs[K][K], pold[K - 1][K - 1];
#pragma unroll
  for (int cc = 0; cc < 2; ++cc)
#pragma unroll
    for (int y = 0; y < NV; ++y)
#pragma unroll
      for (int x = 0; x < NV; ++x) uu[cc][0][y][x] = at(P.u, uc_at(cc, x, y));
#pragma unroll
  for (int y = 0; y < NP; ++y)
#pragma unroll
    for (int x = 0; x < NP; ++x) {
      ds[y][x] = at(P.dinv_s, p_at(x, y));
      if constexpr (MODE == F3_DIVRES) pa[y][x] = P.g ? at(P.g, p_at(x, y)) : T(0);
      else pa[y][x] = at(P.rin, p_at(x, y));
      pc[0][y][x] = (MODE == F3_DIVRES && has_c) ? at(P.p0, p_at(x, y)) : T(0);
    }
#pragma unroll
  for (int y = 0; y < NV; ++y)
#pragma unroll
    for (int x = 0; x < NV; ++x) dv[y][x] = at(op2.dinv, u_at(x, y));
  const T mu = g.mu_cell != nullptr ? g.mu_cell[(uint32_t)ax + (uint32_t)g.n[0] * (uint32_t)ay] : g.mu;
  if (owner) {
#pragma unroll
    for (int y = 0; y < K; ++y)
#pragma unroll
      for (int x = 0; x < K; ++x) bs[y][x] = (LAST && op2.base) ? at(op2.base, u_at(x, y)) : T(0);
    if constexpr (MODE == F3_CHEBS) {
#pragma unroll
      for (int y = 0; y < K - 1; ++y)
#pragma unroll
        for (int x = 0; x < K - 1; ++x) pold[y][x] = (c == 0 && P.p) ? at(P.p, p_at(x, y)) : T(0);
    }
  }
  __asm__ volatile("" ::: "memory");

  // 2. stage 0: t0 = B u + sc M_p pc on the pressure nodes
#pragma unroll
  for (int cc = 0; cc < 2; ++cc)
#pragma unroll
    for (int y = 0; y < NV; ++y)
#pragma unroll
      for (int x = 0; x < NV; ++x) uu[cc][0][y][x] = (active && !vbc(x, y)) ? uu[cc][0][y][x] : T(0);
  T d0[NP][NP];
#pragma unroll
  for (int y = 0; y < NP; ++y)
#pragma unroll
    for (int x = 0; x < NP; ++x) {
      d0[y][x] = ds[y][x] * pa[y][x] * P.inv_theta;   // F3_CHEBS: d_0
      if constexpr (MODE == F3_CHEBS) pc[0][y][x] = d0[y][x];
      pc[0][y][x] = active ? pc[0][y][x] : T(0);
    }
  T t0[1][NP][NP];
  {
    T w[1][NV][NP];
    pass_x<false, false>(R.Gr, uu[0], w, T(1));
    pass_y<false, false>(R.Nr, w, t0, -g.sB[0]);
    pass_x<false, false>(R.Nr, uu[1], w, T(1));
    pass_y<false, true>(R.Gr, w, t0, -g.sB[1]);
  }
  if (has_c) {
    const T sc = (MODE == F3_CHEBS ? g.cp : -g.cp) * g.sM;
    T q[1][NP][NP];
    pass_x<false, false>(R.Mpr, pc, q, T(1));
    pass_y<false, true>(R.Mpr, q, t0, sc);
  }
  hand_over_xy<TX>(t0, lcx, lcy, bxh, byh);
  // z on the nodes this lane holds completely; the pressure output
  T z[NP][NP];
#pragma unroll
  for (int y = 0; y < NP; ++y)
#pragma unroll
    for (int x = 0; x < NP; ++x) {
      if constexpr (MODE == F3_DIVRES) {
        z[y][x] = t0[0][y][x] - pa[y][x];   // r_p
      } else {
        const T rn = pa[y][x] - t0[0][y][x];
        const T dn = P.c1 * d0[y][x] + P.c2 * ds[y][x] * rn;
        z[y][x] = P.tau * ((T(0) + d0[y][x]) + dn);
      }
    }
  if (owner && c == 0) {
#pragma unroll
    for (int y = 0; y < NP; ++y)
#pragma unroll
      for (int x = 0; x < NP; ++x) {
        const bool main = x < K - 1 && y < K - 1;
        if (!main && !(((x < K - 1) | bxh) & ((y < K - 1) | byh))) continue;
        if constexpr (MODE == F3_DIVRES) {
          at(P.rp, p_at(x, y)) = z[y][x];
        } else if (P.p) {
          const T po = main ? pold[main ? y : 0][main ? x : 0] : at(P.p, p_at(x, y));
          at(P.p, p_at(x, y)) = po + z[y][x];
        }
      }
  }
  if constexpr (MODE == F3_DIVRES) {
#pragma unroll
    for (int y = 0; y < NP; ++y)
#pragma unroll
      for (int x = 0; x < NP; ++x) z[y][x] = ds[y][x] * z[y][x] * P.inv_theta;
  }
  gather_high_faces<TX>(z, bxh, byh);

  // 3. stage 1: q_c = B_c^T z (inputs of the lanes holding the whole cell)
  T zm[1][NP][NP], t1[1][NV][NV];
#pragma unroll
  for (int y = 0; y < NP; ++y)
#pragma unroll
    for (int x = 0; x < NP; ++x) zm[0][y][x] = valid1 ? z[y][x] : T(0);
  if (c == 0) {
    T s1[1][NV][NP];
    pass_y<true, false>(R.Nr, zm, s1, T(1));
    pass_x<true, false>(R.Gr, s1, t1, -g.sB[0]);
  } else {
    T s2[1][NP][NV];
    pass_x<true, false>(R.Nr, zm, s2, T(1));
    pass_y<true, false>(R.Gr, s2, t1, -g.sB[1]);
  }
  hand_over_xy<TX>(t1, lcx, lcy, bxh, byh);
  T v[NV][NV];
#pragma unroll
  for (int y = 0; y < NV; ++y)
#pragma unroll
    for (int x = 0; x < NV; ++x) v[y][x] = vbc(x, y) ? T(0) : t1[0][y][x];   // Dirichlet rows of q are 0
  gather_high_faces<TX>(v, bxh, byh);

  // 4. stage 2: t2 = A d0, d0 = D_A^-1 q / theta_A
  const T axk = mu * g.sKx, bxm = g.gr * g.sM, sy = mu * g.sKy;
  T X[NV][NV];
#pragma unroll
  for (int i = 0; i < NV; ++i)
#pragma unroll
    for (int j = 0; j < NV; ++j) X[i][j] = axk * R.Kr[i][j] + bxm * R.Mr[i][j];
  T da[1][NV][NV], t2[1][NV][NV];
#pragma unroll
  for (int y = 0; y < NV; ++y)
#pragma unroll
    for (int x = 0; x < NV; ++x) {
      const T d = dv[y][x] * v[y][x] * op2.inv_theta;
      da[0][y][x] = (valid2 && !vbc(x, y)) ? d : T(0);
    }
  {
    T t[1][NV][NV];
    pass_y<false, false>(R.Mr, da, t, T(1));
    pass_x<false, false>(X, t, t2, T(1));
    pass_y<false, false>(R.Kr, da, t, T(1));
    pass_x<false, true>(R.Mr, t, t2, sy);
  }
  hand_over_xy<TX>(t2, lcx, lcy, bxh, byh);

  // 5. owned nodes through the Chebyshev epilogue
  if (!owner) return;
  using Pre2 = typename OpChebA<T, true, LAST>::Pre;
  auto pre_at = [&](int x, int y, T base) {
    Pre2 q;
    q.r = v[y][x];
    q.x = T(0);
    q.dinv = dv[y][x];
    q.base = base;
    return q;
  };
#pragma unroll
  for (int y = 0; y < K; ++y)
#pragma unroll
    for (int x = 0; x < K; ++x) op2.store_u(u_at(x, y), t2[0][y][x], da[0][y][x], false, pre_at(x, y, bs[y][x]));
  if (bxl | byl) {
#pragma unroll
    for (int y = 0; y < K; ++y)
#pragma unroll
      for (int x = 0; x < K; ++x) {
        if (!vbc(x, y)) continue;
        const T rw = dv[y][x] * v[y][x] * op2.inv_theta;
        op2.store_u(u_at(x, y), rw, rw, true, pre_at(x, y, bs[y][x]));
      }
  }
  if (bxh | byh) {
#pragma unroll
    for (int y = 0; y < NV; ++y)
#pragma unroll
      for (int x = 0; x < NV; ++x) {
        if (x < K && y < K) continue;
        if ((x == K && !bxh) || (y == K && !byh)) continue;
        const BOff gi = u_at(x, y);
        const T rw = dv[y][x] * v[y][x] * op2.inv_theta;
        op2.store_u(gi, rw, rw, true, pre_at(x, y, (LAST && op2.base) ? at(op2.base, gi) : T(0)));
      }
  }
}

template <int K, typename T, class Op1, bool LAST>
__global__ void __launch_bounds__(64)
wave2d_fused_kernel(const Geo2<T> g, const Op1 op1, const OpChebA<T, true, LAST> op2) {
  wave2d_fused_body<K, T, Op1, LAST>(g, op1, op2, xcd_contiguous_tile(blockIdx.x, gridDim.x));
}

// The same two stages on a workgroup of WX x WY waves: one tile of 8 WX x
// 8 WY cells per (workgroup, velocity component) owns (8 WX - 3) x (8 WY - 3)
// cells; faces between the waves go through LDS instead of halo cells.
template <int K, typename T, class Op1, bool LAST, int WX, int WY>
__global__ void __launch_bounds__(64 * WX * WY)
wg2d_fused_kernel(const Geo2<T> g, const Op1 op1, const OpChebA<T, true, LAST> op2) {
  __shared__ WgFaces<WX, WY, K + 1, T> sh;
  wave2d_fused_body<K, T, Op1, LAST, WX, WY>(g, op1, op2, xcd_contiguous_tile(blockIdx.x, gridDim.x), &sh);
}

template <int K, typename T, int MODE, bool LAST>
__global__ void __launch_bounds__(64)
wave2d_fused3_kernel(const Geo2<T> g, const Fuse3P<T> P, const OpChebA<T, true, LAST> op2) {
  wave2d_fused3_body<K, T, MODE, LAST>(g, P, op2, xcd_contiguous_tile(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// The 2D launches above as functors (packed launches over many problems,
// packed.hpp); block b of nb takes tile xcd_contiguous_tile(b, nb) as in a
// launch of its own.
// ---------------------------------------------------------------------------
template <int K, typename T, int BLK, class Op>
struct LTile2 {
  static constexpr int THREADS = 64;
  Geo2<T> g;
  Op op;
  __device__ void run(int b, int nb) const { wave2d_tile<K, T, BLK, Op, -1>(g, op, xcd_contiguous_tile(b, nb)); }
};

template <int K, typename T, int BLK, class Op>
struct LTile2Split {
  static constexpr int THREADS = 64;
  Geo2<T> g;
  Op op;
  __device__ void run(int b, int nb) const {
    constexpr bool OUT_U = (BLK & (BLK_A | BLK_MASS | BLK_BT)) != 0;
    constexpr bool OUT_P = (BLK & (BLK_B | BLK_C)) != 0;
    constexpr int NF = (OUT_U ? 2 : 0) + (OUT_P ? 1 : 0);
    const int bb = xcd_contiguous_tile(b, nb);
    const int f = bb % NF, t = bb / NF;
    if constexpr (OUT_U) {
      if (f == 0) { wave2d_tile<K, T, BLK, Op, 0>(g, op, t); return; }
      if (f == 1) { wave2d_tile<K, T, BLK, Op, 1>(g, op, t); return; }
    }
    if constexpr (OUT_P) wave2d_tile<K, T, BLK, Op, 2>(g, op, t);
  }
};

template <int K, typename T, class Op1, bool LAST>
struct LFused2 {
  static constexpr int THREADS = 64;
  Geo2<T> g;
  Op1 op1;
  OpChebA<T, true, LAST> op2;
  __device__ void run(int b, int nb) const { wave2d_fused_body<K, T, Op1, LAST>(g, op1, op2, xcd_contiguous_tile(b, nb)); }
};

template <int K, typename T, class Op1, bool LAST, int WX, int WY>
struct LFused2Wg {
  static constexpr int THREADS = 64 * WX * WY;
  Geo2<T> g;
  Op1 op1;
  OpChebA<T, true, LAST> op2;
  __device__ void run(int b, int nb) const {
    __shared__ WgFaces<WX, WY, K + 1, T> sh;
    wave2d_fused_body<K, T, Op1, LAST, WX, WY>(g, op1, op2, xcd_contiguous_tile(b, nb), &sh);
  }
};

template <int K, typename T, int MODE, bool LAST>
struct LFused3 {
  static constexpr int THREADS = 64;
  Geo2<T> g;
  Fuse3P<T> P;
  OpChebA<T, true, LAST> op2;
  __device__ void run(int b, int nb) const { wave2d_fused3_body<K, T, MODE, LAST>(g, P, op2, xcd_contiguous_tile(b, nb)); }
};

}  // namespace smg
