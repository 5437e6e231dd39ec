// Set-up kernels on axis-aligned box cells (FP64): the diagonal D_A of the
// velocity block and the Schur-complement diagonal approximations of
// Sec. 3.3.1, each from the 1D cell matrices (the cell matrices of a and b
// are Kronecker products of them, so every entry is a product of 1D entries).
#pragma once
#include "common.hpp"

namespace smg {

// Cells containing lattice node i of a degree-`deg` field along one axis:
// up to two (cell, local index) pairs.
__device__ __forceinline__ int node_cells(int i, int deg, int ncell, int *cell, int *loc) {
  int m = 0;
  const int c = i / deg, r = i - c * deg;
  if (r == 0) {
    if (c - 1 >= 0) { cell[m] = c - 1; loc[m] = deg; ++m; }
    if (c < ncell) { cell[m] = c; loc[m] = 0; ++m; }
  } else {
    cell[m] = c; loc[m] = r; ++m;
  }
  return m;
}

template <int DIM>
__device__ __forceinline__ void unflat(i64 idx, const int *dims, int *out) {
  for (int a = 0; a < DIM; ++a) { out[a] = (int)(idx % dims[a]); idx /= dims[a]; }
}

template <int DIM, int K>
__device__ __forceinline__ double cell_mu(const LevelGeom<double, DIM, K> &g, const int *cell) {
  if (!g.mu_cell) return g.mu;
  i64 ci = cell[0] + (i64)g.n[0] * (cell[1] + (DIM == 3 ? (i64)g.n[1] * cell[2] : 0));
  return g.mu_cell[ci];
}

// (A_tau)_jj for local velocity node j (per direction loc[a]).
template <int DIM, int K>
__device__ __forceinline__ double cell_A_diag(const LevelGeom<double, DIM, K> &g, double mu, const int *loc) {
  double stiff = 0.0, mass = 1.0;
  for (int a = 0; a < DIM; ++a) {
    double t = g.c[a].Kv[loc[a]][loc[a]];
    for (int b = 0; b < DIM; ++b)
      if (b != a) t *= g.c[b].Mv[loc[b]][loc[b]];
    stiff += t;
    mass *= g.c[a].Mv[loc[a]][loc[a]];
  }
  return mu * stiff + g.gr * mass;
}

// D_A = diag(A) per velocity node, 1 on Dirichlet rows, replicated over components.
template <int DIM, int K>
__global__ void k_diag_A(const LevelGeom<double, DIM, K> g, double *D) {
  SMG_GRID_LOOP(node, g.Nv) {
    int l[3] = {0, 0, 0};
    unflat<DIM>(node, g.vd, l);
    bool bc = false;
    for (int a = 0; a < DIM; ++a) bc |= on_box_boundary(l[a], g.vd[a]);
    double s = 0.0;
    if (bc) {
      s = 1.0;
    } else {
      int cs[3][2], ls[3][2], m[3] = {1, 1, 1};
      for (int a = 0; a < DIM; ++a) m[a] = node_cells(l[a], K, g.n[a], cs[a], ls[a]);
      for (int iz = 0; iz < (DIM == 3 ? m[2] : 1); ++iz)
        for (int iy = 0; iy < m[1]; ++iy)
          for (int ix = 0; ix < m[0]; ++ix) {
            int cell[3] = {cs[0][ix], cs[1][iy], DIM == 3 ? cs[2][iz] : 0};
            int loc[3] = {ls[0][ix], ls[1][iy], DIM == 3 ? ls[2][iz] : 0};
            s += cell_A_diag<DIM, K>(g, cell_mu<DIM, K>(g, cell), loc);
          }
    }
    for (int c = 0; c < DIM; ++c) D[c * g.Nv + node] = s;
  }
}

// D~_S per pressure node; kind 0: diag(B diag(A)^-1 B^T) with the assembled B
// entries, 1: sum over cells of diag(B_tau diag(A_tau)^-1 B_tau^T), 2: diag(M_p).
// Constrained velocity columns are excluded; cp diag(M_p) is added (C = cp M_p).
template <int DIM, int K>
__global__ void k_diag_S(const LevelGeom<double, DIM, K> g, int kind, const double *DA, double *DS) {
  constexpr int KP = K - 1;
  SMG_GRID_LOOP(node, g.Np) {
    int l[3] = {0, 0, 0};
    unflat<DIM>(node, g.pd, l);
    int cs[3][2], ls[3][2], m[3] = {1, 1, 1};
    for (int a = 0; a < DIM; ++a) m[a] = node_cells(l[a], KP, g.n[a], cs[a], ls[a]);
    // diag(M_p)
    double mp = 0.0;
    for (int iz = 0; iz < (DIM == 3 ? m[2] : 1); ++iz)
      for (int iy = 0; iy < m[1]; ++iy)
        for (int ix = 0; ix < m[0]; ++ix) {
          const int sel[3] = {ix, iy, iz};
          double t = 1.0;
          for (int a = 0; a < DIM; ++a) t *= g.c[a].Mp[ls[a][sel[a]]][ls[a][sel[a]]];
          mp += t;
        }
    double s = 0.0;
    if (kind == 2) {
      s = mp;
    } else if (kind == 0) {
      // velocity nodes coupled to this pressure node: union of the cells' lattices
      int jlo[3] = {0, 0, 0}, jhi[3] = {0, 0, 0};
      for (int a = 0; a < DIM; ++a) { jlo[a] = K * cs[a][0]; jhi[a] = K * (cs[a][m[a] - 1] + 1); }
      for (int c = 0; c < DIM; ++c)
        for (int jz = jlo[2]; jz <= (DIM == 3 ? jhi[2] : 0); ++jz)
          for (int jy = jlo[1]; jy <= jhi[1]; ++jy)
            for (int jx = jlo[0]; jx <= jhi[0]; ++jx) {
              const int j[3] = {jx, jy, jz};
              bool bc = false;
              for (int a = 0; a < DIM; ++a) bc |= on_box_boundary(j[a], g.vd[a]);
              if (bc) continue;
              // B_ij = - prod_a sum_{cells of a containing both} (a == c ? G : N)[i_loc][j_loc]
              double b = -1.0;
              for (int a = 0; a < DIM; ++a) {
                double f = 0.0;
                for (int t = 0; t < m[a]; ++t) {
                  const int jl = j[a] - K * cs[a][t];
                  if (jl < 0 || jl > K) continue;
                  f += (a == c) ? g.c[a].G[ls[a][t]][jl] : g.c[a].N[ls[a][t]][jl];
                }
                b *= f;
              }
              const i64 jn = jx + (i64)g.vd[0] * (jy + (i64)g.vd[1] * jz);
              s += b * b / DA[c * g.Nv + jn];
            }
    } else {
      for (int iz = 0; iz < (DIM == 3 ? m[2] : 1); ++iz)
        for (int iy = 0; iy < m[1]; ++iy)
          for (int ix = 0; ix < m[0]; ++ix) {
            const int sel[3] = {ix, iy, iz};
            int cell[3] = {0, 0, 0}, il[3] = {0, 0, 0};
            for (int a = 0; a < DIM; ++a) { cell[a] = cs[a][sel[a]]; il[a] = ls[a][sel[a]]; }
            const double mu = cell_mu<DIM, K>(g, cell);
            for (int c = 0; c < DIM; ++c)
              for (int jz = 0; jz <= (DIM == 3 ? K : 0); ++jz)
                for (int jy = 0; jy <= K; ++jy)
                  for (int jx = 0; jx <= K; ++jx) {
                    const int jl[3] = {jx, jy, jz};
                    bool bc = false;
                    for (int a = 0; a < DIM; ++a) bc |= on_box_boundary(K * cell[a] + jl[a], g.vd[a]);
                    if (bc) continue;
                    double b = -1.0;
                    for (int a = 0; a < DIM; ++a) b *= (a == c) ? g.c[a].G[il[a]][jl[a]] : g.c[a].N[il[a]][jl[a]];
                    s += b * b / cell_A_diag<DIM, K>(g, mu, jl);
                  }
          }
    }
    DS[node] = s + g.cp * mp;
  }
}

// ---------------------------------------------------------------------------
// Probing (general cells): indicator of one residue class of lattice nodes
// and extraction of the probed diagonal entries.
// ---------------------------------------------------------------------------
template <int DIM>
__device__ __forceinline__ bool in_class(i64 node, int d0, int d1, int m, int c0, int c1, int c2) {
  const int x = (int)(node % d0);
  const i64 r = node / d0;
  const int y = (int)(r % d1);
  const int z = (int)(r / d1);
  return x % m == c0 && y % m == c1 && (DIM == 2 || z % m == c2);
}

// e = 1 on the nodes of `field` (0: every velocity component, 1: pressure,
// 2 + c: velocity component c only) whose lattice coordinates are congruent
// to (c0, c1, c2) modulo m, else 0.
template <int DIM>
__global__ void k_probe_fill(double *e, i64 Nv, i64 Np, int field, int m, int c0, int c1, int c2, int v0, int v1,
                             int p0, int p1) {
  const i64 nu = (i64)DIM * Nv;
  SMG_GRID_LOOP(i, nu + Np) {
    bool on = false;
    if (i < nu) {
      if (field == 0 || (field >= 2 && i / Nv == field - 2)) on = in_class<DIM>(i % Nv, v0, v1, m, c0, c1, c2);
    } else if (field == 1) {
      on = in_class<DIM>(i - nu, p0, p1, m, c0, c1, c2);
    }
    e[i] = on ? 1.0 : 0.0;
  }
}

// D[i] = y[i] (+ zs z[i]) for the nodes i of the residue class; n nodes per
// component, ncomp components.
template <int DIM>
__global__ void k_probe_take(double *D, const double *y, const double *z, double zs, i64 n, int ncomp, int m, int c0,
                             int c1, int c2, int d0, int d1) {
  SMG_GRID_LOOP(i, n * ncomp) {
    if (!in_class<DIM>(i % n, d0, d1, m, c0, c1, c2)) continue;
    D[i] = y[i] + (z ? zs * z[i] : 0.0);
  }
}

// Velocity values on the Dirichlet nodes (every node on the boundary of the
// box lattice): mode 0 writes out = u_d there and 0 elsewhere, mode 1 writes
// out = u_d there and leaves the other entries.
template <typename T, int DIM>
__global__ void k_dirichlet_values(const T *ud, T *out, i64 Nv, int v0, int v1, int v2, int mode) {
  SMG_GRID_LOOP(i, (i64)DIM * Nv) {
    const i64 node = i % Nv;
    const int x = (int)(node % v0);
    const i64 r = node / v0;
    const int y = (int)(r % v1);
    const int z = (int)(r / v1);
    const bool bc = x == 0 || x == v0 - 1 || y == 0 || y == v1 - 1 || (DIM == 3 && (z == 0 || z == v2 - 1));
    if (bc) out[i] = ud[i];
    else if (mode == 0) out[i] = T(0);
  }
}

template <typename T>
__global__ void k_div_by(T *q, const double *d, i64 n) {
  SMG_GRID_LOOP(i, n) q[i] = (T)((double)q[i] / d[i]);
}

}  // namespace smg
