// Operator application on general (multilinear) cells: meshes given by their
// vertices (Sec. 2: each cell is the image of the unit cell under the
// bi-/trilinear map of its 2^d vertices; Sec. 3.1: K x = sum_tau P_tau K_tau
// P_tau^T x with the cell integrals evaluated by Gauss quadrature, k+1 points
// per direction, and sum factorisation).
//
// At each quadrature point: J = sum_v x_v (x) grad N_v, JxW = det J w_q, the
// physical gradients grad u_c = J^-T grad^ u_c, and the integrands of
//   a(u, v) = int mu grad u_c . grad v_c + gamma rho u_c v_c
//             (or int mu eps(u) : eps(v) + gamma rho u.v, Sec. 2),
//   b(v, q) = -int q div v,   (C p, q) = c_p int p q.
//
// Work decomposition: one wave64 per 64 / (k+1)^d cells, one lane per node /
// quadrature point (for these tensor-product spaces both are (k+1)^d).  The
// 1D passes run through LDS (one pass = each lane contracts k+1 neighbours of
// its line).  Cells are processed in 2^d colours (cells of equal index parity
// share no node), one launch per colour adding into an accumulation vector;
// a separate epilogue pass over all nodes then applies the Dirichlet rows and
// the caller's fused vector algebra (the same functors as the box kernels).
#pragma once
#include <type_traits>

#include "cell_kernel.hpp"
#include "fe1d_const.hpp"

namespace smg {

template <typename T>
struct GenGeo {
  int n[3], vd[3], pd[3];
  i64 Nv, Np;
  int ncol[3];      // cells of the launch colour per direction
  int off[3];       // colour: parity of the cell index per direction
  T mu, gr, cp;
  const T *mu_cell;
  const T *verts;   // (n+1)^d vertices x d coordinates, x fastest
  T *tu, *tp;       // accumulated cell sums (velocity [u_1|..|u_d], pressure)
  int sym;          // viscous term mu eps(u):eps(v) instead of mu grad u : grad v
  int step;         // 2: one colour (cells off + 2 i), 1: every cell
  T *cbu, *cbp;     // every-cell mode: per-cell results [cell][comp][node], [cell][pressure node]
};

// a[i] for a lane-dependent i without dynamic indexing into private memory
template <int N, typename T>
__device__ __forceinline__ T pick(const T (&a)[N], int i) {
  T r = a[0];
#pragma unroll
  for (int j = 1; j < N; ++j) r = (i == j) ? a[j] : r;
  return r;
}

template <int DIM, int K, typename T, int BLK, class Op>
__global__ void __launch_bounds__(64) gen_apply_kernel(const GenGeo<T> g, const Op op) {
  constexpr int NV = K + 1, NP = K;
  constexpr int NN = DIM == 3 ? NV * NV * NV : NV * NV;   // nodes = quadrature points
  constexpr int NPN = DIM == 3 ? NP * NP * NP : NP * NP;  // pressure nodes
  constexpr int CPB = 64 / NN;                             // cells per wave
  constexpr int NVERT = 1 << DIM;
  constexpr cfe::QTab<K, T> Q = cfe::make_qtab<K, T>();
  constexpr bool NEED_U = (BLK & (BLK_A | BLK_MASS | BLK_B)) != 0;
  constexpr bool NEED_P = (BLK & (BLK_BT | BLK_C)) != 0;
  constexpr bool OUT_U = (BLK & (BLK_A | BLK_MASS | BLK_BT)) != 0;
  constexpr bool OUT_P = (BLK & (BLK_B | BLK_C)) != 0;
  __shared__ T lds[CPB][3][NN];

  const int tid = threadIdx.x;
  const int slot = tid / NN;
  const int q = tid - slot * NN;
  const bool in_slot = slot < CPB;
  const int sl = in_slot ? slot : 0;
  const i64 ci = (i64)blockIdx.x * CPB + slot;
  const i64 ncells = (i64)g.ncol[0] * g.ncol[1] * (DIM == 3 ? g.ncol[2] : 1);
  const bool live = in_slot && ci < ncells;
  int cx = 0, cy = 0, cz = 0;
  if (live) {
    const i64 r = ci / g.ncol[0];
    cx = g.step * (int)(ci - r * g.ncol[0]) + g.off[0];
    cy = g.step * (int)(r % g.ncol[1]) + g.off[1];
    cz = DIM == 3 ? g.step * (int)(r / g.ncol[1]) + g.off[2] : 0;
  }
  const i64 cell = cx + (i64)g.n[0] * (cy + (i64)g.n[1] * cz);
  const int qx = q % NV, qy = (q / NV) % NV, qz = DIM == 3 ? q / (NV * NV) : 0;
  const int qd[3] = {qx, qy, qz};
  T *A = lds[sl][0], *Bf = lds[sl][1], *Cf = lds[sl][2];

  // per-lane rows / columns of the 1D quadrature tables
  T rV[3][NV], rD[3][NV], cV[3][NV], cD[3][NV];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      T vr = Q.V[0][i], dr = Q.D[0][i], vc = Q.V[i][0], dc = Q.D[i][0];
#pragma unroll
      for (int j = 1; j < NV; ++j) {
        vr = qd[d] == j ? Q.V[j][i] : vr;
        dr = qd[d] == j ? Q.D[j][i] : dr;
        vc = qd[d] == j ? Q.V[i][j] : vc;
        dc = qd[d] == j ? Q.D[i][j] : dc;
      }
      rV[d][i] = vr;
      rD[d][i] = dr;
      cV[d][i] = vc;
      cD[d][i] = dc;
    }
  auto lidx = [](int x, int y, int z) { return x + NV * (y + NV * z); };
  // one pass along direction d with per-lane coefficients m[i]: out(q) = sum_i m[i] in(q with coordinate d = i)
  auto pass = [&](const T *in, const T (&m)[NV], int d) {
    T s = 0;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int k = d == 0 ? lidx(i, qy, qz) : (d == 1 ? lidx(qx, i, qz) : lidx(qx, qy, i));
      s += m[i] * in[k];
    }
    return s;
  };

  // ---- geometry at this lane's quadrature point
  T Jinv[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  T JxW = 0;
  T mu = g.mu;
  if (live) {
    const T xi[3] = {pick(Q.x, qx), pick(Q.x, qy), DIM == 3 ? pick(Q.x, qz) : T(0)};
    T J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int v = 0; v < NVERT; ++v) {
      const int o[3] = {v & 1, (v >> 1) & 1, (v >> 2) & 1};
      const i64 vid = (cx + o[0]) + (i64)(g.n[0] + 1) * ((cy + o[1]) + (i64)(g.n[1] + 1) * (DIM == 3 ? cz + o[2] : 0));
#pragma unroll
      for (int b = 0; b < DIM; ++b) {
        T dn = o[b] ? T(1) : T(-1);
#pragma unroll
        for (int c = 0; c < DIM; ++c)
          if (c != b) dn *= o[c] ? xi[c] : T(1) - xi[c];
#pragma unroll
        for (int a = 0; a < DIM; ++a) J[a][b] += g.verts[vid * DIM + a] * dn;
      }
    }
    T det;
    if constexpr (DIM == 2) {
      det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
      const T id = T(1) / det;
      Jinv[0][0] = J[1][1] * id;
      Jinv[0][1] = -J[0][1] * id;
      Jinv[1][0] = -J[1][0] * id;
      Jinv[1][1] = J[0][0] * id;
      JxW = det * pick(Q.w, qx) * pick(Q.w, qy);
    } else {
      const T c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
      const T c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
      const T c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
      det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
      const T id = T(1) / det;
      Jinv[0][0] = c00 * id;
      Jinv[1][0] = c01 * id;
      Jinv[2][0] = c02 * id;
      Jinv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
      Jinv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
      Jinv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
      Jinv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
      Jinv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
      Jinv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
      JxW = det * pick(Q.w, qx) * pick(Q.w, qy) * pick(Q.w, qz);
    }
    if (g.mu_cell != nullptr) mu = g.mu_cell[cx + (i64)g.n[0] * (cy + (i64)g.n[1] * cz)];
  }

  // ---- this lane's global velocity node
  const int gx = K * cx + qx, gy = K * cy + qy, gz = K * cz + qz;
  const i64 vnode = gx + (i64)g.vd[0] * (gy + (i64)g.vd[1] * gz);
  const bool vbc = on_box_boundary(gx, g.vd[0]) || on_box_boundary(gy, g.vd[1]) ||
                   (DIM == 3 && on_box_boundary(gz, g.vd[2]));

  // ---- velocity: values and reference gradients at the quadrature points
  T uq[DIM], gref[DIM][3];
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    uq[c] = 0;
    gref[c][0] = gref[c][1] = gref[c][2] = 0;
  }
  if constexpr (NEED_U) {
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      T v = 0;
      if (live && !(Op::ZERO_BC && vbc)) v = op.load_u((i64)c * g.Nv + vnode);
      if (in_slot) A[q] = v;
      __syncthreads();
      T t = pass(A, rV[0], 0);
      if (in_slot) Bf[q] = t;
      __syncthreads();
      t = pass(Bf, rV[1], 1);
      if constexpr (DIM == 3) {
        if (in_slot) A[q] = t;
        __syncthreads();
        t = pass(A, rV[2], 2);
      }
      // values at the quadrature points now in a buffer the gradient passes read
      T *Fq = DIM == 3 ? Bf : A;
      __syncthreads();
      if (in_slot) Fq[q] = t;
      __syncthreads();
      uq[c] = t;
#pragma unroll
      for (int d = 0; d < DIM; ++d) gref[c][d] = pass(Fq, rD[d], d);
      __syncthreads();
    }
  }

  // ---- pressure at the quadrature points (shapes K^d -> (K+1) K^(d-1) -> ...)
  T pq = 0;
  if constexpr (NEED_P) {
    T v = 0;
    if (live && q < NPN) {
      const int px = q % NP, py = (q / NP) % NP, pz = DIM == 3 ? q / (NP * NP) : 0;
      const i64 pn = ((K - 1) * cx + px) + (i64)g.pd[0] * (((K - 1) * cy + py) + (i64)g.pd[1] * ((K - 1) * cz + pz));
      v = op.load_p(pn);
    }
    if (in_slot) A[q] = v;
    __syncthreads();
    // x: (NP, NP, NP) -> (NV, NP, NP)
    {
      const int o = q, ox = o % NV, oy = (o / NV) % NP, oz = o / (NV * NP);
      T s = 0;
      if (o < NV * NP * (DIM == 3 ? NP : 1)) {
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          T m = Q.Vp[0][i];
#pragma unroll
          for (int j = 1; j < NV; ++j) m = ox == j ? Q.Vp[j][i] : m;
          s += m * A[i + NP * (oy + NP * oz)];
        }
      }
      __syncthreads();
      if (in_slot) Bf[q] = s;
      __syncthreads();
    }
    // y: (NV, NP, NP) -> (NV, NV, NP)
    T s = 0;
    {
      const int o = q, ox = o % NV, oy = (o / NV) % NV, oz = o / (NV * NV);
      if (o < NV * NV * (DIM == 3 ? NP : 1)) {
#pragma unroll
        for (int i = 0; i < NP; ++i) {
          T m = Q.Vp[0][i];
#pragma unroll
          for (int j = 1; j < NV; ++j) m = oy == j ? Q.Vp[j][i] : m;
          s += m * Bf[ox + NV * (i + NP * oz)];
        }
      }
    }
    if constexpr (DIM == 3) {
      __syncthreads();
      if (in_slot) A[q] = s;
      __syncthreads();
      // z: (NV, NV, NP) -> (NV, NV, NV)
      T s3 = 0;
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        T m = Q.Vp[0][i];
#pragma unroll
        for (int j = 1; j < NV; ++j) m = qz == j ? Q.Vp[j][i] : m;
        s3 += m * A[qx + NV * (qy + NV * i)];
      }
      s = s3;
    }
    pq = s;
    __syncthreads();
  }

  // ---- integrands at the quadrature point
  T vcoef[DIM], gcoef[DIM][3];
  T pcoef = 0;
  {
    T gphys[DIM][3];
#pragma unroll
    for (int c = 0; c < DIM; ++c)
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        T s = 0;
#pragma unroll
        for (int b = 0; b < DIM; ++b) s += Jinv[b][a] * gref[c][b];
        gphys[c][a] = s;
      }
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      T val = 0;
      if constexpr ((BLK & BLK_A) != 0) val += g.gr * uq[c];
      if constexpr ((BLK & BLK_MASS) != 0) val += uq[c];
      vcoef[c] = val * JxW;
      T G[3] = {0, 0, 0};
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        // test function of component c: mu grad u_c, or mu eps(u)_{c.} (eps:eps = eps:grad)
        if constexpr ((BLK & BLK_A) != 0)
          G[a] += mu * (g.sym ? T(0.5) * (gphys[c][a] + gphys[a][c]) : gphys[c][a]);
        if constexpr ((BLK & BLK_BT) != 0)
          if (a == c) G[a] -= pq;
      }
#pragma unroll
      for (int b = 0; b < DIM; ++b) {
        T s = 0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) s += Jinv[b][a] * G[a];
        gcoef[c][b] = s * JxW;
      }
    }
    if constexpr ((BLK & BLK_B) != 0) {
      T div = 0;
#pragma unroll
      for (int c = 0; c < DIM; ++c) div += gphys[c][c];
      pcoef -= div;
    }
    if constexpr ((BLK & BLK_C) != 0) pcoef += ((BLK & BLK_CPLUS) ? g.cp : -g.cp) * pq;
    pcoef *= JxW;
  }

  // ---- velocity test functions: integrate back, add into the accumulation vector
  if constexpr (OUT_U) {
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
      if (in_slot) {
        A[q] = gcoef[c][0];
        Bf[q] = gcoef[c][1];
        if constexpr (DIM == 3) Cf[q] = gcoef[c][2];
      }
      __syncthreads();
      T w = vcoef[c] + pass(A, cD[0], 0) + pass(Bf, cD[1], 1);
      if constexpr (DIM == 3) w += pass(Cf, cD[2], 2);
      __syncthreads();
      if (in_slot) A[q] = w;
      __syncthreads();
      T t = pass(A, cV[0], 0);
      if (in_slot) Bf[q] = t;
      __syncthreads();
      t = pass(Bf, cV[1], 1);
      if constexpr (DIM == 3) {
        if (in_slot) A[q] = t;
        __syncthreads();
        t = pass(A, cV[2], 2);
      }
      __syncthreads();
      if (live) {
        if (g.cbu != nullptr) g.cbu[(cell * DIM + c) * NN + q] = t;
        else g.tu[(i64)c * g.Nv + vnode] += t;
      }
    }
  }

  // ---- pressure test functions
  if constexpr (OUT_P) {
    if (in_slot) A[q] = pcoef;
    __syncthreads();
    T s = 0;
    if constexpr (DIM == 3) {
      // z: (NV, NV, NV) -> (NV, NV, NP)
      const int o = q, ox = o % NV, oy = (o / NV) % NV, oz = o / (NV * NV);
      if (o < NV * NV * NP) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
          T m = Q.Vp[i][0];
#pragma unroll
          for (int j = 1; j < NP; ++j) m = oz == j ? Q.Vp[i][j] : m;
          s += m * A[ox + NV * (oy + NV * i)];
        }
      }
      __syncthreads();
      if (in_slot) A[q] = s;
      __syncthreads();
    }
    // y: (NV, NV, NP) -> (NV, NP, NP)
    {
      const int o = q, ox = o % NV, oy = (o / NV) % NP, oz = o / (NV * NP);
      s = 0;
      if (o < NV * NP * (DIM == 3 ? NP : 1)) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
          T m = Q.Vp[i][0];
#pragma unroll
          for (int j = 1; j < NP; ++j) m = oy == j ? Q.Vp[i][j] : m;
          s += m * A[ox + NV * (i + NV * oz)];
        }
      }
      __syncthreads();
      if (in_slot) Bf[q] = s;
      __syncthreads();
    }
    // x: (NV, NP, NP) -> (NP, NP, NP)
    {
      const int o = q, ox = o % NP, oy = (o / NP) % NP, oz = o / (NP * NP);
      s = 0;
      if (o < NPN) {
#pragma unroll
        for (int i = 0; i < NV; ++i) {
          T m = Q.Vp[i][0];
#pragma unroll
          for (int j = 1; j < NP; ++j) m = ox == j ? Q.Vp[i][j] : m;
          s += m * Bf[i + NV * (oy + NP * oz)];
        }
      }
      if (live && q < NPN) {
        if (g.cbp != nullptr) {
          g.cbp[cell * NPN + q] = s;
        } else {
          const i64 pn = ((K - 1) * cx + ox) + (i64)g.pd[0] * (((K - 1) * cy + oy) + (i64)g.pd[1] * ((K - 1) * cz + oz));
          g.tp[pn] += s;
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// 3D cells in line layout (every-cell mode, the production path in 3D).
//
// One wave64 per CPW = 64 / (k+1)^2 cells that are consecutive in x.  Lane l
// belongs to cell slot s = l / (k+1)^2 and holds one line of k+1 entries of
// its cell: with r = l % (k+1)^2 and (a, b) = (r % (k+1), r / (k+1)),
//   an x line runs through (y, z) = (a, b), a y line through (x, z) = (a, b),
//   a z line through (x, y) = (a, b).
// A 1D pass along the line costs k+1 FMA per entry with wave-uniform
// coefficients (compile-time constants); lines change direction through
// LDS, each lane writing its line and reading another.  Forward: the nodal
// values are loaded as x lines (contiguous in memory), interpolated to the
// Gauss points along x, y and z; the reference gradients follow from the
// collocation derivative at the Gauss points along each direction.  The
// quadrature-point work runs on z lines: on a trilinear cell the column
// d x / d zeta of J is constant along a z line and the other two columns
// are linear in zeta.  Backward: the transposed passes in reverse order, the
// velocity results leave as x lines (contiguous), into the per-cell results
// the gather kernel sums (gen3_result_index).  Every index stays within
// the cell of the lane's slot; lanes of a slot past the last cell of the
// row (and the spare slot when (k+1)^2 does not divide 64) work on the
// row's last cell and store nothing.
// ---------------------------------------------------------------------------
// LDS position of entry (x, y, z) of a cell slot: strides 1, PY, PZ, slots
// LINE_SLOT apart.  For k+1 = 4 the strides are padded (5, 20, slot 80), which
// takes the bank conflicts of the x and y line accesses of a wave from 4-way
// to none and leaves the z line accesses at 2-way (the unpadded 4, 16, 64
// layout: 4, 4 and 2-4 way).
template <int NV>
struct LineLayout {
  static constexpr int PY = NV == 4 ? 5 : NV;
  static constexpr int PZ = NV == 4 ? 20 : NV * NV;
  static constexpr int SLOT = NV == 4 ? 80 : NV * NV * NV;
};
template <int NV>
__device__ __forceinline__ int line_index(int dir, int a, int b, int i) {
  constexpr int PY = LineLayout<NV>::PY, PZ = LineLayout<NV>::PZ;
  return dir == 0 ? i + PY * a + PZ * b : (dir == 1 ? a + PY * i + PZ * b : a + PY * b + PZ * i);
}

// out[o] = sum_i m[o][i] in[i] (TR: sum_i m[i][o] in[i]); ACC adds to out.
template <bool TR, bool ACC, int NO, int NI, typename T, int R, int C>
__device__ __forceinline__ void line_pass(const T (&m)[R][C], const T (&in)[NI], T (&out)[NO]) {
  static_assert(TR ? (R == NI && C == NO) : (R == NO && C == NI), "line_pass shape");
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    T acc = (TR ? m[0][o] : m[o][0]) * in[0];
#pragma unroll
    for (int i = 1; i < NI; ++i) acc += (TR ? m[i][o] : m[o][i]) * in[i];
    out[o] = ACC ? out[o] + acc : acc;
  }
}

// Cells a launch of gen3_line_kernel covers per block, and its block count.
template <int K>
constexpr int gen3_cells_per_wave() {
  return 64 / ((K + 1) * (K + 1));
}
template <int K, typename T>
inline i64 gen3_blocks(const GenGeo<T> &g) {
  constexpr int CPW = gen3_cells_per_wave<K>();
  return (i64)((g.n[0] + CPW - 1) / CPW) * g.n[1] * g.n[2];
}

// Per-cell results of the line-layout kernel, ordered so that the gather
// reads them along x rows: velocity [comp][cz][cy][lz][ly][cx][lx] and
// pressure [cz][cy][lz][ly][cx][lx] (cell (cx, cy, cz), local node
// (lx, ly, lz) with NS nodes per direction); the x lines a wave writes and a
// gather wave reads are contiguous.
template <int NS>
__host__ __device__ __forceinline__ i64 gen3_result_index(const int (&n)[3], int comp, int cx, int cy, int cz, int lx,
                                                          int ly, int lz) {
  return ((((i64)comp * n[2] + cz) * n[1] + cy) * NS * NS + (i64)lz * NS + ly) * ((i64)n[0] * NS) + (i64)cx * NS + lx;
}

// Block and lane -> cell slot s, line (a, b) and cell (cx, cy, cz) of the
// line-layout kernel; live is false for lanes that store nothing (their cell
// is the last of the row).
struct Gen3Lane {
  int s, a, b, cx, cy, cz;
  bool live;
};
template <int K>
__host__ __device__ __forceinline__ Gen3Lane gen3_lane(const int (&n)[3], int block, int nblocks, int lane) {
  constexpr int NV = K + 1, NL = NV * NV, CPW = gen3_cells_per_wave<K>();
  Gen3Lane l;
  l.s = lane / NL;
  const int r = lane - l.s * NL;
  l.a = r % NV;
  l.b = r / NV;
  // the wave's cells: CPW consecutive cells of one x row; the rows of one
  // XCD are contiguous in (y, z)
  const int wrow = (n[0] + CPW - 1) / CPW;
  const int w = xcd_contiguous_tile(block, nblocks);
  const int wx = w % wrow;
  const int rest = w / wrow;
  l.cy = rest % n[1];
  l.cz = rest / n[1];
  l.live = l.s < CPW && wx * CPW + l.s < n[0];
  l.cx = l.live ? wx * CPW + l.s : n[0] - 1;
  return l;
}

template <int K, typename T, int BLK, class Op>
__global__ void __launch_bounds__(64) gen3_line_kernel(const GenGeo<T> g, const Op op) {
  constexpr int NV = K + 1, NP = K;
  constexpr int NL = NV * NV;                 // lines per cell and direction
  constexpr int SLOTS = (64 + NL - 1) / NL;   // a spare slot when NL does not divide 64
  constexpr cfe::QTab<K, T> Q = cfe::make_qtab<K, T>();
  constexpr bool NEED_U = (BLK & (BLK_A | BLK_MASS | BLK_B)) != 0;
  constexpr bool NEED_P = (BLK & (BLK_BT | BLK_C)) != 0;
  constexpr bool OUT_U = (BLK & (BLK_A | BLK_MASS | BLK_BT)) != 0;
  constexpr bool OUT_P = (BLK & (BLK_B | BLK_C)) != 0;
  __shared__ T lds[3][SLOTS * LineLayout<NV>::SLOT];

  const Gen3Lane ln = gen3_lane<K>(g.n, (int)blockIdx.x, (int)gridDim.x, (int)threadIdx.x);
  const int s = ln.s, a = ln.a, b = ln.b, cx = ln.cx, cy = ln.cy, cz = ln.cz;
  const bool live = ln.live;
  const i64 cell = cx + (i64)g.n[0] * (cy + (i64)g.n[1] * cz);
  T *const B0 = lds[0] + s * LineLayout<NV>::SLOT;
  T *const B1 = lds[1] + s * LineLayout<NV>::SLOT;
  T *const B2 = lds[2] + s * LineLayout<NV>::SLOT;
  auto put = [&](T *B, int dir, const T(&v)[NV]) {
#pragma unroll
    for (int i = 0; i < NV; ++i) B[line_index<NV>(dir, a, b, i)] = v[i];
  };
  auto get = [&](const T *B, int dir, T(&v)[NV]) {
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = B[line_index<NV>(dir, a, b, i)];
  };

  // ---- velocity: values and reference gradients at the points (a, b, k) of the z line
  T uq[3][NV], gq[3][3][NV];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      uq[c][k] = 0;
      gq[c][0][k] = gq[c][1][k] = gq[c][2][k] = 0;
    }
  if constexpr (NEED_U) {
    const int gy = K * cy + a, gz = K * cz + b;
    const bool bc_yz = on_box_boundary(gy, g.vd[1]) || on_box_boundary(gz, g.vd[2]);
    const i64 row = (i64)g.vd[0] * (gy + (i64)g.vd[1] * gz) + K * cx;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T u[NV], t[NV], t2[NV];
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const bool bc = bc_yz || on_box_boundary(K * cx + i, g.vd[0]);
        u[i] = (Op::ZERO_BC && bc) ? T(0) : op.load_u((i64)c * g.Nv + row + i);
      }
      line_pass<false, false, NV, NV>(Q.V, u, t);   // x: nodes -> points
      put(B0, 0, t);
      __syncthreads();
      get(B0, 1, t2);
      line_pass<false, false, NV, NV>(Q.V, t2, t);  // y
      put(B1, 1, t);
      __syncthreads();
      get(B1, 2, t2);
      line_pass<false, false, NV, NV>(Q.V, t2, uq[c]);       // z: values at the points
      line_pass<false, false, NV, NV>(Q.D, uq[c], gq[c][2]);  // d / d zeta
      put(B2, 2, uq[c]);
      __syncthreads();
      get(B2, 0, t2);
      line_pass<false, false, NV, NV>(Q.D, t2, t);  // d / d xi on the x lines
      put(B0, 0, t);
      get(B2, 1, t2);
      line_pass<false, false, NV, NV>(Q.D, t2, t);  // d / d eta on the y lines
      put(B1, 1, t);
      __syncthreads();
      get(B0, 2, gq[c][0]);
      get(B1, 2, gq[c][1]);
      __syncthreads();
    }
  }

  // ---- pressure at the points of the z line (pressure lines: K nodes)
  T pq[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) pq[k] = 0;
  if constexpr (NEED_P) {
    T p[NP], t[NV], t2[NP];
    const bool pl = a < NP && b < NP;
    const i64 prow = (i64)g.pd[0] * ((K - 1) * cy + a + (i64)g.pd[1] * ((K - 1) * cz + b)) + (K - 1) * cx;
#pragma unroll
    for (int i = 0; i < NP; ++i) p[i] = pl ? op.load_p(prow + i) : T(0);
    line_pass<false, false, NV, NP>(Q.Vp, p, t);   // x lines (y, z) = (a, b) < NP
    put(B0, 0, t);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NP; ++j) t2[j] = B0[line_index<NV>(1, a, b, j)];
    line_pass<false, false, NV, NP>(Q.Vp, t2, t);  // y lines (x, z) = (a, b), z < NP
    put(B1, 1, t);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NP; ++k) t2[k] = B1[line_index<NV>(2, a, b, k)];
    line_pass<false, false, NV, NP>(Q.Vp, t2, pq);  // z lines
    __syncthreads();
  }

  // ---- geometry of the trilinear map on the z line (xi, eta) = (x_a, x_b)
  T dE[3], E0[3], dF[3], F0[3], Zc[3];
  {
    const i64 vx = g.n[0] + 1, vxy = vx * (g.n[1] + 1);
    const i64 v0 = cx + vx * cy + vxy * cz;
    T X[8][3];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const i64 vid = v0 + (v & 1) + vx * ((v >> 1) & 1) + vxy * ((v >> 2) & 1);
#pragma unroll
      for (int d = 0; d < 3; ++d) X[v][d] = g.verts[vid * 3 + d];
    }
    const T xi = pick(Q.x, a), eta = pick(Q.x, b);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      // vertex v = ox + 2 oy + 4 oz
      const T e0 = (X[1][d] - X[0][d]) * (T(1) - eta) + (X[3][d] - X[2][d]) * eta;   // d/dxi, zeta = 0
      const T e1 = (X[5][d] - X[4][d]) * (T(1) - eta) + (X[7][d] - X[6][d]) * eta;   // d/dxi, zeta = 1
      const T f0 = (X[2][d] - X[0][d]) * (T(1) - xi) + (X[3][d] - X[1][d]) * xi;     // d/deta, zeta = 0
      const T f1 = (X[6][d] - X[4][d]) * (T(1) - xi) + (X[7][d] - X[5][d]) * xi;     // d/deta, zeta = 1
      E0[d] = e0;
      dE[d] = e1 - e0;
      F0[d] = f0;
      dF[d] = f1 - f0;
      Zc[d] = ((X[4][d] - X[0][d]) * (T(1) - xi) + (X[5][d] - X[1][d]) * xi) * (T(1) - eta) +
              ((X[6][d] - X[2][d]) * (T(1) - xi) + (X[7][d] - X[3][d]) * xi) * eta;
    }
  }
  const T wab = pick(Q.w, a) * pick(Q.w, b);
  const T mu = g.mu_cell != nullptr ? g.mu_cell[cell] : g.mu;

  // ---- integrands at the points of the z line (in place: gq -> test coefficients)
  T vq[3][NV], pc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    T J[3][3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      J[d][0] = E0[d] + Q.x[k] * dE[d];
      J[d][1] = F0[d] + Q.x[k] * dF[d];
      J[d][2] = Zc[d];
    }
    const T c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const T c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const T c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const T det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    T id;
    if constexpr (std::is_same<T, float>::value) id = __builtin_amdgcn_rcpf(det);   // 1 ulp (FP32 cycle)
    else id = T(1) / det;
    T Ji[3][3];   // J^-1
    Ji[0][0] = c00 * id;
    Ji[1][0] = c01 * id;
    Ji[2][0] = c02 * id;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
    const T JxW = det * wab * Q.w[k];
    T gp[3][3];   // physical gradients grad u_c
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int e = 0; e < 3; ++e) gp[c][e] = Ji[0][e] * gq[c][0][k] + Ji[1][e] * gq[c][1][k] + Ji[2][e] * gq[c][2][k];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T val = 0;
      if constexpr ((BLK & BLK_A) != 0) val += g.gr * uq[c][k];
      if constexpr ((BLK & BLK_MASS) != 0) val += uq[c][k];
      vq[c][k] = val * JxW;
      T G[3] = {0, 0, 0};
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        if constexpr ((BLK & BLK_A) != 0) G[e] = mu * (g.sym ? T(0.5) * (gp[c][e] + gp[e][c]) : gp[c][e]);
        if constexpr ((BLK & BLK_BT) != 0)
          if (e == c) G[e] -= pq[k];
      }
#pragma unroll
      for (int d = 0; d < 3; ++d) gq[c][d][k] = (Ji[d][0] * G[0] + Ji[d][1] * G[1] + Ji[d][2] * G[2]) * JxW;
    }
    T pv = 0;
    if constexpr ((BLK & BLK_B) != 0) pv -= gp[0][0] + gp[1][1] + gp[2][2];
    if constexpr ((BLK & BLK_C) != 0) pv += ((BLK & BLK_CPLUS) ? g.cp : -g.cp) * pq[k];
    pc[k] = pv * JxW;
  }

  // ---- velocity test functions, per component; results as x lines
  if constexpr (OUT_U) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T wz[NV], t[NV], t2[NV];
#pragma unroll
      for (int k = 0; k < NV; ++k) wz[k] = vq[c][k];
      line_pass<true, true, NV, NV>(Q.D, gq[c][2], wz);   // + D^T along z
      put(B0, 2, gq[c][0]);
      put(B1, 2, gq[c][1]);
      __syncthreads();
      get(B0, 0, t2);
      line_pass<true, false, NV, NV>(Q.D, t2, t);   // D^T along x
      __syncthreads();
      put(B0, 0, t);
      get(B1, 1, t2);
      line_pass<true, false, NV, NV>(Q.D, t2, t);   // D^T along y
      __syncthreads();
      put(B1, 1, t);
      __syncthreads();
      get(B0, 2, t2);
#pragma unroll
      for (int k = 0; k < NV; ++k) wz[k] += t2[k];
      get(B1, 2, t2);
#pragma unroll
      for (int k = 0; k < NV; ++k) wz[k] += t2[k];
      line_pass<true, false, NV, NV>(Q.V, wz, t);   // z: points -> nodes
      put(B2, 2, t);
      __syncthreads();
      get(B2, 1, t2);
      line_pass<true, false, NV, NV>(Q.V, t2, t);   // y
      __syncthreads();
      put(B0, 1, t);
      __syncthreads();
      get(B0, 0, t2);
      line_pass<true, false, NV, NV>(Q.V, t2, t);   // x
      if (live) {
        T *dst = g.cbu + gen3_result_index<NV>(g.n, c, cx, cy, cz, 0, a, b);
#pragma unroll
        for (int i = 0; i < NV; ++i) dst[i] = t[i];
      }
      __syncthreads();
    }
  }

  // ---- pressure test functions; results as x lines of K nodes
  if constexpr (OUT_P) {
    T t[NP], t2[NV];
    line_pass<true, false, NP, NV>(Q.Vp, pc, t);   // z: points -> pressure nodes
#pragma unroll
    for (int k = 0; k < NP; ++k) B0[line_index<NV>(2, a, b, k)] = t[k];
    __syncthreads();
    get(B0, 1, t2);                                // y lines (x, z) = (a, b), z < K
    line_pass<true, false, NP, NV>(Q.Vp, t2, t);
#pragma unroll
    for (int j = 0; j < NP; ++j) B1[line_index<NV>(1, a, b, j)] = t[j];
    __syncthreads();
    get(B1, 0, t2);                                // x lines (y, z) = (a, b) < K
    line_pass<true, false, NP, NV>(Q.Vp, t2, t);
    if (live && a < NP && b < NP) {
      T *dst = g.cbp + gen3_result_index<NP>(g.n, 0, cx, cy, cz, 0, a, b);
#pragma unroll
      for (int i = 0; i < NP; ++i) dst[i] = t[i];
    }
  }
}

// Dirichlet rows and the caller's epilogue on every node, from the
// accumulated cell sums.
template <int DIM, typename T, int BLK, class Op>
__global__ void gen_epilogue_kernel(const GenGeo<T> g, const Op op) {
  constexpr bool NEED_U = (BLK & (BLK_A | BLK_MASS | BLK_B)) != 0;
  constexpr bool NEED_P = (BLK & (BLK_BT | BLK_C)) != 0;
  constexpr bool OUT_U = (BLK & (BLK_A | BLK_MASS | BLK_BT)) != 0;
  constexpr bool OUT_P = (BLK & (BLK_B | BLK_C)) != 0;
  const i64 nu = OUT_U ? (i64)DIM * g.Nv : 0;
  const i64 total = nu + (OUT_P ? g.Np : 0);
  SMG_GRID_LOOP(i, total) {
    if (i < nu) {
      const i64 node = i % g.Nv;
      const int x = (int)(node % g.vd[0]);
      const i64 r = node / g.vd[0];
      const int y = (int)(r % g.vd[1]);
      const int z = (int)(r / g.vd[1]);
      const bool bc = on_box_boundary(x, g.vd[0]) || on_box_boundary(y, g.vd[1]) ||
                      (DIM == 3 && on_box_boundary(z, g.vd[2]));
      const T v = NEED_U ? op.load_u(i) : T(0);
      const T t = bc ? ((BLK & BLK_A) != 0 ? v : T(0)) : g.tu[i];
      op.store_u(i, t, bc ? t : v, bc, op.fetch_u(i));
    } else {
      const i64 j = i - nu;
      op.store_p(j, g.tp[j], NEED_P ? op.load_p(j) : T(0), op.fetch_p(j));
    }
  }
}

// Every-cell mode: the sum over the cells around a lattice node of their
// per-cell results, cells in increasing index order (fixed summation order).
// deg: node spacing per cell (K for the velocity, K - 1 for the pressure);
// nn: results per cell and component; lattice node (x, y, z).
template <int DIM, int DEG, int NPC, typename T>
__device__ __forceinline__ T gather_cells(const GenGeo<T> &g, const T *cb, int ncomp, int comp, int x, int y, int z) {
  int c0[3], nc[3];
  const int xyz[3] = {x, y, z};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a >= DIM) {
      c0[a] = 0;
      nc[a] = 1;
      continue;
    }
    const int c = xyz[a] / DEG;
    if (xyz[a] % DEG == 0) {
      // a cell boundary: the cells on both sides that exist
      c0[a] = c > 0 ? c - 1 : 0;
      nc[a] = (c > 0 ? 1 : 0) + (c < g.n[a] ? 1 : 0);
    } else {
      c0[a] = c;
      nc[a] = 1;
    }
  }
  constexpr int NS = DEG + 1;  // nodes per cell and direction
  T acc = 0;
  for (int k = 0; k < nc[2]; ++k)
    for (int j = 0; j < nc[1]; ++j)
      for (int i = 0; i < nc[0]; ++i) {
        const int cx = c0[0] + i, cy = c0[1] + j, cz = c0[2] + k;
        const int lx = x - DEG * cx, ly = y - DEG * cy, lz = z - DEG * cz;
        const i64 cell = cx + (i64)g.n[0] * (cy + (i64)g.n[1] * cz);
        acc += cb[(cell * ncomp + comp) * NPC + lx + NS * (ly + NS * lz)];
      }
  return acc;
}

// Every-cell mode epilogue: sums of the per-cell results, then the Dirichlet
// rows and the caller's epilogue as in gen_epilogue_kernel.
template <int DIM, int K, typename T, int BLK, class Op>
__global__ void gen_gather_epilogue_kernel(const GenGeo<T> g, const Op op) {
  constexpr int NV = K + 1, NP = K;
  constexpr int NN = DIM == 3 ? NV * NV * NV : NV * NV;
  constexpr int NPN = DIM == 3 ? NP * NP * NP : NP * NP;
  constexpr bool NEED_U = (BLK & (BLK_A | BLK_MASS | BLK_B)) != 0;
  constexpr bool NEED_P = (BLK & (BLK_BT | BLK_C)) != 0;
  constexpr bool OUT_U = (BLK & (BLK_A | BLK_MASS | BLK_BT)) != 0;
  constexpr bool OUT_P = (BLK & (BLK_B | BLK_C)) != 0;
  const i64 nu = OUT_U ? (i64)DIM * g.Nv : 0;
  const i64 total = nu + (OUT_P ? g.Np : 0);
  SMG_GRID_LOOP(i, total) {
    if (i < nu) {
      const int c = (int)(i / g.Nv);
      const i64 node = i - (i64)c * g.Nv;
      const int x = (int)(node % g.vd[0]);
      const i64 r = node / g.vd[0];
      const int y = (int)(r % g.vd[1]);
      const int z = (int)(r / g.vd[1]);
      const bool bc = on_box_boundary(x, g.vd[0]) || on_box_boundary(y, g.vd[1]) ||
                      (DIM == 3 && on_box_boundary(z, g.vd[2]));
      const T v = NEED_U ? op.load_u(i) : T(0);
      const T tsum = bc ? T(0) : gather_cells<DIM, K, NN>(g, g.cbu, DIM, c, x, y, z);
      const T t = bc ? ((BLK & BLK_A) != 0 ? v : T(0)) : tsum;
      op.store_u(i, t, bc ? t : v, bc, op.fetch_u(i));
    } else {
      const i64 j = i - nu;
      const int x = (int)(j % g.pd[0]);
      const i64 r = j / g.pd[0];
      const int y = (int)(r % g.pd[1]);
      const int z = (int)(r / g.pd[1]);
      const T t = gather_cells<DIM, K - 1, NPN>(g, g.cbp, 1, 0, x, y, z);
      op.store_p(j, t, NEED_P ? op.load_p(j) : T(0), op.fetch_p(j));
    }
  }
}

// n / d for 0 <= n < 2^31 without a division: n m >> (31 + s) with
// s = ceil(log2 d), m = ceil(2^(31+s) / d) < 2^32 (the rounding error of m
// shifts n / d by less than n d / 2^(31+s) / d < 1 / d, which never crosses
// an integer).
struct FastDiv {
  uint32_t d, m, s;
};
inline FastDiv make_fastdiv(uint32_t d) {
  uint32_t s = 0;
  while ((1ull << s) < d) ++s;
  const uint64_t p = 1ull << (31 + s);
  return FastDiv{d, (uint32_t)((p + d - 1) / d), s};
}
__host__ __device__ __forceinline__ uint32_t fast_div(uint32_t n, const FastDiv &f) {
  return (uint32_t)(((uint64_t)n * f.m) >> (31 + f.s));
}

// The cells around lattice coordinate v (spacing deg per cell, n cells) along
// one direction: first cell c0 and count (1 inside a cell, 2 on an interior
// cell boundary, 1 on the domain boundary).
__host__ __device__ __forceinline__ void cells_around(int v, int deg, int n, int &c0, int &nc) {
  const int c = v / deg;
  if (v - c * deg == 0) {
    c0 = c > 0 ? c - 1 : 0;
    nc = (c > 0 ? 1 : 0) + (c < n ? 1 : 0);
  } else {
    c0 = c;
    nc = 1;
  }
}

// Sum of the per-cell results at lattice node (x, y, z) over the cells
// around it (c0, nc per direction), cells in increasing index order.  All
// eight candidate reads are issued unconditionally (a missing second cell
// reads the first one again) and the missing ones add zero, so the loads
// overlap and the sum equals the one over the existing cells in that order.
template <int NS, int DEG, typename T>
__device__ __forceinline__ T sum_cells(const T *res, const int (&n)[3], int comp, int x, int y, int z,
                                       const int (&c0)[3], const int (&nc)[3]) {
  T v[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int cx = c0[0] + ((e & 1) && nc[0] == 2 ? 1 : 0);
    const int cy = c0[1] + ((e & 2) && nc[1] == 2 ? 1 : 0);
    const int cz = c0[2] + ((e & 4) && nc[2] == 2 ? 1 : 0);
    v[e] = res[gen3_result_index<NS>(n, comp, cx, cy, cz, x - DEG * cx, y - DEG * cy, z - DEG * cz)];
  }
  T acc = 0;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const bool ok = (!(e & 1) || nc[0] == 2) && (!(e & 2) || nc[1] == 2) && (!(e & 4) || nc[2] == 2);
    acc += ok ? v[e] : T(0);
  }
  return acc;
}

// 3D every-cell mode epilogue: one thread per velocity node (its three
// components) or pressure node, the sum over the cells around the node of
// their results in increasing cell order, then the Dirichlet rows and the
// caller's epilogue as in gen_gather_epilogue_kernel.  Threads of one XCD
// take a contiguous range of nodes (z slabs, as the cell kernel's waves).
// fv: divisions by the velocity lattice extents vd[0], vd[1]; fp: pressure.
template <int K, typename T, int BLK, class Op>
__global__ void __launch_bounds__(256)
gen3_gather_kernel(const GenGeo<T> g, const Op op, const FastDiv fv0, const FastDiv fv1, const FastDiv fp0,
                   const FastDiv fp1) {
  constexpr int NV = K + 1, NP = K;
  constexpr bool NEED_U = (BLK & (BLK_A | BLK_MASS | BLK_B)) != 0;
  constexpr bool NEED_P = (BLK & (BLK_BT | BLK_C)) != 0;
  constexpr bool OUT_U = (BLK & (BLK_A | BLK_MASS | BLK_BT)) != 0;
  constexpr bool OUT_P = (BLK & (BLK_B | BLK_C)) != 0;
  const uint32_t t = (uint32_t)xcd_contiguous_tile((int)blockIdx.x, (int)gridDim.x) * 256u + threadIdx.x;
  const uint32_t nv = OUT_U ? (uint32_t)g.Nv : 0u;
  if (t < nv) {
    const uint32_t q = fast_div(t, fv0);
    const int x = (int)(t - q * fv0.d);
    const uint32_t zq = fast_div(q, fv1);
    const int y = (int)(q - zq * fv1.d);
    const int z = (int)zq;
    const bool bc = on_box_boundary(x, g.vd[0]) || on_box_boundary(y, g.vd[1]) || on_box_boundary(z, g.vd[2]);
    int c0[3], nc[3];
    cells_around(x, K, g.n[0], c0[0], nc[0]);
    cells_around(y, K, g.n[1], c0[1], nc[1]);
    cells_around(z, K, g.n[2], c0[2], nc[2]);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const i64 i = (i64)c * g.Nv + t;
      const T v = NEED_U ? op.load_u(i) : T(0);
      const T acc = sum_cells<NV, K, T>(g.cbu, g.n, c, x, y, z, c0, nc);
      const T r = bc ? ((BLK & BLK_A) != 0 ? v : T(0)) : acc;
      op.store_u(i, r, bc ? r : v, bc, op.fetch_u(i));
    }
  } else if (OUT_P && t - nv < (uint32_t)g.Np) {
    const uint32_t j = t - nv;
    const uint32_t q = fast_div(j, fp0);
    const int x = (int)(j - q * fp0.d);
    const uint32_t zq = fast_div(q, fp1);
    const int y = (int)(q - zq * fp1.d);
    const int z = (int)zq;
    int c0[3], nc[3];
    cells_around(x, K - 1, g.n[0], c0[0], nc[0]);
    cells_around(y, K - 1, g.n[1], c0[1], nc[1]);
    cells_around(z, K - 1, g.n[2], c0[2], nc[2]);
    const T acc = sum_cells<NP, K - 1, T>(g.cbp, g.n, 0, x, y, z, c0, nc);
    op.store_p(j, acc, NEED_P ? op.load_p(j) : T(0), op.fetch_p(j));
  }
}

// Adjoint-state gradient with respect to the per-cell log-viscosity:
//   out[tau] = - mu_tau int_tau sum_c grad lam_c . grad u_c
//   (- mu_tau int_tau eps(lam) : eps(u) for the deformation-rate form)
// (constrained velocity entries of u and lam taken as zero), every cell of
// the level in one launch; one lane per quadrature point, LDS passes as in
// gen_apply_kernel, then a sum over the cell's lanes.  FP64.
template <int DIM, int K>
__global__ void __launch_bounds__(64) gen_grad_logmu_kernel(const GenGeo<double> g, const double *x,
                                                            const double *lam, double *out) {
  using T = double;
  constexpr int NV = K + 1;
  constexpr int NN = DIM == 3 ? NV * NV * NV : NV * NV;
  constexpr int CPB = 64 / NN;
  constexpr int NVERT = 1 << DIM;
  constexpr cfe::QTab<K, T> Q = cfe::make_qtab<K, T>();
  __shared__ T lds[CPB][2][NN];

  const int tid = threadIdx.x;
  const int slot = tid / NN;
  const int q = tid - slot * NN;
  const bool in_slot = slot < CPB;
  const int sl = in_slot ? slot : 0;
  const i64 ncells = (i64)g.n[0] * g.n[1] * (DIM == 3 ? g.n[2] : 1);
  const i64 ci = (i64)blockIdx.x * CPB + slot;
  const bool live = in_slot && ci < ncells;
  int cx = 0, cy = 0, cz = 0;
  if (live) {
    cx = (int)(ci % g.n[0]);
    const i64 r = ci / g.n[0];
    cy = (int)(r % g.n[1]);
    cz = DIM == 3 ? (int)(r / g.n[1]) : 0;
  }
  const int qx = q % NV, qy = (q / NV) % NV, qz = DIM == 3 ? q / (NV * NV) : 0;
  const int qd[3] = {qx, qy, qz};
  T *A = lds[sl][0], *Bf = lds[sl][1];
  T rV[3][NV], rD[3][NV];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      T vr = Q.V[0][i], dr = Q.D[0][i];
#pragma unroll
      for (int j = 1; j < NV; ++j) {
        vr = qd[d] == j ? Q.V[j][i] : vr;
        dr = qd[d] == j ? Q.D[j][i] : dr;
      }
      rV[d][i] = vr;
      rD[d][i] = dr;
    }
  auto lidx = [](int a, int b, int c) { return a + NV * (b + NV * c); };
  auto pass = [&](const T *in, const T (&m)[NV], int d) {
    T s = 0;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const int k = d == 0 ? lidx(i, qy, qz) : (d == 1 ? lidx(qx, i, qz) : lidx(qx, qy, i));
      s += m[i] * in[k];
    }
    return s;
  };
  // geometry
  T Jinv[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  T JxW = 0, mu = g.mu;
  if (live) {
    const T xi[3] = {pick(Q.x, qx), pick(Q.x, qy), DIM == 3 ? pick(Q.x, qz) : T(0)};
    T J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
#pragma unroll
    for (int v = 0; v < NVERT; ++v) {
      const int o[3] = {v & 1, (v >> 1) & 1, (v >> 2) & 1};
      const i64 vid = (cx + o[0]) + (i64)(g.n[0] + 1) * ((cy + o[1]) + (i64)(g.n[1] + 1) * (DIM == 3 ? cz + o[2] : 0));
#pragma unroll
      for (int b = 0; b < DIM; ++b) {
        T dn = o[b] ? T(1) : T(-1);
#pragma unroll
        for (int c = 0; c < DIM; ++c)
          if (c != b) dn *= o[c] ? xi[c] : T(1) - xi[c];
#pragma unroll
        for (int a = 0; a < DIM; ++a) J[a][b] += g.verts[vid * DIM + a] * dn;
      }
    }
    T det;
    if constexpr (DIM == 2) {
      det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
      const T id = T(1) / det;
      Jinv[0][0] = J[1][1] * id;
      Jinv[0][1] = -J[0][1] * id;
      Jinv[1][0] = -J[1][0] * id;
      Jinv[1][1] = J[0][0] * id;
      JxW = det * pick(Q.w, qx) * pick(Q.w, qy);
    } else {
      const T c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
      const T c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
      const T c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
      det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
      const T id = T(1) / det;
      Jinv[0][0] = c00 * id;
      Jinv[1][0] = c01 * id;
      Jinv[2][0] = c02 * id;
      Jinv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
      Jinv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
      Jinv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
      Jinv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
      Jinv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
      Jinv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
      JxW = det * pick(Q.w, qx) * pick(Q.w, qy) * pick(Q.w, qz);
    }
    if (g.mu_cell != nullptr) mu = g.mu_cell[cx + (i64)g.n[0] * (cy + (i64)g.n[1] * cz)];
  }
  const int gx = K * cx + qx, gy = K * cy + qy, gz = K * cz + qz;
  const i64 vnode = gx + (i64)g.vd[0] * (gy + (i64)g.vd[1] * gz);
  const bool vbc = on_box_boundary(gx, g.vd[0]) || on_box_boundary(gy, g.vd[1]) ||
                   (DIM == 3 && on_box_boundary(gz, g.vd[2]));
  // physical gradient at this lane's point of the field `src` (component c)
  auto grad_at = [&](const double *src, int c, T (&gp)[3]) {
    T v = 0;
    if (live && !vbc) v = src[(i64)c * g.Nv + vnode];
    if (in_slot) A[q] = v;
    __syncthreads();
    T t = pass(A, rV[0], 0);
    if (in_slot) Bf[q] = t;
    __syncthreads();
    t = pass(Bf, rV[1], 1);
    if constexpr (DIM == 3) {
      if (in_slot) A[q] = t;
      __syncthreads();
      t = pass(A, rV[2], 2);
    }
    T *Fq = DIM == 3 ? Bf : A;
    __syncthreads();
    if (in_slot) Fq[q] = t;
    __syncthreads();
    T gr[3] = {0, 0, 0};
#pragma unroll
    for (int d = 0; d < DIM; ++d) gr[d] = pass(Fq, rD[d], d);
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      T s = 0;
#pragma unroll
      for (int b = 0; b < DIM; ++b) s += Jinv[b][a] * gr[b];
      gp[a] = s;
    }
  };
  T gu[DIM][3], gl[DIM][3];
#pragma unroll
  for (int c = 0; c < DIM; ++c) {
    grad_at(x, c, gu[c]);
    grad_at(lam, c, gl[c]);
  }
  T acc = 0;
#pragma unroll
  for (int c = 0; c < DIM; ++c)
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      if (g.sym) acc += T(0.25) * (gu[c][a] + gu[a][c]) * (gl[c][a] + gl[a][c]);
      else acc += gu[c][a] * gl[c][a];
    }
  acc *= JxW;
  if (in_slot) A[q] = acc;
  __syncthreads();
  if (live && q == 0) {
    T s = 0;
    for (int i = 0; i < NN; ++i) s += A[i];
    out[ci] = -mu * s;
  }
}

}  // namespace smg
