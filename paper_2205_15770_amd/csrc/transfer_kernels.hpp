// Level-to-level transfers of the geometric multigrid (Sec. 3.2): the
// prolongation P is the canonical injection of the coarse Q_k / Q_{k-1}
// spaces into the fine ones, i.e. interpolation of the coarse field at the
// fine nodes, a tensor product of 1D weights W[pos][j] = l_j(t_pos) (pos =
// 0..2 deg: fine node within the coarse cell, j = 0..deg: coarse node);
// the restriction is its transpose, R = P^T.  Velocity rows and columns of
// Dirichlet nodes are zero.
//
// prolongation: one thread per fine node, x_f += P w_c.  A block covers a
//   run of fine nodes along x with fixed (y, z), so the y and z weights are
//   uniform across the block and only the x weights vary by lane.
// restriction: one block per run of coarse nodes along x with fixed (y, z):
//   the fine values in the (y, z) support are first summed with the uniform
//   y/z weights into an LDS row (coalesced loads), then each coarse node
//   applies its x weights to that row.  One pass over the fine vector, no
//   intermediate vectors.
#pragma once
#include "common.hpp"

namespace smg {

// one field (velocity components or pressure) of one pair of levels
template <typename T>
struct XferGeo {
  int cdim[3], fdim[3];  // coarse / fine lattice extents (1 beyond the dimension)
  int ncell_f[3];        // fine cells per direction
  i64 coff, foff;        // offset of the field in the coarse / fine level vector
  i64 cstride, fstride;  // distance between components
  T W[28];               // W[pos * (deg + 1) + j]
};

// coarse cell and position 0..2 DEG of fine lattice node f along one direction
template <int DEG>
__device__ __forceinline__ void fine_pos(int f, int nf_cells, int &cc, int &pos) {
  int cf = f / DEG;
  if (cf > nf_cells - 1) cf = nf_cells - 1;
  cc = cf >> 1;
  pos = f - 2 * DEG * cc;
}

template <typename T, int DIM, int DEG, bool BC>
__global__ void __launch_bounds__(128) k_prolong(const T *__restrict__ wc, T *__restrict__ xf, const XferGeo<T> g) {
  constexpr int ND = DEG + 1;
  const int fx = blockIdx.x * 128 + threadIdx.x;
  const int fy = blockIdx.y;
  const int nz = DIM == 3 ? g.fdim[2] : 1;
  const int comp = blockIdx.z / nz;
  const int fz = blockIdx.z - comp * nz;
  if (fx >= g.fdim[0]) return;
  if (BC) {
    const bool fbc = fx == 0 || fx == g.fdim[0] - 1 || fy == 0 || fy == g.fdim[1] - 1 ||
                     (DIM == 3 && (fz == 0 || fz == g.fdim[2] - 1));
    if (fbc) return;  // Dirichlet rows of P are zero
  }
  int ccx, px, ccy, py, ccz = 0, pz = 0;
  fine_pos<DEG>(fx, g.ncell_f[0], ccx, px);
  fine_pos<DEG>(fy, g.ncell_f[1], ccy, py);
  if (DIM == 3) fine_pos<DEG>(fz, g.ncell_f[2], ccz, pz);
  T wx[ND];
  int cxs[ND];
  bool okx[ND];
#pragma unroll
  for (int j = 0; j < ND; ++j) {
    wx[j] = g.W[px * ND + j];
    cxs[j] = DEG * ccx + j;
    okx[j] = !(BC && (cxs[j] == 0 || cxs[j] == g.cdim[0] - 1));
  }
  const T *src = wc + g.coff + (i64)comp * g.cstride;
  T s = 0;
#pragma unroll
  for (int jz = 0; jz < (DIM == 3 ? ND : 1); ++jz) {
    const T wz = DIM == 3 ? g.W[pz * ND + jz] : T(1);
    const int cz = DIM == 3 ? DEG * ccz + jz : 0;
    if (wz == T(0)) continue;  // uniform
    if (DIM == 3 && BC && (cz == 0 || cz == g.cdim[2] - 1)) continue;
#pragma unroll
    for (int jy = 0; jy < ND; ++jy) {
      const T wy = g.W[py * ND + jy];
      const int cy = DEG * ccy + jy;
      if (wy == T(0)) continue;  // uniform
      if (BC && (cy == 0 || cy == g.cdim[1] - 1)) continue;
      const T *row = src + (i64)g.cdim[0] * (cy + (i64)g.cdim[1] * cz);
      T r = 0;
#pragma unroll
      for (int jx = 0; jx < ND; ++jx) r += (okx[jx] ? wx[jx] : T(0)) * row[cxs[jx]];
      s += wz * wy * r;
    }
  }
  T &out = xf[g.foff + (i64)comp * g.fstride + fx + (i64)g.fdim[0] * (fy + (i64)g.fdim[1] * fz)];
  out += s;
}

template <typename T, int DIM, int DEG, bool BC, int CX>
__global__ void __launch_bounds__(256) k_restrict(const T *__restrict__ rf, T *__restrict__ rc, const XferGeo<T> g) {
  constexpr int ND = DEG + 1;
  constexpr int ROW = 2 * (CX - 1) + 4 * DEG + 1;
  __shared__ T tmp[ROW];
  const int cx0 = blockIdx.x * CX;
  const int cy = blockIdx.y;
  const int nz = DIM == 3 ? g.cdim[2] : 1;
  const int comp = blockIdx.z / nz;
  const int cz = blockIdx.z - comp * nz;
  int fx_lo = 2 * cx0 - 2 * DEG;
  if (fx_lo < 0) fx_lo = 0;
  int fx_hi = 2 * (cx0 + CX - 1) + 2 * DEG;
  if (fx_hi > g.fdim[0] - 1) fx_hi = g.fdim[0] - 1;
  const T *src = rf + g.foff + (i64)comp * g.fstride;

  // 1. fine row: sum over the (y, z) support of (cy, cz) with uniform weights
  for (int fx = fx_lo + (int)threadIdx.x; fx <= fx_hi; fx += 256) {
    const bool xbc = BC && (fx == 0 || fx == g.fdim[0] - 1);
    T s = 0;
    const int fz_lo = DIM == 3 ? (2 * cz - 2 * DEG > 0 ? 2 * cz - 2 * DEG : 0) : 0;
    const int fz_hi = DIM == 3 ? (2 * cz + 2 * DEG < g.fdim[2] - 1 ? 2 * cz + 2 * DEG : g.fdim[2] - 1) : 0;
    for (int fz = fz_lo; fz <= fz_hi; ++fz) {
      T wz = 1;
      if (DIM == 3) {
        int cc, pos;
        fine_pos<DEG>(fz, g.ncell_f[2], cc, pos);
        const int j = cz - DEG * cc;
        if (j < 0 || j > DEG) continue;
        wz = g.W[pos * ND + j];
        if (wz == T(0)) continue;
        if (BC && (fz == 0 || fz == g.fdim[2] - 1)) continue;
      }
      const int fy_lo = 2 * cy - 2 * DEG > 0 ? 2 * cy - 2 * DEG : 0;
      const int fy_hi = 2 * cy + 2 * DEG < g.fdim[1] - 1 ? 2 * cy + 2 * DEG : g.fdim[1] - 1;
      for (int fy = fy_lo; fy <= fy_hi; ++fy) {
        int cc, pos;
        fine_pos<DEG>(fy, g.ncell_f[1], cc, pos);
        const int j = cy - DEG * cc;
        if (j < 0 || j > DEG) continue;
        const T wy = g.W[pos * ND + j];
        if (wy == T(0)) continue;
        if (BC && (fy == 0 || fy == g.fdim[1] - 1)) continue;
        s += wz * wy * src[fx + (i64)g.fdim[0] * (fy + (i64)g.fdim[1] * fz)];
      }
    }
    tmp[fx - fx_lo] = xbc ? T(0) : s;
  }
  __syncthreads();

  // 2. x weights
  const int cx = cx0 + (int)threadIdx.x;
  if (threadIdx.x >= CX || cx >= g.cdim[0]) return;
  bool cbc = false;
  if (BC)
    cbc = cx == 0 || cx == g.cdim[0] - 1 || cy == 0 || cy == g.cdim[1] - 1 ||
          (DIM == 3 && (cz == 0 || cz == g.cdim[2] - 1));
  T s = 0;
  if (!cbc) {
#pragma unroll
    for (int o = -2 * DEG; o <= 2 * DEG; ++o) {
      const int fx = 2 * cx + o;
      if (fx < 0 || fx > g.fdim[0] - 1) continue;
      int cc, pos;
      fine_pos<DEG>(fx, g.ncell_f[0], cc, pos);
      const int j = cx - DEG * cc;
      if (j < 0 || j > DEG) continue;
      s += g.W[pos * ND + j] * tmp[fx - fx_lo];
    }
  }
  rc[g.coff + (i64)comp * g.cstride + cx + (i64)g.cdim[0] * (cy + (i64)g.cdim[1] * cz)] = s;
}

}  // namespace smg
