// Level-to-level transfers of the geometric multigrid (Sec. 3.2): the
// prolongation P is the canonical injection of the coarse Q_k / Q_{k-1}
// spaces into the fine ones, i.e. interpolation of the coarse field at the
// fine nodes, a tensor product of 1D weights W[pos][j] = l_j(t_pos) (pos =
// 0..2 deg: fine node within the coarse cell, j = 0..deg: coarse node);
// the restriction is its transpose, R = P^T.  Velocity rows and columns of
// Dirichlet nodes are zero.
//
// prolongation: one thread per fine node, x_f += P w_c, every coarse value of
//   the node's support requested at once.
// restriction: one block per run of coarse nodes along x with fixed (y, z):
//   the fine values in the (y, z) support are first summed with the y/z
//   weights into an LDS row (coalesced loads), then each coarse node applies
//   its x weights to that row.  One pass over the fine vector, no
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

// 1D weight W[pos][j] for a lane-dependent position (the table is a kernel
// argument; the select chain keeps it out of scratch memory)
template <int DEG, typename T>
__device__ __forceinline__ T weight_at(const T *W, int pos, int j) {
  constexpr int ND = DEG + 1;
  T w = W[j];
#pragma unroll
  for (int p = 1; p <= 2 * DEG; ++p) w = pos == p ? W[p * ND + j] : w;
  return w;
}

// Prolongation x_f += P w_c: one thread per fine node; blocks of 256 threads
// run over the flattened (x, y) plane of one z position and component, so no
// block is left mostly empty by lattice extents of the form 2^j + 1.  All
// (deg+1)^d coarse values of the node's support are requested at once (zero
// weights included; coarse Dirichlet nodes get weight 0).
template <typename T, int DIM, int DEG, bool BC>
__device__ __forceinline__ void prolong_block(const T *__restrict__ wc, T *__restrict__ xf, const XferGeo<T> &g, int bx,
                                              int by) {
  constexpr int ND = DEG + 1;
  const int nxy = g.fdim[0] * g.fdim[1];
  const int t = bx * 256 + threadIdx.x;
  const int nz = DIM == 3 ? g.fdim[2] : 1;
  const int comp = by / nz;
  const int fz = by - comp * nz;
  if (t >= nxy) return;
  const int fy = t / g.fdim[0];
  const int fx = t - fy * g.fdim[0];
  if (BC) {
    const bool fbc = fx == 0 || fx == g.fdim[0] - 1 || fy == 0 || fy == g.fdim[1] - 1 ||
                     (DIM == 3 && (fz == 0 || fz == g.fdim[2] - 1));
    if (fbc) return;  // Dirichlet rows of P are zero
  }
  int ccx, px, ccy, py, ccz = 0, pz = 0;
  fine_pos<DEG>(fx, g.ncell_f[0], ccx, px);
  fine_pos<DEG>(fy, g.ncell_f[1], ccy, py);
  if (DIM == 3) fine_pos<DEG>(fz, g.ncell_f[2], ccz, pz);
  T wx[ND], wy[ND], wz[ND];
#pragma unroll
  for (int j = 0; j < ND; ++j) {
    wx[j] = weight_at<DEG>(g.W, px, j);
    wy[j] = weight_at<DEG>(g.W, py, j);
    wz[j] = DIM == 3 ? weight_at<DEG>(g.W, pz, j) : T(j == 0 ? 1 : 0);
    if (BC) {
      const int cx = DEG * ccx + j, cy = DEG * ccy + j, cz = DEG * ccz + j;
      if (cx == 0 || cx == g.cdim[0] - 1) wx[j] = 0;
      if (cy == 0 || cy == g.cdim[1] - 1) wy[j] = 0;
      if (DIM == 3 && (cz == 0 || cz == g.cdim[2] - 1)) wz[j] = 0;
    }
  }
  const T *src = wc + g.coff + (i64)comp * g.cstride + DEG * ccx +
                 (i64)g.cdim[0] * (DEG * ccy + (i64)g.cdim[1] * (DEG * ccz));
  T s = 0;
#pragma unroll
  for (int jz = 0; jz < (DIM == 3 ? ND : 1); ++jz) {
    T r = 0;
#pragma unroll
    for (int jy = 0; jy < ND; ++jy) {
      const T *row = src + (i64)g.cdim[0] * (jy + (i64)g.cdim[1] * jz);
      T q = 0;
#pragma unroll
      for (int jx = 0; jx < ND; ++jx) q += wx[jx] * row[jx];
      r += wy[jy] * q;
    }
    s += wz[jz] * r;
  }
  T &out = xf[g.foff + (i64)comp * g.fstride + fx + (i64)g.fdim[0] * (fy + (i64)g.fdim[1] * fz)];
  out += s;
}

// Restriction r_c = P^T r_f: one block per run of CX coarse nodes along x at
// fixed (y, z) and component.  The fine rows of the (y, z) support with a
// non-zero weight are listed first (the same list for every lane: candidate
// rows tested by one thread each, compacted by wave ballots in candidate
// order, so the summation order is fixed); phase 1 then sums those rows into
// an LDS row, eight rows per round of requests; phase 2 applies each coarse
// node's x weights to the row.  One pass over the fine vector, no
// intermediate vectors.
template <typename T, int DIM, int DEG, bool BC, int CX>
__device__ __forceinline__ void restrict_block(const T *__restrict__ rf, T *__restrict__ rc, T *__restrict__ zc,
                                               const XferGeo<T> &g, int bx, int by, int bz) {
  constexpr int NC = 4 * DEG + 1;  // candidate fine rows per direction
  constexpr int NCAND = DIM == 3 ? NC * NC : NC;
  static_assert(NCAND <= 256, "one candidate per thread");
  constexpr int ROW = 2 * (CX - 1) + 4 * DEG + 1;
  constexpr int UNR = 8;
  __shared__ T tmp[ROW];
  __shared__ T s_w[NCAND];
  __shared__ i64 s_off[NCAND];
  __shared__ int s_cnt[4];
  const int cx0 = bx * CX;
  if (cx0 >= g.cdim[0] || by >= g.cdim[1]) return;  // whole block: beyond this field's lattice
  const int cy = by;
  const int nz = DIM == 3 ? g.cdim[2] : 1;
  const int comp = bz / nz;
  const int cz = bz - comp * nz;
  int fx_lo = 2 * cx0 - 2 * DEG;
  if (fx_lo < 0) fx_lo = 0;
  int fx_hi = 2 * (cx0 + CX - 1) + 2 * DEG;
  if (fx_hi > g.fdim[0] - 1) fx_hi = g.fdim[0] - 1;
  const T *src = rf + g.foff + (i64)comp * g.fstride;

  // weight of fine row f (along a direction) for coarse node c
  auto wrow = [&](int f, int c, int nf_cells, int fdim) -> T {
    if (f < 0 || f > fdim - 1) return T(0);
    if (BC && (f == 0 || f == fdim - 1)) return T(0);
    int cc, pos;
    fine_pos<DEG>(f, nf_cells, cc, pos);
    const int j = c - DEG * cc;
    if (j < 0 || j > DEG) return T(0);
    return weight_at<DEG>(g.W, pos, j);
  };

  // 0. list of the support rows with non-zero weight
  {
    const int t = (int)threadIdx.x;
    T w = 0;
    i64 off = 0;
    if (t < NCAND) {
      const int iy = t % NC, iz = t / NC;
      const int fy = 2 * cy - 2 * DEG + iy;
      w = wrow(fy, cy, g.ncell_f[1], g.fdim[1]);
      int fz = 0;
      if (DIM == 3) {
        fz = 2 * cz - 2 * DEG + iz;
        w *= wrow(fz, cz, g.ncell_f[2], g.fdim[2]);
      }
      off = (i64)g.fdim[0] * (fy + (i64)g.fdim[1] * fz);
    }
    const bool nzw = w != T(0);
    const unsigned long long m = __ballot(nzw);
    const int lane = t % 64, wave = t / 64;
    const int before = __popcll(m & ((1ull << lane) - 1ull));
    if (lane == 0) s_cnt[wave] = __popcll(m);
    __syncthreads();
    int base = 0;
    for (int v = 0; v < wave; ++v) base += s_cnt[v];
    if (nzw) {
      s_w[base + before] = w;
      s_off[base + before] = off;
    }
    __syncthreads();
  }
  const int nrow = s_cnt[0] + s_cnt[1] + s_cnt[2] + s_cnt[3];

  // 1. fine row
  for (int fx = fx_lo + (int)threadIdx.x; fx <= fx_hi; fx += 256) {
    const bool xbc = BC && (fx == 0 || fx == g.fdim[0] - 1);
    T s = 0;
    for (int r0 = 0; r0 < nrow; r0 += UNR) {
      T v[UNR], w[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int r = r0 + u < nrow ? r0 + u : r0;
        w[u] = r0 + u < nrow ? s_w[r] : T(0);
        v[u] = src[s_off[r] + fx];
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) s += w[u] * v[u];
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
      s += weight_at<DEG>(g.W, pos, j) * tmp[fx - fx_lo];
    }
  }
  const i64 ci = g.coff + (i64)comp * g.cstride + cx + (i64)g.cdim[0] * (cy + (i64)g.cdim[1] * cz);
  rc[ci] = s;
  if (zc != nullptr) zc[ci] = T(0);  // the coarse iterate starts at zero (Algorithm 1)
}

// Both fields of a level pair in one launch: blocks [0, nv) of the field
// dimension (y for the prolongation, z for the restriction) carry the
// velocity components (degree K, Dirichlet rows), the rest the pressure
// (degree K - 1); the grid's other extents are those of the larger field.
template <typename T, int DIM, int K>
__global__ void __launch_bounds__(256) k_prolong(const T *__restrict__ wc, T *__restrict__ xf, const XferGeo<T> gv,
                                                 const XferGeo<T> gp, int nv) {
  if ((int)blockIdx.y < nv) prolong_block<T, DIM, K, true>(wc, xf, gv, blockIdx.x, blockIdx.y);
  else prolong_block<T, DIM, K - 1, false>(wc, xf, gp, blockIdx.x, blockIdx.y - nv);
}

// zc (optional): a coarse vector set to zero on every entry written, in the
// same pass.
template <typename T, int DIM, int K, int CX>
__global__ void __launch_bounds__(256) k_restrict(const T *__restrict__ rf, T *__restrict__ rc, T *__restrict__ zc,
                                                  const XferGeo<T> gv, const XferGeo<T> gp, int nv) {
  if ((int)blockIdx.z < nv) restrict_block<T, DIM, K, true, CX>(rf, rc, zc, gv, blockIdx.x, blockIdx.y, blockIdx.z);
  else restrict_block<T, DIM, K - 1, false, CX>(rf, rc, zc, gp, blockIdx.x, blockIdx.y, blockIdx.z - nv);
}

// The two launches above as functors over a flat block index (packed
// launches, packed.hpp): gx (x gy) blocks per field plane as in their grids.
template <typename T, int DIM, int K>
struct LProlong {
  static constexpr int THREADS = 256;
  const T *wc;
  T *xf;
  XferGeo<T> gv, gp;
  int nv, gx;
  __device__ void run(int b, int) const {
    const int bx = b % gx, by = b / gx;
    if (by < nv) prolong_block<T, DIM, K, true>(wc, xf, gv, bx, by);
    else prolong_block<T, DIM, K - 1, false>(wc, xf, gp, bx, by - nv);
  }
};

template <typename T, int DIM, int K, int CX>
struct LRestrict {
  static constexpr int THREADS = 256;
  const T *rf;
  T *rc, *zc;
  XferGeo<T> gv, gp;
  int nv, gx, gy;
  __device__ void run(int b, int) const {
    const int bx = b % gx, r = b / gx, by = r % gy, bz = r / gy;
    if (bz < nv) restrict_block<T, DIM, K, true, CX>(rf, rc, zc, gv, bx, by, bz);
    else restrict_block<T, DIM, K - 1, false, CX>(rf, rc, zc, gp, bx, by, bz - nv);
  }
};

}  // namespace smg
