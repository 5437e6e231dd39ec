// Element-wise, reduction, transfer, diagonal and coarse-solve kernels.
#pragma once
#include "common.hpp"

namespace smg {

constexpr int VB = 256;  // threads per block of the element-wise kernels

inline unsigned grid_for(i64 n, int per_block = VB) {
  i64 g = (n + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > 1048576) g = 1048576;
  return (unsigned)g;
}

template <typename T>
__global__ void k_set(T *y, T v, i64 n) { SMG_GRID_LOOP(i, n) y[i] = v; }

template <typename TO, typename TI>
__global__ void k_copy(TO *y, const TI *x, i64 n) { SMG_GRID_LOOP(i, n) y[i] = (TO)x[i]; }

// y += a x
template <typename T>
__global__ void k_axpy(T *y, T a, const T *x, i64 n) { SMG_GRID_LOOP(i, n) y[i] += a * x[i]; }

// y = x + a z (TO output, any input types)
template <typename TO, typename TI>
__global__ void k_add_scaled(TO *y, const TI *x, TO a, const TO *z, i64 n) {
  SMG_GRID_LOOP(i, n) y[i] = (TO)x[i] + a * z[i];
}

// out = base + s * dinv * r   (Chebyshev of degree 0: damped Jacobi)
template <typename T>
__global__ void k_jacobi(T *out, const T *base, T s, const T *dinv, const T *r, i64 n) {
  SMG_GRID_LOOP(i, n) out[i] = (base ? base[i] : T(0)) + s * dinv[i] * r[i];
}

// p += dp, dp = s * dinv * r
template <typename T>
__global__ void k_jacobi_update(T *p, T *dp, T s, const T *dinv, const T *r, i64 n) {
  SMG_GRID_LOOP(i, n) {
    const T d = s * dinv[i] * r[i];
    dp[i] = d;
    p[i] += d;
  }
}

template <typename TO>
__global__ void k_reciprocal(TO *y, const double *x, i64 n) { SMG_GRID_LOOP(i, n) y[i] = (TO)(1.0 / x[i]); }

// ---------------------------------------------------------------------------
// deterministic reductions: fixed partition into RB blocks, per-block tree
// sums (wave64 shuffles, then LDS), then one block sums the partials in order.
// ---------------------------------------------------------------------------
constexpr int RB = 512;   // number of partial sums

template <typename T>
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double sm[VB / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sm[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int w = 0; w < VB / 64; ++w) s += sm[w];
  }
  __syncthreads();
  return s;
}

// partial[b * nv + j] = sum over the chunk of block b of V_j[i] * w[i]
// (V_j = V + j * ldv), for j < nv; FP64 accumulation.
template <typename T>
__global__ void __launch_bounds__(VB) k_multidot_partial(const T *V, i64 ldv, int nv, const T *w, i64 n, double *partial) {
  const i64 chunk = (n + gridDim.x - 1) / gridDim.x;
  const i64 lo = (i64)blockIdx.x * chunk;
  const i64 hi = lo + chunk < n ? lo + chunk : n;
  for (int j = 0; j < nv; ++j) {
    const T *v = V + (i64)j * ldv;
    double s = 0.0;
    for (i64 i = lo + threadIdx.x; i < hi; i += VB) s += (double)v[i] * (double)w[i];
    s = block_sum<T>(s);
    if (threadIdx.x == 0) partial[(i64)blockIdx.x * nv + j] = s;
  }
}

// out[j] = sum_b partial[b * nv + j]: one block per j, fixed-order tree sum.
static __global__ void __launch_bounds__(VB) k_partial_finish(const double *partial, int nblocks, int nv, double *out) {
  const int j = blockIdx.x;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += VB) s += partial[(i64)b * nv + j];
  s = block_sum<double>(s);
  if (threadIdx.x == 0) out[j] = s;
}

// w *= 1 / sqrt(s2[0])  (normalisation by a norm that stays on the device)
template <typename T>
__global__ void k_scale_inv_sqrt(T *w, const double *s2, i64 n) {
  const double v = s2[0];
  const double f = v > 0.0 ? 1.0 / sqrt(v) : 0.0;
  SMG_GRID_LOOP(i, n) w[i] = (T)((double)w[i] * f);
}

// w -= sum_j h[j] V_j  (h on the device)
template <typename T>
__global__ void k_multi_axpy(T *w, const T *V, i64 ldv, int nv, const double *h, double sign, i64 n) {
  SMG_GRID_LOOP(i, n) {
    double s = 0.0;
    for (int j = 0; j < nv; ++j) s += h[j] * (double)V[(i64)j * ldv + i];
    w[i] = (T)((double)w[i] + sign * s);
  }
}

// ---------------------------------------------------------------------------
// transfers (Sec. 3.2): canonical injection P per field, R = P^T
// ---------------------------------------------------------------------------
struct TransferField {
  int deg;              // polynomial degree of the field (k or k-1)
  int cdim[3], fdim[3]; // lattice extents, coarse and fine
  int ncell_f[3];       // fine cells per direction
  i64 coff, foff;       // offsets of the field in the coarse / fine vectors
  int ncomp;            // consecutive components (d for velocity, 1 for pressure)
  i64 cstride, fstride; // distance between components
  int bc;               // 1: Dirichlet field (velocity)
};

struct TransferTables {
  double W[2][7 * 4];   // W[field][f * (deg+1) + j], f = 0..2deg; field 0 = velocity, 1 = pressure
};

// coarse cell index of fine lattice node f and its position 0..2deg in it
__device__ __forceinline__ void fine_in_coarse(int f, int deg, int nf_cells, int &cc, int &pos) {
  int cf = f / deg;
  if (cf > nf_cells - 1) cf = nf_cells - 1;
  cc = cf >> 1;
  pos = f - 2 * deg * cc;
}

// x_f += P w_c for every field; one thread per fine node and component.
template <typename T, int DIM>
__global__ void k_prolongate_add(const T *wc, T *xf, TransferField fv, TransferField fp, TransferTables tab, i64 n_fine_v, i64 n_fine_p) {
  const i64 total = n_fine_v * fv.ncomp + n_fine_p;
  SMG_GRID_LOOP(gi, total) {
    const bool isv = gi < n_fine_v * fv.ncomp;
    const TransferField &F = isv ? fv : fp;
    const double *W = isv ? tab.W[0] : tab.W[1];
    i64 node, comp = 0;
    if (isv) { comp = gi / n_fine_v; node = gi - comp * n_fine_v; } else { node = gi - n_fine_v * fv.ncomp; }
    int fi[3] = {0, 0, 0};
    i64 r = node;
    for (int a = 0; a < DIM; ++a) { fi[a] = (int)(r % F.fdim[a]); r /= F.fdim[a]; }
    bool fbc = false;
    if (F.bc)
      for (int a = 0; a < DIM; ++a) fbc |= (fi[a] == 0 || fi[a] == F.fdim[a] - 1);
    if (fbc) continue;
    int cc[3], pos[3];
    for (int a = 0; a < DIM; ++a) fine_in_coarse(fi[a], F.deg, F.ncell_f[a], cc[a], pos[a]);
    const int nd = F.deg + 1;
    double s = 0.0;
    const int jz_n = DIM == 3 ? nd : 1;
    for (int jz = 0; jz < jz_n; ++jz) {
      const double wz = DIM == 3 ? W[pos[2] * nd + jz] : 1.0;
      const int cz = DIM == 3 ? F.deg * cc[2] + jz : 0;
      if (wz == 0.0) continue;
      for (int jy = 0; jy < nd; ++jy) {
        const double wy = W[pos[1] * nd + jy];
        if (wy == 0.0) continue;
        const int cy = F.deg * cc[1] + jy;
        for (int jx = 0; jx < nd; ++jx) {
          const double wx = W[pos[0] * nd + jx];
          if (wx == 0.0) continue;
          const int cx = F.deg * cc[0] + jx;
          bool cbc = false;
          if (F.bc)
            cbc = cx == 0 || cx == F.cdim[0] - 1 || cy == 0 || cy == F.cdim[1] - 1 ||
                  (DIM == 3 && (cz == 0 || cz == F.cdim[2] - 1));
          if (cbc) continue;
          const i64 ci = F.coff + comp * F.cstride + cx + (i64)F.cdim[0] * (cy + (i64)F.cdim[1] * cz);
          s += wx * wy * wz * (double)wc[ci];
        }
      }
    }
    const i64 fidx = F.foff + comp * F.fstride + node;
    xf[fidx] = (T)((double)xf[fidx] + s);
  }
}

// One direction of R = P^T: in has fine extent along `dir`, out coarse
// extent; other directions as given by in_dim/out_dim.  `mask_in` zeroes
// Dirichlet inputs (first pass), `mask_out` zeroes Dirichlet outputs (last pass),
// both judged on the full fine/coarse lattices fdim/cdim.
template <typename T>
__global__ void k_restrict_pass(const T *in, T *out, int dir, int deg, int n_cells_f,
                                int in_d0, int in_d1, int in_d2, int out_d0, int out_d1, int out_d2,
                                int ncomp, i64 in_cstride, i64 out_cstride, i64 in_off, i64 out_off,
                                TransferTables tab, int field, int mask_in, int mask_out,
                                int f0, int f1, int f2, int c0, int c1, int c2, int dim) {
  const i64 per = (i64)out_d0 * out_d1 * out_d2;
  const i64 total = per * ncomp;
  const double *W = tab.W[field];
  const int nd = deg + 1;
  const int in_dims[3] = {in_d0, in_d1, in_d2};
  const int fd[3] = {f0, f1, f2}, cd[3] = {c0, c1, c2};
  SMG_GRID_LOOP(gi, total) {
    const i64 comp = gi / per;
    i64 r = gi - comp * per;
    int o[3];
    o[0] = (int)(r % out_d0); r /= out_d0;
    o[1] = (int)(r % out_d1); r /= out_d1;
    o[2] = (int)r;
    // coarse index J along dir
    const int J = o[dir];
    bool obc = false;
    if (mask_out) {
      for (int a = 0; a < dim; ++a) obc |= (o[a] == 0 || o[a] == cd[a] - 1);
    }
    double s = 0.0;
    if (!obc) {
      int flo = 2 * J - 2 * deg, fhi = 2 * J + 2 * deg;
      if (flo < 0) flo = 0;
      if (fhi > in_dims[dir] - 1) fhi = in_dims[dir] - 1;
      for (int f = flo; f <= fhi; ++f) {
        int cc, pos;
        fine_in_coarse(f, deg, n_cells_f, cc, pos);
        const int j = J - deg * cc;
        if (j < 0 || j > deg) continue;
        const double w = W[pos * nd + j];
        if (w == 0.0) continue;
        int ii[3] = {o[0], o[1], o[2]};
        ii[dir] = f;
        if (mask_in) {
          bool ibc = false;
          for (int a = 0; a < dim; ++a) ibc |= (ii[a] == 0 || ii[a] == fd[a] - 1);
          if (ibc) continue;
        }
        const i64 idx = in_off + comp * in_cstride + ii[0] + (i64)in_dims[0] * (ii[1] + (i64)in_dims[1] * ii[2]);
        s += w * (double)in[idx];
      }
    }
    out[out_off + comp * out_cstride + o[0] + (i64)out_d0 * (o[1] + (i64)out_d1 * o[2])] = (T)s;
  }
}

// ---------------------------------------------------------------------------
// coarse solve: x0 = Kinv[0:N0, 0:N0] b0 (border column multiplies zero),
// FP64 arithmetic for any T; one wave per row.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(VB) k_coarse_gemv(const double *Kinv, i64 ld, int n0, const T *b, T *x) {
  const int row = blockIdx.x * (VB / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n0) return;
  double s = 0.0;
  for (int c = lane; c < n0; c += 64) s += Kinv[(i64)row * ld + c] * (double)b[c];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) x[row] = (T)s;
}

// p -= (w . p) / (w . 1) with w = M_p 1 given, for pressure mean removal
static __global__ void k_subtract_scalar(double *p, const double *scal, double denom, i64 n) {
  const double m = scal[0] / denom;
  SMG_GRID_LOOP(i, n) p[i] -= m;
}

}  // namespace smg
