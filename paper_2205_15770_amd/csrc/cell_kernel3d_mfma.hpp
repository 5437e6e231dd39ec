// Matrix-core application of the velocity block A of the Taylor-Hood
// operator on axis-aligned box cells in 3D, Q2 (Sec. 3.1: A u =
// sum_tau P_tau A_tau P_tau^T u, evaluated cell by cell).  A variant of the
// FP32 Chebyshev steps for A, selected by level size (off by default: at
// 64^3 it takes 68 us against 54 us for the column sweep).
//
// On a box level all cells have the widths (h_x, h_y, h_z), so every cell has
// the same 27 x 27 matrix per velocity component,
//   A_tau = mu (sKx Kr(x)Mr(x)Mr + sKy Mr(x)Kr(x)Mr + sKz Mr(x)Mr(x)Kr)
//           + gamma rho sM Mr(x)Mr(x)Mr,
// (per-cell viscosity with gamma = 0: A_tau = mu_tau A_1, and mu_tau scales
// the cell's input).  The cell products of 32 cells are then one dense
// product  Y (32 cells x 27 nodes) = U (32 x 27) A_tau^T,  14 matrix-core
// instructions v_mfma_f32_32x32x2_f32 (inner dimension 27 padded to 28, the
// 27 output nodes to 32 columns).  Dense is 729 multiply-adds per cell and
// component against 567 for the sum-factorised passes, at twice the FP32
// rate the vector ALU issues without packed FP32.
//
// Work decomposition: one wave (its own workgroup) per (tile of 17 x 9 cell
// columns, z chunk, velocity component).  The tile owns 16 x 8 columns:
// column 0 and row 0 are halo columns whose cells are computed only for the
// sums on the tile's low faces.  The wave sweeps its chunk layer by layer
// (the layer below the chunk is a halo layer).  Per layer:
//   * LDS `s_in` holds the layer's three input node planes, 35 x 19 nodes
//     each (masked: zero outside the mesh and, for ZERO_BC, on Dirichlet
//     nodes); the matrix-core A operand is read from it (lane l: cell l % 32
//     of the batch, input node 2 s + l / 32) and the B operand is A_tau, held
//     in 14 registers;
//   * the 16 results per lane (one output node of 16 cells) are written to a
//     per-cell staging area `s_stg` (plain stores, no two lanes on one slot);
//   * every owned node sums the staged results of the (up to) four cells
//     around it in a fixed order (bit-reproducible, no atomics), plus the
//     carry from the layer below; planes 0 and 1 are then complete and are
//     written once through the epilogue functor (Dirichlet rows as in the
//     other box kernels); plane 2's partial sums stay in registers as the
//     next layer's carry.
// Measured at 64^3 (counters): the matrix core is busy a sixth of the
// launch; at one wave per SIMD (the epilogue's in-flight loads need the
// registers, the planes and staging 31 KB of LDS) the layer's loads,
// gathers and stores run serially with its products.
#pragma once
#include <type_traits>
#include "cell_kernel3d.hpp"

namespace smg {
namespace mf3 {
constexpr int CX = 17, CY = 9;                   // computed cell columns per layer
constexpr int OX = CX - 1, OY = CY - 1;          // owned columns per tile
constexpr int PX = 2 * CX + 1, PY = 2 * CY + 1;  // node plane of the patch: 35 x 19
constexpr int PL = PX * PY;                      // 665 nodes
constexpr int NCELL = CX * CY;                   // 153 cells per layer
constexpr int NBLK = (NCELL + 31) / 32;          // 5 batches of 32 cells
constexpr int LPP = (PL + 63) / 64;              // 11 nodes per lane and plane
constexpr int SST = 33;                          // staging row stride (27 nodes + 5 padding + 1)
// staging rows: one per cell of the batches (160), plus a margin that keeps
// the four reads of a node's gather in bounds where the node has fewer cells
constexpr int NROW = 32 * NBLK + CX + 2;
constexpr int NE = (PY - 1) / 2;                 // 9 rows of owned nodes per lane and plane

// LDS offset of local node k = kx + 3 ky + 9 kz of a cell from the cell's
// first node (k = 27, the padding of the inner dimension, reads node 26: a
// finite value times a zero matrix entry)
__host__ __device__ constexpr int node_off(int k) {
  return k >= 27 ? node_off(26) : (k % 3) + PX * ((k / 3) % 3) + PL * (k / 9);
}
// LDS offset of the first node of cell c of the layer (c = i + 17 j)
__host__ __device__ constexpr int cell_base(int c) { return 2 * (c % CX) + 2 * PX * (c / CX); }
}  // namespace mf3

// Launch shape (host): 17 x 9 column tiles owning 16 x 8, three components,
// the z extent cut into chunks of >= 2 cells so that the launch has about
// `waves` waves when the level is large enough.  Sets g.tiles and returns the
// number of blocks (one wave each).
template <typename T>
inline int mfma3d_chunks(Geo3<T> &g, int waves) {
  g.tiles[0] = (g.n[0] + mf3::OX - 1) / mf3::OX;
  g.tiles[1] = (g.n[1] + mf3::OY - 1) / mf3::OY;
  const int cols = g.tiles[0] * g.tiles[1] * 3;
  int nzc = (waves + cols - 1) / cols;
  const int zmax = (g.n[2] + 1) / 2;
  nzc = nzc < 1 ? 1 : (nzc > zmax ? zmax : nzc);
  const int zlen = (g.n[2] + nzc - 1) / nzc;
  g.tiles[2] = (g.n[2] + zlen - 1) / zlen;
  return cols * g.tiles[2];
}

// Block b (after the XCD map) -> component, tiles and chunk; false for an
// empty chunk.
struct Mfma3DTile {
  int comp, tx, ty, z_lo, z_hi, z_start;
};
template <typename T>
__host__ __device__ inline bool mfma3d_decode(const Geo3<T> &g, int b, Mfma3DTile &t) {
  t.comp = b % 3;
  int rest = b / 3;
  t.tx = rest % g.tiles[0];
  rest /= g.tiles[0];
  const int zc = rest % g.tiles[2];
  t.ty = rest / g.tiles[2];
  const int zlen = (g.n[2] + g.tiles[2] - 1) / g.tiles[2];
  t.z_lo = zc * zlen;
  t.z_hi = t.z_lo + zlen < g.n[2] ? t.z_lo + zlen : g.n[2];
  t.z_start = t.z_lo > 0 ? t.z_lo - 1 : 0;
  return t.z_lo < t.z_hi;
}

// Per-lane addressing of mfma3d_kernel: the patch-plane loads, the LDS
// indices of the matrix-core operands, the staging slots and the node
// gathers, and the owned output nodes.  Host and device: the kernel and the
// host replay of its accesses use this same arithmetic.
struct Mfma3DLane {
  int lane, hi, n;
  int gx0, gy0;          // global node of patch node (0, 0)
  int vd0, vd1, vd2;     // velocity lattice extents
  int ox_hi, oy_hi;      // owned nodes: x < ox_hi, y < oy_hi (from patch node (2, 2))
  uint32_t plane_bytes;  // bytes of one lattice plane (one component)
  uint32_t comp_base;    // byte offset of the tile's velocity component
  // gather, x part: node x = 2 + n is node kx0 (1 or 2) of cell i0 and, for
  // even x inside the computed cells (xe), node 0 of cell i0 + 1
  int xp, xph;
  bool xe;
  bool xok, xdir;        // x = gx0 + 2 + n owned / on the boundary
  uint32_t lane_off;     // byte offset of the lane's (clamped) lattice column x
  __host__ __device__ Mfma3DLane(const Geo3<float> &g, const Mfma3DTile &t, int lane_) {
    using namespace mf3;
    lane = lane_;
    hi = lane >> 5;
    n = lane & 31;
    vd0 = g.vd[0];
    vd1 = g.vd[1];
    vd2 = g.vd[2];
    plane_bytes = 4u * (uint32_t)vd0 * (uint32_t)vd1;
    comp_base = (uint32_t)t.comp * g.nv_bytes;
    gx0 = 2 * (OX * t.tx - 1);
    gy0 = 2 * (OY * t.ty - 1);
    ox_hi = t.tx == g.tiles[0] - 1 ? vd0 : gx0 + 2 + 2 * OX;
    oy_hi = t.ty == g.tiles[1] - 1 ? vd1 : gy0 + 2 + 2 * OY;
    const int i0 = (1 + n) >> 1, kx0 = 2 + n - 2 * i0;
    xe = kx0 == 2 && i0 + 1 < CX;
    const int xgl = gx0 + 2 + n;
    xok = xgl < ox_hi;
    xdir = xgl == 0 || xgl == vd0 - 1;
    lane_off = comp_base + 4u * (uint32_t)(xgl < vd0 ? xgl : vd0 - 1);
    // staging offset of (cell i0 + 17 j0, node kx0 + 3 ky0): rows y = 2 + 2 j
    // (hi = 0: j0 = j, ky0 = 2) and y = 3 + 2 j (hi = 1: j0 = j + 1, ky0 = 1)
    // differ by 17 SST - 3
    xp = i0 * SST + kx0;
    xph = xp + hi * (CX * SST - 3);
  }
  // patch-plane node q = lane + 64 j (x fastest over 35): byte offset of its
  // lattice column (clamped into the lattice), inside / on the x-y boundary
  __host__ __device__ uint32_t plane_node(int j, bool &inside, bool &bnd) const {
    using namespace mf3;
    const int q = lane + 64 * j;
    const int x = q % PX, y = q / PX;
    const int gx = gx0 + x, gy = gy0 + y;
    inside = q < PL && gx >= 0 && gx < vd0 && gy >= 0 && gy < vd1;
    bnd = gx == 0 || gx == vd0 - 1 || gy == 0 || gy == vd1 - 1;
    const int cgx = gx < 0 ? 0 : (gx >= vd0 ? vd0 - 1 : gx);
    const int cgy = gy < 0 ? 0 : (gy >= vd1 ? vd1 - 1 : gy);
    return 4u * ((uint32_t)cgx + (uint32_t)vd0 * (uint32_t)cgy);
  }
  // LDS index (input planes) of the A operand of batch b, step s: input node
  // 2 s + hi of cell n of the batch (padding rows read cell 0)
  __host__ __device__ int a_index(int b, int s) const {
    using namespace mf3;
    const int c = 32 * b + n;
    return cell_base(c < NCELL ? c : 0) + node_off(2 * s) + hi * (node_off(2 * s + 1) - node_off(2 * s));
  }
  // LDS staging index of result register r of batch b: node n of the cell
  // in row 8 (r / 4) + 4 hi + r % 4 of the batch (padding rows and columns
  // land in unused slots)
  __host__ __device__ int stg_index(int b, int r) const {
    using namespace mf3;
    return n + 4 * SST * hi + SST * (32 * b + 8 * (r / 4) + (r % 4));
  }
  // owned-node slot j < 9 of a plane: node x = 2 + n, y = 2 + 2 j + hi of
  // the patch (the last row pair has no hi = 1 node: those lanes own
  // nothing there and read the hi = 0 node's staging and input).  The four
  // staging indices of its (up to) four cells in z plane kz and which of
  // them contribute, in summation order.
  __host__ __device__ void gather_index(int j, int kz, int (&a)[4], bool (&use)[4]) const {
    using namespace mf3;
    const int a00 = (j < NE - 1 ? xph : xp) + CX * j * SST + 6 + 9 * kz;
    const bool ye = hi == 0 && j + 1 < CY;
    a[0] = a00;
    a[1] = a00 + SST - 2;
    a[2] = a00 + CX * SST - 6;
    a[3] = a00 + (CX + 1) * SST - 8;
    use[0] = true;
    use[1] = xe;
    use[2] = ye;
    use[3] = xe && ye;
  }
  // LDS index (input planes) of slot j's node in z plane zp
  __host__ __device__ int vin_index(int zp, int j) const {
    using namespace mf3;
    return zp * PL + (2 + 2 * j + (j < NE - 1 ? hi : 0)) * PX + 2 + n;
  }
  // slot j < 9: global address in plane byte offset zoff (clamped into the
  // lattice), owned, on the x-y boundary
  __host__ __device__ void slot(int j, uint32_t zoff, BOff &gi, bool &ok, bool &dir) const {
    using namespace mf3;
    const int gy = gy0 + 2 + 2 * j + hi;
    ok = xok && gy < oy_hi && !(j == NE - 1 && hi);
    dir = xdir || gy == 0 || gy == vd1 - 1;
    gi = BOff{lane_off + zoff + 4u * (uint32_t)vd0 * (uint32_t)(gy < vd1 ? gy : vd1 - 1), 0};
  }
  // slot 9: the patch column x = 34 (the domain's high x face, last tile
  // only), y = 2 + lane: always a Dirichlet row
  __host__ __device__ void slot9(uint32_t zoff, BOff &gi, bool &ok) const {
    using namespace mf3;
    const int gx = gx0 + PX - 1, gy = gy0 + 2 + lane;
    ok = lane < PY - 2 && gx < ox_hi && gy < oy_hi;
    gi = BOff{comp_base + zoff + 4u * ((uint32_t)(gx < vd0 ? gx : vd0 - 1) +
                                       (uint32_t)vd0 * (uint32_t)(gy < vd1 ? gy : vd1 - 1)),
              0};
  }
};

typedef float mf3_v16 __attribute__((ext_vector_type(16)));

// Entry (n, k) of the cell matrix, n = output node (its 1D rows of Kr and Mr
// per direction given), k = input node (compile time).
template <int KK>
__device__ __forceinline__ float mf3_entry(const float (&Kx)[3], const float (&Mx)[3], const float (&Ky)[3],
                                           const float (&My)[3], const float (&Kz)[3], const float (&Mz)[3],
                                           float ax, float bx, float cy, float cz) {
  if constexpr (KK >= 27) {
    return 0.f;
  } else {
    constexpr int kx = KK % 3, ky = (KK / 3) % 3, kz = KK / 9;
    const float X = ax * Kx[kx] + bx * Mx[kx];
    return Mz[kz] * (X * My[ky] + cy * Mx[kx] * Ky[ky]) + cz * Kz[kz] * Mx[kx] * My[ky];
  }
}

template <int S>
__device__ __forceinline__ void mf3_fill_b(float (&Bop)[14], int hi, bool nvalid, const float (&Kx)[3],
                                           const float (&Mx)[3], const float (&Ky)[3], const float (&My)[3],
                                           const float (&Kz)[3], const float (&Mz)[3], float ax, float bx, float cy,
                                           float cz) {
  if constexpr (S < 14) {
    const float e0 = mf3_entry<2 * S>(Kx, Mx, Ky, My, Kz, Mz, ax, bx, cy, cz);
    const float e1 = mf3_entry<2 * S + 1>(Kx, Mx, Ky, My, Kz, Mz, ax, bx, cy, cz);
    Bop[S] = nvalid ? (hi ? e1 : e0) : 0.f;
    mf3_fill_b<S + 1>(Bop, hi, nvalid, Kx, Mx, Ky, My, Kz, Mz, ax, bx, cy, cz);
  }
}

__device__ __forceinline__ float mf3_sel3(int i, float a, float b, float c) { return i == 0 ? a : (i == 1 ? b : c); }

// Op: an epilogue functor with velocity input and output only (the A block).
// Requires K = 2 and FP32; MUC: per-cell viscosity g.mu_cell (then gamma rho
// must be 0), else the uniform g.mu.
template <class Op, bool MUC>
__global__ void __launch_bounds__(64) mfma3d_kernel(const Geo3<float> g, const Op op) {
  using namespace mf3;
  __shared__ float s_in[3 * PL];
  __shared__ float s_stg[NROW * SST];
  Mfma3DTile t;
  if (!mfma3d_decode(g, xcd_contiguous_tile(blockIdx.x, gridDim.x), t)) return;  // whole wave
  const int lane = threadIdx.x;
  const Mfma3DLane L(g, t, lane);
  const int hi = L.hi, n = L.n;
  const int vd2 = L.vd2;
  const uint32_t plane_bytes = L.plane_bytes, comp_base = L.comp_base;
  const int cx0 = OX * t.tx - 1, cy0 = OY * t.ty - 1;  // first computed cell column

  // ---- per-lane node addressing of the plane loads: node q = lane + 64 j
  uint32_t off_xy[LPP];
  uint32_t in_bits = 0, bnd_bits = 0;
#pragma unroll
  for (int j = 0; j < LPP; ++j) {
    bool inside, bnd;
    off_xy[j] = L.plane_node(j, inside, bnd);
    in_bits |= (inside ? 1u : 0u) << j;
    bnd_bits |= (bnd ? 1u : 0u) << j;
  }
  auto load_plane = [&](int gz, float (&v)[LPP]) {
    const uint32_t base = comp_base + (uint32_t)gz * plane_bytes;
#pragma unroll
    for (int j = 0; j < LPP; ++j) v[j] = op.load_u(BOff{base + off_xy[j], 0});
  };
  auto store_plane = [&](int gz, int slot, float (&v)[LPP]) {
    const bool zb = gz == 0 || gz == vd2 - 1;
#pragma unroll
    for (int j = 0; j < LPP; ++j) {
      const bool inside = (in_bits >> j) & 1u;
      const bool bnd = ((bnd_bits >> j) & 1u) | zb;
      const bool keep = inside & !(Op::ZERO_BC & bnd);
      const int q = lane + 64 * j;
      if (q < PL) s_in[slot * PL + q] = keep ? v[j] : 0.f;
    }
  };

  // ---- B operand: the cell matrix, B[k][n] = A_tau[n][k], k = 2 s + hi
  float Bop[14];
  {
    constexpr cfe::TabT<2, float> R = cfe::make_tab_t<2, float>();
    const float mu = MUC ? 1.f : g.mu;
    const float ax = mu * g.sKx, bx = g.gr * g.sM, cy = mu * g.sKy, cz = cy * g.rz;
    const int nn = n < 27 ? n : 26;
    const int nx = nn % 3, ny = (nn / 3) % 3, nz = nn / 9;
    float Kx[3], Mx[3], Ky[3], My[3], Kz[3], Mz[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Kx[i] = mf3_sel3(nx, R.Kr[0][i], R.Kr[1][i], R.Kr[2][i]);
      Mx[i] = mf3_sel3(nx, R.Mr[0][i], R.Mr[1][i], R.Mr[2][i]);
      Ky[i] = mf3_sel3(ny, R.Kr[0][i], R.Kr[1][i], R.Kr[2][i]);
      My[i] = mf3_sel3(ny, R.Mr[0][i], R.Mr[1][i], R.Mr[2][i]);
      Kz[i] = mf3_sel3(nz, R.Kr[0][i], R.Kr[1][i], R.Kr[2][i]);
      Mz[i] = mf3_sel3(nz, R.Mr[0][i], R.Mr[1][i], R.Mr[2][i]);
    }
    mf3_fill_b<0>(Bop, hi, n < 27, Kx, Mx, Ky, My, Kz, Mz, ax, bx, cy, cz);
  }
  // ---- first layer: three input planes
  {
    float v0[LPP], v1[LPP], v2[LPP];
    load_plane(2 * t.z_start, v0);
    load_plane(2 * t.z_start + 1, v1);
    load_plane(2 * t.z_start + 2, v2);
    store_plane(2 * t.z_start, 0, v0);
    store_plane(2 * t.z_start + 1, 1, v1);
    store_plane(2 * t.z_start + 2, 2, v2);
  }
  __syncthreads();

  // A node's sum is formed from the staged results of the (up to) four
  // cells around it in a fixed order; the z = 2 plane's partial sums are
  // carried in registers to the next layer's z = 0 plane (the same nodes,
  // the same lanes).
  auto gather = [&](int j, int kz) {
    int a[4];
    bool use[4];
    L.gather_index(j, kz, a, use);
    const float v00 = s_stg[a[0]], v10 = s_stg[a[1]], v01 = s_stg[a[2]], v11 = s_stg[a[3]];
    float sum = v00;
    sum += use[1] ? v10 : 0.f;
    sum += use[2] ? v01 : 0.f;
    sum += use[3] ? v11 : 0.f;
    return sum;
  };
  // the functor's inputs and the unmasked value (the Dirichlet rows' result)
  // of the ten owned-node slots of a plane
  auto fetch_plane = [&](uint32_t zoff, typename Op::Pre (&pre)[NE + 1], float (&rw)[NE + 1]) {
#pragma unroll
    for (int j = 0; j <= NE; ++j) {
      BOff gi;
      bool ok, dir;
      if (j < NE) L.slot(j, zoff, gi, ok, dir);
      else L.slot9(zoff, gi, ok);
      pre[j] = op.fetch_u(gi);
      rw[j] = op.load_u(gi);
    }
  };
  auto store_plane_out = [&](uint32_t zoff, bool zb, int zp, const float (&sum)[NE],
                             const typename Op::Pre (&pre)[NE + 1], const float (&rw)[NE + 1]) {
#pragma unroll
    for (int j = 0; j < NE; ++j) {
      BOff gi;
      bool ok, dir;
      L.slot(j, zoff, gi, ok, dir);
      dir |= zb;
      const float vin = s_in[L.vin_index(zp, j)];
      // Dirichlet rows: the functor gets the unmasked input as both the
      // operator result and the input (identity row of A)
      if (ok) op.store_u(gi, dir ? rw[j] : sum[j], dir ? rw[j] : vin, dir, pre[j]);
    }
    BOff gi;
    bool ok;
    L.slot9(zoff, gi, ok);
    if (ok) op.store_u(gi, rw[NE], rw[NE], true, pre[NE]);
  };

  float carry[NE];
#pragma unroll
  for (int j = 0; j < NE; ++j) carry[j] = 0.f;

  for (int cl = t.z_start; cl < t.z_hi; ++cl) {
    const bool more = cl + 1 < t.z_hi;
    const bool own = cl >= t.z_lo;
    const uint32_t z0 = (uint32_t)(2 * cl) * plane_bytes;  // node plane 2 cl
    // per-cell viscosity of the batch rows (A operand scale; 0 for padding)
    float sc[NBLK];
#pragma unroll
    for (int b = 0; b < NBLK; ++b) {
      const int c = 32 * b + n;
      float m = 1.f;
      if constexpr (MUC) {
        int cx = cx0 + c % CX, cy = cy0 + c / CX;
        cx = cx < 0 ? 0 : (cx >= g.n[0] ? g.n[0] - 1 : cx);
        cy = cy < 0 ? 0 : (cy >= g.n[1] ? g.n[1] - 1 : cy);
        m = g.mu_cell[(uint32_t)cx + (uint32_t)g.n[0] * ((uint32_t)cy + (uint32_t)g.n[1] * (uint32_t)cl)];
      }
      sc[b] = c < NCELL ? m : 0.f;
    }
    // plane 0's epilogue inputs, in flight during the products
    typename Op::Pre pre0[NE + 1];
    float rw0[NE + 1];
    if (own) fetch_plane(z0, pre0, rw0);

    // ---- cell products, 32 cells per batch, results staged per cell
#pragma unroll
    for (int b = 0; b < NBLK; ++b) {
      float a[14];
#pragma unroll
      for (int s = 0; s < 14; ++s) {
        a[s] = s_in[L.a_index(b, s)];
        if (MUC || 32 * b + 31 >= NCELL) a[s] *= sc[b];
      }
      mf3_v16 acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 14; ++s) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s], Bop[s], acc, 0, 0, 0);
#pragma unroll
      for (int r = 0; r < 16; ++r) s_stg[L.stg_index(b, r)] = acc[r];
    }
    __syncthreads();

    // ---- plane 1's epilogue inputs and the next layer's input planes
    // (on the chunk's last layer the plane loads repeat valid planes and
    // are not used: unconditional loads), in flight during the gathers
    typename Op::Pre pre1[NE + 1];
    float rw1[NE + 1];
    if (own) fetch_plane(z0 + plane_bytes, pre1, rw1);
    float pf1[LPP], pf2[LPP];
    load_plane(more ? 2 * cl + 3 : 2 * cl + 1, pf1);
    load_plane(more ? 2 * cl + 4 : 2 * cl + 2, pf2);
    float sum0[NE], sum1[NE];
#pragma unroll
    for (int j = 0; j < NE; ++j) {
      sum0[j] = carry[j] + gather(j, 0);
      sum1[j] = gather(j, 1);
      carry[j] = gather(j, 2);
    }
    if (own) {
      store_plane_out(z0, 2 * cl == 0, 0, sum0, pre0, rw0);
      store_plane_out(z0 + plane_bytes, false, 1, sum1, pre1, rw1);
      if (cl == g.n[2] - 1) {
        // the top plane of the mesh: Dirichlet rows
        typename Op::Pre pre2[NE + 1];
        float rw2[NE + 1];
        fetch_plane(z0 + 2 * plane_bytes, pre2, rw2);
        float dummy[NE];
#pragma unroll
        for (int j = 0; j < NE; ++j) dummy[j] = 0.f;
        store_plane_out(z0 + 2 * plane_bytes, true, 2, dummy, pre2, rw2);
      }
    }
    if (!more) break;
    __syncthreads();
    // next layer: input plane 2 -> plane 0, planes 1 and 2 from the loads
#pragma unroll
    for (int j = 0; j < LPP; ++j) {
      const int q = lane + 64 * j;
      if (q < PL) s_in[q] = s_in[2 * PL + q];
    }
    store_plane(2 * cl + 3, 1, pf1);
    store_plane(2 * cl + 4, 2, pf2);
    __syncthreads();
  }
}

}  // namespace smg
