// Shared device-side definitions of the multigrid library (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace smg {

typedef int64_t i64;

#define SMG_GRID_LOOP(i, n) \
  for (i64 i = (i64)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (i64)gridDim.x * blockDim.x)

// Per-direction 1D cell matrices scaled to the cell width h of a level:
//   Kv = (1/h) int l_i' l_j'   Mv = h int l_i l_j       (velocity)
//   G  = int psi_i l_j'        N  = h int psi_i l_j     (pressure x velocity)
//   Mp = h int psi_i psi_j                               (pressure)
template <typename T, int K>
struct Coef1D {
  T Kv[K + 1][K + 1];
  T Mv[K + 1][K + 1];
  T G[K][K + 1];
  T N[K][K + 1];
  T Mp[K][K];
};

// Geometry and coefficients of one level for the cell kernels.
template <typename T, int DIM, int K>
struct LevelGeom {
  int n[3];        // cells per direction
  int vd[3];       // velocity lattice extent per direction (K n + 1)
  int pd[3];       // pressure lattice extent per direction ((K-1) n + 1)
  i64 Nv, Np;      // nodes per velocity component, pressure nodes
  int tiles[3];    // tiles per direction
  T mu;            // viscosity when mu_cell == nullptr
  T gr;            // gamma * rho
  T cp;            // c_pressure (C = cp M_p)
  const T *mu_cell;
  const T *verts;  // vertex coordinates of general cells (nullptr: box cells)
  T *gs;           // scratch of length N for the general-cell path
  T *cbu, *cbp;    // per-cell results of the general-cell path (every-cell mode)
  double h[3];     // cell widths
  Coef1D<T, K> c[DIM];
};

// Array access by element index, or by a byte offset v (per lane) plus a
// compile-time byte offset c: the second form maps to global loads/stores with
// a uniform base address, a 32-bit lane offset and an immediate offset.
struct BOff {
  uint32_t v;
  uint32_t c;
};
template <typename T>
__device__ __forceinline__ T &at(T *p, i64 i) { return p[i]; }
template <typename T>
__device__ __forceinline__ const T &at(const T *p, i64 i) { return p[i]; }
template <typename T>
__device__ __forceinline__ T &at(T *p, BOff b) { return *(T *)((char *)p + b.v + b.c); }
template <typename T>
__device__ __forceinline__ const T &at(const T *p, BOff b) { return *(const T *)((const char *)p + b.v + b.c); }

__device__ __forceinline__ bool on_box_boundary(int i, int extent) { return i == 0 || i == extent - 1; }

// ---------------------------------------------------------------------------
// sum-factorisation passes on register arrays indexed [z][y][x]
// out (=|+=) s * sum_i m(o,i) in(i) along one direction; TR selects m^T.
// ---------------------------------------------------------------------------
template <bool TR, bool ACC, int NZ, int NY, int NI, int NO, typename T, int R, int C>
__device__ __forceinline__ void pass_x(const T (&m)[R][C], const T (&in)[NZ][NY][NI], T (&out)[NZ][NY][NO], T s) {
  static_assert(TR ? (R == NI && C == NO) : (R == NO && C == NI), "pass_x shape");
#pragma unroll
  for (int z = 0; z < NZ; ++z)
#pragma unroll
    for (int y = 0; y < NY; ++y)
#pragma unroll
      for (int o = 0; o < NO; ++o) {
        T acc = 0;
#pragma unroll
        for (int i = 0; i < NI; ++i) acc += (TR ? m[i][o] : m[o][i]) * in[z][y][i];
        out[z][y][o] = ACC ? out[z][y][o] + s * acc : s * acc;
      }
}

template <bool TR, bool ACC, int NZ, int NI, int NO, int NX, typename T, int R, int C>
__device__ __forceinline__ void pass_y(const T (&m)[R][C], const T (&in)[NZ][NI][NX], T (&out)[NZ][NO][NX], T s) {
  static_assert(TR ? (R == NI && C == NO) : (R == NO && C == NI), "pass_y shape");
#pragma unroll
  for (int z = 0; z < NZ; ++z)
#pragma unroll
    for (int x = 0; x < NX; ++x)
#pragma unroll
      for (int o = 0; o < NO; ++o) {
        T acc = 0;
#pragma unroll
        for (int i = 0; i < NI; ++i) acc += (TR ? m[i][o] : m[o][i]) * in[z][i][x];
        out[z][o][x] = ACC ? out[z][o][x] + s * acc : s * acc;
      }
}

template <bool TR, bool ACC, int NI, int NO, int NY, int NX, typename T, int R, int C>
__device__ __forceinline__ void pass_z(const T (&m)[R][C], const T (&in)[NI][NY][NX], T (&out)[NO][NY][NX], T s) {
  static_assert(TR ? (R == NI && C == NO) : (R == NO && C == NI), "pass_z shape");
#pragma unroll
  for (int y = 0; y < NY; ++y)
#pragma unroll
    for (int x = 0; x < NX; ++x)
#pragma unroll
      for (int o = 0; o < NO; ++o) {
        T acc = 0;
#pragma unroll
        for (int i = 0; i < NI; ++i) acc += (TR ? m[i][o] : m[o][i]) * in[i][y][x];
        out[o][y][x] = ACC ? out[o][y][x] + s * acc : s * acc;
      }
}

}  // namespace smg
