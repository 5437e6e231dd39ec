// Set-up on vertex-given (multilinear) cells: the local Schur diagonal
//   D~_S,loc = sum_tau P_tau^T diag(B_tau diag(A_tau)^-1 B_tau^T) P_tau
// (Sec. 3.3.1), plus c_p diag(M_p) (C = c_p M_p).  The cell matrices are
// evaluated by the quadrature of the operator kernels (k+1 Gauss points per
// direction, the multilinear vertex map, J^-1 and det J at every point), one
// thread per (cell, pressure node of the cell); constrained velocity columns
// (Dirichlet nodes) are left out.  A second kernel sums the contributions of
// the cells around each pressure node in a fixed order (no atomics).
#pragma once
#include "gen_kernel.hpp"
#include "setup_kernels.hpp"

namespace smg {

template <int DIM, int K>
__global__ void k_schur_loc_cells(const GenGeo<double> g, double cp, double *contrib) {
  constexpr int NV = K + 1, NP = K;
  constexpr int NN = DIM == 3 ? NV * NV * NV : NV * NV;    // velocity nodes = quadrature points
  constexpr int NPN = DIM == 3 ? NP * NP * NP : NP * NP;   // pressure nodes of a cell
  constexpr int NVERT = 1 << DIM;
  constexpr cfe::QTab<K, double> Q = cfe::make_qtab<K, double>();
  const i64 ncells = (i64)g.n[0] * g.n[1] * (DIM == 3 ? g.n[2] : 1);
  SMG_GRID_LOOP(t, ncells * NPN) {
    const i64 cell = t / NPN;
    const int il = (int)(t - cell * NPN);
    const int ip[3] = {il % NP, (il / NP) % NP, DIM == 3 ? il / (NP * NP) : 0};
    const i64 r = cell / g.n[0];
    const int cc[3] = {(int)(cell - r * g.n[0]), (int)(r % g.n[1]), DIM == 3 ? (int)(r / g.n[1]) : 0};
    const double mu = g.mu_cell != nullptr ? g.mu_cell[cell] : g.mu;
    double s = 0.0, mpp = 0.0;
    for (int j = 0; j < NN; ++j) {
      const int jl[3] = {j % NV, (j / NV) % NV, DIM == 3 ? j / (NV * NV) : 0};
      bool free_node = true;
      for (int a = 0; a < DIM; ++a) free_node &= !on_box_boundary(K * cc[a] + jl[a], g.vd[a]);
      double ajj = 0.0, b[3] = {0.0, 0.0, 0.0};
      for (int q = 0; q < NN; ++q) {
        const int ql[3] = {q % NV, (q / NV) % NV, DIM == 3 ? q / (NV * NV) : 0};
        // geometry at the point
        double xi[3] = {0.0, 0.0, 0.0};
        for (int a = 0; a < DIM; ++a) xi[a] = Q.x[ql[a]];
        double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
        for (int v = 0; v < NVERT; ++v) {
          const int o[3] = {v & 1, (v >> 1) & 1, (v >> 2) & 1};
          const i64 vid = (cc[0] + o[0]) + (i64)(g.n[0] + 1) * ((cc[1] + o[1]) + (i64)(g.n[1] + 1) * (DIM == 3 ? cc[2] + o[2] : 0));
          for (int bb = 0; bb < DIM; ++bb) {
            double dn = o[bb] ? 1.0 : -1.0;
            for (int c = 0; c < DIM; ++c)
              if (c != bb) dn *= o[c] ? xi[c] : 1.0 - xi[c];
            for (int a = 0; a < DIM; ++a) J[a][bb] += g.verts[vid * DIM + a] * dn;
          }
        }
        double Ji[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}, det;
        if constexpr (DIM == 2) {
          det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
          Ji[0][0] = J[1][1] / det;
          Ji[0][1] = -J[0][1] / det;
          Ji[1][0] = -J[1][0] / det;
          Ji[1][1] = J[0][0] / det;
        } else {
          const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
          const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
          const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
          det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
          Ji[0][0] = c00 / det;
          Ji[1][0] = c01 / det;
          Ji[2][0] = c02 / det;
          Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
          Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
          Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
          Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
          Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
          Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
        }
        double jxw = det;
        for (int a = 0; a < DIM; ++a) jxw *= Q.w[ql[a]];
        // phi_j and its reference gradient at the point: l_i'(x_q) is the
        // collocation derivative on the Gauss points of the values l_i(x_p)
        double val = 1.0, dref[3] = {1.0, 1.0, 1.0};
        for (int a = 0; a < DIM; ++a) {
          double d1 = 0.0;
          for (int p = 0; p < NV; ++p) d1 += Q.D[ql[a]][p] * Q.V[p][jl[a]];
          const double v1 = Q.V[ql[a]][jl[a]];
          for (int bb = 0; bb < DIM; ++bb) dref[bb] *= (bb == a) ? d1 : v1;
          val *= v1;
        }
        double grad[3] = {0.0, 0.0, 0.0}, g2 = 0.0;
        for (int a = 0; a < DIM; ++a) {
          for (int bb = 0; bb < DIM; ++bb) grad[a] += Ji[bb][a] * dref[bb];
          g2 += grad[a] * grad[a];
        }
        double psi = 1.0;
        for (int a = 0; a < DIM; ++a) psi *= Q.Vp[ql[a]][ip[a]];
        ajj += (mu * g2 + g.gr * val * val) * jxw;
        for (int c = 0; c < DIM; ++c) b[c] -= psi * grad[c] * jxw;
        if (j == 0) mpp += psi * psi * jxw;
      }
      if (free_node)
        for (int c = 0; c < DIM; ++c) s += b[c] * b[c] / ajj;
    }
    contrib[t] = s + cp * mpp;
  }
}

// DS[node] = sum over the cells around the pressure node of their
// contributions, in a fixed order
template <int DIM, int K>
__global__ void k_schur_loc_gather(const GenGeo<double> g, const double *contrib, double *DS) {
  constexpr int KP = K - 1, NP = K;
  constexpr int NPN = DIM == 3 ? NP * NP * NP : NP * NP;
  SMG_GRID_LOOP(node, g.Np) {
    int l[3] = {0, 0, 0};
    unflat<DIM>(node, g.pd, l);
    int cs[3][2] = {{0, 0}, {0, 0}, {0, 0}}, ls[3][2] = {{0, 0}, {0, 0}, {0, 0}}, m[3] = {1, 1, 1};
    for (int a = 0; a < DIM; ++a) m[a] = node_cells(l[a], KP, g.n[a], cs[a], ls[a]);
    double s = 0.0;
    for (int iz = 0; iz < (DIM == 3 ? m[2] : 1); ++iz)
      for (int iy = 0; iy < m[1]; ++iy)
        for (int ix = 0; ix < m[0]; ++ix) {
          const i64 cell = cs[0][ix] + (i64)g.n[0] * (cs[1][iy] + (i64)g.n[1] * (DIM == 3 ? cs[2][iz] : 0));
          const int il = ls[0][ix] + NP * (ls[1][iy] + NP * (DIM == 3 ? ls[2][iz] : 0));
          s += contrib[cell * NPN + il];
        }
    DS[node] = s;
  }
}

}  // namespace smg
