// Host replay of the index arithmetic of the 3D general-cell kernels in line
// layout (gen3_line_kernel, gen3_gather_kernel), with their own helpers
// compiled for the host (gen3_lane, gen3_blocks, fast_div, cells_around):
//   - fast_div against integer division over edge cases and a random sample
//     of [0, 2^31);
//   - for every block and lane of the cell kernel on an n0 x n1 x n2 mesh:
//     velocity, pressure, vertex and viscosity reads inside their arrays, and
//     every per-cell result (gen3_result_index) written by exactly one live
//     lane;
//   - for every thread of the gather: the node coordinates from fast_div,
//     the cells around the node equal to the cells that contain it (brute
//     force), every per-cell result read inside its array.
// Usage: gen3_replay K N0 N1 N2   (exit 0 = all checks pass)
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "gen_kernel.hpp"

using namespace smg;

static long errors = 0, checks = 0;
#define CHECK(cond, ...)                         \
  do {                                           \
    ++checks;                                    \
    if (!(cond)) {                               \
      if (errors < 20) std::printf(__VA_ARGS__); \
      ++errors;                                  \
    }                                            \
  } while (0)

static void check_fast_div() {
  const uint32_t ds[] = {1, 2, 3, 5, 7, 9, 13, 65, 97, 129, 193, 255, 257, 1025, 4097, 65537, 1000003, (1u << 20) + 1,
                         (1u << 30) - 1, (1u << 30) + 3, (1u << 31) - 1};
  std::mt19937_64 rng(12345);
  for (uint32_t d : ds) {
    const FastDiv f = make_fastdiv(d);
    std::vector<uint32_t> ns = {0, 1, 2, d - 1, d, d + 1, 2 * d - 1, 2 * d, (1u << 31) - 1, (1u << 31) - d,
                                (1u << 31) - 1 - ((1u << 31) - 1) % d, (1u << 31) - 2};
    for (int i = 0; i < 200000; ++i) ns.push_back((uint32_t)(rng() % (1ull << 31)));
    for (uint32_t n : ns) {
      if (n >= (1u << 31)) continue;
      CHECK(fast_div(n, f) == n / d, "fast_div %u / %u = %u, expected %u\n", n, d, fast_div(n, f), n / d);
    }
  }
}

template <int K>
static void check_mesh(int n0, int n1, int n2) {
  constexpr int NV = K + 1, NP = K, NN = NV * NV * NV, NPN = NP * NP * NP;
  const int n[3] = {n0, n1, n2};
  const int vd[3] = {K * n0 + 1, K * n1 + 1, K * n2 + 1};
  const int pd[3] = {(K - 1) * n0 + 1, (K - 1) * n1 + 1, (K - 1) * n2 + 1};
  const int64_t Nv = (int64_t)vd[0] * vd[1] * vd[2], Np = (int64_t)pd[0] * pd[1] * pd[2];
  const int64_t ncell = (int64_t)n0 * n1 * n2;
  const int64_t nvert = (int64_t)(n0 + 1) * (n1 + 1) * (n2 + 1);
  GenGeo<double> g{};
  for (int a = 0; a < 3; ++a) {
    g.n[a] = n[a];
    g.vd[a] = vd[a];
    g.pd[a] = pd[a];
  }
  g.Nv = Nv;
  g.Np = Np;
  const int nb = (int)gen3_blocks<K>(g);
  std::vector<int> wu(ncell * 3 * NN, 0), wp(ncell * NPN, 0);
  for (int blk = 0; blk < nb; ++blk)
    for (int lane = 0; lane < 64; ++lane) {
      const Gen3Lane l = gen3_lane<K>(g.n, blk, nb, lane);
      CHECK(l.cx >= 0 && l.cx < n0 && l.cy >= 0 && l.cy < n1 && l.cz >= 0 && l.cz < n2, "cell out of range\n");
      CHECK(l.a >= 0 && l.a < NV && l.b >= 0 && l.b < NV, "line out of range\n");
      CHECK(l.s >= 0 && l.s < (64 + NV * NV - 1) / (NV * NV), "slot out of range\n");
      const int64_t cell = l.cx + (int64_t)n0 * (l.cy + (int64_t)n1 * l.cz);
      // velocity reads: x line of nodes (K cx + i, K cy + a, K cz + b)
      const int gy = K * l.cy + l.a, gz = K * l.cz + l.b;
      const int64_t row = (int64_t)vd[0] * (gy + (int64_t)vd[1] * gz) + K * l.cx;
      for (int c = 0; c < 3; ++c)
        for (int i = 0; i < NV; ++i) {
          const int64_t idx = (int64_t)c * Nv + row + i;
          CHECK(row + i >= 0 && row + i < Nv && idx < 3 * Nv, "velocity read %lld out of range\n", (long long)idx);
          CHECK(K * l.cx + i < vd[0], "velocity x out of the row\n");
        }
      // pressure reads (lines with a, b < K)
      if (l.a < NP && l.b < NP) {
        const int64_t prow = (int64_t)pd[0] * ((K - 1) * l.cy + l.a + (int64_t)pd[1] * ((K - 1) * l.cz + l.b)) +
                             (K - 1) * l.cx;
        for (int i = 0; i < NP; ++i) CHECK(prow + i >= 0 && prow + i < Np, "pressure read out of range\n");
      }
      // vertices and viscosity
      const int64_t vx = n0 + 1, vxy = vx * (n1 + 1);
      const int64_t v0 = l.cx + vx * l.cy + vxy * l.cz;
      for (int v = 0; v < 8; ++v) {
        const int64_t vid = v0 + (v & 1) + vx * ((v >> 1) & 1) + vxy * ((v >> 2) & 1);
        CHECK(vid >= 0 && vid < nvert, "vertex out of range\n");
      }
      CHECK(cell >= 0 && cell < ncell, "viscosity index out of range\n");
      if (!l.live) continue;
      for (int c = 0; c < 3; ++c)
        for (int i = 0; i < NV; ++i) {
          const int64_t o = gen3_result_index<NV>(g.n, c, l.cx, l.cy, l.cz, i, l.a, l.b);
          CHECK(o >= 0 && o < (int64_t)wu.size(), "velocity result out of range\n");
          if (o >= 0 && o < (int64_t)wu.size()) ++wu[o];
        }
      if (l.a < NP && l.b < NP)
        for (int i = 0; i < NP; ++i) {
          const int64_t o = gen3_result_index<NP>(g.n, 0, l.cx, l.cy, l.cz, i, l.a, l.b);
          CHECK(o >= 0 && o < (int64_t)wp.size(), "pressure result out of range\n");
          if (o >= 0 && o < (int64_t)wp.size()) ++wp[o];
        }
    }
  for (size_t i = 0; i < wu.size(); ++i) CHECK(wu[i] == 1, "velocity result %zu written %d times\n", i, wu[i]);
  for (size_t i = 0; i < wp.size(); ++i) CHECK(wp[i] == 1, "pressure result %zu written %d times\n", i, wp[i]);

  // gather: one thread per velocity node, then per pressure node
  const FastDiv fv0 = make_fastdiv(vd[0]), fv1 = make_fastdiv(vd[1]);
  const FastDiv fp0 = make_fastdiv(pd[0]), fp1 = make_fastdiv(pd[1]);
  const int64_t items = Nv + Np;
  const int gb = (int)((items + 255) / 256);
  std::vector<int> seen(items, 0);
  for (int blk = 0; blk < gb; ++blk)
    for (int th = 0; th < 256; ++th) {
      const uint32_t t = (uint32_t)xcd_contiguous_tile(blk, gb) * 256u + (uint32_t)th;
      if (t >= items) continue;
      ++seen[t];
      const bool vel = t < Nv;
      const uint32_t j = vel ? t : t - (uint32_t)Nv;
      const FastDiv &f0 = vel ? fv0 : fp0, &f1 = vel ? fv1 : fp1;
      const uint32_t q = fast_div(j, f0);
      const int x = (int)(j - q * f0.d);
      const uint32_t zq = fast_div(q, f1);
      const int y = (int)(q - zq * f1.d), z = (int)zq;
      const int *ext = vel ? vd : pd;
      CHECK((int64_t)x + ext[0] * ((int64_t)y + (int64_t)ext[1] * z) == j && x < ext[0] && y < ext[1] && z < ext[2],
            "node decomposition of %u wrong\n", j);
      const int deg = vel ? K : K - 1, ns = deg + 1;
      const int xyz[3] = {x, y, z};
      int c0[3], nc[3];
      for (int a = 0; a < 3; ++a) {
        cells_around(xyz[a], deg, n[a], c0[a], nc[a]);
        // brute force: cells c with deg c <= v <= deg (c + 1)
        int bf0 = -1, bfn = 0;
        for (int c = 0; c < n[a]; ++c)
          if (deg * c <= xyz[a] && xyz[a] <= deg * (c + 1)) {
            if (bf0 < 0) bf0 = c;
            ++bfn;
          }
        CHECK(bf0 == c0[a] && bfn == nc[a], "cells around %d (direction %d) wrong\n", xyz[a], a);
      }
      for (int kz = 0; kz < nc[2]; ++kz)
        for (int ky = 0; ky < nc[1]; ++ky)
          for (int kx = 0; kx < nc[0]; ++kx) {
            const int cx = c0[0] + kx, cy = c0[1] + ky, cz = c0[2] + kz;
            const int lx = x - deg * cx, ly = y - deg * cy, lz = z - deg * cz;
            CHECK(lx >= 0 && lx < ns && ly >= 0 && ly < ns && lz >= 0 && lz < ns, "local node out of the cell\n");
            for (int c = 0; c < (vel ? 3 : 1); ++c) {
              const int64_t o = vel ? gen3_result_index<NV>(g.n, c, cx, cy, cz, lx, ly, lz)
                                    : gen3_result_index<NP>(g.n, 0, cx, cy, cz, lx, ly, lz);
              CHECK(o >= 0 && o < (vel ? (int64_t)wu.size() : (int64_t)wp.size()), "gather read out of range\n");
            }
          }
    }
  for (int64_t i = 0; i < items; ++i) CHECK(seen[i] == 1, "item %lld handled %d times\n", (long long)i, seen[i]);
}

int main(int argc, char **argv) {
  if (argc != 5) {
    std::printf("usage: gen3_replay K N0 N1 N2\n");
    return 2;
  }
  const int k = std::atoi(argv[1]), n0 = std::atoi(argv[2]), n1 = std::atoi(argv[3]), n2 = std::atoi(argv[4]);
  check_fast_div();
  if (k == 2) check_mesh<2>(n0, n1, n2);
  else if (k == 3) check_mesh<3>(n0, n1, n2);
  else return 2;
  std::printf("%ld checks, %ld errors\n", checks, errors);
  return errors == 0 ? 0 : 1;
}
