// Host replay of the memory accesses of the 3D box-cell operator kernels
// (column sweep tile3d_kernel, cell block block3d_kernel, cell planes
// block3d_plane_kernel): for every block, lane, cell layer and plane the
// byte offsets the kernels form with Column3D (u_at, p_at, mu index) and the
// block / chunk decomposition they share with the host (sweep3d_decode,
// block3d_decode, sweep3d_chunks) are checked against the lengths of the
// vectors they index: velocity vectors d*Nv entries (x, y, r, d, out of every
// epilogue), pressure vectors Np entries, per-cell viscosity n_x n_y n_z
// entries; and every 32-bit offset against the same offset formed in 64 bits.
//
// The kernels' own access pattern is restated here loop by loop (which
// layers are requested, which nodes are fetched and stored, under which
// masks); the arithmetic that turns (lane, layer, node) into an address is
// the kernels' own code, compiled for the host.
//
// Usage: sweep3d_addr_replay K NX NY NZ [sweep_waves]   (exit 0 = in bounds)
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "cell_kernel3d.hpp"

using namespace smg;

namespace {

struct Bounds {
  uint64_t nu_bytes, np_bytes, ncell;
  long checks = 0, errors = 0;
  void u(const BOff &b, const char *what) { check((uint64_t)b.v + b.c, nu_bytes, what); }
  void p(const BOff &b, const char *what) { check((uint64_t)b.v + b.c, np_bytes, what); }
  void check(uint64_t off, uint64_t len, const char *what) {
    ++checks;
    if (off + 8 > len) {   // 8: the widest element (FP64)
      if (errors < 20) std::fprintf(stderr, "out of bounds: %s offset %llu length %llu\n", what,
                                    (unsigned long long)off, (unsigned long long)len);
      ++errors;
    }
  }
  void mu(uint64_t idx) {
    ++checks;
    if (idx >= ncell) {
      if (errors < 20) std::fprintf(stderr, "out of bounds: mu index %llu of %llu\n", (unsigned long long)idx,
                                    (unsigned long long)ncell);
      ++errors;
    }
  }
};

// 64-bit restatement of Column3D::u_at / p_at for the overflow check
template <int K>
uint64_t u64(const Geo3<double> &g, int c, int ax, int ay, int cz, int x, int y, int z) {
  const uint64_t vd0 = g.vd[0], vd1 = g.vd[1];
  return 8ull * ((uint64_t)c * (g.nv_bytes / 8) + (uint64_t)(K * ax + x) + vd0 * ((uint64_t)(K * ay + y) +
                 vd1 * (uint64_t)(K * cz + z)));
}

}  // namespace

int main(int argc, char **argv) {
  if (argc < 5) {
    std::fprintf(stderr, "usage: %s K NX NY NZ [sweep_waves]\n", argv[0]);
    return 2;
  }
  const int K = std::atoi(argv[1]);
  const int n[3] = {std::atoi(argv[2]), std::atoi(argv[3]), std::atoi(argv[4])};
  const int sweep_waves = argc > 5 ? std::atoi(argv[5]) : 4096;
  int rc = 0;
  auto run = [&](auto kconst) {
    constexpr int KK = decltype(kconst)::value;
    Geo3<double> g{};
    for (int a = 0; a < 3; ++a) {
      g.n[a] = n[a];
      g.vd[a] = KK * n[a] + 1;
      g.pd[a] = (KK - 1) * n[a] + 1;
    }
    const uint64_t Nv = (uint64_t)g.vd[0] * g.vd[1] * g.vd[2];
    const uint64_t Np = (uint64_t)g.pd[0] * g.pd[1] * g.pd[2];
    g.nv_bytes = (uint32_t)(Nv * 8);
    Bounds B{3 * Nv * 8, Np * 8, (uint64_t)n[0] * n[1] * n[2]};
    constexpr int NV = KK + 1, NP = KK;
    // the three kernels' field counts: velocity-only, pressure-only and both
    for (int nf_case = 0; nf_case < 3; ++nf_case) {
      const bool OUT_U = nf_case != 1, OUT_P = nf_case != 0;
      const int NF = (OUT_U ? 3 : 0) + (OUT_P ? 1 : 0);
      // ---------------- column sweep (tile3d_kernel)
      {
        Geo3<double> gs = g;
        const int nb = sweep3d_chunks<SW_TX, SW_TY>(gs, NF, sweep_waves);
        // owner stores per node: every node of an output field exactly once
        std::vector<uint8_t> ucount(OUT_U ? 3 * Nv : 0), pcount(OUT_P ? Np : 0);
        for (int blk = 0; blk < nb; ++blk) {
          const int b = xcd_contiguous_tile(blk, nb);
          for (int lane = 0; lane < 64; ++lane) {
            int field;
            Sweep s;
            int cx, cy;
            if (!sweep3d_decode<SW_TX, SW_TY>(gs, NF, b, lane, field, s, cx, cy)) continue;
            const Column3D<KK, double> col(gs, cx, cy);
            const bool vel = OUT_U && field < 3;
            const int comp = vel ? field : 0;
            // 64-bit cross-check of the column base
            const int ax = cx < 0 ? 0 : (cx >= n[0] ? n[0] - 1 : cx);
            const int ay = cy < 0 ? 0 : (cy >= n[1] ? n[1] - 1 : cy);
            for (int cl = s.z_start; cl < s.z_hi; ++cl) {
              const bool more = cl + 1 < s.z_hi;
              const bool owner = s.col_owner && cl >= s.z_lo;
              const bool last_z = cl == n[2] - 1;
              if (vel) {
                // this layer's planes (first layer: all; later: 1..K requested one layer ahead)
                if (cl == s.z_start)
                  for (int z = 0; z < NV; ++z)
                    for (int y = 0; y < NV; ++y)
                      for (int x = 0; x < NV; ++x) {
                        B.u(col.u_at(comp, cl, x, y, z), "sweep load_u");
                        const BOff o = col.u_at(comp, cl, x, y, z);
                        if ((uint64_t)o.v + o.c != u64<KK>(gs, comp, ax, ay, cl, x, y, z)) ++B.errors;
                      }
                if (cl == s.z_start)
                  for (int z = 0; z < NP; ++z)
                    for (int y = 0; y < NP; ++y)
                      for (int x = 0; x < NP; ++x) B.p(col.p_at(cl, x, y, z), "sweep load_p");
                B.mu(col.mu_index(cl));
                if (more) {
                  B.mu(col.mu_index(cl + 1));
                  for (int z = 1; z < NV; ++z)
                    for (int y = 0; y < NV; ++y)
                      for (int x = 0; x < NV; ++x) B.u(col.u_at(comp, cl + 1, x, y, z), "sweep next layer u");
                  for (int z = 1; z < NP; ++z)
                    for (int y = 0; y < NP; ++y)
                      for (int x = 0; x < NP; ++x) B.p(col.p_at(cl + 1, x, y, z), "sweep next layer p");
                }
                if (owner) {
                  for (int z = 0; z < NV; ++z)
                    for (int y = 0; y < NV; ++y)
                      for (int x = 0; x < NV; ++x) {
                        const bool own = x < KK && y < KK && z < KK;
                        const bool high = !own && !((x == KK && !s.last_x) || (y == KK && !s.last_y) ||
                                                    (z == KK && !last_z));
                        if (own || high) {
                          const BOff o = col.u_at(comp, cl, x, y, z);
                          B.u(o, "sweep fetch/store u");
                          const uint64_t idx = ((uint64_t)o.v + o.c) / 8;
                          if (idx < ucount.size() && ucount[idx] < 255) ++ucount[idx];
                        }
                      }
                }
              } else {
                // pressure wave: velocity components of this layer, one ahead
                if (cl == s.z_start)
                  for (int z = 0; z < NV; ++z)
                    for (int y = 0; y < NV; ++y)
                      for (int x = 0; x < NV; ++x) B.u(col.u_at(0, cl, x, y, z), "sweep p-wave load_u");
                for (int c = 0; c < 3; ++c) {
                  if (c < 2) {
                    for (int z = 0; z < NV; ++z)
                      for (int y = 0; y < NV; ++y)
                        for (int x = 0; x < NV; ++x) B.u(col.u_at(c + 1, cl, x, y, z), "sweep p-wave load_u");
                  } else if (more) {
                    for (int z = 0; z < NV; ++z)
                      for (int y = 0; y < NV; ++y)
                        for (int x = 0; x < NV; ++x) B.u(col.u_at(0, cl + 1, x, y, z), "sweep p-wave next u");
                  }
                }
                if (cl == s.z_start)
                  for (int z = 0; z < NP; ++z)
                    for (int y = 0; y < NP; ++y)
                      for (int x = 0; x < NP; ++x) B.p(col.p_at(cl, x, y, z), "sweep p-wave load_p");
                if (more)
                  for (int z = 0; z < NP; ++z)
                    for (int y = 0; y < NP; ++y)
                      for (int x = 0; x < NP; ++x) B.p(col.p_at(cl + 1, x, y, z), "sweep p-wave next p");
                if (owner) {
                  for (int z = 0; z < NP; ++z)
                    for (int y = 0; y < NP; ++y)
                      for (int x = 0; x < NP; ++x) {
                        const bool main = x < KK - 1 && y < KK - 1 && z < KK - 1;
                        const bool edge = ((x < KK - 1) | s.last_x) & ((y < KK - 1) | s.last_y) & ((z < KK - 1) | last_z);
                        if (main || edge) {
                          const BOff o = col.p_at(cl, x, y, z);
                          B.p(o, "sweep fetch/store p");
                          const uint64_t idx = ((uint64_t)o.v + o.c) / 8;
                          if (idx < pcount.size() && pcount[idx] < 255) ++pcount[idx];
                        }
                      }
                }
              }
            }
          }
        }
        long miss = 0, twice = 0;
        for (const uint8_t c : ucount) miss += c == 0, twice += c > 1;
        for (const uint8_t c : pcount) miss += c == 0, twice += c > 1;
        if (miss || twice) {
          std::fprintf(stderr, "sweep ownership (NF %d): %ld nodes never stored, %ld stored more than once\n", NF,
                       miss, twice);
          B.errors += miss + twice;
        }
      }
      // ---------------- cell block and cell planes (block3d_kernel, block3d_plane_kernel)
      {
        Geo3<double> gb = g;
        const int nb = block3d_tiles(gb, NF);
        for (int blk = 0; blk < nb; ++blk) {
          const int b = xcd_contiguous_tile(blk, nb);
          for (int lane = 0; lane < 64; ++lane) {
            int field, cx, cy;
            Block3D s;
            block3d_decode(gb, NF, b, lane, field, s, cx, cy);
            const Column3D<KK, double> col(gb, cx, cy);
            const bool vel = OUT_U && field < 3;
            B.mu(col.mu_index(s.cz));
            for (int c = 0; c < 3; ++c) {
              if (vel && c != field) continue;
              for (int z = 0; z < NV; ++z)
                for (int y = 0; y < NV; ++y)
                  for (int x = 0; x < NV; ++x) B.u(col.u_at(c, s.cz, x, y, z), "block load_u");
            }
            for (int z = 0; z < NP; ++z)
              for (int y = 0; y < NP; ++y)
                for (int x = 0; x < NP; ++x) B.p(col.p_at(s.cz, x, y, z), "block load_p");
            if (!s.owner) continue;
            if (vel) {
              for (int z = 0; z < NV; ++z)
                for (int y = 0; y < NV; ++y)
                  for (int x = 0; x < NV; ++x) {
                    const bool own = x < KK && y < KK && z < KK;
                    const bool high = !own && !((x == KK && !s.last_x) || (y == KK && !s.last_y) ||
                                                (z == KK && !s.last_z));
                    if (own || high) B.u(col.u_at(field, s.cz, x, y, z), "block fetch/store u");
                  }
            } else {
              for (int z = 0; z < NP; ++z)
                for (int y = 0; y < NP; ++y)
                  for (int x = 0; x < NP; ++x) {
                    const bool main = x < KK - 1 && y < KK - 1 && z < KK - 1;
                    const bool edge = ((x < KK - 1) | s.last_x) & ((y < KK - 1) | s.last_y) & ((z < KK - 1) | s.last_z);
                    if (main || edge) B.p(col.p_at(s.cz, x, y, z), "block fetch/store p");
                  }
            }
          }
        }
      }
    }
    std::printf("K=%d n=%dx%dx%d sweep_waves=%d: %ld accesses checked, %ld out of bounds\n", KK, n[0], n[1], n[2],
                sweep_waves, B.checks, B.errors);
    if (B.errors) rc = 1;
  };
  if (K == 2) run(std::integral_constant<int, 2>{});
  else if (K == 3) run(std::integral_constant<int, 3>{});
  else return 2;
  return rc;
}
