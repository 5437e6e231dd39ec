// Host replay of the memory accesses of the 3D matrix-core cell kernel
// (mfma3d_kernel): for every block, lane and cell layer, the global byte
// offsets and LDS indices the kernel forms -- with its own decomposition
// (mfma3d_chunks, mfma3d_decode) and its own per-lane addressing
// (Mfma3DLane, compiled for the host) -- are checked against the lengths of
// what they index: the velocity vectors (3 Nv FP32 entries), the per-cell
// viscosity, the LDS input planes (3 x 665) and the staging area.  The
// staged values a node's gather adds must be real nodes (< 27) of real cells
// (< 153), and every velocity node must be stored by exactly one lane of the
// launch (owned once, Dirichlet rows included).
//
// The kernel's access pattern is restated here loop by loop (which planes
// are loaded per layer, which slots are fetched and stored, under which
// conditions); the arithmetic that turns (lane, layer, slot) into an
// address is the kernel's own code.
//
// Usage: mfma3d_addr_replay NX NY NZ [waves]   (exit 0 = in bounds)
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "cell_kernel3d_mfma.hpp"

using namespace smg;
using namespace smg::mf3;

int main(int argc, char **argv) {
  if (argc < 4) {
    std::fprintf(stderr, "usage: %s NX NY NZ [waves]\n", argv[0]);
    return 2;
  }
  const int n[3] = {std::atoi(argv[1]), std::atoi(argv[2]), std::atoi(argv[3])};
  const int waves = argc > 4 ? std::atoi(argv[4]) : 2048;
  Geo3<float> g{};
  for (int a = 0; a < 3; ++a) {
    g.n[a] = n[a];
    g.vd[a] = 2 * n[a] + 1;
    g.pd[a] = n[a] + 1;
  }
  const uint64_t Nv = (uint64_t)g.vd[0] * g.vd[1] * g.vd[2];
  g.nv_bytes = (uint32_t)(Nv * 4);
  const uint64_t ubytes = 3 * Nv * 4, ncell = (uint64_t)n[0] * n[1] * n[2];
  long checks = 0, errors = 0;
  auto bad = [&](bool cond, const char *what, long long v) {
    ++checks;
    if (cond) {
      if (errors < 20) std::fprintf(stderr, "out of bounds: %s (%lld)\n", what, v);
      ++errors;
    }
  };
  std::vector<uint8_t> owned(3 * Nv, 0);
  const int nb = mfma3d_chunks(g, waves);
  for (int blk = 0; blk < nb; ++blk) {
    const int b = xcd_contiguous_tile(blk, nb);
    Mfma3DTile t;
    if (!mfma3d_decode(g, b, t)) continue;
    bad(t.comp < 0 || t.comp > 2 || t.tx >= g.tiles[0] || t.ty >= g.tiles[1], "tile decode", b);
    for (int lane = 0; lane < 64; ++lane) {
      const Mfma3DLane L(g, t, lane);
      const int cx0 = OX * t.tx - 1, cy0 = OY * t.ty - 1;
      auto load_plane = [&](int gz, int slot) {
        bad(gz < 0 || gz >= g.vd[2], "plane index", gz);
        for (int j = 0; j < LPP; ++j) {
          bool inside, bnd;
          const uint64_t o = (uint64_t)L.comp_base + (uint64_t)gz * L.plane_bytes + L.plane_node(j, inside, bnd);
          bad(o + 4 > ubytes, "plane load", (long long)o);
          const int q = lane + 64 * j;
          if (slot >= 0 && q < PL) bad(slot * PL + q >= 3 * PL, "plane store (LDS)", slot * PL + q);
        }
      };
      auto epilogue_plane = [&](int cl, int zp, bool zb) {
        const uint32_t zoff = (uint32_t)(2 * cl + zp) * L.plane_bytes;
        for (int j = 0; j <= NE; ++j) {
          BOff gi;
          bool ok, dir = true;
          if (j < NE) L.slot(j, zoff, gi, ok, dir);
          else L.slot9(zoff, gi, ok);
          const uint64_t o = (uint64_t)gi.v + gi.c;
          bad(o + 4 > ubytes, "epilogue fetch/store", (long long)o);
          if (j < NE) bad(L.vin_index(zp, j) >= 3 * PL, "input value (LDS)", L.vin_index(zp, j));
          if (ok) {
            const uint64_t node = o / 4;
            // (the node's Dirichlet test uses the plane flag zb; unused here)
            (void)zb;
            if (node < owned.size() && owned[node] < 255) ++owned[node];
          }
        }
      };
      load_plane(2 * t.z_start, 0);
      load_plane(2 * t.z_start + 1, 1);
      load_plane(2 * t.z_start + 2, 2);
      for (int cl = t.z_start; cl < t.z_hi; ++cl) {
        const bool more = cl + 1 < t.z_hi, own = cl >= t.z_lo;
        // per-cell viscosity of the batch rows (MUC)
        for (int bb = 0; bb < NBLK; ++bb) {
          const int c = 32 * bb + L.n;
          int cx = cx0 + c % CX, cy = cy0 + c / CX;
          cx = cx < 0 ? 0 : (cx >= n[0] ? n[0] - 1 : cx);
          cy = cy < 0 ? 0 : (cy >= n[1] ? n[1] - 1 : cy);
          const uint64_t mi = (uint64_t)cx + (uint64_t)n[0] * ((uint64_t)cy + (uint64_t)n[1] * (uint64_t)cl);
          bad(mi >= ncell, "viscosity index", (long long)mi);
        }
        // products: A operand reads and staging stores
        for (int bb = 0; bb < NBLK; ++bb) {
          for (int s = 0; s < 14; ++s) bad(L.a_index(bb, s) >= 3 * PL || L.a_index(bb, s) < 0, "A operand (LDS)", L.a_index(bb, s));
          for (int r = 0; r < 16; ++r) bad(L.stg_index(bb, r) >= NROW * SST, "staging store (LDS)", L.stg_index(bb, r));
        }
        // gathers of the three z planes
        for (int j = 0; j < NE; ++j)
          for (int kz = 0; kz < 3; ++kz) {
            int a[4];
            bool use[4];
            L.gather_index(j, kz, a, use);
            for (int i = 0; i < 4; ++i) {
              bad(a[i] < 0 || a[i] >= NROW * SST, "gather read (LDS)", a[i]);
              if (use[i]) bad(a[i] % SST >= 27 || a[i] / SST >= NCELL, "gathered slot is not a staged cell node", a[i]);
            }
          }
        if (own) {
          epilogue_plane(cl, 0, 2 * cl == 0);
          epilogue_plane(cl, 1, false);
          if (cl == n[2] - 1) epilogue_plane(cl, 2, true);
        }
        load_plane(more ? 2 * cl + 3 : 2 * cl + 1, more ? 1 : -1);
        load_plane(more ? 2 * cl + 4 : 2 * cl + 2, more ? 2 : -1);
      }
    }
  }
  long miss = 0, twice = 0;
  for (const uint8_t c : owned) miss += c == 0, twice += c > 1;
  if (miss || twice) {
    std::fprintf(stderr, "ownership: %ld nodes never stored, %ld stored more than once\n", miss, twice);
    errors += miss + twice;
  }
  std::printf("n=%dx%dx%d waves=%d blocks=%d: %ld accesses checked, %ld out of bounds\n", n[0], n[1], n[2], waves, nb,
              checks, errors);
  return errors == 0 ? 0 : 1;
}
