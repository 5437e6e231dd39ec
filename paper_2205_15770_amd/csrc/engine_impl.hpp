// Solver engine for one (dimension, degree) pair; instantiated per pair in
// its own translation unit.
#pragma once
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>

#include "cell_kernel2d.hpp"
#include "packed.hpp"
#include "gen_kernel.hpp"
#include "cell_kernel3d.hpp"
#include "cell_kernel3d_mfma.hpp"
#include "gen_setup.hpp"
#include "engine.hpp"
#include "ops.hpp"
#include "setup_kernels.hpp"
#include "transfer_kernels.hpp"
#include "vec_kernels.hpp"

namespace smg {

// Largest 3D Q2 level (cells per direction, all three directions) that runs
// the one-cell-per-lane block kernel instead of the column sweep.  The
// environment variable SMG_BLOCK3D_MAX_N, read when a solver is set up,
// overrides it (0: sweep everywhere).
inline int block3d_max_n_from_env() {
  const char *e = std::getenv("SMG_BLOCK3D_MAX_N");
  return e != nullptr ? std::atoi(e) : 32;
}

// Largest 2D level (cells per direction) on which the smoother fuses the
// operator application producing a Chebyshev right-hand side with the first
// Chebyshev step (one launch instead of two; its 8 x 8 tile owns 5 x 5
// cells, so it recomputes more; measured on the 512^2 solve it pays on
// every level up to 512^2).  SMG_FUSE2D_MAX_N overrides it (0: never).
inline int fuse2d_max_n_from_env() {
  const char *e = std::getenv("SMG_FUSE2D_MAX_N");
  return e != nullptr ? std::atoi(e) : 512;
}

// Largest 2D level (cells per direction) on which an Uzawa step with k_S = 1
// runs as three launches: the velocity update, then the pressure residual
// fused with the first S~ direction and its A_hat^-1 application, then the
// S~ Chebyshev step fused with B^T dp and the final A_hat^-1 application
// (8 x 8 tiles owning 3 x 3 cells).  SMG_FUSE3_2D_MAX_N overrides it (0:
// never).
inline int fuse3_2d_max_n_from_env() {
  const char *e = std::getenv("SMG_FUSE3_2D_MAX_N");
  return e != nullptr ? std::atoi(e) : 128;
}

// Largest 3D Q2 level (cells per direction) whose cell-block launches use
// one wave per output plane of the cells; SMG_PLANE3D_MAX_N overrides it
// (0: never).
inline int plane3d_max_n_from_env() {
  const char *e = std::getenv("SMG_PLANE3D_MAX_N");
  return e != nullptr ? std::atoi(e) : 16;
}

// Waves a 3D column-sweep launch aims at (the z extent is cut into chunks
// of >= 2 cells until the launch has about this many); SMG_SWEEP_WAVES
// overrides it.
inline int sweep_waves_from_env() {
  const char *e = std::getenv("SMG_SWEEP_WAVES");
  const int v = e != nullptr ? std::atoi(e) : 4096;
  return v > 0 ? v : 4096;
}

// Smallest 3D Q2 level (cells per direction, any direction) whose FP32
// Chebyshev steps for A run on the matrix-core cell kernel instead of the
// column sweep: by default none (measured slower than the sweep at 64^3:
// 68 against 54 us); SMG_MFMA3D_MIN_N sets it.  SMG_MFMA3D_WAVES sets the
// waves that launch aims at (z chunks; default 960: at one wave per SIMD
// the 64^3 launch then runs in one round on the 1024 SIMDs).
inline int mfma3d_min_n_from_env() {
  const char *e = std::getenv("SMG_MFMA3D_MIN_N");
  return e != nullptr ? std::atoi(e) : 0;
}
inline int mfma3d_waves_from_env() {
  const char *e = std::getenv("SMG_MFMA3D_WAVES");
  const int v = e != nullptr ? std::atoi(e) : 960;
  return v > 0 ? v : 960;
}
template <class Op>
struct is_cheb_a_op : std::false_type {};
template <typename T, bool F, bool L>
struct is_cheb_a_op<OpChebA<T, F, L>> : std::true_type {};

// 3D general cells: the line-layout cell kernel (1, default) or the one
// with a lane per quadrature point (0); SMG_GEN3_LINES overrides it.
inline int gen3_lines_from_env() {
  const char *e = std::getenv("SMG_GEN3_LINES");
  return e != nullptr ? std::atoi(e) : 1;
}

// Largest 2D level (cells per direction) whose operator launches with a
// pressure output use one wave per (tile, output field) instead of one wave
// per tile for all fields (launches with velocity outputs only always do);
// SMG_SPLIT2D_MAX_N overrides it (0: one wave per tile everywhere).  On the
// 512^2 level such launches are the operator applications K x and the level
// residual, and one wave per tile reads each vector once: FP64 K x 17.9 ->
// 15.6 us, the solves unchanged.
inline int split2d_max_n_from_env() {
  const char *e = std::getenv("SMG_SPLIT2D_MAX_N");
  return e != nullptr ? std::atoi(e) : 256;
}

// Smallest 2D level (cells per direction) whose fused two-stage launches run
// on workgroups of several waves that exchange faces through LDS instead of
// one wave per tile (the tile's halo shrinks from 39 of 64 cells to 87 of
// 256); SMG_WGF2D_MIN_N overrides it (0: never) and SMG_WGF2D_SHAPE picks the
// waves per workgroup (22: 2 x 2, 42: 4 x 2, 44: 4 x 4).
inline int wgf2d_min_n_from_env() {
  const char *e = std::getenv("SMG_WGF2D_MIN_N");
  return e != nullptr ? std::atoi(e) : 512;
}
inline int wgf2d_shape_from_env() {
  const char *e = std::getenv("SMG_WGF2D_SHAPE");
  const int v = e != nullptr ? std::atoi(e) : 22;
  return (v == 42 || v == 22 || v == 44) ? v : 22;
}

// Lanczos (Algorithm 2 asks for a close approximation of lambda_max): steps,
// safety factor and SplitMix64 seeds of the start vectors.
constexpr int LANCZOS_STEPS = 30;
constexpr double LANCZOS_SAFETY = 1.02;
constexpr uint64_t LANCZOS_SEED_A = 1234, LANCZOS_SEED_S = 4321;

// SplitMix64 (Steele, Lea, Flood 2014) as a counter-based generator: output i
// (i = 1, 2, ...) mixes seed + i * 0x9E3779B97F4A7C15.  Mapped to [-1, 1) from
// the top 53 bits.
inline double splitmix64_uniform(uint64_t seed, uint64_t i) {
  uint64_t z = seed + i * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return 2.0 * ((double)(z >> 11) / 9007199254740992.0) - 1.0;
}

// C_{k+1}(3) / (1 + C_{k+1}(3)) of Lemma 1 / Algorithm 2, C_n(3) by the
// Chebyshev three-term recurrence C_{n+1} = 6 C_n - C_{n-1}.
inline double cheb_scaling(int k) {
  double c0 = 1.0, c1 = 3.0;
  for (int n = 1; n < k + 1; ++n) {
    double c2 = 6.0 * c1 - c0;
    c0 = c1;
    c1 = c2;
  }
  return c1 / (1.0 + c1);
}

template <int DIM, int K>
class EngineT : public EngineBase {
 public:
  // one cell per thread; (T-1)^d owned cells plus one low halo layer per tile
  static constexpr int TX = DIM == 2 ? 16 : (K == 2 ? 4 : 3);
  static constexpr int TY = TX;
  static constexpr int TZ = DIM == 2 ? 1 : TX;
  static constexpr int OWN = TX - 1;

  Ref1D ref;
  TransferTables ttab;
  bool general = false;                      // cells given by vertices
  bool gen_op = false;                       // operator through the vertex-given cell kernel
  int block3d_max_n = block3d_max_n_from_env();
  int split2d_max_n = split2d_max_n_from_env();
  int wgf2d_min_n = wgf2d_min_n_from_env();
  int wgf2d_shape = wgf2d_shape_from_env();
  int gen3_lines = gen3_lines_from_env();
  int sweep_waves = sweep_waves_from_env();
  int mfma3d_min_n = mfma3d_min_n_from_env();
  int mfma3d_waves = mfma3d_waves_from_env();
  int fuse2d_max_n = fuse2d_max_n_from_env();
  int fuse3_2d_max_n = fuse3_2d_max_n_from_env();
  int plane3d_max_n = plane3d_max_n_from_env();
  std::vector<std::vector<double>> hverts;   // per level, host copy (node coordinates)
  double *Kinv = nullptr;
  int coarse_ld = 0;   // leading dimension of Kinv: n0 + 1 (bordered) or n0
  int n0 = 0;
  double sigma = 0, tau = 0;
  // FGMRES storage
  int restart = 30;
  double *V = nullptr, *Z = nullptr, *partial = nullptr, *dvec = nullptr;
  float *b32 = nullptr, *x32 = nullptr;
  double *lz[4] = {nullptr, nullptr, nullptr, nullptr};  // Lanczos temporaries
  double mp1_sum = 0;
  // The preconditioning cycle (zero initial guess, fixed internal buffers) is
  // captured once per precision into a HIP graph and replayed; this removes
  // the host launch cost of its several hundred small kernels.
  struct CycleGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  CycleGraph cg[2];
  hipStream_t cap_stream = nullptr;
  double *b64 = nullptr, *x64 = nullptr;

  void invalidate_graphs() override {
    for (CycleGraph &c : cg) {
      if (c.exec) (void)hipGraphExecDestroy(c.exec);
      if (c.graph) (void)hipGraphDestroy(c.graph);
      c.exec = nullptr;
      c.graph = nullptr;
    }
  }
  ~EngineT() override {
    invalidate_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }

  // x_L = cycle(0, b_L) for the internal buffers of precision `dt`, by graph
  // replay (captured on first use) or, while kernel timing is on, eagerly.
  void cycle_from_zero(int dt) {
    if (profiling || !use_graphs) {
      if (dt == SMG_F32) { vset<float>(x32, 0.0f, lv[L].N); cycle_t<float>(L, x32, b32, true); }
      else { vset<double>(x64, 0.0, lv[L].N); cycle_t<double>(L, x64, b64, true); }
      return;
    }
    CycleGraph &c = cg[dt];
    if (!c.exec) {
      if (!cap_stream) SMG_HIP(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
      hipStream_t saved = stream;
      stream = cap_stream;
      SMG_HIP(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal));
      try {
        if (dt == SMG_F32) { vset<float>(x32, 0.0f, lv[L].N); cycle_t<float>(L, x32, b32, true); }
        else { vset<double>(x64, 0.0, lv[L].N); cycle_t<double>(L, x64, b64, true); }
      } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(cap_stream, &g);
        if (g) (void)hipGraphDestroy(g);
        stream = saved;
        throw;
      }
      SMG_HIP(hipStreamEndCapture(cap_stream, &c.graph));
      stream = saved;
      SMG_HIP(hipGraphInstantiate(&c.exec, c.graph, nullptr, nullptr, 0));
    }
    SMG_HIP(hipGraphLaunch(c.exec, stream));
  }

  // ---------------------------------------------------------------- helpers
  template <typename T>
  Work<T> &work(int l) {
    if constexpr (std::is_same<T, double>::value) return lv[l].w64;
    else return lv[l].w32;
  }

  template <typename T>
  LevelGeom<T, DIM, K> geom(int l, bool unit_cp = false) {
    const LevelInfo &I = lv[l];
    LevelGeom<T, DIM, K> g;
    std::memset(&g, 0, sizeof(g));
    for (int a = 0; a < 3; ++a) {
      g.n[a] = I.n[a];
      g.vd[a] = I.vd[a];
      g.pd[a] = I.pd[a];
      g.tiles[a] = (a < DIM) ? (I.n[a] + OWN - 1) / OWN : 1;
    }
    g.Nv = I.Nv;
    g.Np = I.Np;
    g.mu = (T)desc.mu;
    g.gr = (T)(desc.gamma * desc.rho);
    g.cp = (T)(unit_cp ? 1.0 : desc.c_pressure);
    g.mu_cell = work<T>(l).mu_cell;
    g.verts = work<T>(l).verts;
    g.gs = work<T>(l).t1;
    g.cbu = work<T>(l).cbu;
    g.cbp = work<T>(l).cbp;
    for (int a = 0; a < 3; ++a) g.h[a] = I.h[a];
    const int nv = K + 1, np = K;
    for (int a = 0; a < DIM; ++a) {
      const double h = I.h[a];
      for (int i = 0; i < nv; ++i)
        for (int j = 0; j < nv; ++j) {
          g.c[a].Kv[i][j] = (T)(ref.Kv[i * nv + j] / h);
          g.c[a].Mv[i][j] = (T)(ref.Mv[i * nv + j] * h);
        }
      for (int i = 0; i < np; ++i) {
        for (int j = 0; j < nv; ++j) {
          g.c[a].G[i][j] = (T)(ref.G[i * nv + j]);
          g.c[a].N[i][j] = (T)(ref.N[i * nv + j] * h);
        }
        for (int j = 0; j < np; ++j) g.c[a].Mp[i][j] = (T)(ref.Mp[i * np + j] * h);
      }
    }
    return g;
  }

  void check_launch() { SMG_HIP(hipGetLastError()); }

  // 2D box-cell geometry of the wave-tile kernels; `own` cells per tile and direction
  template <typename T>
  Geo2<T> geo2(const LevelGeom<T, DIM, K> &g, int own) const {
    Geo2<T> g2;
    std::memset(&g2, 0, sizeof(g2));
    for (int a = 0; a < 2; ++a) {
      g2.n[a] = g.n[a];
      g2.vd[a] = g.vd[a];
      g2.pd[a] = g.pd[a];
      g2.tiles[a] = (g.n[a] + own - 1) / own;
    }
    g2.nv_bytes = (uint32_t)(g.Nv * (int64_t)sizeof(T));
    g2.mu = g.mu;
    g2.gr = g.gr;
    g2.cp = g.cp;
    g2.mu_cell = g.mu_cell;
    const double hx = g.h[0], hy = g.h[1];
    g2.sKx = (T)(hy / hx);
    g2.sKy = (T)(hx / hy);
    g2.sM = (T)(hx * hy);
    g2.sB[0] = (T)hy;
    g2.sB[1] = (T)hx;
    return g2;
  }

  template <typename T, int BLK, class Op>
  void tile(const LevelGeom<T, DIM, K> &g, const Op &op) {
    hipEvent_t ea = nullptr, eb = nullptr;
    if (profiling) {
      ea = next_event();
      eb = next_event();
      SMG_HIP(hipEventRecord(ea, stream));
    }
    if (rec && (gen_op || DIM != 2)) throw Error{SMG_EUNSUPPORTED, "batched launches: 2D box cells only"};
    if (gen_op) {
      gen_tile<T, BLK, Op>(g, op);
    } else if constexpr (DIM == 2) {
      // 8 x 8 cells per wave, one cell per lane
      const Geo2<T> g2 = geo2<T>(g, 7);
      const unsigned nb2 = (unsigned)(g2.tiles[0] * g2.tiles[1]);
      constexpr unsigned NF2 = ((BLK & (BLK_A | BLK_MASS | BLK_BT)) ? 2 : 0) + ((BLK & (BLK_B | BLK_C)) ? 1 : 0);
      constexpr bool VEL_ONLY = (BLK & (BLK_B | BLK_C)) == 0;
      if (NF2 > 1 && split2d_max_n > 0 && (VEL_ONLY || std::max(g.n[0], g.n[1]) <= split2d_max_n)) {
        // one wave per (tile, output field): fewer instructions per wave.
        // Blocks with only velocity outputs read nothing twice this way; the
        // others read p (and u) once per field, which pays on small levels.
        if (rec) rec_add(LTile2Split<K, T, BLK, Op>{g2, op}, nb2 * NF2);
        else hipLaunchKernelGGL((wave2d_split_kernel<K, T, BLK, Op>), dim3(nb2 * NF2), dim3(64), 0, stream, g2, op);
      } else {
        if (rec) rec_add(LTile2<K, T, BLK, Op>{g2, op}, nb2);
        else hipLaunchKernelGGL((wave2d_kernel<K, T, BLK, Op>), dim3(nb2), dim3(64), 0, stream, g2, op);
      }
    } else if constexpr (K != 2) {
      // Q3-Q2 in 3D always runs on the vertex-given cell kernel (gen_op)
      throw Error{SMG_EUNSUPPORTED, "3D Q3-Q2 box kernel"};
    } else {
      // SW_TX x SW_TY cell columns per wave, one wave per output field; the z extent
      // is cut into chunks so that the launch has about sweep_waves waves
      // (4096: four per SIMD) when the level is large enough, chunks of >= 2
      // cells.
      constexpr int NF = ((BLK & (BLK_A | BLK_MASS | BLK_BT)) ? 3 : 0) + ((BLK & (BLK_B | BLK_C)) ? 1 : 0);
      Geo3<T> g3;
      std::memset(&g3, 0, sizeof(g3));
      for (int a = 0; a < 3; ++a) {
        g3.n[a] = g.n[a];
        g3.vd[a] = g.vd[a];
        g3.pd[a] = g.pd[a];
      }
      g3.nv_bytes = (uint32_t)(g.Nv * (int64_t)sizeof(T));
      g3.mu = g.mu;
      g3.gr = g.gr;
      g3.cp = g.cp;
      g3.mu_cell = g.mu_cell;
      const double hx = g.h[0], hy = g.h[1], hz = g.h[2];
      g3.sKx = (T)(hy * hz / hx);
      g3.sKy = (T)(hx * hz / hy);
      g3.rz = (T)((hy * hy) / (hz * hz));
      g3.sM = (T)(hx * hy * hz);
      g3.sB[0] = (T)(hy * hz);
      g3.sB[1] = (T)(hx * hz);
      g3.sB[2] = (T)(hx * hy);
      if (std::max(g.n[0], std::max(g.n[1], g.n[2])) <= block3d_max_n) {
        // small level: 4 x 4 x 4 cells per wave, one cell per lane, no sweep
        const unsigned nbb = (unsigned)block3d_tiles(g3, NF);
        if (std::max(g.n[0], std::max(g.n[1], g.n[2])) <= plane3d_max_n)
          // smallest levels: one wave per output plane of the cells
          hipLaunchKernelGGL((block3d_plane_kernel<K, T, BLK, Op>), dim3(nbb), dim3(64 * (K + 1)), 0, stream, g3, op);
        else
          hipLaunchKernelGGL((block3d_kernel<K, T, BLK, Op>), dim3(nbb), dim3(64), 0, stream, g3, op);
      } else {
        bool done = false;
        if constexpr (std::is_same<T, float>::value && BLK == BLK_A && is_cheb_a_op<Op>::value) {
          // uniform box cells: the cell matrix is shared, 32 cells per
          // matrix-core product (per-cell viscosity only with gamma rho = 0)
          if (mfma3d_min_n > 0 && std::max(g.n[0], std::max(g.n[1], g.n[2])) >= mfma3d_min_n &&
              (g.mu_cell == nullptr || g.gr == 0)) {
            const unsigned nbm = (unsigned)mfma3d_chunks(g3, mfma3d_waves);
            if (g.mu_cell != nullptr)
              hipLaunchKernelGGL((mfma3d_kernel<Op, true>), dim3(nbm), dim3(64), 0, stream, g3, op);
            else
              hipLaunchKernelGGL((mfma3d_kernel<Op, false>), dim3(nbm), dim3(64), 0, stream, g3, op);
            done = true;
          }
        }
        if (!done) {
          const unsigned nb3 = (unsigned)sweep3d_chunks<SW_TX, SW_TY>(g3, NF, sweep_waves);
          hipLaunchKernelGGL((tile3d_kernel<K, T, BLK, Op, SW_TX, SW_TY>), dim3(nb3), dim3(64), 0, stream, g3, op);
        }
      }
    }
    check_launch();
    if (profiling) {
      SMG_HIP(hipEventRecord(eb, stream));
      char key[160];
      std::snprintf(key, sizeof(key), "%s/v%d/blk%d/%s/%dx%dx%d", Op::NAME, Op::VARIANT, BLK,
                    std::is_same<T, double>::value ? "f64" : "f32", g.n[0], g.n[1], g.n[2]);
      constexpr bool NU = (BLK & (BLK_A | BLK_MASS | BLK_B)) != 0, NP = (BLK & (BLK_BT | BLK_C)) != 0;
      constexpr bool OU = (BLK & (BLK_A | BLK_MASS | BLK_BT)) != 0, OP = (BLK & (BLK_B | BLK_C)) != 0;
      const double bytes = op.algo_bytes(NU, NP, OU, OP, (double)(DIM * g.Nv), (double)g.Np);
      prof.push_back(ProfRec{key, ea, eb, bytes});
    }
  }

  // General (vertex-given) cells: 2^d colour launches accumulate the cell
  // sums into the level scratch, then one pass applies Dirichlet rows and
  // the epilogue functor.
  template <typename T, int BLK, class Op>
  void gen_tile(const LevelGeom<T, DIM, K> &g, const Op &op) {
    GenGeo<T> gg;
    std::memset(&gg, 0, sizeof(gg));
    for (int a = 0; a < 3; ++a) {
      gg.n[a] = g.n[a];
      gg.vd[a] = g.vd[a];
      gg.pd[a] = g.pd[a];
    }
    gg.Nv = g.Nv;
    gg.Np = g.Np;
    gg.mu = g.mu;
    gg.gr = g.gr;
    gg.cp = g.cp;
    gg.mu_cell = g.mu_cell;
    gg.verts = g.verts;
    gg.sym = desc.form == SMG_FORM_EPS ? 1 : 0;
    gg.tu = g.gs;
    gg.tp = g.gs + (int64_t)DIM * g.Nv;
    const int64_t n_all = (int64_t)DIM * g.Nv + g.Np;
    if (g.cbu != nullptr) {
      // every cell in one launch, results per cell; the epilogue sums them
      // per node (two launches instead of 2^d colours + epilogue)
      constexpr int NN = DIM == 3 ? (K + 1) * (K + 1) * (K + 1) : (K + 1) * (K + 1);
      constexpr int CPB = 64 / NN;
      gg.step = 1;
      for (int a = 0; a < 3; ++a) {
        gg.off[a] = 0;
        gg.ncol[a] = a < DIM ? gg.n[a] : 1;
      }
      gg.cbu = g.cbu;
      gg.cbp = g.cbp;
      const int64_t ncells = (int64_t)gg.n[0] * gg.n[1] * (DIM == 3 ? gg.n[2] : 1);
      if constexpr (DIM == 3) {
        if (gen3_lines && gg.Nv + gg.Np < ((int64_t)1 << 31)) {
          // line layout (CPW cells per wave), then the gather with one
          // thread per node (32-bit node indices)
          hipLaunchKernelGGL((gen3_line_kernel<K, T, BLK, Op>), dim3((unsigned)gen3_blocks<K>(gg)), dim3(64), 0, stream,
                             gg, op);
          check_launch();
          constexpr bool OU = (BLK & (BLK_A | BLK_MASS | BLK_BT)) != 0, OP = (BLK & (BLK_B | BLK_C)) != 0;
          const int64_t items = (OU ? gg.Nv : 0) + (OP ? gg.Np : 0);
          hipLaunchKernelGGL((gen3_gather_kernel<K, T, BLK, Op>), dim3((unsigned)((items + 255) / 256)), dim3(256), 0,
                             stream, gg, op, make_fastdiv((uint32_t)gg.vd[0]), make_fastdiv((uint32_t)gg.vd[1]),
                             make_fastdiv((uint32_t)gg.pd[0]), make_fastdiv((uint32_t)gg.pd[1]));
          check_launch();
          return;
        } else {
          hipLaunchKernelGGL((gen_apply_kernel<DIM, K, T, BLK, Op>), dim3((unsigned)((ncells + CPB - 1) / CPB)),
                             dim3(64), 0, stream, gg, op);
        }
      } else {
        hipLaunchKernelGGL((gen_apply_kernel<DIM, K, T, BLK, Op>), dim3((unsigned)((ncells + CPB - 1) / CPB)), dim3(64),
                           0, stream, gg, op);
      }
      check_launch();
      hipLaunchKernelGGL((gen_gather_epilogue_kernel<DIM, K, T, BLK, Op>), dim3(grid_for(n_all)), dim3(VB), 0, stream,
                         gg, op);
      check_launch();
      return;
    }
    gen_accumulate<T, BLK, Op>(gg, op);
    hipLaunchKernelGGL((gen_epilogue_kernel<DIM, T, BLK, Op>), dim3(grid_for(n_all)), dim3(VB), 0, stream, gg, op);
    check_launch();
  }

  // cell sums of all 2^d colours into gg.tu / gg.tp (zeroed first)
  template <typename T, int BLK, class Op>
  void gen_accumulate(GenGeo<T> &gg, const Op &op) {
    const int64_t n_all = (int64_t)DIM * gg.Nv + gg.Np;
    vset<T>(gg.tu, (T)0, n_all);
    gg.step = 2;
    gg.cbu = nullptr;
    gg.cbp = nullptr;
    constexpr int NN = DIM == 3 ? (K + 1) * (K + 1) * (K + 1) : (K + 1) * (K + 1);
    constexpr int CPB = 64 / NN;
    for (int colour = 0; colour < (1 << DIM); ++colour) {
      int64_t ncells = 1;
      for (int a = 0; a < 3; ++a) {
        gg.off[a] = a < DIM ? (colour >> a) & 1 : 0;
        gg.ncol[a] = a < DIM ? (gg.n[a] - gg.off[a] + 1) / 2 : 1;
        ncells *= gg.ncol[a];
      }
      if (ncells == 0) continue;
      const unsigned nb = (unsigned)((ncells + CPB - 1) / CPB);
      hipLaunchKernelGGL((gen_apply_kernel<DIM, K, T, BLK, Op>), dim3(nb), dim3(64), 0, stream, gg, op);
      check_launch();
    }
  }

  // finest-level vertex coordinates for the general-cell kernels (box meshes:
  // the lattice of the box, built on first use)
  void ensure_vertices() {
    if (lv[L].w64.verts) return;
    const LevelInfo &I = lv[L];
    const int nz = DIM == 3 ? I.n[2] + 1 : 1;
    std::vector<double> hv((size_t)(I.n[0] + 1) * (I.n[1] + 1) * nz * DIM);
    size_t o = 0;
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j <= I.n[1]; ++j)
        for (int i = 0; i <= I.n[0]; ++i) {
          const int ii[3] = {i, j, k};
          for (int a = 0; a < DIM; ++a) hv[o++] = desc.box_lo[a] + I.h[a] * ii[a];
        }
    lv[L].w64.verts = dalloc<double>((int64_t)hv.size());
    SMG_HIP(hipMemcpyAsync(lv[L].w64.verts, hv.data(), hv.size() * sizeof(double), hipMemcpyHostToDevice, stream));
    SMG_HIP(hipStreamSynchronize(stream));
  }

  // adjoint-state gradients on the finest level (FP64)
  void gradient(const double *x, const double *lam, double *g_logmu, double *g_f) override {
    ensure_vertices();
    auto g = geom<double>(L);
    GenGeo<double> gg;
    std::memset(&gg, 0, sizeof(gg));
    for (int a = 0; a < 3; ++a) {
      gg.n[a] = g.n[a];
      gg.vd[a] = g.vd[a];
      gg.pd[a] = g.pd[a];
    }
    gg.Nv = g.Nv;
    gg.Np = g.Np;
    gg.mu = g.mu;
    gg.mu_cell = g.mu_cell;
    gg.verts = lv[L].w64.verts;
    gg.sym = desc.form == SMG_FORM_EPS ? 1 : 0;
    gg.tu = g.gs;
    gg.tp = g.gs + (int64_t)DIM * g.Nv;
    if (g_logmu) {
      constexpr int NN = DIM == 3 ? (K + 1) * (K + 1) * (K + 1) : (K + 1) * (K + 1);
      constexpr int CPB = 64 / NN;
      const int64_t ncells = (int64_t)g.n[0] * g.n[1] * g.n[2];
      hipLaunchKernelGGL((gen_grad_logmu_kernel<DIM, K>), dim3((unsigned)((ncells + CPB - 1) / CPB)), dim3(64), 0,
                         stream, gg, x, lam, g_logmu);
      check_launch();
    }
    if (g_f) {
      // M_v (Z lam_u) on every node: cell sums of the mass form, no Dirichlet rows
      gen_accumulate<double, BLK_MASS>(gg, OpApply<double>{lam, nullptr, nullptr, nullptr});
      hipLaunchKernelGGL((k_copy<double, double>), dim3(grid_for((int64_t)DIM * g.Nv)), dim3(VB), 0, stream, g_f,
                         (const double *)gg.tu, (i64)((int64_t)DIM * g.Nv));
      check_launch();
    }
  }

  // Diagonals of general cells by probing with the operator kernels:
  // velocity nodes whose lattice coordinates agree modulo k+1 share no cell,
  // so A e (e = indicator of one residue class) equals diag(A) on that class;
  // pressure nodes whose coordinates agree modulo 3 (k = 2) / 5 (k = 3)
  // share no velocity node of their cells, so B D_A^-1 B^T e equals
  // diag(B D_A^-1 B^T) there (and M_p e equals diag(M_p)).
  void probe_diagonals(int l) {
    LevelInfo &I = lv[l];
    auto g = geom<double>(l);
    auto gu = geom<double>(l, true);
    double *e = lz[0], *q = lz[1], *s = lz[2], *mpe = lz[3];
    const int mv = K + 1;
    const int ncv = DIM == 3 ? mv * mv * mv : mv * mv;
    // the deformation-rate form couples the components at a node: probe one
    // component at a time there
    const bool per_comp = desc.form == SMG_FORM_EPS;
    for (int comp = 0; comp < (per_comp ? DIM : 1); ++comp)
      for (int col = 0; col < ncv; ++col) {
        const int c0 = col % mv, c1 = (col / mv) % mv, c2 = DIM == 3 ? col / (mv * mv) : 0;
        hipLaunchKernelGGL((k_probe_fill<DIM>), dim3(grid_for(I.N)), dim3(VB), 0, stream, e, I.Nv, I.Np,
                           per_comp ? 2 + comp : 0, mv, c0, c1, c2, I.vd[0], I.vd[1], I.pd[0], I.pd[1]);
        check_launch();
        tile<double, BLK_A>(g, OpApply<double>{e, nullptr, q, nullptr});
        const int64_t o = per_comp ? comp * I.Nv : 0;
        hipLaunchKernelGGL((k_probe_take<DIM>), dim3(grid_for(I.Nu)), dim3(VB), 0, stream, I.DA + o,
                           (const double *)(q + o), (const double *)nullptr, 0.0, I.Nv, per_comp ? 1 : DIM, mv, c0, c1,
                           c2, I.vd[0], I.vd[1]);
        check_launch();
      }
    const int mp = K == 2 ? 3 : 5;
    const int ncp = DIM == 3 ? mp * mp * mp : mp * mp;
    const bool schur_p = desc.schur_diag == SMG_SCHUR_P;
    for (int col = 0; col < ncp; ++col) {
      const int c0 = col % mp, c1 = (col / mp) % mp, c2 = DIM == 3 ? col / (mp * mp) : 0;
      hipLaunchKernelGGL((k_probe_fill<DIM>), dim3(grid_for(I.N)), dim3(VB), 0, stream, e, I.Nv, I.Np, 1, mp, c0, c1,
                         c2, I.vd[0], I.vd[1], I.pd[0], I.pd[1]);
      check_launch();
      const double *ep = e + I.Nu;
      // M_p e (unit c_p)
      tile<double, BLK_C | BLK_CPLUS>(gu, OpApply<double>{nullptr, ep, nullptr, mpe});
      if (schur_p) {
        // D~_S_p = diag(M_p) (+ c_p diag(M_p))
        hipLaunchKernelGGL((k_probe_take<DIM>), dim3(grid_for(I.Np)), dim3(VB), 0, stream, I.DS, (const double *)mpe,
                           (const double *)mpe, desc.c_pressure, I.Np, 1, mp, c0, c1, c2, I.pd[0], I.pd[1]);
      } else {
        // D~_S_d = diag(B D_A^-1 B^T) (+ c_p diag(M_p))
        tile<double, BLK_BT>(g, OpApply<double>{nullptr, ep, q, nullptr});
        hipLaunchKernelGGL((k_div_by<double>), dim3(grid_for(I.Nu)), dim3(VB), 0, stream, q, (const double *)I.DA, I.Nu);
        check_launch();
        tile<double, BLK_B>(g, OpApply<double>{q, nullptr, nullptr, s});
        hipLaunchKernelGGL((k_probe_take<DIM>), dim3(grid_for(I.Np)), dim3(VB), 0, stream, I.DS, (const double *)s,
                           (const double *)mpe, desc.c_pressure, I.Np, 1, mp, c0, c1, c2, I.pd[0], I.pd[1]);
      }
      check_launch();
    }
  }

  // D~_S_loc on vertex-given cells (Sec. 3.3.1): cell contributions by
  // quadrature, then one fixed-order sum per pressure node (replaces the D~_S
  // the probing left).
  void local_schur_diagonal_general(int l) {
    LevelInfo &I = lv[l];
    auto g = geom<double>(l);
    GenGeo<double> gg;
    std::memset(&gg, 0, sizeof(gg));
    for (int a = 0; a < 3; ++a) {
      gg.n[a] = g.n[a];
      gg.vd[a] = g.vd[a];
      gg.pd[a] = g.pd[a];
    }
    gg.Nv = g.Nv;
    gg.Np = g.Np;
    gg.mu = g.mu;
    gg.gr = g.gr;
    gg.cp = g.cp;
    gg.mu_cell = g.mu_cell;
    gg.verts = g.verts;
    constexpr int NPN = DIM == 3 ? K * K * K : K * K;
    const int64_t nt = (int64_t)g.n[0] * g.n[1] * (DIM == 3 ? g.n[2] : 1) * NPN;
    if (nt > I.N) throw Error{SMG_EINVAL, "local Schur diagonal: cell contributions exceed the work vector"};
    double *contrib = lz[2];
    hipLaunchKernelGGL((k_schur_loc_cells<DIM, K>), dim3(grid_for(nt)), dim3(VB), 0, stream, gg, desc.c_pressure,
                       contrib);
    check_launch();
    hipLaunchKernelGGL((k_schur_loc_gather<DIM, K>), dim3(grid_for(I.Np)), dim3(VB), 0, stream, gg,
                       (const double *)contrib, I.DS);
    check_launch();
  }

  // D_S~ = diag(B A_hat^-1 B^T) (+ c_p diag(M_p)), A_hat^-1 = sigma Cheb(A, D_A, k_A)
  // (Sec. 3.3.1, the diagonal the cheaper choices approximate), by probing:
  // B^T e_j lives on the cells around pressure node j, each of the k_A
  // applications of A inside Cheb widens that by one cell layer, and B e_i
  // reads the cells around node i; pressure nodes of one class are
  // (k - 1)(k_A + 3) + 1 lattice steps apart in some direction, which is more
  // than that reach, so the probe returns the diagonal entry on its class.
  // Needs D_A, beta_A and the level's FP64 work vectors.
  void exact_schur_diagonal(int l) {
    LevelInfo &I = lv[l];
    Work<double> &W = work<double>(l);
    auto g = geom<double>(l);
    auto gu = geom<double>(l, true);
    double *e = lz[0], *s = lz[2], *mpe = lz[3];
    const int mp = (K - 1) * (desc.cheb_deg_A + 3) + 1;
    const int ncp = DIM == 3 ? mp * mp * mp : mp * mp;
    for (int col = 0; col < ncp; ++col) {
      const int c0 = col % mp, c1 = (col / mp) % mp, c2 = DIM == 3 ? col / (mp * mp) : 0;
      hipLaunchKernelGGL((k_probe_fill<DIM>), dim3(grid_for(I.N)), dim3(VB), 0, stream, e, I.Nv, I.Np, 1, mp, c0, c1,
                         c2, I.vd[0], I.vd[1], I.pd[0], I.pd[1]);
      check_launch();
      const double *ep = e + I.Nu;
      tile<double, BLK_C | BLK_CPLUS>(gu, OpApply<double>{nullptr, ep, nullptr, mpe});
      tile<double, BLK_BT>(g, OpApply<double>{nullptr, ep, W.q, nullptr});
      cheb_A<double>(l, W.q, nullptr, W.w, sigma);
      tile<double, BLK_B>(g, OpApply<double>{W.w, nullptr, nullptr, s});
      hipLaunchKernelGGL((k_probe_take<DIM>), dim3(grid_for(I.Np)), dim3(VB), 0, stream, I.DS, (const double *)s,
                         (const double *)mpe, desc.c_pressure, I.Np, 1, mp, c0, c1, c2, I.pd[0], I.pd[1]);
      check_launch();
    }
    hipLaunchKernelGGL((k_reciprocal<double>), dim3(grid_for(I.Np)), dim3(VB), 0, stream, W.dinvS, (const double *)I.DS, (i64)I.Np);
    check_launch();
    hipLaunchKernelGGL((k_reciprocal<float>), dim3(grid_for(I.Np)), dim3(VB), 0, stream, work<float>(l).dinvS, (const double *)I.DS, (i64)I.Np);
    check_launch();
  }

  bool has_c() const { return desc.c_pressure != 0.0; }

  template <typename T>
  void vset(T *y, T v, int64_t n) {
    if (rec) rec_add(LSet<T>{y, v, (i64)n}, grid_for(n));
    else hipLaunchKernelGGL((k_set<T>), dim3(grid_for(n)), dim3(VB), 0, stream, y, v, (i64)n);
    check_launch();
  }

  // append a launch functor to the recorder (batched execution)
  template <class L>
  void rec_add(const L &l, unsigned nb) {
    static_assert(std::is_trivially_copyable<L>::value, "launch functors are copied as bytes");
    LaunchRec r;
    r.tag = rec->tag;
    r.kernel = (const void *)&k_packed<L>;
    r.nblocks = nb;
    r.threads = L::THREADS;
    r.align = alignof(L);
    r.bytes.resize(sizeof(L));
    std::memcpy(r.bytes.data(), &l, sizeof(L));
    rec->recs.push_back(std::move(r));
  }

  // ---------------------------------------------------------------- blocks
  template <typename T>
  void vmult_t(int l, const T *x, T *y) {
    auto g = geom<T>(l);
    OpApply<T> op{x, x + lv[l].Nu, y, y + lv[l].Nu};
    if (has_c()) tile<T, BLK_A | BLK_BT | BLK_B | BLK_C>(g, op);
    else tile<T, BLK_A | BLK_BT | BLK_B>(g, op);
  }

  // bytes of the per-cell results of one operator application on level l
  // (vertex-given cells; 0 for the box-cell kernels), the pressure part
  // starting at a 256-byte boundary
  int64_t vmult_scratch_bytes(int l, int dt) const override {
    if (!gen_op) return 0;
    constexpr int64_t NN = DIM == 3 ? (K + 1) * (K + 1) * (K + 1) : (K + 1) * (K + 1);
    constexpr int64_t NPN = DIM == 3 ? K * K * K : K * K;
    const int64_t es = dt == SMG_F32 ? 4 : 8;
    const int64_t nc = (int64_t)lv[l].n[0] * lv[l].n[1] * (DIM == 3 ? lv[l].n[2] : 1);
    return (nc * DIM * NN * es + 255) / 256 * 256 + nc * NPN * es;
  }

  void vmult_scratch(int l, int dt, const void *x, void *y, void *scratch) override {
    const bool saved = profiling;   // kernel timing would create events
    profiling = false;
    try {
      if (dt == SMG_F32) vmult_scratch_t<float>(l, (const float *)x, (float *)y, scratch);
      else vmult_scratch_t<double>(l, (const double *)x, (double *)y, scratch);
    } catch (...) {
      profiling = saved;
      throw;
    }
    profiling = saved;
  }

  template <typename T>
  void vmult_scratch_t(int l, const T *x, T *y, void *scratch) {
    auto g = geom<T>(l);
    if (gen_op) {
      constexpr int64_t NN = DIM == 3 ? (K + 1) * (K + 1) * (K + 1) : (K + 1) * (K + 1);
      const int64_t nc = (int64_t)lv[l].n[0] * lv[l].n[1] * (DIM == 3 ? lv[l].n[2] : 1);
      g.cbu = (T *)scratch;
      g.cbp = (T *)((char *)scratch + (nc * DIM * NN * (int64_t)sizeof(T) + 255) / 256 * 256);
    }
    OpApply<T> op{x, x + lv[l].Nu, y, y + lv[l].Nu};
    if (has_c()) tile<T, BLK_A | BLK_BT | BLK_B | BLK_C>(g, op);
    else tile<T, BLK_A | BLK_BT | BLK_B>(g, op);
  }

  template <typename T>
  void residual_t(int l, const T *x, const T *b, T *r) {
    auto g = geom<T>(l);
    const int64_t nu = lv[l].Nu;
    OpResidual<T> op{x, x + nu, b, b + nu, r, r + nu};
    if (has_c()) tile<T, BLK_A | BLK_BT | BLK_B | BLK_C>(g, op);
    else tile<T, BLK_A | BLK_BT | BLK_B>(g, op);
  }

  // Non-homogeneous Dirichlet data by lifting: b <- b - K u~ (Dirichlet
  // columns kept, u~ = u_d on the Dirichlet nodes, 0 elsewhere), Dirichlet
  // rows of b set to 0; the solution of K x0 = b plus u~ solves the problem
  // with x = u_d on the boundary.
  template <typename T>
  void lift_t(int l, const T *ud, T *b) {
    const LevelInfo &I = lv[l];
    Work<T> &W = work<T>(l);
    hipLaunchKernelGGL((k_dirichlet_values<T, DIM>), dim3(grid_for(I.Nu)), dim3(VB), 0, stream, ud, W.ru, (i64)I.Nv,
                       I.vd[0], I.vd[1], I.vd[2], 0);
    check_launch();
    auto g = geom<T>(l);
    tile<T, BLK_A | BLK_B>(g, OpLift<T>{W.ru, b, b + I.Nu, b, b + I.Nu});
  }

  template <typename T>
  void insert_dirichlet_t(int l, const T *ud, T *x) {
    const LevelInfo &I = lv[l];
    hipLaunchKernelGGL((k_dirichlet_values<T, DIM>), dim3(grid_for(I.Nu)), dim3(VB), 0, stream, ud, x, (i64)I.Nv,
                       I.vd[0], I.vd[1], I.vd[2], 1);
    check_launch();
  }

  template <typename T>
  void block_t(int l, int blk, const T *x, T *y) {
    auto g = geom<T>(l);
    switch (blk) {
      case SMG_BLOCK_K: vmult_t<T>(l, x, y); break;
      case SMG_BLOCK_A: tile<T, BLK_A>(g, OpApply<T>{x, nullptr, y, nullptr}); break;
      case SMG_BLOCK_BT: tile<T, BLK_BT>(g, OpApply<T>{nullptr, x, y, nullptr}); break;
      case SMG_BLOCK_B: tile<T, BLK_B>(g, OpApply<T>{x, nullptr, nullptr, y}); break;
      case SMG_BLOCK_MP:
        tile<T, BLK_C | BLK_CPLUS>(geom<T>(l, true), OpApply<T>{nullptr, x, nullptr, y});
        break;
      case SMG_BLOCK_MASS: {
        auto gm = g;
        tile<T, BLK_MASS>(gm, OpMass<T>{x, y});
        break;
      }
      default: throw Error{SMG_EINVAL, "unknown block"};
    }
  }

  // --------------------------------------------------------- Chebyshev (A)
  // out = base + s * Cheb(A, D_A, k_A) r   (Sec. 3.3.1; three-term recurrence)
  // i0 > 0: continue after a first step done elsewhere (its r, x, d in the
  // level's Chebyshev state vectors)
  template <typename T>
  void cheb_A(int l, const T *r, const T *base, T *out, double s, int i0 = 0) {
    Work<T> &W = work<T>(l);
    const int64_t nu = lv[l].Nu;
    const double beta = lv[l].beta_A, theta = 0.75 * beta, delta = 0.25 * beta, s1 = theta / delta;
    const int k = desc.cheb_deg_A;
    if (k == 0) {
      if (rec) rec_add(LJacobi<T>{out, base, (T)(s / theta), W.dinvA, r, (i64)nu}, grid_for(nu));
      else hipLaunchKernelGGL((k_jacobi<T>), dim3(grid_for(nu)), dim3(VB), 0, stream, out, base, (T)(s / theta), W.dinvA, r, (i64)nu);
      check_launch();
      return;
    }
    auto g = geom<T>(l);
    double rho = 1.0 / s1;
    for (int i = 0; i < i0; ++i) rho = 1.0 / (2.0 * s1 - rho);
    for (int i = i0; i < k; ++i) {
      const double rn = 1.0 / (2.0 * s1 - rho);
      OpChebA<T, true, true> o;  // field holder; copied into the right instantiation below
      std::memset(&o, 0, sizeof(o));
      o.rin = (i == 0) ? r : W.cr;
      o.dinv = W.dinvA;
      o.d = W.cd[i % 2];
      o.x = W.cx;
      o.r_out = W.cr;
      o.x_out = W.cx;
      o.d_out = W.cd[(i + 1) % 2];
      o.base = base;
      o.out = out;
      o.inv_theta = (T)(1.0 / theta);
      o.c1 = (T)(rn * rho);
      o.c2 = (T)(2.0 * rn / delta);
      o.s = (T)s;
      const bool first = i == 0, last = i == k - 1;
      if (first && last) tile<T, BLK_A>(g, cast_op<OpChebA<T, true, true>>(o));
      else if (first) tile<T, BLK_A>(g, cast_op<OpChebA<T, true, false>>(o));
      else if (last) tile<T, BLK_A>(g, cast_op<OpChebA<T, false, true>>(o));
      else tile<T, BLK_A>(g, cast_op<OpChebA<T, false, false>>(o));
      rho = rn;
    }
  }

  // out = base + s * Cheb(A, D_A, k_A) r where r comes from op1 (q = B^T d
  // of OpGrad, or the residual of OpResidual), the application of op1 and the
  // first Chebyshev step in one launch (2D box levels of at most
  // fuse2d_max_n cells per direction).  Returns false, launching nothing,
  // where the fused kernel does not apply; the caller then runs op1 and
  // cheb_A separately.
  template <typename T, class Op1>
  bool cheb_A_fused(int l, const Op1 &op1, const T *base, T *out, double s) {
    if constexpr (DIM != 2) {
      return false;
    } else {
      const int k = desc.cheb_deg_A;
      if (general || k < 1 || fuse2d_max_n <= 0 || std::max(lv[l].n[0], lv[l].n[1]) > fuse2d_max_n) return false;
      Work<T> &W = work<T>(l);
      const double beta = lv[l].beta_A, theta = 0.75 * beta, delta = 0.25 * beta, s1 = theta / delta;
      const double rho = 1.0 / s1, rn = 1.0 / (2.0 * s1 - rho);
      OpChebA<T, true, true> o;
      std::memset(&o, 0, sizeof(o));
      o.dinv = W.dinvA;
      o.r_out = W.cr;
      o.x_out = W.cx;
      o.d_out = W.cd[1];
      o.base = base;
      o.out = out;
      o.inv_theta = (T)(1.0 / theta);
      o.c1 = (T)(rn * rho);
      o.c2 = (T)(2.0 * rn / delta);
      o.s = (T)s;
      auto g = geom<T>(l);
      const Geo2<T> g2 = geo2<T>(g, 5);
      const unsigned nb = (unsigned)(g2.tiles[0] * g2.tiles[1] * 2);
      hipEvent_t ea = nullptr, eb = nullptr;
      if (profiling) {
        ea = next_event();
        eb = next_event();
        SMG_HIP(hipEventRecord(ea, stream));
      }
      const bool wg = wgf2d_min_n > 0 && std::max(lv[l].n[0], lv[l].n[1]) >= wgf2d_min_n;
      if (wg) {
        if (wgf2d_shape == 22) fused_wg_launch<T, Op1, 2, 2>(g, op1, o, k);
        else if (wgf2d_shape == 44) fused_wg_launch<T, Op1, 4, 4>(g, op1, o, k);
        else fused_wg_launch<T, Op1, 4, 2>(g, op1, o, k);
      } else if (rec) {
        if (k == 1) rec_add(LFused2<K, T, Op1, true>{g2, op1, o}, nb);
        else rec_add(LFused2<K, T, Op1, false>{g2, op1, cast_op<OpChebA<T, true, false>>(o)}, nb);
      } else if (k == 1)
        hipLaunchKernelGGL((wave2d_fused_kernel<K, T, Op1, true>), dim3(nb), dim3(64), 0, stream, g2, op1, o);
      else
        hipLaunchKernelGGL((wave2d_fused_kernel<K, T, Op1, false>), dim3(nb), dim3(64), 0, stream, g2, op1,
                           cast_op<OpChebA<T, true, false>>(o));
      check_launch();
      if (profiling) {
        SMG_HIP(hipEventRecord(eb, stream));
        char key[160];
        std::snprintf(key, sizeof(key), "%s+cheb_A/v%d/%s/%s/%dx%dx%d", Op1::NAME, k == 1 ? 3 : 1, wg ? "fusedwg" : "fused",
                      std::is_same<T, double>::value ? "f64" : "f32", g.n[0], g.n[1], g.n[2]);
        // algorithmic bytes, every vector read or written once: the producer's
        // inputs (residual: u, p, f; B^T d: d), then D_A^-1, the base unless
        // it is the residual's u, and the output (k = 1), or the recurrence's
        // r, x, d and D_A^-1 (k > 1)
        const double nu = (double)(DIM * g.Nv), np = (double)g.Np;
        constexpr bool RES = std::is_same<Op1, OpResidual<T>>::value;
        bool base_read = base != nullptr;
        if constexpr (RES) base_read = base_read && (const void *)base != (const void *)op1.xu;
        const double bytes =
            sizeof(T) * ((RES ? 2 * nu + np : np) + nu * (k == 1 ? (base_read ? 3 : 2) : 4));
        prof.push_back(ProfRec{key, ea, eb, bytes});
      }
      if (k > 1) cheb_A<T>(l, nullptr, base, out, s, 1);
      return true;
    }
  }

  // The fused pair on workgroups of WX x WY waves (2D box levels).
  template <typename T, class Op1, int WX, int WY>
  void fused_wg_launch(const LevelGeom<T, DIM, K> &g, const Op1 &op1, const OpChebA<T, true, true> &o, int k) {
    Geo2<T> g2 = geo2<T>(g, 5);
    g2.tiles[0] = (g.n[0] + 8 * WX - 4) / (8 * WX - 3);
    g2.tiles[1] = (g.n[1] + 8 * WY - 4) / (8 * WY - 3);
    const unsigned nb = (unsigned)(g2.tiles[0] * g2.tiles[1] * 2);
    if (rec) {
      if (k == 1) rec_add(LFused2Wg<K, T, Op1, true, WX, WY>{g2, op1, o}, nb);
      else rec_add(LFused2Wg<K, T, Op1, false, WX, WY>{g2, op1, cast_op<OpChebA<T, true, false>>(o)}, nb);
    } else if (k == 1) {
      hipLaunchKernelGGL((wg2d_fused_kernel<K, T, Op1, true, WX, WY>), dim3(nb), dim3(64 * WX * WY), 0, stream, g2,
                         op1, o);
    } else {
      hipLaunchKernelGGL((wg2d_fused_kernel<K, T, Op1, false, WX, WY>), dim3(nb), dim3(64 * WX * WY), 0, stream,
                         g2, op1, cast_op<OpChebA<T, true, false>>(o));
    }
  }

  template <class To, class From>
  static To cast_op(const From &f) {
    static_assert(sizeof(To) == sizeof(From), "op layout");
    To t;
    std::memcpy(&t, &f, sizeof(To));
    return t;
  }

  // ------------------------------------------------------- Chebyshev (S~)
  // dp = tau * Cheb(S~, D~_S, k_S) rp, and p += dp when p != nullptr.
  template <typename T>
  void cheb_S(int l, const T *rp, T *dp, T *p) {
    Work<T> &W = work<T>(l);
    const int64_t np = lv[l].Np;
    const double beta = lv[l].beta_S, theta = 0.75 * beta, delta = 0.25 * beta, s1 = theta / delta;
    const int k = desc.cheb_deg_S;
    if (k == 0) {
      if (rec && p)
        rec_add(LJacobiUpdate<T>{p, dp, (T)(tau / theta), W.dinvS, rp, (i64)np}, grid_for(np));
      else if (rec)
        rec_add(LJacobi<T>{dp, (const T *)nullptr, (T)(tau / theta), W.dinvS, rp, (i64)np}, grid_for(np));
      else if (p)
        hipLaunchKernelGGL((k_jacobi_update<T>), dim3(grid_for(np)), dim3(VB), 0, stream, p, dp, (T)(tau / theta), W.dinvS, rp, (i64)np);
      else
        hipLaunchKernelGGL((k_jacobi<T>), dim3(grid_for(np)), dim3(VB), 0, stream, dp, (const T *)nullptr, (T)(tau / theta), W.dinvS, rp, (i64)np);
      check_launch();
      return;
    }
    auto g = geom<T>(l);
    double rho = 1.0 / s1;
    for (int i = 0; i < k; ++i) {
      const double rn = 1.0 / (2.0 * s1 - rho);
      const bool first = i == 0, last = i == k - 1;
      // q = B^T d_i, w = A_hat^-1 q
      if (first) {
        const OpGrad<T, true> og{rp, W.dinvS, nullptr, (T)(1.0 / theta), W.q};
        if (!cheb_A_fused<T>(l, og, (const T *)nullptr, W.w, sigma)) {
          tile<T, BLK_BT>(g, og);
          cheb_A<T>(l, W.q, nullptr, W.w, sigma);
        }
      } else {
        const OpGrad<T, false> og{nullptr, nullptr, W.sd[i % 2], (T)0, W.q};
        if (!cheb_A_fused<T>(l, og, (const T *)nullptr, W.w, sigma)) {
          tile<T, BLK_BT>(g, og);
          cheb_A<T>(l, W.q, nullptr, W.w, sigma);
        }
      }
      // t = B w + C d_i and the recurrence
      OpChebS<T, true, true> o;
      std::memset(&o, 0, sizeof(o));
      o.w = W.w;
      o.rin = first ? rp : W.sr;
      o.dinv_s = W.dinvS;
      o.d = W.sd[i % 2];
      o.x = W.sx;
      o.r_out = W.sr;
      o.x_out = W.sx;
      o.d_out = W.sd[(i + 1) % 2];
      o.p = p;
      o.dp = dp;
      o.inv_theta = (T)(1.0 / theta);
      o.c1 = (T)(rn * rho);
      o.c2 = (T)(2.0 * rn / delta);
      o.tau = (T)tau;
      if (first && last) div_cheb<T>(g, cast_op<OpChebS<T, true, true>>(o));
      else if (first) div_cheb<T>(g, cast_op<OpChebS<T, true, false>>(o));
      else if (last) div_cheb<T>(g, cast_op<OpChebS<T, false, true>>(o));
      else div_cheb<T>(g, cast_op<OpChebS<T, false, false>>(o));
      rho = rn;
    }
  }

  template <typename T, class Op>
  void div_cheb(const LevelGeom<T, DIM, K> &g, const Op &op) {
    if (has_c()) tile<T, BLK_B | BLK_C | BLK_CPLUS>(g, op);
    else tile<T, BLK_B>(g, op);
  }

  // out = S~ d = B A_hat^-1 B^T d + C d
  template <typename T>
  void S_tilde(int l, const T *d, T *out) {
    Work<T> &W = work<T>(l);
    auto g = geom<T>(l);
    tile<T, BLK_BT>(g, OpGrad<T, false>{nullptr, nullptr, d, (T)0, W.q});
    cheb_A<T>(l, W.q, nullptr, W.w, sigma);
    OpApply<T> op{W.w, d, nullptr, out};
    if (has_c()) tile<T, BLK_B | BLK_C | BLK_CPLUS>(g, op);
    else tile<T, BLK_B>(g, op);
  }

  // ------------------------------------------------------ Uzawa smoother
  // One inexact symmetric Uzawa step in the form consistent with the compact
  // form x <- x + K_hat^-1 (b - K x) of Sec. 3.3.1:
  //   u_hat = u + A_hat^-1 (f - A u - B^T p)
  //   dp    = S_hat^-1 (B u_hat - C p - g),   p <- p + dp
  //   u     = u_hat - A_hat^-1 B^T dp
  // velocity_update_t forms the first line (zero_init: u = 0, p = 0, the
  // residual is f), uzawa_step the whole step.
  template <typename T>
  void velocity_update_t(int l, const T *x, const T *b, T *uhat, bool zero_init = false) {
    Work<T> &W = work<T>(l);
    const int64_t nu = lv[l].Nu;
    const T *u = x, *p = x + nu, *f = b;
    if (zero_init) {
      cheb_A<T>(l, f, nullptr, uhat, sigma);
    } else {
      const OpResidual<T> op{u, p, f, nullptr, W.ru, nullptr};
      if (!cheb_A_fused<T>(l, op, u, uhat, sigma)) {
        tile<T, BLK_A | BLK_BT>(geom<T>(l), op);
        cheb_A<T>(l, W.ru, u, uhat, sigma);
      }
    }
  }

  template <typename T>
  void uzawa_step(int l, T *x, const T *b, bool zero_init) {
    Work<T> &W = work<T>(l);
    const int64_t nu = lv[l].Nu;
    T *u = x, *p = x + nu;
    const T *gp = b + nu;
    auto g = geom<T>(l);
    velocity_update_t<T>(l, x, b, W.uhat, zero_init);
    if (uzawa_tail_fused3<T>(l, u, p, gp)) return;
    OpDivResidual<T> od{W.uhat, p, gp, W.rp};
    if (has_c()) tile<T, BLK_B | BLK_C>(g, od);
    else tile<T, BLK_B>(g, od);
    cheb_S<T>(l, W.rp, W.dp, p);
    const OpGrad<T, false> og{nullptr, nullptr, W.dp, (T)0, W.q};
    if (!cheb_A_fused<T>(l, og, (const T *)W.uhat, u, -sigma)) {
      tile<T, BLK_BT>(g, og);
      cheb_A<T>(l, W.q, W.uhat, u, -sigma);
    }
  }

  // The rest of an Uzawa step after u_hat, in two launches of the
  // three-stage kernel (2D box levels of at most fuse3_2d_max_n cells per
  // direction, k_S = 1, k_A >= 1):
  //   1. r_p = B u_hat - C p - g, d_0 = D~_S^-1 r_p / theta_S,
  //      w = Cheb(A, D_A, k_A) B^T d_0;
  //   2. dp = the Chebyshev step for S~ from w and d_0, p += dp,
  //      u = u_hat - sigma Cheb(A, D_A, k_A) B^T dp.
  // Returns false, launching nothing, where it does not apply.
  template <typename T>
  bool uzawa_tail_fused3(int l, T *u, T *p, const T *gp) {
    if constexpr (DIM != 2) {
      return false;
    } else {
      const int kA = desc.cheb_deg_A, kS = desc.cheb_deg_S;
      if (general || kA < 1 || kS != 1 || fuse3_2d_max_n <= 0 ||
          std::max(lv[l].n[0], lv[l].n[1]) > fuse3_2d_max_n)
        return false;
      Work<T> &W = work<T>(l);
      const double bA = lv[l].beta_A, thA = 0.75 * bA, deA = 0.25 * bA, s1A = thA / deA;
      const double rhoA = 1.0 / s1A, rnA = 1.0 / (2.0 * s1A - rhoA);
      const double bS = lv[l].beta_S, thS = 0.75 * bS, deS = 0.25 * bS, s1S = thS / deS;
      const double rhoS = 1.0 / s1S, rnS = 1.0 / (2.0 * s1S - rhoS);
      OpChebA<T, true, true> o;
      std::memset(&o, 0, sizeof(o));
      o.dinv = W.dinvA;
      o.r_out = W.cr;
      o.x_out = W.cx;
      o.d_out = W.cd[1];
      o.inv_theta = (T)(1.0 / thA);
      o.c1 = (T)(rnA * rhoA);
      o.c2 = (T)(2.0 * rnA / deA);
      Fuse3P<T> P;
      std::memset(&P, 0, sizeof(P));
      P.dinv_s = W.dinvS;
      P.inv_theta = (T)(1.0 / thS);
      P.c1 = (T)(rnS * rhoS);
      P.c2 = (T)(2.0 * rnS / deS);
      P.tau = (T)tau;
      auto g = geom<T>(l);
      const Geo2<T> g2 = geo2<T>(g, 3);
      const unsigned nb = (unsigned)(g2.tiles[0] * g2.tiles[1] * 2);
      const double nu = (double)(DIM * g.Nv), np = (double)g.Np;
      for (int stage = 0; stage < 2; ++stage) {
        if (stage == 0) {
          P.u = W.uhat;
          P.p0 = p;
          P.g = gp;
          P.rp = W.rp;
          o.base = nullptr;
          o.out = W.w;
          o.s = (T)sigma;
        } else {
          P.u = W.w;
          P.rin = W.rp;
          P.p = p;
          o.base = W.uhat;
          o.out = u;
          o.s = (T)(-sigma);
        }
        hipEvent_t ea = nullptr, eb = nullptr;
        if (profiling) {
          ea = next_event();
          eb = next_event();
          SMG_HIP(hipEventRecord(ea, stream));
        }
        if (rec) {
          if (stage == 0 && kA == 1) rec_add(LFused3<K, T, F3_DIVRES, true>{g2, P, o}, nb);
          else if (stage == 0) rec_add(LFused3<K, T, F3_DIVRES, false>{g2, P, cast_op<OpChebA<T, true, false>>(o)}, nb);
          else if (kA == 1) rec_add(LFused3<K, T, F3_CHEBS, true>{g2, P, o}, nb);
          else rec_add(LFused3<K, T, F3_CHEBS, false>{g2, P, cast_op<OpChebA<T, true, false>>(o)}, nb);
        } else if (stage == 0) {
          if (kA == 1)
            hipLaunchKernelGGL((wave2d_fused3_kernel<K, T, F3_DIVRES, true>), dim3(nb), dim3(64), 0, stream, g2, P, o);
          else
            hipLaunchKernelGGL((wave2d_fused3_kernel<K, T, F3_DIVRES, false>), dim3(nb), dim3(64), 0, stream, g2, P,
                               cast_op<OpChebA<T, true, false>>(o));
        } else {
          if (kA == 1)
            hipLaunchKernelGGL((wave2d_fused3_kernel<K, T, F3_CHEBS, true>), dim3(nb), dim3(64), 0, stream, g2, P, o);
          else
            hipLaunchKernelGGL((wave2d_fused3_kernel<K, T, F3_CHEBS, false>), dim3(nb), dim3(64), 0, stream, g2, P,
                               cast_op<OpChebA<T, true, false>>(o));
        }
        check_launch();
        if (profiling) {
          SMG_HIP(hipEventRecord(eb, stream));
          char key[160];
          std::snprintf(key, sizeof(key), "%s+grad+cheb_A/v%d/fused3/%s/%dx%dx%d",
                        stage == 0 ? "div_residual" : "cheb_S", kA == 1 ? 3 : 1,
                        std::is_same<T, double>::value ? "f64" : "f32", g.n[0], g.n[1], g.n[2]);
          // velocity input of B, the pressure vectors, D_A^-1, the velocity outputs
          const double pres = stage == 0 ? (has_c() ? 4 : 3) : (P.p ? 4 : 2);
          const double bytes = sizeof(T) * (nu + pres * np + nu * (kA == 1 ? (stage == 1 ? 3 : 2) : 4));
          prof.push_back(ProfRec{key, ea, eb, bytes});
        }
        if (kA > 1) cheb_A<T>(l, nullptr, o.base, o.out, stage == 0 ? sigma : -sigma, 1);
      }
      return true;
    }
  }

  template <typename T>
  void smooth_t(int l, T *x, const T *b, int steps, bool zero_init) {
    for (int s = 0; s < steps; ++s) uzawa_step<T>(l, x, b, zero_init && s == 0);
  }

  // ------------------------------------------------------------ transfers
  template <typename T>
  XferGeo<T> xfer_geo(int lf, bool velocity) {
    XferGeo<T> g;
    std::memset(&g, 0, sizeof(g));
    const LevelInfo &f = lv[lf], &c = lv[lf - 1];
    for (int a = 0; a < 3; ++a) {
      g.cdim[a] = velocity ? c.vd[a] : c.pd[a];
      g.fdim[a] = velocity ? f.vd[a] : f.pd[a];
      g.ncell_f[a] = f.n[a];
    }
    g.coff = velocity ? 0 : c.Nu;
    g.foff = velocity ? 0 : f.Nu;
    g.cstride = velocity ? c.Nv : 0;
    g.fstride = velocity ? f.Nv : 0;
    for (int i = 0; i < 28; ++i) g.W[i] = (T)ttab.W[velocity ? 0 : 1][i];
    return g;
  }

  // both fields in one launch each (see k_prolong / k_restrict)
  template <typename T>
  void prolongate_t(int lf, const T *wc, T *xf) {
    const XferGeo<T> gv = xfer_geo<T>(lf, true), gp = xfer_geo<T>(lf, false);
    const int nzv = (DIM == 3 ? gv.fdim[2] : 1) * DIM, nzp = DIM == 3 ? gp.fdim[2] : 1;
    const int64_t nxy = std::max((int64_t)gv.fdim[0] * gv.fdim[1], (int64_t)gp.fdim[0] * gp.fdim[1]);
    const dim3 grid((unsigned)((nxy + 255) / 256), (unsigned)(nzv + nzp));
    if (rec) rec_add(LProlong<T, DIM, K>{wc, xf, gv, gp, nzv, (int)grid.x}, grid.x * grid.y);
    else hipLaunchKernelGGL((k_prolong<T, DIM, K>), grid, dim3(256), 0, stream, wc, xf, gv, gp, nzv);
    check_launch();
  }

  // zc (optional): a coarse vector zeroed in the same pass
  template <typename T>
  void restrict_t(int lf, const T *rf, T *rc, T *zc = nullptr) {
    constexpr int CX = 128;
    const XferGeo<T> gv = xfer_geo<T>(lf, true), gp = xfer_geo<T>(lf, false);
    const int nzv = (DIM == 3 ? gv.cdim[2] : 1) * DIM, nzp = DIM == 3 ? gp.cdim[2] : 1;
    const int nx = std::max(gv.cdim[0], gp.cdim[0]), ny = std::max(gv.cdim[1], gp.cdim[1]);
    const dim3 grid((unsigned)((nx + CX - 1) / CX), (unsigned)ny, (unsigned)(nzv + nzp));
    if (rec) rec_add(LRestrict<T, DIM, K, CX>{rf, rc, zc, gv, gp, nzv, (int)grid.x, (int)grid.y}, grid.x * grid.y * grid.z);
    else hipLaunchKernelGGL((k_restrict<T, DIM, K, CX>), grid, dim3(256), 0, stream, rf, rc, zc, gv, gp, nzv);
    check_launch();
  }

  // --------------------------------------------------------- coarse solve
  template <typename T>
  void coarse_t(const T *b0, T *x0) {
    const unsigned nb = (unsigned)((n0 + (VB / 64) - 1) / (VB / 64));
    if (rec) rec_add(LCoarseGemv<T>{Kinv, (i64)coarse_ld, n0, b0, x0}, nb);
    else hipLaunchKernelGGL((k_coarse_gemv<T>), dim3(nb), dim3(VB), 0, stream, Kinv, (i64)coarse_ld, n0, b0, x0);
    check_launch();
  }

  // ---------------------------------------------------------- the cycle
  // Algorithm 1 with cycle index desc.cycle_index; level 0 is the direct solve.
  template <typename T>
  void cycle_t(int l, T *x, const T *b, bool zero_init) {
    // stage tags for batched execution (depth d below the finest level): on
    // the way down 4d (pre-smoothing), 4d + 1 (residual), 4d + 2
    // (restriction), 4d + 3 the coarse solve; on the way up ASCENT + 2(64 -
    // d) (prolongation), + 1 (post-smoothing) -- increasing along the V-cycle
    // of every hierarchy, whatever its depth
    constexpr int ASCENT = 1000;
    const int d = L - l;
    if (l == 0) {
      set_tag(4 * d + 3);
      coarse_t<T>(b, x);
      return;
    }
    Work<T> &W = work<T>(l);
    Work<T> &C = work<T>(l - 1);
    set_tag(4 * d);
    smooth_t<T>(l, x, b, desc.smooth_steps, zero_init);
    set_tag(4 * d + 1);
    residual_t<T>(l, x, b, W.r);
    set_tag(4 * d + 2);
    restrict_t<T>(l, W.r, C.b, C.x);   // also C.x = 0
    for (int j = 0; j < desc.cycle_index; ++j) cycle_t<T>(l - 1, C.x, C.b, j == 0);
    set_tag(ASCENT + 2 * (64 - d));
    prolongate_t<T>(l, C.x, x);
    set_tag(ASCENT + 2 * (64 - d) + 1);
    smooth_t<T>(l, x, b, desc.smooth_steps, false);
  }

  // ------------------------------------------------- batched execution
  void record_cycle(int dt, Recorder &r) override {
    if (desc.cycle_index != 1) throw Error{SMG_EUNSUPPORTED, "batched cycle: V-cycle only"};
    if (profiling) throw Error{SMG_EINVAL, "batched cycle: kernel timing is on"};
    rec = &r;
    try {
      r.tag = -1;
      if (dt == SMG_F32) {
        vset<float>(x32, 0.0f, lv[L].N);
        cycle_t<float>(L, x32, b32, true);
      } else {
        vset<double>(x64, 0.0, lv[L].N);
        cycle_t<double>(L, x64, b64, true);
      }
    } catch (...) {
      rec = nullptr;
      throw;
    }
    rec = nullptr;
  }
  void record_vmult(Recorder &r, const double *x, double *y) override {
    rec = &r;
    try {
      vmult_t<double>(L, x, y);
    } catch (...) {
      rec = nullptr;
      throw;
    }
    rec = nullptr;
  }
  void record_residual(Recorder &r, const double *x, const double *b, double *res) override {
    rec = &r;
    try {
      residual_t<double>(L, x, b, res);
    } catch (...) {
      rec = nullptr;
      throw;
    }
    rec = nullptr;
  }
  BatchView batch_view() override {
    BatchView v;
    v.N = lv[L].N;
    v.restart = restart;
    v.V = V;
    v.Z = Z;
    v.b64 = b64;
    v.x64 = x64;
    v.b32 = b32;
    v.x32 = x32;
    v.partial = partial;
    v.precision = desc.precision;
    v.c_zero = !has_c();
    return v;
  }
  void normalize_solution(double *x) override { remove_pressure_mean(x); }
  void set_variants(int split2d, int fuse2d, int fuse3_2d) override {
    if (split2d >= 0) split2d_max_n = split2d;
    if (fuse2d >= 0) fuse2d_max_n = fuse2d;
    if (fuse3_2d >= 0) fuse3_2d_max_n = fuse3_2d;
    invalidate_graphs();
  }

  // ---------------------------------------------------------- reductions
  // dvec[0..nv) = V_j . w (V_j = V + j * ldv), FP64, deterministic.
  void multidot(const double *Vb, int64_t ldv, int nv, const double *w, int64_t n, double *outdev) {
    hipLaunchKernelGGL((k_multidot_partial<double>), dim3(RB), dim3(VB), 0, stream, Vb, (i64)ldv, nv, w, (i64)n, partial);
    check_launch();
    hipLaunchKernelGGL(k_partial_finish, dim3(nv), dim3(VB), 0, stream, partial, RB, nv, outdev);
    check_launch();
  }
  double dot(const double *a, const double *b, int64_t n) {
    multidot(a, 0, 1, b, n, dvec);
    SMG_HIP(hipMemcpyAsync(hpin + 1000, dvec, sizeof(double), hipMemcpyDeviceToHost, stream));
    SMG_HIP(hipStreamSynchronize(stream));
    return hpin[1000];
  }
  double norm(const double *a, int64_t n) { return std::sqrt(dot(a, a, n)); }

  // only for C = 0, where the pressure is fixed up to a constant
  void remove_pressure_mean(double *x) {
    if (has_c()) return;
    const LevelInfo &I = lv[L];
    multidot(I.mp1, 0, 1, x + I.Nu, I.Np, dvec);
    hipLaunchKernelGGL(k_subtract_scalar, dim3(grid_for(I.Np)), dim3(VB), 0, stream, x + I.Nu, (const double *)dvec, mp1_sum, (i64)I.Np);
    check_launch();
  }

  // transpose of remove_pressure_mean: g_p -= M_p 1 (1 . g_p) / (1 . M_p 1);
  // nothing to do for C != 0, where solutions are not normalised
  void pressure_mean_adjoint(double *g) override {
    if (has_c()) return;
    const LevelInfo &I = lv[L];
    multidot(unit_vec(I.Np), 0, 1, g + I.Nu, I.Np, dvec);
    hipLaunchKernelGGL(k_subtract_weighted, dim3(grid_for(I.Np)), dim3(VB), 0, stream, g + I.Nu, (const double *)I.mp1,
                       (const double *)dvec, mp1_sum, (i64)I.Np);
    check_launch();
  }

  // ------------------------------------------------------------- set-up
  double lanczos(int l, int which) {
    const LevelInfo &I = lv[l];
    const int64_t n = which == 0 ? I.Nu : I.Np;
    const double *D = which == 0 ? I.DA : I.DS;
    const uint64_t seed = which == 0 ? LANCZOS_SEED_A : LANCZOS_SEED_S;
    std::vector<double> v0(n);
    for (int64_t i = 0; i < n; ++i) v0[i] = splitmix64_uniform(seed, (uint64_t)i + 1);
    if (which == 0) {
      // start in the free (unconstrained) velocity subspace
      for (int c = 0; c < DIM; ++c)
        for (int64_t node = 0; node < I.Nv; ++node) {
          int64_t r = node;
          bool bc = false;
          for (int a = 0; a < DIM; ++a) {
            int ia = (int)(r % I.vd[a]);
            r /= I.vd[a];
            bc |= (ia == 0 || ia == I.vd[a] - 1);
          }
          if (bc) v0[c * I.Nv + node] = 0.0;
        }
    }
    double *q = lz[0], *qp = lz[1], *w = lz[2], *t = lz[3];
    SMG_HIP(hipMemcpyAsync(q, v0.data(), n * sizeof(double), hipMemcpyHostToDevice, stream));
    vset<double>(qp, 0.0, n);
    auto Dmul = [&](double *y, const double *x) {  // y = D x
      hipLaunchKernelGGL((k_jacobi<double>), dim3(grid_for(n)), dim3(VB), 0, stream, y, (const double *)nullptr, 1.0, D, x, (i64)n);
      check_launch();
    };
    Dmul(t, q);
    const double nq = std::sqrt(dot(q, t, n));
    std::vector<double> qs(n);
    // q /= ||q||_D  (host round trip keeps this set-up code simple)
    SMG_HIP(hipMemcpyAsync(qs.data(), q, n * sizeof(double), hipMemcpyDeviceToHost, stream));
    SMG_HIP(hipStreamSynchronize(stream));
    for (auto &v : qs) v /= nq;
    SMG_HIP(hipMemcpyAsync(q, qs.data(), n * sizeof(double), hipMemcpyHostToDevice, stream));
    std::vector<double> al, be;
    double bprev = 0.0;
    const double *dinv = which == 0 ? lv[l].w64.dinvA : lv[l].w64.dinvS;
    for (int j = 0; j < LANCZOS_STEPS && j < n; ++j) {
      // t = M q
      if (which == 0) {
        auto g = geom<double>(l);
        tile<double, BLK_A>(g, OpApply<double>{q, nullptr, t, nullptr});
      } else {
        S_tilde<double>(l, q, t);
      }
      const double a = dot(q, t, n);
      // w = D^-1 t - a q - bprev qp
      hipLaunchKernelGGL((k_jacobi<double>), dim3(grid_for(n)), dim3(VB), 0, stream, w, (const double *)nullptr, 1.0, dinv, t, (i64)n);
      check_launch();
      hipLaunchKernelGGL((k_axpy<double>), dim3(grid_for(n)), dim3(VB), 0, stream, w, -a, (const double *)q, (i64)n);
      check_launch();
      hipLaunchKernelGGL((k_axpy<double>), dim3(grid_for(n)), dim3(VB), 0, stream, w, -bprev, (const double *)qp, (i64)n);
      check_launch();
      al.push_back(a);
      Dmul(t, w);
      const double b = std::sqrt(std::max(dot(w, t, n), 0.0));
      if (!(b > 1e-14 * std::fabs(a))) break;
      be.push_back(b);
      // qp = q; q = w / b
      hipLaunchKernelGGL((k_copy<double, double>), dim3(grid_for(n)), dim3(VB), 0, stream, qp, (const double *)q, (i64)n);
      check_launch();
      hipLaunchKernelGGL((k_jacobi<double>), dim3(grid_for(n)), dim3(VB), 0, stream, q, (const double *)nullptr, 1.0 / b, unit_vec(n), w, (i64)n);
      check_launch();
      bprev = b;
    }
    return LANCZOS_SAFETY * tridiag_max_eig(al, be);
  }

  double *ones = nullptr;
  int64_t ones_n = 0;
  const double *unit_vec(int64_t n) {
    if (ones_n < n) throw Error{SMG_EINVAL, "internal: ones vector too short"};
    return ones;
  }

  // largest eigenvalue of the symmetric tridiagonal (alpha, beta) by bisection
  // on the Sturm sequence count.
  static double tridiag_max_eig(const std::vector<double> &a, const std::vector<double> &b) {
    const int m = (int)a.size();
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < m; ++i) {
      double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i < m - 1 ? std::fabs(b[i]) : 0.0);
      lo = std::min(lo, a[i] - r);
      hi = std::max(hi, a[i] + r);
    }
    auto count_below = [&](double x) {  // number of eigenvalues < x
      int cnt = 0;
      double d = 1.0;
      for (int i = 0; i < m; ++i) {
        d = a[i] - x - (i > 0 ? b[i - 1] * b[i - 1] / d : 0.0);
        if (d == 0.0) d = -1e-300;
        if (d < 0) ++cnt;
      }
      return cnt;
    };
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (count_below(mid) >= m) hi = mid;
      else lo = mid;
      if (hi - lo <= 1e-15 * std::max(1.0, std::fabs(hi))) break;
    }
    return hi;
  }

  void build_coarse() {
    const LevelInfo &I = lv[0];
    n0 = (int)I.N;
    double *e = dalloc<double>(n0);
    double *cols = dalloc<double>((int64_t)n0 * n0);
    for (int j = 0; j < n0; ++j) {
      vset<double>(e, 0.0, n0);
      const double one = 1.0;
      SMG_HIP(hipMemcpyAsync(e + j, &one, sizeof(double), hipMemcpyHostToDevice, stream));
      vmult_t<double>(0, e, cols + (int64_t)j * n0);
    }
    std::vector<double> Kc((size_t)n0 * n0), m(n0, 0.0);
    SMG_HIP(hipMemcpyAsync(Kc.data(), cols, sizeof(double) * Kc.size(), hipMemcpyDeviceToHost, stream));
    SMG_HIP(hipMemcpyAsync(m.data() + I.Nu, I.mp1, sizeof(double) * I.Np, hipMemcpyDeviceToHost, stream));
    SMG_HIP(hipStreamSynchronize(stream));
    // C = 0: constant pressures span ker K_0, and the border [K_0 m; m^T 0]
    // fixes the pressure mean; C = c_p M_p with c_p > 0: K_0 is regular and
    // is inverted as it is
    const bool border = !has_c();
    const int nb = n0 + (border ? 1 : 0);
    coarse_ld = nb;
    std::vector<double> A((size_t)nb * nb, 0.0), Inv((size_t)nb * nb, 0.0);
    for (int i = 0; i < n0; ++i)
      for (int j = 0; j < n0; ++j) A[(size_t)i * nb + j] = Kc[(size_t)j * n0 + i];  // column j = K e_j
    if (border)
      for (int i = 0; i < n0; ++i) {
        A[(size_t)i * nb + n0] = m[i];
        A[(size_t)n0 * nb + i] = m[i];
      }
    for (int i = 0; i < nb; ++i) Inv[(size_t)i * nb + i] = 1.0;
    // Gauss-Jordan elimination with partial pivoting
    for (int c = 0; c < nb; ++c) {
      int piv = c;
      for (int r = c + 1; r < nb; ++r)
        if (std::fabs(A[(size_t)r * nb + c]) > std::fabs(A[(size_t)piv * nb + c])) piv = r;
      if (A[(size_t)piv * nb + c] == 0.0) throw Error{SMG_EINVAL, "singular coarse matrix"};
      if (piv != c)
        for (int j = 0; j < nb; ++j) {
          std::swap(A[(size_t)c * nb + j], A[(size_t)piv * nb + j]);
          std::swap(Inv[(size_t)c * nb + j], Inv[(size_t)piv * nb + j]);
        }
      const double d = 1.0 / A[(size_t)c * nb + c];
      for (int j = 0; j < nb; ++j) {
        A[(size_t)c * nb + j] *= d;
        Inv[(size_t)c * nb + j] *= d;
      }
      for (int r = 0; r < nb; ++r) {
        if (r == c) continue;
        const double f = A[(size_t)r * nb + c];
        if (f == 0.0) continue;
        for (int j = 0; j < nb; ++j) {
          A[(size_t)r * nb + j] -= f * A[(size_t)c * nb + j];
          Inv[(size_t)r * nb + j] -= f * Inv[(size_t)c * nb + j];
        }
      }
    }
    Kinv = dalloc<double>((int64_t)nb * nb);
    SMG_HIP(hipMemcpyAsync(Kinv, Inv.data(), sizeof(double) * Inv.size(), hipMemcpyHostToDevice, stream));
    SMG_HIP(hipStreamSynchronize(stream));
  }

  template <typename T>
  void alloc_work(int l) {
    LevelInfo &I = lv[l];
    Work<T> &W = work<T>(l);
    W.x = dalloc<T>(I.N);
    W.b = dalloc<T>(I.N);
    W.r = dalloc<T>(I.N);
    W.ru = dalloc<T>(I.Nu);
    W.uhat = dalloc<T>(I.Nu);
    W.q = dalloc<T>(I.Nu);
    W.w = dalloc<T>(I.Nu);
    W.cr = dalloc<T>(I.Nu);
    W.cx = dalloc<T>(I.Nu);
    W.cd[0] = dalloc<T>(I.Nu);
    W.cd[1] = dalloc<T>(I.Nu);
    W.rp = dalloc<T>(I.Np);
    W.dp = dalloc<T>(I.Np);
    W.sr = dalloc<T>(I.Np);
    W.sx = dalloc<T>(I.Np);
    W.sd[0] = dalloc<T>(I.Np);
    W.sd[1] = dalloc<T>(I.Np);
    if (!W.t1) W.t1 = dalloc<T>(I.N);
    W.t2 = dalloc<T>(I.N);
    W.dinvA = dalloc<T>(I.Nu);
    W.dinvS = dalloc<T>(I.Np);
    hipLaunchKernelGGL((k_reciprocal<T>), dim3(grid_for(I.Nu)), dim3(VB), 0, stream, W.dinvA, (const double *)I.DA, (i64)I.Nu);
    check_launch();
    hipLaunchKernelGGL((k_reciprocal<T>), dim3(grid_for(I.Np)), dim3(VB), 0, stream, W.dinvS, (const double *)I.DS, (i64)I.Np);
    check_launch();
  }

  void setup() override {
    ref = make_ref1d(K);
    {
      // the device kernels use the compile-time copies of these tables
      constexpr cfe::Tab<K> ct = cfe::make_tab<K>();
      double e = 0;
      for (int i = 0; i <= K; ++i)
        for (int j = 0; j <= K; ++j) {
          e = std::max(e, std::fabs(ct.Kr[i][j] - ref.Kv[i * (K + 1) + j]));
          e = std::max(e, std::fabs(ct.Mr[i][j] - ref.Mv[i * (K + 1) + j]));
        }
      for (int i = 0; i < K; ++i) {
        for (int j = 0; j <= K; ++j) {
          e = std::max(e, std::fabs(ct.Gr[i][j] - ref.G[i * (K + 1) + j]));
          e = std::max(e, std::fabs(ct.Nr[i][j] - ref.N[i * (K + 1) + j]));
        }
        for (int j = 0; j < K; ++j) e = std::max(e, std::fabs(ct.Mpr[i][j] - ref.Mp[i * K + j]));
      }
      if (e > 1e-14) throw Error{SMG_EINVAL, "internal: compile-time 1D tables differ from the set-up tables"};
    }
    sigma = cheb_scaling(desc.cheb_deg_A);
    tau = cheb_scaling(desc.cheb_deg_S);
    std::memset(&ttab, 0, sizeof(ttab));
    {
      std::vector<double> Wv = prolongation_weights(ref.zv), Wp = prolongation_weights(ref.zp);
      std::copy(Wv.begin(), Wv.end(), ttab.W[0]);
      std::copy(Wp.begin(), Wp.end(), ttab.W[1]);
    }
    stream = (hipStream_t)desc.stream;
    L = desc.n_levels - 1;
    lv.resize(desc.n_levels);
    for (int l = 0; l <= L; ++l) {
      LevelInfo &I = lv[l];
      I.Nv = 1;
      I.Np = 1;
      for (int a = 0; a < 3; ++a) {
        if (a < DIM) {
          I.n[a] = desc.n_coarse[a] << l;
          I.vd[a] = K * I.n[a] + 1;
          I.pd[a] = (K - 1) * I.n[a] + 1;
          I.h[a] = (desc.box_hi[a] - desc.box_lo[a]) / I.n[a];
        } else {
          I.n[a] = 1;
          I.vd[a] = 1;
          I.pd[a] = 1;
          I.h[a] = 1.0;
        }
        I.Nv *= I.vd[a];
        I.Np *= I.pd[a];
      }
      I.Nu = DIM * I.Nv;
      I.N = I.Nu + I.Np;
    }
    // the operator kernels address a level vector's velocity block by 32-bit
    // byte offsets
    if ((double)lv[L].Nu * sizeof(double) >= 4294967296.0)
      throw Error{SMG_EUNSUPPORTED, "finest level too large: velocity block exceeds 4 GiB"};
    // per-cell viscosity: finest as given, coarser levels by averaging children
    if (desc.mu_cell) {
      std::vector<std::vector<double>> mu(desc.n_levels);
      const LevelInfo &F = lv[L];
      const int64_t ncf = (int64_t)F.n[0] * F.n[1] * F.n[2];
      mu[L].assign(desc.mu_cell, desc.mu_cell + ncf);
      for (int l = L - 1; l >= 0; --l) {
        const LevelInfo &I = lv[l], &J = lv[l + 1];
        mu[l].assign((size_t)I.n[0] * I.n[1] * I.n[2], 0.0);
        const double wgt = 1.0 / (1 << DIM);
        for (int cz = 0; cz < I.n[2]; ++cz)
          for (int cy = 0; cy < I.n[1]; ++cy)
            for (int cx = 0; cx < I.n[0]; ++cx) {
              double s = 0.0;
              for (int dz = 0; dz < (DIM == 3 ? 2 : 1); ++dz)
                for (int dy = 0; dy < 2; ++dy)
                  for (int dx = 0; dx < 2; ++dx)
                    s += mu[l + 1][(2 * cx + dx) + (int64_t)J.n[0] * ((2 * cy + dy) + (int64_t)J.n[1] * (DIM == 3 ? 2 * cz + dz : 0))];
              mu[l][cx + (int64_t)I.n[0] * (cy + (int64_t)I.n[1] * cz)] = s * wgt;
            }
      }
      for (int l = 0; l <= L; ++l) {
        const int64_t nc = (int64_t)mu[l].size();
        lv[l].w64.mu_cell = dalloc<double>(nc);
        lv[l].w32.mu_cell = dalloc<float>(nc);
        SMG_HIP(hipMemcpyAsync(lv[l].w64.mu_cell, mu[l].data(), nc * sizeof(double), hipMemcpyHostToDevice, stream));
        hipLaunchKernelGGL((k_copy<float, double>), dim3(grid_for(nc)), dim3(VB), 0, stream, lv[l].w32.mu_cell, (const double *)lv[l].w64.mu_cell, (i64)nc);
        check_launch();
      }
    }
    int64_t nmax = 0;
    for (int l = 0; l <= L; ++l) nmax = std::max(nmax, lv[l].N);
    ones = dalloc<double>(nmax);
    ones_n = nmax;
    vset<double>(ones, 1.0, nmax);
    for (int i = 0; i < 4; ++i) lz[i] = dalloc<double>(nmax);
    partial = dalloc<double>((int64_t)RB * 256);
    dvec = dalloc<double>(1024);
    SMG_HIP(hipHostMalloc((void **)&hpin, sizeof(double) * 1024, hipHostMallocDefault));
    SMG_HIP(hipEventCreateWithFlags(&hpin_ready, hipEventDisableTiming));
    // general cells: vertex coordinates of every level (level l takes the
    // finest-level vertex at the same lattice point)
    // the deformation-rate form and Q3-Q2 in 3D run on the vertex-given cell
    // kernel: a box mesh is handed to it as its vertex lattice (box-cell
    // diagonals, node coordinates and the local Schur diagonal still apply
    // to 3D Q3-Q2 box meshes)
    std::vector<double> lattice;
    const double *fverts = desc.fine_vertices;
    general = desc.fine_vertices != nullptr || desc.form == SMG_FORM_EPS;
    if (!fverts && (desc.form == SMG_FORM_EPS || (DIM == 3 && K == 3))) {
      const LevelInfo &F = lv[L];
      const int nz = DIM == 3 ? F.n[2] + 1 : 1;
      lattice.resize((size_t)(F.n[0] + 1) * (F.n[1] + 1) * nz * DIM);
      size_t o = 0;
      for (int k = 0; k < nz; ++k)
        for (int j = 0; j <= F.n[1]; ++j)
          for (int i = 0; i <= F.n[0]; ++i) {
            const int ijk[3] = {i, j, k};
            for (int a = 0; a < DIM; ++a)
              lattice[o++] = desc.box_lo[a] + (desc.box_hi[a] - desc.box_lo[a]) * ijk[a] / (double)F.n[a];
          }
      fverts = lattice.data();
    }
    if (fverts) {
      gen_op = true;
      hverts.resize(L + 1);
      const LevelInfo &F = lv[L];
      const int64_t fx = F.n[0] + 1, fy = F.n[1] + 1;
      for (int l = 0; l <= L; ++l) {
        const LevelInfo &I = lv[l];
        const int s = 1 << (L - l);
        const int nz = DIM == 3 ? I.n[2] + 1 : 1;
        std::vector<double> &hv = hverts[l];
        hv.resize((size_t)(I.n[0] + 1) * (I.n[1] + 1) * nz * DIM);
        size_t o = 0;
        for (int k = 0; k < nz; ++k)
          for (int j = 0; j <= I.n[1]; ++j)
            for (int i = 0; i <= I.n[0]; ++i) {
              const int64_t fv = (int64_t)i * s + fx * ((int64_t)j * s + fy * (int64_t)k * s);
              for (int a = 0; a < DIM; ++a) hv[o++] = fverts[fv * DIM + a];
            }
        lv[l].w64.verts = dalloc<double>((int64_t)hv.size());
        lv[l].w32.verts = dalloc<float>((int64_t)hv.size());
        SMG_HIP(hipMemcpyAsync(lv[l].w64.verts, hv.data(), hv.size() * sizeof(double), hipMemcpyHostToDevice, stream));
        hipLaunchKernelGGL((k_copy<float, double>), dim3(grid_for((int64_t)hv.size())), dim3(VB), 0, stream,
                           lv[l].w32.verts, (const double *)lv[l].w64.verts, (i64)hv.size());
        check_launch();
      }
    }
    // diagonals and M_p 1 on every level
    for (int l = 0; l <= L; ++l) {
      LevelInfo &I = lv[l];
      I.DA = dalloc<double>(I.Nu);
      I.DS = dalloc<double>(I.Np);
      I.mp1 = dalloc<double>(I.Np);
      lv[l].w64.t1 = dalloc<double>(I.N);
      lv[l].w32.t1 = dalloc<float>(I.N);
      if (gen_op) {
        // per-cell results of the one-launch general-cell operator
        constexpr int64_t NN = DIM == 3 ? (K + 1) * (K + 1) * (K + 1) : (K + 1) * (K + 1);
        constexpr int64_t NPN = DIM == 3 ? K * K * K : K * K;
        const int64_t nc = (int64_t)I.n[0] * I.n[1] * (DIM == 3 ? I.n[2] : 1);
        lv[l].w64.cbu = dalloc<double>(nc * DIM * NN);
        lv[l].w64.cbp = dalloc<double>(nc * NPN);
        lv[l].w32.cbu = dalloc<float>(nc * DIM * NN);
        lv[l].w32.cbp = dalloc<float>(nc * NPN);
      }
      auto g = geom<double>(l);
      if (general) {
        probe_diagonals(l);
        if (desc.schur_diag == SMG_SCHUR_LOC) local_schur_diagonal_general(l);
      } else {
        hipLaunchKernelGGL((k_diag_A<DIM, K>), dim3(grid_for(I.Nv)), dim3(VB), 0, stream, g, I.DA);
        check_launch();
        // (the exact diagonal starts as the _d one and is replaced below)
        const int kind = desc.schur_diag == SMG_SCHUR_LOC ? 1 : (desc.schur_diag == SMG_SCHUR_P ? 2 : 0);
        hipLaunchKernelGGL((k_diag_S<DIM, K>), dim3(grid_for(I.Np)), dim3(VB), 0, stream, g, kind, (const double *)I.DA, I.DS);
        check_launch();
      }
      auto gu = geom<double>(l, true);
      tile<double, BLK_C | BLK_CPLUS>(gu, OpApply<double>{nullptr, ones, nullptr, I.mp1});
      alloc_work<double>(l);
      alloc_work<float>(l);
    }
    {
      std::vector<double> h(lv[L].Np);
      SMG_HIP(hipMemcpyAsync(h.data(), lv[L].mp1, h.size() * sizeof(double), hipMemcpyDeviceToHost, stream));
      SMG_HIP(hipStreamSynchronize(stream));
      mp1_sum = 0;
      for (double v : h) mp1_sum += v;
    }
    // Chebyshev intervals (Algorithm 2); level 0 is solved directly
    for (int l = 1; l <= L; ++l) {
      lv[l].beta_A = lanczos(l, 0);
      if (desc.schur_diag == SMG_SCHUR_EXACT) exact_schur_diagonal(l);
      lv[l].beta_S = lanczos(l, 1);
    }
    build_coarse();
    // FGMRES storage
    restart = desc.fgmres_restart;
    V = dalloc<double>((int64_t)(restart + 1) * lv[L].N);
    Z = dalloc<double>((int64_t)restart * lv[L].N);
    b32 = dalloc<float>(lv[L].N);
    x32 = dalloc<float>(lv[L].N);
    b64 = dalloc<double>(lv[L].N);
    x64 = dalloc<double>(lv[L].N);
    SMG_HIP(hipStreamSynchronize(stream));
  }

  // -------------------------------------------------------- public (dt)
#define SMG_DISPATCH(dt, call_f64, call_f32) \
  do {                                        \
    if ((dt) == SMG_F64) { call_f64; }        \
    else { call_f32; }                        \
  } while (0)

  void vmult(int l, int dt, const void *x, void *y) override {
    SMG_DISPATCH(dt, vmult_t<double>(l, (const double *)x, (double *)y), vmult_t<float>(l, (const float *)x, (float *)y));
  }
  void residual(int l, int dt, const void *x, const void *b, void *r) override {
    SMG_DISPATCH(dt, residual_t<double>(l, (const double *)x, (const double *)b, (double *)r),
                 residual_t<float>(l, (const float *)x, (const float *)b, (float *)r));
  }
  void apply_block(int l, int dt, int blk, const void *x, void *y) override {
    SMG_DISPATCH(dt, block_t<double>(l, blk, (const double *)x, (double *)y), block_t<float>(l, blk, (const float *)x, (float *)y));
  }
  void lift_dirichlet(int l, int dt, const void *ud, void *b) override {
    SMG_DISPATCH(dt, lift_t<double>(l, (const double *)ud, (double *)b), lift_t<float>(l, (const float *)ud, (float *)b));
  }
  void insert_dirichlet(int l, int dt, const void *ud, void *x) override {
    SMG_DISPATCH(dt, insert_dirichlet_t<double>(l, (const double *)ud, (double *)x),
                 insert_dirichlet_t<float>(l, (const float *)ud, (float *)x));
  }
  void chebyshev(int l, int dt, int which, const void *r, void *out) override {
    if (which == 0)
      SMG_DISPATCH(dt, cheb_A<double>(l, (const double *)r, nullptr, (double *)out, sigma),
                   cheb_A<float>(l, (const float *)r, nullptr, (float *)out, sigma));
    else
      SMG_DISPATCH(dt, cheb_S<double>(l, (const double *)r, (double *)out, nullptr),
                   cheb_S<float>(l, (const float *)r, (float *)out, nullptr));
  }
  void velocity_update(int l, int dt, const void *x, const void *b, void *uhat) override {
    SMG_DISPATCH(dt, velocity_update_t<double>(l, (const double *)x, (const double *)b, (double *)uhat),
                 velocity_update_t<float>(l, (const float *)x, (const float *)b, (float *)uhat));
  }
  void smooth(int l, int dt, void *x, const void *b, int steps) override {
    SMG_DISPATCH(dt, smooth_t<double>(l, (double *)x, (const double *)b, steps, false),
                 smooth_t<float>(l, (float *)x, (const float *)b, steps, false));
  }
  void restrict_(int lf, int dt, const void *rf, void *rc) override {
    SMG_DISPATCH(dt, restrict_t<double>(lf, (const double *)rf, (double *)rc), restrict_t<float>(lf, (const float *)rf, (float *)rc));
  }
  void prolongate_add(int lf, int dt, const void *wc, void *xf) override {
    SMG_DISPATCH(dt, prolongate_t<double>(lf, (const double *)wc, (double *)xf), prolongate_t<float>(lf, (const float *)wc, (float *)xf));
  }
  void coarse_solve(int dt, const void *b0, void *x0) override {
    SMG_DISPATCH(dt, coarse_t<double>((const double *)b0, (double *)x0), coarse_t<float>((const float *)b0, (float *)x0));
  }
  void vcycle(int l, int dt, void *x, const void *b) override {
    SMG_DISPATCH(dt, cycle_t<double>(l, (double *)x, (const double *)b, false), cycle_t<float>(l, (float *)x, (const float *)b, false));
  }

  // z = M^-1 v: one cycle from zero, in the precision of the descriptor
  void precondition(const double *v, double *z) {
    const int64_t N = lv[L].N;
    if (desc.precision == SMG_PRECOND_F64) {
      hipLaunchKernelGGL((k_copy<double, double>), dim3(grid_for(N)), dim3(VB), 0, stream, b64, v, (i64)N);
      check_launch();
      cycle_from_zero(SMG_F64);
      hipLaunchKernelGGL((k_copy<double, double>), dim3(grid_for(N)), dim3(VB), 0, stream, z, (const double *)x64, (i64)N);
      check_launch();
    } else {
      hipLaunchKernelGGL((k_copy<float, double>), dim3(grid_for(N)), dim3(VB), 0, stream, b32, v, (i64)N);
      check_launch();
      cycle_from_zero(SMG_F32);
      hipLaunchKernelGGL((k_copy<double, float>), dim3(grid_for(N)), dim3(VB), 0, stream, z, (const float *)x32, (i64)N);
      check_launch();
    }
  }

  static bool finite(double v) { return std::isfinite(v); }

  smg_status solve(double *x, const double *b, double rtol, int maxit, smg_solve_info *info) override {
    auto t0 = std::chrono::steady_clock::now();
    const int64_t N = lv[L].N;
    const int m = restart;
    // ||b|| and the initial residual norm with one copy back
    residual_t<double>(L, x, b, V);
    multidot(b, 0, 1, b, N, dvec);
    multidot(V, 0, 1, V, N, dvec + 1);
    SMG_HIP(hipMemcpyAsync(hpin + 1000, dvec, 2 * sizeof(double), hipMemcpyDeviceToHost, stream));
    SMG_HIP(hipStreamSynchronize(stream));
    const double bnorm = std::sqrt(hpin[1000]), beta0 = std::sqrt(hpin[1001]);
    int hist_len = 0;
    auto record = [&](double v) {
      if (info && info->history && hist_len < info->history_capacity) info->history[hist_len] = v;
      ++hist_len;
    };
    smg_status st = SMG_OK;
    int it = 0;
    double rel = 0.0;
    if (bnorm == 0.0) {
      vset<double>(x, 0.0, N);
      record(0.0);
    } else {
      double beta = beta0;
      rel = beta / bnorm;
      record(rel);
      std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1);
      // pinned: hbuf = this iteration's coefficients and norm (dvec[0..512]),
      // y = the correction's coefficients (host to device, dvec[0..m))
      double *hbuf = hpin, *y = hpin + 600;
      while (it < maxit && rel > rtol) {
        hipLaunchKernelGGL((k_jacobi<double>), dim3(grid_for(N)), dim3(VB), 0, stream, V, (const double *)nullptr, 1.0 / beta, unit_vec(N), (const double *)V, (i64)N);
        check_launch();
        std::fill(gv.begin(), gv.end(), 0.0);
        std::fill(H.begin(), H.end(), 0.0);
        gv[0] = beta;
        int jdone = 0;
        bool broke = false;
        // z_j = M^-1 v_j and w = K z_j of iteration j already queued (ahead)
        bool queued = false;
        double rel_prev = rel, rel_prev2 = -1.0;
        for (int j = 0; j < m; ++j) {
          double *vj = V + (int64_t)j * N, *zj = Z + (int64_t)j * N, *w = V + (int64_t)(j + 1) * N;
          if (!queued) {
            precondition(vj, zj);
            vmult_t<double>(L, zj, w);
          }
          queued = false;
          // classical Gram-Schmidt, twice; coefficients and the norm stay on
          // the device until one copy per iteration
          for (int pass = 0; pass < 2; ++pass) {
            double *hd = dvec + 256 * pass;
            multidot(V, N, j + 1, w, N, hd);
            hipLaunchKernelGGL((k_multi_axpy<double>), dim3(grid_for(N)), dim3(VB), 0, stream, w, (const double *)V, (i64)N, j + 1, (const double *)hd, -1.0, (i64)N);
            check_launch();
          }
          multidot(w, 0, 1, w, N, dvec + 512);
          hipLaunchKernelGGL((k_scale_inv_sqrt<double>), dim3(grid_for(N)), dim3(VB), 0, stream, w, (const double *)(dvec + 512), (i64)N);
          check_launch();
          SMG_HIP(hipMemcpyAsync(hbuf, dvec, sizeof(double) * 513, hipMemcpyDeviceToHost, stream));
          SMG_HIP(hipEventRecord(hpin_ready, stream));
          // While the host waits for this iteration's coefficients, queue the
          // next iteration's preconditioner and operator (they need only
          // v_{j+1}, normalised on the device) unless this iteration may
          // reach the tolerance: the residual estimate is extrapolated
          // geometrically from the last two (a factor 100 per iteration at
          // the start of a cycle).  Queued work of an iteration that does not
          // run is discarded; it changes no result.
          {
            const double pred = rel_prev2 > 0.0 ? rel_prev * (rel_prev / rel_prev2) : rel_prev * 1e-2;
            if (j + 1 < m && it + 1 < maxit && pred > 2.0 * rtol) {
              double *zn = Z + (int64_t)(j + 1) * N, *wn = V + (int64_t)(j + 2) * N;
              precondition(w, zn);
              vmult_t<double>(L, zn, wn);
              queued = true;
            }
          }
          SMG_HIP(hipEventSynchronize(hpin_ready));
          for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] += hbuf[i] + hbuf[256 + i];
          const double hn = std::sqrt(std::max(hbuf[512], 0.0));
          H[(size_t)(j + 1) * m + j] = hn;
          if (!finite(hn)) { broke = true; break; }
          for (int i = 0; i < j; ++i) {
            const double t = cs[i] * H[(size_t)i * m + j] + sn[i] * H[(size_t)(i + 1) * m + j];
            H[(size_t)(i + 1) * m + j] = -sn[i] * H[(size_t)i * m + j] + cs[i] * H[(size_t)(i + 1) * m + j];
            H[(size_t)i * m + j] = t;
          }
          const double den = std::hypot(H[(size_t)j * m + j], H[(size_t)(j + 1) * m + j]);
          cs[j] = H[(size_t)j * m + j] / den;
          sn[j] = H[(size_t)(j + 1) * m + j] / den;
          H[(size_t)j * m + j] = den;
          H[(size_t)(j + 1) * m + j] = 0.0;
          gv[j + 1] = -sn[j] * gv[j];
          gv[j] = cs[j] * gv[j];
          ++it;
          jdone = j + 1;
          rel = std::fabs(gv[j + 1]) / bnorm;
          if (!finite(rel)) { broke = true; break; }
          record(rel);
          rel_prev2 = rel_prev;
          rel_prev = rel;
          if (rel <= rtol || it >= maxit) break;
        }
        if (broke) { st = SMG_EBREAKDOWN; break; }
        for (int i = jdone - 1; i >= 0; --i) {
          double s = gv[i];
          for (int c = i + 1; c < jdone; ++c) s -= H[(size_t)i * m + c] * y[c];
          y[i] = s / H[(size_t)i * m + i];
        }
        SMG_HIP(hipMemcpyAsync(dvec, y, sizeof(double) * jdone, hipMemcpyHostToDevice, stream));
        hipLaunchKernelGGL((k_multi_axpy<double>), dim3(grid_for(N)), dim3(VB), 0, stream, x, (const double *)Z, (i64)N, jdone, (const double *)dvec, 1.0, (i64)N);
        check_launch();
        residual_t<double>(L, x, b, V);
        beta = norm(V, N);
        rel = beta / bnorm;
        if (!finite(rel)) { st = SMG_EBREAKDOWN; break; }
        if (hist_len > 0 && info && info->history && hist_len - 1 < info->history_capacity) info->history[hist_len - 1] = rel;
      }
      if (st == SMG_OK && rel > rtol) st = SMG_ENOTCONV;
    }
    remove_pressure_mean(x);
    SMG_HIP(hipStreamSynchronize(stream));
    if (info) {
      info->iterations = it;
      info->rel_residual = rel;
      info->rate_q = 0.0;
      info->history_len = std::min(hist_len, info->history_capacity);
      info->t_solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      info->t_setup_ms = t_setup_ms;
    }
    return st;
  }

  smg_status solve_stationary(double *x, const double *b, double rtol, int maxit, smg_solve_info *info) override {
    auto t0 = std::chrono::steady_clock::now();
    const int64_t N = lv[L].N;
    double *r = lv[L].w64.r;
    residual_t<double>(L, x, b, r);
    const double r0 = norm(r, N);
    std::vector<double> hist{r0};
    smg_status st = SMG_OK;
    int it = 0;
    while (it < maxit && hist.back() > rtol * r0) {
      cycle_t<double>(L, x, b, false);
      residual_t<double>(L, x, b, r);
      const double rn = norm(r, N);
      ++it;
      hist.push_back(rn);
      if (!finite(rn) || rn > 1e3 * r0) { st = SMG_EBREAKDOWN; break; }
    }
    if (st == SMG_OK && hist.back() > rtol * r0) st = SMG_ENOTCONV;
    remove_pressure_mean(x);
    SMG_HIP(hipStreamSynchronize(stream));
    if (info) {
      info->iterations = it;
      info->rel_residual = r0 > 0 ? hist.back() / r0 : 0.0;
      const int j = (int)hist.size() - 1, s = std::min(3, j);
      info->rate_q = (j > 0 && hist[j - s] > 0) ? std::pow(hist[j] / hist[j - s], 1.0 / s) : 0.0;
      int n = 0;
      for (size_t i = 0; i < hist.size(); ++i)
        if (info->history && (int)i < info->history_capacity) { info->history[i] = r0 > 0 ? hist[i] / r0 : 0.0; ++n; }
      info->history_len = n;
      info->t_solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
      info->t_setup_ms = t_setup_ms;
    }
    return st;
  }

  void node_coordinates(int l, double *xyz) override {
    const LevelInfo &I = lv[l];
    if (general) {
      // image of the GLL lattice under each cell's multilinear map
      const std::vector<double> &hv = hverts[l];
      for (int64_t node = 0; node < I.Nv; ++node) {
        int64_t r = node;
        int c[3] = {0, 0, 0};
        double t[3] = {0, 0, 0};
        for (int a = 0; a < DIM; ++a) {
          const int i = (int)(r % I.vd[a]);
          r /= I.vd[a];
          c[a] = i / K;
          if (c[a] > I.n[a] - 1) c[a] = I.n[a] - 1;
          t[a] = ref.zv[i - c[a] * K];
        }
        for (int a = 0; a < DIM; ++a) xyz[node * DIM + a] = 0.0;
        for (int v = 0; v < (1 << DIM); ++v) {
          double w = 1.0;
          int o[3] = {v & 1, (v >> 1) & 1, (v >> 2) & 1};
          for (int b = 0; b < DIM; ++b) w *= o[b] ? t[b] : 1.0 - t[b];
          const int64_t vid = (c[0] + o[0]) + (int64_t)(I.n[0] + 1) * ((c[1] + o[1]) + (int64_t)(I.n[1] + 1) * (DIM == 3 ? c[2] + o[2] : 0));
          for (int a = 0; a < DIM; ++a) xyz[node * DIM + a] += w * hv[vid * DIM + a];
        }
      }
      return;
    }
    for (int64_t node = 0; node < I.Nv; ++node) {
      int64_t r = node;
      for (int a = 0; a < DIM; ++a) {
        const int i = (int)(r % I.vd[a]);
        r /= I.vd[a];
        int c = i / K;
        if (c > I.n[a] - 1) c = I.n[a] - 1;
        const double t = ref.zv[i - c * K];
        xyz[node * DIM + a] = desc.box_lo[a] + I.h[a] * (c + t);
      }
    }
  }
};

}  // namespace smg
