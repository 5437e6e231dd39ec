// Host-side solver engine: level hierarchy, set-up (Algorithm 2), smoother
// (inexact symmetric Uzawa, Sec. 1 / Sec. 3.3.1), multigrid cycle
// (Algorithm 1), outer FGMRES and the stationary protocol (Sec. 4.1).
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "../../include/smg.h"
#include "fe1d.hpp"

namespace smg {

struct Error {
  smg_status code;
  std::string msg;
};

#define SMG_HIP(call)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw ::smg::Error{SMG_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

// Per-precision workspace of one level.
template <typename T>
struct Work {
  T *x = nullptr, *b = nullptr, *r = nullptr;        // level iterate / rhs / residual (length N)
  T *ru = nullptr, *uhat = nullptr, *q = nullptr, *w = nullptr;  // velocity (d Nv)
  T *cr = nullptr, *cx = nullptr, *cd[2] = {nullptr, nullptr};  // Chebyshev state, A
  T *rp = nullptr, *dp = nullptr;                     // pressure (Np)
  T *sr = nullptr, *sx = nullptr, *sd[2] = {nullptr, nullptr};  // Chebyshev state, S~
  T *t1 = nullptr, *t2 = nullptr;                     // scratch (length N): general-cell accumulation
  T *cbu = nullptr, *cbp = nullptr;                   // general cells: per-cell results (cells x d x (k+1)^d, cells x k^d)
  T *dinvA = nullptr, *dinvS = nullptr;               // inverse diagonals
  T *mu_cell = nullptr;                               // per-cell viscosity (optional)
  T *verts = nullptr;                                 // vertex coordinates (general cells)
};

struct LevelInfo {
  int n[3] = {1, 1, 1};
  int vd[3] = {1, 1, 1}, pd[3] = {1, 1, 1};
  int64_t Nv = 0, Np = 0, Nu = 0, N = 0;
  double h[3] = {1, 1, 1};
  double beta_A = 0, beta_S = 0;
  double *DA = nullptr, *DS = nullptr;  // FP64 diagonals
  double *mp1 = nullptr;                // M_p 1 (pressure mean weights)
  Work<double> w64;
  Work<float> w32;
};

// A kernel launch recorded instead of run: the launch functor's bytes (see
// packed.hpp), its block count and the packed kernel that runs many of them.
struct LaunchRec {
  int tag = 0;                  // stage of the multigrid cycle (merge key)
  const void *kernel = nullptr; // k_packed<L>
  unsigned nblocks = 0, threads = 0;
  size_t align = 8;
  std::vector<unsigned char> bytes;
};
struct Recorder {
  int tag = 0;
  std::vector<LaunchRec> recs;
};

// Internal buffers of a solver that a batched driver works on.
struct BatchView {
  int64_t N = 0;              // finest-level vector length
  int restart = 0;            // FGMRES basis size
  double *V = nullptr, *Z = nullptr;   // Krylov bases (restart + 1, restart vectors of N)
  double *b64 = nullptr, *x64 = nullptr;
  float *b32 = nullptr, *x32 = nullptr;
  double *partial = nullptr;  // RB x (restart + 1) reduction partials
  int precision = 0;
  bool c_zero = true;         // C = 0: solutions are normalised to pressure mean zero
};

class EngineBase {
 public:
  virtual ~EngineBase() {}
  smg_desc desc;
  std::vector<LevelInfo> lv;
  hipStream_t stream = nullptr;
  int L = 0;  // finest level index
  double t_setup_ms = 0;  // wall time of setup()

  virtual void setup() = 0;
  virtual void vmult(int l, int dt, const void *x, void *y) = 0;
  virtual void residual(int l, int dt, const void *x, const void *b, void *r) = 0;
  virtual void apply_block(int l, int dt, int blk, const void *x, void *y) = 0;
  virtual void lift_dirichlet(int l, int dt, const void *ud, void *b) = 0;
  virtual void insert_dirichlet(int l, int dt, const void *ud, void *x) = 0;
  virtual void chebyshev(int l, int dt, int which, const void *r, void *out) = 0;
  virtual void velocity_update(int l, int dt, const void *x, const void *b, void *uhat) = 0;
  virtual void smooth(int l, int dt, void *x, const void *b, int steps) = 0;
  virtual void restrict_(int lf, int dt, const void *rf, void *rc) = 0;
  virtual void prolongate_add(int lf, int dt, const void *wc, void *xf) = 0;
  virtual void coarse_solve(int dt, const void *b0, void *x0) = 0;
  virtual void vcycle(int l, int dt, void *x, const void *b) = 0;
  virtual smg_status solve(double *x, const double *b, double rtol, int maxit, smg_solve_info *info) = 0;
  virtual smg_status solve_stationary(double *x, const double *b, double rtol, int maxit, smg_solve_info *info) = 0;
  virtual void node_coordinates(int l, double *xyz) = 0;
  virtual void gradient(const double *x, const double *lam, double *g_logmu, double *g_f) = 0;
  virtual void pressure_mean_adjoint(double *g) = 0;
  // y = K_l x with the per-cell partial results of vertex-given cells in a
  // caller-provided device buffer instead of the level's own (box-cell
  // kernels need none); no allocation, no kernel timing.
  virtual int64_t vmult_scratch_bytes(int l, int dt) const = 0;
  virtual void vmult_scratch(int l, int dt, const void *x, void *y, void *scratch) = 0;
  virtual void invalidate_graphs() {}
  bool use_graphs = true;

  // Batched execution: with `rec` set, the launch sites of the 2D box-cell
  // cycle and operator append functors to it instead of launching.
  Recorder *rec = nullptr;
  void set_tag(int t) {
    if (rec) rec->tag = t;
  }
  // the preconditioning cycle from zero on the internal buffers (b32/x32 or
  // b64/x64 by dt), the finest-level y = K x and r = b - K x (FP64)
  virtual void record_cycle(int dt, Recorder &r) = 0;
  virtual void record_vmult(Recorder &r, const double *x, double *y) = 0;
  virtual void record_residual(Recorder &r, const double *x, const double *b, double *res) = 0;
  virtual BatchView batch_view() = 0;
  // the normalisation smg_solve applies to its result (pressure mean zero for C = 0)
  virtual void normalize_solution(double *x) = 0;
  // kernel-variant limits of the 2D levels (cells per direction; negative: keep)
  virtual void set_variants(int split2d, int fuse2d, int fuse3_2d) = 0;

  // Optional kernel timing: HIP events recorded around each operator-kernel
  // launch on the launch stream, aggregated per kernel key.
  struct ProfRec {
    std::string key;
    hipEvent_t a, b;
    double bytes;  // algorithmic HBM bytes of the launch
  };
  bool profiling = false;
  std::vector<ProfRec> prof;
  std::vector<hipEvent_t> event_pool;
  size_t event_used = 0;
  hipEvent_t next_event() {
    if (event_used == event_pool.size()) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) throw Error{SMG_EDEVICE, std::string("hipEventCreate: ") + hipGetErrorString(r)};
      event_pool.push_back(e);
    }
    return event_pool[event_used++];
  }
  void profile_reset() {
    prof.clear();
    event_used = 0;
  }
  void destroy_events() {
    for (hipEvent_t e : event_pool) (void)hipEventDestroy(e);
    event_pool.clear();
    event_used = 0;
  }
  std::string profile_report();

  std::vector<void *> allocations;
  template <typename T>
  T *dalloc(int64_t n) {
    void *p = nullptr;
    if (n <= 0) n = 1;
    hipError_t e = hipMalloc(&p, sizeof(T) * (size_t)n);
    if (e != hipSuccess) throw Error{SMG_ENOMEM, std::string("hipMalloc failed: ") + hipGetErrorString(e)};
    allocations.push_back(p);
    return (T *)p;
  }
  // pinned host mirror of the small device result vector (reduction
  // results copied back once per Krylov iteration; pinned, so the copies
  // are true asynchronous DMA transfers)
  double *hpin = nullptr;
  // marks the arrival of those results while later work is already queued
  hipEvent_t hpin_ready = nullptr;
  void free_all() {
    destroy_events();
    for (void *p : allocations) (void)hipFree(p);
    allocations.clear();
    if (hpin) (void)hipHostFree(hpin);
    hpin = nullptr;
    if (hpin_ready) (void)hipEventDestroy(hpin_ready);
    hpin_ready = nullptr;
  }
};

EngineBase *make_engine(const smg_desc &d);

}  // namespace smg
