// C ABI of the multigrid library (declarations and contracts in include/smg.h).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include <chrono>
#include <map>
#include <mutex>
#include <vector>

#include "batch.hpp"
#include "engine.hpp"

std::string smg::EngineBase::profile_report() {
  SMG_HIP(hipStreamSynchronize(stream));
  struct Agg {
    long count = 0;
    double ms = 0.0, bytes = 0.0;
  };
  std::map<std::string, Agg> agg;
  for (const ProfRec &r : prof) {
    float ms = 0.0f;
    SMG_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    Agg &e = agg[r.key];
    e.count += 1;
    e.ms += ms;
    e.bytes += r.bytes;
  }
  std::string out;
  char line[320];
  for (const auto &kv : agg) {
    std::snprintf(line, sizeof(line), "%s %ld %.6f %.6e\n", kv.first.c_str(), kv.second.count, kv.second.ms, kv.second.bytes);
    out += line;
  }
  return out;
}

namespace smg {
EngineBase *make_engine_2_2();
EngineBase *make_engine_2_3();
EngineBase *make_engine_3_2();
EngineBase *make_engine_3_3();
}  // namespace smg

struct smg_ctx {
  smg::EngineBase *eng = nullptr;
  int device = 0;
  void *scratch = nullptr;   // this device's address of `scratch` below (nullptr if unavailable)
};

// Fixed device buffer of smg_vmult_noalloc: the per-cell partial results of
// vertex-given cells.  One copy per GPU the library runs on, held until the
// process ends.  Host code never passes `scratch` itself to a kernel (on the
// host the name is only a stand-in): its device address comes from
// hipGetSymbolAddress, once per device (scratch_address below).
#define SMG_NOALLOC_SCRATCH_BYTES (16u << 20)
static __device__ __align__(256) unsigned char scratch[SMG_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_addr;   // device -> address of `scratch` there

// The address of `scratch` on device `dev`, which must be the current device.
hipError_t scratch_address(int dev, void **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it != g_scratch_addr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void *p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_addr[dev] = p;
  *out = p;
  return hipSuccess;
}
}  // namespace

namespace {

thread_local std::string g_last_error;

smg_status fail(smg_status code, const std::string &msg) {
  g_last_error = msg;
  return code;
}

#define SMG_TRY(body)                                              \
  try {                                                            \
    body;                                                          \
    g_last_error.clear();                                          \
    return SMG_OK;                                                 \
  } catch (const smg::Error &e) {                                  \
    return fail(e.code, e.msg);                                    \
  } catch (const std::exception &e) {                              \
    return fail(SMG_EDEVICE, std::string("exception: ") + e.what()); \
  }

smg_status check_ctx(const smg_ctx *ctx) {
  if (!ctx || !ctx->eng) return fail(SMG_EINVAL, "null context");
  return SMG_OK;
}

smg_status check_level(const smg_ctx *ctx, int level, int min_level = 0) {
  smg_status s = check_ctx(ctx);
  if (s != SMG_OK) return s;
  if (level < min_level || level > ctx->eng->L)
    return fail(SMG_EINVAL, "level " + std::to_string(level) + " out of range [" + std::to_string(min_level) + ", " +
                                std::to_string(ctx->eng->L) + "]");
  return SMG_OK;
}

smg_status check_dtype(int dt) {
  if (dt != SMG_F64 && dt != SMG_F32) return fail(SMG_EINVAL, "dtype must be SMG_F64 (0) or SMG_F32 (1)");
  return SMG_OK;
}

smg_status check_ptrs(std::initializer_list<const void *> ps) {
  for (const void *p : ps)
    if (!p) return fail(SMG_EINVAL, "null vector pointer");
  return SMG_OK;
}

smg_status validate(const smg_desc *d) {
  if (!d) return fail(SMG_EINVAL, "null descriptor");
  if (d->dim != 2 && d->dim != 3) return fail(SMG_EINVAL, "dim must be 2 or 3");
  if (d->fe_degree < 2) return fail(SMG_EINVAL, "fe_degree must be >= 2 (Taylor-Hood Q_k-Q_{k-1})");
  if (d->fe_degree > 3) return fail(SMG_EUNSUPPORTED, "fe_degree > 3 is not built");
  if (d->n_levels < 2 || d->n_levels > 16) return fail(SMG_EINVAL, "n_levels must be in [2, 16]");
  double ncells = 1.0;
  for (int a = 0; a < d->dim; ++a) {
    if (d->n_coarse[a] < 2) return fail(SMG_EINVAL, "n_coarse must be >= 2 in every direction (no cell with two opposite boundary faces)");
    if (!(d->box_hi[a] > d->box_lo[a])) return fail(SMG_EINVAL, "box_hi must exceed box_lo");
    const double n = (double)d->n_coarse[a] * std::ldexp(1.0, d->n_levels - 1);
    if (n * d->fe_degree + 1 > 2.0e9) return fail(SMG_EINVAL, "mesh too large");
    ncells *= n;
  }
  if (ncells > 4.0e9) return fail(SMG_EINVAL, "mesh too large");
  if (!(d->mu > 0) && !d->mu_cell) return fail(SMG_EINVAL, "mu must be > 0");
  if (!(d->gamma >= 0) || !(d->rho > 0)) return fail(SMG_EINVAL, "need gamma >= 0 and rho > 0");
  if (!(d->c_pressure >= 0)) return fail(SMG_EINVAL, "c_pressure must be >= 0");
  if (d->cheb_deg_A < 0 || d->cheb_deg_A > 16 || d->cheb_deg_S < 0 || d->cheb_deg_S > 16)
    return fail(SMG_EINVAL, "Chebyshev degrees must be in [0, 16]");
  if (d->smooth_steps < 1 || d->smooth_steps > 64) return fail(SMG_EINVAL, "smooth_steps must be in [1, 64]");
  if (d->cycle_index < 1 || d->cycle_index > 2) return fail(SMG_EINVAL, "cycle_index must be 1 (V) or 2 (W)");
  if (d->schur_diag < 0 || d->schur_diag > 3) return fail(SMG_EINVAL, "schur_diag must be 0, 1, 2 or 3");
  if (d->precision != SMG_PRECOND_F64 && d->precision != SMG_PRECOND_F32) return fail(SMG_EINVAL, "precision must be 0 or 1");
  if (d->fgmres_restart < 1 || d->fgmres_restart > 200) return fail(SMG_EINVAL, "fgmres_restart must be in [1, 200]");
  if (d->form != SMG_FORM_GRAD && d->form != SMG_FORM_EPS) return fail(SMG_EINVAL, "form must be 0 (grad) or 1 (eps)");
  if (d->form == SMG_FORM_EPS && d->schur_diag == SMG_SCHUR_LOC)
    return fail(SMG_EUNSUPPORTED, "the local Schur diagonal is built for the gradient form only");
  if (d->mu_cell) {
    double nf = 1.0;
    for (int a = 0; a < d->dim; ++a) nf *= (double)d->n_coarse[a] * std::ldexp(1.0, d->n_levels - 1);
    for (int64_t i = 0; i < (int64_t)nf; ++i)
      if (!(d->mu_cell[i] > 0) || !std::isfinite(d->mu_cell[i])) return fail(SMG_EINVAL, "mu_cell entries must be finite and > 0");
  }
  return SMG_OK;
}

}  // namespace

extern "C" {

void smg_desc_default(smg_desc *d) {
  if (!d) return;
  std::memset(d, 0, sizeof(*d));
  d->dim = 2;
  d->fe_degree = 2;
  d->n_coarse[0] = d->n_coarse[1] = d->n_coarse[2] = 4;
  d->n_levels = 3;
  for (int a = 0; a < 3; ++a) {
    d->box_lo[a] = 0.0;
    d->box_hi[a] = 1.0;
  }
  d->fine_vertices = nullptr;
  d->mu = 1.0;
  d->mu_cell = nullptr;
  d->gamma = 0.0;
  d->rho = 1.0;
  d->c_pressure = 0.0;
  d->cheb_deg_A = 1;
  d->cheb_deg_S = 1;
  d->smooth_steps = 2;
  d->cycle_index = 1;
  d->schur_diag = SMG_SCHUR_D;
  d->precision = SMG_PRECOND_F64;
  d->fgmres_restart = 30;
  d->stream = nullptr;
  d->form = SMG_FORM_GRAD;
}

smg_status smg_create(const smg_desc *desc, smg_ctx **out) {
  if (!out) return fail(SMG_EINVAL, "null output pointer");
  *out = nullptr;
  smg_status s = validate(desc);
  if (s != SMG_OK) return s;
  smg::EngineBase *eng = nullptr;
  if (desc->dim == 2 && desc->fe_degree == 2) eng = smg::make_engine_2_2();
  else if (desc->dim == 2 && desc->fe_degree == 3) eng = smg::make_engine_2_3();
  else if (desc->dim == 3 && desc->fe_degree == 2) eng = smg::make_engine_3_2();
  else eng = smg::make_engine_3_3();
  eng->desc = *desc;
  eng->desc.fine_vertices = desc->fine_vertices;  // read during setup only
  eng->desc.mu_cell = desc->mu_cell;              // read during setup only
  smg_ctx *ctx = new smg_ctx();
  ctx->eng = eng;
  try {
    int dev = 0;
    SMG_HIP(hipGetDevice(&dev));
    ctx->device = dev;
    const auto t0 = std::chrono::steady_clock::now();
    eng->setup();
    eng->t_setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    // the allocation-free entry point's buffer on this device (set-up, so that
    // the entry point itself makes no runtime call besides its launches)
    void *sp = nullptr;
    if (scratch_address(dev, &sp) == hipSuccess) ctx->scratch = sp;
    else (void)hipGetLastError();   // leave no sticky error for the next call
    eng->desc.mu_cell = nullptr;
    eng->desc.fine_vertices = nullptr;
  } catch (const smg::Error &e) {
    eng->free_all();
    delete eng;
    delete ctx;
    return fail(e.code, e.msg);
  } catch (const std::exception &e) {
    eng->free_all();
    delete eng;
    delete ctx;
    return fail(SMG_EDEVICE, e.what());
  }
  *out = ctx;
  g_last_error.clear();
  return SMG_OK;
}

smg_status smg_destroy(smg_ctx *ctx) {
  if (!ctx) return SMG_OK;
  if (ctx->eng) {
    (void)hipStreamSynchronize(ctx->eng->stream);
    ctx->eng->invalidate_graphs();
    ctx->eng->free_all();
    delete ctx->eng;
  }
  delete ctx;
  return SMG_OK;
}

smg_status smg_sizes(const smg_ctx *ctx, int level, int64_t *n_u, int64_t *n_p) {
  smg_status s = check_level(ctx, level);
  if (s != SMG_OK) return s;
  if (n_u) *n_u = ctx->eng->lv[level].Nu;
  if (n_p) *n_p = ctx->eng->lv[level].Np;
  return SMG_OK;
}

smg_status smg_set_stream(smg_ctx *ctx, void *stream) {
  smg_status s = check_ctx(ctx);
  if (s != SMG_OK) return s;
  ctx->eng->stream = (hipStream_t)stream;
  ctx->eng->desc.stream = stream;
  return SMG_OK;
}

smg_status smg_vmult(smg_ctx *ctx, int level, int dtype, const void *x, void *y) {
  smg_status s = check_level(ctx, level);
  if (s == SMG_OK) s = check_dtype(dtype);
  if (s == SMG_OK) s = check_ptrs({x, y});
  if (s != SMG_OK) return s;
  if (x == y) return fail(SMG_EINVAL, "x and y must be distinct");
  SMG_TRY(ctx->eng->vmult(level, dtype, x, y));
}

smg_status smg_vmult_noalloc(smg_ctx *ctx, int level, int dtype, const void *x, void *y) {
  smg_status s = check_level(ctx, level);
  if (s == SMG_OK) s = check_dtype(dtype);
  if (s == SMG_OK) s = check_ptrs({x, y});
  if (s != SMG_OK) return s;
  if (x == y) return fail(SMG_EINVAL, "x and y must be distinct");
  const int64_t need = ctx->eng->vmult_scratch_bytes(level, dtype);
  if (need > (int64_t)SMG_NOALLOC_SCRATCH_BYTES)
    return fail(SMG_EINVAL, "level " + std::to_string(level) + " needs " + std::to_string(need) +
                                " bytes of scratch, more than the fixed " + std::to_string(SMG_NOALLOC_SCRATCH_BYTES) +
                                " of smg_vmult_noalloc (use smg_vmult)");
  if (need > 0 && ctx->scratch == nullptr)
    return fail(SMG_EDEVICE, "hipGetSymbolAddress of the fixed scratch buffer failed at smg_create");
  SMG_TRY(ctx->eng->vmult_scratch(level, dtype, x, y, ctx->scratch));
}

smg_status smg_residual(smg_ctx *ctx, int level, int dtype, const void *x, const void *b, void *r) {
  smg_status s = check_level(ctx, level);
  if (s == SMG_OK) s = check_dtype(dtype);
  if (s == SMG_OK) s = check_ptrs({x, b, r});
  if (s != SMG_OK) return s;
  if (r == x || r == b) return fail(SMG_EINVAL, "r may alias neither x nor b");
  SMG_TRY(ctx->eng->residual(level, dtype, x, b, r));
}

smg_status smg_apply_block(smg_ctx *ctx, int level, int dtype, int block, const void *x, void *y) {
  smg_status s = check_level(ctx, level);
  if (s == SMG_OK) s = check_dtype(dtype);
  if (s == SMG_OK) s = check_ptrs({x, y});
  if (s != SMG_OK) return s;
  if (block < SMG_BLOCK_K || block > SMG_BLOCK_MP) return fail(SMG_EINVAL, "unknown block");
  if (x == y) return fail(SMG_EINVAL, "x and y must be distinct");
  SMG_TRY(ctx->eng->apply_block(level, dtype, block, x, y));
}

smg_status smg_lift_dirichlet(smg_ctx *ctx, int level, int dtype, const void *u_d, void *b) {
  smg_status s = check_level(ctx, level);
  if (s == SMG_OK) s = check_dtype(dtype);
  if (s == SMG_OK) s = check_ptrs({u_d, b});
  if (s != SMG_OK) return s;
  if (u_d == b) return fail(SMG_EINVAL, "u_d and b must be distinct");
  SMG_TRY(ctx->eng->lift_dirichlet(level, dtype, u_d, b));
}

smg_status smg_insert_dirichlet(smg_ctx *ctx, int level, int dtype, const void *u_d, void *x) {
  smg_status s = check_level(ctx, level);
  if (s == SMG_OK) s = check_dtype(dtype);
  if (s == SMG_OK) s = check_ptrs({u_d, x});
  if (s != SMG_OK) return s;
  if (u_d == x) return fail(SMG_EINVAL, "u_d and x must be distinct");
  SMG_TRY(ctx->eng->insert_dirichlet(level, dtype, u_d, x));
}

smg_status smg_get_diagonal(const smg_ctx *ctx, int level, int which, double *out) {
  smg_status s = check_level(ctx, level);
  if (s == SMG_OK) s = check_ptrs({out});
  if (s != SMG_OK) return s;
  if (which != 0 && which != 1) return fail(SMG_EINVAL, "which must be 0 (D_A) or 1 (D~_S)");
  const smg::LevelInfo &I = ctx->eng->lv[level];
  SMG_TRY({
    SMG_HIP(hipMemcpyAsync(out, which == 0 ? I.DA : I.DS, sizeof(double) * (which == 0 ? I.Nu : I.Np),
                           hipMemcpyDeviceToDevice, ctx->eng->stream));
    SMG_HIP(hipStreamSynchronize(ctx->eng->stream));
  });
}

smg_status smg_get_eigs(const smg_ctx *ctx, int level, double *beta_A, double *beta_S) {
  smg_status s = check_level(ctx, level);
  if (s != SMG_OK) return s;
  if (beta_A) *beta_A = ctx->eng->lv[level].beta_A;
  if (beta_S) *beta_S = ctx->eng->lv[level].beta_S;
  return SMG_OK;
}

smg_status smg_set_eigs(smg_ctx *ctx, int level, double beta_A, double beta_S) {
  smg_status s = check_level(ctx, level, 1);
  if (s != SMG_OK) return s;
  if (!(beta_A > 0) || !(beta_S > 0) || !std::isfinite(beta_A) || !std::isfinite(beta_S))
    return fail(SMG_EINVAL, "eigenvalue bounds must be finite and > 0");
  ctx->eng->lv[level].beta_A = beta_A;
  ctx->eng->lv[level].beta_S = beta_S;
  ctx->eng->invalidate_graphs();  // the bounds are baked into the captured cycle
  return SMG_OK;
}

smg_status smg_chebyshev(smg_ctx *ctx, int level, int dtype, int which, const void *r, void *out) {
  smg_status s = check_level(ctx, level, 1);
  if (s == SMG_OK) s = check_dtype(dtype);
  if (s == SMG_OK) s = check_ptrs({r, out});
  if (s != SMG_OK) return s;
  if (which != 0 && which != 1) return fail(SMG_EINVAL, "which must be 0 (A) or 1 (S)");
  if (r == out) return fail(SMG_EINVAL, "r and out must be distinct");
  SMG_TRY(ctx->eng->chebyshev(level, dtype, which, r, out));
}

smg_status smg_velocity_update(smg_ctx *ctx, int level, int dtype, const void *x, const void *b, void *uhat) {
  smg_status s = check_level(ctx, level, 1);
  if (s == SMG_OK) s = check_dtype(dtype);
  if (s == SMG_OK) s = check_ptrs({x, b, uhat});
  if (s != SMG_OK) return s;
  if (uhat == x || uhat == b) return fail(SMG_EINVAL, "uhat must not alias x or b");
  SMG_TRY(ctx->eng->velocity_update(level, dtype, x, b, uhat));
}

smg_status smg_smooth(smg_ctx *ctx, int level, int dtype, void *x, const void *b, int steps) {
  smg_status s = check_level(ctx, level, 1);
  if (s == SMG_OK) s = check_dtype(dtype);
  if (s == SMG_OK) s = check_ptrs({x, b});
  if (s != SMG_OK) return s;
  if (steps < 0) return fail(SMG_EINVAL, "steps must be >= 0");
  if (x == b) return fail(SMG_EINVAL, "x and b must be distinct");
  SMG_TRY(ctx->eng->smooth(level, dtype, x, b, steps));
}

smg_status smg_restrict(smg_ctx *ctx, int fine_level, int dtype, const void *r_fine, void *r_coarse) {
  smg_status s = check_level(ctx, fine_level, 1);
  if (s == SMG_OK) s = check_dtype(dtype);
  if (s == SMG_OK) s = check_ptrs({r_fine, r_coarse});
  if (s != SMG_OK) return s;
  SMG_TRY(ctx->eng->restrict_(fine_level, dtype, r_fine, r_coarse));
}

smg_status smg_prolongate_add(smg_ctx *ctx, int fine_level, int dtype, const void *w_coarse, void *x_fine) {
  smg_status s = check_level(ctx, fine_level, 1);
  if (s == SMG_OK) s = check_dtype(dtype);
  if (s == SMG_OK) s = check_ptrs({w_coarse, x_fine});
  if (s != SMG_OK) return s;
  SMG_TRY(ctx->eng->prolongate_add(fine_level, dtype, w_coarse, x_fine));
}

smg_status smg_coarse_solve(smg_ctx *ctx, int dtype, const void *b0, void *x0) {
  smg_status s = check_ctx(ctx);
  if (s == SMG_OK) s = check_dtype(dtype);
  if (s == SMG_OK) s = check_ptrs({b0, x0});
  if (s != SMG_OK) return s;
  if (b0 == x0) return fail(SMG_EINVAL, "b0 and x0 must be distinct");
  SMG_TRY(ctx->eng->coarse_solve(dtype, b0, x0));
}

smg_status smg_vcycle(smg_ctx *ctx, int level, int dtype, void *x, const void *b) {
  smg_status s = check_level(ctx, level);
  if (s == SMG_OK) s = check_dtype(dtype);
  if (s == SMG_OK) s = check_ptrs({x, b});
  if (s != SMG_OK) return s;
  if (x == b) return fail(SMG_EINVAL, "x and b must be distinct");
  SMG_TRY(ctx->eng->vcycle(level, dtype, x, b));
}

smg_status smg_solve(smg_ctx *ctx, double *x, const double *b, double rtol, int maxit, smg_solve_info *info) {
  smg_status s = check_ctx(ctx);
  if (s == SMG_OK) s = check_ptrs({x, b});
  if (s != SMG_OK) return s;
  if (!(rtol > 0) || maxit < 0) return fail(SMG_EINVAL, "need rtol > 0 and maxit >= 0");
  if (x == b) return fail(SMG_EINVAL, "x and b must be distinct");
  try {
    smg_status r = ctx->eng->solve(x, b, rtol, maxit, info);
    if (r == SMG_ENOTCONV) g_last_error = "iteration limit reached before the tolerance";
    else if (r == SMG_EBREAKDOWN) g_last_error = "breakdown (NaN/Inf) in FGMRES";
    else g_last_error.clear();
    return r;
  } catch (const smg::Error &e) {
    return fail(e.code, e.msg);
  }
}

smg_status smg_solve_stationary(smg_ctx *ctx, double *x, const double *b, double rtol, int maxit, smg_solve_info *info) {
  smg_status s = check_ctx(ctx);
  if (s == SMG_OK) s = check_ptrs({x, b});
  if (s != SMG_OK) return s;
  if (!(rtol > 0) || maxit < 0) return fail(SMG_EINVAL, "need rtol > 0 and maxit >= 0");
  if (x == b) return fail(SMG_EINVAL, "x and b must be distinct");
  try {
    smg_status r = ctx->eng->solve_stationary(x, b, rtol, maxit, info);
    if (r == SMG_ENOTCONV) g_last_error = "iteration limit reached before the tolerance";
    else if (r == SMG_EBREAKDOWN) g_last_error = "breakdown: NaN/Inf or residual growth by more than 1e3";
    else g_last_error.clear();
    return r;
  } catch (const smg::Error &e) {
    return fail(e.code, e.msg);
  }
}

smg_status smg_node_coordinates(const smg_ctx *ctx, int level, double *xyz) {
  smg_status s = check_level(ctx, level);
  if (s == SMG_OK) s = check_ptrs({xyz});
  if (s != SMG_OK) return s;
  SMG_TRY(ctx->eng->node_coordinates(level, xyz));
}

struct smg_batch {
  smg::BatchDriver drv;
  std::vector<smg_ctx *> ctxs;
  int device = 0;
  int variant = 0;
};

namespace {
// Kernel-variant choices the batch autotuner times: the largest 2D level
// (cells per direction) that runs one wave per output field, the two-stage
// fused launches (tiles owning 5 x 5 cells) and the three-stage launches
// (3 x 3); the others run one wave per 8 x 8 tile owning 7 x 7 cells.
// Variant 0 is the solvers' default.
constexpr int kBatchVariants[][3] = {
    {256, 512, 128}, {0, 0, 0}, {256, 0, 0}, {256, 256, 0}, {256, 256, 128}, {256, 256, 256}, {512, 512, 128}};
constexpr int kNumBatchVariants = (int)(sizeof(kBatchVariants) / sizeof(kBatchVariants[0]));

smg_status check_batch(const smg_batch *b) {
  if (!b) return fail(SMG_EINVAL, "null batch");
  return SMG_OK;
}
}  // namespace

smg_status smg_batch_create(smg_ctx *const *ctxs, int n, void *stream, smg_batch **out) {
  if (!out) return fail(SMG_EINVAL, "null output pointer");
  *out = nullptr;
  if (!ctxs || n < 1) return fail(SMG_EINVAL, "need n >= 1 contexts");
  for (int i = 0; i < n; ++i) {
    smg_status s = check_ctx(ctxs[i]);
    if (s != SMG_OK) return s;
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) return fail(SMG_EINVAL, "a context appears twice in the batch");
    const smg_desc &d = ctxs[i]->eng->desc;
    if (d.dim != 2) return fail(SMG_EUNSUPPORTED, "batched solves: 2D problems only");
    if (d.cycle_index != 1) return fail(SMG_EUNSUPPORTED, "batched solves: V-cycle only");
    if (d.form != SMG_FORM_GRAD) return fail(SMG_EUNSUPPORTED, "batched solves: gradient form only");
    if (ctxs[i]->device != ctxs[0]->device) return fail(SMG_EINVAL, "batched contexts must share one device");
  }
  smg_batch *b = new smg_batch();
  try {
    b->device = ctxs[0]->device;
    b->ctxs.assign(ctxs, ctxs + n);
    std::vector<smg::EngineBase *> e;
    for (int i = 0; i < n; ++i) e.push_back(ctxs[i]->eng);
    b->drv.stream = (hipStream_t)stream;
    b->drv.init(e);
    b->drv.build_cycle();
  } catch (const smg::Error &e) {
    delete b;
    return fail(e.code, e.msg);
  } catch (const std::exception &e) {
    delete b;
    return fail(SMG_EDEVICE, std::string("exception: ") + e.what());
  }
  *out = b;
  g_last_error.clear();
  return SMG_OK;
}

smg_status smg_batch_destroy(smg_batch *b) {
  if (!b) return SMG_OK;
  (void)hipStreamSynchronize(b->drv.stream);
  delete b;
  return SMG_OK;
}

smg_status smg_batch_solve(smg_batch *b, double *const *x, const double *const *rhs, double rtol, int maxit,
                           smg_solve_info *infos) {
  smg_status s = check_batch(b);
  if (s != SMG_OK) return s;
  if (!x || !rhs) return fail(SMG_EINVAL, "null vector arrays");
  for (size_t i = 0; i < b->ctxs.size(); ++i) {
    s = check_ptrs({x[i], rhs[i]});
    if (s != SMG_OK) return s;
    if (x[i] == rhs[i]) return fail(SMG_EINVAL, "x and b must be distinct");
  }
  if (!(rtol > 0) || maxit < 0) return fail(SMG_EINVAL, "need rtol > 0 and maxit >= 0");
  try {
    smg_status r = b->drv.solve(x, rhs, rtol, maxit, infos);
    if (r == SMG_ENOTCONV) g_last_error = "iteration limit reached before the tolerance (some problem)";
    else if (r == SMG_EBREAKDOWN) g_last_error = "breakdown (NaN/Inf) in FGMRES (some problem)";
    else g_last_error.clear();
    return r;
  } catch (const smg::Error &e) {
    return fail(e.code, e.msg);
  } catch (const std::exception &e) {
    return fail(SMG_EDEVICE, std::string("exception: ") + e.what());
  }
}

smg_status smg_batch_precondition(smg_batch *b, const double *const *v, double *const *z) {
  smg_status s = check_batch(b);
  if (s != SMG_OK) return s;
  if (!v || !z) return fail(SMG_EINVAL, "null vector arrays");
  for (size_t i = 0; i < b->ctxs.size(); ++i) {
    s = check_ptrs({v[i], z[i]});
    if (s != SMG_OK) return s;
  }
  SMG_TRY(b->drv.precondition(v, z));
}

smg_status smg_batch_info(const smg_batch *b, int *packed_launches_per_cycle, int *variant) {
  smg_status s = check_batch(b);
  if (s != SMG_OK) return s;
  if (packed_launches_per_cycle)
    *packed_launches_per_cycle = b->drv.cycle_plan ? (int)b->drv.cycle_plan->launches.size() : 0;
  if (variant) *variant = b->variant;
  return SMG_OK;
}

namespace {
void batch_autotune_impl(smg_batch *b, int probe_cycles, int *best, double *times_ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  SMG_HIP(hipEventCreate(&e0));
  SMG_HIP(hipEventCreate(&e1));
  double tbest = 1e300;
  int ibest = 0;
  try {
    for (int c = 0; c < kNumBatchVariants; ++c) {
      for (smg::EngineBase *e : b->drv.eng)
        e->set_variants(kBatchVariants[c][0], kBatchVariants[c][1], kBatchVariants[c][2]);
      b->drv.build_cycle();
      SMG_HIP(hipGraphLaunch(b->drv.gexec, b->drv.stream));   // warm-up
      SMG_HIP(hipEventRecord(e0, b->drv.stream));
      for (int k = 0; k < probe_cycles; ++k) SMG_HIP(hipGraphLaunch(b->drv.gexec, b->drv.stream));
      SMG_HIP(hipEventRecord(e1, b->drv.stream));
      SMG_HIP(hipEventSynchronize(e1));
      float ms = 0.0f;
      SMG_HIP(hipEventElapsedTime(&ms, e0, e1));
      if (times_ms) times_ms[c] = ms / probe_cycles;
      if (ms < 0.97 * tbest) {   // a clear gain only: near-equal timings keep the earlier choice
        tbest = ms;
        ibest = c;
      }
    }
  } catch (...) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  for (smg::EngineBase *e : b->drv.eng)
    e->set_variants(kBatchVariants[ibest][0], kBatchVariants[ibest][1], kBatchVariants[ibest][2]);
  b->drv.build_cycle();
  b->variant = ibest;
  if (best) *best = ibest;
}
}  // namespace

smg_status smg_batch_autotune(smg_batch *b, int probe_cycles, int *best, double *times_ms, int *ncand) {
  smg_status s = check_batch(b);
  if (s != SMG_OK) return s;
  if (probe_cycles < 1) return fail(SMG_EINVAL, "probe_cycles must be >= 1");
  if (ncand) *ncand = kNumBatchVariants;
  SMG_TRY(batch_autotune_impl(b, probe_cycles, best, times_ms));
}

smg_status smg_gradient(smg_ctx *ctx, const double *x, const double *lam, double *g_logmu, double *g_f) {
  smg_status s = check_ctx(ctx);
  if (s == SMG_OK) s = check_ptrs({x, lam});
  if (s != SMG_OK) return s;
  SMG_TRY(ctx->eng->gradient(x, lam, g_logmu, g_f));
}

smg_status smg_pressure_mean_adjoint(smg_ctx *ctx, double *g) {
  smg_status s = check_ctx(ctx);
  if (s == SMG_OK) s = check_ptrs({g});
  if (s != SMG_OK) return s;
  SMG_TRY(ctx->eng->pressure_mean_adjoint(g));
}

smg_status smg_profile(smg_ctx *ctx, int enable) {
  smg_status s = check_ctx(ctx);
  if (s != SMG_OK) return s;
  SMG_TRY({
    SMG_HIP(hipStreamSynchronize(ctx->eng->stream));
    ctx->eng->profile_reset();
    ctx->eng->profiling = enable != 0;
  });
}

smg_status smg_profile_report(smg_ctx *ctx, char *buf, int64_t cap, int64_t *len) {
  smg_status s = check_ctx(ctx);
  if (s != SMG_OK) return s;
  if (cap < 0) return fail(SMG_EINVAL, "cap must be >= 0");
  SMG_TRY({
    std::string r = ctx->eng->profile_report();
    if (len) *len = (int64_t)r.size();
    if (buf && cap > 0) {
      const size_t n = std::min((size_t)(cap - 1), r.size());
      std::memcpy(buf, r.data(), n);
      buf[n] = '\0';
    }
  });
}

const char *smg_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
