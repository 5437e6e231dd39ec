/*
 * smg.h -- C ABI of a matrix-free monolithic geometric multigrid solver for
 * Q_k-Q_{k-1} Taylor-Hood discretisations of the Stokes and generalized
 * Stokes problems on box meshes, for AMD Instinct MI355X (gfx950).
 *
 * Method: Jodlbauer, Langer, Wick, Zulehner, "Matrix-free Monolithic
 * Multigrid Methods for Stokes and Generalized Stokes Problems":
 *   problem and mixed weak form        Sec. 1 (Eqs. of Stokes / generalized
 *                                      Stokes), Sec. 2 (forms a, b, <F,v>)
 *   matrix-free operator K x           Sec. 3.1 (K x = sum P_tau K_tau P_tau^T x,
 *                                      sum factorisation)
 *   transfers                          Sec. 3.2 (canonical injection, R = P^T)
 *   smoother                           Sec. 1 (inexact symmetric Uzawa),
 *                                      Sec. 3.3.1 (Chebyshev-Jacobi, Lemma 1,
 *                                      Schur diagonals, Algorithm 2)
 *   multigrid cycle, coarse solve      Algorithm 1, Sec. 4.1
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Mesh: the box [box_lo, box_hi] with n_coarse[a] * 2^l cells in direction a
 * on level l = 0 (coarsest) ... n_levels-1 (finest); optionally the finest
 * vertices are given (bi-/trilinear cells), coarser levels take the finest
 * vertex at the same lattice point.
 *
 * Vector layout on level l: [u_1 | ... | u_d | p], each velocity component on
 * the (k n_x + 1) x (k n_y + 1) [x (k n_z + 1)] node lattice, the pressure on
 * the ((k-1) n_x + 1) x ... lattice, lexicographic with x fastest.  Length
 * N = d * Nv + Np (see smg_sizes).  Every velocity node on the box boundary
 * carries a Dirichlet condition, homogeneous for the operators: they act as
 * the identity on those entries and ignore them as inputs of the free rows
 * (non-zero boundary values are lifted, smg_lift_dirichlet).
 *
 * Memory: every vector argument is a DEVICE pointer owned by the caller, on
 * the device that was current at smg_create, of the element type `dtype`
 * (SMG_F64: double, SMG_F32: float), contiguous, of the length stated.  The
 * library owns all level data and workspace, allocated once in smg_create and
 * released in smg_destroy; apart from two first-use items (the HIP graph of
 * the preconditioning cycle, on the first smg_solve; on box meshes the vertex
 * lattice of smg_gradient, on its first call) no other entry point allocates
 * device memory.
 *
 * Streams: all device work is enqueued on the stream of the context
 * (smg_desc.stream or smg_set_stream; NULL = the default stream).  Entry
 * points other than smg_create, smg_solve, smg_solve_stationary and the
 * smg_get_* queries return without synchronising.
 *
 * Errors: every entry point returns an smg_status; on failure a message is
 * available from smg_last_error() (per thread).  Invalid arguments are
 * rejected before any device work is enqueued.
 */
#ifndef SMG_H
#define SMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct smg_ctx smg_ctx;

typedef enum {
  SMG_OK = 0,
  SMG_EINVAL = -1,        /* invalid argument or descriptor                 */
  SMG_ENOMEM = -2,        /* device or host allocation failed               */
  SMG_EDEVICE = -3,       /* a HIP runtime call failed                      */
  SMG_ENOTCONV = -4,      /* iteration limit reached before the tolerance   */
  SMG_EBREAKDOWN = -5,    /* NaN/Inf or residual growth in an iteration     */
  SMG_EUNSUPPORTED = -6   /* valid but not built (e.g. fe_degree 4)         */
} smg_status;

typedef enum { SMG_F64 = 0, SMG_F32 = 1 } smg_dtype;

/* Approximations of the Schur-complement diagonal, Sec. 3.3.1:
 *   SMG_SCHUR_D   diag(B diag(A)^-1 B^T)                     (assembled B entries)
 *   SMG_SCHUR_LOC sum_tau diag(B_tau diag(A_tau)^-1 B_tau^T) (cell-local;
 *                 Dirichlet columns left out; box cells from the 1D cell
 *                 matrices, vertex-given cells by quadrature; gradient form
 *                 only: SMG_EUNSUPPORTED with SMG_FORM_EPS)
 *   SMG_SCHUR_P   diag(M_p)                                  (pressure mass)
 *   SMG_SCHUR_EXACT diag(B A_hat^-1 B^T), A_hat^-1 = sigma Cheb(A, D_A, k_A):
 *                 the diagonal the three choices above approximate; built
 *                 at set-up by probing (about ((k-1)(k_A+3)+1)^d applications
 *                 of A_hat^-1 per level), for comparisons on small meshes
 * With c_pressure != 0 the diagonal of C = c_pressure M_p is added.        */
typedef enum { SMG_SCHUR_D = 0, SMG_SCHUR_LOC = 1, SMG_SCHUR_P = 2, SMG_SCHUR_EXACT = 3 } smg_schur_diag;

/* Blocks of K = [A B^T; B -C] for smg_apply_block (Sec. 1, saddle-point
 * system; Sec. 2, forms a and b):
 *   SMG_BLOCK_K    y = K x                       x, y length N
 *   SMG_BLOCK_A    y = A u                       u, y length d*Nv
 *   SMG_BLOCK_BT   y = B^T p                     p length Np, y length d*Nv (0 on Dirichlet rows)
 *   SMG_BLOCK_B    y = B u                       u length d*Nv, y length Np
 *   SMG_BLOCK_MASS y = M_v f per component       f, y length d*Nv; f is used at
 *                  every node (also on the boundary), y is 0 on Dirichlet rows:
 *                  the load vector <F, v> of a nodal FE field f (Sec. 2).
 *   SMG_BLOCK_MP   y = M_p p                     p, y length Np: the pressure mass
 *                  matrix (its row sums M_p 1 weight the pressure mean).      */
typedef enum {
  SMG_BLOCK_K = 0, SMG_BLOCK_A = 1, SMG_BLOCK_BT = 2, SMG_BLOCK_B = 3, SMG_BLOCK_MASS = 4, SMG_BLOCK_MP = 5
} smg_block;

typedef enum { SMG_PRECOND_F64 = 0, SMG_PRECOND_F32 = 1 } smg_precision;

/* Viscous term of the bilinear form a (Sec. 2):
 *   SMG_FORM_GRAD  a(u,v) = int mu grad u : grad v + gamma rho u.v
 *   SMG_FORM_EPS   a(u,v) = int mu eps(u) : eps(v) + gamma rho u.v,
 *                  eps(u) = (grad u + grad u^T) / 2 (as printed, no factor 2);
 *                  couples the velocity components.  Runs on every mesh
 *                  through the quadrature-point kernel of vertex-given cells
 *                  (a box mesh is passed to it as its vertex lattice);
 *                  SMG_SCHUR_LOC is not available with it.               */
typedef enum { SMG_FORM_GRAD = 0, SMG_FORM_EPS = 1 } smg_form;

typedef struct {
  int dim;                 /* 2 or 3                                                  */
  int fe_degree;           /* k: velocity Q_k, pressure Q_{k-1}; k = 2 or 3            */
  int n_coarse[3];         /* cells per direction on level 0, each >= 2 (App. A:       */
                           /* no cell with two opposite boundary faces)                */
  int n_levels;            /* number of levels, >= 2                                   */
  double box_lo[3], box_hi[3];
  const double *fine_vertices; /* HOST, ((n_f+1)^d x d) vertex coordinates of the      */
                           /* finest mesh, x fastest; NULL = Cartesian box lattice.    */
                           /* Boundary vertices must lie on the box boundary.          */
  double mu;               /* viscosity (> 0), used when mu_cell == NULL               */
  const double *mu_cell;   /* HOST, per finest cell (x fastest), > 0; coarse cells     */
                           /* take the mean of their 2^d children.                     */
  double gamma, rho;       /* generalized Stokes reaction gamma*rho >= 0 (Eq. 2)       */
  double c_pressure;       /* C = c_pressure * M_p >= 0 (Sec. 1 allows C >= 0)          */
  int cheb_deg_A;          /* k_A >= 0  (Algorithm 2)                                  */
  int cheb_deg_S;          /* k_S >= 0                                                 */
  int smooth_steps;        /* m >= 1 pre- and post-smoothing steps (Algorithm 1)       */
  int cycle_index;         /* 1 = V-cycle, 2 = W-cycle (Algorithm 1)                   */
  int schur_diag;          /* smg_schur_diag                                           */
  int precision;           /* smg_precision: the multigrid preconditioner in smg_solve */
  int fgmres_restart;      /* Krylov basis size of smg_solve, 1..200                   */
  void *stream;            /* hipStream_t, or NULL                                     */
  int form;                /* smg_form: the viscous term of the form a (Sec. 2)        */
} smg_desc;

typedef struct {
  int iterations;          /* outer iterations performed                              */
  double rel_residual;     /* ||b - K x||_2 / ||b||_2 at return, FP64                  */
  double rate_q;           /* stationary protocol: (r_j / r_{j-3})^(1/3), Sec. 4.1     */
  double t_solve_ms;       /* wall time of the call                                    */
  double t_setup_ms;       /* wall time of smg_create for this context (hierarchy,     */
                           /* diagonals, eigenvalue bounds, coarse inverse)            */
  double *history;         /* HOST array provided by the caller or NULL; receives the  */
  int history_capacity;    /* relative residual per iteration (entry 0 = initial)      */
  int history_len;         /* entries written                                          */
} smg_solve_info;

/* Fill *desc with defaults: 2D, k = 2, 4x4 coarse cells, 3 levels, unit box,
 * mu = rho = 1, gamma = c_pressure = 0, (k_A, k_S, m) = (1, 1, 2), V-cycle,
 * SMG_SCHUR_D, FP64 preconditioner, restart 30, default stream.              */
void smg_desc_default(smg_desc *desc);

/* Build the level hierarchy, the diagonals D_A and D~_S of every level
 * (Sec. 3.3.1), the eigenvalue bounds beta_A ~ lambda_max(D_A^-1 A) and
 * beta_S ~ lambda_max(D~_S^-1 S~) by Lanczos (Algorithm 2; the paper asks for
 * a close approximation: 30 Lanczos steps in the D inner product from a
 * SplitMix64 start vector, times 1.02), the dense inverse of the bordered
 * coarse matrix [K_0 m; m^T 0], m = (0, M_p 1) (Sec. 4.1, direct coarse solve;
 * the border fixes the pressure mean; with c_pressure > 0, K_0 is regular and
 * is inverted without the border), and all workspace.  Synchronises.
 * Errors: EINVAL for an invalid descriptor, EUNSUPPORTED for dim/degree not
 * built, ENOMEM, EDEVICE.  On success *out owns everything until smg_destroy. */
smg_status smg_create(const smg_desc *desc, smg_ctx **out);
smg_status smg_destroy(smg_ctx *ctx);

/* Sizes of level `level`: velocity DoFs d*Nv, pressure DoFs Np (N = sum). */
smg_status smg_sizes(const smg_ctx *ctx, int level, int64_t *n_u, int64_t *n_p);
smg_status smg_set_stream(smg_ctx *ctx, void *stream);

/* y = K_l x (Sec. 3.1): the cell-wise sum-factorised application of the
 * saddle-point operator.  x, y length N, distinct. */
smg_status smg_vmult(smg_ctx *ctx, int level, int dtype, const void *x, void *y);

/* y = K_l x as smg_vmult, allocating nothing: for callers that cannot
 * allocate device memory while they run (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  The per-cell partial
 * results that the vertex-given (multilinear) cell kernels produce before
 * summing them per node live in one fixed 16 MiB device buffer per GPU
 * (a static device array, held until the process ends; its address is
 * looked up once per device in smg_create) instead of the level's own
 * buffer; box-cell kernels need no such buffer.  Levels whose partial
 * results need more than 16 MiB (about 9,500 3D Q3 cells in FP64, 23,500 3D
 * Q2 cells, 95,000 2D Q2 cells) are rejected with SMG_EINVAL before any
 * device work.  Every call on one GPU shares that buffer: calls that overlap
 * on one GPU (other streams, other threads, other contexts) race and must be
 * ordered by the caller.  Kernel timing (smg_profile) does not record these
 * launches.  x, y as smg_vmult; asynchronous on the context's stream. */
smg_status smg_vmult_noalloc(smg_ctx *ctx, int level, int dtype, const void *x, void *y);

/* r = b - K_l x (Algorithm 1, residual step).  r may alias neither x nor b. */
smg_status smg_residual(smg_ctx *ctx, int level, int dtype, const void *x, const void *b, void *r);

/* One block of K (see smg_block).  x and y distinct. */
smg_status smg_apply_block(smg_ctx *ctx, int level, int dtype, int block, const void *x, void *y);

/* Non-homogeneous Dirichlet data (Sec. 2: u = u_D on the boundary; the
 * paper's driven-cavity examples) by lifting.  u_d is a velocity vector of
 * length d*Nv whose entries on the Dirichlet nodes (every node on the box
 * boundary) are the prescribed values; its other entries are not used.
 * smg_lift_dirichlet updates the right-hand side b (length N) in place:
 *   b_u <- b_u - (A u~ + 0) on free rows,  b_u <- 0 on Dirichlet rows,
 *   b_p <- b_p - B u~,
 * where u~ = u_d on the Dirichlet nodes, 0 elsewhere, and A, B keep their
 * Dirichlet columns (the operator before constraints).  The solution x0 of
 * K x0 = b (homogeneous on the boundary, e.g. by smg_solve) then gives the
 * solution of the problem with data u_D as x0 + u~, which
 * smg_insert_dirichlet forms by writing u_d into the Dirichlet entries of x.
 * b (resp. x) and u_d must be distinct device arrays of the level's dtype.
 * Uses the level's internal work vectors (not concurrently with a solve on
 * the same handle).  Errors: EINVAL (level, dtype, NULL or aliasing). */
smg_status smg_lift_dirichlet(smg_ctx *ctx, int level, int dtype, const void *u_d, void *b);
smg_status smg_insert_dirichlet(smg_ctx *ctx, int level, int dtype, const void *u_d, void *x);

/* Copy the FP64 diagonal D_A (which = 0, length d*Nv; 1 on Dirichlet rows) or
 * D~_S (which = 1, length Np) of level l into the device array out. */
smg_status smg_get_diagonal(const smg_ctx *ctx, int level, int which, double *out);

/* The Chebyshev interval bounds beta_A, beta_S of level l (Algorithm 2).
 * smg_set_eigs overrides them (e.g. to share values with another
 * implementation); the scaling sigma, tau depends only on k_A, k_S. */
smg_status smg_get_eigs(const smg_ctx *ctx, int level, double *beta_A, double *beta_S);
smg_status smg_set_eigs(smg_ctx *ctx, int level, double beta_A, double beta_S);

/* out = sigma Cheb(A, D_A, k_A) r (which = 0, vectors length d*Nv) or
 * out = tau Cheb(S~, D~_S, k_S) r, S~ = B A_hat^-1 B^T + C (which = 1, length
 * Np): the scaled Chebyshev-Jacobi preconditioners A_hat^-1, S_hat^-1 of
 * Sec. 3.3.1, by the three-term Chebyshev recurrence from a zero start. */
smg_status smg_chebyshev(smg_ctx *ctx, int level, int dtype, int which, const void *r, void *out);

/* uhat = u + sigma Cheb(A, D_A, k_A) (f - A u - B^T p): the velocity update
 * that opens an inexact symmetric Uzawa step (Sec. 1, Sec. 3.3.1), on level
 * l >= 1.  x = (u, p) and b = (f, g) are level vectors (length N, layout of
 * smg_vmult); uhat (caller-owned device memory) has the velocity length d*Nv.
 * Constrained velocity rows are treated as in smg_smooth.  On 2D box levels
 * up to the two-stage fusion threshold this is the one launch the smoother
 * uses (residual and first Chebyshev step fused), elsewhere the residual and
 * the Chebyshev steps run as separate launches.  SMG_EINVAL for uhat
 * aliasing x or b. */
smg_status smg_velocity_update(smg_ctx *ctx, int level, int dtype, const void *x, const void *b, void *uhat);

/* `steps` inexact symmetric Uzawa steps (Sec. 1; compact form of Sec. 3.3.1)
 * on level l >= 1, in place on x (length N) for right-hand side b. */
smg_status smg_smooth(smg_ctx *ctx, int level, int dtype, void *x, const void *b, int steps);

/* r_c = R r_f = P^T r_f from level `fine_level` to fine_level-1 (Sec. 3.2). */
smg_status smg_restrict(smg_ctx *ctx, int fine_level, int dtype, const void *r_fine, void *r_coarse);

/* x_f += P w_c from level fine_level-1 to fine_level (Sec. 3.2). */
smg_status smg_prolongate_add(smg_ctx *ctx, int fine_level, int dtype, const void *w_coarse, void *x_fine);

/* x_0 = K_0^+ b_0 on level 0 by the dense bordered inverse, computed in FP64
 * for either dtype (Sec. 4.1).  b_0 should satisfy 1^T b_p = 0.  With
 * c_pressure > 0: x_0 = K_0^-1 b_0 (no border, no condition on b_0). */
smg_status smg_coarse_solve(smg_ctx *ctx, int dtype, const void *b0, void *x0);

/* One multigrid cycle (Algorithm 1, cycle index of the descriptor) on level
 * l for K_l x = b, in place on x (initial guess). */
smg_status smg_vcycle(smg_ctx *ctx, int level, int dtype, void *x, const void *b);

/* Solve K x = b on the finest level to ||b - K x|| <= rtol ||b|| by FP64
 * flexible GMRES(fgmres_restart), right-preconditioned by one multigrid cycle
 * per iteration in the precision of desc.precision (FP32: the FP64 Krylov
 * vector is cast to FP32, the FP32 cycle is applied, the result is cast back;
 * the coarse solve stays FP64).  x (FP64, length N) is the initial guess and
 * the result; for c_pressure = 0 the pressure of the result is shifted to
 * M_p-weighted mean zero (with c_pressure > 0 it is unique and left as is).
 * Returns ENOTCONV if maxit iterations do not reach rtol (x holds the last
 * iterate), EBREAKDOWN on NaN/Inf.  Synchronises; info may be NULL. */
smg_status smg_solve(smg_ctx *ctx, double *x, const double *b, double rtol, int maxit, smg_solve_info *info);

/* The paper's protocol (Sec. 4.1): stationary multigrid x <- MG(x, b) in FP64
 * until ||b - K x|| <= rtol ||b - K x_0|| or maxit cycles; info->rate_q is the
 * mean reduction of the last three iterations. */
smg_status smg_solve_stationary(smg_ctx *ctx, double *x, const double *b, double rtol, int maxit, smg_solve_info *info);

/* Batched solves of independent problems (Sec. 1: the generalized Stokes
 * problem; Sec. 4.3 reports convergence rates robust in gamma, which lets one
 * smoother parameter set serve every problem of a batch).  A batch groups
 * existing contexts -- 2D, box cells, gradient form, V-cycle, one device,
 * one preconditioner precision -- of any sizes and gamma.  Every stage of
 * the multigrid cycle runs for all problems in one packed launch (a launch
 * whose table gives each problem's kernel arguments and block range; the
 * problems whose level takes another kernel variant form another launch of
 * the same stage), and the whole batched cycle is one HIP graph launch.
 *
 * smg_batch_create: records every context's preconditioning cycle, packs it
 * and captures the graph (allocates the packed tables, the graph and the
 * reduction buffers; synchronises).  `stream` (hipStream_t or NULL) carries
 * all batch work.  The contexts must stay alive, unused outside the batch
 * while a batch call runs, and outlive the batch.  Errors: EINVAL,
 * EUNSUPPORTED (3D, vertex-given cells, the eps form, W-cycle), EDEVICE. */
typedef struct smg_batch smg_batch;
smg_status smg_batch_create(smg_ctx *const *ctxs, int n, void *stream, smg_batch **out);
smg_status smg_batch_destroy(smg_batch *batch);

/* Solve K_i x_i = b_i for every problem i to ||b_i - K_i x_i|| <= rtol ||b_i||:
 * FGMRES(m) per problem (m = the smallest fgmres_restart of the batch),
 * right-preconditioned by one cycle in each context's precision, with the
 * problems' Krylov iterations in lockstep: each problem keeps its own basis,
 * coefficients and stopping test (its iterations are those of smg_solve), and
 * each step -- residual, norms, the copies around the cycle, the batched
 * cycle, the operator, both Gram-Schmidt passes, the normalisation -- is one
 * packed launch for all problems, with one copy of all problems'
 * coefficients to the host per iteration.  x[i], b[i]: HOST arrays of n
 * DEVICE FP64 pointers (length N_i of the finest level); x[i] is the initial
 * guess.  infos: HOST array of n (may be NULL).  Pressures are normalised as
 * by smg_solve.  Returns the first failing problem's status (ENOTCONV,
 * EBREAKDOWN); every problem is attempted.  Synchronises. */
smg_status smg_batch_solve(smg_batch *batch, double *const *x, const double *const *b, double rtol, int maxit,
                           smg_solve_info *infos);

/* z_i = M_i^-1 v_i (one cycle from zero, in each context's precision) for
 * every problem with one graph launch; v, z: HOST arrays of DEVICE FP64
 * pointers.  Synchronises. */
smg_status smg_batch_precondition(smg_batch *batch, const double *const *v, double *const *z);

/* Packed launches per batched cycle and the kernel-variant choice in use. */
smg_status smg_batch_info(const smg_batch *batch, int *packed_launches_per_cycle, int *variant);

/* Autotuner of the batch's tile shapes: for each built-in choice of which 2D
 * levels run one wave per output field, the two-stage fused launches (tiles
 * owning 5 x 5 cells) and the three-stage launches (3 x 3 cells) instead of
 * one wave per 8 x 8 tile owning 7 x 7 cells, re-packs the batched cycle and
 * times probe_cycles graph launches of it; keeps the fastest (a later choice
 * must be 3 % faster) for the batch's contexts.  times_ms: HOST array of at
 * least 16 entries or NULL; *ncand receives the number of choices. */
smg_status smg_batch_autotune(smg_batch *batch, int probe_cycles, int *best, double *times_ms, int *ncand);

/* HOST array xyz (Nv x d, node-major) <- physical coordinates of the velocity
 * lattice nodes of level l (for evaluating nodal data such as f). */
smg_status smg_node_coordinates(const smg_ctx *ctx, int level, double *xyz);

/* Adjoint-state gradients on the finest level.  For the solution x of
 * K(mu) x = [Z M_v f; 0] (Z zeroes the Dirichlet rows; f a nodal velocity
 * field) and an objective J(x), let lam solve K lam = dJ/dx (K = K^T, so
 * smg_solve with that right-hand side).  K depends on the per-cell viscosity
 * only through mu_tau int_tau grad u : grad v (Sec. 2, form a; with
 * SMG_FORM_EPS mu_tau int_tau eps(u) : eps(v)), hence
 *   g_logmu[tau] = dJ/d log mu_tau = -mu_tau int_tau grad lam_u : grad u
 *                  (-mu_tau int_tau eps(lam_u) : eps(u) with SMG_FORM_EPS),
 *   g_f          = dJ/df          = M_v Z lam_u   (every velocity node),
 * with the Dirichlet entries of x and lam taken as zero (cell integrals by
 * the operator's quadrature, on box or vertex-given cells).
 * x, lam: DEVICE FP64, length N of the finest level.  g_logmu: DEVICE FP64,
 * one entry per finest cell (x fastest), or NULL.  g_f: DEVICE FP64, length
 * d*Nv, or NULL.  Asynchronous on the context's stream. */
smg_status smg_gradient(smg_ctx *ctx, const double *x, const double *lam, double *g_logmu, double *g_f);

/* Transpose of the pressure normalisation that smg_solve applies to its
 * result (Sec. 2: the pressure space is L^2_0; the returned pressure has
 * M_p-weighted mean zero, p <- p - 1 (m . p) / (m . 1), m = M_p 1), for
 * adjoint computations: with J depending on the normalised solution, the
 * adjoint right-hand side is g <- g_p - m (1 . g_p) / (m . 1) on the pressure
 * block (velocity block unchanged).  With c_pressure > 0 the solution is not
 * normalised and g is left as it is.  g: DEVICE FP64, length N of the finest
 * level, in place.  Asynchronous on the context's stream. */
smg_status smg_pressure_mean_adjoint(smg_ctx *ctx, double *g);

/* Kernel timing for measurement: with enable != 0, every later operator-kernel
 * launch of this context is bracketed by two HIP events recorded on the
 * context's stream (previous records are discarded); enable == 0 stops.
 * smg_profile_report synchronises the stream and writes one line per kernel
 * key "name/vVARIANT/blkBLOCKS/dtype/NXxNYxNZ count total_ms total_bytes" into buf
 * (NUL-terminated, truncated to cap bytes); *len receives the full length.
 * total_bytes is the algorithmic HBM traffic of those launches: each vector
 * the kernel reads or writes counted once.
 * Intended for benchmarks: the events add a little host overhead per launch. */
smg_status smg_profile(smg_ctx *ctx, int enable);
smg_status smg_profile_report(smg_ctx *ctx, char *buf, int64_t cap, int64_t *len);

/* Message of the last failed call on this thread ("" if none). */
const char *smg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SMG_H */
