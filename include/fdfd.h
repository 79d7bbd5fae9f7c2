/*
 * fdfd.h -- C ABI of the MI355X sparse direct solver for repeated 2D FDFD
 * solves with a cached factorisation.
 *
 * The operations follow the problem statement of the paper (Sec. II):
 *   - solve the discretised Maxwell system A(eps) x = b            (Eq. 2)
 *   - solve the adjoint system A^T lam = (dF/dx)^T                 (Eq. 4)
 *   - form dF/deps_n = -2 Re(lam^T dA/deps_n x) = -2 w^2 Re(lam_n x_n) (Eq. 3)
 *   - cache the symbolic factorisation across iterations and wavelengths,
 *     and the numeric factorisation across the forward and adjoint solves and
 *     across right-hand sides (the three caching levels of Sec. II).
 *
 * Operator.  Grid of nx * ny cells, unknown n = i + nx*j, grid units
 * (dx = 1, c = 1, omega = 2*pi*dx/lambda), Dirichlet E = 0 outside the grid,
 * stretched-coordinate PML of npml_x / npml_y cells on each side:
 *   A = Sx_c^-1 Dxb Sx_f^-1 Dxf + Sy_c^-1 Dyb Sy_f^-1 Dyf + w^2 diag(eps_r),
 *   s(p) = 1 + i sigma(p)/w, sigma = (32/npml) d(p)^3,
 *   d(p) = max(npml - p, p - (n - npml), 0)/npml,
 * at cell centres p = i + 1/2 and faces p = i.  A is not symmetric inside the
 * PML; S*A with S = diag(sx_c[i] sy_c[j]) is complex symmetric, so the library
 * factors S*A = L D L^T (no conjugation) in nested-dissection order and uses
 *   x = (SA)^-1 (S b),   lam = S (SA)^-1 g   (A^T = (SA) S^-1).
 *
 * Memory.  Every pointer named *_dev is device memory owned by the caller and
 * must stay valid until the work enqueued on the given stream completes.
 * Complex vectors are interleaved complex128 (re, im doubles), laid out
 * [nsys][nrhs][N] with N = nx*ny in grid order.  The plan owns all other
 * device memory (analysis tables, factors of every system, workspaces).
 *
 * Streams and errors.  Calls enqueue on hip_stream (a hipStream_t; NULL is
 * the null stream) and return without synchronising, except fdfd_analyze,
 * fdfd_query and fdfd_destroy.  The enqueued work reads no per-call state from
 * the host, so a caller may record refactor / solve / adjoint calls into its
 * own HIP graph (stream capture) and replay it: each replay uses the values
 * then in the captured buffers, and the omegas given at capture (plans made
 * with FDFD_PROFILE or FDFD_TRACE excepted).  Argument and state errors are
 * returned at once and enqueue nothing.  Numeric conditions found on the device (pivot
 * perturbation, non-finite values, refinement that misses its tolerance) are
 * recorded in a device status word and reported by fdfd_query.  No C++
 * exception crosses this interface.  A plan is not thread safe.
 */
#ifndef FDFD_H_
#define FDFD_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FDFD_OK = 0,
  FDFD_ERR_ARG = 1,      /* invalid argument (null pointer, bad size)          */
  FDFD_ERR_STATE = 2,    /* call out of order, e.g. solve before refactor      */
  FDFD_ERR_NOMEM = 3,    /* device allocation failed or exceeds mem_cap_bytes  */
  FDFD_ERR_HIP = 4,      /* a HIP runtime call failed                          */
  FDFD_ERR_NUMERIC = 5,  /* non-finite values, or refinement missed its tolerance */
  FDFD_WARN_PIVOT = 6    /* >= 1 pivot was perturbed; results are refined      */
} fdfd_status;

typedef enum {
  FDFD_C128 = 0,    /* complex128 factors and solves                            */
  FDFD_C64_IR = 1   /* complex64 factors; FP64 residuals and iterative refinement */
} fdfd_prec;

/* fdfd_desc.flags */
#define FDFD_ANALYZE_HOST_ONLY 1  /* symbolic analysis only: no device memory;  */
                                  /* only fdfd_query / fdfd_get_table work     */
#define FDFD_PROFILE 2            /* bracket every kernel launch with HIP events */
                                  /* (read with fdfd_kernel_stats)             */
#define FDFD_GRAPH 4              /* record the launch chain of each refactor,  */
                                  /* solve and adjoint call in a HIP graph once */
                                  /* per argument set (pointers, sizes, omegas, */
                                  /* refinement settings) and replay it; not    */
                                  /* with FDFD_PROFILE or FDFD_TRACE            */
#define FDFD_POL_TE 8             /* the TE (Hz) operator instead of TM (Ez):   */
                                  /* the same five-point pattern (one analysis */
                                  /* serves both) with the permittivity inside */
                                  /* the derivatives, on the faces (the mean  */
                                  /* of the two cells a face separates; a grid */
                                  /* edge face takes its one cell's value):    */
                                  /* A = Sx_c^-1 Dxb (eps_x Sx_f)^-1 Dxf       */
                                  /*   + Sy_c^-1 Dyb (eps_y Sy_f)^-1 Dyf       */
                                  /*   + omega^2 I.  The gradient of           */
                                  /* fdfd_adjoint_grad then collects each      */
                                  /* cell's share of its four faces' terms     */
                                  /* -2 Re(lam^T dA/deps_f x) (the curl-curl   */
                                  /* operator of Eq. (1) written for H; the    */
                                  /* paper states E only)                      */

typedef struct {
  int32_t nx, ny;          /* grid cells, nx, ny >= 2                           */
  int32_t npml_x, npml_y;  /* PML cells per side, 2*npml < n                    */
  int32_t nsys;            /* same-pattern systems factored together (>= 1)    */
  int32_t max_rhs;         /* largest nrhs passed to the solves (>= 1)         */
  int32_t prec;            /* fdfd_prec                                         */
  int32_t device;          /* HIP device ordinal, -1 = current device          */
  int32_t leaf;            /* cells per undivided dissection leaf, 0 = default */
  int32_t flags;           /* FDFD_ANALYZE_HOST_ONLY | FDFD_PROFILE | FDFD_GRAPH */
                           /* | FDFD_POL_TE                                     */
  int32_t small_lds;       /* LDS bytes a front may use in the one-workgroup-  */
                           /* per-front kernel (the bottom levels whose fronts */
                           /* all fit run there, the rest as 64 x 64 tile     */
                           /* tasks); 0 = default (64 KiB), -1 = tiles only   */
  int32_t reserved;        /* must be 0                                         */
  int64_t mem_cap_bytes;   /* refuse plans needing more device memory, 0 = off  */
  /* Schedule knobs (layout of the work only, never the solution; 0 = the   */
  /* default, or the environment variable of the same name if it is set):   */
  int32_t syrk_group;      /* pivot blocks one Schur-tile task accumulates     */
                           /* before it writes the tile (default 8; -1 = all) */
  int32_t split_kb;        /* L21 size (KiB) from which the sweeps take a      */
                           /* front's update rows as 64-row chunk items       */
                           /* (default 128; -1 = never)                       */
  int32_t block_split;     /* pivot blocks from which the sweeps take a front's */
                           /* pivot part one 64-row block per item (default 6; */
                           /* -1 = never)                                      */
  int32_t reserved2;       /* must be 0                                         */
} fdfd_desc;

typedef struct fdfd_plan_s* fdfd_plan;

/* Per-plan figures.  Counts are per system unless said otherwise. */
typedef struct {
  int64_t n;                 /* unknowns                                          */
  int64_t nfronts;           /* fronts in the separator tree                      */
  int64_t nlevels;           /* tree height (levels of the level schedule)        */
  int64_t nnz_factor;        /* lower-triangular entries of L (incl. D)           */
  int64_t factor_bytes;      /* bytes of one system's factor panels               */
  int64_t update_bytes;      /* bytes of one system's update blocks               */
  int64_t device_bytes;      /* all device memory held by the plan                */
  double refactor_flops;     /* real flops of one numeric factorisation           */
  double schur_flops;        /* of which in the Schur-complement updates          */
  int32_t max_front, max_pivots;
  int32_t leaf;
  int32_t n_perturbed;       /* pivots perturbed by the last refactor, all systems */
  double min_pivot_ratio;    /* min |d_k| / ||SA||_max over the last refactor      */
  int32_t ir_steps_solve;    /* refinement steps taken by the last fdfd_solve      */
  int32_t ir_steps_adjoint;  /* ... by the last fdfd_adjoint_grad                  */
  double rel_residual_solve;   /* max over columns of ||Sb - SAx|| / ||Sb||        */
  double rel_residual_adjoint; /* max over columns of ||g - SA lam'|| / ||g||      */
  int32_t device_flags;      /* raw device status bits                            */
  int32_t small_levels;      /* bottom tree levels run one workgroup per front    */
  double refactor_ms;        /* device time of the last fdfd_refactor (HIP events */
  double solve_ms;           /* around its launches), of the last fdfd_solve and  */
  double adjoint_ms;         /* of the last fdfd_adjoint_grad; -1 if none yet     */
  int32_t rhs_group;         /* right-hand sides per sweep pass at max_rhs: the   */
                             /* sweeps hold a front's right-hand-side block in   */
                             /* LDS, so more columns take more passes            */
  int32_t syrk_group;        /* the schedule knobs in effect (fdfd_desc; -1:     */
  int32_t split_kb;          /* all blocks / never)                              */
  int32_t block_split;
  int32_t small_lds;         /* the one-workgroup kernel's LDS budget in effect  */
  int32_t reserved3;         /* 0                                                 */
  double analyze_ms;         /* host time of fdfd_analyze's symbolic analysis    */
                             /* (the nested-dissection ordering and the fronts)  */
  double setup_ms;           /* host time of the rest of fdfd_analyze: schedule, */
                             /* device arena allocation and table uploads        */
} fdfd_info;

/*
 * Symbolic analysis, once per grid (the cached symbolic factorisation of
 * Sec. II): nested dissection, separator tree, front layout, index maps and
 * level schedule, then device allocation of every arena.  Host work plus one
 * upload.  *out receives a new plan on success and NULL otherwise.
 * Read here from the environment, for measurement only (all optional):
 *   FDFD_SMALL_LDS  LDS budget (bytes) of the one-workgroup front kernel when
 *                   desc->small_lds is 0;
 *   FDFD_SPLIT_KB   desc->split_kb when that is 0;
 *   FDFD_BLOCK_SPLIT, FDFD_SYRK_GROUP  the schedule knobs of fdfd_desc of
 *                   the same name when the desc leaves them at 0 (for
 *                   FDFD_BLOCK_SPLIT and FDFD_SYRK_GROUP, 0 means never /
 *                   all blocks);
 *   FDFD_WAVE_FRONTS at most this many bottom levels factored one wavefront
 *                   per front (each level's fronts must have at most 64 rows
 *                   and 40 pivots, or 128 rows and 16 pivots; 0 = none,
 *                   default all that qualify);
 *   FDFD_WAVE_MIN_FRONTS fronts a level of up to 128 rows needs for that
 *                   (default 16 per CU; per system, so a batch of systems
 *                   is factored exactly as each system alone);
 *   FDFD_SWEEP_RHS  at most this many right-hand sides per sweep pass (the
 *                   passes also never take more than fit the LDS);
 *   FDFD_SWEEP_GROUP height of the bottom-level subtrees one wavefront
 *                   sweeps whole, children before parents (default: the
 *                   highest level up to 3 with 16 fronts per CU; 0 = one
 *                   front at a time);
 *   FDFD_PIVOT_TAU  static pivot threshold relative to the matrix norm;
 *   FDFD_TRACE      file for per-task timestamps (written by fdfd_query).
 * max_rhs is not limited by the front sizes: the sweeps hold a front's
 * right-hand-side block in LDS and take the columns in as many passes as
 * needed (fdfd_info.rhs_group per pass); a front whose single column does not
 * fit is refused with FDFD_ERR_ARG, and so is a front of m rows with
 * m * m * (bytes per complex entry) >= 2 GiB (m > 11585 in complex128, about
 * a 7700 x 7700 grid).
 */
fdfd_status fdfd_analyze(const fdfd_desc* desc, fdfd_plan* out);

/*
 * Numeric factorisation of S*A(eps, w_s) for every system s (Sec. II,
 * numerical factorisation).  eps_dev: float64 [ny][nx] per system, system s at
 * eps_dev + s*eps_sys_stride (stride 0 = one map shared by all systems).
 * omega_host: nsys host doubles, w = 2*pi*dx/lambda.  The factor stays valid
 * for every later solve until the next refactor (Sec. II, caching 1 and 3).
 */
fdfd_status fdfd_refactor(fdfd_plan plan, const double* eps_dev, int64_t eps_sys_stride,
                          const double* omega_host, void* hip_stream);

/*
 * Forward solve A x = b for nrhs right-hand sides per system (Eq. 2 and
 * Eq. 5) with the cached factor.  b_dev, x_dev: complex128 [nsys][nrhs][N].
 * In FDFD_C128 mode max_ir may be 0.  Each refinement step computes the
 * residual S b - S A x in FP64, solves for a correction with the factor and
 * adds it in FP64; refinement stops once every column satisfies
 * ||Sb - SAx|| <= ir_tol ||Sb|| (ir_tol <= 0: 1e-12), after at most max_ir
 * steps.  1 <= nrhs <= max_rhs.
 */
fdfd_status fdfd_solve(fdfd_plan plan, const void* b_dev, void* x_dev, int32_t nrhs,
                       int32_t max_ir, double ir_tol, void* hip_stream);

/*
 * For callers that cannot allocate device memory during the solve (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): fdfd_solve with the same arguments, results and errors, whose
 * work vectors (elimination-order and update vectors, split-front hand-over
 * buffers, FP64 residual and partial norms) live in one
 * file-scope device array of FDFD_NOALLOC_SCRATCH_BYTES (64 MiB) instead of
 * the plan's arenas.  It calls no hipMalloc, hipFree or other allocating
 * routine (the plan, made earlier by fdfd_analyze, is an input); nothing in
 * the array has to start at zero (each launch writes what it reads).  Every call on a GPU
 * shares that GPU's array, which keeps the last call's contents: calls that
 * overlap on one GPU (other streams, other plans, other threads) race, and the
 * caller must serialise them.  Returns FDFD_ERR_ARG, enqueuing nothing, when
 * nsys x nrhs columns of this plan need more than the array holds (about
 * 64 bytes per cell and column in complex128, plus the update vectors: one
 * column of a 500 x 500 grid fits, 2000 x 2000 does not), and FDFD_ERR_STATE
 * for plans made with FDFD_PROFILE.
 */
#define FDFD_NOALLOC_SCRATCH_BYTES (64ll << 20)
fdfd_status fdfd_solve_noalloc(fdfd_plan plan, const void* b_dev, void* x_dev, int32_t nrhs,
                               int32_t max_ir, double ir_tol, void* hip_stream);

/*
 * Adjoint solve A^T lam = g (Eq. 4 and Eq. 6) with the same cached factor
 * (S A is symmetric, so lam = S (SA)^-1 g needs no second factorisation),
 * then the gradient of Eq. (3): grad_n = -2 w_s^2 Re(lam_n x_n), summed over
 * the nrhs right-hand sides.
 *   x_dev       complex128 [nsys][nrhs][N]   forward fields from fdfd_solve
 *   g_dev       complex128 [nsys][nrhs][N]   (dF/dx)^T per column
 *   lambda_dev  complex128 [nsys][nrhs][N]   adjoint fields, may be NULL
 *   grad_dev    float64 [nsys][N], or [N] with FDFD_GRAD_SUM_SYSTEMS
 * FDFD_GRAD_ACCUMULATE adds to grad_dev instead of overwriting it.
 * Refinement as in fdfd_solve.
 */
#define FDFD_GRAD_ACCUMULATE 1
#define FDFD_GRAD_SUM_SYSTEMS 2
fdfd_status fdfd_adjoint_grad(fdfd_plan plan, const void* x_dev, const void* g_dev,
                              int32_t nrhs, int32_t max_ir, double ir_tol,
                              void* lambda_dev, double* grad_dev, int32_t flags,
                              void* hip_stream);

/*
 * Synchronises the plan's last stream, then fills *info.  Returns
 * FDFD_ERR_NUMERIC if the device recorded non-finite values or a refinement
 * that missed its tolerance, FDFD_WARN_PIVOT if pivots were perturbed, else
 * FDFD_OK.
 */
fdfd_status fdfd_query(fdfd_plan plan, fdfd_info* info);

/*
 * Host copies of the analysis tables, for inspection and tests:
 *   FDFD_TABLE_PERM    int32 [N]        elimination position -> grid index
 *   FDFD_TABLE_FRONTS  int32 [nfronts][4] (first position, pivots, update rows, parent)
 *   FDFD_TABLE_UPDATE  int32 [sum of update rows] update rows (positions), front by front
 *   FDFD_TABLE_TASKS   int32 [ntasks][5] the tile task graph of one system, in
 *                      claim order: (type, front, k, I, J) with type 0 assembly,
 *                      1 pivot-block LDL^T, 2 panel solve, 3 update of a pivot-
 *                      column tile by block k, 4 inverse completion, 5 fused
 *                      chain step, 6 Schur-complement tile over the blocks
 *                      [k & 0xffff, k >> 16); preceded by one int32 holding
 *                      ntasks (so the table has 1 + 5 ntasks entries)
 *   FDFD_TABLE_SWEEP_ITEMS int32 the bottom levels' sweep items: nitems, the
 *                      subtree height H, then nitems + 1 offsets into the
 *                      fronts list that follows (each item's fronts,
 *                      children before parents)
 * count is the capacity of out in int32 elements.  Returns FDFD_ERR_ARG if it
 * is too small.  Works for host-only plans.
 */
#define FDFD_TABLE_PERM 0
#define FDFD_TABLE_FRONTS 1
#define FDFD_TABLE_UPDATE 2
#define FDFD_TABLE_TASKS 3
#define FDFD_TABLE_SWEEP_ITEMS 4
fdfd_status fdfd_get_table(fdfd_plan plan, int32_t which, int32_t* out, int64_t count);

/*
 * Per-kernel measurement (not part of the method; a measurement aid).  For a
 * plan analysed with FDFD_PROFILE, every kernel launch is bracketed by a pair
 * of HIP events on its stream and tagged with the algorithmic work it
 * performs: factor and vector bytes that must move for the sweeps and the
 * residual, real flops of the partial LDL^T for the factorisation kernels.
 * fdfd_kernel_stats synchronises the plan's stream, fills up to max_entries
 * records (one per kernel, in a fixed order), stores the count in *n_out, and
 * resets the totals.  Returns FDFD_ERR_STATE for a plan without FDFD_PROFILE.
 */
typedef struct {
  char name[32];        /* kernel name, e.g. "fwd_sweep"                      */
  int64_t launches;     /* launches since the previous call                   */
  double total_ms;      /* summed event time of those launches                */
  double alg_bytes;     /* summed algorithmic bytes (0 if flop-bound)         */
  double alg_flops;     /* summed algorithmic real flops (0 if byte-bound)    */
} fdfd_kernel_stat;
fdfd_status fdfd_kernel_stats(fdfd_plan plan, fdfd_kernel_stat* out, int32_t max_entries,
                              int32_t* n_out);

/*
 * Design parametrisation (Sec. III, Sec. IV): the map from the optimiser's
 * variables theta in [0, 1], one per design pixel, to the permittivity of the
 * design block, and its backward pass.  Stateless; the work runs on the
 * current HIP device, enqueued on hip_stream.
 *   filter      rho_i = sum_j w(d_ij) theta_j / S_i,  S_i = sum_j w(d_ij),
 *               with the conic weights w(d) = max(0, 1 - d / radius) of the
 *               distance d (cells) between pixel centres, over the block only
 *               (the paper's smoothing filter of 200 nm radius is radius =
 *               200 nm / dx cells);
 *   projection  P(x) = (tanh(beta eta) + tanh(beta (x - eta)))
 *                    / (tanh(beta eta) + tanh(beta (1 - eta)))
 *               (the paper's sigmoid-like projection towards two materials);
 *   material    eps = eps_min + P(rho) (eps_max - eps_min).
 * Layouts: theta, rho, work and dF/dtheta are float64 [h][w] device arrays;
 * eps and dF/deps are float64 [ny][nx] maps with the block at (i0, j0)
 * (nx = w, ny = h, i0 = j0 = 0 for a compact block).  Caller-owned.
 * Errors: FDFD_ERR_ARG (enqueues nothing; text from fdfd_param_last_error),
 * FDFD_ERR_HIP on a launch failure.
 */
typedef struct {
  int32_t w, h;          /* design block, cells along x and y (>= 1)           */
  int32_t i0, j0;        /* its corner in the eps map                          */
  int32_t nx, ny;        /* the eps map                                         */
  double radius;         /* filter radius in cells, (0, 12]                     */
  double beta, eta;      /* projection steepness (> 0) and threshold (0 < eta < 1) */
  double eps_min, eps_max;
} fdfd_param_desc;

/* Forward: rho_dev <- filtered theta (kept for the backward pass); the block
 * of eps_dev <- eps_min + P(rho) (eps_max - eps_min); the rest of eps_dev is
 * not touched. */
fdfd_status fdfd_param_forward(const fdfd_param_desc* desc, const double* theta_dev, double* rho_dev,
                               double* eps_dev, void* hip_stream);

/* Backward: grad_theta_dev <- dF/dtheta from dF/deps (the block of
 * grad_eps_dev is read) and rho from the forward pass.  work_dev: h * w
 * doubles of scratch. */
fdfd_status fdfd_param_backward(const fdfd_param_desc* desc, const double* rho_dev, const double* grad_eps_dev,
                                double* work_dev, double* grad_theta_dev, void* hip_stream);

/* Text of the calling thread's last fdfd_param_* error. */
const char* fdfd_param_last_error(void);

/* Static text of a status code. */
const char* fdfd_status_str(fdfd_status s);

/* Text of the plan's last error (empty string if none; never NULL). */
const char* fdfd_last_error(fdfd_plan plan);

/* Frees the plan and all its device memory after synchronising its stream. */
void fdfd_destroy(fdfd_plan plan);

#ifdef __cplusplus
}
#endif

#endif /* FDFD_H_ */
