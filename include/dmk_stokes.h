/*
 * dmk_stokes.h -- C ABI of the MI355X (gfx950) DMK Stokeslet library.
 *
 * Computes the 3D Stokeslet point sums of the paper's Introduction
 * (eq. stokes_stress_sum with the Stokeslet of eq. stokeslet_def_deriv,
 * viscosity 1):
 *
 *   free space:  u_j(x_b) = sum_{a != b} S_jl(x_b - x_a) f_{a,l},
 *   periodic:    u_j(x_b) = sum_a sum_{p in Z^3}* S_jl(x_b - x_a + p) f_{a,l}
 *                on the unit cell [0,1)^3 (eq. periodic_sum), with the k = 0
 *                Fourier term dropped: zero mean flow (eq. ewald_far and the
 *                remark after it);
 *
 *   S_jl(y) = (1/8pi) (delta_jl / |y| + y_j y_l / |y|^3),
 *
 * by the dual-space multilevel kernel-splitting method with the prolate
 * (PSWF) splitting of the biharmonic kernel (Sec. "The DMK method", split of
 * eqs. biharmonicks/bsplitdef, residual kernel eq. res_stokeslet, parameters
 * of Table tab:params).  A pair of distinct but coincident points contributes
 * nothing (to within tol: its mollified part, carried by the far field, is
 * cancelled in the near field).
 *
 * Memory: every array argument of the plan/eval calls is a DEVICE pointer
 * (hipMalloc'd or a torch CUDA tensor's data pointer) owned by the caller.
 * The plan copies and reorders what it needs, so `points` may be freed once
 * dmk_stokes_plan returns.  dmk_stokes_eval only enqueues work on the plan's
 * stream and returns; `forces` and `velocities` must stay valid until the
 * stream reaches that point.  Host-only diagnostics take host pointers.
 *
 * Errors: every call returns a dmk_status; on failure no plan is created
 * (*out is set to NULL) and dmk_last_error() describes the cause in a
 * thread-local string.  Calls never throw across the ABI.
 */
#ifndef DMK_STOKES_H
#define DMK_STOKES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dmk_plan_s* dmk_plan_t;

typedef enum {
    DMK_OK = 0,
    DMK_ERR_ARG = -1,          /* null / non-device pointer, n < 1, n_rhs < 1, bad option */
    DMK_ERR_UNSUPPORTED = -2,  /* dim != 3 */
    DMK_ERR_DOMAIN = -3,       /* periodic point outside [0,1)^3 */
    DMK_ERR_NONFINITE = -4,    /* NaN or Inf among the points */
    DMK_ERR_TOL = -5,          /* tol outside [1e-12, 1e-3] (mixed precision: [1e-6, 1e-3]) */
    DMK_ERR_OOM = -6,          /* device allocation failed or exceeds opts.mem_cap_bytes */
    DMK_ERR_HIP = -7           /* a HIP runtime call failed */
} dmk_status;

/* FP64: every buffer and operation in double precision.
 * MIXED: the far-field buffers (proxy charges and potentials, plane-wave
 * expansions, stage intermediates, the points' Lagrange values) are stored as
 * float, halving their memory and traffic, and the two point <-> proxy-grid
 * contractions run on FP32 matrix cores: the proxy charges (Step 2a) with FP32
 * products summed in blocks of 64 points into FP64 sums, the far field at the
 * points with the contraction over one grid axis in FP32 and the rest in FP64.
 * The near field (whose radial polynomials are evaluated in FP64), the tree
 * geometry and the accumulation at the points stay FP64.  Relative errors
 * gain about 2e-7, so MIXED needs tol >= 1e-6. */
typedef enum { DMK_PREC_FP64 = 0, DMK_PREC_MIXED = 1 } dmk_precision;

/* Window of the kernel split (eqs. wfunchat_prol_G / wfunc_prol_G):
 * PROLATE is the PSWF window of the paper's method (Table tab:params, left
 * columns); GAUSSIAN is the classical Hasimoto window (right columns,
 * q = (6/pi) sigma^-2), offered for tol in [1e-6, 1e-3]. */
typedef enum { DMK_WINDOW_PROLATE = 0, DMK_WINDOW_GAUSSIAN = 1 } dmk_window;

/* Kernel of a plan.  STOKESLET: the sums above.  STRESSLET: the double-layer
 * sums of eq. stokes_stress_sum with the stresslet of eq. stresslet_def_deriv,
 *   u_j(x_b) = sum_{a != b} T_jlm(x_b - x_a) f_{a,l} n_{a,m},
 *   T_jlm(y) = -(3/4pi) y_j y_l y_m / |y|^5,
 * split by the same PSWF mollifier (residual eq. res_stresslet with the
 * functions of eq. T-offd; Fourier side eq. moll_stresslet) with the stresslet
 * columns of Table tab:params (p stepped up one compiled order per row: 12,
 * 23, 36, 48).  Offered with the prolate window, in free space and on the
 * periodic unit cell; there the k = 0 Fourier term is the one the paper fixes
 * for the stresslet (after eq. ewald_far),
 *   u^(0)(x_b) = -sum_a (x_b - x_a)(f_a . n_a),
 * with positions in [0,1)^3 as given (so the sum depends on which image of a
 * point is passed, by -p (f.n) for a shift p).  Evaluated with
 * dmk_stokes_eval_stresslet. */
typedef enum { DMK_KERNEL_STOKESLET = 0, DMK_KERNEL_STRESSLET = 1 } dmk_kernel;

/* Method of a plan.  DMK: the multilevel method above.  EWALD: the
 * single-level spectral Ewald sum with the same prolate split, for the
 * periodic cell (the uniform-data variant the paper's introduction points to,
 * Sec. "Ewald summation"): with r_c = 2^-L, L the smallest level whose cells
 * hold at most leaf_size points on average,
 *   u = sum over neighbouring cells of the residual Stokeslet at scale r_c
 *     + sum_{0 < |kappa_i| <= K} (I - k k^T/k^2) gammahat(k r_c)/k^2 F(k) e^{i k.x},
 *   k = 2 pi kappa, |k_i| < c / r_c,
 * the Fourier sum by spreading to an oversampled M^3 grid with a prolate
 * gridding kernel, a 3D FFT, scaling, an inverse FFT and interpolation.
 * Offered for one periodic problem (no batch, no separate targets), the
 * Stokeslet, the prolate window, FP64, tol in [1e-9, 1e-3]. */
typedef enum { DMK_METHOD_DMK = 0, DMK_METHOD_EWALD = 1 } dmk_method;

typedef struct {
    int precision;        /* dmk_precision */
    int leaf_size;        /* maximum points per leaf; 0 = the tolerance's default */
    void* stream;         /* hipStream_t for all work of the plan; NULL = null stream */
    size_t mem_cap_bytes; /* refuse plans whose device buffers exceed this; 0 = no cap */
    int flags;            /* DMK_FLAG_* bits */
    int near_lanes;       /* near field: source lanes per target (1, 2, 4 or 8; a wave
                             then holds 64, 32, 16 or 8 targets); 0 = automatic */
    int q;                /* window parameter q = 3c/pi (sets c and the plane-wave
                             counts n1 = 2q-1, nper = 2 ceil(q/6) - 1); 0 = the
                             Table tab:params row chosen by tol, else in [4, 40] */
    int p;                /* Chebyshev points per dimension of every proxy grid;
                             0 = the row's value, else 11, 12, 14, 16, 20, 22, 23,
                             26, 28, 30, 33, 36, 40, 43, 44 or 48 */
    int rhs_batch;        /* force vectors evaluated together by one near-field pass
                             (the pair geometry and radial polynomials are shared):
                             1, 2, 4 or 8; 0 = 8.  Sets the size of the plan's
                             force/velocity work buffers (48 bytes per point each) */
    int window;           /* dmk_window (0 = prolate) */
    int kernel;           /* dmk_kernel (0 = Stokeslet) */
    int method;           /* dmk_method (0 = DMK) */
    int stage_rows;       /* rows per workgroup of the separable proxy / plane-wave stages:
                             16, 32 or 64; 0 = chosen per stage by its LDS footprint
                             (a value a stage cannot take falls back to that choice) */
    int eval_points;      /* points per workgroup of the far-field evaluation at the
                             points: 128 or 256 (256 only for p <= 16, 23, 30, else
                             128); 0 = 128 */
} dmk_opts;

/* record HIP events around each phase of dmk_stokes_eval (read back with
 * dmk_stokes_phase_ms) */
#define DMK_FLAG_PHASE_TIMING 1
/* the points are complete when the plan call is made (no writes to them are
 * pending on any stream): the plan is built on the library's own
 * non-blocking stream, so its device work and host tree construction overlap
 * work already queued on opts.stream (e.g. the previous plan's evaluation).
 * Without the flag the plan is built in order on opts.stream. */
#define DMK_FLAG_CONCURRENT_PLAN 2
/* dmk_stokes_eval captures its launches into a HIP graph the first time it
 * sees a (forces, n_rhs, velocities) triple and replays that graph, on
 * opts.stream, for later calls with the same triple (new force values in the
 * same buffer are picked up).  Phase timing is not recorded in this mode. */
#define DMK_FLAG_GRAPH 4
/* keep the points of every leaf in Morton order.  By default a plan reorders
 * them, inside each leaf (sources and targets separately), by recursive
 * balanced bisection across the longest side of the bounding box, so that the
 * runs of 8 to 64 points that the near field takes as target groups and source
 * chunks are compact and its per-group pruning discards more out-of-support
 * pairs (Step 4 evaluates the residual only within r_lambda).  The sums are
 * the same up to rounding either way. */
#define DMK_FLAG_MORTON_ORDER 8
/* build the octree, its level restriction and the neighbour lists on the host
 * (sequential construction, from the same device-sorted keys) instead of on
 * the device.  Both constructions give the same tree and lists; the flag is a
 * reference for checks. */
#define DMK_FLAG_HOST_TREE 16

/* phases reported by dmk_stokes_phase_ms (an evaluation runs the near field
 * first, then the far-field phases in index order, then the finish) */
#define DMK_PHASE_ANTERP 0     /* leaf proxy charges (Step 2a) */
#define DMK_PHASE_MERGE 1      /* upward merge (Step 2b) */
#define DMK_PHASE_OUTGOING 2   /* outgoing plane waves */
#define DMK_PHASE_TRANSLATE 3  /* colleague translation + difference symbol (Step 3b) */
#define DMK_PHASE_INCOMING 4   /* incoming plane waves -> proxy potentials */
#define DMK_PHASE_ROOT 5       /* root convolution (Step 3a) */
#define DMK_PHASE_INTERP 6     /* downward interpolation */
#define DMK_PHASE_LEAF_EVAL 7  /* far field at the points */
#define DMK_PHASE_NEAR 8       /* force gather + residual pair sums + self term (Step 4) */
#define DMK_PHASE_FINALIZE 9   /* constant, scaling, unpermute */
#define DMK_NUM_PHASES 10

typedef struct {
    /* parameters (Table tab:params, Stokeslet; q, c = K_max = q pi/3) */
    double tol, c;
    int q, p, n1, nper, leaf_size;
    int deg_P, deg_Q;           /* degrees of the near-field radial polynomials */
    /* tree */
    int levels;                 /* deepest level + 1 */
    int periodic;
    int64_t n_points, n_boxes, n_leaves, n_nonempty_boxes, n_nonempty_leaves;
    int64_t near_pairs;         /* sum over near-list entries of |target leaf| * |source leaf| */
    int64_t n_senders, n_receivers;
    double center[3], box_len;  /* unit box <-> input coordinates */
    size_t device_bytes;
    double plan_ms;             /* wall time of the plan call */
    /* wall time of the plan's parts: bounding box, Morton keys + sort + key
     * download, host octree, host lists, device buffers, uploads + final sync */
    double plan_phase_ms[6];
    int near_lanes;             /* source lanes per target of the near-field kernel */
    int precision;              /* dmk_precision of the plan */
    int window;                 /* dmk_window of the plan */
    double sigma;               /* Gaussian shape parameter (0 for the prolate window) */
    int kernel;                 /* dmk_kernel of the plan */
    int method;                 /* dmk_method of the plan */
    /* spectral Ewald plans: grid points per dimension M, mode bound K
     * (|kappa_i| <= K), gridding kernel width in grid points; levels = L + 1 */
    int ewald_grid, ewald_modes, ewald_width;
    /* 1 when no two distinct points coincide (found at plan time): the near
     * field then skips pairs at r = 0 and adds the self term per target */
    int no_coincident;
} dmk_plan_info;

/*
 * Builds a plan: parameters and tables for `tol`, the level-restricted
 * adaptive octree of the points, neighbour lists and device buffers.
 *   points    device, (n,3) row-major float64.  Free space: any finite
 *             coordinates (mapped to the unit box by their bounding cube).
 *             Periodic: inside the unit cell [0,1)^3.
 *   n         number of points (sources = targets), >= 1
 *   dim       must be 3
 *   periodic  0 = free space, 1 = periodic unit cell
 *   tol       requested relative l2 accuracy, in [1e-12, 1e-3]; the plan uses
 *             the Table tab:params row with the largest tolerance <= tol
 *   out       receives the plan (NULL on failure)
 * Synchronises the stream once (tree sizes are needed on the host).
 */
int dmk_stokes_plan(const double* points, int64_t n, int dim, int periodic, double tol, dmk_plan_t* out);

/* As dmk_stokes_plan with options (opts may be NULL = defaults). */
int dmk_stokes_plan_ex(const double* points, int64_t n, int dim, int periodic, double tol, const dmk_opts* opts,
                       dmk_plan_t* out);

/*
 * Builds a plan for a target set separate from the sources:
 *   u(t) = sum_s S(t - x_s) f_s   (a target coinciding with a source: that pair contributes nothing)
 *   sources   device, (n_sources,3) row-major float64
 *   targets   device, (n_targets,3) row-major float64
 * One octree covers both sets (split while a box holds more than leaf_size
 * points, sources and targets together); within each leaf the sources come first, so proxy
 * charges and the near field's source side run over sources only and the far
 * field is evaluated at targets only.  dmk_stokes_eval then takes forces
 * (n_rhs, n_sources, 3) and writes velocities (n_rhs, n_targets, 3).  Built in
 * order on opts.stream (DMK_FLAG_CONCURRENT_PLAN is refused); allocates and
 * frees a temporary device copy of both point sets.  Other arguments as
 * dmk_stokes_plan_ex; plan_info counts n_points = n_sources + n_targets.
 */
int dmk_stokes_plan_targets(const double* sources, int64_t n_sources, const double* targets, int64_t n_targets,
                            int dim, int periodic, double tol, const dmk_opts* opts, dmk_plan_t* out);

/*
 * Builds one plan over n_problems independent problems (each its own free-space
 * sum, or its own periodic unit cell), evaluated together: every pass of
 * dmk_stokes_eval covers all problems in one launch per stage.
 *   points      device, (n,3) row-major float64, the problems concatenated:
 *               problem b is points[offsets[b] .. offsets[b+1])
 *   offsets     HOST array of n_problems + 1 int64: offsets[0] = 0, strictly
 *               increasing (every problem has at least one point), n = offsets[n_problems]
 *   n_problems  in [1, 2^20]
 * Each problem gets its own bounding cube and octree (a forest); points of
 * different problems never interact.  forces / velocities of dmk_stokes_eval
 * follow the same concatenated order.  Other arguments as dmk_stokes_plan_ex;
 * plan_info reports the forest (center/box_len: problem 0).
 */
int dmk_stokes_plan_batch(const double* points, const int64_t* offsets, int n_problems, int dim, int periodic,
                          double tol, const dmk_opts* opts, dmk_plan_t* out);

/*
 * Evaluates the sums for n_rhs force vectors on the plan's points.
 *   forces      device, (n_rhs, n, 3) float64, caller's point order (n_sources
 *               rows per vector for a plan with separate targets)
 *   velocities  device, (n_rhs, n, 3) float64, overwritten (n_targets rows per
 *               vector for a plan with separate targets)
 * The vectors are taken in batches of up to dmk_opts.rhs_batch: the far-field
 * passes run per vector, the near field once per batch.  Stream-ordered, no
 * host synchronisation; several calls on one plan must not overlap (they share
 * the plan's work buffers).
 */
int dmk_stokes_eval(dmk_plan_t plan, const double* forces, int n_rhs, double* velocities);

/*
 * Evaluates the stresslet sums (dmk_kernel STRESSLET) for n_rhs pairs of
 * vectors on a plan built with dmk_opts.kernel = DMK_KERNEL_STRESSLET:
 *   u_j(x_b) = sum_{a != b} T_jlm(x_b - x_a) f_{a,l} n_{a,m}
 *   forces, normals  device, (n_rhs, n_sources, 3) float64 each, caller's order
 *                    (n_sources = n for a plan without separate targets)
 *   velocities       device, (n_rhs, n_targets, 3) float64, overwritten
 * The far field carries the 6 components of the symmetric part of f n^T
 * through the proxy and plane-wave passes; the difference-kernel symbol of eq.
 * moll_stresslet contracts them to 3 velocity components before the
 * translation.  Vectors run one after the other.  A pair of distinct but
 * coincident points contributes nothing; there is no self term.  Returns
 * DMK_ERR_ARG for a Stokeslet plan.  Stream-ordered, like dmk_stokes_eval.
 */
int dmk_stokes_eval_stresslet(dmk_plan_t plan, const double* forces, const double* normals, int n_rhs,
                              double* velocities);

/*
 * Autotuner: picks the leaf size (maximum points per leaf), the near-field
 * lane split and the tile shapes of the far-field kernels (stage_rows,
 * eval_points) for this workload by timing plan + evaluation on the caller's
 * points.  Leaf sizes 0.5, 0.75, 1, 1.35, 1.8 and 2.4 times the starting size
 * (opts->leaf_size, else the tolerance's default) are tried with the starting
 * lane split, then 2 and 8 lanes at the best size, then stage rows 16, 32 and
 * 64 and 128 / 256 evaluation points at the best size and split; each trial
 * keeps the fastest of three runs.  The choice is cached per process for the workload class
 * (n and n_problems to the nearest power of two, periodicity, tol, precision,
 * n_rhs, q, p): a later call for the same class returns at once.
 *   points, n                as dmk_stokes_plan_ex (device points)
 *   offsets, n_problems      as dmk_stokes_plan_batch, or offsets = NULL for one problem
 *   opts                     starting options (may be NULL); copied into *tuned
 *   n_rhs                    force vectors per evaluation to tune for (1..64)
 *   tuned                    receives opts with leaf_size, near_lanes, stage_rows and
 *                            eval_points set
 *   best_ms                  receives the best trial's plan + eval milliseconds (may be NULL)
 * Allocates and frees two (n_rhs, n, 3) device buffers; synchronises opts->stream.
 */
int dmk_stokes_autotune(const double* points, int64_t n, const int64_t* offsets, int n_problems, int dim,
                        int periodic, double tol, const dmk_opts* opts, int n_rhs, dmk_opts* tuned, double* best_ms);

/* Fills *info (host struct) with the plan's parameters and statistics. */
int dmk_stokes_plan_info(dmk_plan_t plan, dmk_plan_info* info);

/*
 * Tree export for checks (host arrays, each sized by dmk_plan_info):
 *   leaf_level[L], leaf_coord[3L] (integer box coordinates at that level),
 *   leaf_count[L] for all L = n_leaves leaves (empty ones included), and
 *   point_leaf[n]: index of the leaf holding each point (caller's order).
 * Any pointer may be NULL to skip that array.  Synchronises the stream.
 */
int dmk_stokes_tree_leaves(dmk_plan_t plan, int32_t* leaf_level, int64_t* leaf_coord, int64_t* leaf_count,
                           int64_t* point_leaf);

/*
 * Milliseconds spent in each phase of the most recent dmk_stokes_eval call on
 * this plan, out[DMK_NUM_PHASES] host array: the far-field phases of its first
 * force vector, the near field and finish of its first batch of vectors
 * (dmk_opts.rhs_batch).  Needs DMK_FLAG_PHASE_TIMING; synchronises on the
 * recorded events.
 */
int dmk_stokes_phase_ms(dmk_plan_t plan, double* out);

/*
 * Near-field pair statistics of the plan (host int64 outputs, NULL to skip):
 *   listed     sum over near-list entries of |target leaf| * |source leaf|
 *   evaluated  (target, source) pairs the near-field kernel evaluates: for each
 *              wave's target group, the sources lying within r_lambda of the
 *              group's bounding box (64-point source chunks are first pruned
 *              by their own boxes)
 *   in_support pairs with 0 < |x_t - x_s + shift| < r_lambda (the residual's
 *              support, Corollary eq. reskernelproperty)
 * Runs a counting kernel; synchronises the stream.
 */
int dmk_stokes_near_stats(dmk_plan_t plan, int64_t* listed, int64_t* evaluated, int64_t* in_support);

/* Releases the plan (NULL-safe).  Waits for the plan's most recent
 * evaluation to finish; its device buffers then return to the library's
 * per-process cache and are reused by later plans of similar size. */
void dmk_stokes_destroy(dmk_plan_t plan);

/* Frees the cached device buffers of destroyed plans (hipFree) and the
 * cached FFT plans of destroyed spectral Ewald plans. */
void dmk_stokes_release_cached_memory(void);

/* Thread-local description of the last failure of this thread. */
const char* dmk_last_error(void);

/* ---- host-only diagnostics (no GPU needed; host pointers) ------------------ */

/* Parameters the plan would use for tol (other fields zero). */
int dmk_stokes_params(double tol, dmk_plan_info* info);
/* The same for a given window (dmk_window). */
int dmk_stokes_params_ex(double tol, int window, dmk_plan_info* info);
/* The same for a given window and kernel (dmk_kernel); for the stresslet,
 * deg_P and deg_Q are the degrees of its radial functions A and D. */
int dmk_stokes_params_kernel(double tol, int window, int kernel, dmk_plan_info* info);

/*
 * Window and near-field radial functions at unit scale for tol, at n radii:
 *   out[4i+0] = phi(rho)            (eq. wfunc_prol_G)
 *   out[4i+1] = Phi(rho)            (eq. def_erfc_like_fcn)
 *   out[4i+2] = P(rho^2), out[4i+3] = Q(rho^2), the polynomial fits with
 *     S_R(y) = S(y) - [P(s) I + Q(s) y y^T]/(4 pi),  s = |y|^2 < 1
 *     (eq. res_stokeslet/Soffdiag rearranged).
 */
int dmk_stokes_radial(double tol, const double* rho, int64_t n, double* out);

/* Grid of a spectral Ewald plan (DMK_METHOD_EWALD) for n periodic points:
 * fills method, levels (split level + 1), ewald_grid (M), ewald_modes (K),
 * ewald_width (w), q, c and leaf_size (0 = the tolerance's default). */
int dmk_stokes_ewald_params(double tol, int64_t n, int leaf_size, dmk_plan_info* info);

/*
 * Near-field radial functions of the residual stresslet at unit scale for tol
 * (stresslet row of Table tab:params), at n radii: out[2i] = A(rho^2),
 * out[2i+1] = D(rho^2), the polynomial fits with
 *   T_R(y) : (f n^T) = T(y) : (f n^T) + (3/2pi) A(s) (y.f)(y.n) y
 *                      + (1/4pi) D(s) [(y.n) f + (y.f) n + (f.n) y],  s = |y|^2 < 1,
 * i.e. A = (1 - R_Toffd(rho)) / (2 rho^5), D = R_Tdiag(rho) / (2 rho^3) (eq. T-offd).
 */
int dmk_stokes_radial_stresslet(double tol, const double* rho, int64_t n, double* out);

/* Window transform and biharmonic mollifier (eq. gammaB_in_phi) at n wave
 * numbers: out[2i] = phihat(k), out[2i+1] = gammahat(k). */
int dmk_stokes_mollifier(double tol, const double* k, int64_t n, double* out);

/*
 * Builds the level-restricted octree of host points on the host (same tree
 * construction as dmk_stokes_plan, keys computed on the CPU) and exports its
 * leaves like dmk_stokes_tree_leaves.  Arrays hold `cap` leaves; when the tree
 * has more, returns DMK_ERR_ARG with *n_leaves set so the caller can retry.
 *   points      host (n,3) float64; leaf_size > 0; periodic 0/1 (points in [0,1)^3)
 */
int dmk_stokes_host_tree(const double* points, int64_t n, int leaf_size, int periodic, int64_t cap,
                         int32_t* leaf_level, int64_t* leaf_coord, int64_t* leaf_count, int64_t* n_leaves,
                         int64_t* n_near_pairs);

/* ---- device stage entry point ------------------------------------------------ */

/*
 * Residual-kernel sums by brute force over all sources, at scale r_lambda:
 *   out[i] = sum_a S_R^{r_lambda}(t_i - s_a) f_a,
 * S_R as in eq. res_stokeslet evaluated at r / r_lambda (the scaling remark
 * of Sec. "The Stokes kernels"), with the same device pair routine as the
 * near field of dmk_stokes_eval.  A pair with r = 0 contributes the residual
 * without its singular part, -S_M(0) f = -(phi(0)/(2 pi r_lambda)) f (eq.
 * S_self): in the full sum this cancels the mollified part of a coincident
 * pair, and for the pair of a target with itself it is the self term.
 *   targets (m,3), sources (ns,3), forces (ns,3), out (m,3): device float64
 *   stream: hipStream_t or NULL.  Stream-ordered.
 */
int dmk_stokes_residual_sum(const double* targets, int64_t m, const double* sources, const double* forces,
                            int64_t ns, double r_lambda, double tol, void* stream, double* out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * sums as dmk_stokes_residual_sum, with the same kernel, on the same
 * arguments, bit for bit, but the SoA staging of targets, sources and forces
 * lives in a fixed device workspace of 2^21 doubles (16 MiB) that the library
 * holds on each GPU it runs on until the process ends.  No device memory is
 * allocated or freed and the call does not synchronise: it enqueues copies
 * into the workspace and the kernel on `stream` and returns.
 *   3 m + 6 ns must not exceed 2^21 (e.g. m = ns = 233016); larger sizes
 *   return DMK_ERR_ARG (dmk_stokes_residual_sum has no such limit).
 * Every call on one GPU uses that GPU's single workspace: calls that may
 * overlap on one GPU (different streams, or host threads) race and must be
 * serialised by the caller.  The workspace keeps the last call's staged
 * values; nothing in it needs to start at zero.
 */
int dmk_stokes_residual_sum_noalloc(const double* targets, int64_t m, const double* sources, const double* forces,
                                    int64_t ns, double r_lambda, double tol, void* stream, double* out);

/*
 * The same for the residual stresslet (eq. res_stresslet with eq. T-offd, at
 * scale r_lambda), with the near-field pair routine of the stresslet plans:
 *   out[i] = sum_a T_R^{r_lambda}(t_i - s_a) : (f_a n_a^T);
 * pairs with r = 0 contribute nothing.  normals (ns,3) device float64; other
 * arguments as dmk_stokes_residual_sum.
 */
int dmk_stokes_residual_sum_stresslet(const double* targets, int64_t m, const double* sources, const double* forces,
                                      const double* normals, int64_t ns, double r_lambda, double tol, void* stream,
                                      double* out);

#ifdef __cplusplus
}
#endif

#endif /* DMK_STOKES_H */
