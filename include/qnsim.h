/*
 * qnsim.h -- C ABI of the MI355X (gfx950) quasi-Newton hyperelastic step.
 *
 * The library advances a tetrahedral mesh by implicit-Euler time steps. Each
 * step minimises
 *     g(x) = 1/(2 h^2) tr((x - y)^T M (x - y)) + E(x)                 (Eq. PD)
 * with y = x_n + h v_n + h^2 M^{-1} f_ext (section 3), by a fixed number of
 * quasi-Newton iterations (section 4.1, Algorithm 1): a descent direction from
 * the L-BFGS two-loop recursion (section 4.2, Algorithm 2) whose initial
 * Hessian is the constant, prefactored matrix A = M/h^2 + L with
 * L = sum_e V_e k_e G_e^T G_e (section 3, Eqs. PDmatrixForm / PDsolution;
 * section 4.1 for k_e), and a backtracking Armijo line search (section 4.1,
 * "Line search"). Every step of the hot path runs in HIP kernels; the host
 * only orders, factors and uploads A once per mesh (qnsim_prepare).
 *
 * Conventions (all entry points):
 *  - Every function returns an int status: QNSIM_OK (0) or a negative
 *    QNSIM_E_* code. No C++ exception crosses the ABI.
 *  - On error, output buffers are left untouched and the context stays usable;
 *    qnsim_last_error() returns a message describing the last failure.
 *  - All pointers are owned by the caller. The library copies what it needs
 *    and keeps no caller pointer after a call returns.
 *  - Positions, velocities and forces are row-major n x 3 arrays of doubles in
 *    the caller's vertex numbering; tetrahedra are row-major T x 4 int32
 *    vertex indices (any orientation).
 *  - Host entry points (qnsim_step) synchronise before returning. Device entry
 *    points (qnsim_step_device) take device pointers and a hipStream_t passed
 *    as void*, are ordered after earlier work on that stream, and state when
 *    they return (steps return when they are done; probes are stream-ordered).
 *  - Calls on one context must not overlap (a context is not thread-safe);
 *    distinct contexts are independent.
 */
#ifndef QNSIM_H
#define QNSIM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------- */
#define QNSIM_OK 0
#define QNSIM_E_INVALID -1     /* null pointer, size or index out of range     */
#define QNSIM_E_NONFINITE -2   /* NaN or Inf in an input array                  */
#define QNSIM_E_DEGENERATE -3  /* rest tetrahedron with (near) zero volume      */
#define QNSIM_E_INVERTED -4    /* Neo-Hookean element with J <= 0 at input x    */
#define QNSIM_E_STIFFNESS -5   /* stiffness fit k <= 0 for a material           */
#define QNSIM_E_NOT_SPD -6     /* Cholesky factorisation of A failed            */
#define QNSIM_E_H_MISMATCH -7  /* step h differs from the h A was factored for  */
#define QNSIM_E_STATE -8       /* call out of order (e.g. step before prepare)  */
#define QNSIM_E_NOMEM -9       /* host or device allocation failed              */
#define QNSIM_E_DEVICE -10     /* HIP runtime error                             */
#define QNSIM_E_BUDGET -11     /* pool: the simulation does not fit the budget  */

/* ---- material types (section 4.1, Valanis-Landel materials; section 5) --- */
#define QNSIM_NEOHOOKEAN 0  /* mu/2 (I1-3) - mu log J + lam/2 (log J)^2          */
#define QNSIM_STVK 1        /* mu tr(E^2) + lam/2 tr(E)^2, E = (F^T F - I)/2     */
#define QNSIM_SPLINE 2      /* sum a(s_i) + lam/2 (J-1)^2, a'' piecewise linear  */
#define QNSIM_COROTATED 3   /* mu |F-R|^2 + lam/2 tr(R^T F - I)^2                */
#define QNSIM_POLYNOMIAL 4  /* sum mu (s_i - 1)^4                                */
#define QNSIM_MOONEY_RIVLIN 5 /* mu/2 (I1-3) + mu2/2 (I2-3) - (mu + 2 mu2) log J
                                 + lam/2 (log J)^2, I2 = ((tr C)^2 - tr C^2)/2,
                                 C = F^T F (compressible; mu2 = 0 is Neo-Hookean) */

/* ---- precision modes ---------------------------------------------------- */
#define QNSIM_FP64 0   /* every kernel in FP64                                   */
#define QNSIM_MIXED 1  /* FP32 element energies/stresses; FP64 solves, dot
                          products, curvature pairs and line-search sums         */

typedef struct qnsim qnsim_t; /* opaque; owns all its host and device memory */

/* Solver options. qnsim_options_default() fills the paper's settings:
 * 10 iterations per step and L-BFGS window m = 5 (section 5, Table StatAll),
 * Armijo gamma = 0.3 and backtracking factor 0.5 (section 4.1), stiffness fit
 * interval [0.5, 1.5] (section 5), at most 30 halvings per line search,
 * gravity (0, 0, -9.81) m/s^2, FP64, device 0, dense_top 6144,
 * subtree_cap 384, level_merge 1. */
typedef struct {
  int32_t iterations;   /* quasi-Newton iterations per step (>= 1)           */
  int32_t history;      /* L-BFGS window m (0..16); 0 = plain PD direction   */
  int32_t max_halvings; /* line-search trials per iteration = max_halvings+1 */
  int32_t precision;    /* QNSIM_FP64 or QNSIM_MIXED                         */
  int32_t device;       /* HIP device ordinal                                */
  int32_t dense_top;    /* largest column count of the dense top block of the
                           prefactored solve (0 = off, at most 6144); the
                           top levels of the supernode tree are merged into
                           it when a latency/bandwidth cost model favours it */
  double gamma;         /* Armijo constant in (0, 1)                         */
  double backtrack;     /* step-length factor after a failed trial, (0, 1)   */
  double fit_lo;        /* stiffness fit interval [fit_lo, fit_hi]           */
  double fit_hi;
  double gravity[3];    /* uniform body acceleration added to f_ext / m      */
  int32_t subtree_cap;  /* the lowest levels of the supernode tree whose
                           supernodes all have at most subtree_cap rows are
                           solved one subtree per workgroup (0 = off, at
                           most 384)                                        */
  int32_t level_merge;  /* 1: whole levels of the supernode tree may merge
                           into their parents when a latency/bandwidth cost
                           model favours it; 0: off                          */
  int32_t step_graph;   /* 1: the fixed kernel sequence of a step is captured
                           once in a HIP graph per set of state buffers and
                           replayed; 0: kernels launched one by one         */
  int32_t trials_per_cycle; /* line-search trials enqueued per iteration
                           (1..8; a longer line search continues in the next
                           cycle); default 2                                 */
  int32_t direction;    /* QNSIM_DIR_LBFGS (Algorithm 2) or QNSIM_DIR_CHEBYSHEV
                           (section 5, Algorithm 3: the comparison method;
                           needs history = 0)                               */
  int32_t cheb_delay;   /* Chebyshev: iterations S with omega = 1 (>= 1; 10)   */
  double cheb_rho;      /* Chebyshev: spectral-radius estimate rho in (0, 1)  */
  int32_t device_factor; /* 1: qnsim_prepare runs the ordering and symbolic
                           analysis on the host and the numeric factorisation
                           of A on the device (as qnsim_refactor); the host
                           holds no factor values (qnsim_export_factor returns
                           QNSIM_E_STATE). 0 (default): both on the host.
                           Pools use 0.                                      */
  int32_t elem_tile;    /* tets (and free vertices) per element-pass block:
                           128, 256 or 512 (0: 256). Pools pick it per group
                           with qnsim_pool_tune.                            */
} qnsim_options;

#define QNSIM_DIR_LBFGS 0
#define QNSIM_DIR_CHEBYSHEV 1  /* d = omega (x^ - x_{k-1}) + x_{k-1} - x_k, x^ = x_k - A^{-1} grad g,
                                  omega = 1 (k < S), 2/(2 - rho^2) (k = S),
                                  4/(4 - rho^2 omega_k) (k > S); an ascent
                                  direction falls back to d = -A^{-1} grad g */

/* One material. mu, lambda in Pa; density in kg/m^3. For QNSIM_SPLINE,
 * spline_d2[j] is a''(s) at the knot s_j = 0.2 + 0.4 j (j = 0..7); a'' is
 * linear between knots and constant beyond the end knots, with
 * a'(1) = a(1) = 0 (the paper's spline curves are not published; this is the
 * spline family the library implements). Ignored for other types. */
typedef struct {
  int32_t type;
  int32_t reserved;
  double mu;
  double lambda;
  double density;
  double spline_d2[8];
  /* Anisotropic fibre term (section 4, "Anisotropy") added to the base
   * material: fiber_kappa / 2 (|F d| - 1)^2 with d = fiber_dir / |fiber_dir|
   * the rest-pose fibre direction. fiber_kappa = 0: none; > 0 needs a
   * non-zero direction. It does not change the stiffness k of A. */
  double fiber_kappa;
  double fiber_dir[3];
  /* QNSIM_MOONEY_RIVLIN: shear modulus of the I2 term (>= 0, Pa); ignored
   * for other types. Its stiffness k is the Neo-Hookean rule's with shear
   * modulus mu + 2 mu2 (the stress profile of the stiffness rule is the same
   * function of the stretch). */
  double mu2;
} qnsim_material;

/* Per-step counters (filled by qnsim_step / qnsim_step_device when non-null). */
typedef struct {
  int32_t iterations_run; /* quasi-Newton iterations executed                */
  int32_t ls_trials;      /* objective evaluations in line searches          */
  int32_t ls_exhausted;   /* 1 if a line search found no acceptable step     */
  int32_t lbfgs_skipped;  /* curvature pairs rejected (rho <= 1e-10|s||t|)   */
  int32_t fallbacks;      /* x_1 := x (infeasible y) or non-descent resets   */
  int32_t reserved;
  double g_first;         /* g(x_1)                                           */
  double g_last;          /* g at the returned state                          */
  double grad_norm_first; /* |grad g(x_1)|                                    */
  double grad_norm_last;  /* |grad g(x_final)| (one extra gradient pass), or
                             NaN unless requested with qnsim_set_diagnostics  */
} qnsim_stats;

/* Factor and schedule facts, for reports and tests. */
typedef struct {
  int32_t n_free;         /* free vertices = order of A                       */
  int32_t n_supernodes;
  int32_t n_levels;       /* supernode tree height + 1                        */
  int32_t max_front;      /* largest supernode rows (columns + below-diag)    */
  int32_t dense_top_cols; /* columns of the dense top block (0 if none)      */
  int32_t subtree_levels; /* lowest levels solved one subtree per workgroup   */
  int64_t nnz_L;          /* stored factor entries (incl. explicit zeros)     */
  int64_t nnz_L_exact;    /* structural nonzeros of the Cholesky factor       */
  int64_t factor_bytes;   /* device bytes of the solve blocks                 */
  double factor_flops;    /* host factorisation flops                         */
  double prepare_seconds; /* wall time of the last qnsim_prepare              */
} qnsim_factor_info;

/* Fill *opts with the defaults listed above. */
int qnsim_options_default(qnsim_options* opts);

/* Create a context. opts may be NULL (defaults). Does not touch the GPU. */
int qnsim_create(const qnsim_options* opts, qnsim_t** out);

/* Destroy a context and free its host and device memory. NULL is a no-op. */
void qnsim_destroy(qnsim_t* ctx);

/* Rest mesh: n_verts rest positions (n x 3) and n_tets tetrahedra (T x 4).
 * Rejects indices out of range, repeated vertices in a tet, non-finite
 * coordinates and tets with |det Dm| <= 1e-12 * (longest edge)^3
 * (QNSIM_E_DEGENERATE). Invalidates a previous prepare. */
int qnsim_set_mesh(qnsim_t* ctx, int32_t n_verts, const double* rest_xyz,
                   int32_t n_tets, const int32_t* tets);

/* Pinned (Dirichlet) vertices: they keep their input positions, enter the
 * element deformation gradients, and are eliminated from A and the solver
 * vectors. n_pinned = 0 clears the set. Invalidates a previous prepare.
 * (The paper states no boundary conditions; its scenes hold vertices fixed,
 * section 5. Elimination keeps A = M/h^2 + L of section 3, Eq. PDsolution,
 * symmetric positive definite on the free vertices.) */
int qnsim_set_pinned(qnsim_t* ctx, int32_t n_pinned, const int32_t* idx);

/* Materials: n_mat entries; tet_mat[T] gives each tet's material index, or
 * NULL to use material 0 everywhere. Invalidates a previous prepare. Each
 * material is an energy density Psi(F) of the deformation gradient of a
 * tetrahedron (section 4.1: isotropic Valanis-Landel energies written in the
 * principal stretches, Neo-Hookean and StVK among them; spline-based
 * materials; section 4, "Anisotropy" for the fibre term); its stiffness k
 * for A comes from Eq. stiffness (section 4.1). */
int qnsim_set_materials(qnsim_t* ctx, int32_t n_mat, const qnsim_material* mats,
                        const int32_t* tet_mat);

/* Host precompute for time step h (section 3; section 4.1): element rest data,
 * lumped masses, per-material stiffness k by the least-squares fit of
 * Eq. stiffness over [fit_lo, fit_hi], A = M/h^2 + L on the free vertices,
 * nested-dissection ordering, supernodal Cholesky factorisation and the
 * level-scheduled solve blocks; then uploads everything to the device. */
int qnsim_prepare(qnsim_t* ctx, double h);

/* Same host precompute as qnsim_prepare without any device work; used to
 * inspect the factorisation on machines without a GPU. A later qnsim_prepare
 * with the same h reuses it. */
int qnsim_analyze(qnsim_t* ctx, double h);

/* One time step from host arrays (n x 3): x, v in; x_out, v_out out (may alias
 * x and v). The step minimises g of Eq. PD (section 3) with
 * y = x + h v + h^2 M^{-1} f_ext by Algorithm 1 (section 4.1) with the
 * direction of Algorithm 2 (section 4.2), and returns x' = x_{K+1},
 * v' = (x' - x)/h. f_ext may be NULL (gravity only). h must equal the
 * prepared h.
 * Returns QNSIM_E_INVERTED if a Neo-Hookean element has J <= 0 at x.
 * Synchronises. stats may be NULL. */
int qnsim_step(qnsim_t* ctx, const double* x, const double* v, double h,
               const double* f_ext, double* x_out, double* v_out, qnsim_stats* stats);

/* One time step from device arrays (n x 3 doubles, caller's numbering): the
 * same step as qnsim_step (Eq. PD, section 3; Algorithms 1 and 2, sections
 * 4.1 and 4.2), on the given stream (hipStream_t as void*; NULL = the null stream: the step then
 * runs on the context's own stream, after the work already submitted to the
 * null stream). x_out / v_out may alias x / v. The inverted-input check of
 * qnsim_step is not made here: an infeasible x shows up as a non-finite
 * g_first. The step's work is ordered after earlier work on the stream; the
 * call returns when it is done (the device decides when every iteration has
 * ended, the host reads a 64-byte status). With options.step_graph the fixed
 * kernel sequence is captured once per set of buffers and replayed. */
int qnsim_step_device(qnsim_t* ctx, const double* d_x, const double* d_v, double h,
                      const double* d_fext, double* d_x_out, double* d_v_out,
                      void* stream, qnsim_stats* stats);

/* Autotuning of a prepared context (prepared for h) on its own workload:
 * times reps steps (after one untimed step) from the device state (d_x,
 * d_v), n x 3 float64 in caller order, which is not modified. what = 1: the
 * solve schedule among four (levels only; bottom subtrees per workgroup;
 * plus level merging; plus the dense top block: dense_top / subtree_cap /
 * level_merge = 0/0/0, 0/384/0, 0/384/1, 6144/384/1), each a new host
 * analysis and factorisation for h (section 3: the prefactored A); what =
 * 2: the element tile among 128, 256, 512 (the per-element gradient of
 * section 4.1); what = 4: line-search trials enqueued per iteration
 * (trials_per_cycle 1, 2 or 3: the step's fixed launch sequence, with
 * Algorithm 1's line search unchanged); bits combine, 0 = 7: the schedule,
 * then the tile, then the trials. The context keeps the fastest options
 * and stays prepared for h; the options are reported in *info with the
 * measured milliseconds per step (NaN: not timed). Results with different
 * schedules or tiles agree to rounding; the trials per cycle change no
 * result.
 * Errors: QNSIM_E_INVALID, QNSIM_E_STATE / QNSIM_E_H_MISMATCH (not prepared
 * for h), QNSIM_E_NOMEM, QNSIM_E_DEVICE, QNSIM_E_NOT_SPD; on an error the
 * options return to their values before the call and the context is left
 * unprepared. Synchronous; the context must not be stepping. */
typedef struct {
  int32_t dense_top;     /* options kept */
  int32_t subtree_cap;
  int32_t level_merge;
  int32_t elem_tile;
  int32_t trials_per_cycle;
  int32_t reserved;
  double schedule_ms[4]; /* ms per step for the four schedules, in the order above */
  double tile_ms[3];     /* ms per step with the kept schedule, tiles 128, 256, 512 */
  double trials_ms[3];   /* ms per step with the kept schedule and tile, 1, 2, 3 trials per cycle */
} qnsim_tune_info;
int qnsim_tune(qnsim_t* ctx, double h, const double* d_x, const double* d_v, int32_t reps,
               int32_t what, qnsim_tune_info* info);

/* Run `steps` consecutive time steps on device arrays, advancing (d_x, d_v)
 * in place (stream as qnsim_step_device), and accumulate counters into stats
 * (if non-null). Used to time trajectories; each step reads back one status. */
int qnsim_run_device(qnsim_t* ctx, double* d_x, double* d_v, double h,
                     const double* d_fext, int32_t steps, void* stream,
                     qnsim_stats* stats);

/* Request the extra gradient pass that fills grad_norm_last (0 = off). */
int qnsim_set_diagnostics(qnsim_t* ctx, int32_t final_gradient);

/* Plane colliders (section 4.3): the half-spaces n . x >= c given as rows
 * (nx, ny, nz, c) of planes (n_planes x 4; n is normalised, c scaled with it;
 * at most 16; n_planes = 0 removes them). At the start of every iteration of
 * a step, each free vertex that penetrates or touches a plane (n . x_k <= c)
 * and is not separating from it (its motion since the start of the step,
 * x_k - x_n, does not point along n) gets the energy term
 * stiffness (n . x - c)^2 of its deepest such plane (the paper's
 * ((S x - t)^T n)^2, t the projection on the plane, with a weight); the terms
 * stay fixed through that iteration's line search and enter g and grad g but
 * not A, so nothing is refactored. May be called before or after prepare.
 * The probes (qnsim_eval_device) evaluate g without them. */
int qnsim_set_colliders(qnsim_t* ctx, int32_t n_planes, const double* planes, double stiffness);

/* Per-tet stiffness k (T doubles), available after qnsim_analyze/prepare:
 * the slope of the least-squares line through the material's stress-stretch
 * profile over [fit_lo, fit_hi] (section 4.1, Eq. stiffness). */
int qnsim_get_stiffness(const qnsim_t* ctx, double* k);

/* Lumped vertex masses (n doubles), available after qnsim_analyze/prepare. */
int qnsim_get_masses(const qnsim_t* ctx, double* mass);

/* Factor and schedule facts, available after qnsim_analyze/prepare. */
int qnsim_get_factor_info(const qnsim_t* ctx, qnsim_factor_info* info);

/* The Cholesky factor as CSC of the permuted free-vertex matrix, so that
 * A[perm][:, perm] = L L^T. perm[i] = caller vertex id of the i-th free
 * unknown (n_free int32). colptr (n_free+1 int64), rowidx / values (nnz_L_exact
 * int32 / double). Any output pointer may be NULL to skip it. */
int qnsim_export_factor(const qnsim_t* ctx, int32_t* perm, int64_t* colptr,
                        int32_t* rowidx, double* values);

/* Numeric refactorisation on the device for a new time step h. A = M/h^2 +
 * sum_e V_e k_e G_e^T G_e (section 3, Eq. PDsolution; section 4.1,
 * Eq. stiffness for k_e) depends on h, and the method
 * prefactors it once per step size. This keeps the ordering and the
 * supernodal structure of the prepared factor and recomputes its values on
 * the device: a multifrontal Cholesky factorisation level by level of the
 * supernode tree, then the solve blocks in place. The first call builds a
 * device plan (host work linear in the mesh, plus a device workspace of
 * sum over supernodes of (rows)^2 doubles, kept until the context is
 * re-prepared or destroyed); later calls do no host work besides launching.
 * After success, steps and solves use h, and qnsim_export_factor returns
 * QNSIM_E_STATE (the host copy of the factor belongs to the analysed h) until
 * the next qnsim_prepare. *device_ms (nullable): device time of the
 * refactorisation. Errors: QNSIM_E_STATE (not prepared), QNSIM_E_INVALID (h
 * not positive and finite, or a front wider than 20000 rows),
 * QNSIM_E_NOT_SPD (a pivot not positive: the previous factor and h stay in
 * force), QNSIM_E_NOMEM, QNSIM_E_DEVICE. Synchronises. */
int qnsim_refactor(qnsim_t* ctx, double h, double* device_ms);

/* ---- kernel-level entry points (device arrays, caller's numbering) ------ */

/* Objective and gradient at positions d_x with inertia target d_y (n x 3):
 * *g_out = g(x) (Eq. PD, free vertices), d_grad (n x 3) = grad g with zero
 * rows at pinned vertices. Synchronises. */
int qnsim_eval_device(qnsim_t* ctx, const double* d_x, const double* d_y,
                      double* g_out, double* d_grad, void* stream);

/* Per-element energy density Psi (T doubles) and first Piola stress P
 * (T x 9, row-major 3x3 per tet) at positions d_x, evaluated as the element
 * pass does in the context's precision mode (QNSIM_MIXED: FP32 from the
 * displacement gradient, returned widened to FP64). Synchronises. */
int qnsim_element_stress_device(qnsim_t* ctx, const double* d_x, double* d_psi,
                                double* d_P, void* stream);

/* r = A^{-1} q with the prefactored matrix (section 3, Eq. PDsolution): d_q and
 * d_r are n x 3 in the caller's numbering; rows of pinned vertices are ignored
 * in q and set to zero in r. Stream-ordered. */
int qnsim_solve_device(qnsim_t* ctx, const double* d_q, double* d_r, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve
 * of qnsim_solve_device, with the same arguments, kernels and results (bit
 * for bit), whose working memory (permuted right-hand side and solution,
 * forward intermediate, update layers, dense top block right-hand side) lives
 * in a fixed 16 MiB device array of the library instead of the context's
 * buffers; it calls no allocation routine. Each GPU holds its own copy of the
 * array until the process ends, and every call on a GPU shares it: calls that
 * overlap on one GPU (other streams or threads) race and must be serialised
 * by the caller. The array keeps the last call's contents; the call clears
 * what must start at zero. Returns QNSIM_E_INVALID when the mesh needs more
 * working memory than the array holds (about 9 n_free + the update layers
 * doubles: the 40^3 block fits), QNSIM_E_STATE before qnsim_prepare,
 * QNSIM_E_DEVICE on a HIP error. Stream-ordered, like qnsim_solve_device. */
int qnsim_solve_device_noalloc(qnsim_t* ctx, const double* d_q, double* d_r, void* stream);

/* ---- measurement -------------------------------------------------------- */

/* Kernels that qnsim_time_kernel can time in isolation. */
#define QNSIM_KERNEL_ELEMENT 0  /* element pass of a line-search trial: energy and
                                   gradient contributions at x_k + alpha d   */
#define QNSIM_KERNEL_GATHER 1   /* gradient gather (inertia + element terms)     */
#define QNSIM_KERNEL_SOLVE 2    /* r = A^{-1} q: all forward and backward levels */

/* Time `reps` back-to-back launches of one kernel of the step on the
 * context's stream with HIP events, on the device state left by the last step
 * (call after at least one step). *avg_ms = mean time per launch (for
 * QNSIM_KERNEL_SOLVE: per complete solve). Synchronises. The kernels' inputs
 * are not changed; their outputs are scratch of the next step. */
int qnsim_time_kernel(qnsim_t* ctx, int32_t kernel, int32_t reps, double* avg_ms);

/* Descriptive text of a status code, and of the context's last failure. */
const char* qnsim_strerror(int code);
const char* qnsim_last_error(const qnsim_t* ctx);

/* ==== Pools: many resident simulations on one GPU ========================
 *
 * A pool keeps many independent simulations (mesh, materials, prefactored A
 * and state x, v) resident in device memory and advances any subset of them
 * by one implicit-Euler step each, with the same method and options as a
 * single context (sections 3-4). Admitted simulations are grouped; a group
 * is one concatenated device mesh (A block diagonal) whose every phase (line
 * -search trials, gradient gather, two-loop recursion, prefactored solve) is
 * one kernel launch over all its stepping simulations, each simulation
 * keeping its own line search and curvature pairs. A simulation's result in
 * a group equals its result alone (same factor options, same reductions).
 *
 * Lifecycle: qnsim_pool_add (host precompute, the simulation is staged) ->
 * qnsim_pool_commit (staged simulations are uploaded into new groups while
 * the device-memory budget allows) -> qnsim_pool_step (synchronous batched
 * step) or the serving loop (qnsim_pool_serve_start, qnsim_pool_submit,
 * qnsim_pool_wait). Pools use dense_top = 0 and level_merge = 0: a level
 * launch of a group serves all its simulations, so merging levels would only
 * add bytes. Every simulation uses the pool's h (qnsim_pool_set_h changes
 * it) and gravity, plus its own external force if one is set
 * (qnsim_pool_set_force) or the request's (qnsim_pool_submit_force).
 * qnsim_pool_tune picks each group's element tile. Functions of one pool may
 * be called from several threads. */
typedef struct qnsim_pool qnsim_pool_t;

/* One simulation: mesh (as qnsim_set_mesh), pinned vertices (as
 * qnsim_set_pinned; pinned may be NULL when n_pinned = 0), materials (as
 * qnsim_set_materials; tet_mat may be NULL) and the initial state x0, v0
 * (n x 3; NULL: x0 = rest positions, v0 = 0). */
typedef struct {
  int32_t n_verts;
  const double* rest_xyz;
  int32_t n_tets;
  const int32_t* tets;
  int32_t n_pinned;
  const int32_t* pinned;
  int32_t n_mat;
  const qnsim_material* mats;
  const int32_t* tet_mat;
  const double* x0;
  const double* v0;
} qnsim_mesh_desc;

typedef struct {
  int32_t sims_staged;     /* added, not yet resident                           */
  int32_t sims_resident;   /* admitted into a group and not removed             */
  int32_t groups;          /* device meshes                                     */
  int32_t serving;         /* 1 while the request loop runs                     */
  int64_t budget_bytes;    /* device-memory budget of the pool                  */
  int64_t used_bytes;      /* device memory held by the groups                  */
  int64_t steps_done;      /* simulation steps completed since creation         */
  int64_t batches_done;    /* batched group steps since creation                */
  int64_t nnz_L;           /* structural nonzeros of the resident factors       */
  int64_t n_free;          /* free vertices of the resident simulations         */
  int64_t n_tets;          /* tetrahedra of the resident simulations            */
  int32_t groups_made;     /* groups created (the range of group indices)       */
  int32_t reserved;
} qnsim_pool_info;

/* Creates a pool for time step h with a device-memory budget in bytes
 * (> 0). opts as qnsim_create (NULL: defaults); dense_top and level_merge
 * are forced to 0. */
int qnsim_pool_create(const qnsim_options* opts, double h, int64_t budget_bytes,
                      qnsim_pool_t** out);
/* Stops the request loop (finishing queued requests) and frees everything. */
void qnsim_pool_destroy(qnsim_pool_t* pool);

/* Validates and analyses n simulations on the host (in parallel) and stages
 * them; ids[i] receives the id of descs[i]. On error nothing is staged;
 * errors are those of qnsim_set_mesh / set_pinned / set_materials /
 * qnsim_prepare's analysis, for the first failing description. */
int qnsim_pool_add(qnsim_pool_t* pool, int32_t n, const qnsim_mesh_desc* descs, int32_t* ids);

/* Uploads staged simulations (in id order) into new groups of at most
 * max_group_sims simulations (<= 0: one group), skipping any whose estimated
 * device memory does not fit the remaining budget (they stay staged).
 * *n_admitted (nullable) receives the number admitted. Allowed while the
 * request loop runs: the admission is planned under the pool's lock, the
 * groups are built and uploaded without it (resident groups keep stepping on
 * their own streams), and the new simulations become resident, able to take
 * requests, when their group is published. A group whose removed members
 * hold at least half of its estimated memory is first rebuilt with its live
 * members while the old group keeps serving them; once the old group is not
 * stepping, their states and forces are copied to the new group on the
 * device (under the pool's lock) and it replaces the old one, before the new
 * groups are built; the memory it frees counts for the admission. One commit
 * runs at a time (later ones wait); on a failure the simulations of the
 * failed group and of the groups after it stay staged and the first error
 * is returned. */
int qnsim_pool_commit(qnsim_pool_t* pool, int32_t max_group_sims, int32_t* n_admitted);

/* Removes a resident or staged simulation; a group's device memory is freed
 * when its last simulation is removed, or returned by the next commit's
 * rebuild when removed members hold half of it. */
int qnsim_pool_remove(qnsim_pool_t* pool, int32_t id);

/* One step of each listed resident simulation (distinct ids): groups run
 * concurrently, each as one batched step of its listed simulations; the
 * others keep their state. stats (nullable) receives one record per id.
 * Synchronous. Not allowed while the request loop runs (QNSIM_E_STATE). */
int qnsim_pool_step(qnsim_pool_t* pool, int32_t n, const int32_t* ids, qnsim_stats* stats);

/* State of a resident simulation (host arrays, n x 3, its own numbering). */
/* External force of a resident simulation (section 3: f_ext in the inertial
 * target y = x + h v + h^2 M^{-1} f_ext): n x 3 float64 in newtons, caller
 * order, copied; NULL removes it. It acts, with the pool's gravity, in every
 * later step of the simulation (batched or served) until changed: a step
 * uses the force set before it starts. The first force set in a group
 * allocates one n x 3 array for the whole group (counted in the pool's used
 * bytes, outside the admission budget). Waits for a running step of the
 * group. Errors: QNSIM_E_INVALID (not resident), QNSIM_E_NONFINITE,
 * QNSIM_E_NOMEM, QNSIM_E_DEVICE. */
int qnsim_pool_set_force(qnsim_pool_t* pool, int32_t id, const double* f_ext);
int qnsim_pool_get_state(qnsim_pool_t* pool, int32_t id, double* x, double* v);
int qnsim_pool_set_state(qnsim_pool_t* pool, int32_t id, const double* x, const double* v);

/* Request loop: `lanes` (1..8) host threads each take the group with the
 * oldest queued request that is not already stepping, step all its
 * simulations that have a queued request (one request per simulation per
 * batch, in arrival order), and complete those requests; requests that
 * arrive meanwhile join that group's next batch, and different groups step
 * concurrently on their own streams. */
int qnsim_pool_serve_start(qnsim_pool_t* pool, int32_t lanes);
/* Queues one step request for a resident simulation; *ticket identifies it. */
int qnsim_pool_submit(qnsim_pool_t* pool, int32_t id, int64_t* ticket);
/* As qnsim_pool_submit, with an external force for this step only (section
 * 3: f_ext in y; n x 3 float64 in newtons, caller order, copied at submit;
 * NULL: as qnsim_pool_submit): the step that serves the request uses it in
 * place of the simulation's own force (qnsim_pool_set_force), which later
 * steps use again. Errors as qnsim_pool_submit, and QNSIM_E_NONFINITE. */
int qnsim_pool_submit_force(qnsim_pool_t* pool, int32_t id, const double* f_ext, int64_t* ticket);
/* Waits for a request (at most timeout_s seconds; < 0: no limit) and
 * returns its status: the step's own error, or QNSIM_E_STATE on time-out or
 * an unknown ticket. stats and latency_s (time from submit to completion;
 * both nullable) are filled on success. A ticket can be waited for once. */
int qnsim_pool_wait(qnsim_pool_t* pool, int64_t ticket, double timeout_s, qnsim_stats* stats,
                    double* latency_s);
/* Stops the request loop after the queued requests are done. */
int qnsim_pool_serve_stop(qnsim_pool_t* pool);

int qnsim_pool_get_info(qnsim_pool_t* pool, qnsim_pool_info* info);

/* Where simulation id is: QNSIM_SIM_STAGED (added, not admitted, or being
 * admitted by a running commit), QNSIM_SIM_RESIDENT (in a group; *group, if
 * non-null, receives its index) or QNSIM_SIM_REMOVED (*group = -1). */
#define QNSIM_SIM_STAGED 0
#define QNSIM_SIM_RESIDENT 1
#define QNSIM_SIM_REMOVED 2
int qnsim_pool_status(qnsim_pool_t* pool, int32_t id, int32_t* status, int32_t* group);

/* Change the pool's time step to h (section 3, Eq. PDsolution: A = M/h^2 + L
 * depends on h). Every resident group's A is refactored on the device (as
 * qnsim_refactor; the first call per group builds its refactorisation plan,
 * whose device memory is outside the pool's budget); staged simulations are
 * analysed again on the host for h. Later steps use h. Needs the request loop
 * stopped (QNSIM_E_STATE) and waits for running steps. On a failure the
 * groups already refactored return to the previous h and the error is
 * returned (QNSIM_E_NOT_SPD, QNSIM_E_NOMEM, QNSIM_E_DEVICE). *device_ms
 * (nullable): the device time of the refactorisations. */
int qnsim_pool_set_h(qnsim_pool_t* pool, double h, double* device_ms);
/* Autotuning of a pool's groups: the element tile of the element pass (the
 * per-element gradient of E, section 4.1) and, optionally, the line-search
 * trials enqueued per iteration. For each resident group, times reps batched
 * steps of all its members (after one untimed step) with each candidate
 * element tile (candidates: a mask of 1 = 128, 2 = 256, 4 = 512 tets per
 * block; 0: all three), on a copy of the members' states, and keeps the
 * fastest candidate: the group's device mesh is rebuilt with that tile (for
 * a tile other than the current one, a second copy of the group's device
 * mesh exists during the call). Members' states are unchanged. Later steps
 * of a simulation equal, bit for bit, its steps alone with elem_tile set to
 * its group's tile. tiles: n_groups entries, the chosen tile of each group
 * in admission order (0: group with no resident member); step_ms (nullable):
 * n_groups x 3 measured milliseconds per step for the tiles 128, 256, 512
 * (NaN: not a candidate). trials (nullable): with the kept tile, also time
 * 1, 2 and 3 line-search trials enqueued per iteration (trials_per_cycle; no
 * result changes) and keep the fastest for the group; n_groups entries, the
 * kept value (0: group with no resident member); trials_ms (nullable):
 * n_groups x 3 milliseconds per step. Needs the request loop stopped
 * (QNSIM_E_STATE); waits for running steps; other pool calls wait until it
 * returns. Errors: QNSIM_E_INVALID (bad mask, reps outside 1..1000),
 * QNSIM_E_NOMEM / QNSIM_E_DEVICE (the rebuild failed: the group keeps its
 * mesh). */
int qnsim_pool_tune(qnsim_pool_t* pool, int32_t candidates, int32_t reps, int32_t n_groups,
                    int32_t* tiles, double* step_ms, int32_t* trials, double* trials_ms);
/* As qnsim_time_kernel, on group `group` (0-based, in admission order) with
 * every simulation of the group taking part; after at least one step of the
 * group. Not while the request loop runs. */
int qnsim_pool_time_kernel(qnsim_pool_t* pool, int32_t group, int32_t kernel, int32_t reps,
                           double* avg_ms);
const char* qnsim_pool_last_error(const qnsim_pool_t* pool);

#ifdef __cplusplus
}
#endif

#endif /* QNSIM_H */
