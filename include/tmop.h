/*
 * tmop.h -- C ABI of the MI355X partially assembled TMOP library.
 *
 * The library evaluates the TMOP objective of high-order node-movement mesh
 * optimisation, its gradient and its Hessian action with partial assembly
 * (matrix-free, sum-factorized) on quad (2D) and hex (3D) meshes of order p,
 * and drives the Newton-MINRES solve with its backtracking line search.
 *
 *   Mesh nodes           x (Sec. 2.1, eq. eq_x): a global vector of d x N_x
 *                        coordinates, the element map x = sum_i x_{E,i} w_i.
 *   Target / metric      T = A W^{-1} (Sec. 2.2, eqs. eq_A, eq_T); shape
 *                        metrics mu_2 (quads) and mu_303 (hexes), size metric
 *                        mu_55, shape+size metrics mu_7 and mu_9 (quads)
 *                        (Sec. 2.2, Sec. 4.1).
 *   Objective            F(x) = sum_E int mu(T) (Sec. 2.2, eq. eq_F_full, first
 *                        term, spatial weight 1; Sec. 3.3, eq. D0_expression).
 *   Gradient             Sec. 3.3, eq. eq_vm_pa_grad.
 *   Hessian action       Sec. 3.4, eq. eq_vm_pa_hess, with the quadrature data
 *                        stored once per Newton step and applied matrix-free.
 *   Hessian diagonal     Sec. 3.4 (Jacobi preconditioning from tensor
 *                        contractions).
 *   Solve                Sec. 2.3: x <- x - alpha dx, dx = H^{-1} g by MINRES
 *                        with Jacobi preconditioning; alpha halved from 1 until
 *                        det A > 0 at every quadrature point, F < 1.2 F_old and
 *                        |g| < 1.2 |g_old|; stop when |g|/|g_0| <= eps.
 *
 * Conventions for every entry point:
 *   - Vectors are caller-owned DEVICE buffers of doubles, SoA by component:
 *     x[c * N_x + g], c < dim.  For a structured box of n_0 x n_1 (x n_2)
 *     elements the global node g is lexicographic on the (n_k p + 1) grid,
 *     first axis fastest; local element nodes are lexicographic
 *     i = i_0 + (p+1) (i_1 + (p+1) i_2).
 *   - The reference element is [0,1]^d; the 1D basis is the Lagrange basis on
 *     the p+1 Gauss-Lobatto-Legendre points of [0,1]; quadrature is the
 *     tensor Gauss-Legendre rule with nq1d points per direction.
 *   - Fixed (essential) DoFs enter as H_c = P H P + (I - P), g_c = P g, where P
 *     zeroes the fixed entries.  By default every component of every node on
 *     the boundary of a structured box is fixed.
 *   - Calls are asynchronous on the stream given at creation except those
 *     that return host scalars, which synchronise that stream.
 *   - Every function returns a tmop_status; on failure tmop_last_error()
 *     returns a thread-local message.  No C++ exception crosses this ABI.
 *   - The context owns its workspace (quadrature tensor, element-vector
 *     scratch, reduction scratch, solver vectors); it never frees or keeps
 *     pointers the caller passes in, except elem_to_node / ess_mask, which
 *     must stay valid for the context's lifetime.
 */
#ifndef TMOP_H
#define TMOP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TMOP_OK = 0,
    TMOP_ERR_INVALID_ARG = 1,   /* bad pointer, size, order or combination   */
    TMOP_ERR_UNSUPPORTED = 2,   /* valid request this build has no kernel for */
    TMOP_ERR_INVERTED = 3,      /* det A <= 0 at a quadrature point of input */
    TMOP_ERR_LINESEARCH = 4,    /* no step length accepted                   */
    TMOP_ERR_NOT_CONVERGED = 5, /* max_newton reached                         */
    TMOP_ERR_NONFINITE = 6,     /* NaN / Inf in input or iterate              */
    TMOP_ERR_OOM = 7,           /* device allocation failed                   */
    TMOP_ERR_BUDGET = 8,        /* request larger than a pool's HBM budget    */
    TMOP_ERR_BUSY = 9,          /* pool full right now; retry later           */
    TMOP_ERR_HIP = 10,          /* HIP runtime error                          */
    TMOP_ERR_STATE = 11         /* call out of order (e.g. apply before setup) */
} tmop_status;

enum { TMOP_FP64 = 0, TMOP_MIXED = 1 };       /* tmop_params.precision */
enum { TMOP_ESS_BOUNDARY = 0, TMOP_ESS_NONE = 1, TMOP_ESS_MASK = 2 };
enum { TMOP_HESS_TENSOR = 0, TMOP_HESS_COMPACT = 1 };  /* tmop_params.hess_storage */
enum { TMOP_QUAD_GL = 0, TMOP_QUAD_GLL = 1 };          /* tmop_params.quad_rule */
enum { TMOP_SWEEPS_PENCIL = 0, TMOP_SWEEPS_MFMA = 1 };  /* tmop_set_sweeps */

typedef struct tmop_ctx tmop_ctx;

/* Mesh description.  Structured box: elem_to_node == NULL, nx, ny (, nz) > 0.
 * General mesh: elem_to_node = device int32 array [num_elems][(p+1)^dim]
 * (lexicographic local order), num_elems and num_nodes set. */
typedef struct {
    int dim;                      /* 2 or 3 */
    int order_p;                  /* 1..4 */
    int nx, ny, nz;               /* elements per axis (structured box) */
    int num_elems;                /* general mesh only */
    int num_nodes;                /* general mesh only: N_x */
    const int32_t *elem_to_node;  /* device, or NULL for the structured box */
    int ess_mode;                 /* TMOP_ESS_BOUNDARY (box only) / _NONE / _MASK */
    const uint8_t *ess_mask;      /* device [dim*N_x], nonzero = fixed, for _MASK */
} tmop_mesh_desc;

/* Discretisation, target and precision. */
typedef struct {
    int metric;     /* dim 2: 2 (mu_2 = |T|^2/(2 tau) - 1), 7 (mu_7 = |T - T^{-t}|^2),
                       9 (mu_9 = tau mu_7) or 55 (mu_55 = (tau - 1)^2);
                       dim 3: 303 (mu_303 = |T|^2/(3 tau^{2/3}) - 1) or 55.
                       Others: TMOP_ERR_UNSUPPORTED */
    int nq1d;       /* quadrature points per direction, p+1 .. p+3 */
    int has_W;      /* 0: ideal target W = I; 1: use the constant W below */
    double W[9];    /* constant target matrix, row-major dim x dim, det > 0 */
    int precision;  /* TMOP_FP64, or TMOP_MIXED: FP32 quadrature data and
                       FP32 Hessian action (FP32 accumulation); energy,
                       gradient, det, line search and reductions stay FP64 */
    int hess_storage; /* TMOP_HESS_TENSOR: per point the packed symmetric
                       d^2 x d^2 second-derivative tensor times the weight
                       (45 / 10 entries, Sec. 3.4); TMOP_HESS_COMPACT: per
                       point T and the four weighted scalar coefficients of
                       the metric's second derivative (13 / 8 entries), the
                       tensor applied in closed form in the action.  Same
                       results; the compact form moves 3.5x fewer bytes. */
    int quad_rule;  /* 1D rule of the tensor quadrature (Sec. 3.1 builds the
                       element rule from a 1D rule without naming it):
                       TMOP_QUAD_GL (0, default) Gauss-Legendre, or
                       TMOP_QUAD_GLL (1) Gauss-Lobatto-Legendre (nq1d >= 2;
                       includes the element's faces, so the det test also
                       covers its vertices).  Pooled solves take GL only. */
} tmop_params;

typedef struct {
    double rel_grad_tol;  /* stop when |g_c|/|g_c(x_0)| <= this (e.g. 1e-8)   */
    int max_newton;       /* Newton iteration cap                             */
    int max_minres;       /* MINRES iterations per Newton step (e.g. 50)      */
    double minres_rtol;   /* relative preconditioned-residual tolerance       */
    int max_halvings;     /* line-search halvings before TMOP_ERR_LINESEARCH  */
    int jacobi;           /* 1: Jacobi-preconditioned MINRES, 0: plain        */
    double g0_norm;       /* > 0: |g_c(x_0)| of an earlier run (resume); else computed */
} tmop_solve_params;

typedef struct {
    int newton_its;       /* accepted Newton updates   */
    int minres_its_total; /* MINRES iterations, summed */
    int halvings_total;   /* line-search halvings      */
    int status;           /* tmop_status of the solve  */
    double F0, F;         /* initial and final objective                */
    double g0_norm, g_norm; /* initial and final |g_c| (l2, all DoFs)  */
    double t_setup_ms, t_minres_ms, t_linesearch_ms, t_total_ms; /* phase times */
    /* Hessian actions inside MINRES, timed with HIP events on the context's
     * stream when timing is enabled (tmop_set_timing); zero otherwise. */
    double t_apply_ms;      /* summed device time of the actions (element + gather) */
    double t_apply_elem_ms; /* summed device time of the element kernel alone       */
    int n_apply;            /* number of timed actions                              */
    int reserved;
} tmop_solve_report;

/* One entry of a solve's per-iteration record (Sec. 2.3): the objective and
 * |g_c| at the mesh after k accepted Newton updates (k = 0: the initial mesh),
 * and the MINRES iterations and line-search halvings of the update that led
 * to it (0 for k = 0). */
typedef struct {
    double F;
    double g_norm;
    int minres_its;
    int halvings;
} tmop_iter_record;

/* ---------------------------------------------------------------------- */
/* Context                                                                 */
/* ---------------------------------------------------------------------- */

/* Create a context on the current HIP device; hip_stream may be NULL (the
 * null stream).  Allocates the workspace for the Hessian tensor of this mesh
 * (N_e N_q d^2(d^2+1)/2 entries of 8 or 4 bytes) and the element scratch.
 * Errors: INVALID_ARG, UNSUPPORTED (order/nq combination without a kernel),
 * OOM. */
int tmop_create(tmop_ctx **out, const tmop_mesh_desc *mesh, const tmop_params *prm,
                void *hip_stream);
int tmop_destroy(tmop_ctx *ctx);

/* Device bytes a context for this mesh/params would allocate (excluding the
 * solver's work vectors when with_solver == 0). */
int tmop_workspace_bytes(const tmop_mesh_desc *mesh, const tmop_params *prm, int with_solver,
                         size_t *bytes);

/* Number of global nodes N_x and DoFs d*N_x of the context's mesh. */
int tmop_sizes(const tmop_ctx *ctx, int *num_nodes, int *num_dofs);

/* The 1D node positions (p+1 values on [0,1]) the library places element
 * nodes at, written to host memory; lets a caller build uniform meshes. */
int tmop_basis_nodes(int order_p, double *nodes_host);

/* ---------------------------------------------------------------------- */
/* Evaluations (Sec. 3.3, 3.4)                                             */
/* ---------------------------------------------------------------------- */

/* F(x) to host.  Synchronises.  If det A <= 0 at a quadrature point the
 * return is TMOP_ERR_INVERTED and *F_host = +inf. */
int tmop_energy(tmop_ctx *ctx, const double *x_dev, double *F_host);

/* min over all quadrature points of det A(x), to host.  Synchronises. */
int tmop_min_det(tmop_ctx *ctx, const double *x_dev, double *mindet_host);

/* F and min det A in one pass (both to host).  Synchronises.  Returns
 * TMOP_ERR_INVERTED (F = +inf) when min det <= 0. */
int tmop_energy_mindet(tmop_ctx *ctx, const double *x_dev, double *F_host, double *mindet_host);

/* g_c = P dF/dx (device, d*N_x).  Asynchronous. */
int tmop_gradient(tmop_ctx *ctx, const double *x_dev, double *g_dev);

/* F, min det A (to host), g_c (device, d*N_x) and |g_c|^2 (to host) at one
 * point in one element pass: the gradient kernel also sums the energy terms
 * (Sec. 3.3), as the line search of the Newton solver needs all four.
 * Synchronises.  F, min det A and g_c are bitwise those of
 * tmop_energy_mindet and tmop_gradient, and |g_c|^2 is the sum of squares
 * of g_c in the library's reduction order.  Returns TMOP_ERR_INVERTED
 * (F = +inf, g_c of no use) when det T <= 0 at a quadrature point.  Any
 * host pointer may be NULL. */
int tmop_energy_gradient(tmop_ctx *ctx, const double *x_dev, double *F_host,
                         double *mindet_host, double *g_dev, double *g2_host);

/* Store the per-quadrature-point Hessian data of F at x (symmetric
 * d^2 x d^2 tensor times quadrature weight, d^2(d^2+1)/2 entries per point).
 * Asynchronous.  Subsequent apply/diag calls use it. */
int tmop_hessian_setup(tmop_ctx *ctx, const double *x_dev);

/* y = H_c v with the data of the last setup.  Asynchronous.  In MIXED
 * precision the element work runs in FP32; v and y stay FP64 in memory.
 * v and y must not alias.  Errors: STATE if no setup was done. */
int tmop_hessian_apply(tmop_ctx *ctx, const double *v_dev, double *y_dev);

/* Diagonal of H_c (fixed entries 1) from the last setup.  Asynchronous. */
int tmop_hessian_diag(tmop_ctx *ctx, double *d_dev);

/* tmop_hessian_setup at x followed by tmop_hessian_diag into d_dev (device,
 * d*N_x), in one element pass where the class allows it (hex classes whose
 * n_q^3 points times elements per workgroup fit one workgroup pass, pencil
 * sweeps; tensor or compact storage): the per-point data feeds the
 * diagonal's contraction on chip instead of being read back from HBM
 * (Sec. 3.4; the Newton solver's Jacobi preconditioner uses this).  The stored data and d
 * are bitwise those of the two separate calls.  Asynchronous. */
int tmop_hessian_setup_diag(tmop_ctx *ctx, const double *x_dev, double *d_dev);

/* ---------------------------------------------------------------------- */
/* Newton-MINRES solve (Sec. 2.3)                                          */
/* ---------------------------------------------------------------------- */

/* Optimise x in place.  Returns the solve status (also in rep->status). */
int tmop_solve(tmop_ctx *ctx, double *x_dev_inout, const tmop_solve_params *sp,
               tmop_solve_report *rep);

/* One Newton step with exactly n_minres MINRES iterations from x, without
 * the convergence test: setup, diagonal, MINRES, line search and update of x
 * in place.  Reports as tmop_solve.  Used to time a fixed amount of work. */
int tmop_newton_step(tmop_ctx *ctx, double *x_dev_inout, int n_minres, int jacobi,
                     tmop_solve_report *rep);

/* Preconditioned MINRES on H_c dx = b with the last setup (and, when
 * jacobi != 0, the diagonal of the last setup).  dx is overwritten.
 * *its receives the iteration count.  Synchronises. */
int tmop_minres(tmop_ctx *ctx, const double *b_dev, double *dx_dev, int max_its, double rtol,
                int jacobi, int *its);

/* MINRES (Paige and Saunders' recurrences, Sec. 2.3) forms its solution as a
 * combination of the preconditioned Lanczos vectors.  When max_its + 1 of them
 * (each N_dof doubles, rounded up to 256 bytes) fit in max_bytes and in free
 * device memory, and max_its <= 255, tmop_minres, tmop_solve and
 * tmop_newton_step keep them resident in a buffer the context owns (grown on
 * demand, freed by tmop_destroy) and form dx once after the loop; otherwise
 * every iteration updates dx with the three-term recurrence.  Both give the
 * same iterates up to rounding.  Default: no limit; 0 always selects the
 * three-term update.  Takes effect on the next solve. */
int tmop_set_lanczos_bank_limit(tmop_ctx *ctx, size_t max_bytes);

/* ---------------------------------------------------------------------- */
/* Batched and served solves                                               */
/* ---------------------------------------------------------------------- */

/* A pool advances many independent solves (structured boxes of any order,
 * dimension, precision and storage) together through the Newton-MINRES loop
 * of Sec. 2.3.  Each phase (setup, diagonal, MINRES iterations, line-search
 * trials) is one launch per kernel class (dim, p, n_q, storage, precision)
 * over the elements of every participating solve, and six MINRES iterations
 * are replayed as one HIP graph.  Every solve owns a contiguous region of one
 * device arena of hbm_budget bytes; a solve's arithmetic does not depend on
 * the other solves in the pool (its reductions run over its own data in a
 * fixed order), so its result is the same alone and in the mix.
 *
 * Calls on one pool are not thread-safe; the pool runs on its own HIP
 * stream and synchronises with the caller's stream where it reads or writes
 * caller buffers. */
typedef struct tmop_pool tmop_pool;

/* Create a pool with an arena of hbm_budget bytes and up to max_slots
 * concurrent solves.  The pool's work runs on hip_stream when it is not
 * NULL (the caller keeps it alive until tmop_pool_destroy), else on a
 * non-blocking stream the pool creates and destroys.  Errors: INVALID_ARG,
 * OOM. */
int tmop_pool_create(tmop_pool **out, size_t hbm_budget, int max_slots, void *hip_stream);
int tmop_pool_destroy(tmop_pool *pool);

/* Arena bytes one solve of this mesh/params takes (vectors, quadrature data,
 * element scratch).  Structured boxes only (elem_to_node must be NULL). */
int tmop_pool_request_bytes(const tmop_mesh_desc *mesh, const tmop_params *prm, size_t *bytes);

/* Admit one solve: copies the caller's device nodes x_dev (d*N_x doubles,
 * read after the work queued on src_stream) into the pool, and with
 * ess_mode TMOP_ESS_MASK also the mask (d*N_x bytes, counted in the slot's
 * region), so neither buffer is needed after the call.  Each solve keeps its
 * own solve parameters (MINRES cap and tolerance included).  Returns the slot
 * index.  Errors: BUDGET (the request alone exceeds the budget), BUSY (no
 * free slot or no free arena region now: retry after a release),
 * UNSUPPORTED, INVALID_ARG.  Does not run any solver work. */
int tmop_pool_admit(tmop_pool *pool, const tmop_mesh_desc *mesh, const tmop_params *prm,
                    const tmop_solve_params *sp, const double *x_dev, void *src_stream,
                    int *slot);

/* Admit one solve whose objective carries the limiting term (Sec. 2.2, eq.
 * eq_F_full, second integral; Sec. 3.5, eq. eq_pa_limiting), as
 * tmop_set_limiting does for a context: F gains coef * sum_E int_{E_t}
 * |x - x0|^2 / delta^2, with its gradient and its mass-like Hessian.
 * x0_dev: device [dim*N_x] reference nodes, copied into the slot's region
 * (read after the work queued on src_stream); coef >= 0 and delta > 0, else
 * TMOP_ERR_INVALID_ARG; coef = 0 admits a plain solve.  The region is
 * tmop_pool_request_bytes plus the reference nodes (d*N_x doubles rounded
 * up to 256 bytes).  Slots with the term run their own kernel launches (the
 * Hessian action in its base tile shape).  Otherwise as tmop_pool_admit. */
int tmop_pool_admit_limited(tmop_pool *pool, const tmop_mesh_desc *mesh, const tmop_params *prm,
                            const tmop_solve_params *sp, const double *x_dev, const double *x0_dev,
                            double coef, double delta, void *src_stream, int *slot);

/* Advance every unfinished solve by one Newton iteration (new solves first
 * get their initial energy, det check and gradient).  *n_active receives the
 * number of unfinished solves.  Synchronises the pool's stream. */
int tmop_pool_step(tmop_pool *pool, int *n_active);

/* Status of a slot: *done = 1 once the solve has finished (report.status
 * tells how); the report carries iteration counts, F, |g| and the wall time
 * since admission. */
int tmop_pool_poll(tmop_pool *pool, int slot, int *done, tmop_solve_report *rep);

/* Copy a slot's current nodes to the caller's device buffer.  The copy runs
 * on the pool's stream and has completed when the call returns, so x_dev
 * may be used on any stream (dst_stream is not needed and may be NULL). */
int tmop_pool_result(tmop_pool *pool, int slot, double *x_dev, void *dst_stream);

/* Evaluate one slot's operators with the pool's own batched kernels (the
 * launches of tmop_pool_step, gated to this slot), for checking a pooled
 * solve against a plain evaluation; between steps only.
 *   TMOP_EVAL_ENERGY:   F and min det A at in_dev = x (d*N_x doubles) to
 *                       out_host[0..1]; TMOP_ERR_INVERTED (F = +inf) when
 *                       min det <= 0 (Sec. 3.3, eq. D0_expression).
 *   TMOP_EVAL_GRADIENT: g_c at in_dev = x to out_dev (Sec. 3.3, eq.
 *                       eq_vm_pa_grad).
 *   TMOP_EVAL_SETUP:    store the slot's quadrature data at in_dev = x
 *                       (Sec. 3.4).
 *   TMOP_EVAL_APPLY:    out_dev = H_c in_dev from the slot's last setup
 *                       (Sec. 3.4, eq. eq_vm_pa_hess); FP32 element work for
 *                       a mixed-precision slot.
 *   TMOP_EVAL_DIAG:     out_dev = diagonal of H_c (fixed entries 1).
 * Inputs are read after the work queued on `stream`; outputs are complete on
 * return.  Overwrites only the slot's per-step scratch (trial nodes and
 * gradient, MINRES work vectors, diagonal, quadrature data, element
 * scratch), which the next tmop_pool_step recomputes.  Errors: INVALID_ARG,
 * STATE (APPLY / DIAG before any setup of the slot), INVERTED. */
enum { TMOP_EVAL_ENERGY = 0, TMOP_EVAL_GRADIENT = 1, TMOP_EVAL_SETUP = 2, TMOP_EVAL_APPLY = 3,
       TMOP_EVAL_DIAG = 4 };
int tmop_pool_evaluate(tmop_pool *pool, int slot, int what, const double *in_dev, double *out_dev,
                       double *out_host, void *stream);

/* Free a slot and its arena region. */
int tmop_pool_release(tmop_pool *pool, int slot);

/* Bytes in use, budget, and occupied slots. */
int tmop_pool_info(tmop_pool *pool, size_t *used_bytes, size_t *budget_bytes, int *slots_used);

/* HIP-graph replay of the pool's Newton steps (Sec. 2.3):
 *   0  no graphs: every launch issued by the host;
 *   1  (default) a block of six lockstep MINRES iterations captured once and
 *      replayed, the host checking every twelve iterations whether any slot
 *      still iterates, and deciding each line-search round;
 *   2  the whole Newton step captured once per pool layout and replayed once
 *      per tmop_pool_step: setup, Jacobi diagonal, every MINRES iteration
 *      (slots stop on the device), the first two line-search rounds and the
 *      stop test, with accept / halve decided per slot on the device; the
 *      host reads the per-slot state back once per step, and runs any further
 *      line-search rounds one by one (a slot still halving after two).
 * Every mode gives bitwise the same iterates.  Other values:
 * TMOP_ERR_INVALID_ARG. */
int tmop_pool_set_graph(tmop_pool *pool, int enable);

/* Enable or disable (default) resident MINRES Lanczos vectors for solves
 * admitted later (as tmop_set_lanczos_bank_limit for a context): an admitted
 * solve whose region plus (max_minres + 1) N_dof vectors (each rounded up to
 * 256 bytes) and 16 KB of scalars fits the free budget keeps them and forms
 * dx once per MINRES call; otherwise it takes the three-term update.
 * tmop_pool_request_bytes reports the size without them, so a budget sized
 * from it may admit fewer solves at once with this enabled.
 * tmop_batch_solve enables it and sizes its pool to hold them.  Same
 * iterates up to rounding. */
int tmop_pool_set_lanczos_bank(tmop_pool *pool, int enable);

/* Autotuner of the pool: for every kernel class with resident meshes, time
 * the batched Hessian action of each tile shape (as tmop_autotune) over
 * `reps` launches on the pool's stream, keep the fastest for the class and
 * record it for the process.  Call between steps (it overwrites the slots'
 * element scratch only); results are unchanged by the tile shape. */
int tmop_pool_autotune(tmop_pool *pool, int reps);

/* Thread-local description of the last pool error. */
const char *tmop_pool_last_error(void);

/* Solve count independent meshes together (a pool sized to fit them all,
 * resident Lanczos vectors, Hessian-action tile shapes autotuned per kernel
 * class after admission, each Newton step one replay of a HIP graph as in
 * tmop_pool_set_graph mode 2):
 * x_devs[k] holds mesh k's nodes on entry and the optimised nodes on return;
 * reps[k] its report.  Returns the first error, if any. */
int tmop_batch_solve(int count, const tmop_mesh_desc *meshes, const tmop_params *prms,
                     double *const *x_devs, const tmop_solve_params *sps,
                     tmop_solve_report *reps, void *hip_stream);

/* ---------------------------------------------------------------------- */
/* Timing helpers                                                          */
/* ---------------------------------------------------------------------- */

/* Time the Hessian action on the context's stream with HIP events recorded
 * on that stream (milliseconds per action): elem_ms is the mean time of the
 * element kernel over n actions with events around each kernel; total_ms is
 * the mean time of a whole action (element kernel plus node gather) over n
 * further actions run back to back, events only before and after the run.
 * 2n actions in all; y_dev receives the result. */
int tmop_time_apply(tmop_ctx *ctx, const double *v_dev, double *y_dev, int n, double *elem_ms,
                    double *total_ms);

/* Autotuner of the Hessian action's tile shape (elements per workgroup):
 * times the element kernel of the action for each tile shape the class has
 * (half, base and double the base max(1, 256 / n_q^d) elements per workgroup,
 * where they fit the LDS) over `reps` launches on the context's stream, keeps the
 * fastest for this context and records it for the class (dim, p, n_q,
 * storage, precision), so that contexts and pools created later in the
 * process start with it.  Needs tmop_hessian_setup; leaves y_dev = H v.
 * The tile shape changes no result (every element is computed alike).
 * epb (may be NULL): the chosen elements per workgroup. */
int tmop_autotune(tmop_ctx *ctx, const double *v_dev, double *y_dev, int reps, int *epb);

/* Elements per workgroup of the context's current Hessian-action tile. */
int tmop_tile_epb(tmop_ctx *ctx, int *epb);

/* Use the Hessian-action tile with epb elements per workgroup (one of the
 * shapes tmop_autotune considers), else TMOP_ERR_UNSUPPORTED. */
int tmop_set_tile(tmop_ctx *ctx, int epb);

/* Limiting term (Sec. 2.2, eq. eq_F_full, second integral; Sec. 3.5, eq.
 * eq_pa_limiting): adds coef * sum_E int_{E_t} |x - x0|^2 / delta^2 to F, with
 * its gradient and its mass-like Hessian, to every later evaluation and solve
 * of the context.  x0_dev: device [dim*N_x] reference node positions (SoA),
 * copied into the context on its stream (the caller may free it afterwards);
 * NULL removes the term.  coef >= 0 and delta > 0, else TMOP_ERR_INVALID_ARG.
 * The Jacobi diagonal is recomputed on its next use. */
int tmop_set_limiting(tmop_ctx *ctx, const double *x0_dev, double coef, double delta);

/* The per-iteration record of the context's last tmop_solve: copies
 * min(cap, entries) records into the host array out (newton_its + 1 entries
 * for a solve that ran) and sets *n to the number of entries (also when cap
 * is smaller).  out may be NULL when cap is 0.  Errors: INVALID_ARG. */
int tmop_solve_history(tmop_ctx *ctx, tmop_iter_record *out, int cap, int *n);

/* How the forward sum-factorized contractions (Sec. 3.2: the Jacobian at
 * the points from three 1D contractions with B and G) of the energy, gradient
 * and FP64 Hessian setup kernels run: TMOP_SWEEPS_PENCIL (default), one lane
 * per 1D line with the tables in scalar registers; or TMOP_SWEEPS_MFMA, each
 * contraction as 16 x 16 x 4 FP64 matrix-core products.  Same values up to
 * rounding order.  MFMA exists for hex classes with nq1d <= 5 (else
 * TMOP_ERR_UNSUPPORTED) and is not used while a limiting term is set; the
 * Hessian action and diagonal always use the pencil form.  Errors:
 * INVALID_ARG, UNSUPPORTED. */
int tmop_set_sweeps(tmop_ctx *ctx, int mode);

/* Enable (1) or disable (0) HIP-event timing of the Hessian actions inside
 * MINRES; results land in tmop_solve_report.t_apply_ms / n_apply. */
int tmop_set_timing(tmop_ctx *ctx, int enable);

/* ---------------------------------------------------------------------- */
/* No-allocation evaluation                                                */
/* ---------------------------------------------------------------------- */

/* Largest number of element tiles (workgroups of the energy kernel, each of
 * max(1, 256 / nq1d^dim) elements) tmop_energy_mindet_noalloc accepts. */
#define TMOP_NOALLOC_MAX_TILES 65536

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * energy and min det of tmop_energy_mindet without a context, with no device
 * or pinned allocation by the library.  The per-workgroup partial sums go to
 * a fixed 1.5 MiB device array of the library (3 x TMOP_NOALLOC_MAX_TILES
 * doubles; each GPU the library runs on holds its own copy until the process
 * ends).  m: a structured box (elem_to_node must be NULL, else
 * TMOP_ERR_UNSUPPORTED; ess fields ignored); prm: metric, nq1d, target and
 * quad_rule as for tmop_create (precision and storage ignored: the energy is
 * FP64).  x_dev: device [dim*N_x] nodes.  out_dev: caller-owned device
 * doubles [3]: out[0] = F (meaningless when out[2] > 0), out[1] = min det A
 * over all quadrature points, out[2] = number of points with det A <= 0.
 * Asynchronous on hip_stream (NULL: the null stream); out_dev is ready when
 * the stream reaches the call.  A box whose elements fill more than
 * TMOP_NOALLOC_MAX_TILES tiles returns TMOP_ERR_INVALID_ARG.  Every call on
 * one GPU shares that GPU's array (the partials are written in full before
 * they are read, so nothing needs clearing): calls that overlap in time on
 * one GPU (different streams or host threads) race and must be ordered by
 * the caller.  The result is bitwise that of tmop_energy_mindet for the same
 * mesh and parameters. */
int tmop_energy_mindet_noalloc(const tmop_mesh_desc *m, const tmop_params *prm,
                               const double *x_dev, double *out_dev, void *hip_stream);

/* Thread-local description of the last error. */
const char *tmop_last_error(void);

/* Library version string. */
const char *tmop_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TMOP_H */
