/*
 * bhem_shell.h -- C ABI of the MI355X (gfx950) BHEM thin-shell library.
 *
 * The library evaluates the Kirchhoff-Love thin-shell model discretised by
 * bicubic Hermite patches (Ni et al., "Simulating Parametric Thin Shells by
 * Bicubic Hermite Elements", arXiv 2312.14839) and advances it by one
 * implicit-Euler step:
 *   - per-patch 4x4 Gauss quadrature of the StVK membrane + bending energy,
 *     its gradient and its exact (or pseudo) Hessian (Sec. 3.3, Appendix B);
 *   - assembly of those Hessians, the consistent mass matrix (Eq. mass) and
 *     the areal gravity load into a 12x12-block sparse matrix;
 *   - Newton's method with a line search on the incremental potential of the
 *     implicit Euler scheme (Sec. 6.1), whose linear systems are solved by a
 *     block-Jacobi preconditioned conjugate gradient on the GPU.
 *
 * Conventions shared by every entry point
 *   Generalized coordinates.  Each node stores x, dx/dxi1, dx/dxi2 and
 *   d2x/dxi1dxi2 (Sec. 4.1), i.e. 12 doubles per node, ordered
 *   [3*kind + component]; arrays of nodal values are [nodes][12] row-major
 *   float64.  Derivative coordinates are derivatives with respect to xi, not
 *   to the per-cell parameter theta.
 *   Grids.  Shell s is an n1 x n2 grid of patches; node (i, j) has index
 *   j*(n1+1) + i, or j*n1 + (i mod n1) when periodic1 is set (the node column
 *   at xi1 = n1 dxi1 is the column at 0, Sec. 4.2 "Periodic boundary
 *   conditions").  With several shells the node arrays are concatenated in
 *   the order of the descriptors.
 *   Memory.  Pointers whose name ends in _dev are device pointers valid on the
 *   context's stream; _host are host pointers.  The caller owns every pointer
 *   it passes; the library copies what it needs during shell_create and keeps
 *   no caller pointer.  All device work is ordered on the context's stream.
 *   Calls that return host values synchronise that stream before returning.
 *   Errors.  Every call returns a shell_status (0 = success, < 0 = error);
 *   no exception crosses the ABI.  shell_last_error() describes the last
 *   error of a context.  SHELL_E_DEVICE means a HIP call failed; destroy the
 *   context afterwards.  A context is not thread safe: use one per stream.
 */
#ifndef BHEM_SHELL_H
#define BHEM_SHELL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct shell_ctx shell_ctx;
typedef int32_t shell_status;

enum {
    SHELL_OK = 0,
    SHELL_E_INVAL = -1,          /* invalid argument; the context is unchanged */
    SHELL_E_NOMEM = -2,          /* device allocation failed */
    SHELL_E_DEVICE = -3,         /* a HIP runtime call failed */
    SHELL_E_NOT_CONVERGED = -4,  /* Newton or CG iteration cap; outputs hold the last iterate */
    SHELL_E_INDEFINITE = -5,     /* regulariser reached its cap without a positive definite system */
    SHELL_E_NONFINITE = -6,      /* non-finite input or result */
    SHELL_E_LINESEARCH = -7      /* no step along the Newton direction lowered the energy */
};

enum { SHELL_FP64 = 0, SHELL_MIXED = 1 };             /* Hessian/SpMV precision */
enum { SHELL_HESS_EXACT = 0, SHELL_HESS_PSEUDO = 1 };  /* Appendix B.2, last paragraph */
enum { SHELL_WS_NONE = 0, SHELL_WS_MLP = 1 };          /* initial Newton iterate of each step */

/* One shell (Sec. 4.1-4.2; material of Sec. 3.3; loads of Sec. 4.3). */
typedef struct {
    int32_t n1, n2;              /* patches along xi1 and xi2, each >= 1 */
    int32_t periodic1;           /* 1: node column n1 is node column 0 (needs n1 >= 3) */
    double dxi1, dxi2;           /* parameter cell size, > 0 */
    const double *ref_host;      /* [nodes][12] reference (rest) generalized coordinates */
    const uint8_t *fixed_host;   /* [nodes][12], 1 = prescribed DOF (Sec. 4.2); NULL = none */
    double young, poisson;       /* Y > 0, 0 <= nu < 0.5; lambda = Y nu/(1 - nu^2), mu = Y/(2(1 + nu)) */
    double thickness, density;   /* h > 0, rho > 0 */
    double gravity[3];           /* areal dead load rho h g (Sec. 4.3, "External Forces") */
    double damping;              /* mass-proportional Rayleigh coefficient alpha >= 0 [1/s]: damping
                                    force -alpha M qdot in the Newton steps (Table 2 lists a Rayleigh
                                    coefficient without its form; this is the mass-proportional reading) */
} shell_desc;

typedef struct {
    int32_t precision;           /* SHELL_FP64 or SHELL_MIXED (FP32 Hessian, matrix and inner CG;
                                    FP64 gradient, residual, refinement and block inverses) */
    int32_t hessian;             /* SHELL_HESS_EXACT or SHELL_HESS_PSEUDO */
    int32_t warm_start;          /* SHELL_WS_NONE or SHELL_WS_MLP (needs shell_mlp_set_params first) */
    int32_t newton_maxit;        /* > 0 */
    int32_t pcg_maxit;           /* > 0, per linear solve */
    double newton_rtol;          /* Newton stops at ||g|| <= max(newton_rtol ||g_0||, rounding floor) */
    double pcg_rtol;             /* CG stops at ||b - A x|| <= pcg_rtol ||b|| (FP64 residual) */
    int32_t device;              /* HIP device ordinal */
    void *stream;                /* hipStream_t, NULL = the default stream */
    int32_t graphs;              /* 1: the fixed launch sequences of a Newton iteration (assembly and
                                    factorisation, CG, line-search trial, rounding floor) run as HIP
                                    graphs captured once per context and time-step size; 0: direct
                                    launches.  Off while event timing is on. */
    int32_t cg_resident;         /* 1: where a CG block has few enough row passes, the solver keeps
                                    its own rows' residual, solution and product in registers
                                    instead of device memory; 0: always in device memory (same
                                    arithmetic, for comparison) */
    int32_t device_newton;       /* 1: each Newton iteration (Sec. 6.1) is one launch sequence, a
                                    single HIP graph when graphs is on: assembly, factorisation, the
                                    CG (mixed form: up to 2 refinement sweeps), the slope, up to 2
                                    line-search trials and the next convergence test, every decision
                                    taken on the device per shell; the host reads the shells' state
                                    once per iteration and finishes only a shell that needs the
                                    regulariser, more sweeps or more trials, with the same arithmetic
                                    as the host-driven iteration (0).  Not with point constraints or
                                    event timing on, which use the host-driven iteration.  The
                                    iteration's time counts as t_pcg_ms. */
} shell_opts;

/* Per-shell statistics of one shell_newton_step. */
typedef struct {
    int32_t status;              /* shell_status of this shell */
    int32_t newton_iters;        /* Newton iterations taken */
    int32_t pcg_iters_total;     /* CG iterations over all Newton iterations */
    int32_t ls_backtracks;       /* rejected line-search trials */
    int32_t refine_sweeps;       /* FP64 refinement sweeps (mixed precision) */
    int32_t warm_start_used;     /* 1 if the Newton iteration started from the learned guess */
    double grad_norm0, grad_norm, grad_floor, reg_delta;
    double t_assemble_ms, t_pcg_ms, t_step_ms;   /* whole-context wall times */
    double alm_residual;         /* max |c| over this shell's point constraints at the last check */
    int32_t alm_outer;           /* multiplier updates taken (shell_set_point_constraints) */
} shell_step_stats;

/* Default options: FP64, exact Hessian, no warm start, newton_rtol = pcg_rtol
 * = 1e-10, 50 Newton and 100000 CG iterations, device 0, default stream,
 * graphs on, register-resident CG vectors on, device-driven Newton
 * iterations on. */
void shell_default_opts(shell_opts *o);

/* Create a context for n_shells shells (batching: one context holds all of
 * them, concatenated).  Copies the descriptors' arrays, builds the patch
 * colouring and the 12x12-block sparsity pattern (Sec. 4.3, "Properties of
 * the mass matrix": blocks couple nodes that share a patch) and allocates all
 * device memory.  On error *out is NULL and shell_last_error(NULL) tells why. */
shell_status shell_create(const shell_desc *shells, int32_t n_shells, const shell_opts *o, shell_ctx **out);

/* Destroy a context and free its device memory.  NULL is allowed. */
void shell_destroy(shell_ctx *c);

/* Message of the last error of c (of the last failed create if c is NULL). */
const char *shell_last_error(const shell_ctx *c);

/* Sizes: total nodes, total patches, and block non-zeros of the full matrix
 * (both triangles; the device stores the diagonal and upper-triangle blocks,
 * (nnzb + total_nodes) / 2 of them). */
shell_status shell_sizes(const shell_ctx *c, int32_t *total_nodes, int32_t *total_patches, int64_t *nnzb);

/* Elastic energy V_e of every shell at q (Sec. 3.3 energy density integrated
 * by the 16-point rule of Appendix A.2), its gradient (Appendix B.1,
 * Eq. matrix) and, if assemble_hessian != 0, its Hessian (Appendix B.2,
 * exact or pseudo per the options) assembled into the context's matrix.
 *   q_dev        [total_nodes][12] generalized coordinates
 *   energy_host  [n_shells] or NULL
 *   grad_dev     [total_nodes][12] or NULL; no constraint is applied
 * Returns SHELL_E_NONFINITE if an energy is not finite. */
shell_status shell_energy_grad_hess(shell_ctx *c, const double *q_dev, double *energy_host, double *grad_dev,
                                    int32_t assemble_hessian);

/* Assemble K(q) + mass_scale * M into the context's matrix (M of Eq. mass;
 * K the elastic Hessian; elastic = 0 drops K, giving mass_scale * M). */
shell_status shell_assemble(shell_ctx *c, const double *q_dev, double mass_scale, int32_t elastic);

/* Copy shell s's part of the context's matrix to the host as BSR with local
 * node indices: row_ptr[nodes_s + 1], col_idx[nnzb_s], vals[nnzb_s][12][12]
 * (FP64 even in mixed precision).  Call with NULL arrays to get *nnzb only.
 * The device keeps the diagonal and upper-triangle blocks only (the Hessian
 * is symmetric); the full pattern is returned, each block below the
 * diagonal the transpose of its mirror image: exactly the matrix that
 * shell_spmv and the CG apply. */
shell_status shell_get_bsr(shell_ctx *c, int32_t shell, int32_t *nnzb, int32_t *row_ptr, int32_t *col_idx,
                           double *vals);

/* y = A x with the context's matrix; rows and columns of prescribed DOFs are
 * left out when masked != 0 (y is 0 there).  FP64 vectors. */
shell_status shell_spmv(shell_ctx *c, const double *x_dev, double *y_dev, int32_t masked);

/* Solve A x = b (prescribed DOFs masked out; b must be 0 there) with the
 * block-Jacobi CG at the options' precision, from x = 0.  iters_host and
 * relres_host ([n_shells] each, may be NULL) receive per-shell counts and
 * final ||b - A x|| / ||b|| (FP64).  SHELL_E_INDEFINITE if a diagonal block
 * or p^T A p is not positive. */
shell_status shell_pcg_solve(shell_ctx *c, const double *b_dev, double *x_dev, double rtol, int32_t maxit,
                             int32_t *iters_host, double *relres_host);

/* One implicit-Euler step of every shell (Sec. 6.1): minimise
 *   E(q) = (1/2 dt^2)(q - qhat)^T M (q - qhat) + V_e(q) - f^T (q - qhat),
 *   qhat = q_n + dt v_n,
 * over the free DOFs, prescribed DOFs held at q_presc (or q_n if NULL);
 * then v_{n+1} = (q_{n+1} - q_n)/dt.  Newton with a backtracking line
 * search (quadratic, then cubic interpolation); block-Jacobi CG for the
 * Newton systems; diagonal regulariser A + delta diag(A), delta = 1e-6..1e2,
 * when a block or p^T A p is not positive (Sec. 6.1, "The Hessian matrix").
 *   q_n_dev, v_n_dev, q_presc_dev  [total_nodes][12]
 *   q_np1_dev, v_np1_dev           [total_nodes][12] outputs (may not alias inputs)
 *   stats_host                     [n_shells] or NULL
 * Returns the worst shell status. */
shell_status shell_newton_step(shell_ctx *c, double dt, const double *q_n_dev, const double *v_n_dev,
                               const double *q_presc_dev, double *q_np1_dev, double *v_np1_dev,
                               shell_step_stats *stats_host);

/* External nodal generalized forces f_dev[total_nodes][12] (device, copied;
 * NULL clears them), added to the areal gravity load of every later
 * shell_newton_step: the incremental potential gains -f^T (q - qhat).  On
 * prescribed DOFs they have no effect.  A point force at a parameter point
 * is the vector shell_point_load builds (Sec. 4.3, "External Forces"). */
shell_status shell_set_nodal_forces(shell_ctx *c, const double *f_dev);

/* Pressure on each shell (Sec. 4.3, "External Forces", f = p n):
 * pressure_host[n_shells] in Pa, per unit current area along the normal
 * a_1 x a_2 / |a_1 x a_2| of the parametrisation (positive inflates a
 * cylinder whose xi1 runs around its axis counter-clockwise and xi2 along
 * it); NULL or all zero removes it.  A follower load: in shell_newton_step
 * it is evaluated at the step's start, F_I = p sum_gp w Phi^I (a_1 x a_2)(q_n),
 * and acts as a dead load within the step (added to the nodal forces), so
 * every Newton system stays symmetric; its load stiffness, which is not
 * symmetric, is not used.  A non-finite pressure is rejected with
 * SHELL_E_INVAL. */
shell_status shell_set_pressure(shell_ctx *c, const double *pressure_host);

/* The nodal generalized forces of the context's pressures at state q_dev:
 * f_dev[total_nodes][12] (device), unmasked.  Enqueued on the context's
 * stream. */
shell_status shell_pressure_load(shell_ctx *c, const double *q_dev, double *f_dev);

/* Positional constraint at a midsurface point (Sec. 4.2: the position or a
 * tangent of the midsurface prescribed at an arbitrary parameter point, not
 * only at a node), imposed in shell_newton_step by the augmented Lagrangian
 * method (Sec. 6.1): with c = x^(kind)(xi) - target (3 rows per constraint,
 * linear in q) each Newton solve minimises the incremental potential plus
 * -lambda.c + (penalty/2)|c|^2; when it has converged and max |c| over a
 * shell's constraints exceeds tol, that shell's multipliers are updated,
 * lambda <- lambda - penalty c, and its Newton iteration resumes (at least
 * one more iteration, newton_maxit again, the convergence test relative to
 * the step's initial gradient), at most max_outer times (then
 * SHELL_E_NOT_CONVERGED).  At the result lambda is the constraint force:
 * grad of the incremental potential = C^T lambda. */
typedef struct {
    int32_t shell;               /* shell index */
    int32_t kind;                /* 0: x, 1: x_xi1, 2: x_xi2 at the point */
    double xi1, xi2;             /* parameter coordinates, in [0, n1 dxi1] x [0, n2 dxi2] (xi1 modulo
                                    n1 dxi1 on a periodic shell), patch as shell_point_load */
    double target[3];
} shell_point_constraint;

typedef struct {
    double penalty;              /* > 0, the coefficient of (1/2)|c|^2 */
    double tol;                  /* > 0, max |c| at which a shell's outer iteration stops */
    int32_t max_outer;           /* >= 0, multiplier updates per step at most */
} shell_alm_opts;

/* Set the point constraints of the context (n = 0 or pts NULL removes
 * them) and zero their multipliers.  Constraints on prescribed DOFs act
 * on the free DOFs only.  SHELL_E_INVAL for a shell index, kind or point
 * out of range, a non-finite target or invalid options.  Takes effect in
 * the next shell_newton_step; shell_energy_grad_hess, shell_assemble and
 * the other building blocks do not include them. */
shell_status shell_set_point_constraints(shell_ctx *c, const shell_point_constraint *pts, int32_t n,
                                         const shell_alm_opts *o);

/* Multipliers lambda_host[n][3] of the constraints in the order they were
 * set: after a step, its constraint forces; kept as the next step's start
 * (shell_set_point_multipliers replaces them, e.g. after moving targets). */
shell_status shell_get_point_multipliers(const shell_ctx *c, double *lambda_host);
shell_status shell_set_point_multipliers(shell_ctx *c, const double *lambda_host);

/* Consistent nodal load of a point force: adds Phi^I(xi) force into the
 * host array f_nodal[nodes of this shell][12] for the 16 shape functions of
 * the patch containing (xi1, xi2) (parameter coordinates in [0, n1 dxi1] x
 * [0, n2 dxi2]; xi1 taken modulo n1 dxi1 for a periodic shell), so that
 * f_nodal . q equals force . x(xi) for every state q.  Needs no context. */
shell_status shell_point_load(const shell_desc *d, double xi1, double xi2, const double *force, double *f_nodal);

/* Device-time accounting per kernel group, measured with HIP events on the
 * context's stream (adds a stream synchronisation after each timed launch,
 * so enable it only to measure). */
enum {
    SHELL_T_ENERGY_GRAD = 0,   /* patch energy + gradient kernels (and their reductions) */
    SHELL_T_HESSIAN = 1,       /* patch Hessian + colour scatter kernels (all colours) */
    SHELL_T_BJ = 2,            /* block-Jacobi factorisation */
    SHELL_T_CG = 3,            /* persistent CG kernel */
    SHELL_T_SPMV = 4,          /* stand-alone SpMV / residual kernels */
    SHELL_T_NGROUPS = 5
};
typedef struct {
    double ms[SHELL_T_NGROUPS];          /* accumulated device milliseconds */
    int64_t launches[SHELL_T_NGROUPS];   /* timed launches (a group of colour passes counts once) */
    int64_t patch_evals;                 /* patches through the Hessian kernel */
    int64_t cg_iter_rows;                /* sum over CG launches and shells of iterations x node rows */
    int64_t cg_iter_blocks;              /* same with block non-zeros */
    int64_t cg_iters_max;                /* sum over CG launches of the largest shell iteration count */
} shell_timing;

/* Reset the counters and turn event timing on (enable != 0) or off. */
shell_status shell_timing_enable(shell_ctx *c, int32_t enable);
/* Copy the counters accumulated since the last shell_timing_enable. */
shell_status shell_timing_get(const shell_ctx *c, shell_timing *out);

/* Phase trace of the persistent CG (enable != 0: on).  While on, every CG
 * launch records, for each of its blocks (a block owns contiguous node rows
 * of one shell) and each of its first 64 iterations, six timestamps of the
 * GPU's constant 100 MHz clock taken by the block's first thread: the
 * iteration's start, the end of the update phase (own rows: vectors and
 * preconditioner), the end of the wait for the neighbouring blocks, the end
 * of its own share of the product phase, its arrival at the iteration's
 * reduce-barrier (every wavefront of the block done and its partial sums
 * published; 0 for a shell held by one block, which needs no grid barrier)
 * and the barrier's exit.  Results are unchanged by tracing. */
shell_status shell_cg_trace_enable(shell_ctx *c, int32_t enable);
/* The last CG launch's trace: *nblocks blocks x *iters iterations x 6
 * timestamps into ts_host (host, [nblocks][iters][6], may be NULL to query
 * the sizes; zeros where an iteration was not reached or tracing is off). */
shell_status shell_cg_trace_get(shell_ctx *c, int32_t *nblocks, int32_t *iters, uint64_t *ts_host);

/* Autotuner of the batched form's launch shapes.  CG layout: the persistent
 * CG kernel covers each shell's node rows with contiguous row blocks; the
 * tunable layout is the threads per block (256, 512 or 1024) and the rows
 * per block (the fewest that keep every block resident at once, or 1, 2 or
 * 4 times that rounded up to the rows one pass of a block covers, or one
 * block per shell where a block covers the largest shell in two passes).
 * shell_autotune times cg_iters CG iterations of every candidate on K(qbar)
 * + M (overwriting the context's matrix) and keeps the fastest.  Patch
 * kernel tiles: the patches (wavefronts) per block of the Hessian kernel
 * (4 or 8) and the patches per block of the energy and gradient
 * kernel (4, 8 or 16, 16 threads each), each chosen by the wall time of one
 * assembly / one evaluation at qbar.  Results are cached for the process by
 * (device, nodes, shells, block non-zeros, precision); a cached choice is
 * applied without timing the candidates (candidates = 0, from_cache = 1).
 * Times are wall-clock microseconds: per CG iteration, per assembly, per
 * evaluation. */
typedef struct {
    int32_t threads, rows_per_block, blocks;   /* chosen layout */
    int32_t default_threads, default_rows_per_block;   /* layout before the call */
    int32_t candidates, from_cache;
    double us_per_iter, us_per_iter_default;
    int32_t hess_waves, energy_patches;        /* chosen patch kernel tiles */
    double hess_us, hess_us_default, energy_us, energy_us_default;
} shell_tune_result;
shell_status shell_autotune(shell_ctx *c, int32_t cg_iters, shell_tune_result *out);

/* Set the patch kernel tiles by hand: hess_waves patches (wavefronts) per
 * block of the Hessian kernel (4 or 8), energy_patches patches per
 * block of the energy and gradient kernel (4, 8 or 16).  Results do not
 * depend on them (each patch is computed by one wavefront or 16 lanes, and
 * patches of one colour share no matrix block).  SHELL_E_INVAL otherwise. */
shell_status shell_set_patch_tiles(shell_ctx *c, int32_t hess_waves, int32_t energy_patches);

/* Form of the Hessian assembly (Appendix B.2 scattered into the stored
 * triangle).  single_launch = 0: one launch per patch colour, each adding
 * its patches' blocks into the matrix (patches of one colour share no
 * block).  single_launch = 1: one launch over all patches writing their
 * stored local blocks to a scratch array of the context, then one that
 * sums each stored block's contributions in colour order -- the same
 * additions in the same order, so the same matrix bit for bit, with two
 * launches instead of one per colour.  It needs every patch's Hessian
 * block resident on the device at once (shells of up to a few thousand
 * patches); contexts that allow it start with it.  SHELL_E_INVAL where
 * single_launch = 1 is not allowed. */
shell_status shell_set_assembly(shell_ctx *c, int32_t single_launch);

/* ------------------------------------------------------------------
 * Learned warm start of the Newton iteration.  This is an extension: the
 * paper has no learned component.  Its conclusions note that positions and
 * their parametric derivatives carry different units (Sec. 8, "Loss
 * functions"); the features are therefore scaled per DOF kind.
 *
 * A per-node network 60 -> 128 -> 128 -> 12 (ReLU, ReLU, linear):
 *   h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), y = h2 W3 + b3,
 * products in bfloat16 (round to nearest even) with FP32 accumulation,
 * FP32 master parameters.  Parameter vector (float, row-major, this order):
 *   W1[60][128], b1[128], W2[128][128], b2[128], W3[128][12], b3[12].
 * Each step's Newton iteration starts at q_s (qhat = q_n + dt v_n on free
 * DOFs, prescribed values on the others) and ends at q_{n+1}; its
 * correction is D = q_{n+1} - q_s on free DOFs.  Features of node n of shell
 * s at the start of a step, for DOF kind k = w / 3 (x, x_1, x_2, x_12) of
 * the node's 12 DOFs w = 3k + component:
 *   x[w]      = (q_s - qbar)[n][w] / s_u[s][k]   (displacement from the reference)
 *   x[12 + w] = b[n][w] / s_b[s][k]             (b = -grad E(q_s), 0 on prescribed DOFs)
 *   x[24 + w] = Dprev[n][w] / s_d[s][k]          (the previous step's correction)
 *   x[36 + w] = (L b)[n][w] / s_b[s][k],  x[48 + w] = (L Dprev)[n][w] / s_d[s][k]
 * with s_*[s][k] the root mean square of that quantity over the free DOFs of
 * kind k of shell s (1 if it is zero), and L the node's 3x3 grid stencil
 * (L f)[n] = (4 sum of f over the four edge neighbours + sum over the four
 * diagonal ones) / 20 - f[n], a missing neighbour (an open edge) counted as
 * the node itself.  The network predicts the change of
 * the correction, w = s_d y on free DOFs.  The Newton iteration then starts
 * at q_s + c1 Dprev + c2 w, c the Galerkin solution of the quadratic model
 * of the incremental potential E in span{Dprev, w} (its Hessian from the
 * gradient differences grad E(q_s + d) - grad E(q_s), d = Dprev, w), if that
 * point satisfies the Armijo condition on E and at least halves
 * ||grad E|| (else the same is tried with Dprev alone).  Otherwise, for
 * shells whose previous step did not converge
 * (and at a context's first step), and where the network's output is not
 * finite, it starts at q_s exactly as without a warm start.
 * Convergence is still measured against ||grad E(q_s)||.
 * ------------------------------------------------------------------ */
#define SHELL_MLP_IN 60
#define SHELL_MLP_HIDDEN 128
#define SHELL_MLP_OUT 12
#define SHELL_MLP_PARAMS 25868

/* Load the network's parameters (theta_host: SHELL_MLP_PARAMS floats, host
 * memory, copied) and reset the Adam state.  Required before a step with
 * warm_start = SHELL_WS_MLP.  SHELL_E_NONFINITE for a non-finite value. */
shell_status shell_mlp_set_params(shell_ctx *c, const float *theta_host);

/* Copy the current parameters to theta_host (SHELL_MLP_PARAMS floats). */
shell_status shell_mlp_get_params(shell_ctx *c, float *theta_host);

/* Inference: out_dev[n][12] = y(feat_dev[n][60]), device arrays, n >= 0. */
shell_status shell_mlp_forward(shell_ctx *c, const float *feat_dev, float *out_dev, int64_t n);

/* Loss and gradient of one mini-batch: samples idx_dev[batch] (int64,
 * device, each in [0, n_samples), checked: SHELL_E_INVAL otherwise) of
 * feat_dev[n_samples][60] / tgt_dev[n_samples][12]; loss = mean over the
 * batch of sum_w (y_w - t_w)^2.  batch is a positive multiple of 32.
 * loss_host (1 double) and grad_host (SHELL_MLP_PARAMS floats) may be NULL.
 * The parameters are not changed. */
shell_status shell_mlp_loss_grad(shell_ctx *c, const float *feat_dev, const float *tgt_dev, int64_t n_samples,
                                 const int64_t *idx_dev, int32_t batch, double *loss_host, float *grad_host);

/* Train on n_samples device samples: steps Adam steps (beta 0.9, 0.999,
 * eps 1e-8, learning rate lr) on mini-batches of `batch` samples drawn with
 * replacement by a splitmix64 hash of (seed, step, i).  batch is a positive
 * multiple of 32.  loss_host ([steps] doubles or NULL) receives each step's
 * mini-batch loss before its update. */
shell_status shell_mlp_train(shell_ctx *c, const float *feat_dev, const float *tgt_dev, int64_t n_samples,
                             int32_t batch, int32_t steps, float lr, uint64_t seed, double *loss_host);

/* Record training samples during shell_newton_step: after each step,
 * per_shell nodes of every shell that converged and has a previous
 * correction (picked by a hash of seed, call and sample index) append their
 * features at the step's start (feat_dev[.][60]) and the target
 * t = (D - Dprev) / s_d (tgt_dev[.][12]), while capacity samples are not
 * exceeded.  The buffers are the caller's device memory and must outlive
 * the recording; feat_dev = NULL stops recording.  The sample count
 * restarts at 0. */
shell_status shell_mlp_record(shell_ctx *c, float *feat_dev, float *tgt_dev, int64_t capacity, int32_t per_shell,
                              uint64_t seed);

/* Samples recorded since the last shell_mlp_record. */
shell_status shell_mlp_recorded(const shell_ctx *c, int64_t *count);

/* ------------------------------------------------- collision handling
 * Sec. 6.2 ("Collision Handling") for colliders of simple shape: the shell
 * midsurface is sampled uniformly and every sample tested against the
 * colliders; the step is rolled back to the earliest contact; impulses with
 * zero restitution (and Coulomb friction) on the earliest simultaneous
 * contacts, each a linear constraint on the generalized velocities, solved
 * together in the least-squares sense; then every resolved contact point is
 * pushed a small distance off the collider, a constraint on the generalized
 * positions solved the same way. */
enum { SHELL_COLLIDER_PLANE = 0, SHELL_COLLIDER_SPHERE = 1 };

typedef struct {
    int32_t kind;                /* SHELL_COLLIDER_PLANE or SHELL_COLLIDER_SPHERE; static */
    double point[3];             /* plane: a point of it; sphere: its centre */
    double normal[3];            /* plane: its normal (normalised by the call); the shell stays on the side it
                                    points to */
    double radius;               /* sphere: radius > 0; the shell stays outside */
} shell_collider;

typedef struct {
    int32_t samples;             /* s: each patch sampled at the s x s parameter points ((a + 1/2)/s, (b + 1/2)/s);
                                    1..16 */
    double friction;             /* Coulomb coefficient mu >= 0 (0: frictionless) */
    double push_out;             /* distance each resolved contact point is moved off its collider (1e-4 m) */
    double simultaneous;         /* contacts within simultaneous * dt of the earliest are resolved together */
    double rtol;                 /* relative residual of the constraint solves */
} shell_collide_opts;

typedef struct {
    double t_contact;            /* time of the earliest contact after the step's start; +inf: none */
    int32_t contacts;            /* resolved contacts (pushed out) */
    int32_t approaching;         /* of those, the ones moving into their collider (impulses) */
    int32_t impulse_iters;       /* CG iterations on J M^-1 J^T of the velocity constraints */
    int32_t push_iters;          /* the same for the position constraints */
} shell_collide_stats;

/* samples 3, friction 0, push_out 1e-4, simultaneous 1e-3, rtol 1e-12. */
void shell_collide_default_opts(shell_collide_opts *o);

/* One collision pass after an implicit step from q_n to q_np1 with velocity
 * v (= (q_np1 - q_n)/dt, e.g. from shell_newton_step) of every shell of the
 * context:
 *   1. each sample moves on a straight line over the step (the generalized
 *      coordinates move linearly); its contact time is the earliest tau in
 *      [0, dt] at which it reaches a collider (0 if it starts inside);
 *   2. tau_min = the earliest; the state is rolled back to
 *      q_r = q_n + (tau_min / dt)(q_np1 - q_n), the velocity kept;
 *   3. the samples with contact times <= tau_min + simultaneous * dt are the
 *      contacts, each with the collider's normal n at its point;
 *   4. on those moving into their collider (n . v(xi) < 0): constraints
 *      n . v(xi) = 0 (friction > 0: also the tangential velocity 0), with
 *      v(xi) = sum_I Phi^I(xi) qdot_I; dqdot = M^-1 J^T lambda, lambda the
 *      minimum-norm solution of (J M^-1 J^T) lambda = -J qdot (M the
 *      consistent mass matrix, Eq. mass; prescribed DOFs do not move); with
 *      friction each tangential impulse is then scaled into the cone
 *      |lambda_t| <= friction * lambda_n (0 if lambda_n <= 0);
 *   5. for every contact the position constraint n . (x(xi) - p) = push_out
 *      (p its point on the collider), solved the same way: dq = M^-1 J^T mu.
 * Outputs: q_out = q_r + dq, v_out = v + dqdot, and the stats (t_contact: the
 * step has advanced by tau_min, which the caller takes as the step's length).
 * Without a contact q_out = q_np1, v_out = v, t_contact = +inf.
 *   q_n_dev, q_np1_dev, v_dev, q_out_dev, v_out_dev  [total_nodes][12];
 *   outputs may not alias inputs; colliders_host: n_colliders (host, copied);
 *   opts NULL: the defaults.
 * Overwrites the context's matrix with the mass matrix (the next Newton
 * step assembles its own); SHELL_E_INVAL for invalid colliders or options. */
shell_status shell_collide(shell_ctx *c, double dt, const double *q_n_dev, const double *q_np1_dev,
                           const double *v_dev, const shell_collider *colliders_host, int32_t n_colliders,
                           const shell_collide_opts *opts, double *q_out_dev, double *v_out_dev,
                           shell_collide_stats *stats_host);

/* ---------------------------------------------- ray--patch intersection
 * Sec. 5: a bicubic Hermite patch is a bicubic Bezier surface, whose
 * control-point bounding boxes bound it (convex-hull property); Sec. 5.1
 * finds the closest intersection of a ray with a set of such surfaces. */

/* Bezier control points of every patch of the context at state q_dev
 * [total_nodes][12] (Sec. 5, the Bernstein form of the patch).
 * ctrl_dev [total_patches][4][4][3] float64: p_ij of patch p at
 * ((4p + i)*4 + j)*3, i along xi1 (local parameter u in [0, 1]), j along xi2
 * (v); patch (pi, pj) of shell s is patch_begin(s) + pj*n1 + pi, shells in
 * descriptor order.  Enqueued on the context's stream. */
shell_status shell_bezier(shell_ctx *c, const double *q_dev, double *ctrl_dev);

#define SHELL_RAY_HEAP_MAX 64

typedef struct {
    double eps;            /* a candidate whose control-point box has a diagonal <= eps |d| is an answer;
                              its tau interval is then narrower than eps (tau in units of |d|); > 0 */
    double newton_tol;     /* Newton converged when |x(u,v) - x0 - tau d| <= newton_tol (length); > 0 */
    double hole;           /* half-width of the box abandoned around a Newton hit, as a fraction of the
                              candidate rectangle's width in each direction (Fig. subany); in (0, 0.5) */
    int32_t newton_iters;  /* 0: midpoint subdivision only, the first answer popped is the result;
                              1..64: Newton's method from each candidate's centre, at most this many steps */
    int32_t max_depth;     /* subdivision depth at which a candidate is an answer whatever its size; 1..60 */
    int32_t heap_cap;      /* candidates one ray may hold; 1..SHELL_RAY_HEAP_MAX */
    int32_t device;        /* HIP device */
    void *stream;          /* hipStream_t; NULL = the null stream */
} shell_ray_opts;

/* eps 1e-10, newton_tol 1e-12, hole 1e-3, newton_iters 8, max_depth 60,
 * heap_cap SHELL_RAY_HEAP_MAX, device 0, stream NULL. */
void shell_ray_default_opts(shell_ray_opts *o);

/* Static ray--patch intersection (Sec. 5.1): for each ray x0 + tau d the
 * smallest tau >= 0 at which it meets one of the n_patches Bezier patches,
 * by subdivision of the patches with a min-heap of candidate rectangles
 * keyed by the tau at which the ray enters their control-point box
 * (Eq. ineqray), optionally accelerated by Newton's method.
 *   ctrl_dev  [n_patches][4][4][3], e.g. written by shell_bezier (any
 *             Bezier patches in that layout); n_patches >= 0, < 2^24.
 *   rays_dev  [n_rays][6] float64: origin xyz, direction xyz.
 *   hit_dev   [n_rays][3] float64 out: tau, u, v of the closest hit in the
 *             patch's own parameters; tau = +inf when there is none.
 *   patch_dev [n_rays] int32 out: the hit's patch, -1 for a miss, -2 when
 *             there is no result: more root candidates than heap_cap, or
 *             the cooperative search (which takes over a ray after 512
 *             candidates or when its heap of heap_cap nears full, with room
 *             for 2,048 candidates and 16,384 rays per call) ran out of room,
 *             or 2^18 candidates examined; -3 for an invalid ray (zero or
 *             non-finite direction, non-finite origin).
 *   pops_dev  [n_rays] int32 out, or NULL: candidates the ray examined.
 * Device pointers valid on opts->stream; the caller owns them.  Enqueued on
 * that stream; no synchronisation.  Cost per ray is linear in n_patches
 * (every patch's box is tested; there is no scene hierarchy).  Invalid
 * sizes or options return SHELL_E_INVAL before anything is enqueued, a
 * failed launch SHELL_E_DEVICE; shell_last_error(NULL) describes both. */
shell_status shell_ray_cast(const double *ctrl_dev, int32_t n_patches, const double *rays_dev, int64_t n_rays,
                            const shell_ray_opts *opts, double *hit_dev, int32_t *patch_dev, int32_t *pops_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * search as shell_ray_cast, with the same arguments, validation and
 * results, except that rays go to the cooperative search through a fixed
 * device buffer of the library instead of a per-call stream-ordered
 * allocation.  The call allocates and frees nothing.
 *   The buffer holds SHELL_RAY_NOALLOC_TAIL_RAYS handed-over rays (about
 *   15 MiB of device memory, held on every device the library runs on until
 *   the process ends); no input size is rejected for it: rays that find it
 *   full report -2, as shell_ray_cast's do past its 16,384.  Its counter is
 *   cleared by a kernel on opts->stream at the start of each call.
 *   Every call on one device shares that device's buffer: calls that
 *   overlap on one GPU (other streams, other threads) race and must be
 *   serialised by the caller. */
#define SHELL_RAY_NOALLOC_TAIL_RAYS 4096
shell_status shell_ray_cast_noalloc(const double *ctrl_dev, int32_t n_patches, const double *rays_dev,
                                    int64_t n_rays, const shell_ray_opts *opts, double *hit_dev,
                                    int32_t *patch_dev, int32_t *pops_dev);

/* Dynamic ray--patch intersection (Sec. 5.2): for each point moving as
 * x0 + t w over one step t in [0, dt], the earliest t at which it meets one
 * of the patches whose control points move as p + t v (Eq. ineqccd bounds
 * the times at which the point can be inside a candidate's box), by the
 * same subdivision search as shell_ray_cast with keys = earliest feasible
 * times.  Control-point velocities are shell_bezier of the nodal velocities
 * (the Bezier form is linear in the nodal values).
 *   ctrl_dev, vel_dev [n_patches][4][4][3]: control points at t = 0 and
 *             their velocities.
 *   points_dev [n_points][6]: x0 xyz, w xyz.
 *   hit_dev   [n_points][3] out: t, u, v of the first contact; t = +inf
 *             when there is none within the step.
 *   patch_dev, pops_dev: as for shell_ray_cast (-3: non-finite point).
 *   opts: as for shell_ray_cast, except that eps is a length: a candidate
 *         whose box at its earliest time has a diagonal <= eps is an answer
 *         (its earliest time and rectangle centre).
 * Same ownership, stream and error rules as shell_ray_cast; dt > 0. */
shell_status shell_ccd(const double *ctrl_dev, const double *vel_dev, int32_t n_patches, const double *points_dev,
                       int64_t n_points, double dt, const shell_ray_opts *opts, double *hit_dev, int32_t *patch_dev,
                       int32_t *pops_dev);

#ifdef __cplusplus
}
#endif

#endif /* BHEM_SHELL_H */
