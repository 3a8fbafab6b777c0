/*
 * stmg.h - C ABI of the MI355X hp space-time multigrid library.
 *
 * The library solves the slab system of the instationary Stokes equations
 * discretised with Q_{r+1}/P_r^disc elements in space and DG(k) in time
 * (Margenberg, Bause, Munch, arXiv 2502.09159: Problem "Discrete variational
 * problem", Sec. 2.2; algebraic form Eq. (InAlg), (DefDtauh), (GloSys) of
 * Sec. 3.2) with FGMRES preconditioned by one hp space-time multigrid V-cycle
 * (Alg. 1 of Sec. 4.3; transfers of App. A; cell Vanka smoother Eq. (vanka0),
 * (vanka) of Sec. 4.2).
 *
 * Conventions
 *  - Every function returns stmg_status (0 = ok, < 0 = error); no C++
 *    exception crosses the ABI.  stmg_last_error() returns a message for the
 *    last failing call on a context (owned by the context).
 *  - Vectors passed to compute calls are caller-owned DEVICE pointers to
 *    contiguous FP64 arrays in the layout of Eq. (DefX):
 *        X = (V_1, P_1, ..., V_N, P_N),  V_n = (V_n^1..V_n^{k+1}),
 *        P_n = (P_n^1..P_n^{k+1});
 *    V_n^a is component-major over the global Gauss-Lobatto velocity nodes
 *    (nn = n (r+1) + 1 per direction, x fastest), P_n^a is cell-major (cells
 *    x fastest) over the C(r+d, d) shifted-Legendre modes of each cell,
 *    ordered by total degree, then with the x exponent largest first.
 *    Dirichlet velocity dofs are part of the vector; the operator acts as
 *    the identity on them.
 *  - The caller must not free or resize vectors during a call.  All calls
 *    are synchronous: work is issued on the context's stream and completed
 *    before the call returns.  A context is used by one host thread at a
 *    time.
 *  - Level 0 is the finest level (the paper numbers levels coarsest first).
 *  - The context owns all setup data (geometry, smoother factors, coarse
 *    inverse, work vectors) and frees it in stmg_destroy.
 */
#ifndef STMG_H
#define STMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  STMG_OK = 0,
  STMG_EINVAL = -1,       /* bad argument: null pointer, unsupported r/k/d/N */
  STMG_ENOMEM = -2,       /* host or device allocation failed */
  STMG_EDEVICE = -3,      /* a HIP runtime call failed */
  STMG_ENOCONV = -4,      /* solve reached max_it before the tolerance */
  STMG_ESINGULAR = -5,    /* a local or coarse factorisation broke down */
  STMG_EUNSUPPORTED = -6  /* configuration the library does not support */
} stmg_status;

typedef struct stmg_ctx stmg_ctx;

typedef enum {
  STMG_FP64 = 0,        /* every level in FP64 */
  STMG_MIXED_FP32 = 1   /* V-cycle in FP32 inside FP64 FGMRES */
} stmg_precision;

typedef enum {
  STMG_VANKA_FACTORED = 0, /* local inverse applied in Schur-factored form */
  STMG_VANKA_DENSE = 1,    /* local inverse stored as one dense b x b block */
  STMG_VANKA_DECOUPLED = 2, /* the same local inverse, decoupled in time: one
                               spatial Stokes block per eigenvalue of the
                               temporal matrix */
  STMG_VANKA_AUTO = 3       /* per level, the faster of the two factored forms
                               on MI355X: decoupled on levels with at least 64
                               velocity nodes per cell, Schur-factored below
                               (default) */
} stmg_vanka_mode;

typedef enum {
  STMG_LOCAL_EXACT = 0,   /* the exact patch inverse of Eq. (vanka0) (default) */
  STMG_LOCAL_DIAGONAL = 1 /* diagonal Vanka, a cheaper smoother (the conclusion
                             of the paper asks for cheaper local solves): the
                             patch matrix with its spatial mass and stiffness
                             blocks replaced by their diagonals, the temporal
                             coupling and the divergence kept exact; applied
                             in the decoupled form (vanka_mode is ignored) */
} stmg_local_solver;

/* nu(x) callback: evaluate the viscosity at npts physical points xyz
 * (npts x dim, row-major) into nu_out (npts).  Called on the host during
 * stmg_setup only. */
typedef void (*stmg_nu_fn)(int npts, const double* xyz, double* nu_out, void* user);

typedef struct {
  int dim;               /* 2 or 3 */
  int n_cells_1d;        /* fine mesh: n^d cells on [0,1]^d, n = n_coarse_1d 2^j */
  int n_coarse_1d;       /* cells per direction of the coarsest h-level (>= 1) */
  double deform_amp;     /* vertices x_i += amp * prod_j sin(2 pi x_j) */
  int r, k;              /* velocity Q_{r+1}, pressure P_r^disc, DG(k) */
  int n_sub;             /* N subintervals of the slab */
  double tau;            /* uniform subinterval length */
  double nu;             /* constant viscosity (used when nu_fn == NULL) */
  stmg_nu_fn nu_fn;      /* optional nu(x) */
  void* nu_user;
  int r_min, k_min;      /* p-coarsening floors (>= 1 and >= 0) */
  int time_h_coarsening; /* 1: also coarsen the slab in time (N -> N/2) */
  int placement;         /* 0: Alg. 2 + Alg. 3 of Sec. 4.4 (temporal coarsening
                            on the coarsest levels); 1: halve r and k together
                            on the fine mesh first */
  int nu_pre, nu_post;   /* Vanka sweeps before/after the coarse correction */
  double omega;          /* Vanka relaxation */
  int precision;         /* stmg_precision */
  int vanka_mode;        /* stmg_vanka_mode */
  int local_solver;      /* stmg_local_solver */
  int device;            /* HIP device ordinal */
  void* stream;          /* hipStream_t to issue work on, or NULL (default) */
} stmg_params;

/* Fill p with the defaults (3D, n=4, r=1, k=1, N=2, tau=0.05, nu=1,
 * r_min=k_min=1, no temporal h-coarsening, placement 0, one pre/post sweep,
 * omega=0.8, FP64, automatic Vanka form, device 0, default stream). */
stmg_status stmg_default_params(stmg_params* p);

/* Build the level list of the hp hierarchy without touching a GPU
 * (Sec. 4.4: p before h, space before time, space-time coarsening at the
 * coarse end).  levels_out receives up to max_levels rows of
 * (n_cells_1d, r, k, n_sub); *n_levels the number of levels (finest first). */
stmg_status stmg_hierarchy(const stmg_params* p, int max_levels, int* levels_out, int* n_levels);

/* Set up all levels on the device: mesh hierarchy, geometry, temporal
 * matrices (Eq. (DefKMC)), cell-patch matrices and their FP64
 * factorisations (Eq. (vanka0)), transfer tables (App. A) and the bordered
 * coarse-level inverse.  *out receives a new context. */
stmg_status stmg_setup(const stmg_params* p, stmg_ctx** out);
stmg_status stmg_destroy(stmg_ctx* ctx);
const char* stmg_last_error(const stmg_ctx* ctx);

/* Execution options, for tests and tuning (they change the work split, not
 * the result beyond rounding order):
 *  STMG_OPT_APPLY_SUBINTERVALS: subintervals of a cell that one wave of the
 *    operator's cell kernel walks through, carrying the jump term of Eq.
 *    (InAlg) in registers (0 = automatic: all N unless the grid would not
 *    fill the chip; values are clamped to [1, N]);
 *  STMG_OPT_NET_CHUNK: space-time cells per inference chunk of the learned
 *    correction (0 = default 65536; at most 65536);
 *  STMG_OPT_APPLY_LOOP_ORDER: loop order of the operator's cell kernel on 3D
 *    FP32 levels (0 = automatic: components outer; 1 = components outer, one
 *    component's geometry live at a time; 2 = components inner, the pressure
 *    and continuity rows shared by the components).
 *  STMG_OPT_INJECT_NONFINITE: test hook; a value v >= 1 overwrites the
 *    output of the v-th preconditioner application of every following
 *    stmg_solve with NaN (as an FP32 overflow in the V-cycle would leave it),
 *    to exercise the fallback described at stmg_solve; 0 = off.
 * Returns STMG_EINVAL for an unknown option or value. */
typedef enum {
  STMG_OPT_APPLY_SUBINTERVALS = 1,
  STMG_OPT_NET_CHUNK = 2,
  STMG_OPT_APPLY_LOOP_ORDER = 3,
  STMG_OPT_INJECT_NONFINITE = 4
} stmg_option;
stmg_status stmg_set_option(stmg_ctx* ctx, int option, int64_t value);

/* Record per-phase device times (smoother, rest of the V-cycle, outer
 * operator applies, other) in stmg_solve_info; adds event overhead. */
stmg_status stmg_set_phase_timing(stmg_ctx* ctx, int on);

/* Sizes of a level: total dofs, velocity dofs per slice, pressure dofs per
 * slice; *n_levels receives the number of levels. */
stmg_status stmg_sizes(const stmg_ctx* ctx, int level, int64_t* n_dofs, int64_t* n_vel_space,
                       int64_t* n_p_space, int* n_levels);

/* y = S_level x (Eq. (GloSys) on that level), FP64.  x and y must not alias. */
stmg_status stmg_apply_operator(stmg_ctx* ctx, int level, const double* x, double* y);

/* y = S_level x evaluated in the V-cycle's precision: in a mixed context x
 * is rounded to FP32, the FP32 operator of the V-cycle is applied and y is
 * widened back to FP64; in an FP64 context this equals stmg_apply_operator.
 * x and y are FP64 device vectors and must not alias. */
stmg_status stmg_apply_operator_vcycle_precision(stmg_ctx* ctx, int level, const double* x, double* y);

/* r = b - S_level x, FP64. */
stmg_status stmg_residual(stmg_ctx* ctx, int level, const double* b, const double* x, double* r);

/* `steps` cell Vanka iterations x <- x + omega D^{-1} sum_T R_T^T A_T^{-1} R_T (b - S x)
 * (Eq. (vanka) with valence weighting), FP64, x updated in place. */
stmg_status stmg_smooth(stmg_ctx* ctx, int level, const double* b, double* x, int steps);

/* x += omega D^{-1} sum_T R_T^T A_T^{-1} R_T r: the smoother's correction
 * step alone (the local solves of Eq. (vanka0) for a given residual r), in
 * the context's precision (inputs cast when the context is mixed). */
stmg_status stmg_vanka_correction(stmg_ctx* ctx, int level, const double* r, double* x);

/* Allocation-free variant of stmg_vanka_correction, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same correction, bit for bit, but the
 * smoother's scratch (the cell-local velocity corrections and, in a mixed
 * context, the FP32 copies of r and x) comes from a fixed device buffer of
 * STMG_NOALLOC_SCRATCH_BYTES bytes that the library holds on every GPU it
 * runs on until the process ends.  The call allocates nothing (the context
 * must exist already).  Returns STMG_EINVAL, with a message naming the size,
 * if the level needs more scratch than the buffer holds (about 64^3-node
 * levels of Q3 x DG(1) with 8 subintervals in FP32 need more).  Every call on
 * one GPU uses the same buffer: calls that overlap in time on one GPU (other
 * host threads or streams, any context) race, and the caller must serialise
 * them. */
#define STMG_NOALLOC_SCRATCH_BYTES (64u << 20)
stmg_status stmg_vanka_correction_noalloc(stmg_ctx* ctx, int level, const double* r, double* x);

/* Benchmark helper: run one kernel class `reps` times back to back on the
 * level's internal work vectors, in the context's precision (the V-cycle's),
 * on the context's stream, and return the mean device time of one
 * application in *avg_ms (HIP events).  which = 0: Vanka correction (local
 * solves and node gather); 1: operator residual b - S x (cell kernel and node
 * gather); 2: the Vanka local solves alone (factored smoother only); 3: the
 * operator's cell kernel alone.  The work vectors' contents are overwritten. */
stmg_status stmg_kernel_time(stmg_ctx* ctx, int which, int level, int reps, double* avg_ms);

/* coarse = P^T fine (restriction, App. A) from `level` to `level + 1`. */
stmg_status stmg_restrict(stmg_ctx* ctx, int level, const double* fine, double* coarse);

/* fine = P coarse (prolongation, App. A) from `level + 1` to `level`. */
stmg_status stmg_prolongate(stmg_ctx* ctx, int level, const double* coarse, double* fine);

/* x = exact solution on the coarsest level with per-slice mean-zero pressure
 * (bordered FP64 inverse; Alg. 1 step 3). */
stmg_status stmg_coarse_solve(stmg_ctx* ctx, const double* b, double* x);

/* x = V(b): one V-cycle from a zero initial guess on the finest level, in the
 * context's precision (Alg. 1 with Alg. 4-7). */
stmg_status stmg_vcycle(stmg_ctx* ctx, const double* b, double* x);

typedef struct {
  int iterations;          /* preconditioner applications */
  double rel_residual;     /* explicit ||b - S x|| / ||b|| at exit */
  double t_solve_s;        /* wall time of the solve (device events) */
  double t_smoother_s;     /* time in Vanka sweeps */
  double t_mg_other_s;     /* V-cycle minus smoothing (applies, transfers, coarse) */
  double t_operator_s;     /* FGMRES operator applies outside the V-cycle */
  double t_other_s;        /* orthogonalisation and the rest */
  int learned_disabled;    /* 1 if the learned correction was switched off */
  int history_len;
  const double* history;   /* residual estimates, owned by the context */
  int vcycle_fallbacks;    /* steps whose V-cycle output was not finite and
                              that were redone with the unpreconditioned
                              direction */
  int learned_steps;       /* learned corrections applied before the switch-off */
} stmg_solve_info;

/* FGMRES (right preconditioned by stmg_vcycle, CGS2, x0 = 0) on the finest
 * level until ||b - S x|| <= rtol ||b|| (explicitly rechecked), restarted
 * every STMG_RESTART iterations (fewer if device memory is short).  Returns
 * STMG_ENOCONV if max_it preconditioner applications were not enough (x then
 * holds the last iterate).  info may be NULL.  The returned x has mean-zero
 * pressure in every slice.  Failure handling: if a V-cycle returns a
 * non-finite direction (seen in the Gram-Schmidt coefficients that every
 * step reads back), that step is redone with z_j = the V-cycle's input (no
 * preconditioning for that step) and counted in info->vcycle_fallbacks; if
 * that is not finite either, STMG_ESINGULAR. */
#define STMG_RESTART 64
stmg_status stmg_solve(stmg_ctx* ctx, const double* b, double* x, double rtol, int max_it,
                       stmg_solve_info* info);

/* ------------------------------------------------------------------------
 * Time marching over slabs (Eq. (AlgSysTMS) of Sec. 3.2, with a slab of N
 * subintervals in place of one) with inhomogeneous Dirichlet data.  The
 * temporal dofs of a subinterval sit at the right Radau points t_a of DG(k)
 * (stmg_time_nodes), so the last one is the end value that the next slab's
 * jump term C^1 V_0 takes.  Dirichlet data are lifted: the library solves
 * S x0 = b with b = f - S_full gD - C^1 v0 on free rows and 0 on Dirichlet
 * rows (S_full keeps the Dirichlet columns; gD is g on Dirichlet velocity
 * entries, 0 elsewhere) and returns x = x0 + gD.
 * ------------------------------------------------------------------------ */

/* The k+1 reference Radau points t_a in (-1, 1] of the finest level's DG(k)
 * basis (t_hat: host array of k+1 values); temporal dof a of subinterval n
 * sits at t0 + tau (n + (t_a + 1) / 2). */
stmg_status stmg_time_nodes(const stmg_ctx* ctx, double* t_hat);

/* b = f - S_full gD - C^1 v0 on free velocity rows and pressure rows, 0 on
 * Dirichlet rows (device FP64 slab vectors; f may be NULL for zero forcing,
 * g NULL for homogeneous data; v0 is a device array of d x nodes velocity
 * values (one slice of V, component-major), NULL for v0 = 0). */
stmg_status stmg_slab_rhs(stmg_ctx* ctx, const double* f, const double* v0, const double* g, double* b);

/* v_end = the velocity of the last temporal dof of the last subinterval of
 * the slab vector x (d x nodes values, device). */
stmg_status stmg_slab_end_value(stmg_ctx* ctx, const double* x, double* v_end);

/* One slab of the time-marching scheme: b from stmg_slab_rhs, FGMRES as in
 * stmg_solve (tolerance relative to ||b||), then x = x0 + gD.  Returns what
 * stmg_solve returns. */
stmg_status stmg_solve_slab(stmg_ctx* ctx, const double* f, const double* v0, const double* g, double* x,
                            double rtol, int max_it, stmg_solve_info* info);

/* n_slabs slabs in a row: slab s solves with forcing f + s n_dofs (or 0),
 * Dirichlet data g + s n_dofs (or 0) and v0 = the end value of slab s - 1
 * (the given v0, or 0, for s = 0), into x + s n_dofs.  iterations (host,
 * n_slabs values, may be NULL) receives the FGMRES iterations per slab.
 * Stops at the first slab that fails (STMG_ENOCONV names it). */
stmg_status stmg_march(stmg_ctx* ctx, int n_slabs, const double* f, const double* g, const double* v0, double* x,
                       double rtol, int max_it, int* iterations);

/* x <- x with the L2 mean of the pressure removed in every slice (device
 * vector, finest level). */
stmg_status stmg_project_pressure_mean_zero(stmg_ctx* ctx, double* x);

/* ------------------------------------------------------------------------
 * Learned correction (an addition to the paper's method): after every Vanka
 * sweep on a 3D level with the Q2/P1 x DG(1) element, a 3-layer 3x3x3
 * convolutional network maps each space-time cell's residual (15 channels:
 * 6 velocity, 8 pressure broadcast, 1 Dirichlet mask; scaled by its 2-norm
 * s_T) to a correction (6 velocity channels at the nodes, 8 pressure values
 * averaged over the nodes; times s_T), summed over cells with the valence
 * weighting of the Vanka patches.  BF16 operands on the matrix cores, FP32
 * accumulation.  The correction c is added with the step alpha = <r, S c> /
 * <S c, S c> that minimises the level's residual 2-norm, so it cannot raise
 * it; if that step would remove less than 2% of |r|^2 (alpha <= 0 included)
 * the correction is skipped and the network is switched off for the rest of
 * the solve.  A level with another element whose next
 * coarser level has the network's element on the same mesh (e.g. the finest
 * Q3/P2 x DG(1) level above the Q2/P1 x DG(1) level) takes the correction
 * P c_coarse(P^T r) through that level: residual restricted, network
 * correction there, prolongated (App. A transfers), then the same step.
 * Weights: STMG_NET_PARAMS FP32 values, W1 (32x15x27), W2 (32x32x27),
 * W3 (14x32x27), each [c_out][c_in][offset], offset (dx+1)+3(dy+1)+9(dz+1).
 * ------------------------------------------------------------------------ */
#define STMG_NET_PARAMS 52704

/* Copy host weights into the context (allocates the network state). */
stmg_status stmg_learned_load(stmg_ctx* ctx, const float* weights_host, size_t n);
/* Read the current weights back (e.g. after training). */
stmg_status stmg_learned_weights(const stmg_ctx* ctx, float* weights_host, size_t n);
/* Switch the correction inside stmg_vcycle / stmg_solve: on = 0 off; 1 on
 * every level it reaches (directly or through the next level); 2 only on
 * levels with the network's element. */
stmg_status stmg_learned_enable(stmg_ctx* ctx, int on);

/* Training pairs on the finest level (3D, r=1, k=1): run the first V-cycle
 * from x = 0 for right-hand side b and record (r, e = xstar - x) after the
 * presmoothing sweep and after the postsmoothing sweep.  r_out and e_out are
 * device FP64 arrays of 2 * n_dofs (pair 0, then pair 1). */
stmg_status stmg_learned_record(stmg_ctx* ctx, const double* b, const double* xstar, double* r_out, double* e_out);

/* Train with Adam (lr, beta = 0.9/0.999) on n_pairs device FP32 pairs
 * (r_pairs, e_pairs: n_pairs x n_dofs of the finest level) for `epochs`
 * passes; a batch is `batch` consecutive space-time cells of one pair, the
 * batch order is a permutation drawn from `seed`.  The loss of every step,
 * sum |net - e|^2 / sum |e|^2 over the batch, goes to loss_hist (host, at
 * least epochs * n_pairs * ceil(cells per pair / batch) values). */
stmg_status stmg_learned_train_pairs(stmg_ctx* ctx, const float* r_pairs, const float* e_pairs, int n_pairs,
                                     uint64_t seed, int epochs, int batch, float lr, float* loss_hist);

/* The whole training of the learned correction in one call, on an FP64
 * context whose finest level has the network's element (3D, r=1, k=1):
 * ceil(n_pairs / 2) random forcings (velocity entries U[-1,1) on interior
 * nodes from a SplitMix64 stream seeded by `seed` and the forcing's index,
 * pressure rows 0), each solved to 1e-12 by plain multigrid FGMRES, give two
 * (residual, error) pairs each (stmg_learned_record); then Adam with
 * learning rate lr, batches of 4096 space-time cells, `epochs` passes
 * (stmg_learned_train_pairs).  Starts from the loaded weights, or from a
 * He-normal initialisation drawn from the seed if none are loaded.  The
 * trained weights (STMG_NET_PARAMS FP32 values) go to weights_out (host) and
 * stay loaded.  The pairs live in device memory for the call only
 * (2 n_pairs n_dofs FP32 values). */
stmg_status stmg_learned_train(stmg_ctx* ctx, int n_pairs, uint64_t seed, int epochs, float lr, float* weights_out);

/* Test hooks on one level, FP64 in and out:
 * u = sum_T R_T^T s_T net(R_T r / s_T) (the correction, no residual check) on
 * a level with the network's element, or P of it applied to P^T r on a level
 * that reaches one through the next level (FP64 contexts only);
 * the gradient on a level with the network's element (3D, r=1, k=1):
 * grad = d/dW [sum |net - e|^2 / sum |e|^2] over all cells of the level. */
stmg_status stmg_learned_correction(stmg_ctx* ctx, int level, const double* r, double* u);
stmg_status stmg_learned_gradient(stmg_ctx* ctx, int level, const double* r, const double* e, float* grad_host,
                                  double* loss);

#ifdef __cplusplus
}
#endif
#endif /* STMG_H */
