/*
 * bamg.h -- C ABI of the MI355X (gfx950) Bootstrap AMG library for the
 * stationary vector of an irreducible Markov chain.
 *
 * Method: Bolten, Brandt, Brannick, Frommer, Kahl, Livshits, "A Bootstrap
 * Algebraic Multilevel method for Markov Chains" (arXiv:1004.1451).
 *   - Problem (Section 1, eq. ax; Section 2): A is column stochastic and
 *     irreducible; find x > 0 with A x = x, i.e. B x = 0 with B = I - A.
 *   - Setup (Algorithm 3 with mu = 1, then the recomputation of every P, B, T
 *     described in Section 1): omega-Jacobi relaxation of r test vectors,
 *     least-squares interpolation (Algorithm 2, eq. LSfuncrowi), averaging
 *     restriction Q, Petrov-Galerkin B_{l+1} = Q B_l P and T_{l+1} = Q T_l P,
 *     injection, the coarsest eigenproblem B_L x = lam T_L x, interpolation
 *     and relaxation of the eigenvector approximations.
 *   - Solve (Section 4.2): flexible GMRES on B x = 0, right-preconditioned by
 *     the V(nu_pre, nu_post) cycle of eq. mgerrorprop with the minimal-norm
 *     (Moore-Penrose) solve on the coarsest level.
 *
 * Conventions shared by every entry point:
 *   - CSR of A: row = destination state, column = source state, so every
 *     column sums to one.  Columns ascending within each row, no duplicates.
 *     row_ptr has n+1 int32 entries, col_idx and val nnz entries.
 *   - States lie on an nx x ny grid, state s = a*ny + b (0 <= a < nx,
 *     0 <= b < ny); coarsening keeps the points with a and b even.  Every
 *     nonzero of A must join states within Chebyshev distance 1 on that grid
 *     (with wrap-around when periodic).
 *   - Or the chain has no grid (bamg_grid {0, 0, 0}; single-chain setup
 *     only): compatible relaxation (Section 3.1, Algorithm 1) chooses the
 *     coarse points of every level, starting from the standard independent
 *     set of the matrix graph, and N_i holds the coarse points joined to i by
 *     a stored entry (eq. neighbor_def with z = 1).  The pattern of A must be
 *     symmetric (an undirected graph, like the unstructured planar graphs of
 *     Section 5); omega-Jacobi relaxation and LS interpolation only.
 *   - "device" pointers are HIP device memory of the current device; "host"
 *     pointers are ordinary host memory.  The library never frees caller
 *     memory.  A handle owns everything it allocates and is bound to the
 *     stream given at setup; it is not thread-safe.
 *   - Return value 0 on success or a negative BAMG_E* code; no exception or
 *     abort crosses the ABI.  bamg_last_error() gives a message for the last
 *     failure of the calling thread.
 *   - Environment: BAMG_POISON=1 fills every floating-point allocation of a
 *     handle with NaN bits (integer ones with zero) when it is made; for
 *     tests that no kernel reads memory it has not written.  Costs one fill.
 */
#ifndef BAMG_H
#define BAMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BAMG_OK 0
#define BAMG_EINVAL (-1)        /* bad argument, shape, pattern or grid      */
#define BAMG_ENOTSTOCH (-2)     /* negative entry or |column sum - 1| > 1e-12 */
#define BAMG_EZERODIAG (-3)     /* b_ii <= 0 (distributive relaxation is not built) */
#define BAMG_EUNSUPPORTED (-4)  /* stencil wider than the 3x3 grid box, a grid
                                   that cannot be coarsened to the requested depth,
                                   or (without a grid) an unsymmetric pattern, a
                                   point with more than 16 coarse neighbours or a
                                   coarse row needing more than 2048 products */
#define BAMG_ENOMEM (-5)        /* device allocation failed or mem_budget exceeded */
#define BAMG_EDEVICE (-6)       /* a HIP runtime error (message kept)         */
#define BAMG_ENOCONV (-7)       /* tolerance not reached within max_cycles; x and
                                   info still hold the best normalised iterate */
#define BAMG_ESINGULAR (-8)     /* coarsest pivot below 1e-12 of its column     */

#define BAMG_FP64 0             /* every step in FP64                            */
#define BAMG_MIXED 1            /* FP32 relaxation, Galerkin products and V-cycle
                                   (its coarsest product by an FP32 copy of B_L^+),
                                   and the coarsest Arnoldi products by that copy;
                                   FP64 norms, the coarsest inverse and
                                   eigenproblem, and the outer iteration          */

#define BAMG_RELAX_JACOBI 0     /* omega-Jacobi: x <- x + omega D^-1 (f - B x)    */
#define BAMG_RELAX_MCGS 1       /* multicolour Gauss-Seidel (Section 3 names
                                   Gauss-Seidel beside Jacobi): the points of a
                                   level are coloured by grid position, two
                                   colours per direction (three along a periodic
                                   side of odd length), so no two points within
                                   Chebyshev distance 1 share one; a sweep
                                   updates colour 0, 1, ... in order,
                                   x_i <- x_i + gs_omega (f_i - (B x)_i) / b_ii.
                                   Every operator must couple only points of
                                   different colours: bamg_setup accepts only
                                   operators within the 3 x 3 grid box and every
                                   coarse operator stays within it, so this
                                   holds; each level is still checked (a
                                   violation fails with BAMG_EINVAL).            */

#define BAMG_INTERP_LS 0        /* least-squares interpolation (Algorithm 2)     */
#define BAMG_INTERP_MLP 1       /* learned weights with the LS fit as judge      */

#define BAMG_USE_GUESS 1u       /* bamg_solve: start from the caller's x         */
#define BAMG_PARNOLDI 2u        /* bamg_solve: the multigrid-preconditioned
                                   Arnoldi method of Section 4.3 instead of
                                   FGMRES: Arnoldi on C B (C = one cycle) from
                                   the start vector; after each step the Ritz
                                   vector of the eigenvalue of H_j closest to 0,
                                   scaled to sum 1, is the iterate; restarted
                                   from it every gmres_m steps.  cycles counts
                                   applications of C; history holds the residual
                                   after each step.                              */

typedef struct bamg_ctx* bamg_handle;

typedef struct {
    int32_t nx, ny;   /* grid sides, nx*ny == n                              */
    int32_t periodic; /* 1: wrap in both directions (sides must stay even)    */
} bamg_grid;

typedef struct {
    int32_t levels;      /* number of levels including the finest; 0 = coarsen
                            while n_l > coarse_max                          */
    int32_t coarse_max;  /* used when levels == 0                             */
    int32_t nu_setup;    /* Jacobi sweeps on test / eigenvectors per level    */
    int32_t nu_pre, nu_post; /* V(nu_pre, nu_post) cycle                       */
    double omega;        /* Jacobi weight (Section 3: 0.7)                    */
    int32_t caliber;     /* c: max interpolatory points per fine point        */
    int32_t n_eig;       /* k: coarsest eigenpairs including the null vector  */
    int32_t arnoldi_m;   /* Krylov dimension of the coarsest eigensolve       */
    int32_t gmres_m;     /* restart length of flexible GMRES (1 .. 63)         */
    int32_t precision;   /* BAMG_FP64 or BAMG_MIXED                            */
    int32_t interp;      /* BAMG_INTERP_LS or BAMG_INTERP_MLP                  */
    const float* mlp_weights; /* device, BAMG_MLP_NPARAM floats; needed for MLP */
    uint64_t seed;       /* seed of the initial test vectors                  */
    size_t mem_budget;   /* bytes; 0 = unlimited                               */
    int32_t profile;     /* 1: time the level-0 sweeps and Galerkin products
                            with HIP events (reported in bamg_stats)          */
    int32_t stop_after;  /* 0: full setup; 1: after the first down-leg;
                            2: after the coarsest eigensolve; 3: after the
                            up-leg (inspection only)                          */
    int32_t cycle_mode;  /* 0: decide on the first cycle (graph when the cycle
                            is launch-bound); 1: eager launches; 2: HIP graph
                            of one cycle, captured once and replayed          */
    int32_t setup_passes;/* 2 (0 = default): down-leg, up-leg, then every P, B,
                            T recomputed from U and V; 1: the first pass only
                            (the cycle uses the first-pass hierarchy)          */
    int32_t collect;     /* 1: keep the first-pass features and the final
                            slot weights of every level for bamg_export
                            (BAMG_X_FEATURES, BAMG_X_SLOTW): training data    */
    float mlp_judge;     /* learned form: keep the network's row when the LS
                            functional at it is <= mlp_judge x the fit's
                            minimum (default 2)                               */
    int32_t relax;       /* BAMG_RELAX_JACOBI (omega-Jacobi, default) or
                            BAMG_RELAX_MCGS (multicolour Gauss-Seidel) for the
                            test-vector, eigenvector and cycle sweeps         */
    double gs_omega;     /* weight of the Gauss-Seidel update (default 1)     */
    int32_t mu;          /* cycle index of the setup cycle (Algorithm 3): 1 =
                            V-cycle (default), 2 = W-cycle (every level fits,
                            recurses and brings the eigenvectors up twice, the
                            second time fitting to U and V)                   */
    /* chains without a grid (bamg_grid {0, 0, 0}): compatible relaxation,
       Section 3.1, Algorithm 1 */
    double cr_theta;     /* CR tolerance theta (default 0.85)                  */
    int32_t cr_nu;       /* F-relaxation sweeps per estimate (default 8)       */
    int32_t cr_rounds;   /* at most this many CR relaxations per level (64)    */
    int32_t nbr_dist;    /* z of eq. neighbor_def: path length of the candidate
                            sets N_i (only 1 is built)                        */
    const char* mlp_weights_path; /* learned form: network file written by
                            bamg_mlp_train_spec, read when mlp_weights is NULL */
} bamg_options;

typedef struct {
    int32_t cycles;        /* preconditioner applications (V-cycles)          */
    int32_t restarts;      /* completed GMRES restart cycles                  */
    int32_t converged;     /* 1 if ||B x||_1/||x||_1 <= tol                     */
    int32_t history_len;
    double residual_l1;    /* ||B x||_1 / ||x||_1 of the returned x (FP64)      */
    double clamped_mass;   /* mass removed by clamping negative entries       */
    double history[256];   /* true relative residual after each restart       */
} bamg_solve_info;

typedef struct {
    int32_t n_levels;
    int32_t n_v;            /* columns of eigenvector approximations          */
    double op_complexity;   /* sum nnz(B_l) / nnz(B_0)                         */
    double coarsest_min_pivot; /* smallest Gauss-Jordan pivot of the coarsest inverse:
                                  diagonal blocks' pivots / max |B_L entry|; on
                                  grids without the periodic arrow also the
                                  joins' pivots of I - C G (dimensionless) */
    double t_setup_ms, t_solve_ms;   /* host wall clock of the last calls      */
    /* with options.profile: HIP-event time and launch count of the level-0
       test-vector sweeps (every launch), of the launch that forms both
       Galerkin products B_1 = Q (B_0 P) and T_1 = Q (T_0 P) (T_0 = I) and of
       the least-squares fit of the first setup pass, each with the
       algorithmic bytes of one such launch */
    double sweep_ms, galerkin_ms, lsfit_ms;
    int32_t sweep_launches, galerkin_launches, lsfit_launches;
    int64_t sweep_bytes, galerkin_bytes, lsfit_bytes; /* algorithmic bytes per launch */
    int32_t cycle_graph;    /* 1: cycles replay a captured graph              */
    double cycle_host_us, cycle_gpu_us; /* first cycle (cycle_mode 0): host launch
                                           time and GPU time                 */
    int32_t sweep_vw, sweep_bs; /* launch shape of the level-0 multi-vector sweep:
                                   columns per thread, threads per workgroup
                                   (VW 1, 2, 3, 4, 6 or 12; autotuned once per shape and process;
                                   BAMG_SWEEP_VARIANT="VW,BS[,RP]" forces one) */
    double tune_ms;         /* process total spent timing launch candidates
                               (level-0 and coarse sweeps; the fused Galerkin
                               launch's 14, 28 or 56 coarse rows per
                               workgroup, BAMG_GAL_ROWS forcing one); with
                               BAMG_TUNE_CACHE=<file> the choices are read
                               from and written to that JSON file          */
    int64_t mlp_points;     /* learned form: F points judged (all levels)      */
    int64_t mlp_fallback;   /* of which fell back to the least-squares row     */
    /* with options.profile: the rank-64 updates of the dense coarsest inverse
       (coarsest levels without block structure): HIP-event time, launches,
       and their flops (2 nb (m - nb)^2 each, m = n_L - 1)                */
    double dense_update_ms;
    int32_t dense_update_launches;
    double dense_update_flops;
    int32_t sweep_ell;      /* 1: the level-0 sweeps, the cycle's level-0 residual
                               and the outer SpMV read a 4-wide ELL copy of B_0
                               (every row has at most 4 entries)            */
    /* with options.profile, the other level-0 launches of the setup, same
       form: the copy of both products from their ELL-9 form into CSR, and
       the least-squares fit of the recompute pass (U and V) */
    double gal_csr_ms, lsfit2_ms;
    int32_t gal_csr_launches, lsfit2_launches;
    int64_t gal_csr_bytes, lsfit2_bytes;
    int32_t sweep_rp;       /* row pieces per thread of the level-0 sweep (1, or
                               2 on the ELL-4 copy; autotuned with sweep_vw)  */
    int32_t arnoldi_steps;  /* Arnoldi steps of the last coarsest eigensolve:
                               min(40, n_L - 1), or m = 20 or 30 when every
                               wanted Ritz pair's relative residual
                               |h_{m+1,m} s_m| / |theta| is at most 1e-9 after
                               m steps (checked at 20, then 30;
                               BAMG_ARNOLDI_CHECK=0 in the environment turns
                               the checks off)                                  */
} bamg_stats;

typedef struct {
    int64_t n;          /* rows of B_l                                        */
    int32_t nx, ny, periodic;
    int64_t nnz_b, nnz_t; /* T_0 = I is not stored: nnz_t = 0 on level 0     */
    int64_t nnz_p;      /* entries of P_l (0 on the coarsest level)           */
    int32_t r;          /* columns of U_l                                     */
    int32_t n_v;        /* columns of V_l                                     */
    int32_t cr_rounds;  /* CR relaxations that chose this level's C points
                           (0 on grids and on the coarsest level)            */
} bamg_level_info;

/* Items of bamg_export (arrays of one level, copied to host memory). */
#define BAMG_X_B_ROWPTR 1   /* int32[n+1]                                   */
#define BAMG_X_B_COL 2      /* int32[nnz_b]                                 */
#define BAMG_X_B_VAL 3      /* double[nnz_b]                                */
#define BAMG_X_T_ROWPTR 4
#define BAMG_X_T_COL 5
#define BAMG_X_T_VAL 6
#define BAMG_X_P_COL 7      /* int32[4n], ELL: slot s of row i at 4i+s, -1 = empty,
                               used slots first in ascending column order    */
#define BAMG_X_P_VAL 8      /* double[4n]                                   */
#define BAMG_X_U 9          /* double[n*r], row-major: the relaxed test vectors */
#define BAMG_X_V 10         /* double[n*n_v], row-major eigenvector approximations */
#define BAMG_X_LAMBDA 11    /* double[2*n_v]: (re, im) of the eigenvalue of each
                               column (both columns of a pair carry the pair's
                               Im > 0 member)                                */
#define BAMG_X_VKIND 12     /* int32[n_v]: 0 real, 1 real part, 2 imaginary part */
#define BAMG_X_X0 13        /* double[n]: setup's state-vector approximation */
#define BAMG_X_W 14         /* double[n*n] (coarsest level): B_L^+ row-major   */
#define BAMG_X_Y 15         /* double[n] (coarsest level): null vector, 1^T T y = 1 */
#define BAMG_X_U0 16        /* double[n*r] level 0: the initial test vectors   */
#define BAMG_X_FEATURES 17  /* float[n*24] first-pass features of every point
                               (zero rows for C points); needs options.collect */
#define BAMG_X_SLOTW 18     /* float[n*4] final interpolation weights in slot
                               order (lexicographic (da, db)); needs collect  */
#define BAMG_X_SLOTW0 19    /* float[n*4] the first pass's fitted weights in slot
                               order (least-squares form); needs collect      */
#define BAMG_X_CMAP 20      /* int32[n] (level without a grid, not the coarsest):
                               coarse index of each C point (its rank among the
                               C points), -1 for an F point                   */
#define BAMG_X_CR_RHO 21    /* double[cr_rounds]: the estimate of eq. meas1 of
                               every CR relaxation of the level               */

/* Fill *opt with the defaults: levels 0, coarse_max 1024, nu_setup 4,
   V(2,2), omega 0.7, caliber 4, n_eig 6, arnoldi_m 40, gmres_m 50,
   FP64, LS interpolation, seed 0, no budget, no profiling, 2 setup passes,
   mlp_judge 2, omega-Jacobi relaxation (gs_omega 1), mu 1; without a grid
   cr_theta 0.85, cr_nu 8, cr_rounds 64, nbr_dist 1 (Section 3.1). */
void bamg_options_default(bamg_options* opt);

/* Build the hierarchy for A (device CSR, see conventions) with r initial test
   vectors.  The caller's arrays are only read during the call and may be freed
   once it returns.  stream: a hipStream_t (NULL = default stream); every
   kernel of this handle runs on it.  On success *out owns the hierarchy.
   grid {0, 0, 0}: no grid, coarsened by compatible relaxation (see the
   conventions); levels then counts the levels to build (0: coarsen while
   n_l > coarse_max) and EUNSUPPORTED reports a level CR cannot coarsen.
   Errors: EINVAL (null pointer, n < 1, r < 1, bad CSR, nx*ny != n),
   ENOTSTOCH, EZERODIAG, EUNSUPPORTED, ENOMEM, EDEVICE, ESINGULAR.
   Irreducibility is a precondition and is not checked. */
int bamg_setup(int64_t n, const int32_t* row_ptr, const int32_t* col_idx,
               const double* val, bamg_grid grid, int32_t r,
               const bamg_options* opt, void* stream, bamg_handle* out);

/* Solve B x = 0 to ||B x||_1 / ||x||_1 <= tol with at most max_cycles
   preconditioner applications.  x: device, n doubles; read as the starting
   vector with BAMG_USE_GUESS, otherwise the setup's approximation is used.
   On return x >= 0 and sum(x) = 1.  info (host) may be NULL.  Returns 0,
   ENOCONV (x and info hold the best iterate), EINVAL or EDEVICE.  The call
   returns after the stream has finished. */
int bamg_solve(bamg_handle h, double* x, double tol, int32_t max_cycles,
               uint32_t flags, bamg_solve_info* info);

/* Batched setup: nchains independent chains in one handle, solved together.
   The same construction as bamg_setup, applied to every chain (Algorithm 3
   per chain); chains never interact.  The caller concatenates the chains
   block-diagonally: chain c owns rows and columns [chain_row_off[c],
   chain_row_off[c+1]) of the CSR (host int64 array of nchains+1 offsets,
   chain_row_off[0] = 0, n = chain_row_off[nchains]); a column outside the
   row's own chain is EINVAL.  grids: host array of nchains grids, one per
   chain (local state numbering).  Chains may differ in size and depth; with
   levels = 0 each chain coarsens until its own size <= coarse_max.  Every
   chain's coarsest grid must have ny <= 64 when nchains > 1 (EUNSUPPORTED
   otherwise).  bamg_export is limited to nchains = 1; the other entry points
   work on all chains at once.  1 <= nchains <= 4096.  Same errors as
   bamg_setup. */
int bamg_setup_batched(int32_t nchains, const int64_t* chain_row_off,
                       const int32_t* row_ptr, const int32_t* col_idx,
                       const double* val, const bamg_grid* grids, int32_t r,
                       const bamg_options* opt, void* stream, bamg_handle* out);

/* Solve every chain of a batched handle (or of a bamg_setup handle, as one
   chain) with lockstep flexible GMRES: each chain keeps its own Krylov
   scalars and stops on its own tolerance.  x: device, n doubles in the
   caller's concatenated order; each chain's block ends >= 0 and sums to 1.
   chain_status (host int32[nchains], may be NULL): 1 converged, 0 not.
   chain_residual (host double[nchains], may be NULL): ||B_c x_c||_1/||x_c||_1.
   info: cycles, restarts and history hold the worst chain.  Returns 0 when
   every chain converged, otherwise ENOCONV; EINVAL, EDEVICE. */
int bamg_solve_batched(bamg_handle h, double* x, double tol, int32_t max_cycles,
                       uint32_t flags, int32_t* chain_status,
                       double* chain_residual, bamg_solve_info* info);

/* The multilevel eigensolver iteration used as a stand-alone solver (Section
   4.1: the MLE steps of Algorithm 3 yield the state-vector approximation
   V_0[:, 0]).  Runs further setup cycles on the handle's hierarchy (with
   options.mu as set up), each fitting every P_l to U_l and the previous cycle's
   eigenvector approximations V_l, until ||B x||_1 / ||x||_1 <= tol for x =
   V_0[:, 0] / sum, or max_cycles cycles.  x: caller-owned device array of n
   doubles, written with that x clamped to x >= 0 and scaled to sum 1.  info
   (host, may be NULL): cycles = MLE cycles run, history = residual after each.
   The handle keeps the last cycle's hierarchy (bamg_solve uses it).  Returns
   BAMG_ENOCONV when the tolerance is not met, BAMG_EUNSUPPORTED for a handle
   of several chains, BAMG_EINVAL for NULL pointers, tol <= 0 or max_cycles < 0. */
int bamg_mle_iterate(bamg_handle h, double* x, double tol, int32_t max_cycles, bamg_solve_info* info);

/* Release everything the handle owns.  NULL is allowed.  The handle's stream
   is drained first; its device buffers go back to the library's process-wide
   cache (per device, size classes within 1/16 of a power of two) for the next
   setup, and are returned to HIP only by bamg_trim. */
int bamg_free(bamg_handle h);

/* Return every cached device buffer not owned by a live handle to HIP
   (hipFree).  Handles stay valid.  Returns 0. */
int bamg_trim(void);

/* Message of the last failing call on this thread ("" if none). */
const char* bamg_last_error(void);

/* Statistics of the last setup / solve (host struct). */
int bamg_get_stats(bamg_handle h, bamg_stats* st);

/* Sizes of level l (0 = finest). */
int bamg_level_info_get(bamg_handle h, int32_t l, bamg_level_info* out);

/* Copy item `what` (BAMG_X_*) of level l into host memory dst of `bytes`
   bytes; EINVAL if the item does not exist on that level or bytes is too
   small.  Synchronises the handle's stream. */
int bamg_export(bamg_handle h, int32_t l, int32_t what, void* dst, size_t bytes);

/* One application of the V-cycle preconditioner on level 0: e = C f
   (device vectors of n doubles; for a batched handle all chains at once, in
   the caller's concatenated order).  Synchronises the stream. */
int bamg_apply_vcycle(bamg_handle h, const double* f, double* e);

/* ---- Learned interpolation (the learned form of the first-pass fit) ----
   A 24-64-64-4 ReLU network maps the 24 features of an F point's
   least-squares problem (Section 3.2, eq. LSfuncrowi: the slot mask, the
   operator row -b_ij/b_ii at the 8 neighbour offsets, b_s/G_ss,
   b_s/sqrt(sigma G_ss), sqrt(G_ss/sigma)) to a correction of its 4 fitted
   slot weights (the setup adds it to the first-pass fit, then judges).  Params:
   BAMG_MLP_NPARAM FP32 values, row-major W1[64][24], b1[64], W2[64][64],
   b2[64], W3[4][64], b3[4].  Every product runs on the matrix cores with
   bfloat16 operands (round to nearest even) and FP32 accumulation.  Features
   and targets are device FP32 arrays, n x 24 and n x 4; the first 4 features
   (the slot mask) mask the loss.  All calls synchronise the stream. */
#define BAMG_MLP_NPARAM 6020

typedef struct {
    int32_t epochs;      /* passes over the training set (default 8)           */
    int32_t batch;       /* points per Adam step, multiple of 256 (4096)       */
    float lr, beta1, beta2, eps;   /* Adam (1e-3, 0.9, 0.999, 1e-8)            */
    uint64_t seed;       /* batch sampling (with replacement); 0 = in order     */
} bamg_mlp_train_opts;

typedef struct {
    int32_t steps;
    double train_loss_first, train_loss_last;   /* batch losses               */
    double val_loss_first, val_loss_last;       /* before / after training    */
    double ms;                                  /* wall time of the call      */
    int32_t val_len;
    double val_history[64];                     /* after each epoch           */
} bamg_mlp_train_info;

/* He-uniform weights U(-sqrt(6/fan_in), sqrt(6/fan_in)) from the counter
   generator, zero biases.  params: device, BAMG_MLP_NPARAM floats. */
int bamg_mlp_init(uint64_t seed, float* params, void* stream);

/* out[i] = network(feat[i]) for n points (device arrays). */
int bamg_mlp_forward(const float* feat, int64_t n, const float* params, float* out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the same
   inference as bamg_mlp_forward, bit for bit, staged through a static device
   array of the library (8.02 MiB per GPU, held until the process ends)
   instead of allocated buffers.  n <= 131072 points (larger n returns
   BAMG_EINVAL); feat (n x 24), params and out (n x 4) are the caller's device
   arrays, stream a stream of the current device.  Calls on one GPU share the
   array: calls that overlap on one GPU (other streams, other threads) race.
   Calls no allocating routine.  Synchronises the stream. */
int bamg_mlp_forward_noalloc(const float* feat, int64_t n, const float* params, float* out, void* stream);

/* Masked mean squared error over all n points (one batch) and its gradient
   (device, BAMG_MLP_NPARAM floats); *loss on the host. */
int bamg_mlp_loss_grad(const float* feat, const float* tgt, int64_t n, const float* params, float* grad,
                       double* loss, void* stream);

/* Adam on params (in place) over (feat, tgt); the loss on (vfeat, vtgt),
   nv >= 0 points, is reported before, after each epoch and at the end.
   opt and info are host structs (opt NULL = defaults; info may be NULL). */
int bamg_mlp_train(const float* feat, const float* tgt, int64_t n, const float* vfeat, const float* vtgt, int64_t nv,
                   float* params, const bamg_mlp_train_opts* opt, bamg_mlp_train_info* info, void* stream);

/* Training pairs of the learned form from a handle set up with
   options.collect (least-squares form): for every F point of every
   non-coarsest level, its 24 first-pass features (feat, n x 24) and, as the
   target, the correction of its fitted slot weights, final minus first-pass
   (tgt, n x 4), in level order.  Only ordinary points are kept: at least one
   valid slot, every feature within +-16 and every correction within +-1.
   feat and tgt are device arrays of cap rows, or both NULL to count only;
   *count (host) = the pairs.  BAMG_EINVAL if they exceed cap (*count still
   set).  Synchronises the handle's stream. */
int bamg_mlp_collect(bamg_handle h, float* feat, float* tgt, int64_t cap, int64_t* count);

/* The training set of the learned form, built by the library itself: n_chains
   jittered tandem queues (Section 5, Table 2 rates 11/31, 10/31, 10/31, each
   times 1 + jitter (2u - 1)), chain c of side side_min + floor((side_max -
   side_min + 1) u_c), u_c from the counter generator (seed, stream 8, c),
   rates from (seed, stream 3, 3 (1000 + c) + k); each set up in FP64 with
   r test vectors and `levels` levels, its pairs collected as by
   bamg_mlp_collect; the last n_val chains validate. */
typedef struct {
    int32_t n_chains;    /* training and validation chains (32)                */
    int32_t n_val;       /* of which the last n_val validate (4)               */
    int32_t side_min, side_max; /* grid sides N + 1 (256, 1024)                */
    double jitter;       /* relative rate jitter (0.2)                          */
    uint64_t seed;       /* chain sides and rates (0)                           */
    int32_t r, levels;   /* setups that collect the pairs (12, 6)               */
    uint64_t init_seed;  /* He-uniform initial weights (5)                      */
    bamg_mlp_train_opts train; /* Adam (8 epochs, batch 4096, lr 1e-3, seed 6) */
} bamg_train_spec;

/* Fills *spec with the defaults above. */
void bamg_train_spec_default(bamg_train_spec* spec);

/* Builds the training set of *spec, initialises a network (bamg_mlp_init
   with init_seed) and trains it (bamg_mlp_train with spec->train).  The
   parameters go to params (device, BAMG_MLP_NPARAM floats) when not NULL and
   to the file out_path when not NULL ("BAMGMLP1", int32 count, FP32 values;
   options.mlp_weights_path reads it); info (host) may be NULL.  Allocates
   and frees its own device memory; synchronises the stream. */
int bamg_mlp_train_spec(const bamg_train_spec* spec, const char* out_path, float* params,
                        bamg_mlp_train_info* info, void* stream);

/* nu omega-Jacobi sweeps X <- X + omega D^-1 (F - B X) on caller data
   (Section 3, eq. amg_relax): B = I - A from device CSR of A (as in
   bamg_setup, validated the same way), X device n x R row-major (in place),
   F device n x R or NULL for the homogeneous problem.  Runs the same kernel
   as the setup.  Synchronises the stream. */
int bamg_relax(int64_t n, const int32_t* row_ptr, const int32_t* col_idx,
               const double* val, double* X, const double* F, int32_t R,
               double omega, int32_t nu, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* BAMG_H */
