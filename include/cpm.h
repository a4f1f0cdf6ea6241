/*
 * cpm.h -- C ABI of the MI355X Closest Point Method multigrid library (libcpm.so).
 *
 * Problem (Chen & Macdonald, Sec. 2.1, eq. (2.1)): solve  -Lap_S u + c u = f  on a closed
 * curve or surface S given by its closest-point function cp, c > 0 constant.  f is known
 * on S and extended off S by f~(x) = f(cp(x)).
 *
 * Discretization (Sec. 3.1): a band of grid nodes x_i = h * i (i integer) within
 * sqrt(lam2) * h of S; tensor-product cubic Lagrange interpolation at cp(x_i) (matrix E,
 * 4^d weights per node); (2d+1)-point Laplacian L = N - (2d/h^2) I; the CPM matrix
 * A = c I - M, M = E L - gamma (I - E), gamma = 2d/h^2 (eq. (3.3)), which equals
 * A u = delta u - E (N u) with delta = c + 2d/h^2.
 *
 * Solver (Sec. 4, Algorithm 4.1): V(nu1, nu2) cycles with Ruuth-Merriman Jacobi smoothing
 * (Jacobi on cI - L followed by closest-point extension, eqs. (4.2a)-(4.2b)), damped by
 * omega outside the extension; closest-point restriction / prolongation between bands of
 * spacing h and 2h (Sec. 4.3, linear interpolation as in Sec. 4.6); a direct solve on the
 * coarsest level.  The residual is r = E(f + N u) - delta u = E f - A u and the solve stops
 * when ||r||_inf / ||E f||_inf < rtol.
 *
 * Conventions for every call:
 *   - Vectors are contiguous device arrays (double unless stated) of length n(level), in
 *     band order: grid multi-indices sorted lexicographically with x fastest, then y, z.
 *   - f is given as samples f(cp(x_i)) at the band nodes of level 0.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).  Calls are
 *     asynchronous on that stream unless stated; device buffers belong to the caller.
 *   - A band handle is immutable after cpm_build_band except for cached coarse-level
 *     factorizations and captured graphs; do not use one handle from two host threads
 *     at once.
 *   - Every function returns a cpm_status; nothing throws across the ABI.  On failure
 *     cpm_last_error() returns a message for the calling thread.
 */
#ifndef CPM_H
#define CPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  CPM_OK = 0,
  CPM_E_INVALID = 1,  /* bad argument (null pointer, level out of range, bad sizes)      */
  CPM_E_BAND = 2,     /* a stencil leaves the band (band radius too small for the grid) */
  CPM_E_NOMEM = 3,    /* host or device allocation failed                                */
  CPM_E_HIP = 4,      /* a HIP runtime call failed                                       */
  CPM_E_NOCONV = 5,   /* max_cycles reached before rtol                                  */
  CPM_E_DIVERGED = 6, /* NaN / Inf residual                                              */
  CPM_E_WORKSPACE = 7 /* workspace too small                                             */
} cpm_status;

/* CPM_DZIUK: the level set (x1 - x3^2)^2 + x2^2 + x3^2 = 1 shifted by center (R, r unused),
 * the level-set example of Sec. 4.6.5; its closest points are computed by
 * Newton's method from the nearest of a fixed set of surface samples. */
typedef enum { CPM_CIRCLE = 0, CPM_SPHERE = 1, CPM_TORUS = 2, CPM_DZIUK = 3 } cpm_surface_kind;

/* Analytic surfaces of the paper's examples (Sec. 3.4, 4.6).  circle: 2-D, centre
 * center[0..1], radius R.  sphere: centre, radius R.  torus: centre, axis along z,
 * tube-centre radius R, tube radius r. */
typedef struct {
  int kind;
  double center[3];
  double R;
  double r;
} cpm_surface;

/* Grid hierarchy: finest spacing h0, h_l = h0 * 2^l for l = 0..levels-1, band radius^2 =
 * lam2 * h_l^2 on each level (lam2 <= 0 selects 13 in 2-D, 17 in 3-D). */
typedef struct {
  double h0;
  int levels;
  double lam2;
} cpm_grid;

typedef enum { CPM_F64 = 0, CPM_MIXED = 1 } cpm_precision;
typedef enum {
  CPM_SMOOTH_JACOBI = 0,
  CPM_SMOOTH_LEARNED = 1,
  CPM_SMOOTH_STANDARD = 2,
  CPM_SMOOTH_STANDARD_RB = 3
} cpm_smoother;

/* Solver parameters.  precision CPM_MIXED: float32 smoothing / extension / transfers on
 * every level, float64 outer residual, refinement update and coarsest solve.
 * smoother CPM_SMOOTH_JACOBI: the Ruuth-Merriman step (Sec. 4.2), damped by omega.
 * smoother CPM_SMOOTH_LEARNED: the learned local smoother (cpm_set_smoother_weights) on
 * the two finest levels, Jacobi elsewhere, with a fallback to Jacobi (see cpm_stats).
 * smoother CPM_SMOOTH_STANDARD: the standard relaxation of Sec. 4.5 (CPM_F64 only): the
 * cycle solves A u = f itself (no extension of f), smooths with Jacobi on A,
 * u <- u + omega diag(A)^{-1} (f - A u), passes the residual f - A (E u) to the coarse grid
 * and solves the coarsest level with A_c^{-1}; its progress is measured by the relative
 * increment ||u_k - u_{k-1}||_inf / ||u_k||_inf (the paper's stopping test), which is what
 * relres / relres_history / relres_out and rtol then refer to (the cycle's fixed point does
 * not make f - A u vanish).
 * smoother CPM_SMOOTH_STANDARD_RB: the same standard relaxation with Gauss-Seidel in red-black
 * order instead of Jacobi (Sec. 4.5 names Gauss-Seidel as the alternative): each sweep applies
 * the damped correction omega diag(A)^{-1} (f - A u) to the nodes whose grid index sum is even,
 * then, from that iterate, to the others (nodes of one colour that A couples are updated
 * together).  Everything else as for CPM_SMOOTH_STANDARD. */
typedef struct {
  double c;
  int nu1;
  int nu2;
  double omega;
  int precision;
  int smoother;
  int learned_sweeps; /* learned smoother: sweeps before and after the coarse correction on
                         the levels where it runs (0 = nu1 / nu2 as everywhere else) */
  int gamma;          /* cycle index: visits of the next coarser level per level (1 = V-cycle,
                         2 = W-cycle; 0 is taken as 1; the coarsest level is solved once) */
  int fmg;            /* cpm_solve only: 1 = start from the full-multigrid (nested iteration)
                         approximation instead of the given u: f restricted to every level,
                         coarsest solved, then per finer level cubic closest-point
                         interpolation of the coarser solution and one cycle (smoother
                         CPM_SMOOTH_JACOBI; the start runs in double precision, also before
                         CPM_MIXED cycles, whose workspace then holds the double-precision
                         layout too) */
  int residual_mode;  /* CPM_RESIDUAL_CONSISTENT (0): the residual passed to the coarse grid
                         is E f - A u (= E(f + N u) - delta u), whose fixed point solves
                         A u = E f.  CPM_RESIDUAL_VERBATIM (1): Algorithm 4.1 step 2 as printed,
                         r = f - (cI - L) u = f + N u - delta u at every node, and the coarsest
                         level solves A_c e = f_c; its residual stagnates at the extension's
                         discretization error (Sec. 4.6.1 notes this), so progress is the
                         relative increment ||u_k - u_{k-1}||_inf / ||u_k||_inf (the paper's
                         stopping test), which relres and rtol then refer to (precision
                         CPM_F64, smoother CPM_SMOOTH_JACOBI, constant coefficient).  With
                         the standard relaxation it selects the plain residual f - A u (the
                         printed step with A in place of A~) instead of f - A (E u); the fixed
                         point then solves A u = f */
  int el_degree;      /* degree p of the interpolation in front of L in M = E_p L - gamma
                         (I - E_3): 3 (or 0) the cubic of every cycle; 1 the sparser operator of
                         Remark 3.2 (Table 3.1), with the standard relaxation only */
} cpm_params;

#define CPM_RESIDUAL_CONSISTENT 0
#define CPM_RESIDUAL_VERBATIM 1

#define CPM_MAX_HISTORY 256

typedef struct {
  int cycles;                               /* V-cycles (outer steps) executed          */
  double relres;                            /* final ||E f - A u||_inf / ||E f||_inf   */
  double relres_history[CPM_MAX_HISTORY];   /* after each cycle                         */
  int fallback_cycle;                       /* learned smoother: cycle at which it was
                                               replaced by Jacobi, -1 if never           */
  double seconds;                           /* wall time of the solve loop on the host  */
  int tile_block;                           /* batched: workgroup size chosen by the
                                               autotuner (0 for single solves)           */
  int tile_blocks_per_cu;                   /* batched: resident workgroups per CU       */
  int host_syncs;                           /* batched: host synchronizations of the
                                               solve loop (one per graph launch)          */
  int cycles_per_launch;                    /* batched: cycles captured per graph launch */
} cpm_stats;

typedef struct cpm_band_s* cpm_band;

/* Device allocator for the arrays a band owns (index tables, closest-point fractions,
 * coarsest-level matrices, scalars, smoother weights): alloc(ctx, bytes) returns device
 * memory or NULL, release(ctx, p) frees it, so a framework's caching allocator (torch's) can
 * back a band.  Bands use the allocator registered when they are built, until they are
 * freed; NULL for both restores hipMalloc / hipFree.  Process-wide; set it before building
 * bands, not while another thread builds one.  CPM_E_INVALID if only one function is given.
 * (Workspaces and vectors are the caller's own memory and never go through it.) */
cpm_status cpm_set_allocator(void* (*alloc)(void* ctx, size_t bytes), void (*release)(void* ctx, void* ptr),
                             void* ctx);

/* Build the band hierarchy (Sec. 3.1, Sec. 4.3): band nodes, closest points, cubic
 * extension stencils, Laplacian neighbours and the linear restriction / prolongation
 * stencils of every level; checks that every stencil node and every Laplacian neighbour
 * of a stencil node lies in the band (CPM_E_BAND otherwise).  Index construction runs on
 * the host in IEEE double without contraction, then the arrays are copied to the device
 * on `stream` (the call synchronizes it).  *out receives a handle owned by the caller
 * (release with cpm_band_free). */
cpm_status cpm_build_band(const cpm_surface* surface, const cpm_grid* grid, void* stream,
                          cpm_band* out);

/* Build `count` band hierarchies (surfaces[k], grids[k]) as cpm_build_band does, several
 * at once on the host's cores (each band single-threaded), for batches of problems.  out
 * receives count handles; on failure none is left allocated and the error names the first
 * failing band. */
cpm_status cpm_build_bands(int count, const cpm_surface* surfaces, const cpm_grid* grids, void* stream,
                           cpm_band* out);

/* Release a handle and all device memory it owns.  NULL is accepted. */
cpm_status cpm_band_free(cpm_band band);

/* Number of levels, embedding dimension. */
cpm_status cpm_band_levels(cpm_band band, int* levels, int* dim);

/* Size n and spacing h of one level (any output may be NULL), and flags:
 * CPM_BAND_BEYOND_REACH when the band radius sqrt(lam2) h of the level reaches the surface's
 * reach (Sec. 2.1: the closest point is unique only within it; radius R for a circle or
 * sphere, min(r, R - r) for a torus, the smallest radius of curvature for the level set).
 * Such coarse levels are allowed: nodes at a tie take the documented closest point on S. */
#define CPM_BAND_BEYOND_REACH 1
/* CPM_BAND_RESID_SUBSET: the residual passed to the restriction into the next level is formed
 * only at the fine nodes that the restriction's linear stencils read (Sec. 4.3: it samples
 * the residual near the surface; about a third of a 3-D level), the other entries of that
 * vector being left as they were. */
#define CPM_BAND_RESID_SUBSET 2
cpm_status cpm_band_info(cpm_band band, int level, int64_t* n, double* h, int* flags);

/* Copy one level's grid multi-indices (n x dim int32, row-major) and closest points
 * (n x dim double, row-major) into caller-owned host buffers (either may be NULL). */
cpm_status cpm_band_export(cpm_band band, int level, int32_t* idx_host, double* cp_host);

/* Copy one level's addressing into caller-owned host buffers (any may be NULL):
 *   runE  n x 4^(dim-1): band index of the first node of each x-run of the cubic stencil
 *         of cp(x_i), run (b, c) at column b + 4c (y offset b, z offset c);
 *   nbr   n x 2*dim: band index of the -x,+x,-y,+y(,-z,+z) neighbour, -1 if absent;
 *   runP  n x 2^(dim-1): x-runs of the linear stencil of cp(x_i) in level+1's band
 *         (prolongation; undefined on the coarsest level);
 *   runR  n x 2^(dim-1): x-runs of the linear stencil of cp(x_i) in level-1's band
 *         (restriction; undefined on level 0). */
cpm_status cpm_band_export_stencils(cpm_band band, int level, int32_t* runE, int32_t* nbr,
                                    int32_t* runP, int32_t* runR);

/* Bytes of device workspace a vcycle / solve with these parameters needs (CPM_MIXED with
 * fmg: the larger of the mixed and the double-precision layouts). */
cpm_status cpm_workspace_size(cpm_band band, const cpm_params* params, size_t* bytes);

typedef enum { CPM_DTYPE_F64 = 0, CPM_DTYPE_F32 = 1 } cpm_dtype;

/* Au = (c + 2d/h^2) u - E (N u) on one level (eq. (3.3), matrix-free).  u and Au are device
 * vectors of length n(level) of type dtype (CPM_DTYPE_F64: double, CPM_DTYPE_F32: float,
 * the arithmetic then in float) that must not overlap; work is a device buffer of at least
 * n(level) elements of that type. */
cpm_status cpm_apply(cpm_band band, int level, int dtype, double c, const void* u, void* Au, void* work,
                     void* stream);

/* cpm_apply without a workspace, for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops): the work vector is a file-scope device array of 32 MiB that
 * every GPU the library runs on holds until the process ends (4 Mi doubles / 8 Mi floats).
 * Levels whose work vector would exceed it are refused with CPM_E_WORKSPACE.  No device
 * memory is allocated or freed.  All calls on one GPU share that array: calls that overlap in
 * time on one GPU (two streams, or two host threads) race and must be ordered by the caller. */
cpm_status cpm_apply_static(cpm_band band, int level, int dtype, double c, const void* u, void* Au, void* stream);

/* A u for the family of Sec. 3.1: A = c I - M, M = E_p L - gamma (I - E_3), gamma = 2d/h^2,
 * p = 3 (cpm_apply) or p = 1 (Remark 3.2: linear interpolation in front of the Laplacian, a
 * sparser matrix with the same second order, the operator of Table 3.1):
 * A u = delta u - E_1 (N u) + gamma (E_1 u - E_3 u).  double device vectors of length
 * n(level), u and Au not overlapping; work holds n(level) doubles. */
cpm_status cpm_apply_pq(cpm_band band, int level, int p, double c, const double* u, double* Au, double* work,
                        void* stream);

/* One application of the extension: out = E g on one level (degree-3 closest-point
 * interpolation, Sec. 3.1).  double device vectors of length n(level), not overlapping. */
cpm_status cpm_extend(cpm_band band, int level, const double* g, double* out, void* stream);

/* Variable diffusion coefficient: -div_S(a grad_S u) + c u = f (Sec. 2.2; the variable-
 * coefficient sphere example, Sec. 4.6.6).  a is a host array of n(level)
 * doubles, a(cp(x_i)) > 0 for the nodes of `level` in band order (closest points from
 * cpm_band_export), copied.  The discrete operator is the flux form
 * L~ = sum over axes of D^b diag(A^f a) D^f, smoothed with the Ruuth-Merriman step on
 * cI - L~ (Jacobi, then the extension); a level's residual is r = D (E u~ - u), u~ the
 * undamped Jacobi step and D = c + sigma its diagonal, and the coarsest level solves the
 * smoother's fixed-point equation densely.  The coefficient takes effect once every level
 * has one; a = NULL (any level) removes it from all levels.  While set, solves accept
 * precision CPM_F64 with smoother CPM_SMOOTH_JACOBI only; relres is ||r|| / ||D E (f / D)||.
 * cpm_apply and the batched solver keep the constant-coefficient operator.  Synchronous. */
cpm_status cpm_set_diffusion(cpm_band band, int level, const double* a);

/* One V(nu1, nu2) cycle in place on u (Algorithm 4.1) for right-hand side f.  work has
 * cpm_workspace_size bytes.  If relres_out is not NULL the call synchronizes the stream
 * and stores ||E f - A u||_inf / ||E f||_inf of the new iterate (the relative increment
 * for the standard relaxation and CPM_RESIDUAL_VERBATIM).  Only precision CPM_F64 with smoother
 * CPM_SMOOTH_JACOBI, CPM_SMOOTH_STANDARD or CPM_SMOOTH_STANDARD_RB is accepted here. */
cpm_status cpm_vcycle(cpm_band band, const cpm_params* params, const double* f, double* u,
                      void* work, size_t work_bytes, double* relres_out, void* stream);

/* Repeat cycles from the given u (set it to 0 for the paper's start) until
 * ||E f - A u||_inf / ||E f||_inf < rtol or max_cycles.  Synchronous on return.  In
 * CPM_MIXED precision each outer step is one float32 V-cycle on the correction equation
 * A e = r with r evaluated in double.  With params->fmg the given u is replaced by the
 * full-multigrid start first (its one cycle per level is not counted in stats->cycles).
 * Returns CPM_E_NOCONV / CPM_E_DIVERGED with stats filled; CPM_E_NOCONV also before
 * max_cycles when the stopping quantity has not dropped below 0.99 of its best value for 8
 * cycles (it has reached the rounding floor of its evaluation: the residual's cancellation
 * between delta u and E(N u) grows like the 2d/h^2 of the finest level). */
cpm_status cpm_solve(cpm_band band, const cpm_params* params, const double* f, double* u,
                     void* work, size_t work_bytes, double rtol, int max_cycles,
                     cpm_stats* stats, void* stream);

/* Run a fixed number of cycles as one captured HIP graph launch per `cycles_per_launch`
 * cycles, without host synchronization between launches (throughput measurement).  The
 * relative residual after every cycle is written to relres_dev (device, >= cycles
 * doubles).  Same precision / smoother rules as cpm_solve. */
cpm_status cpm_run_cycles(cpm_band band, const cpm_params* params, const double* f, double* u,
                          void* work, size_t work_bytes, int cycles, int cycles_per_launch,
                          double* relres_dev, void* stream);

/* Average duration in microseconds of one launch of a V-cycle kernel on one level, timed
 * with HIP events on `stream` over `reps` back-to-back launches: which = 0 the
 * extension pass fused with Jacobi smoothing (the dominant kernel), 1 the neighbour-sum
 * pass, 2 restriction into `level` (level >= 1), 3 prolongation from level+1 into `level`
 * (level < levels-1), 4 the fused learned-smoother update from a fixed residual, held in
 * float32 as the learned sweep keeps it (level < 2,
 * weights set, CPM_E_INVALID otherwise), 5 the fused one-pass sweep (levels that have its
 * addressing, CPM_E_INVALID otherwise), 6 the tiled sweep (levels that have its tables,
 * CPM_E_INVALID otherwise).  Level 0 runs on f and u, other levels on workspace vectors; the
 * values left in u are those of repeated smoothing.  Synchronous. */
cpm_status cpm_time_kernel(cpm_band band, const cpm_params* params, int which, int level, int reps,
                           const double* f, double* u, void* work, size_t work_bytes, double* avg_us,
                           void* stream);

/* Batched solve of nprob independent problems (different surfaces, spacings and sizes)
 * with the same parameters (the mixed-precision iterative refinement of cpm_solve, Jacobi
 * smoother, V-cycles): every phase of the V-cycle runs as one launch over the tiles of all
 * problems, and 8 consecutive V-cycles of the whole batch are one captured HIP graph.
 * Each problem stops on the device, through its own flag, when it reaches rtol or
 * max_cycles, so it performs exactly the cycles of its own solve; the host reads the
 * number of finished problems once per graph launch.  The workgroup size of the batched
 * launches is timed on the first solve of a batch (its bands, their sizes, the device) and
 * reused by later solves of the same batch.  A problem with E f = 0 gets u = 0 and no
 * cycle.  f[k], u[k] are device vectors of problem k (u[k]: the start, normally 0);
 * work has cpm_workspace_size_batched bytes.  precision must be CPM_MIXED.  stats: nprob
 * entries (NULL allowed).  Returns CPM_E_NOCONV if any problem missed rtol,
 * CPM_E_DIVERGED if any residual was not finite.  Synchronous on return. */
cpm_status cpm_workspace_size_batched(int nprob, const cpm_band* bands, const cpm_params* params,
                                      size_t* bytes);
cpm_status cpm_solve_batched(int nprob, const cpm_band* bands, const cpm_params* params,
                             const double* const* f, double* const* u, void* work,
                             size_t work_bytes, double rtol, int max_cycles, cpm_stats* stats,
                             void* stream);

/* Autotuner: for every level, time the two passes of a smoothing sweep with each candidate
 * launch configuration on this band's addressing (extension: gathers with workgroups of
 * 128 / 256 / 512 lanes or LDS-staged; neighbour sum: 128 / 256 / 512 lanes), then the fused
 * one-pass sweep (E f + (E N) u, levels up to 2^21 nodes: gathers with 128 / 256 / 512 lanes
 * or LDS-staged) against that pair, and keep the fastest in the handle.  The environment
 * variables CPM_SWEEP=fused|split and CPM_SWEEP_LDS=0, read when the band is built, pin the
 * sweep form and keep the fused pass off LDS.  Allocates two temporary vectors;
 * synchronous. */
cpm_status cpm_autotune(cpm_band band, void* stream);

/* Launch configuration chosen for one level (after cpm_autotune, or the defaults); any
 * output pointer may be NULL.  fused = 1 when the level sweeps with the fused pass;
 * sweep_lds = 1 when that pass is LDS-staged (sweep_block is then its fixed 256 lanes);
 * tiled = 1 when the level sweeps with the tiled pass (3-D levels of 2^18 nodes or more whose
 * tables exist: f + N u formed in LDS over each tile's box, then the extension, one pass);
 * ext_prefetch = 1 when the LDS-staged extension loads each node's own data (band index, run
 * offsets, fractions, u) before its workgroup stages the interpolated values; ext_slots =
 * stencil slots per workgroup of the LDS-staged extension (its 256 lanes take 1, 2 or 4 slots
 * each, fixed when the band is built; 0 on a level without the staging tables). */
cpm_status cpm_band_tuning(cpm_band band, int level, int* use_lds, int* ext_block, int* nsum_block, int* fused,
                           int* sweep_block, int* sweep_lds, int* tiled, int* ext_prefetch, int* ext_slots);

/* Set one level's launch configuration by hand (for instance one found by cpm_autotune in
 * an earlier process): use_lds = LDS-staged extension (levels that have its tables),
 * ext_block / nsum_block / sweep_block in {128, 256, 512}, fused = sweep with the fused pass
 * (levels that have its addressing), sweep_lds = that pass LDS-staged (levels that have its
 * tables; its workgroup is then 256), tiled = sweep with the tiled pass (levels that have its
 * tables; not together with fused), ext_prefetch = the LDS-staged extension's early loads
 * (with use_lds only).  CPM_E_INVALID, with nothing changed, for a configuration the level
 * does not support.  Drops the band's captured cycle graphs. */
cpm_status cpm_set_band_tuning(cpm_band band, int level, int use_lds, int ext_block, int nsum_block, int fused,
                               int sweep_block, int sweep_lds, int tiled, int ext_prefetch);

/* ---- learned smoother ---------------------------------------------------------------
 * Network (per node): x = [r_patch / s (27 values: residual on the 3x3x3 grid patch
 * around the node, 0 outside the band, x fastest), the node's 12 one-dimensional cubic
 * weights (x, y, z; 4 each), 25 zeros] (64 features), s = max |r_patch| (update 0 when
 * s = 0); hidden = relu(W1 x + b1) (64), y = w2 . hidden + b2; update
 * u_i += (s / delta) * y.  W1 is 64 x 64 row-major (out, in), all weights bfloat16
 * (uint16 bit patterns), arithmetic float32. */
#define CPM_MLP_IN 64
#define CPM_MLP_HIDDEN 64
#define CPM_MLP_FEATURES 39

/* Copy weights (W1 64*64, b1 64, w2 64, b2 1, bf16 bit patterns) into the band handle;
 * the learned smoother uses them.  rho_plain is the per-cycle contraction of the plain
 * method above which the solve falls back to Jacobi. */
cpm_status cpm_set_smoother_weights(cpm_band band, const uint16_t* w_bf16, double rho_plain);

/* Forward pass on m feature rows: X (m x 64 bf16 bit patterns, device), W (device, same
 * packing as cpm_set_smoother_weights), Y (m floats, device), H (m x 64 floats, device,
 * hidden activations kept for the backward pass; may be NULL). */
cpm_status cpm_mlp_forward(int64_t m, const uint16_t* X, const uint16_t* W, float* Y, float* H,
                           void* stream);

/* Backward pass of the mean squared loss (1/m) sum (Y - T)^2 : gradients w.r.t. W1, b1,
 * w2, b2 in float32 (G, device, 64*64 + 64 + 64 + 1 floats, overwritten).  X, W as in the
 * forward pass, H and Y from it, T targets (m floats). */
cpm_status cpm_mlp_backward(int64_t m, const uint16_t* X, const uint16_t* W, const float* H,
                            const float* Y, const float* T, float* G, void* stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected with step >= 1) on the
 * float32 master weights w_master using gradient G; m1, m2 are the moment buffers (zero
 * before step 1); w_bf16 receives the rounded weights.  All device arrays of
 * 64*64 + 64 + 64 + 1 elements. */
cpm_status cpm_mlp_adam(int step, float lr, float* w_master, float* m1, float* m2, const float* G,
                        uint16_t* w_bf16, void* stream);

/* Features of the learned smoother for every node of level 0 or 1: the residual
 * r = E(f + N u) - delta u of (u, f) is evaluated in double, then X (n x 64 bf16, device,
 * rows in band order) and the patch scale s (n floats, device) are written.  work is a
 * device buffer of at least 2 n(level) doubles.  Used to generate training data from
 * plain solves. */
cpm_status cpm_smoother_features(cpm_band band, int level, double c, const double* f,
                                 const double* u, uint16_t* X, float* s, void* work,
                                 void* stream);

/* Training pairs of the learned smoother at every node of level 0 or 1: X and s as
 * cpm_smoother_features, and the target T (n floats, device) = r_i / s_i clipped to
 * [-clip, clip] (0 where s_i = 0), the undamped Ruuth-Merriman correction of u_i (eqs.
 * (4.2a)-(4.2b): u_i moves by r_i / delta with r = E f - A u, eq. (3.3)) in the network's
 * units.  work: at least 2 n(level) doubles (it keeps the residual in its second half). */
cpm_status cpm_smoother_pairs(cpm_band band, int level, double c, const double* f, const double* u, uint16_t* X,
                              float* T, float* s, double clip, void* work, void* stream);

/* Mean squared loss (1/m) sum (Y - T)^2 of m outputs against targets (device floats), summed
 * in double in a fixed order, into one device double. */
cpm_status cpm_mlp_loss(int64_t m, const float* Y, const float* T, double* loss, void* stream);

const char* cpm_status_string(int status);
const char* cpm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* CPM_H */
