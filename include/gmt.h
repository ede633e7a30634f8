/*
 * gmt.h -- C ABI of the MI355X periodic geometric-multigrid homogenization library.
 *
 * The library computes the effective stiffness C_H (6x6) of a periodic binary
 * voxel cell under linear elasticity, or the effective conductivity kappa_H
 * (3x3) under steady heat conduction, by solving the periodic cell problems
 * K u = f (paper Sec. 3.1, eq. linear_system; App. F) with a matrix-free,
 * element-by-element geometric multigrid on the sparse active-voxel hierarchy
 * (Sec. 4.1, Sec. 4.6, Alg. 1 / Alg. 2, App. E).
 *
 * Conventions (fixed by this library where the paper is silent):
 *   - a voxel cell is N^3 uint8 (0 = void, nonzero = solid), linear index
 *     x + N*(y + N*z), x fastest; voxel size 1, |Omega| = N^3;
 *   - levels are numbered as in the paper, l = 1 (finest) .. L (coarsest);
 *     level l has N_l = N / 2^(l-1) voxels per axis;
 *   - active elements / nodes of a level are sorted by linear index and
 *     identified by their rank (0-based id);
 *   - hex8 local corner a + 2b + 4c sits at offset (a, b, c) of its voxel;
 *   - a vector holds c load cases of d DOFs per node in the layout
 *     [n_n][c][d] row-major (elastic c = 6, d = 3, Voigt order
 *     11, 22, 33, 23, 13, 12 with engineering shear; thermal c = 3, d = 1);
 *   - gauge: the solution returned by gmt_solve has every DOF of node id 0
 *     of level 1 equal to zero (a translation of any solution).
 *
 * Memory and streams: every pointer named d_* is device memory owned by the
 * caller; h_* is host memory owned by the caller.  The hierarchy owns its
 * internal buffers (obtained through gmt_params.alloc when given, else
 * hipMalloc) and frees them in gmt_destroy.  Calls enqueue work on the given
 * hipStream_t (NULL = the null stream); calls that return host values
 * synchronize that stream before returning.  A hierarchy may be used from one
 * host thread at a time.
 *
 * Errors: every call returns a gmt_status; GMT_OK = 0.  Nothing aborts.
 * gmt_last_error() returns a thread-local message for the last failure.
 */
#ifndef GMT_H
#define GMT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GMT_OK = 0,
  GMT_E_INVAL = 1,    /* bad argument: size, level, dtype, null pointer, empty cell */
  GMT_E_NOMEM = 2,    /* an allocation failed */
  GMT_E_HIP = 3,      /* a HIP runtime call failed (message names it) */
  GMT_E_NOCONV = 4,   /* the iteration budget ran out or the residual went non-finite */
  GMT_E_SINGULAR = 5, /* coarsest-level Cholesky met a non-positive pivot */
  GMT_E_STATE = 6     /* call not valid for this hierarchy (e.g. wrong physics) */
} gmt_status;

typedef enum { GMT_ELASTIC = 0, GMT_THERMAL = 1 } gmt_physics;
typedef enum { GMT_F64 = 0, GMT_F32 = 1 } gmt_dtype;
/* Smoothers: Chebyshev iteration for D^-1 K, weighted Jacobi, and the
 * 8-colour Gauss-Seidel / SOR smoother of Sec. 4.6 (parallel smoothing): nodes
 * coloured by the parities of their coordinates, the colours updated in turn
 * with u_i += omega D_i^-1 r_i (D = diag K); the pre-smoother runs the colours
 * 0..7, the post-smoother 7..0 (its adjoint), so the cycle stays symmetric. */
typedef enum { GMT_SMOOTH_CHEBYSHEV = 0, GMT_SMOOTH_JACOBI = 1, GMT_SMOOTH_GS = 2 } gmt_smoother;

/* Multigrid schedules (Sec. 6.3, schedule study): per visit of a level, its
 * coarse correction problem gets one visit of the next level (V), two visits
 * in a row (W), or an F-visit followed by a V-visit (F).  The exact coarsest
 * solve is never repeated.  Injected corrections (Alg. 2) start a level at its
 * first entry in the cycle only. */
typedef enum { GMT_CYCLE_V = 0, GMT_CYCLE_W = 1, GMT_CYCLE_F = 2 } gmt_schedule;

typedef struct gmt_hier* gmt_hier_t;

/* Parameters of one cell.  Zero-initialise and set what you need; zero
 * fields take the defaults named below. */
typedef struct {
  int32_t physics;      /* gmt_physics */
  double E, nu;         /* isotropic solid (elastic); default E = 1, nu = 0.3 */
  double kappa;         /* conductivity (thermal); default 1 */
  int32_t levels;       /* L >= 1; N must be divisible by 2^(L-1) and N_L >= 2 */
  int32_t power_iters;  /* power iterations for lambda_max(D^-1 K); default 20 */
  uint64_t seed;        /* seed of the power-iteration start vector */
  /* optional allocator for the hierarchy's internal device buffers */
  void* (*alloc)(size_t bytes, void* ctx);
  void (*release)(void* ptr, void* ctx);
  void* alloc_ctx;
  /* gauge of the solutions gmt_solve reports (the cell problem fixes u only up to
   * a rigid translation per case): 0 (default) node 0 pinned, u(node 0) = 0;
   * 1 zero mean of every component over the fine nodes (the gauge of Sec. 4.5).
   * C_H does not depend on it. */
  int32_t gauge;
} gmt_params;

typedef struct {
  int32_t N;   /* voxels per axis on this level */
  int32_t n_e; /* active elements */
  int32_t n_n; /* active nodes */
  int32_t c;   /* load cases (6 elastic, 3 thermal) */
  int32_t d;   /* DOFs per node (3 elastic, 1 thermal) */
  double lambda_max; /* power-iteration estimate of the largest eigenvalue of D^-1 K */
  /* launch shape of this level's FP32 operator sweeps (the FP64 ones in
   * [1]), as chosen by the timing autotuner before the first solve (or the
   * defaults before it ran): kernel variant, workgroup size, 1 = workgroups
   * numbered XCD-contiguously */
  int32_t sweep_variant[2];
  int32_t sweep_block[2];
  int32_t sweep_xcd[2];
} gmt_level_desc;

/* Smoothing and schedule of one cycle.  For every level l (1..L-1) the
 * smoother is weighted Jacobi u += omega D^-1 (f - K u) (nu sweeps), the
 * degree-nu Chebyshev iteration for D^-1 K on [lo, hi], or nu 8-colour
 * Gauss-Seidel / SOR sweeps with weight omega.  Host arrays of length L
 * indexed by level-1; NULL arrays take the defaults omega = 4/(3 lambda_max)
 * (Jacobi) or 1 (Gauss-Seidel; SOR weights must lie in (0, 2)),
 * lo = lambda_max / 30, hi = 1.1 lambda_max.  Zero-initialised options give a
 * V-cycle with degree-2 Chebyshev smoothing. */
typedef struct {
  int32_t nu1, nu2;   /* pre / post smoothing degree; default 2 / 2 when both 0 */
  int32_t smoother;   /* gmt_smoother */
  const double* omega;
  const double* lo;
  const double* hi;
  int32_t schedule;   /* gmt_schedule */
} gmt_cycle_opts;

typedef struct {
  double tol;         /* stop when max_m ||f_m - K u_m|| / ||f_m|| <= tol (FP64); default 1e-5 */
  int32_t max_iter;   /* total inner PCG iterations; default 500 */
  int32_t precision;  /* GMT_F64: all-FP64; GMT_F32: FP32 inner PCG + FP64 refinement.
                         An ill-conditioned cell leaves the FP32 recurrence: when an FP32
                         inner solve stalls or passes 120 iterations short of its target
                         (its update is kept), or an FP32 step does not halve the FP64
                         residual (that step is undone), the solve continues with FP64
                         CG vectors, dot products and K.p around the FP32 V-cycle. */
  int32_t max_outer;  /* FP64 refinement steps; default 8 */
  int32_t check_every;/* inner convergence check period (host sync); default 1 */
  gmt_cycle_opts cycle;
  int32_t graph;      /* 1: inner PCG iterations run as replays of captured hipGraph
                         blocks of 1 or 4 iterations (host check between blocks);
                         0: kernel-by-kernel launches, check every check_every */
  int32_t zero_start; /* 1: start from u = 0 whatever d_u holds on entry (the first
                         residual is then f itself: no operator sweep, no layout pass
                         over d_u); 0: start from d_u */
} gmt_solve_opts;

typedef struct {
  int32_t iterations;      /* inner PCG iterations (V-cycles) spent */
  int32_t outer;           /* FP64 residual evaluations / refinement steps */
  int32_t converged;       /* 1 when max_m rel_res[m] <= tol */
  int32_t c;               /* load cases reported */
  double rel_res[6];       /* final FP64 relative residual per case */
  double rel_res_init[6];  /* FP64 relative residual of the initial guess */
} gmt_solve_report;

/* Sec. 4.1 (active set, occupancy, eq. gmgcoarsenode) and App. E.1 (transfer
 * stencils), plus the Galerkin operators of Sec. 4.6, the Jacobi diagonal, a
 * lambda_max estimate per level and the factor of the pinned coarsest matrix.
 * d_voxels: N^3 uint8 on the device.  Fails with GMT_E_INVAL for an empty
 * cell or bad N / levels, and for a cell whose solid voxels form more than one
 * node-connected component (periodic; voxels sharing a node are connected):
 * each component could translate on its own and one pinned node fixes only
 * one of them (the message names the count).  GMT_E_SINGULAR if the coarsest
 * factorisation fails. */
gmt_status gmt_build_hierarchy(const uint8_t* d_voxels, int32_t N, const gmt_params* params,
                               void* stream, gmt_hier_t* out);

void gmt_destroy(gmt_hier_t h);

gmt_status gmt_level_info(gmt_hier_t h, int32_t level, gmt_level_desc* out);

/* Exports the integer maps of one level (Sec. 4.1.1, eq. gmgcoarsenode; App. E.2
 * stencil tuple).  Any pointer may be NULL to skip it.  Sizes: elem_lin[n_e],
 * node_lin[n_n], occ8[n_n] (bit a+2b+4c set iff the element at offset
 * (a-1, b-1, c-1) from the node is active), elem_nodes[n_e][8],
 * prol_idx[n_n][8] and prol_w[n_n][8] (level < L only: id of coarse corner
 * o_k = (k&1, k>>1&1, k>>2&1) of the parent cell, -1 / 0.0 where w_k = 0). */
gmt_status gmt_export_maps(gmt_hier_t h, int32_t level, int32_t* d_elem_lin, int32_t* d_node_lin,
                           uint8_t* d_occ8, int32_t* d_elem_nodes, int32_t* d_prol_idx,
                           double* d_prol_w, void* stream);

/* Galerkin element matrices of level l >= 2 (Sec. 4.6, K_c = R_loc K_patch P_loc):
 * d_K[n_e][8d][8d] FP64.  Level 1 returns the voxel K_e for every element. */
gmt_status gmt_export_element_matrices(gmt_hier_t h, int32_t level, double* d_K, void* stream);

/* diag(K^l) as d_D[n_n][d] FP64. */
gmt_status gmt_export_diagonal(gmt_hier_t h, int32_t level, double* d_D, void* stream);

/* f = sum_e A_e^T K_e X0 (App. F.1 f_e = K_e X0, X0 the affine unit-strain field),
 * d_f[n_n][c][d] of level 1 in dtype. */
gmt_status gmt_load_vector(gmt_hier_t h, void* d_f, int32_t dtype, void* stream);

/* y = K^l u = sum_e A_e^T K_e A_e u, matrix-free (Sec. 4.6). */
gmt_status gmt_apply_K(gmt_hier_t h, int32_t level, const void* d_u, void* d_y, int32_t dtype,
                       void* stream);

/* r = f - K^l u. */
gmt_status gmt_residual(gmt_hier_t h, int32_t level, const void* d_f, const void* d_u, void* d_r,
                        int32_t dtype, void* stream);

/* nu smoothing steps on level l < L in place on d_u (weighted Jacobi with
 * omega = p1; Chebyshev on [lo, hi] = [p1, p2]; Gauss-Seidel / SOR with
 * omega = p1, colours 0..7 when p2 = 0 (pre-smoother) or 7..0 when p2 = 1
 * (post-smoother)); the pre- and post-smoother of Alg. 1. */
gmt_status gmt_smooth(gmt_hier_t h, int32_t level, const void* d_f, void* d_u, int32_t nu,
                      int32_t smoother, double p1, double p2, int32_t dtype, void* stream);

/* f_{l+1} = R r_l with R = P^T, unscaled, in gather form (App. E.2). */
gmt_status gmt_restrict(gmt_hier_t h, int32_t level, const void* d_rf, void* d_fc, int32_t dtype,
                        void* stream);

/* u_l += P u_{l+1} (App. E.2 weighted gather). */
gmt_status gmt_prolong_add(gmt_hier_t h, int32_t level, const void* d_uc, void* d_uf, int32_t dtype,
                           void* stream);

/* Exact solve of the coarsest level: node 0's DOFs pinned to zero, RHS there
 * ignored, u = K_L,pinned^-1 f (replaces the coarsest GS of Alg. 1/2). */
gmt_status gmt_coarse_solve(gmt_hier_t h, const void* d_f, void* d_u, int32_t dtype, void* stream);

/* One cycle (Alg. 2; V, W or F by opts->schedule) in place on d_u (level-1
 * vector, its initial guess u^1).
 * d_e_init: NULL, or an array of L pointers indexed by level-1 whose entries
 * 2..L-1 (indices 1..L-2) may be NULL or point to injected corrections
 * e^l[n_n^l][c][d] (the coarse-level injection of Alg. 2); entry L is unused (exact
 * coarsest solve). */
gmt_status gmt_vcycle(gmt_hier_t h, const void* d_f, void* d_u, const void* const* d_e_init,
                      const gmt_cycle_opts* opts, int32_t dtype, void* stream);

/* Solve K u = f to opts->tol (relative residual, Sec. 5.2, evaluated in FP64)
 * by conjugate gradients preconditioned with one cycle per iteration
 * (opts->cycle: V or W, both symmetric; F is rejected with GMT_E_INVAL),
 * starting from the guess in d_u (zeros = the plain solver).  d_f and d_u are
 * FP64 level-1 vectors; on return d_u holds the solution in the gauge
 * u(node 0) = 0.  A guess whose residual is not finite, or larger than the
 * load itself (worse than the zero guess), is replaced by zero before the
 * first iteration (rel_res_init still reports it).  Returns GMT_E_NOCONV
 * (with the report filled) when the budget is spent.  Synchronizes the
 * stream. */
gmt_status gmt_solve(gmt_hier_t h, const void* d_f, void* d_u, const gmt_solve_opts* opts,
                     gmt_solve_report* report, void* stream);

/* Batched solve of n independent cells (each its own hierarchy: any N,
 * elastic or thermal, any number of levels), the same problem as gmt_solve
 * for each: d_f[i] / d_u[i] are that cell's FP64 level-1 vectors.  Cells are
 * taken largest first from one shared queue by n_workers host threads (<= 0:
 * 4), each driving its own HIP stream, so small cells overlap on the GPU; each
 * cell's inner PCG replays captured hipGraph blocks when opts->graph is set.
 * All work buffers are allocated on the calling thread before the workers
 * start.  reports[i] / status[i] (either may be NULL) receive each cell's
 * outcome; the call returns the first non-OK status (GMT_E_NOCONV included)
 * or GMT_OK.  The caller's stream is synchronized first; the call returns when
 * every cell is done. */
gmt_status gmt_solve_batch(gmt_hier_t const* hs, int32_t n, const void* const* d_f, void* const* d_u,
                           const gmt_solve_opts* opts, int32_t n_workers, gmt_solve_report* reports,
                           gmt_status* status, void* stream);


/* h_rel[c] = ||f_m - K u_m||_2 / ||f_m||_2 per case in FP64 (a case whose load
 * is below 1e-12 of the largest case is normalised by the largest ||f||). */
gmt_status gmt_relative_residual(gmt_hier_t h, const void* d_f, const void* d_u, int32_t dtype,
                                 double* h_rel, void* stream);

/* Effective tensor (App. F.1 / F.2):
 * C_H = 1/N^3 sum_e (X0 - u_e)^T K_e (X0 - u_e), evaluated in FP64 through the
 * equivalent assembled form (n_e C0 - F^T U - U^T F + U^T K U) / N^3.
 * h_CH: c x c row-major host array.  Synchronizes the stream. */
gmt_status gmt_homogenize(gmt_hier_t h, const void* d_u, int32_t dtype, double* h_CH, void* stream);

/* ------------------------------------------------------------------------
 * SIMP inverse homogenization (App. F.3).  A density field rho (one value per
 * voxel element, rho_min <= rho <= 1) gives every element the tensor
 * C_e = (rho_min + rho_e^p) C0 (eq. ch): element matrix s_e K0.  Elements with
 * rho_e <= prune are left out of the active set (pruning of near-void voxels).
 * The hierarchy of such a cell is built by gmt_build_density_hierarchy and then
 * used with every call above (gmt_load_vector gives f = sum_e s_e A_e^T K0 X0,
 * gmt_homogenize the C_H of the scaled elements, gmt_solve the GMG-PCG with
 * Galerkin operators of the scaled elements), except the learned initializer
 * (gmt_nn_setup: binary cells only) and level-1 gmt_export_element_matrices.
 * ------------------------------------------------------------------------ */
typedef struct {
  double p;        /* penalization exponent, >= 1 (e.g. 3) */
  double rho_min;  /* additive stiffness floor, > 0 */
  double prune;    /* elements with rho <= prune are inactive, 0 <= prune < 1 */
} gmt_simp_params;

/* d_rho: device FP64 [N^3], x fastest (the voxel order of gmt_build_hierarchy).
 * params->levels >= 2.  Errors as gmt_build_hierarchy. */
gmt_status gmt_build_density_hierarchy(const double* d_rho, int32_t N, const gmt_simp_params* sp,
                                       const gmt_params* params, void* stream, gmt_hier_t* out);

/* Analytic sensitivities (App. F.3) from a solution d_u (device FP64, ABI
 * layout [n_n][c][d], level 1): with d_e = X0 - u_e and g_e = p rho_e^(p-1) / N^3,
 * d_dC (device [N^3][c][c] or NULL) receives dC_H[i][j]/drho_e = g_e d_e^(i)T K0 d_e^(j),
 * d_dJ (device [N^3] or NULL) receives dJ/drho_e = sum_ij h_G[i][j] dC_H[i][j]/drho_e
 * for host weights h_G = dJ/dC_H (c x c row-major; required with d_dJ).  Both are
 * dense over the voxel grid, zero for inactive elements.  Synchronizes the stream.
 * GMT_E_STATE for a binary hierarchy. */
gmt_status gmt_simp_sensitivity(gmt_hier_t h, const double* d_u, const double* h_G, double* d_dJ, double* d_dC,
                                void* stream);

/* Objectives of App. F.3 on the compliance S = C_H^-1 (elastic 6x6, host):
 * GMT_SIMP_YOUNG  J = (S00 + S11 + S22) / 3,  GMT_SIMP_SHEAR  J = (S33 + S44 + S55) / 3,
 * GMT_SIMP_BULK   J = sum_{i,j < 3} Sij;  h_G = dJ/dC_H = -S^T W S^T (6x6 row-major).
 * GMT_E_SINGULAR when C_H is singular. */
typedef enum { GMT_SIMP_YOUNG = 0, GMT_SIMP_SHEAR = 1, GMT_SIMP_BULK = 2 } gmt_simp_objective_kind;
gmt_status gmt_simp_objective(const double* h_CH, int32_t kind, double* h_J, double* h_G);

/* Sensitivity filter on the dense periodic N^3 grid (device FP64, x fastest):
 * out_e = sum_f H_ef rho_f dc_f / (max(1e-3, rho_e) sum_f H_ef),
 * H_ef = max(0, rmin - |x_e - x_f|) over periodic voxel distances, 1 < rmin <= 8.
 * d_out must not alias the inputs. */
gmt_status gmt_simp_filter(const double* d_rho, const double* d_dc, int32_t N, double rmin, double* d_out,
                           void* stream);

/* Optimality-Criteria step with move limits on n densities (device FP64):
 * rho_new = min(1, rho + move, max(rho_lo, rho - move, rho (max(-dc, 0) / lam)^eta)),
 * lam found by bisection on [0, 1e9] so that sum(rho_new) = volfrac * n
 * (h_lambda receives it).  Synchronizes the stream; d_rho_new must not alias. */
gmt_status gmt_simp_oc(const double* d_rho, const double* d_dc, size_t n, double volfrac, double move, double eta,
                       double rho_lo, double* d_rho_new, double* h_lambda, void* stream);

/* ------------------------------------------------------------------------
 * Learned initializer (Sec. 4.2-4.5 with a sparse-convolution backbone): a
 * U-Net on the same active node sets P_1..P_L, periodic neighbour maps, the
 * 8-bit occupancy embedded by a 256-entry table, learned 27-tap pooling from
 * the fine nodes 2x + k and unpooling along the same connectivity, and a
 * three-layer head per level l < L that predicts u_hat^1 (l = 1) and the
 * corrections e_hat^l (1 < l < L).  BF16 weights and activations, FP32 sums.
 *
 * Flat FP32 parameter layout (caller-owned), in this order:
 *   E [256][C1];  for l = 1..L: We_l [27][C_l][C_l], be_l [C_l];
 *   for l = 1..L-1: Wp_l [27][C_l][C_{l+1}], bp_l [C_{l+1}], Wu_l [27][C_{l+1}][C_l],
 *   bu_l [C_l], Wd_l [27][C_l][C_l], bd_l [C_l], W1_l [C_l][H], b1_l [H], W2_l [H][H],
 *   b2_l [H], W3_l [H][q], b3_l [q]      (q = c*d; tap t <-> offset (t%3-1, t/3%3-1, t/9-1));
 *   with cfg.attention = 1, after all of the above: for l = 1..L: Wq_l, Wk_l, Wv_l,
 *   Wo_l, each [C_l][C_l].
 *
 * Attention blocks (cfg.attention = 1; Sec. 4.2-4.3, the paper's serialized
 * window attention with Ra-RoPE): after the encoder convolution of level l,
 *   q = bf16(a Wq), k = bf16(a Wk), v = bf16(a Wv),
 *   o = bf16(Attn(q, k, v)),  s = bf16(a + o Wo),
 * and s takes the place of a as the pooling input, the decoder skip and (at
 * the coarsest level) the decoder's start.  Attn is softmax attention with
 * heads of 8 channels (C_l / 8 heads) inside windows of W_l = min(256 * 2^(l-1),
 * 1024) consecutive nodes of the level's serialization: the Morton order of
 * the node coordinates under the cyclic view (l-1) mod 3 of the axes
 * ((x, y, z), (y, z, x), (z, x, y); bit b of the view's first, second, third
 * coordinate at code bit 3b, 3b+1, 3b+2).  Queries and keys are rotated per
 * channel pair k of a head by 2 pi (k div 3 + 1) p_{k mod 3} / N_l, p the
 * node's coordinates on the level (Ra-RoPE: exactly periodic).  Scores are
 * scaled by 1/sqrt(8); sums and the softmax in FP32.
 * ------------------------------------------------------------------------ */
#define GMT_NN_MAX_LEVELS 8
typedef struct {
  int32_t levels;                       /* 2..the hierarchy's L: the network runs on levels 1..levels */
  int32_t channels[GMT_NN_MAX_LEVELS];  /* C_l in {16, 32, 64} */
  int32_t head;                         /* H = 32 */
  int32_t attention;                    /* 0: convolutional U-Net; 1: with an attention block per level */
} gmt_nn_config;

/* Number of FP32 parameters of the network for a physics (q = 18 or 3). */
gmt_status gmt_nn_param_count(const gmt_nn_config* cfg, int32_t physics, size_t* n_params);

/* Builds the network's neighbour tables and activation buffers for a hierarchy. */
gmt_status gmt_nn_setup(gmt_hier_t h, const gmt_nn_config* cfg, void* stream);

/* Forward pass.  With L' = cfg.levels: d_out is an array of L' pointers indexed
 * by level-1; entry l-1 (l = 1..L'-1) receives the level-l prediction
 * [n_l][c][d] FP32 (u_hat^1 for l = 1, e_hat^l otherwise) or is NULL to skip
 * it; entry L'-1 is unused.  (L' < L: a network of fewer levels than the
 * hierarchy, e.g. trained on coarser cells, predicts for levels 1..L'-1 only.)
 * Every prediction is centred: the mean over the level's nodes of each of its
 * c*d columns is removed (zero-mean gauge, Sec. 4.5). */
gmt_status gmt_nn_forward(gmt_hier_t h, const float* d_params, float* const* d_out, void* stream);

/* Backward pass of the last forward: d_grad += d/dparams sum_l <d_gout[l], out[l]>
 * (same indexing as gmt_nn_forward; NULL entries contribute nothing). */
gmt_status gmt_nn_backward(gmt_hier_t h, const float* const* d_gout, float* d_grad, void* stream);

/* Inspection of the last forward: copies one stored BF16 activation of
 * level l (1..L), widened to FP32 [n_l][width], into d_out.  which: 0 = h
 * (encoder input), 1 = a (encoder output), 2 = t (decoder merge), 3 = d
 * (decoder output), 4 = z1, 5 = z2 (head hidden layers); 2..5 exist for
 * l < L only.  With attention blocks also: 6 = s (block output, node order),
 * and, in serialization order (row r is node order[r]), 7 = q, 8 = k, 9 = v
 * (BF16) and 10 = the FP32 attention output before its BF16 rounding; 6 is a
 * itself without attention, 7..10 fail with GMT_E_STATE.  h_width receives the
 * row width (C_l, or the head width). */
gmt_status gmt_nn_activation(gmt_hier_t h, int32_t level, int32_t which, float* d_out, int32_t* h_width,
                             void* stream);

/* Supervised term of training on solved cells (the plain solver's solution as
 * the target of u_hat^1; used with the label-free loss of gmt_vcycle_loss):
 * with t_c the target d_target [n_1][c][d] (FP32) centred per column like the
 * predictions, h_loss = alpha |d_pred - t_c|^2 / |t_c|^2 (FP64 sums in a fixed
 * order), and, if d_grad is not NULL, d_grad += its gradient with respect to
 * d_pred (the gradient to pass, with the V-cycle loss's, to gmt_nn_backward).
 * GMT_E_INVAL for a target that is zero after centring.  Synchronizes. */
gmt_status gmt_nn_supervised_loss(gmt_hier_t h, const float* d_pred, const float* d_target, double alpha,
                                  float* d_grad, double* h_loss, void* stream);

/* Serialization of level l (1..cfg.levels) of a network set up with attention:
 * d_order[r] (n_l int32, device) receives the node id of rank r in the level's
 * Morton order (view (l-1) mod 3).  GMT_E_STATE without attention blocks. */
gmt_status gmt_nn_serialization(gmt_hier_t h, int32_t level, int32_t* d_order, void* stream);

/* AdamW step on FP32 master weights (bias-corrected moments, step >= 1,
 * decoupled weight decay wd, gradient multiplied by grad_scale first). */
gmt_status gmt_nn_adamw(float* d_params, const float* d_grad, float* d_m, float* d_v, size_t n, double lr,
                        double beta1, double beta2, double eps, double wd, int32_t step, double grad_scale,
                        void* stream);

/* Training helpers on flat FP32 vectors: h_out = ||d_x||_2^2 (FP64 sum), and
 * the exponential moving average d_ema = decay * d_ema + (1 - decay) * d_x. */
gmt_status gmt_nn_norm2(const float* d_x, size_t n, double* h_out, void* stream);
gmt_status gmt_nn_ema(float* d_ema, const float* d_x, size_t n, double decay, void* stream);

/* gmt_nn_norm2 without any allocation, for callers that cannot allocate device
 * memory (code under graph capture, tight training loops, allocator-free
 * harnesses).  Same result as gmt_nn_norm2 (FP64 partial sums per 2048 values,
 * summed in a fixed order).  The partial sums live in one fixed device array of
 * the library (8192 FP64 partials + the total, 64 KiB per GPU, kept until the
 * process ends), so n is limited to 8192 * 2048 = 16 777 216 values: a larger n
 * returns GMT_E_INVAL before anything is launched.  The array is per GPU and
 * shared by every call on it: calls that overlap on one GPU (other streams or
 * threads) race and must be serialised by the caller.  Synchronizes the stream. */
gmt_status gmt_nn_norm2_noalloc(const float* d_x, size_t n, double* h_out, void* stream);

/* One V-cycle of Alg. 2 (Chebyshev or Jacobi smoothing; other smoothers and
 * schedules are rejected with GMT_E_INVAL) started from network outputs, in FP32, and the
 * physics loss of Sec. 4.5:  L = log10(||f - K u^1||_2 + 1e-12)
 * + lambda * sum_{case,dof} (sum_i u^1_i)^2  (norm over all cases and DOFs).
 * d_pred: L pointers by level-1 (entry 0 = u_hat^1 [n_1][c][d], required;
 * entries 1..L-2 = e_hat^l or NULL) FP32.  Outputs (each optional): d_u1, the
 * V-cycle result [n_1][c][d] FP32; h_out[0] = loss, h_out[1] = ||r||, and
 * h_out[2..2+c) the per-case relative residuals; d_gpred (same indexing as
 * d_pred, NULL entries skipped) receives dL/d(pred) through the exact adjoint
 * of the V-cycle.  Synchronizes the stream. */
gmt_status gmt_vcycle_loss(gmt_hier_t h, const float* const* d_pred, const gmt_cycle_opts* opts,
                           double lambda, float* d_u1, double* h_out, float* const* d_gpred, void* stream);

/* Instrumentation (tracing/profiling): times `reps` Chebyshev sweeps of
 * level l (the fused K.u + smoother update, on internal FP32 or FP64 work
 * vectors, no layout staging) with HIP events recorded on the given stream and
 * returns the mean duration of one sweep in h_ms.  Level 1 sweeps launch two
 * kernels (all-solid interior nodes, boundary nodes).  Synchronizes the stream. */
gmt_status gmt_time_sweep(gmt_hier_t h, int32_t level, int32_t reps, int32_t dtype, double* h_ms,
                          void* stream);

/* Instrumentation: after a gmt_nn_forward of a network with attention blocks,
 * times `reps` launches of level l's window-attention forward kernel on the
 * stored q, k, v (rewriting the same outputs) with HIP events on the given
 * stream; h_ms receives the mean duration of one launch.  GMT_E_STATE without
 * attention blocks.  Synchronizes the stream. */
gmt_status gmt_nn_time_attention(gmt_hier_t h, int32_t level, int32_t reps, double* h_ms, void* stream);

const char* gmt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GMT_H */
