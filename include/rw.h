/* rw.h — C ABI of the MI355X random-walker solver (librw.so).
 *
 * Problem (random-walker segmentation, the operator the paper lists in
 * Sec. III-A and benchmarks hierarchically in Sec. IV-B, Table III):
 *   6-connected voxel grid, Gaussian edge weights
 *       w_ij = exp(-beta (g_i - g_j)^2) + w_eps,
 *   g = (v - norm_lo) / (norm_hi - norm_lo) the normalised intensity;
 *   L = D - W; seeded voxels M carry Dirichlet data m^s = [label == s];
 *   every label s solves L_U x^s = -B^T m^s on the unseeded voxels U by
 *   Jacobi-preconditioned conjugate gradients, stopped when
 *   ||r|| <= tol ||b||.  Edges never leave the volume.
 *
 * Layout: every grid is C order [nz][ny][nx], x fastest; multi-grid arrays
 * are planar, [count][nz][ny][nx].  Labels: uint8, 0 = unseeded, 1..K = seed
 * label, label 1 = background.
 *
 * Ownership: every data pointer is caller-owned DEVICE memory unless marked
 * "host".  The library never allocates device memory for data: scratch comes
 * from the caller's workspace (rw_*_workspace_bytes).  A context owns only a
 * private HIP stream, events, a small pinned host buffer for convergence
 * polling, and cached graph executables.
 *
 * Streams: `stream` is a hipStream_t passed as void* (NULL = the legacy
 * default stream).  Work runs on the context's stream, ordered after all work
 * already queued on `stream`, and `stream` is made to wait for it.  Calls that
 * poll convergence return after their device work is complete.  Calls on one
 * context must not overlap (one host thread per context).
 *
 * Errors: negative statuses are failures, detected before any output is
 * written unless stated; RW_NOT_CONVERGED (positive) means the last iterate
 * was written.  rw_last_error() gives a per-thread message.
 */
#ifndef RW_H_
#define RW_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RW_MAX_LABELS 16

typedef enum {
    RW_OK = 0,
    RW_NOT_CONVERGED = 1,     /* max_iter reached: last iterate written, stats valid */
    RW_ERR_INVALID_ARG = -1,  /* null pointer, bad size, bad option, label > K */
    RW_ERR_NO_SEEDS = -2,     /* no seed at all, or a solved label has no seed */
    RW_ERR_SINGULAR = -3,     /* an unseeded voxel has zero degree (all weights 0) */
    RW_ERR_BREAKDOWN = -4,    /* CG breakdown: p.Ap <= 0 or not finite */
    RW_ERR_NONFINITE = -5,    /* NaN/Inf in the input or in the weights */
    RW_ERR_WORKSPACE = -6,    /* workspace missing or smaller than required */
    RW_ERR_HIP = -7,          /* a HIP runtime call failed (see rw_last_error) */
    RW_ERR_UNSUPPORTED = -8   /* combination of options not implemented */
} rw_status;

typedef enum { RW_DT_U16 = 1, RW_DT_F32 = 2, RW_DT_F64 = 3 } rw_dtype;

typedef enum {
    RW_PREC_FP64 = 0,  /* float64 weights, vectors and reductions */
    RW_PREC_MIXED = 1  /* float32 weights and vectors, float64 dot products,
                          float64 residual + iterative refinement */
} rw_precision;

/* Grid size in voxels.  Supported grids: every side in [1, 2^30], a plane
 * nx * ny of at most 2^29 voxels and at most 2^40 voxels in all; calls given
 * larger grids return RW_ERR_INVALID_ARG before any device work, and the
 * workspace-size functions return 0. */
typedef struct {
    int64_t nx, ny, nz;
} rw_dims;

/* Input volume.  g = (v - norm_lo) / (norm_hi - norm_lo); norm_hi <= norm_lo
 * means a constant image (g = 0, all weights 1 + w_eps). */
typedef struct {
    const void* data; /* device, [nz][ny][nx] of `dtype` */
    int32_t dtype;    /* rw_dtype */
    rw_dims dims;
    double norm_lo, norm_hi;
} rw_volume;

typedef struct {
    const uint8_t* labels; /* device, [nz][ny][nx]; 0 = unseeded, 1..num_labels */
    int32_t num_labels;    /* K, 1 <= K <= RW_MAX_LABELS */
} rw_seeds;

typedef struct {
    double beta;          /* >= 0 */
    double w_eps;         /* added to every weight; >= 0 in normal use */
    double tol;           /* relative residual, > 0 (1e-6) */
    double inner_tol;     /* mixed, refine_mode 1: relative tolerance of the
                             refinement steps after the first (1e-3) */
    double update_delta;  /* mixed, refine_mode 0: the residual is recomputed in
                             float64 whenever the recurrence residual has fallen
                             by this factor since the last recomputation (0.1;
                             volume time series converge far sooner at 0.5, whose
                             float32 recurrence drifts faster) */
    int32_t max_iter;     /* CG iterations per label and call (20000) */
    int32_t max_refine;   /* mixed, refine_mode 1: refinement steps (5) */
    int32_t precision;    /* rw_precision */
    int32_t solve_all_labels; /* 0: solve labels 2..K, background = 1 - sum;
                                 1: solve all K labels independently */
    int32_t check_interval;   /* CG iterations between convergence polls (16) */
    int32_t use_graph;        /* 1: replay each poll interval as a HIP graph */
    int32_t kernel_timing;    /* 1: time every CG pass with events (no graph) */
    int32_t refine_mode;      /* mixed: 0 = one CG run whose residual is
                                 recomputed in float64 as it falls (reliable
                                 updates), 1 = restarted iterative refinement */
    const void* x0;       /* device, initial guess or NULL.  rw_solve: [R][nz][ny][nx]
                             float64 for the solved labels (NULL = 0); rw_solve_bricks:
                             [K][fine voxels] float32 as prob_out (NULL = upsampled
                             coarse).  Read on unseeded voxels. */
    int64_t brick_voxels; /* rw_solve_bricks, rw_autotune_bricks: voxels of the
                             level's nominal (unclipped) brick, the key of the tile
                             table, so that a batch of clipped border bricks (a
                             region of interest, a seed edit) runs on the same
                             tiles, and so the same reduction order, as the whole
                             level; 0 = the largest brick of the batch */
} rw_options;

/* Statistics of one call (host memory). */
typedef struct {
    int32_t iters[RW_MAX_LABELS];        /* CG iterations per solved label (summed over
                                            refinement steps) */
    int32_t label_status[RW_MAX_LABELS]; /* per solved label: rw_status */
    double rel_residual[RW_MAX_LABELS];  /* final true float64 ||b - Ax|| / ||b|| */
    int32_t num_solved;                  /* R */
    int32_t refinements;                 /* mixed: float64 residual recomputations
                                            after the first */
    int32_t tile_by, tile_zc;            /* stencil tile used (64 vx x by columns,
                                            zc planes; vx and xcd at the end) */
    double device_ms;                    /* whole call on the device (events) */
    double loop_ms;                      /* CG iteration loops only */
    /* kernel_timing = 1: summed durations of the CG passes over the iterations
       in which at least one label was still iterating, their launch count,
       and sum over those iterations of the number of labels iterating */
    double pass_ms[2];
    int64_t pass_launches[2];
    int64_t rhs_iterations;
    /* algorithmic work of the CG passes: sum over the launches that did work
       of the voxels of the boxes (volume or bricks) with a label iterating,
       and of those voxels times the number of labels iterating */
    int64_t box_voxel_iterations;
    int64_t rhs_voxel_iterations;
    int64_t active_bricks;               /* brick solves: bricks solved */
    int64_t unknowns;                    /* unseeded voxels solved for */
    int32_t tile_vx;                     /* columns per lane (1, 2, 4) */
    int32_t tile_xcd;                    /* 1: XCD-aware tile order */
    int32_t brick_blocks;                /* brick solves: blocks of the one persistent
                                            launch (0: one launch per CG pass) */
    int32_t tile_tuned;                  /* 1: the tile shape came from the autotuner's
                                            table (librw.tune), 0: the built-in default */
    int32_t tile_by2, tile_zc2;          /* rows and planes of CG pass 2's tiles (whole
                                            volumes may run pass 2 on other tiles than
                                            pass 1) */
} rw_stats;

/* Fine-level brick: origin and size in voxels of the fine grid (or of its
 * sub-volume, see rw_subvolume). */
typedef struct {
    int32_t ox, oy, oz, sx, sy, sz;
} rw_brick;

/* A brick's own volume in a pool (streamed solves): a box of the fine grid
 * stored contiguously, C order, starting at element `offset` of the pool's
 * intensity, label and output arrays; (gx, gy, gz) is the global fine
 * position of its origin.  Its faces are the volume's faces for the solver
 * (no edge leaves it), so a brick with a one-voxel halo on every side that
 * is inside the global volume sees exactly its global neighbourhood. */
typedef struct {
    int64_t offset;
    int32_t nx, ny, nz;
    int32_t gx, gy, gz;
} rw_subvolume;

typedef struct rw_context rw_context;

/* Context: creates a private stream on the current device. */
rw_status rw_context_create(rw_context** out);
void rw_context_destroy(rw_context* ctx);

const char* rw_status_string(rw_status s);
const char* rw_last_error(void);
void rw_default_options(rw_options* opts);

/* Output assembly (the segmentation is the label of highest probability,
 * Sec. IV-B): labels_out[i] = argmax over L of prob[L-1][i], lowest label on
 * ties.  prob: device [K][n] float32 (RW_DT_F32) or float64 (RW_DT_F64);
 * labels_out: device uint8 [n], values 1..K.  Invalid arguments return
 * RW_ERR_INVALID_ARG before any device work. */
rw_status rw_argmax(rw_context* ctx, const void* prob, int32_t dtype, int32_t num_labels,
                    int64_t n, uint8_t* labels_out, void* stream);

/* Normalisation range (min, max) of a volume, computed on the device.
 * lo_hi: host, 2 doubles.  NaN in the volume -> RW_ERR_NONFINITE. */
rw_status rw_minmax(rw_context* ctx, const rw_volume* vol, double* lo_hi, void* stream);

/* Materialised edge weights and Jacobi inverse diagonal.
 * w_out: [3][nz][ny][nx] (float64 for RW_PREC_FP64, float32 for MIXED);
 *   w_out[a][v] is the weight of edge (v, v + e_a), a = 0 (x), 1 (y), 2 (z);
 *   the last plane along each axis is 0 (no edge).
 * dinv_out: NULL or [nz][ny][nx] of the same type: 1 / sum of the (up to six)
 *   weights at v when v is unseeded, 0 on seeds (seeds must then be given). */
rw_status rw_build_weights(rw_context* ctx, const rw_volume* vol, double beta, double w_eps,
                           int32_t precision, void* w_out, void* dinv_out,
                           const rw_seeds* seeds_or_null, void* stream);

/* The operator q = L_U p of the Dirichlet system, matrix free, weights
 * recomputed from the volume (the CG kernel's own stencil).  p: [nz][ny][nx]
 * float64 (FP64) or float32 (MIXED), must be 0 on seeded voxels; q_out: same
 * type and shape, meaningful on unseeded voxels.  ws: workspace of
 * rw_operator_workspace_bytes. */
size_t rw_operator_workspace_bytes(rw_dims dims, int32_t precision);
rw_status rw_apply_operator(rw_context* ctx, const rw_volume* vol, const rw_seeds* seeds,
                            double beta, double w_eps, int32_t precision, const void* p,
                            void* q_out, void* ws, size_t ws_bytes, void* stream);

/* Whole-volume solve.
 * prob_out: [K][nz][ny][nx], float64 for RW_PREC_FP64, float32 for MIXED;
 *   seeds exact; with solve_all_labels = 0 label 1 is 1 - sum of the others.
 * argmax_out: NULL or uint8 [nz][ny][nx], 1-based label of the largest
 *   probability, lowest label on ties.
 * ws: workspace of rw_solve_workspace_bytes(dims, K, precision, solve_all).
 * stats: host, may be NULL. */
size_t rw_solve_workspace_bytes(rw_dims dims, int32_t num_labels, int32_t precision,
                                int32_t solve_all_labels);
rw_status rw_solve(rw_context* ctx, const rw_volume* vol, const rw_seeds* seeds,
                   const rw_options* opts, void* prob_out, uint8_t* argmax_out, void* ws,
                   size_t ws_bytes, rw_stats* stats, void* stream);

/* 4-D random walker (Sec. V-B: the random walker applied to a volume time
 * series): the grid [nt][nz][ny][nx] in which every voxel is joined to its
 * two neighbours along x, y, z and t (8-connected), the same Gaussian
 * weights and Dirichlet problem as rw_solve.
 * vol: data [nt][nz][ny][nx] (C order, x fastest); vol->dims is ONE time
 *   step's (nx, ny, nz); nt time steps, nz * nt at most 2^30.
 * seeds: labels [nt][nz][ny][nx].  prob_out: [K][nt][nz][ny][nx];
 * argmax_out: NULL or [nt][nz][ny][nx].  Options, precisions, statuses and
 * outputs otherwise as rw_solve.
 * ws: rw_solve4d_workspace_bytes(dims, nt, K, precision, solve_all_labels). */
size_t rw_solve4d_workspace_bytes(rw_dims dims, int32_t nt, int32_t num_labels,
                                  int32_t precision, int32_t solve_all_labels);
rw_status rw_solve4d(rw_context* ctx, const rw_volume* vol, int32_t nt, const rw_seeds* seeds,
                     const rw_options* opts, void* prob_out, uint8_t* argmax_out, void* ws,
                     size_t ws_bytes, rw_stats* stats, void* stream);

/* rw_solve without device allocation, for callers that cannot allocate
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc).  The workspace is a static device array of
 * rw_solve_noalloc_max_bytes() bytes (64 MiB) that the library holds on
 * every device it runs on until the process ends: solves whose
 * rw_solve_workspace_bytes exceeds it return RW_ERR_WORKSPACE before any
 * device work (e.g. float64 solves of up to about 2 million voxels with two
 * labels, 1 million with three).  Every call on one device shares the array,
 * so calls that overlap on one device (several contexts or threads) race.
 * Launches are plain (opts->use_graph and kernel_timing are ignored); the
 * context (rw_context_create) is the only set-up, and this call allocates no
 * device or pinned memory.  Arguments and results otherwise as rw_solve. */
size_t rw_solve_noalloc_max_bytes(void);
rw_status rw_solve_noalloc(rw_context* ctx, const rw_volume* vol, const rw_seeds* seeds,
                           const rw_options* opts, void* prob_out, uint8_t* argmax_out,
                           rw_stats* stats, void* stream);

/* One LOD step (levels of detail built by smoothing and downsampling, the
 * paper's Sec. III-D): g_out[c] = mean of the (up to) 2x2x2 fine values of g
 * in block c, g the normalised intensity of `fine` (pass a previous level's
 * output as RW_DT_F32/F64 with norm_lo 0, norm_hi 1); coarse size ceil(n/2)
 * per axis.  out_dtype: RW_DT_F32 or RW_DT_F64 (g_out's type).
 * labels_out (optional, needs fine_labels): coarse seed map, label s iff the
 * block holds seeds of s and of no other label (conflicts -> 0). */
rw_status rw_downsample(rw_context* ctx, const rw_volume* fine, const uint8_t* fine_labels,
                        int32_t out_dtype, void* g_out, uint8_t* labels_out, void* stream);

/* Brick activity from coarse probabilities (coarse-to-fine step of the
 * hierarchical random walker, Sec. IV-B).
 * coarse_prob: [K][coarse dims], float32 (coarse_dtype RW_DT_F32) or float64.
 * Upsampling: fine index i <-> coarse coordinate (i + 0.5)/factor - 0.5,
 *   clamped to [0, n_c - 1], trilinear, in float64.
 * Tiling: per axis cuts at grid_offset (0 = none), then every brick_size
 *   voxels; bricks_out (host, capacity >= candidates) receives every
 *   candidate brick in z-major grid order, active_out (host) one flag each.
 * Active: some voxel of the brick or of its in-volume face shell has
 *   lo_thr < p_s < hi_thr (strict) for some label s, or a seed in the brick
 *   differs from the upsampled argmax (lowest label on ties). */
rw_status rw_classify_bricks(rw_context* ctx, const void* coarse_prob, int32_t coarse_dtype,
                             rw_dims coarse_dims, int32_t num_labels, int32_t factor,
                             const uint8_t* fine_labels, rw_dims fine_dims,
                             const int32_t brick_size[3] /* x, y, z */,
                             const int32_t grid_offset[3] /* x, y, z */, double lo_thr,
                             double hi_thr, rw_brick* bricks_out, uint8_t* active_out,
                             int32_t capacity, int32_t* n_candidates, void* stream);

/* rw_classify_bricks with the seed rule taken from a seed list instead of a
 * dense fine label map (the out-of-core form: the fine labels need not be
 * on the device).  seed_index: device int64 [n_seeds], flat fine-grid
 * indices (z * ny + y) * nx + x; seed_label: device uint8 [n_seeds], 1..K.
 * Entries outside the grid or with label 0 are ignored.  The result equals
 * rw_classify_bricks on the label map holding exactly these seeds. */
rw_status rw_classify_bricks_sparse(rw_context* ctx, const void* coarse_prob,
                                    int32_t coarse_dtype, rw_dims coarse_dims, int32_t num_labels,
                                    int32_t factor, const int64_t* seed_index,
                                    const uint8_t* seed_label, int64_t n_seeds, rw_dims fine_dims,
                                    const int32_t brick_size[3], const int32_t grid_offset[3],
                                    double lo_thr, double hi_thr, rw_brick* bricks_out,
                                    uint8_t* active_out, int32_t capacity, int32_t* n_candidates,
                                    void* stream);

/* What a seed edit reaches, for an incremental re-solve of a hierarchical
 * solution (the paper's interactive segmentation, Sec. IV-B): on the brick
 * grid of rw_classify_bricks (same brick_size, grid_offset; candidates in
 * the same order),
 *   edited_out[b] = 1 if brick b holds a voxel whose label differs between
 *     old_labels and new_labels, or one of such a voxel's six face
 *     neighbours (its face shell holds the voxel), else 0;
 *   moved_out[b] = the largest |new_coarse - old_coarse| over the K labels
 *     and over the coarse cells of b's footprint (fine origin / factor to
 *     ceil(fine end / factor)) and one cell around it.
 * old_labels, new_labels: device uint8 fine label maps; old_coarse,
 * new_coarse: device [K][coarse dims] of coarse_dtype (F32 or F64).
 * edited_out (uint8), moved_out (double): host arrays of capacity >=
 * candidates; *n_candidates receives the count (a call with capacity 0
 * only counts, returning RW_ERR_INVALID_ARG). */
rw_status rw_seed_edit_bricks(rw_context* ctx, const uint8_t* old_labels,
                              const uint8_t* new_labels, rw_dims fine_dims,
                              const void* old_coarse, const void* new_coarse,
                              int32_t coarse_dtype, rw_dims coarse_dims, int32_t num_labels,
                              int32_t factor, const int32_t brick_size[3],
                              const int32_t grid_offset[3], uint8_t* edited_out,
                              double* moved_out, int32_t capacity, int32_t* n_candidates,
                              void* stream);

/* Batched solve of many bricks of the fine level in one set of launches
 * (each CG pass of every brick in one launch, over a compacted list of the
 * tiles of the bricks still iterating; per-brick, per-label convergence).
 * Each brick solves the random walker restricted to it: unknowns are its
 * unseeded voxels; Dirichlet data are its seeds and every in-volume face
 * neighbour outside it (seed value if seeded, else the upsampled coarse
 * probability).  Initial guess: opts->x0 = NULL gives the upsampled coarse
 * probabilities; otherwise opts->x0 is a device float32 [K][voxels of `fine`]
 * array in the layout of prob_out (a previous result may be passed back, as
 * for a warm-started re-solve after a seed edit), read on the bricks'
 * unseeded voxels for the solved labels.  Stopping ||r|| <= tol ||b|| per
 * brick and label (b of the brick system).  Precision MIXED (float32 CG,
 * float64 dots, float64 residual refreshes) or FP64.  Bricks must lie inside
 * their volume.
 * bricks: host array of n_bricks.
 * subvols: NULL (every brick lies in `fine`), or host array of n_bricks: brick
 *   i lies in sub-volume i of the pool `fine` (its data and labels, with
 *   fine->dims the pool's total size as (n, 1, 1)); coarse upsampling uses
 *   global positions.
 * prob_out: [K][voxels of `fine`] float32: the voxels of the bricks are
 *   overwritten (at their pool positions), other voxels untouched.
 * brick_iters: NULL or host int32 [n_bricks][R] CG iterations per brick/label.
 * ws: rw_bricks_workspace_bytes(...), sized for every tile shape a brick
 *   solve may use (the default and every rw_autotune_bricks candidate). */
size_t rw_bricks_workspace_bytes(const rw_brick* bricks, int32_t n_bricks, int32_t num_labels,
                                 int32_t precision, int32_t solve_all_labels);
rw_status rw_solve_bricks(rw_context* ctx, const rw_volume* fine, const rw_seeds* fine_seeds,
                          const void* coarse_prob, int32_t coarse_dtype, rw_dims coarse_dims,
                          int32_t factor, const rw_brick* bricks, const rw_subvolume* subvols,
                          int32_t n_bricks, const rw_options* opts, float* prob_out,
                          int32_t* brick_iters, void* ws, size_t ws_bytes, rw_stats* stats,
                          void* stream);

/* Upsampled coarse probabilities written into the fine grid for every voxel
 * of the listed bricks (the inactive ones), seeds exact.  prob_out: [K][voxels
 * of the label array] float32.  subvols: as for rw_solve_bricks (NULL: the
 * bricks lie in the fine grid of fine_dims; else fine_dims is the pool size
 * as (n, 1, 1) and brick i lies in sub-volume i). */
rw_status rw_fill_bricks(rw_context* ctx, const void* coarse_prob, int32_t coarse_dtype,
                         rw_dims coarse_dims, int32_t num_labels, int32_t factor,
                         const uint8_t* fine_labels, rw_dims fine_dims, const rw_brick* bricks,
                         const rw_subvolume* subvols, int32_t n_bricks, float* prob_out,
                         void* stream);

/* Adjoint gradient of a loss L of the probabilities of a float64 rw_solve
 * (the differentiable form of the random walker of Sec. III-A; the
 * operator L_U is symmetric, so each adjoint system uses the forward one).
 * prob: [K][nz][ny][nx] float64, the forward probabilities as rw_solve wrote
 *   them with the same opts->solve_all_labels (seeds exact).
 * grad_prob: [K][nz][ny][nx] float64, dL/dprob (read on unseeded voxels).
 * For every solved label s (2..K, or 1..K with solve_all_labels = 1):
 *   rhs_s = dL/dx^s, minus dL/dx^1 when label 1 is the complement 1 - sum of
 *     the solved labels (solve_all_labels = 0: a loss of the background
 *     reaches label s through that sum);
 *   L_U lam_s = rhs_s on the unseeded voxels (lam_s = 0 on seeds), by the
 *     float64 Jacobi-PCG of rw_solve to opts->tol;
 *   c_e = (lam_i - lam_j)(x_i - x_j) w_e per edge e = (i, j);
 * and the contributions of all solved labels add:
 *   dL/dbeta = sum_s sum_e c_e (g_i - g_j)^2,
 *   dL/dg_i  = sum_s sum_{e=(i,j)} 2 beta c_e (g_i - g_j)   (g normalised;
 *     a raw-intensity gradient is dL/dg_i / (norm_hi - norm_lo)).
 * grad_g_out: NULL or device [nz][ny][nx] float64 (overwritten).
 * grad_beta_out: NULL or a device float64 scalar (overwritten).
 * stats: per solved label the adjoint iterations, status and residual.
 * Validation failures return before any device work; an adjoint solve that
 * fails returns its status with the outputs undefined.
 * ws: rw_backward_workspace_bytes(dims). */
size_t rw_backward_workspace_bytes(rw_dims dims);
rw_status rw_solve_backward(rw_context* ctx, const rw_volume* vol, const rw_seeds* seeds,
                            const rw_options* opts, const double* prob, const double* grad_prob,
                            double* grad_g_out, double* grad_beta_out, void* ws, size_t ws_bytes,
                            rw_stats* stats, void* stream);

/* Tile-shape autotuner of the whole-volume stencil kernels (64 vx x by
 * columns, each lane owning vx columns 64 apart, one row per wave; zc planes;
 * XCD-aware tile order on/off): runs 2 * check_interval CG iterations of
 * rw_solve on this volume for each candidate (vx in {1, 2, 4}, 4 for mixed
 * precision only; by in {4, 8}, 8 with vx = 2 only; zc in {16, 32, 64}; order
 * in {plain, XCD-aware}) with every pass timed by events, and records the
 * fastest for later solves of the same precision, number of solved labels and
 * size class (floor(log2 voxels)) in this process.  prob_scratch: output
 * buffer as for rw_solve (overwritten); ws as for rw_solve; best: host, 4 ints
 * (vx, zc, xcd, by) or NULL. */
rw_status rw_autotune(rw_context* ctx, const rw_volume* vol, const rw_seeds* seeds,
                      const rw_options* opts, void* prob_scratch, void* ws, size_t ws_bytes,
                      int32_t* best, void* stream);

/* Tile-shape autotuner of the batched brick solves (tiles of 64 columns by
 * by * rpl rows, each lane owning rpl rows by apart; zc planes; worklist in
 * plain or XCD-aware order): runs 2 * check_interval CG iterations of
 * rw_solve_bricks on these bricks for each candidate ((by, rpl) in {(8, 2),
 * (4, 2), (16, 1), (8, 1), (4, 1)}, zc in {16, 32, 64}, both orders), times
 * every pass by events, and records the shape with the least pass time per
 * voxel-iteration for later brick solves of the same precision, number of
 * solved labels and size class of the largest brick (floor(log2 voxels)) in
 * this process.  Arguments as for rw_solve_bricks; prob_scratch receives
 * partial solutions (overwritten by every candidate), ws must hold
 * rw_bricks_workspace_bytes (which covers every candidate shape); best: host,
 * 4 ints (by, rpl, zc, xcd order) or NULL. */
rw_status rw_autotune_bricks(rw_context* ctx, const rw_volume* fine, const rw_seeds* seeds,
                             const void* coarse_prob, int32_t coarse_dtype, rw_dims coarse_dims,
                             int32_t factor, const rw_brick* bricks, const rw_subvolume* subvols,
                             int32_t n_bricks, const rw_options* opts, float* prob_scratch,
                             void* ws, size_t ws_bytes, int32_t* best, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* RW_H_ */
