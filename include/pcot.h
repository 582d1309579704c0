/*
 * pcot.h - C ABI of the MI355X (gfx950) library that runs polyhedral loop nests
 * (iterative stencils and interval dynamic programming) under single-level
 * tiling and under cache-oblivious recursive decomposition.
 *
 * Problem statement followed (paper: "PCOT: Cache Oblivious Tiling of
 * Polyhedral Programs", arXiv 1802.00166):
 *   - the input is a fully permutable loop nest, described by its domain and
 *     its dependences (Section 3, Tiling; Section 4.1 Approach Overview);
 *   - tiles are hyper-rectangles of runtime sizes b_i; the tile size is the
 *     base-case (leaf) threshold of the recursive decomposition (Section 3.3,
 *     Terminology: Tile Size);
 *   - the schedule is either single-level tiling visiting tiles in
 *     lexicographic or wavefront order, or the cache-oblivious recursion that
 *     halves the padded bounding box into 2^d orthants (Section 4.2), skips
 *     zero and empty orthants (Section 4.3) and pads the bounding box to
 *     b_i * 2^k_i (Section 4.5).
 * Stencils are skewed (t, i) -> (t, i + t) in every spatial dimension to make
 * the nest fully permutable (Section 4.3.2, the Heat-2D skewing example;
 * appendix on memory allocation, the 1D-Jacobi schedule), and values are
 * stored in two buffers indexed by t mod 2 (the appendix's motivating
 * example), which is a schedule-independent allocation for these radius-1
 * stencils.
 *
 * Conventions for every entry point
 *   - Pointers named "device" are HIP device pointers; everything else is
 *     host memory.  The caller owns every buffer it passes.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Run calls only enqueue work and return; results and device-side errors
 *     are visible after the stream is synchronised (pcot_stream_status).
 *   - Returns PCOT_OK (0) or a negative pcot_status; pcot_last_error() then
 *     gives a message (thread-local, valid until the next call on the thread).
 *   - No C++ exception crosses this boundary.
 */
#ifndef PCOT_H
#define PCOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ enums --- */

typedef enum {
    PCOT_JACOBI1D_3PT = 1, /* u'[i] = ((u[i-1] + u[i]) + u[i+1]) / 3                        */
    PCOT_JACOBI2D_5PT = 2, /* u' = 0.2 * ((((c + n) + s) + e) + w), n = u[y-1][x], e = u[y][x+1] */
    PCOT_HEAT3D_7PT = 3,   /* u' = u + 0.125 * ((dx + dy) + dz), dx = (u[x+1] - 2u) + u[x-1]   */
    PCOT_GS2D_5PT = 4,     /* in-place Gauss-Seidel: sweep t visits the interior row by row,
                              u[y][x] = 0.2 * ((((c + n) + s) + e) + w) with n, w already of
                              sweep t (dependences inside a time step; Section 6.2, Table 2).
                              f64, tiled schedules 1..4 only                                  */
    PCOT_FDTD2D = 5,       /* three-statement 2D Yee update per step, in place (an imperfect
                              nest, run after the embedding transformation, Section 4.4):
                                ey[i][j] -= 0.25 (hz[i][j] - hz[i-1][j])       1 <= i < ny
                                ex[i][j] += 0.25 (hz[i][j] - hz[i][j-1])       1 <= j < nx
                                hz[i][j] -= 0.5 ((ey[i+1][j] - ey[i][j]) - (ex[i][j+1] - ex[i][j]))
                                                                 i < ny-1, j < nx-1
                              in / out hold ex, ey, hz one after another (3 ny nx elements);
                              dims are ny, nx >= 1 (no frame: every cell belongs to the nest).
                              f64; PCOT_NAIVE (three kernels per step) or schedules 1..4  */
    PCOT_MOTIV1D = 6       /* the appendix's motivating 1D program (Memory Allocation):
                                x'[i] = 0.25 (((x[i-1] + x[i]) + x[i+1]) + x[0])  1 <= i <= N-2
                                x'[0] = 0.5 x[0] + 0.25,  x'[N-1] = 0.5 x[N-1] + 0.25
                              every interior point reads the previous step's left boundary
                              (an affine, many-to-one dependence).  Run with the appendix's
                              schedule-independent allocation: two buffers for the interior,
                              single-assignment arrays of T+1 values for each boundary cell
                              (in the workspace).  f64; PCOT_NAIVE or schedules 1..4; tile t,
                              s[0] as for the 1D stencil                                   */
} pcot_kind;

typedef enum {
    PCOT_F64 = 0,  /* storage and arithmetic in binary64                                   */
    PCOT_F32 = 1,  /* storage and arithmetic in binary32                                   */
    PCOT_BF16 = 2  /* bfloat16 storage (uint16 bit patterns), binary32 arithmetic, each
                      stored value rounded to nearest-even bfloat16                        */
} pcot_dtype;

typedef enum {
    PCOT_NAIVE = 0,    /* untiled: one sweep over the field per time step (a Jacobi-1D field
                          whose two levels fit in one CU's LDS runs all steps in one block)   */
    PCOT_SLT_LEX = 1,  /* single-level tiling, tiles in lexicographic order (Section 1, 3.2)   */
    PCOT_SLT_WAVE = 2, /* single-level tiling, tiles ordered by wavefront, then lexicographic  */
    PCOT_COT_SEQ = 3,  /* recursive decomposition, orthants in lexicographic order (Sec. 4.2)  */
    PCOT_COT_PAR = 4,  /* recursive decomposition, orthants grouped by wavefront at each level
                          (the task/taskwait grouping of the parallel version, Sec. 4.2)      */
    PCOT_TRAP = 5,     /* 2D stencil only: trapezoid tiles from a hyperspace cut of y and x in
                          every time band (upright tiles shrink, inverted ones grow; the four
                          phases UU, UV, VU, VV of a band each start all their tiles at once):
                          the concurrent-start schedules the paper compares against (Sec. 5.3,
                          Pochoir's Heat-3D scaling; related work, Frigo-Strumpen cuts)      */
    PCOT_DIAMOND = 6   /* PCOT_TRAP with the cut shifted by half a period in every other band,
                          so each upright tile sits on the inverted one below it (hexagonal /
                          diamond tiles with concurrent start; related work, diamond tiling)  */
} pcot_schedule;

typedef int32_t pcot_status;
#define PCOT_OK 0
#define PCOT_ERR_INVALID (-1)     /* bad kind, dtype, dims, T, tile or pointer              */
#define PCOT_ERR_UNSUPPORTED (-2) /* valid tile that the executors cannot run (registers/LDS) */
#define PCOT_ERR_OVERFLOW (-3)    /* DP: (N-1)*pmax^3 does not fit in int64                  */
#define PCOT_ERR_HIP (-4)         /* a HIP runtime call failed                              */
#define PCOT_ERR_WORKSPACE (-5)   /* workspace missing or smaller than required            */
#define PCOT_ERR_TIMEOUT (-6)     /* device watchdog: a tile waited too long for its inputs */
#define PCOT_ERR_DEVICE (-7)      /* device-side validation failed (e.g. p out of range)    */
#define PCOT_ERR_HOST (-8)        /* host-side failure (out of host memory for a plan)      */

/* Leaf (tile) sizes.  t: time steps per tile; s[0..d-1]: spatial sizes, outer
 * to inner, in skewed coordinates (j = i + t).  The same numbers are the
 * base-case thresholds of the recursive schedules.  For the interval DP,
 * s[0], s[1], s[2] are the (i, j, k) block sizes and t is unused.
 * For PCOT_TRAP / PCOT_DIAMOND: t = band height b_t, s[0], s[1] = footprints
 * F_y, F_x (points held per tile, one-point halo included, each >= 2 b_t + 2):
 * upright tiles start F - 2 wide, inverted ones F - 2 b_t; executors exist
 * for f64 with (b_t, F_y, F_x) in {(16, 64, 128), (8, 64, 128), (8, 32, 128)}. */
typedef struct {
    int32_t t;
    int32_t s[3];
} pcot_tile;

/* ------------------------------------------------------------ stencils --- */

/* Bytes of workspace pcot_stencil_run needs for this problem (0 when the
 * arguments are invalid; see pcot_last_error).  Covers the second
 * time-level buffer, tile dependency counters and the device error word. */
size_t pcot_stencil_workspace(int32_t kind, int32_t dtype, const int64_t* dims, int64_t T,
                              const pcot_tile* tile, int32_t schedule);

/* Run T time steps of stencil `kind` on the field `in`, writing u_T to `out`.
 *   dims      host, d entries (d = 1, 2, 3 for the three kinds), array extents
 *             outer to inner INCLUDING the boundary; each >= 3.  Row-major,
 *             innermost index contiguous, no padding.
 *   T         >= 0 time steps.  T = 0 copies in to out.
 *   tile      host; ignored for PCOT_NAIVE (may be NULL then).
 *   in        device, read only, prod(dims) elements of `dtype`.
 *   out       device, prod(dims) elements; must not overlap `in` or the
 *             workspace.  Boundary cells (outer face) are copied from `in`
 *             unchanged; interior cells receive u_T.
 *   workspace device, at least pcot_stencil_workspace(...) bytes, 256-byte
 *             aligned; contents are scratch between calls.  Calls that share
 *             a workspace must be ordered on one stream.
 * Every schedule and every valid tile gives the same bits (the method only
 * reorders points of a fully permutable nest; each point uses the fixed
 * operation order of its update rule, without contraction to FMA).
 * Size limit of the tiled schedules: the executors address a field with
 * 32-bit byte offsets, so field bytes + 2 outermost slices (rows in 2D,
 * planes in 3D) + 4 KiB must stay below 0x7FFFFFF0 (just under 2 GiB);
 * larger fields return PCOT_ERR_UNSUPPORTED here and from
 * pcot_stencil_workspace (0) and the batched calls.  PCOT_NAIVE has no such
 * limit. */
/* The tiles of a PCOT_TRAP / PCOT_DIAMOND plan of the 2D stencil, in queue
 * order (a topological order of their dependences).  Per tile, 12 int32 in
 * `tiles` (host, cap tiles): lo_y, hi_y, slo_y, shi_y, fo_y, lo_x, hi_x,
 * slo_x, shi_x, fo_x, t0, nt: level l (0 <= l < nt, time step t0 + l) of the
 * tile computes u_{t0+l+1} over [lo + slo*l, hi + shi*l) in each dimension,
 * intersected with the interior; fo is the first index of the executor's
 * register footprint.  `edges` (host, edge_cap pairs): (predecessor,
 * successor) tile indices; *n_edges receives their number.  traffic[0],
 * traffic[1] (host, nullable) receive the elements the executor loads and
 * stores for the whole plan (its algorithmic HBM traffic).  Returns the tile
 * count, or -1 (pcot_last_error).  Host only. */
int64_t pcot_stencil_trap_plan(const int64_t* dims, int64_t T, const pcot_tile* tile, int32_t schedule,
                               int32_t* tiles, int64_t cap, int32_t* edges, int64_t edge_cap,
                               int64_t* n_edges, int64_t* traffic);

pcot_status pcot_stencil_run(int32_t kind, int32_t dtype, const int64_t* dims, int64_t T,
                             const pcot_tile* tile, int32_t schedule, const void* in, void* out,
                             void* workspace, size_t ws_bytes, void* stream);

/* Is `tile` runnable by the tiled executors for this kind and dtype?  Returns
 * PCOT_OK, PCOT_ERR_UNSUPPORTED or PCOT_ERR_INVALID without touching the GPU. */
pcot_status pcot_stencil_tile_supported(int32_t kind, int32_t dtype, const pcot_tile* tile);

/* Batched form: n independent instances of one kind and dtype, each with its
 * own dims, T and tile, run by one persistent launch that takes tiles of all
 * instances from one device queue.
 *   dims   host, n*3 (unused trailing entries ignored), in/out host arrays of
 *          n device pointers.  T, tiles host arrays of n.
 *   workspace >= pcot_stencil_workspace_batched(...).
 * Schedules: PCOT_SLT_WAVE or PCOT_COT_PAR (order within each instance);
 * the instances' tile sequences are interleaved by fractional progress
 * through each sequence, ties going to the instance with more updates. */
size_t pcot_stencil_workspace_batched(int32_t kind, int32_t dtype, int32_t n, const int64_t* dims,
                                      const int64_t* T, const pcot_tile* tiles, int32_t schedule);
pcot_status pcot_stencil_run_batched(int32_t kind, int32_t dtype, int32_t n, const int64_t* dims,
                                     const int64_t* T, const pcot_tile* tiles, int32_t schedule,
                                     const void* const* in, void* const* out, void* workspace,
                                     size_t ws_bytes, void* stream);

/* Number of leaves (non-empty tiles) the planner emits for this problem, and
 * optionally their visiting order: `order` (host, may be NULL) receives up to
 * `cap` entries of 4 int32 each (time tile index, then spatial tile indices
 * outer to inner, unused entries 0).  Host only; no GPU work. */
int64_t pcot_stencil_plan(int32_t kind, const int64_t* dims, int64_t T, const pcot_tile* tile,
                          int32_t schedule, int32_t* order, int64_t cap);

/* Device error-norm reduction in binary64 for reporting precision forms:
 * over the interior of a field of `dims` (d entries), with x of `dtype` and
 * the reference r in binary64 (both device), writes (host) out[0] =
 * max|x-r|, out[1] = max|r|, out[2] = sum (x-r)^2, out[3] = sum r^2.
 * Synchronises the stream. */
pcot_status pcot_error_norms(int32_t dtype, int32_t d, const int64_t* dims, const void* x,
                             const double* r, double* out, void* stream);

/* Allocation-free variant of pcot_error_norms, for callers that cannot
 * allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc).  Same two reduction passes, same bits.
 *   x, r   device, as in pcot_error_norms.
 *   out    DEVICE, 4 doubles: max|x-r|, max|r|, sum (x-r)^2, sum r^2.
 * The first pass's partial sums live in a static device array of the
 * library (1024 x 4 doubles = 32 KiB per GPU, held until the process ends;
 * its address is looked up once per device on the first call).  Every call
 * rewrites all of it, so no clearing is needed; calls that overlap on one
 * GPU (different streams, no ordering between them) race on it.  Only
 * enqueues: no synchronisation, no hipMalloc / hipFree, no host-device copy.
 * Inputs with more than PCOT_NORMS_STATIC_MAX_POINTS interior points return
 * PCOT_ERR_UNSUPPORTED. */
#define PCOT_NORMS_STATIC_MAX_POINTS (1LL << 36)
pcot_status pcot_error_norms_static(int32_t dtype, int32_t d, const int64_t* dims, const void* x,
                                    const double* r, double* out, void* stream);

/* --------------------------------------------------------- interval DP --- */

/* Matrix-chain / optimal parenthesization (the interval DP of the paper's OSP
 * benchmark, Section 5.1.2, tiled in all three dimensions after the
 * Guibas-Kung-Thompson reordering of the reduction):
 *   C[i][i] = 0,  C[i][j] = min_{i<=k<j} C[i][k] + C[k+1][j] + p[i-1] p[k] p[j].
 *   p      device, N+1 int64 dimensions, each in [1, pmax].
 *   pmax   caller's bound on p; selects 32-bit arithmetic when
 *          (N-1)*pmax^3 < 2^32 (exact then), int64 otherwise;
 *          PCOT_ERR_OVERFLOW when (N-1)*pmax^3 >= 2^62.  The kernels check
 *          1 <= p <= pmax and report PCOT_ERR_DEVICE through
 *          pcot_stream_status if not.
 *   C      device, N*N int64 row-major; C[(i-1)*N + (j-1)] receives the
 *          cost of A_i..A_j for i <= j.  The lower triangle is set to 0.
 *   tile   s[0] = s[1] = block size b of the square (i, j) tiles, b in
 *          {16, 32, 64} (the finishing pass holds three b x b tiles in LDS:
 *          b = 128 would not fit); s[2] = k-chunk, a multiple of 16: the
 *          off-diagonal splits of a tile pair are cut into work items of
 *          this many splits; t unused.  Other sizes: PCOT_ERR_UNSUPPORTED /
 *          PCOT_ERR_INVALID.
 *   schedule PCOT_SLT_WAVE (tile diagonals in order) or PCOT_COT_PAR
 *          (recursive halving of the padded (i, j) triangle; leaves grouped by
 *          the wavefronts of each split).
 * Every schedule and tile gives identical (exact integer) results.
 * Plan limit: the off-diagonal k range of every tile pair is cut into
 * k-chunk items; more than 2^31-1 items (e.g. N = 65536 with b = 32 and
 * k-chunk 16) returns PCOT_ERR_UNSUPPORTED. */
size_t pcot_dp_workspace(int64_t N, const pcot_tile* tile, int32_t schedule);
pcot_status pcot_dp_run(const int64_t* p, int64_t N, int64_t pmax, const pcot_tile* tile,
                        int32_t schedule, int64_t* C, void* workspace, size_t ws_bytes,
                        void* stream);

/* Optimal parenthesization from the final cost table of pcot_dp_run: for
 * every cell i < j (1-based A_i..A_j), split[(i-1)*N + (j-1)] = the smallest k,
 * i <= k < j, with C[i][k] + C[k+1][j] + p[i-1] p[k] p[j] = C[i][j] (the
 * bracketing (A_i..A_k)(A_{k+1}..A_j); a sequential scan of k with a strict
 * comparison picks the same k).  Cells on and below the diagonal get 0.
 *   p      device, N+1 int64 (the same dimensions as the DP run).
 *   C      device, N*N int64 as written by pcot_dp_run (read only).
 *   split  device, N*N int64, written.
 * A separate pass over the finished table, so it does not depend on the
 * order in which the tiled DP reduced its splits; it costs up to about as
 * much work as the DP itself.  Only enqueues. */
pcot_status pcot_dp_split(const int64_t* p, int64_t N, const int64_t* C, int64_t* split, void* stream);

/* ------------------------------------------------- autotuning and model --- */

/* The paper explores tile sizes by timing a grid of candidates per kernel
 * (Section 5.2, the tile-size exploration, and its variability figures);
 * pcot_tune does the same on the GPU over the tile grids below, and a small
 * learned cost model, trained on such sweeps, predicts a good (tile,
 * schedule) without timing every candidate.  The sweep stays the reference
 * the model is measured against. */

#define PCOT_MATRIX_CHAIN 4 /* pcot_problem.kind of the interval DP */

typedef struct {
    int32_t kind;    /* pcot_kind, or PCOT_MATRIX_CHAIN                                  */
    int32_t dtype;   /* stencils: pcot_dtype; DP: ignored                                */
    int64_t dims[3]; /* stencils: extents outer..inner incl. boundary; DP: dims[0] = N  */
    int64_t T;       /* stencils: time steps; DP: pmax                                   */
} pcot_problem;

/* One timed (or predicted) candidate. */
typedef struct {
    float feat[8];    /* model features, pcot_features()                          */
    float ms;         /* median time of one run call, milliseconds                */
    pcot_tile tile;
    int32_t schedule;
} pcot_record;

typedef enum {
    PCOT_TUNE_SWEEP = 0,       /* time every candidate                                 */
    PCOT_TUNE_MODEL = 1,       /* predict every candidate, time none                   */
    PCOT_TUNE_MODEL_VERIFY = 2 /* predict every candidate, time the topk best-predicted */
} pcot_tune_mode;

typedef struct pcot_model pcot_model;

typedef struct {
    int32_t mode;            /* pcot_tune_mode                                          */
    int32_t reps;            /* timed runs per candidate, median kept (<= 0: 5)          */
    int32_t warmup;          /* untimed runs per candidate (< 0: 2)                     */
    int32_t topk;            /* MODEL_VERIFY: candidates re-timed (<= 0: 3)             */
    uint32_t sched_mask;     /* bit s: schedule s is a candidate; 0 = every tiled one   */
    const pcot_model* model; /* required by the MODEL modes                             */
} pcot_tune_opts;

/* Candidate grid of a problem (host only):
 *   Jacobi-1D: b_t in {16,32,64,128,256} x b_x in {64,128,256}
 *   Jacobi-2D: b_t in {4,8,16,32,64} x b_y in {16,32,64,128,256} x b_x in {64,128,256}
 *   Heat-3D:   b_t in {2,4,8} x b_z in {16,64,256} x b_y in {2,4,8,16}, b_x = 64
 *   DP:        b in {32,64} (s[0] = s[1]) x k-chunk in {32,64,128,256}
 * each crossed with the schedules of sched_mask (stencils: the four tiled
 * schedules; DP: SLT_WAVE and COT_PAR), keeping only runnable tiles.  Writes
 * up to `cap` entries to tiles/scheds (either may be NULL) and returns the
 * number of candidates, or -1 on invalid arguments. */
int64_t pcot_tune_candidates(const pcot_problem* prob, uint32_t sched_mask, pcot_tile* tiles,
                             int32_t* scheds, int64_t cap);

/* Model features of (problem, tile, schedule) (host only), all log2 of
 * positive sizes unless stated:
 *   stencils: [outer extent (product of all but the innermost; 1D: n),
 *              inner extent (1D: 1), T, b_t, outer tile (product; 1D: 1),
 *              b_inner (1D: b_x), element bytes, schedule code]
 *   DP:       [N, b, k-chunk, pmax, schedule code, 0, 0, 0] */
pcot_status pcot_features(const pcot_problem* prob, const pcot_tile* tile, int32_t schedule, float* feat);

/* Tunes one problem on the GPU: allocates its own buffers (input filled with
 * zeros, DP dims 1 + (37 i mod pmax)), times or predicts the candidates per
 * opts, and returns the best in best/best_sched/best_ms (any may be NULL).
 * Up to `cap` records (every candidate timed or predicted) are written to
 * `records` (may be NULL) and their number to *n_records.  Synchronous. */
pcot_status pcot_tune(const pcot_problem* prob, const pcot_tune_opts* opts, pcot_tile* best,
                      int32_t* best_sched, double* best_ms, pcot_record* records, size_t cap,
                      size_t* n_records, void* stream);

/* Training options of the cost model (two hidden ReLU layers of 64, binary32,
 * predicting ln(ms) from standardised features; mean squared error; Adam with
 * beta1 = 0.9, beta2 = 0.999, eps = 1e-8). */
typedef struct {
    int32_t epochs; /* <= 0: 300                              */
    int32_t batch;  /* 1..256; <= 0: 256                      */
    float lr;       /* <= 0: 1e-3                             */
    uint64_t seed;  /* He-uniform initialisation and shuffling */
} pcot_train_opts;

/* Trains a model on n records with the device training kernel and returns it
 * in *out (free with pcot_model_free); *final_loss (may be NULL) receives the
 * last epoch's mean squared error in standardised ln(ms).  Synchronous. */
pcot_status pcot_model_train(const pcot_record* records, size_t n, const pcot_train_opts* opts,
                             pcot_model** out, float* final_loss, void* stream);
/* Predicted ms of n records' features (host arrays), on the device. */
pcot_status pcot_model_predict_ms(const pcot_model* model, const pcot_record* records, size_t n,
                                  float* ms, void* stream);
/* Best predicted candidate of a problem (the MODEL mode of pcot_tune). */
pcot_status pcot_model_predict(const pcot_model* model, const pcot_problem* prob, uint32_t sched_mask,
                               pcot_tile* best, int32_t* best_sched, double* pred_ms, void* stream);
/* Text file: magic line, 8 feature means, 8 feature scales, target mean and
 * scale, then the 4801 parameters. */
pcot_status pcot_model_save(const pcot_model* model, const char* path);
pcot_status pcot_model_load(const char* path, pcot_model** out);
void pcot_model_free(pcot_model* model);

/* The network itself, for verification against an independent reference.
 * `params` holds 4801 floats: W1 [64][8], b1 [64], W2 [64][64], b2 [64],
 * W3 [64], b3 (row-major, output index first).  All arrays are host memory;
 * the computation runs on the device and the call synchronises.
 *   pcot_mlp_forward: yhat[i] for rows X[i][0..7], i < n.
 *   pcot_mlp_grad:    mean squared error of one batch (n <= 256) and its
 *                     gradient with respect to every parameter.
 *   pcot_mlp_train:   `epochs` passes of Adam over batches of `batch` rows
 *                     taken in the order given (order: epochs x n row
 *                     indices); params, m, v updated in place, the Adam step
 *                     count continuing from step0; epoch_loss (may be NULL)
 *                     receives each epoch's mean loss before its updates. */
#define PCOT_MLP_PARAMS 4801
pcot_status pcot_mlp_forward(const float* params, const float* X, int32_t n, float* yhat, void* stream);
pcot_status pcot_mlp_grad(const float* params, const float* X, const float* y, int32_t n, float* grad,
                          float* loss, void* stream);
pcot_status pcot_mlp_train(float* params, float* m, float* v, const float* X, const float* y, int32_t n,
                           const int32_t* order, int32_t epochs, int32_t batch, int32_t step0, float lr,
                           float* epoch_loss, void* stream);

/* ------------------------------------------------------------ status --- */

/* Synchronises `stream` and reads the device error word that the last run on
 * `workspace` left: PCOT_OK, PCOT_ERR_TIMEOUT or PCOT_ERR_DEVICE. */
pcot_status pcot_stream_status(void* workspace, void* stream);

/* Message for the last non-OK status returned on this thread ("" if none). */
const char* pcot_last_error(void);

/* Measurement: when enabled, every run records a HIP event pair on its
 * stream around its dominant kernel (the tiled executor, or the DP tile
 * kernels).  pcot_kernel_timing(1) starts a new measurement (discarding old
 * events); pcot_kernel_timing_read waits for the recorded events and returns
 * the summed kernel time (ms) and the number of timed launches. */
pcot_status pcot_kernel_timing(int32_t enable);
pcot_status pcot_kernel_timing_read(double* total_ms, int64_t* count);

/* Library version string. */
const char* pcot_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PCOT_H */
