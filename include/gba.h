/*
 * gba.h -- C ABI of the MI355X (gfx950) Levenberg-Marquardt bundle-adjustment
 * solver.
 *
 * The method is the LM graph optimiser of Graphite (arXiv 2509.26581) applied
 * to bundle adjustment: minimise half the sum of robustified squared
 * Mahalanobis reprojection errors (Background, Eq. 1-2, Huber kernel Eq. 7) by
 * repeatedly solving the damped normal equations
 *     (J^T W J + lambda D^T D) dx = -J^T W r            (Background, Eq. 4-6)
 * with D^T D the clamped Hessian diagonal (Sec. IV-D).  On the GPU the point
 * blocks are eliminated (Schur complement) and the reduced camera system is
 * solved by block-Jacobi preconditioned conjugate gradients with implicit,
 * matrix-free products built from the stored Jacobian blocks (Sec. IV-D:
 * implicit PCG over the graph structure, block-Jacobi preconditioner).
 *
 * Camera model (the BAL camera; the paper benchmarks BAL but does not write
 * the model out): 9 parameters per camera (w[3] angle-axis, t[3], f, k1, k2),
 *     P = R(w) X + t,  p = -P_xy / P_z,  pixel = f (1 + k1|p|^2 + k2|p|^4) p,
 *     residual r = pixel - observation.
 *
 * Conventions common to every call:
 *   - Every function returns gba_status: GBA_OK (0) or a negative GBA_ERR_*.
 *     No exception crosses the ABI.  After an error, gba_last_error(g) returns
 *     a message for that handle.
 *   - Host pointers are read (or written) before the call returns; the caller
 *     keeps ownership of every array it passes.  Arrays are row-major,
 *     contiguous, in the units stated.
 *   - Device memory is obtained from the allocator callbacks given to
 *     gba_create (or hipMalloc/hipFree when both are NULL) and released by
 *     gba_destroy.  All work is issued on the stream given to gba_set_stream
 *     (default: the null stream of the chosen device).
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - Vertex ids are arbitrary int64 values, unique per kind (Sec. IV-A:
 *     vertices are added with a user identifier).  Results are returned in
 *     the order the vertices were added.
 */
#ifndef GBA_H
#define GBA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int gba_status;

#define GBA_OK 0
#define GBA_ERR_INVALID_ARG (-1)  /* bad size, NULL pointer, bad enum        */
#define GBA_ERR_UNKNOWN_ID (-2)   /* an edge or set_fixed names no vertex    */
#define GBA_ERR_DUPLICATE_ID (-3) /* a vertex id added twice                 */
#define GBA_ERR_NONFINITE (-4)    /* NaN/Inf in parameters or observations   */
#define GBA_ERR_OOM (-5)          /* the allocator returned NULL             */
#define GBA_ERR_HIP (-6)          /* a HIP runtime call failed               */
#define GBA_ERR_STATE (-7)        /* call not valid in the current state     */
#define GBA_ERR_UNSUPPORTED (-8)  /* configuration the library cannot run   */
#define GBA_ERR_BUDGET (-9)       /* serving: request larger than the budget */
#define GBA_PENDING 1             /* serving: result not ready (not an error) */

typedef struct gba_graph gba_graph;

/* Precision policy (Sec. IV-D: vertex precision and linear-system precision
 * chosen separately; Table I runs FP64, FP32 and FP32 with BF16 storage). */
typedef enum {
    GBA_FP64 = 0,        /* everything in FP64                               */
    GBA_MIXED_FP32 = 1,  /* FP32 Jacobians, Hessian blocks and PCG vectors;
                            FP64 cost, gain ratio, PCG dot products, step
                            acceptance and 3x3 point-block inversion          */
    GBA_MIXED_BF16 = 2   /* as MIXED_FP32, plus BF16 storage of the Jacobian
                            copy read by the PCG products                     */
} gba_precision;

/* Robust kernel on s = r^T Omega r (Background, Eq. 7). */
typedef enum {
    GBA_LOSS_SQUARED = 0, /* rho(s) = s                                        */
    GBA_LOSS_HUBER = 1    /* rho(s) = s if s <= delta^2, else 2 delta sqrt(s) - delta^2 */
} gba_loss;

/* Preconditioner of the reduced camera system (Sec. IV-D). */
typedef enum {
    GBA_PRECOND_IDENTITY = 0,
    GBA_PRECOND_BLOCK_JACOBI = 1  /* exact 9x9 diagonal blocks of the Schur complement */
} gba_precond;

/* Why gba_solve stopped (report.termination). */
typedef enum {
    GBA_TERM_NONE = 0,
    GBA_TERM_MAX_ITERS = 1,        /* max_iters trials were run               */
    GBA_TERM_COST_TOL = 2,         /* accepted step with (F - F')/F < tol     */
    GBA_TERM_STEP_TOL = 3,         /* |dx| <= tol (|x| + tol)                 */
    GBA_TERM_LAMBDA_OVERFLOW = 4,  /* damping exceeded 1e32                   */
    GBA_TERM_NUMERICAL_FAILURE = 5,/* initial cost not finite                 */
    GBA_TERM_NO_WORK = 6           /* no active edge or no free vertex        */
} gba_termination;

/* Device allocator supplied by the caller (e.g. PyTorch's caching
 * allocator).  alloc returns NULL on failure; free accepts what alloc gave. */
typedef void* (*gba_alloc_fn)(size_t bytes, void* ctx);
typedef void (*gba_free_fn)(void* ptr, void* ctx);

/* Solver options.  Defaults from gba_default_options().  The PCG knobs follow
 * the paper's PCG solver (maximum iterations, tolerance, rejection ratio;
 * Sec. IV-A listing and Sec. V-C settings). */
typedef struct gba_options {
    double initial_lambda;     /* initial damping (default 1e-4)             */
    double min_diag;           /* clamp of diag(H) used for damping (1e-6)   */
    double max_diag;           /* (1e32)                                     */
    int pcg_max_iters;         /* (100)                                      */
    double pcg_tol;            /* (1e-6)                                     */
    int pcg_tol_relative;      /* 1: |r_k| <= tol |r_0|; 0: |r_k| <= tol (1) */
    double pcg_rejection_ratio;/* stop PCG and keep the best iterate when
                                  |r_k| > ratio * min_m<=k |r_m|; <= 0 or Inf
                                  disables (default: disabled)               */
    int precond;               /* gba_precond (BLOCK_JACOBI)                 */
    int timing;                /* 1: time phases with HIP events (0)         */
    int accumulation;          /* camera-side sums of the Schur products:
                                  GBA_ACC_AUTO (default): one point-major pass
                                  with per-workgroup LDS partials when one
                                  problem's 9 x n_cams FP64 vector fits in LDS,
                                  else two passes (point-major, then
                                  camera-major over a camera-major copy of
                                  the stored Jacobian); GBA_ACC_LDS /
                                  GBA_ACC_CAMERA_PASS force one (LDS fails with
                                  UNSUPPORTED when it does not fit).  In the
                                  two-pass form of a single problem with more
                                  than 1,024 cameras (no fixed order), the PCG
                                  product's camera pass runs over camera
                                  blocks of 1,024 (edges in point order inside
                                  a block, LDS partials per block, its own
                                  Jacobian copy; the persistent PCG schedule
                                  takes the camera-major pass instead);
                                  GBA_ACC_CAMERA_BLOCKS forces that form at
                                  any size.  Read when the device graph is
                                  built.                                      */
    int tiles_per_block;       /* point tiles (whole points, <= 64 edges) per
                                  workgroup of the point passes; 0 (default):
                                  max(16, n_tiles / n_CU).  Read when the device
                                  graph is built; the server takes its sizes
                                  from gba_server_config instead.             */
    int deterministic;         /* 1: every reduction runs in a fixed order, so
                                  a solve repeats bit for bit (run twice, graph
                                  replay or eager launches, alone or in a
                                  served mix).  The camera-side sums of the
                                  Schur products then take the camera-major
                                  second pass (GBA_ACC_CAMERA_PASS); combined
                                  with GBA_ACC_LDS it is INVALID_ARG.  0
                                  (default): LDS partials combined by atomics,
                                  results repeat to rounding.  Read when the
                                  device graph is built.                      */
    int jacobi_scaling;        /* 1: scale the camera columns of the Jacobian by
                                  s_k = 1 / (1 + sqrt(H_kk)), H_kk the Hessian
                                  diagonal (Sec. IV-D column rescaling).  PCG
                                  on the scaled reduced system is PCG with the
                                  preconditioner diag(s)^2, which is what the
                                  identity preconditioner then applies; under
                                  block Jacobi the scaling cancels exactly (the
                                  blocks of the scaled system are the scaled
                                  blocks), so it changes nothing there.  (0)  */
    int pcg_schedule;          /* how the PCG iterations of a damped step are
                                  launched: GBA_PCG_CHUNKED = chunks of
                                  iterations (three kernels each) replayed as
                                  HIP graphs, the host checking the PCG state
                                  between chunks; GBA_PCG_PERSISTENT = one
                                  cooperative kernel runs every iteration of
                                  every problem of the batch (product,
                                  reduction and update as phases separated by
                                  grid barriers), each problem stopping on its
                                  own device-side decision, and the rest of the
                                  trial follows without a host check;
                                  GBA_PCG_AUTO (0) = chunked (on MI355X each
                                  grid barrier costs every workgroup a
                                  device-scope L2 write-back and invalidation,
                                  more than the graph's launch gaps it
                                  replaces).  Per-phase timing (`timing`)
                                  always launches chunks.                     */
    int jacobian;              /* GBA_JACOBIAN_ANALYTIC (0): closed-form edge
                                  Jacobians (Sec. IV-B); GBA_JACOBIAN_AUTODIFF:
                                  forward-mode automatic differentiation
                                  (Sec. IV-C): the residual evaluated on dual
                                  numbers, one seeded input per evaluation
                                  giving one Jacobian column.  The solver's
                                  linearisation evaluates an edge's 12 columns
                                  in its lane; gba_eval_edges runs one lane per
                                  (edge, column).  Same storage either way.
                                  GBA_JACOBIAN_DYNAMIC (full solver only):
                                  no stored Jacobian; every product and pass
                                  that needs J recomputes it from the
                                  parameters (Sec. IV-B dynamic Jacobians,
                                  the minimum-memory form).                  */
    int solver;                /* GBA_SOLVER_SCHUR (0): PCG on the reduced
                                  camera system after eliminating the point
                                  blocks; GBA_SOLVER_FULL: PCG on the whole
                                  damped system H + lambda D (cameras and
                                  points together) with block-Jacobi 9x9 and
                                  3x3 diagonal blocks, the paper's own form
                                  (Sec. IV-D).  FULL needs each problem's
                                  camera vector in LDS (UNSUPPORTED above
                                  ~2,200 cameras) and no fixed-order mode.
                                  Read when the device graph is built.       */
} gba_options;

#define GBA_SOLVER_SCHUR 0
#define GBA_SOLVER_FULL 1

#define GBA_JACOBIAN_ANALYTIC 0
#define GBA_JACOBIAN_AUTODIFF 1
#define GBA_JACOBIAN_DYNAMIC 2

#define GBA_PCG_AUTO 0
#define GBA_PCG_CHUNKED 1
#define GBA_PCG_PERSISTENT 2

#define GBA_ACC_AUTO 0
#define GBA_ACC_LDS 1
#define GBA_ACC_CAMERA_PASS 2
#define GBA_ACC_CAMERA_BLOCKS 3

/* Summary of one gba_solve call. */
typedef struct gba_report {
    double initial_cost;       /* F at the start: 1/2 sum rho(s_e)           */
    double final_cost;
    double final_lambda;
    int trials;                /* linear solves run (accepted or not)        */
    int accepted;
    int pcg_iters_total;
    int termination;           /* gba_termination                            */
    double ms_total;           /* wall time of the call (host clock)         */
    double ms_linearize;       /* HIP-event times, when options.timing = 1   */
    double ms_precond;
    double ms_pcg;
    double ms_other;
    double ms_matvec;          /* summed duration of the matvec kernels      */
    int matvec_count;
    int reserved_i;
    size_t workspace_bytes;    /* device bytes held by the graph             */
} gba_report;

/* One LM trial (for comparisons and diagnostics). */
typedef struct gba_trial {
    double cost;               /* F before the trial                         */
    double candidate_cost;     /* F(x + dx)                                  */
    double lambda;             /* damping used                               */
    double model_decrease;     /* L = -(b^T dx + 1/2 dx^T H dx)              */
    double step_norm;          /* |dx|                                       */
    int accepted;
    int pcg_iters;
} gba_trial;

void gba_default_options(gba_options* out);

/* Create an empty graph on `device` with the given precision policy.
 * alloc/free may both be NULL (hipMalloc/hipFree are then used). */
gba_status gba_create(gba_precision precision, int device, gba_alloc_fn alloc,
                      gba_free_fn free_fn, void* ctx, gba_graph** out);

/* Issue all device work on this hipStream_t (e.g. torch's current stream). */
gba_status gba_set_stream(gba_graph* g, void* hip_stream);

/* Pre-size host staging for the given counts (Sec. IV-A: descriptors reserve
 * memory before vertices and constraints are added).  Optional. */
gba_status gba_reserve(gba_graph* g, int64_t n_cams, int64_t n_pts, int64_t n_edges);

/* Add n cameras: ids[n], params[n x 9] = (w0 w1 w2 t0 t1 t2 f k1 k2). */
gba_status gba_add_cameras(gba_graph* g, int64_t n, const int64_t* ids,
                           const double* params);

/* Add n points: ids[n], xyz[n x 3]. */
gba_status gba_add_points(gba_graph* g, int64_t n, const int64_t* ids,
                          const double* xyz);

/* Add n reprojection edges (binary constraints, Sec. IV-A): camera and point
 * ids, uv[n x 2] observed pixel, info[n x 3] = (O00, O01, O11) of the 2x2
 * information matrix Omega (symmetric positive definite), or NULL for the
 * identity (the paper's nullptr-means-identity precision matrix).  Edges are
 * numbered in insertion order starting at 0. */
gba_status gba_add_edges(gba_graph* g, int64_t n, const int64_t* cam_ids,
                         const int64_t* pt_ids, const double* uv,
                         const double* info);

/* Hold a vertex constant (kind 0 = camera, 1 = point; Sec. IV-A set_fixed). */
gba_status gba_set_fixed(gba_graph* g, int kind, int64_t id, int fixed);

/* Include (1) or exclude (0) an edge (Sec. IV-A set_active / optimisation
 * level).  Excluded edges contribute neither cost nor linear terms. */
gba_status gba_set_edge_active(gba_graph* g, int64_t edge_index, int active);

/* Robust kernel for every edge (Background, Eq. 7); delta > 0 for Huber. */
gba_status gba_set_robust_kernel(gba_graph* g, gba_loss loss, double delta);

gba_status gba_set_options(gba_graph* g, const gba_options* opts);

/* Build the device graph (id maps, point-major and camera-major edge orders,
 * workspace) and upload it.  gba_solve calls it when the graph changed. */
gba_status gba_prepare(gba_graph* g);

/* Run up to max_iters LM trials from the current parameters (tol as in
 * gba_termination): the Levenberg-Marquardt iteration of the Background
 * section (the damped normal equations of Eq. normal-equations, solved by PCG
 * as in the mixed-precision solver section; the step kept when the cost
 * falls).  Synchronous: returns after the results are on device and the
 * report is filled (report may be NULL).  Returns GBA_OK whenever the solver
 * ran, including on early termination. */
gba_status gba_solve(gba_graph* g, int max_iters, double tol, gba_report* report);

/* Restore the parameters given at insertion time (device-side copy). */
gba_status gba_reset(gba_graph* g);

/* Current cost F = 1/2 sum rho(s_e) over active edges (FP64): the total
 * error of Eq. total-error with the robust kernel applied per edge. */
gba_status gba_get_cost(gba_graph* g, double* cost);

/* Current parameters (the vertices x of Eq. total-error), insertion order:
 * out[n_cams x 9] / out[n_pts x 3]; out is host memory the caller owns. */
gba_status gba_get_cameras(gba_graph* g, double* out);
gba_status gba_get_points(gba_graph* g, double* out);

/* Per-trial log of the last gba_solve: writes min(max_entries, trials)
 * entries and the count to *n_out. */
gba_status gba_get_trials(gba_graph* g, int max_entries, gba_trial* out, int* n_out);

/* Step-level entry points of the hot path, for verification.  All outputs
 * are host arrays in insertion order; entries of inactive edges are zero.
 *
 * gba_eval_edges: residual r[n_edges x 2] (pixel - observation), unweighted
 * Jacobians jc[n_edges x 2 x 9] (d r / d camera) and jp[n_edges x 2 x 3]
 * (d r / d point) at the current parameters, and the IRLS weight w[n_edges] =
 * rho'(r^T Omega r).  Jacobian columns of fixed vertices are zero.  Any
 * output pointer may be NULL. */
gba_status gba_eval_edges(gba_graph* g, double* r, double* jc, double* jp, double* w);

/* gba_eval_edges_noalloc: for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the outputs of gba_eval_edges, computed by the same kernels,
 * without any device or host allocation.  The graph must already be on the
 * device (gba_prepare, or a solve, after the last change): GBA_ERR_STATE
 * otherwise.  At most GBA_NOALLOC_MAX_EDGES inserted edges: GBA_ERR_UNSUPPORTED
 * otherwise.  The working memory is a fixed device array of the library
 * (about 14 MB, one per GPU, held until the process ends) that every call on
 * that GPU shares: calls that overlap on one GPU race on it.  Synchronous
 * (returns after the outputs are in the caller's arrays). */
#define GBA_NOALLOC_MAX_EDGES 65536
gba_status gba_eval_edges_noalloc(gba_graph* g, double* r, double* jc, double* jp, double* w);

/* gba_eval_normal_equations: the blocks of H = sum J^T w Omega J and
 * b = sum J^T w Omega r (Eq. 5) at the current parameters: hcc[n_cams x 81],
 * bc[n_cams x 9], hpp[n_pts x 9], bp[n_pts x 3] (row-major 9x9 / 3x3). */
gba_status gba_eval_normal_equations(gba_graph* g, double* hcc, double* bc,
                                     double* hpp, double* bp);

/* gba_eval_step: one damped step at the current parameters and damping
 * lambda, computed as the hot path does (point elimination, PCG on the
 * reduced camera system with the options' settings, back-substitution):
 * dcam[n_cams x 9], dpt[n_pts x 3]; *pcg_iters receives the PCG count. */
gba_status gba_eval_step(gba_graph* g, double lambda, double* dcam, double* dpt,
                         int* pcg_iters);

/* gba_time_matvec (measurement): linearise at the current parameters, form
 * the damped reduced camera system at `lambda` as gba_eval_step does, run one
 * PCG iteration, then run `launches` Schur products (the PCG hot loop's
 * dominant kernel, with the iteration's stop decision it takes first) back to
 * back on the graph's stream between two HIP events; *avg_us receives the
 * average duration of one product in microseconds.  The parameters are not
 * changed. */
gba_status gba_time_matvec(gba_graph* g, double lambda, int launches, double* avg_us);

/* gba_hbm_probe (measurement): read the `bytes` (a positive multiple of 16)
 * of device memory at `buf` once per launch with 16-byte loads, `launches`
 * times back to back on `stream` (a hipStream_t, NULL: the null stream) of
 * `device`, between two HIP events; each of the 2048 workgroups writes one
 * 8-byte word to the device array `sink` (2048 words, caller-owned).  A
 * launch reads exactly `bytes` and writes 16 KiB, which calibrates the HBM
 * byte counters of a profiler; *avg_us receives the average duration of one
 * launch.  INVALID_ARG for null pointers, a size that is not a positive
 * multiple of 16, or launches < 1. */
gba_status gba_hbm_probe(int device, const void* buf, size_t bytes, double* sink, int launches,
                         void* stream, double* avg_us);

const char* gba_last_error(const gba_graph* g);

/* Release all device and host memory of the graph.  NULL is ignored. */
void gba_destroy(gba_graph* g);

/* ====================================================================
 * Serving: many small (local) bundle-adjustment problems solved
 * concurrently on one GPU.
 *
 * Requests are admitted while both a slot and device memory are free (the
 * memory budget bounds the device bytes of every resident request: its
 * uploaded image plus its share of the batch workspace).  Resident problems
 * are packed into one batch whose kernels work on problem-aligned
 * decompositions: each workgroup serves one problem, so every problem keeps
 * its own damping, PCG state, scalars and accept / reject decisions, and the
 * LM iterations of all resident problems advance together (one batched trial
 * at a time).  A request that arrives while others run is uploaded
 * asynchronously and joins the batch at the next trial boundary; a finished
 * problem leaves it.  With fixed decomposition sizes (always the case in the
 * server) a problem's arithmetic does not depend on its batch mates: its
 * result is the same alone and in any mix.
 *
 * The paper batches constraints and vertices of one graph for its kernels
 * (Sec. IV-B); serving several graphs at once is this library's production
 * form of the same method, not a construct of the paper.
 *
 * Threading: gba_server_submit / poll / stats may be called from any thread;
 * one internal thread drives the device.
 * ==================================================================== */
typedef struct gba_server gba_server;

/* One request: a complete problem with dense, request-local indices. */
typedef struct gba_problem {
    int32_t n_cams;
    int32_t n_pts;
    int64_t n_edges;
    const double* cams;          /* [n_cams x 9] as in gba_add_cameras          */
    const double* pts;           /* [n_pts x 3]                                 */
    const int32_t* cam_idx;      /* [n_edges] in [0, n_cams)                    */
    const int32_t* pt_idx;       /* [n_edges] in [0, n_pts)                     */
    const double* uv;            /* [n_edges x 2] observed pixels               */
    const double* info;          /* [n_edges x 3] or NULL (identity)            */
    const uint8_t* cam_fixed;    /* [n_cams] nonzero = constant, or NULL        */
    const uint8_t* pt_fixed;     /* [n_pts] or NULL                             */
    int32_t max_iters;           /* LM trials (as gba_solve)                    */
    int32_t reserved;
    double tol;                  /* as gba_solve                                */
} gba_problem;

/* Result of one request.  cams / pts are caller buffers sized for the
 * request (or NULL to skip); the rest is filled by gba_server_poll. */
typedef struct gba_result {
    double* cams;                /* [n_cams x 9]                                */
    double* pts;                 /* [n_pts x 3]                                 */
    gba_report report;           /* ms_total = service time (admission to result) */
    double latency_ms;           /* submission to result                        */
    double queue_ms;             /* submission to admission                     */
    int32_t batch_peak;          /* most problems resident with it in one trial */
    int32_t reserved;
} gba_result;

typedef struct gba_server_config {
    gba_precision precision;     /* (GBA_MIXED_FP32)                            */
    int device;                  /* (0)                                         */
    size_t hbm_budget_bytes;     /* device bytes for all resident requests (4 GiB) */
    int max_slots;               /* resident requests at most (64; <= 4096)     */
    gba_loss loss;               /* (GBA_LOSS_HUBER)                            */
    double delta;                /* (1.0)                                       */
    gba_options options;         /* as gba_set_options (defaults)               */
    const char* tune_db;         /* tuning database written by the autotuner, or
                                    NULL for built-in sizes; read at creation   */
    int tiles_per_block;         /* > 0 overrides the database                  */
    int edges_per_block;
    int pts_per_block;
    int pcg_sync_every;
    int reserved[8];
} gba_server_config;

typedef struct gba_serving_stats {
    int64_t submitted, admitted, rejected, completed, collected;
    int64_t in_flight;           /* resident now                                */
    int64_t queued;              /* waiting for admission                       */
    int64_t trials_run;          /* batched LM trials issued                    */
    int64_t repacks;             /* batch rebuilds on membership change         */
    double mean_batch;           /* mean resident problems per batched trial   */
    double p50_latency_ms, p99_latency_ms;  /* over completed requests          */
    double p50_service_ms, p99_service_ms;
    double solves_per_s;         /* completed / (last completion - first submission) */
    size_t bytes_in_use, bytes_peak, budget;
    int tiles_per_block, edges_per_block, pts_per_block, pcg_sync_every;  /* in use */
} gba_serving_stats;

void gba_server_default_config(gba_server_config* out);

/* Create a server: reserves the budget on the device (one allocation from
 * alloc / free, or hipMalloc when both are NULL) and starts its thread. */
gba_status gba_server_create(const gba_server_config* cfg, gba_alloc_fn alloc,
                             gba_free_fn free_fn, void* ctx, gba_server** out);

/* Copy a request (all arrays are read before return), validate it and
 * queue it.  GBA_ERR_BUDGET when it can never fit the budget. */
gba_status gba_server_submit(gba_server* s, const gba_problem* req, uint64_t* ticket);

/* Collect a result: GBA_PENDING while the request runs (wait = 0), or block
 * until it is done (wait != 0).  A collected ticket is forgotten. */
gba_status gba_server_poll(gba_server* s, uint64_t ticket, int wait, gba_result* out);

gba_status gba_server_stats(gba_server* s, gba_serving_stats* out);

/* Message of the last failed server call or of a failure of its thread. */
const char* gba_server_last_error(gba_server* s);

/* Stop the thread (finishing resident requests is not waited for) and
 * release everything.  NULL is ignored. */
void gba_server_destroy(gba_server* s);

/* ====================================================================
 * Visual-inertial factors (Background Eq. 8; Sec. V-C): the inertial
 * residual between consecutive keyframes from preintegrated IMU
 * measurements, and rectified stereo reprojection.  Evaluation calls for
 * verification and for building solvers on them; device memory is allocated
 * and freed inside each call, inputs and outputs are host arrays owned by the
 * caller.
 *
 * Keyframe state (15 doubles): rotation world <- body as an angle-axis
 * vector (3), position (3) and velocity (3) in the world frame, gyroscope
 * bias (3), accelerometer bias (3).  Jacobian columns are the local
 * perturbations R Exp(dtheta) (right), p + dp, v + dv, b + db.  Gravity is
 * (0, 0, -9.81) in the world frame.
 * ==================================================================== */

#define GBA_VI_PRE_STRIDE 148   /* doubles per preintegrated interval */

/* gba_vi_preintegrate: IMU preintegration of n intervals (on-manifold
 * discrete propagation).  Interval f holds the samples
 * [sample_off[f], sample_off[f+1]) of gyro / acc (3 doubles each, one every
 * dt seconds) and is integrated with the bias estimates bias0[6f..6f+5]
 * (b_g, then b_a).  out[148 f ..]: dt_total, dR (3x3 row-major), dv, dp, the
 * bias Jacobians dR/db_g, dv/db_g, dv/db_a, dp/db_g, dp/db_a (3x3 each), the
 * biases b_g0, b_a0, and the covariance (9x9 over [dphi, dv, dp]) from the
 * continuous noise densities sigma_g, sigma_a.  INVALID_ARG for a negative
 * n, decreasing offsets, sample_off[0] != 0, dt <= 0 or negative sigmas. */
gba_status gba_vi_preintegrate(int device, int n, const int64_t* sample_off, const double* gyro,
                               const double* acc, double dt, const double* bias0, double sigma_g,
                               double sigma_a, double* out);

/* gba_vi_eval_inertial: the inertial factors between keyframes f and f + 1
 * (f = 0 .. n_kf - 2) from states[15 n_kf] and their preintegrated intervals
 * pre[148 (n_kf - 1)]: r[9 f ..] = (r_R, r_v, r_p) with
 *   r_R = Log((dR Exp(JRg dbg))^T Ri^T Rj),
 *   r_v = Ri^T (vj - vi - g dt) - (dv + Jvg dbg + Jva dba),
 *   r_p = Ri^T (pj - pi - vi dt - g dt^2 / 2) - (dp + Jpg dbg + Jpa dba),
 * dbg, dba the bias of keyframe f minus the interval's b_g0, b_a0; J[216 f ..]
 * the 9 x 24 Jacobian (row-major) over dtheta_i, dp_i, dv_i, dbg_i, dba_i,
 * dtheta_j, dp_j, dv_j by forward-mode AD (one lane per column). */
gba_status gba_vi_eval_inertial(int device, int n_kf, const double* states, const double* pre,
                                double* r, double* J);

/* gba_vi_eval_stereo: rectified stereo reprojection of n_obs observations
 * (keyframe kf[e], point pt[e], obs[3e..] = u_l, v_l, u_r) with
 * intr = (fx, fy, cx, cy, baseline): Xc = R^T (X - p), u_l = fx Xc_x / Xc_z
 * + cx, v_l = fy Xc_y / Xc_z + cy, u_r = u_l - fx baseline / Xc_z;
 * r[3e..] = prediction - obs, J[27 e ..] the 3 x 9 Jacobian over dtheta, dp
 * of the keyframe and dX of the point (forward-mode AD).  UNKNOWN_ID for an
 * index out of range. */
gba_status gba_vi_eval_stereo(int device, int n_kf, const double* states, int64_t n_pts,
                              const double* pts, int64_t n_obs, const int64_t* kf, const int64_t* pt,
                              const double* obs, const double* intr, double* r, double* J);

/* A visual-inertial bundle-adjustment problem (Background Eq. 8; Sec. V-C):
 * keyframe states (angle-axis of R world <- body, p, v, b_g, b_a; 15 doubles
 * each, updated in place), map points (3 doubles each, updated in place),
 * stereo observations (keyframe kf[e], point pt[e], u_l, v_l, u_r) with the
 * rectified pair intr = (fx, fy, cx, cy, baseline), and the preintegrated
 * interval of each consecutive keyframe pair (gba_vi_preintegrate's output,
 * GBA_VI_PRE_STRIDE doubles per interval).  The cost is
 *   F = 1/2 sum_stereo rho(|r|^2 / sigma_px^2)          (Huber with threshold
 *       huber_delta2 on the squared norm; 0: squared loss)
 *     + 1/2 sum_inertial r^T cov^-1 r                    (gba_vi_eval_inertial)
 *     + 1/2 sum_bias r^T Omega_b r,  r = b_{f+1} - b_f,
 *       Omega_b = diag(I3 / (sigma_gw^2 dt), I3 / (sigma_aw^2 dt)).
 * The first keyframe is held fixed (the gauge). */
typedef struct gba_vi_problem {
    int32_t n_kf;              /* keyframes, >= 2                            */
    int32_t reserved0;
    int64_t n_pts;
    int64_t n_obs;
    double* states;            /* [15 n_kf] in/out                           */
    double* pts;               /* [3 n_pts] in/out                           */
    const int64_t* kf;         /* [n_obs]                                    */
    const int64_t* pt;         /* [n_obs]                                    */
    const double* obs;         /* [3 n_obs]                                  */
    const double* intr;        /* [5]                                        */
    const double* pre;         /* [GBA_VI_PRE_STRIDE (n_kf - 1)]             */
    double sigma_px;           /* > 0                                        */
    double huber_delta2;       /* >= 0                                       */
    double sigma_gw;           /* gyroscope bias random-walk density, > 0    */
    double sigma_aw;           /* accelerometer bias random-walk density     */
} gba_vi_problem;

typedef struct gba_vi_options {
    int pcg_max_iters;         /* PCG iterations per trial (100)             */
    int solver;                /* GBA_SOLVER_SCHUR (default): the points
                                  eliminated, PCG on the keyframe system S;
                                  GBA_SOLVER_FULL: PCG on the whole system  */
    double pcg_tol;            /* stop at |r| <= pcg_tol |r0| (1e-8)         */
    double initial_lambda;     /* 1e-4                                       */
    double min_diag, max_diag; /* clip of the damping diagonal (1e-6, 1e32)  */
    int precision;             /* GBA_FP64 (default), or GBA_MIXED_FP32: the
                                  per-observation array the PCG products
                                  stream (W = J_k^T J_p in the Schur form, the
                                  whitened 3 x 9 stereo J in the whole-system
                                  form) stored in FP32, all arithmetic and
                                  every other array FP64                     */
    int reserved1;
    double pcg_rejection_ratio;/* stop PCG and keep the best iterate when
                                  |r_k| > ratio * min_m<=k |r_m| (the
                                  paper's VI runs use 10); <= 0 or Inf
                                  disables (default: disabled)               */
} gba_vi_options;

void gba_vi_default_options(gba_vi_options* out);

/* gba_vi_solve: up to max_iters Levenberg-Marquardt trials on a
 * visual-inertial problem (Background Eq. 8; Sec. V-C), with the acceptance,
 * damping and stop rules of gba_solve (tol as in gba_termination), FP64
 * arithmetic (precision below), in one of two forms of the damped step:
 *   GBA_SOLVER_SCHUR: the point blocks eliminated (Eq. 5-6 on the keyframe /
 *     point partition), PCG on the keyframe system S (keyframe-keyframe
 *     blocks from the inertial terms and from the points two keyframes
 *     share) preconditioned by S's 15 x 15 diagonal blocks (exact when a
 *     keyframe observes each point at most once), then the point steps by
 *     back-substitution; the PCG tolerance applies to S's residual;
 *   GBA_SOLVER_FULL: the paper's form for it, PCG on the whole damped system
 *     over keyframe states and points, block-Jacobi preconditioned (15 x 15
 *     keyframe blocks, 3 x 3 point blocks).  Host arrays in and out (copied to and from
 * device memory the call allocates and frees; report.ms_other is that set-up
 * (orderings, allocation, uploads), report.ms_total - ms_other the LM
 * trials and the download, workspace_bytes the device bytes); report and the
 * first max_log
 * trials in log (n_log: their count) may be NULL / 0.  INVALID_ARG for
 * missing arrays, n_kf < 2, non-positive noise parameters, an unknown solver
 * form or precision, UNKNOWN_ID for
 * an index out of range, OOM when device memory runs out. */
gba_status gba_vi_solve(int device, const gba_vi_problem* prob, int max_iters, double tol,
                        const gba_vi_options* opts, gba_report* report, gba_trial* log,
                        int max_log, int* n_log);

#ifdef __cplusplus
}
#endif

#endif /* GBA_H */
