// Host-side building blocks shared by the graph API (gba_api.hip) and the
// serving loop (gba_serve.hip): the staged data of one problem, its sorted
// image (edge orders, tiles, runs, chunks in problem-local indices), the
// union plan of several problems (offsets, work decompositions, workspace
// layout), the device batch holding them, and the per-problem
// Levenberg-Marquardt driver.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "gba.h"
#include "gba_internal.h"

namespace gba {

// Staged (host) data of one problem, in insertion order.
struct HostProblem {
    std::vector<double> cam_params;   // [nc][9] current values
    std::vector<double> pt_params;    // [np][3]
    std::vector<double> cam_init;     // values at insertion
    std::vector<double> pt_init;
    std::vector<unsigned char> cam_fixed, pt_fixed;
    std::vector<int> e_cam, e_pt;     // per edge, insertion order
    std::vector<double> e_uv;         // [n][2]
    std::vector<double> e_info;       // [n][3] (empty when every edge has Omega = I)
    std::vector<unsigned char> e_active;
    int nc() const { return (int)cam_fixed.size(); }
    int np() const { return (int)pt_fixed.size(); }
    int n_edges() const { return (int)e_cam.size(); }
    bool any_free() const;
};

// Counts of one problem's image.
struct ImageCounts {
    int nc = 0, np = 0, ne = 0, n_tiles = 0, n_runs = 0, n_chunks = 0;
    bool info = false;
};

// Sorted image of one problem, problem-local indices.  Edge arrays are
// point-major (by point, then camera, then insertion) unless prefixed cm_
// (camera-major: by camera, then point).  SoA arrays are [k][ne].
struct HostImage {
    ImageCounts n;
    std::vector<int> e_cam, e_pt;            // [ne]
    std::vector<double> obs;                 // [2][ne]
    std::vector<double> sinfo;               // [3][ne] upper factor of Omega (when n.info)
    std::vector<int> tile_off;               // [n_tiles + 1]
    std::vector<int> cm_run_off;             // [n_runs + 1]
    std::vector<int> cm_pt;                  // [ne]
    std::vector<double> cm_obs;              // [2][ne]
    std::vector<double> cm_sinfo;            // [3][ne]
    std::vector<int> chunk_run_off;          // [n_chunks + 1]
    std::vector<int> chunk_cam;              // [n_chunks]
    std::vector<int> cam_chunk_off;          // [nc + 1]
    std::vector<int> pm_edge;                // point-major position -> insertion index
};

gba_status make_image(const HostProblem& h, HostImage& img, std::string& msg);

// Work-decomposition sizes.  0 selects the automatic size, which depends on
// the whole batch; non-zero sizes make every problem's decomposition (and so
// its rounding) independent of what else is in the batch.
struct Tuning {
    int tiles_per_block = 0;    // point tiles per point-pass workgroup
    int edges_per_block = 0;    // edges per cost workgroup
    int pts_per_block = 0;      // points per damping workgroup
    int pcg_sync_every = 8;     // PCG iterations launched between host checks
    int accumulation = GBA_ACC_AUTO;   // camera sums of the point passes
    int deterministic = 0;      // fixed-order reductions only (camera-major second pass)
    int solver = 0;             // GBA_SOLVER_* (full: point vectors and partials are laid out)
    int dynamic = 0;            // 1: dynamic Jacobians (no stored Jacobian copies)
};

struct HostDecomp {
    std::vector<int> blk;       // begin, end, problem per workgroup
    std::vector<int> prob_blk;  // [P + 1]
    int nblk() const { return (int)blk.size() / 3; }
};

// Layout of P problems packed one after the other.
struct UnionPlan {
    int P = 0;
    ImageCounts tot;
    std::vector<int> cam_off, pt_off, edge_off, tile_off, run_off, chunk_off;  // [P + 1]
    HostDecomp pp, red, cam, edges, pts;
    std::vector<int> part_off;   // [max(1, pp.nblk())]
    long long part_total = 0;
    int max_cams = 0;
    int lds_pp = 0;            // dynamic LDS bytes of the point passes (one-pass scheme)
    bool cam_pass = false;     // camera vector of some problem exceeds LDS (or fixed-order
                               // sums were asked for): two passes
    bool deterministic = false;
    bool full = false;         // full-Hessian PCG
    bool dynamic = false;      // no stored Jacobian
    bool cam_blocks = false;   // the camera-blocked product pass (one problem)
    int bo_nblk = 0, bo_chunk_cap = 0;   // its blocks, and a bound on its chunks
    int bo_target = 1;         // edges per chunk aimed at
    std::vector<int> cam_prob, pt_prob;   // problem of each union camera / point
};

struct DeviceInfo {
    int n_cu = 256;
    size_t max_lds = 65536;
};

// precision: the LDS camera sums of the point passes are in the vector type
// (FP64 or FP32), which decides whether a problem's camera vector fits
gba_status plan_union(const std::vector<const ImageCounts*>& probs, const Tuning& tune,
                      const DeviceInfo& dev, int precision, UnionPlan& u, std::string& msg);

// Device workspace of a union: assigns the DeviceGraph pointers inside
// [base, base + bytes) when base is non-null; returns the byte count.
size_t layout_union(const UnionPlan& u, int precision, void* base, DeviceGraph* d);

struct Allocator {
    gba_alloc_fn alloc = nullptr;
    gba_free_fn free_fn = nullptr;
    void* ctx = nullptr;
    void* allocate(size_t bytes) const;
    void release(void* p) const;
};

// Per-problem LM state (host).
struct ProblemLM {
    double F = 0.0, lam = 1e-4, nu = 2.0;
    double F0 = 0.0;
    int trials = 0, accepted = 0, pcg_total = 0;
    int max_iters = 0;
    double tol = 0.0;
    int term = GBA_TERM_NONE;
    bool running = false;
    std::vector<gba_trial> log;
};

constexpr int kMaxPcgChunk = 64;   // PCG iterations per replayed chunk, at most

// One or more problems resident on the device.
struct Batch {
    int precision = 0;
    hipStream_t stream = nullptr;
    Allocator allocator;
    bool owns_arena = true;
    void* arena = nullptr;
    size_t arena_bytes = 0;
    DeviceGraph dg{};
    UnionPlan plan;
    int P = 0;
    std::vector<std::vector<int>> pm_edge; // per problem: point-major position -> insertion index
    // PCG chunks replayed as HIP graphs (kernel arguments captured by value).
    // Between rebuilds the only fields that change are the parameter
    // pointers, swapped with the candidate's on an accepted step of a single
    // problem; only the dynamic-Jacobian product reads them, so its graphs
    // are kept per orientation of that swap and checked against the pointers.
    bool use_graphs = false;
    bool pcg_warm = false;          // one eager chunk ran (kernel attributes set)
    hipStream_t cap_stream = nullptr;   // capture only (the null stream cannot be captured)
    struct PcgGraph {
        hipGraphExec_t exec = nullptr;
        int iters = 0, max_iters = 0;
        double min_diag = 0, max_diag = 0, ratio = 0;
        const double* cam = nullptr;
        const double* pt = nullptr;
    } pcg_graph[kMaxPcgChunk + 1][2];   // by chunk length and parameter orientation
    void drop_graphs();
    // PCG iterations of the last damped step (the largest over the problems):
    // with graphs, the next step's first chunk is sized from it
    int last_pcg_iters = 0;
    int persistent_ok = -1;         // launch_pcg_persistent usable for this layout (-1: not checked)
    int jacobian = 0;               // GBA_JACOBIAN_* of the linearisation (options)
    // Hpp / bp of the current layout cleared once (points without edges keep 0)
    bool blocks_zeroed = false;
    // pinned host mirrors of the per-problem device arrays (capacity h_cap)
    int h_cap = 0;
    TrialScalars* h_scal = nullptr;
    PcgState* h_pcg = nullptr;
    // device addresses of the mapped h_scal / h_pcg: the trial finisher and
    // the PCG kernels (start, stop) write these copies, so the host reads
    // them after a synchronize
    TrialScalars* d_scal_host = nullptr;
    PcgState* d_pcg_host = nullptr;
    double* h_lam = nullptr;
    int* h_accept = nullptr;
    ~Batch();
    void release();               // workspace only (mirrors are kept)
    gba_status ensure_mirrors(int P, std::string& msg);
};

// Counts and flags of a union on b.dg (no pointers).
void set_union_scalars(Batch& b, int precision, int loss, double delta);

// Build a batch from problems (in the given order): sort, plan, allocate the
// workspace from the allocator, upload.  Parameters are taken from
// HostProblem::cam_params / pt_params.
gba_status build_batch(const std::vector<const HostProblem*>& probs, int precision, int loss,
                       double delta, const DeviceInfo& dev, const Tuning& tune,
                       const Allocator& alloc, hipStream_t stream, Batch& out, std::string& msg);

// Upload the decompositions and problem tables of b.plan into b.dg (async on
// b.stream; the host arrays of b.plan must stay alive until it completes).
gba_status upload_plan(Batch& b, std::string& msg);

// Timing hooks of one solve (HIP events on the batch stream).
struct Timers {
    bool on = false;
    std::vector<hipEvent_t> ev;
    double ms_mv = 0.0;
    int n_mv = 0;
    double ms_phase[4] = {0, 0, 0, 0};  // linearize, precondition, pcg, other
    hipError_t init();
    ~Timers();
};

// Start the LM state of the problems flagged in `fresh` (cost at the current
// parameters; running when they have active edges and free vertices), then
// linearise the batch when any problem runs.
gba_status batch_begin(Batch& b, const std::vector<const HostProblem*>& probs,
                       std::vector<ProblemLM>& lm, const std::vector<char>& fresh,
                       const gba_options& o, Timers* tm, std::string& msg);

// One LM trial for every running problem (damped solve, candidate cost,
// accept / reject, commit, re-linearisation).  Problems that terminate stop
// running.
gba_status batch_trial(Batch& b, std::vector<ProblemLM>& lm, const gba_options& o,
                       const Tuning& tune, Timers* tm, std::string& msg);

// Linearisation at the current parameters: per-edge residuals and Jacobians
// and, unless raw outputs are requested, the camera blocks (Hcc, bc, W).
gba_status batch_linearize(Batch& b, const RawOut* raw, Timers* tm, std::string& msg);

// Damped solve of every problem at its damping b.h_lam[p] (negative: idle),
// back-substitution and candidate cost; trial scalars land in b.h_scal.
gba_status batch_damped_step(Batch& b, const gba_options& o, const Tuning& tune, Timers* tm,
                             std::string& msg);

// Measurement: set up the damped reduced system at damping b.h_lam[p] (as
// batch_damped_step does), then run `launches` Schur products back to back
// between two events; *ms = average per product.
gba_status batch_time_matvec(Batch& b, const gba_options& o, int launches, double* ms,
                             std::string& msg);

// Current cost of every problem into b.h_scal[p].cost.
gba_status batch_cost(Batch& b, std::string& msg);

// Copy the current parameters of problem p to host arrays (problem order).
gba_status batch_download(Batch& b, int p, double* cams, double* pts, std::string& msg);

}  // namespace gba
