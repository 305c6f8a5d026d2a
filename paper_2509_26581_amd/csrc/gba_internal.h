// Internal interface between the host driver (gba_api.hip) and the gfx950
// kernels (gba_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gba {

constexpr int kWave = 64;
constexpr int kTileEdges = 64;        // edges per point tile (one wavefront)
constexpr int kChunkRuns = 1024;      // camera-major runs per workgroup chunk
constexpr int kHccN = 45;             // unique entries of a symmetric 9x9
constexpr int kHppN = 6;              // unique entries of a symmetric 3x3
constexpr int kHinvStride = 8;        // padded row of the damped inverse point blocks

// symmetric 9x9 packed upper triangle, row-major: index of (r, c), r <= c
__host__ __device__ constexpr int sym9(int r, int c) {
    return r <= c ? r * 9 - (r * (r - 1)) / 2 + (c - r) : c * 9 - (c * (c - 1)) / 2 + (r - c);
}
// symmetric 3x3 packed: 00 01 02 11 12 22
__host__ __device__ constexpr int sym3(int r, int c) {
    return r <= c ? r * 3 - (r * (r - 1)) / 2 + (c - r) : c * 3 - (c * (c - 1)) / 2 + (r - c);
}

enum Mode { kModeFP64 = 0, kModeFP32 = 1, kModeBF16 = 2 };

// Per-trial scalars read back by the host after each LM trial.
struct TrialScalars {
    double cost;         // F at the candidate (or at x for the initial eval)
    double b_dot_dx;     // b^T dx
    double quad;         // sum_e |J_e dx_e|^2 (weighted Jacobian)
    double step2;        // |dx|^2 over free variables
    double x2;           // |x|^2 over free variables
    int pcg_iters;
    int pcg_reason;
};

// PCG scalar state, written by the single-workgroup update kernels.
struct PcgState {
    double rz;           // r^T z of the current iterate
    double rr;           // r^T r
    double rr0;
    double min_rr;
    double thresh;       // stop when rr <= thresh
    int iters;
    int done;            // 0 running, 1 converged, 2 max iters, 3 breakdown, 4 rejected
    int use_best;
    int pad;
};

// Device view of one graph.  All arrays are device pointers.  Edge arrays are
// in point-major order (sorted by point, then camera) unless prefixed cm_
// (camera-major order, sorted by camera, then point).
struct DeviceGraph {
    int nc, np, ne;
    int n_tiles;         // point tiles (whole points, <= 64 edges, or one long point)
    int n_runs;          // camera-major runs of equal (camera, point)
    int n_chunks;        // camera-major workgroup chunks
    int has_info;
    int loss;            // 0 squared, 1 huber
    double delta;
    int mode;            // Mode
    int jac_bytes;       // bytes per stored Jacobian entry for the PCG copy

    // topology
    const int* tile_off;      // [n_tiles + 1] edge offsets
    const int* e_cam;         // [ne]
    const int* e_pt;          // [ne]
    const double* obs;        // [2][ne]
    const double* sinfo;      // [3][ne] upper Cholesky factor of Omega, or null
    const int* cm_run_off;    // [n_runs + 1] offsets into cm_* arrays
    const int* cm_pt;         // [ne]
    const double* cm_obs;     // [2][ne]
    const double* cm_sinfo;   // [3][ne] or null
    const int* chunk_run_off; // [n_chunks + 1]
    const int* chunk_cam;     // [n_chunks]
    const int* cam_chunk_off; // [nc + 1]
    const unsigned char* cam_fixed;  // [nc]
    const unsigned char* pt_fixed;   // [np]

    // parameters (FP64 master copies; candidate buffers swap with these)
    double* cam;              // [nc][9]
    double* pt;               // [np][3]
    double* cam_c;            // candidates
    double* pt_c;
    double* dpt;              // [np][3] point step of the last damped solve
    const double* cam_init;   // as inserted, for reset
    const double* pt_init;

    // linearisation (T = double or float; J copy may be bf16)
    void* jc;                 // [18][ne] weighted Jacobian w.r.t. camera (FP64/FP32/BF16)
    void* jp;                 // [6][ne]  weighted Jacobian w.r.t. point
    void* rw;                 // [2][ne]  weighted residual
    void* hpp;                // [6][np]
    void* bp;                 // [3][np]
    void* hcc;                // [45][nc] stored as [nc][45]
    void* wrun;               // [27][n_runs] W = sum_run J_c^T J_p per camera-major run
    void* bc;                 // [nc][9]
    double* hpp_inv;          // [np][8] damped inverse (FP64), 6 unique entries per 64-byte row
    void* minv;               // [nc][45] preconditioner inverse blocks

    // Schur / PCG vectors, [nc][9]
    void* v_x;
    void* v_r;
    void* v_z;
    void* v_p;
    void* v_q;
    void* v_best;

    // partial sums
    void* cam_partial;        // [grid_pp][9 nc]
    double* pq_partial;       // [grid_red]
    double* dot_partial;      // [2][pcg workgroups] r^T z, r^T r
    double* chunk_partial;    // [n_chunks][54]
    double* red_partial;      // [grid_edges][4] misc per-block sums
    double* cost_partial;     // [grid_edges]
    double* damp_partial;     // [grid_pts]
    PcgState* pcg;
    TrialScalars* scal;

    // launch geometry
    int grid_pp;              // workgroups of the point passes (one partial each)
    int block_pp;             // threads per point-pass workgroup
    int lds_pp;               // dynamic LDS bytes of the point passes
    int grid_red;             // workgroups of the partial reduction
    int grid_edges;           // workgroups of the per-edge passes
    int grid_pts;             // workgroups of the per-point kernels
};

struct LaunchCtx {
    hipStream_t stream;
};

// ---- launchers (gba_kernels.hip) --------------------------------------
// debug outputs of gba_eval_edges, point-major, all may be null
struct RawOut {
    double* r;   // [2][ne]
    double* jc;  // [18][ne]
    double* jp;  // [6][ne]
    double* w;   // [ne]
};

hipError_t launch_linearize(const DeviceGraph& g, hipStream_t s, const RawOut* raw);
hipError_t launch_cost(const DeviceGraph& g, hipStream_t s, const double* cam, const double* pt);
hipError_t launch_damp(const DeviceGraph& g, hipStream_t s, double lambda, double min_diag,
                       double max_diag);
hipError_t launch_precond(const DeviceGraph& g, hipStream_t s, double lambda, double min_diag,
                          double max_diag, int block_jacobi);
hipError_t launch_rhs(const DeviceGraph& g, hipStream_t s);
hipError_t launch_pcg_init(const DeviceGraph& g, hipStream_t s, double tol, int relative);
hipError_t launch_pcg_iter(const DeviceGraph& g, hipStream_t s, double lambda, double min_diag,
                           double max_diag, int max_iters, double reject_ratio,
                           hipEvent_t ev_mv0, hipEvent_t ev_mv1);
hipError_t launch_backsub(const DeviceGraph& g, hipStream_t s);
hipError_t launch_finish(const DeviceGraph& g, hipStream_t s);
hipError_t launch_assemble(const DeviceGraph& g, hipStream_t s);

}  // namespace gba
