// Internal interface between the host drivers (gba_api.hip, gba_serve.hip)
// and the gfx950 kernels (gba_kernels.hip).  Not part of the public ABI.
//
// A device graph holds P >= 1 independent bundle-adjustment problems laid out
// one after the other (cameras, points, point-major edges and tiles of a
// problem are contiguous).  A single solve is P = 1; the serving loop packs
// many resident problems into one graph.  Every kernel works on a
// problem-aligned decomposition: each workgroup handles items of exactly one
// problem, so per-workgroup partial sums add up per problem without atomics,
// and each problem carries its own damping, PCG state and trial scalars.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gba {

constexpr int kWave = 64;
constexpr int kTileEdges = 64;        // edges per point tile (one wavefront)
constexpr int kChunkRuns = 1024;      // camera-major runs per workgroup chunk
constexpr int kHinvStride = 8;        // padded row of the damped inverse point blocks
constexpr int kCamsPerBlock = 28;     // cameras per PCG-vector workgroup (252 components)
constexpr int kPcgBlock = 256;        // threads of the PCG-vector workgroups
constexpr int kCamPassBlock = 256;    // threads of the camera-major pass workgroups
constexpr int kCamBlock = 1024;       // cameras per block of the camera-blocked product pass
constexpr int kCamBlockThreads = 1024;   // threads of its workgroups
constexpr int kRedComps = 64;         // components per partial-reduction workgroup
constexpr int kMaxProblems = 4096;    // problems per device graph
constexpr int kMaxDevices = 64;       // devices tracked for per-device kernel attributes
#ifndef GBA_PP_BLOCK
#define GBA_PP_BLOCK 1024
#endif
constexpr int kPointPassBlock = GBA_PP_BLOCK;  // threads per point-pass workgroup

// symmetric 9x9 packed upper triangle, row-major: index of (r, c), r <= c
__host__ __device__ constexpr int sym9(int r, int c) {
    return r <= c ? r * 9 - (r * (r - 1)) / 2 + (c - r) : c * 9 - (c * (c - 1)) / 2 + (r - c);
}
// symmetric 3x3 packed: 00 01 02 11 12 22
__host__ __device__ constexpr int sym3(int r, int c) {
    return r <= c ? r * 3 - (r * (r - 1)) / 2 + (c - r) : c * 3 - (c * (c - 1)) / 2 + (r - c);
}

enum Mode { kModeFP64 = 0, kModeFP32 = 1, kModeBF16 = 2 };

// Per-problem scalars of one LM trial, read back by the host.
struct TrialScalars {
    double cost;         // F at the candidate (or at x for the initial eval)
    double b_dot_dx;     // b^T dx
    double quad;         // sum_e |J_e dx_e|^2 (weighted Jacobian)
    double step2;        // |dx|^2 over free variables
    double x2;           // |x|^2 over free variables
    int pcg_iters;
    int pcg_reason;
    int barrier_err;     // the persistent PCG's grid barrier gave up waiting (never expected)
    int pad_;
};

// Per-problem PCG state.
struct PcgState {
    double rz;           // r^T z of the current iterate
    double rr;           // r^T r
    double rr0;
    double min_rr;
    double thresh;       // stop when rr <= thresh
    int iters;
    int done;            // 0 running, 1 converged, 2 max iters, 3 breakdown, 4 rejected, 5 idle problem
    int use_best;
    int act;             // decisions only: the work of this iteration (kAct* bits)
    double beta;         // of the last step
    int fresh;           // no step taken yet (the first direction is p = z)
    int pad_;
};

// Work of one PCG iteration, decided at its start from the previous step's
// dot products (PcgState::act of a decision).
constexpr int kActRun = 1;        // a step with p = z + beta p
constexpr int kActFresh = 2;      // the first step, p = z
constexpr int kActKeepBest = 4;   // best = x before the step (rejection ratio)
constexpr int kActRestore = 8;    // x = best (stopped by the rejection ratio)
constexpr int kActState = 16;     // the state changed: the apply kernel stores it
constexpr int kActStep = kActRun | kActFresh;

// Problem-aligned work decomposition: workgroup b handles items
// [blk[3b], blk[3b+1]) of problem blk[3b+2]; the workgroups of problem p are
// prob_blk[p] .. prob_blk[p+1]-1.
struct Decomp {
    const int* blk;
    const int* prob_blk;
    int nblk;
};

__device__ __forceinline__ int decomp_block(const Decomp& d, int b, int& begin, int& end) {
    begin = d.blk[3 * b];
    end = d.blk[3 * b + 1];
    return d.blk[3 * b + 2];
}

// Device view of one graph.  All arrays are device pointers.  Edge arrays are
// in point-major order (sorted by problem, point, camera) unless prefixed cm_
// (camera-major order, sorted by camera, then point).
struct DeviceGraph {
    int nc, np, ne;
    int n_tiles;         // point tiles (whole points of one problem, <= 64 edges, or one long point)
    int n_runs;          // camera-major runs of equal (camera, point)
    int n_chunks;        // camera-major workgroup chunks
    int n_probs;         // P
    int has_info;
    int loss;            // 0 squared, 1 huber
    double delta;
    int mode;            // Mode
    int jac_bytes;       // bytes per stored Jacobian entry

    // topology
    // camera-blocked order of the PCG product's camera pass (two-pass form,
    // one problem; bo_chunks == 0: off): edges grouped by block of kCamBlock
    // cameras, in point order inside a block, cut into chunks (one workgroup
    // each, within one block); the chunk's LDS sums of J_c^T J_p z_j per
    // camera of the block go to bo_partial[chunk][kCamBlock][9] (vector type)
    int bo_chunks;
    int bo_nblk;
    const int* bo_off;        // [bo_chunks + 1] edge ranges (block order)
    const int* bo_blk;        // [bo_chunks] block of each chunk
    const int* bo_blk_chunk;  // [bo_nblk + 1] chunks of each block
    const int* bo_perm;       // [ne] point-major edge of each block-order edge
    const int* bo_pt;         // [ne]
    const int* bo_cam;        // [ne]
    void* jst_bo;             // the stored Jacobian in block order
    void* bo_partial;

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

    // problems
    const int* cam_prob;      // [nc] problem of each camera
    const int* pt_prob;       // [np]
    const int* prob_cam_off;  // [P + 1] camera range of each problem
    double* lam;              // [P] damping of the current trial; negative: problem idle (no PCG)
    int* accept;              // [P] 1: commit the candidate of this problem
    PcgState* pcg;            // [P]
    TrialScalars* scal;       // [P]
    PcgState* pcg_dec;        // [P] decision of the current PCG iteration (from the product)
    PcgState* pcg_host;       // [P] mapped host copies of pcg (at the start and once stopped), or null
    TrialScalars* scal_host;  // [P]

    // parameters (FP64 master copies and candidates)
    double* cam;              // [nc][9]
    double* pt;               // [np][3]
    double* cam_c;            // candidates
    double* pt_c;
    double* dpt;              // [np][3] point step of the last damped solve
    double* cam_init;         // as inserted, for reset
    double* pt_init;

    // linearisation (T = double or float blocks; Jacobian FP64 / FP32 / BF16)
    void* jst;                // stored weighted Jacobian, 24 entries per edge in 16-byte chunks
                              // (layout: jac_chunk in gba_device.h), ceil(ne/64)*64 edges
    void* rw;                 // [2][ne]  weighted residual
    void* hpp;                // [6][np]
    void* bp;                 // [3][np]
    void* hcc;                // [nc][45]
    void* bc;                 // [nc][9]
    void* hpp_inv;            // [np][8] damped inverse (inverted in FP64, stored in the block
                              // type), 6 unique entries per row
    void* jst_cm;             // camera-major copy of jst, same layout
    void* zbuf;               // [np][4] point vectors between the two passes (vector type)
    void* minv;               // [nc][45] preconditioner inverse blocks

    // Schur / PCG vectors, [nc][9]
    void* v_x;
    void* v_r;
    void* v_z;
    void* v_p;
    void* v_q;
    void* v_best;

    // decompositions and partial sums
    Decomp dc_pp;             // point tiles (RHS, matvec, back-substitution)
    Decomp dc_red;            // camera components, <= kRedComps per workgroup
    Decomp dc_cam;            // cameras, <= kCamsPerBlock per workgroup
    Decomp dc_edges;          // edges (cost)
    Decomp dc_pts;            // points (damping)
    const int* pp_part_off;   // [dc_pp.nblk] offset of each point-pass partial vector
    double* cam_partial;      // point-pass camera partials
    double* pq_partial;       // [dc_red.nblk]
    double* dot_partial;      // [2][dc_cam.nblk] r^T z, r^T r
    double* camupd_partial;   // [3][dc_cam.nblk] b^T dc, |dc|^2, |c|^2
    double* chunk_partial;    // [n_chunks][54]
    double* red_partial;      // [4][dc_pp.nblk] back-substitution sums
    double* cost_partial;     // [dc_edges.nblk]
    double* damp_partial;     // [dc_pts.nblk]

    // launch geometry
    int block_pp;             // threads per point-pass workgroup
    int lds_pp;               // dynamic LDS bytes of the point passes (9 x max cameras of a problem)
    int pcg_max_iters;        // PCG stop rules, set by the PCG launchers
    double pcg_ratio;
    int cam_pass;             // 1: a problem's camera vector exceeds LDS (or fixed-order sums
                              // were asked for); the RHS and the Schur product take two
                              // passes (point-major: z_j into zbuf; camera-major over
                              // jst_cm: sums per chunk)
    int deterministic;        // 1: every sum in an order that depends only on the problem
                              // (not on the batch it is packed with)
    // Small problems: the last reduction workgroup of a problem to finish
    // runs that problem's PCG update (no update launch); red_count[P] counts
    // the finished reduction workgroups per problem (cleared at each PCG start
    // and by the last arrival)
    int fuse_apply;
    unsigned int* red_count;
    unsigned int* gbar;       // [kGbarWords] grid barrier of the persistent PCG: arrivals,
                              // generation, error flag; group arrival counters
                              // kGbarLine words apart
    int jacobian;             // GBA_JACOBIAN_*: closed form, forward-mode AD, dynamic (closed form)
    // full-Hessian PCG (the solver form without point elimination)
    int full;                 // 1: PCG on the whole damped system
    int dynamic;              // 1: no stored Jacobian; products recompute it from the parameters
    void* w_x;                // [np][3] point parts of the PCG vectors (vector type)
    void* w_r;
    void* w_z;
    void* w_p;
    void* w_q;
    void* w_best;
    double* pdot_partial;     // [2][dc_pts.nblk] point parts of r^T z, r^T r
    double* ppq_partial;      // [dc_pp.nblk] point part of p^T q
    double min_diag, max_diag;  // damping clamp (set by the full system's launchers)
};

// The storage types a kernel is instantiated with must be those of the
// graph's precision mode (another type would address the buffers with the
// wrong strides, past their ends); kernels check and return at once.
template <typename VT>
__device__ __forceinline__ bool vec_type_ok(const DeviceGraph& g) {
    return (sizeof(VT) == 8) == (g.mode == kModeFP64);
}
template <typename JS>
__device__ __forceinline__ bool jac_type_ok(const DeviceGraph& g) {
    return sizeof(JS) == (size_t)g.jac_bytes;
}

// ---- launchers (gba_kernels.hip) --------------------------------------
// outputs of gba_eval_edges in the caller's layout: edge q = pos[e] (the
// insertion index of point-major edge e) at r[2q..], jc[18q..] (row-major
// 2 x 9), jp[6q..] (2 x 3), w[q]; any of the four may be null
struct RawOut {
    double* r;
    double* jc;
    double* jp;
    double* w;
    const int* pos;   // [ne] point-major position -> insertion index
};

// Batch assembly on the device: copy (or fill) element ranges, adding a
// constant to 32-bit indices.  One workgroup per PackChunk.
enum PackKind { kPackI32 = 0, kPackF64 = 1, kPackU8 = 2, kPackFillI32 = 3, kPackFillF64 = 4 };
struct PackDesc {
    const void* src;   // unused by the fill kinds
    void* dst;
    long long n;       // elements
    int add;           // kPackI32: added to every element; kPackFillI32: the value
    int kind;          // PackKind
    double fval;       // kPackFillF64: the value
};
constexpr int kPackChunk = 4096;  // elements per workgroup
struct PackChunk {
    int desc;
    int begin;         // first element of this chunk
};
hipError_t launch_pack(const PackDesc* desc, const PackChunk* chunks, int n_chunks, hipStream_t s);

// p[0..n) = v with a fill kernel (no memset node, so it may be captured)
hipError_t launch_fill_f64(double* p, double v, size_t n, hipStream_t s);

// zero_blocks: clear Hpp and bp first (points without edges are never written;
// needed once per device-graph layout)
hipError_t launch_linearize(const DeviceGraph& g, hipStream_t s, const RawOut* raw, bool zero_blocks);
hipError_t launch_assemble(const DeviceGraph& g, hipStream_t s);
hipError_t launch_cost(const DeviceGraph& g, hipStream_t s, const double* cam, const double* pt);
hipError_t launch_cost_finish(const DeviceGraph& g, hipStream_t s);
hipError_t launch_damp(const DeviceGraph& g, hipStream_t s, double min_diag, double max_diag);
// jacobi_scaling: with the identity preconditioner, apply diag(s)^2 with
// s_k = 1 / (1 + sqrt(Hcc_kk)) (the column-scaled system); no effect under
// block Jacobi
hipError_t launch_precond(const DeviceGraph& g, hipStream_t s, double min_diag, double max_diag,
                          int block_jacobi, int jacobi_scaling);
hipError_t launch_rhs(const DeviceGraph& g, hipStream_t s);
// true: launch_precond also forms the reduced RHS (then launch_rhs is not
// needed); false: call launch_rhs first
bool precond_forms_rhs(const DeviceGraph& g, int block_jacobi);
hipError_t launch_pcg_init(const DeviceGraph& g, hipStream_t s, double tol, int relative);
hipError_t launch_pcg_iter(const DeviceGraph& g, hipStream_t s, double min_diag, double max_diag,
                           int max_iters, double reject_ratio, hipEvent_t ev_mv0,
                           hipEvent_t ev_mv1);
// the Schur product of a PCG iteration alone (its decision and the q
// partials, no update)
hipError_t launch_matvec(const DeviceGraph& g, hipStream_t s, int max_iters, double reject_ratio);
// Every PCG iteration of every problem in one cooperative launch (the
// phases of launch_pcg_iter separated by grid barriers), after
// launch_pcg_init.  hipErrorNotSupported when the device has no cooperative
// launch or the grid would not be co-resident.
// Its workgroups are point-pass sized: the product and the reduction run as
// launched, the vector updates and the camera-major pass as kSubs launched
// workgroups side by side.
constexpr int kPersistentBlock = kPointPassBlock;
// the fused update runs when every problem has at most this many cameras (at
// most four camera-aligned update workgroups, one pass of the reduction's
// 1024 threads)
constexpr int kFuseApplyCams = 4 * (kPcgBlock / 9);
// The grid barrier counts arrivals in kGbarGroups groups (workgroup index
// modulo kGbarGroups), each counter on its own 128-byte line, then the groups
// at the top: no one address takes every workgroup's atomic.
constexpr int kGbarGroups = 8;
constexpr int kGbarLine = 32;                                  // words per 128-byte line
constexpr int kGbarWords = kGbarLine * (1 + kGbarGroups);
static_assert(kPersistentBlock % kPcgBlock == 0 && kPersistentBlock % kCamPassBlock == 0,
              "persistent workgroups hold whole vector and camera-pass workgroups");
hipError_t launch_pcg_persistent(const DeviceGraph& g, hipStream_t s, double min_diag, double max_diag,
                                 int max_iters, double reject_ratio);
// whether launch_pcg_persistent can run this graph on the current device
bool pcg_persistent_ok(const DeviceGraph& g);
hipError_t launch_backsub(const DeviceGraph& g, hipStream_t s);
hipError_t launch_finish(const DeviceGraph& g, hipStream_t s);
hipError_t launch_commit(const DeviceGraph& g, hipStream_t s);
// streaming read of n16 16-byte words (byte-counter calibration); one word
// per workgroup into sink[kProbeBlocks]
constexpr int kProbeBlocks = 2048;
hipError_t launch_hbm_probe(const void* buf, size_t n16, double* sink, hipStream_t s);

}  // namespace gba
