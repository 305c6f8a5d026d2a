// gfx950 kernels of one Levenberg-Marquardt iteration of bundle adjustment:
// edge linearisation, block assembly, point-block damping and inversion,
// Schur right-hand side, block-Jacobi preconditioner of the reduced camera
// system, preconditioned conjugate gradients with fused implicit Schur
// products, back-substitution, candidate cost and model decrease.
//
// Layout conventions (see gba_internal.h): edge arrays are structure-of-
// arrays in point-major order, so a wavefront reads the Jacobian entries of 64
// consecutive edges with one coalesced load per entry; camera vectors are
// [n_cams][9]; per-point blocks are [6][n_pts] / [3][n_pts].
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <mutex>
#include <type_traits>

#include "gba.h"
#include "gba_autodiff.h"
#include "gba_device.h"
#include "gba_internal.h"

namespace gba {

// An edge's residual and Jacobian in FP64: closed form, or (kAD) forward-mode
// automatic differentiation with the 12 columns evaluated one after another
// in this lane (the fused passes need the whole edge in one lane).
template <bool kAD>
__device__ __forceinline__ void edge_eval(const double* __restrict__ cam, const double* __restrict__ X,
                                          double ou, double ov, EdgeEval<double>& ev) {
    if constexpr (kAD) {
        // one dual evaluation live at a time (the loop is kept rolled); the
        // column lands in its register slot through selects
#pragma unroll 1
        for (int k = 0; k < 12; ++k) {
            double r[2], col[2];
            bal_jacobian_column<double>(cam, X, ou, ov, k, r, col);
#pragma unroll
            for (int m = 0; m < 9; ++m) {
                ev.jc[0][m] = m == k ? col[0] : ev.jc[0][m];
                ev.jc[1][m] = m == k ? col[1] : ev.jc[1][m];
            }
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                ev.jp[0][m] = 9 + m == k ? col[0] : ev.jp[0][m];
                ev.jp[1][m] = 9 + m == k ? col[1] : ev.jp[1][m];
            }
            ev.r[0] = r[0];
            ev.r[1] = r[1];
        }
    } else {
        bal_eval<double, true>(cam, X, ou, ov, ev);
    }
}

// ==========================================================================
// Linearisation: per edge residual and closed-form Jacobian, robust
// whitening (Eq. 7 kernel on s = r^T Omega r, IRLS weight), storage of the
// weighted blocks, and point-side sums Hpp_j = sum J_p^T J_p, bp_j =
// sum J_p^T r (Eq. 5) by segmented wavefront reductions over the point's
// contiguous edges.  One wavefront per tile of whole points.  The camera
// model is evaluated in FP64 in every precision mode and the Jacobian rounded
// once to its storage type JS (T is the block type): an FP32 evaluation
// leaves the gradient with components along the gauge directions, where the
// reduced system has only the damping as curvature, and the PCG then needs
// more iterations.  The linear system is built from the stored Jacobian, the
// gradient b from the FP64 one, so the LM fixed point is that of the FP64
// problem.  kRaw: also write the FP64 evaluation in the caller's layout (the
// edge evaluation entry point), a separate instantiation.  kAD: the Jacobian
// by forward-mode automatic differentiation.
// ==========================================================================
template <typename T, typename JS, bool kRaw, bool kAD>
__global__ __launch_bounds__(256) void k_linearize(DeviceGraph g, RawOut raw) {
    if (!vec_type_ok<T>(g) || !jac_type_ok<JS>(g)) return;   // instantiated for another mode
    const int l = lane_id();
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int nwaves = (gridDim.x * blockDim.x) >> 6;
    T* rw = (T*)g.rw;
    T* Hpp = (T*)g.hpp;
    T* bp = (T*)g.bp;
    const int ne = g.ne;
    for (int t = wave; t < g.n_tiles; t += nwaves) {
        const int e0 = g.tile_off[t], e1 = g.tile_off[t + 1];
        const int n = e1 - e0;
        double acc[9];
#pragma unroll
        for (int k = 0; k < 9; ++k) acc[k] = 0.0;
        int j_first = g.e_pt[e0];
        uint64_t starts = 0;
        int head = 0, end = 63;
        for (int c0 = 0; c0 < n; c0 += kWave) {
            const int idx = c0 + l;
            const bool valid = idx < n;
            const int e = e0 + (valid ? idx : 0);
            const int j = g.e_pt[e];
            const int i = g.e_cam[e];
            EdgeEval<double> ev;
            edge_eval<kAD>(g.cam + 9 * i, g.pt + 3 * j, g.obs[e], g.obs[ne + e], ev);
            double s, rho, w;
            whiten<double, true>(ev, g.sinfo, ne, e, g.loss, g.delta, g.cam_fixed[i] != 0,
                            g.pt_fixed[j] != 0, s, rho, w);
            if (valid) {
                if (!g.dynamic) jac_save<JS>(g.jst, e, ev.jc, ev.jp);
                rw[e] = (T)ev.r[0];
                rw[ne + e] = (T)ev.r[1];
                if (kRaw) {
                    // unweighted values for verification, at the edge's
                    // insertion index in the caller's layout
                    EdgeEval<double> ed;
                    bal_eval<double, true>(g.cam + 9 * i, g.pt + 3 * j, g.obs[e], g.obs[ne + e], ed);
                    const size_t q = (size_t)raw.pos[e];
                    const bool cf = g.cam_fixed[i] != 0, pf = g.pt_fixed[j] != 0;
                    if (raw.r) {
                        raw.r[2 * q] = ed.r[0];
                        raw.r[2 * q + 1] = ed.r[1];
                    }
                    if (raw.jc)
                        for (int a = 0; a < 2; ++a)
                            for (int k = 0; k < 9; ++k) raw.jc[18 * q + 9 * a + k] = cf ? 0.0 : ed.jc[a][k];
                    if (raw.jp)
                        for (int a = 0; a < 2; ++a)
                            for (int k = 0; k < 3; ++k) raw.jp[6 * q + 3 * a + k] = pf ? 0.0 : ed.jp[a][k];
                    if (raw.w) raw.w[q] = (double)w;
                }
            }
            // point-side contributions of this edge: the Hessian block from the
            // stored (rounded) Jacobian, the gradient from the FP64 one
            double jr[2][3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                jr[0][k] = jac_round<JS>(ev.jp[0][k]);
                jr[1][k] = jac_round<JS>(ev.jp[1][k]);
            }
            double h[9];
            h[0] = jr[0][0] * jr[0][0] + jr[1][0] * jr[1][0];
            h[1] = jr[0][0] * jr[0][1] + jr[1][0] * jr[1][1];
            h[2] = jr[0][0] * jr[0][2] + jr[1][0] * jr[1][2];
            h[3] = jr[0][1] * jr[0][1] + jr[1][1] * jr[1][1];
            h[4] = jr[0][1] * jr[0][2] + jr[1][1] * jr[1][2];
            h[5] = jr[0][2] * jr[0][2] + jr[1][2] * jr[1][2];
            h[6] = ev.jp[0][0] * ev.r[0] + ev.jp[1][0] * ev.r[1];
            h[7] = ev.jp[0][1] * ev.r[0] + ev.jp[1][1] * ev.r[1];
            h[8] = ev.jp[0][2] * ev.r[0] + ev.jp[1][2] * ev.r[1];
            if (n <= kWave) {
                const bool st = !valid || idx == 0 || g.e_pt[e - 1] != j;
                starts = __ballot(st);
                segment_of(starts, l, head, end);
                const SegScan seg(st);
#pragma unroll
                for (int k = 0; k < 9; ++k) acc[k] = seg.sum(valid ? h[k] : 0.0);
                if (valid && end == l) {   // the segment's last lane holds its sums
#pragma unroll
                    for (int k = 0; k < 6; ++k) Hpp[k * g.np + j] = (T)acc[k];
#pragma unroll
                    for (int k = 0; k < 3; ++k) bp[k * g.np + j] = (T)acc[6 + k];
                }
            } else {
#pragma unroll
                for (int k = 0; k < 9; ++k) acc[k] += valid ? h[k] : 0.0;
            }
        }
        if (n > kWave) {
            // one long point: full-wavefront sums
#pragma unroll
            for (int k = 0; k < 9; ++k) acc[k] = wave_sum(acc[k]);
            if (l == 0) {
#pragma unroll
                for (int k = 0; k < 6; ++k) Hpp[k * g.np + j_first] = (T)acc[k];
#pragma unroll
                for (int k = 0; k < 3; ++k) bp[k * g.np + j_first] = (T)acc[6 + k];
            }
        }
    }
}

// ==========================================================================
// Cost F = 1/2 sum_e rho(s_e) (Eq. 1 with the Eq. 7 kernel) in FP64 at the
// given parameters; per-workgroup partial sums.
// ==========================================================================
__global__ __launch_bounds__(256) void k_cost(DeviceGraph g, const double* __restrict__ cam,
                                              const double* __restrict__ pt) {
    __shared__ double red[16];
    int eb, ee;
    decomp_block(g.dc_edges, blockIdx.x, eb, ee);
    double acc = 0.0;
    const int ne = g.ne;
    for (int e = eb + (int)threadIdx.x; e < ee; e += blockDim.x) {
        const int i = g.e_cam[e], j = g.e_pt[e];
        EdgeEval<double> ev;
        bal_eval<double, false>(cam + 9 * i, pt + 3 * j, g.obs[e], g.obs[ne + e], ev);
        double s, rho, w;
        whiten<double, false>(ev, g.sinfo, ne, e, g.loss, g.delta, false, false, s, rho, w);
        acc += 0.5 * rho;
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) g.cost_partial[blockIdx.x] = acc;
}

// ==========================================================================
// Forward-mode AD Jacobians in the caller's layout (the edge evaluation entry
// point with GBA_JACOBIAN_AUTODIFF): one lane per (edge, column) pair; each
// lane evaluates the residual once on dual numbers with its column's input
// seeded and writes that column; the lane of column 0 also writes the
// residual and the robust weight.
// ==========================================================================
__global__ __launch_bounds__(256) void k_jacobian_autodiff(DeviceGraph g, RawOut raw) {
    const size_t total = 12 * (size_t)g.ne;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t t = blockIdx.x * (size_t)blockDim.x + threadIdx.x; t < total; t += stride) {
        const int e = (int)(t / 12), k = (int)(t % 12);
        const int i = g.e_cam[e], j = g.e_pt[e];
        double r[2], col[2];
        bal_jacobian_column<double>(g.cam + 9 * i, g.pt + 3 * j, g.obs[e], g.obs[g.ne + e], k, r, col);
        const size_t q = (size_t)raw.pos[e];
        if (k < 9) {
            const bool cf = g.cam_fixed[i] != 0;
            if (raw.jc) {
                raw.jc[18 * q + k] = cf ? 0.0 : col[0];
                raw.jc[18 * q + 9 + k] = cf ? 0.0 : col[1];
            }
        } else {
            const bool pf = g.pt_fixed[j] != 0;
            if (raw.jp) {
                raw.jp[6 * q + (k - 9)] = pf ? 0.0 : col[0];
                raw.jp[6 * q + 3 + (k - 9)] = pf ? 0.0 : col[1];
            }
        }
        if (k == 0) {
            if (raw.r) {
                raw.r[2 * q] = r[0];
                raw.r[2 * q + 1] = r[1];
            }
            if (raw.w) {
                EdgeEval<double> ev;
                ev.r[0] = r[0];
                ev.r[1] = r[1];
                double s, rho, w;
                whiten<double, false>(ev, g.sinfo, g.ne, e, g.loss, g.delta, false, false, s, rho, w);
                raw.w[q] = w;
            }
        }
    }
}

// ==========================================================================
// Point blocks: Hpp_lambda = Hpp + lambda diag(clamp(diag Hpp)) (Eq. 4-6 with
// the clamped diagonal, lambda of the point's problem), inverted in FP64 by
// Cholesky; fixed points get a zero inverse (no unknowns).  Also initialises the candidate points and
// the |x|^2 partial sums over free points.
// ==========================================================================
template <typename T>
__global__ __launch_bounds__(256) void k_damp_points(DeviceGraph g, double min_diag, double max_diag) {
    if (!vec_type_ok<T>(g)) return;   // instantiated for another mode
    __shared__ double red[16];
    int pb, pe;
    const int prob = decomp_block(g.dc_pts, blockIdx.x, pb, pe);
    const double lambda = fabs(g.lam[prob]);   // negative: problem idle this trial
    const T* Hpp = (const T*)g.hpp;
    double x2 = 0.0;
    for (int j = pb + (int)threadIdx.x; j < pe; j += blockDim.x) {
        const bool fixed = g.pt_fixed[j] != 0;
        double A[3][3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) A[r][c] = (double)Hpp[sym3(r, c) * g.np + j];
#pragma unroll
        for (int r = 0; r < 3; ++r) A[r][r] += lambda * fmin(fmax(A[r][r], min_diag), max_diag);
        bool ok = !fixed && spd_inverse<3>(A);
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = r; c < 3; ++c) ((T*)g.hpp_inv)[kHinvStride * j + sym3(r, c)] = (T)(ok ? A[r][c] : 0.0);
        const double p0 = g.pt[3 * j], p1 = g.pt[3 * j + 1], p2 = g.pt[3 * j + 2];
        g.pt_c[3 * j] = p0;
        g.pt_c[3 * j + 1] = p1;
        g.pt_c[3 * j + 2] = p2;
        g.dpt[3 * j] = 0.0;
        g.dpt[3 * j + 1] = 0.0;
        g.dpt[3 * j + 2] = 0.0;
        if (!fixed) x2 += p0 * p0 + p1 * p1 + p2 * p2;
    }
    x2 = block_sum(x2, red);
    if (threadIdx.x == 0) g.damp_partial[blockIdx.x] = x2;
}

// ==========================================================================
// Camera-major accumulation over runs of equal (camera, point), one
// workgroup per chunk of one camera's runs; partial sums per chunk.
//   kAssemble: recompute the run's edge Jacobians from the parameters (no
//              gathers of stored Jacobians) and sum Hcc_i = sum J_c^T J_c
//              (45 unique), bc_i = sum J_c^T r (9); store the rounded
//              Jacobian in camera-major order (jst_cm).
//   kPrecond:  sum over runs of W Hpp_lambda^{-1} W^T, W = sum over the run's
//              edges of J_c^T J_p, from jst_cm: the point-elimination term of
//              the 9x9 diagonal block of the Schur complement.
//   kPrecondRhs: kPrecond and the reduced RHS sums sum J_c^T J_p Hpp^-1 bp_j
//              (chunk slots 45..53).
// ==========================================================================
enum { kAssemble = 0, kPrecond = 1, kPrecondRhs = 2 };

// y += J_c^T (J_p t) for one edge (the reduced RHS term of a run).
template <typename A>
__device__ __forceinline__ void rhs_term(const A (&jc)[2][9], const A (&jp)[2][3],
                                         const A (&t)[3], A (&y)[9]) {
    const A u0 = jp[0][0] * t[0] + jp[0][1] * t[1] + jp[0][2] * t[2];
    const A u1 = jp[1][0] * t[0] + jp[1][1] * t[1] + jp[1][2] * t[2];
#pragma unroll
    for (int k = 0; k < 9; ++k) y[k] += jc[0][k] * u0 + jc[1][k] * u1;
}

template <typename T, typename JS, int kMode, bool kAD = false>
__global__ __launch_bounds__(256) void k_cam_accumulate(DeviceGraph g) {
    if (!vec_type_ok<T>(g) || !jac_type_ok<JS>(g)) return;   // instantiated for another mode
    constexpr int K = 45;
    __shared__ double red[4][54];
    const int chunk = blockIdx.x;
    const int cam = g.chunk_cam[chunk];
    const int rb = g.chunk_run_off[chunk], re = g.chunk_run_off[chunk + 1];
    const bool cfix = g.cam_fixed[cam] != 0;
    // block entries: the assembly evaluates the camera model in FP64 (see
    // the linearisation) and sums in FP64; the preconditioner computes and
    // accumulates its per-thread sums in the block type (FP32 in the mixed
    // modes: the blocks are a preconditioner, kept >= FP32); wavefront,
    // workgroup and chunk sums in FP64
    using AccT = std::conditional_t<kMode == kAssemble, double, T>;
    AccT acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = (AccT)0;
    // kPrecondRhs: the reduced RHS sums of the camera ride on the same pass over
    // the runs (accumulated as the block entries)
    AccT y[9];
    double gb[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        y[k] = (AccT)0;
        gb[k] = 0.0;
    }
    const int ne = g.ne;
    if (kMode == kAssemble) {
        // edge-parallel over the chunk's edges (no per-run state here): the
        // chain of dependent loads per edge is point index -> point
        const int qb = g.cm_run_off[rb], qe = g.cm_run_off[re];
        for (int q = qb + (int)threadIdx.x; q < qe; q += blockDim.x) {
            const int j = g.cm_pt[q];
            const bool pfix = g.pt_fixed[j] != 0;
            {
                EdgeEval<double> ev;
                edge_eval<kAD>(g.cam + 9 * cam, g.pt + 3 * j, g.cm_obs[q], g.cm_obs[ne + q], ev);
                double s, rho, w;
                whiten<double, true>(ev, g.cm_sinfo, ne, q, g.loss, g.delta, cfix, pfix, s, rho, w);
                // gradient from the unrounded Jacobian, before it is rounded
#pragma unroll
                for (int a = 0; a < 9; ++a) gb[a] += ev.jc[0][a] * ev.r[0] + ev.jc[1][a] * ev.r[1];
                double jc[2][9], jp[2][3];
#pragma unroll
                for (int a = 0; a < 9; ++a) {
                    jc[0][a] = jac_round<JS>(ev.jc[0][a]);
                    jc[1][a] = jac_round<JS>(ev.jc[1][a]);
                }
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    jp[0][a] = jac_round<JS>(ev.jp[0][a]);
                    jp[1][a] = jac_round<JS>(ev.jp[1][a]);
                }
                // camera-major copy of the stored Jacobian (the preconditioner
                // pass and the two-pass products read it)
                if (!g.dynamic) jac_save<JS>(g.jst_cm, q, jc, jp);
                int k = 0;
#pragma unroll
                for (int a = 0; a < 9; ++a)
#pragma unroll
                    for (int b = a; b < 9; ++b, ++k)
                        acc[k] += jc[0][a] * jc[0][b] + jc[1][a] * jc[1][b];
            }
        }
    } else {
        // edge-parallel over the chunk's edges too: a run of edges on one
        // (camera, point) pair (equal consecutive points; the chunk starts and
        // ends on run boundaries) is handled by its first edge, so the chain
        // of dependent loads per edge is point index -> inverse point block
        const int qb = g.cm_run_off[rb], qe = g.cm_run_off[re];
        const T* __restrict__ bp = (const T*)g.bp;
        for (int q0 = qb + (int)threadIdx.x; q0 < qe; q0 += blockDim.x) {
            const int j = g.cm_pt[q0];
            if (q0 > qb && g.cm_pt[q0 - 1] == j) continue;   // inside a run
            T b0 = 0, b1 = 0, b2 = 0;
            if (kMode == kPrecondRhs) {
                b0 = bp[j];
                b1 = bp[g.np + j];
                b2 = bp[2 * g.np + j];
            }
            const bool single = q0 + 1 == qe || g.cm_pt[q0 + 1] != j;
            AccT W[9][3];
            AccT Hi[3][3];
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
                for (int c = 0; c < 3; ++c) Hi[r][c] = (AccT)((const T*)g.hpp_inv)[kHinvStride * j + sym3(r, c)];
            AccT jc[2][9], jp[2][3];
            jac_load<JS>(g.jst_cm, q0, jc, jp);
            // the reduced RHS term of the run: J_c^T J_p t with
            // t = Hpp_lambda^-1 bp_j
            AccT t[3];
#pragma unroll
            for (int r = 0; r < 3; ++r)
                t[r] = Hi[r][0] * (AccT)b0 + Hi[r][1] * (AccT)b1 + Hi[r][2] * (AccT)b2;
            if (kMode == kPrecondRhs) rhs_term(jc, jp, t, y);
            if (single) {
                // one edge: W Hpp^-1 W^T = J_c^T A J_c with the 2x2
                // A = J_p Hpp^-1 J_p^T (fewer operations than forming W)
                AccT JH[2][3];
#pragma unroll
                for (int r = 0; r < 2; ++r)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        JH[r][c] = jp[r][0] * Hi[0][c] + jp[r][1] * Hi[1][c] + jp[r][2] * Hi[2][c];
                const AccT A00 = JH[0][0] * jp[0][0] + JH[0][1] * jp[0][1] + JH[0][2] * jp[0][2];
                const AccT A01 = JH[0][0] * jp[1][0] + JH[0][1] * jp[1][1] + JH[0][2] * jp[1][2];
                const AccT A11 = JH[1][0] * jp[1][0] + JH[1][1] * jp[1][1] + JH[1][2] * jp[1][2];
                AccT AJ[2][9];
#pragma unroll
                for (int b = 0; b < 9; ++b) {
                    AJ[0][b] = A00 * jc[0][b] + A01 * jc[1][b];
                    AJ[1][b] = A01 * jc[0][b] + A11 * jc[1][b];
                }
                int k = 0;
#pragma unroll
                for (int a = 0; a < 9; ++a)
#pragma unroll
                    for (int b = a; b < 9; ++b, ++k)
                        acc[k] += jc[0][a] * AJ[0][b] + jc[1][a] * AJ[1][b];
            } else {
                // several edges on one (camera, point) pair: W = sum J_c^T J_p
#pragma unroll
                for (int a = 0; a < 9; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) W[a][b] = jc[0][a] * jp[0][b] + jc[1][a] * jp[1][b];
                for (int q = q0 + 1; q < qe && g.cm_pt[q] == j; ++q) {
                    jac_load<JS>(g.jst_cm, q, jc, jp);
                    if (kMode == kPrecondRhs) rhs_term(jc, jp, t, y);
#pragma unroll
                    for (int a = 0; a < 9; ++a)
#pragma unroll
                        for (int b = 0; b < 3; ++b) W[a][b] += jc[0][a] * jp[0][b] + jc[1][a] * jp[1][b];
                }
                AccT WH[9][3];
#pragma unroll
                for (int a = 0; a < 9; ++a)
#pragma unroll
                    for (int c = 0; c < 3; ++c)
                        WH[a][c] = W[a][0] * Hi[0][c] + W[a][1] * Hi[1][c] + W[a][2] * Hi[2][c];
                int k = 0;
#pragma unroll
                for (int a = 0; a < 9; ++a)
#pragma unroll
                    for (int b = a; b < 9; ++b, ++k)
                        acc[k] += WH[a][0] * W[b][0] + WH[a][1] * W[b][1] + WH[a][2] * W[b][2];
            }
        }
    }
    // workgroup reduction of the accumulators (kPrecondRhs: 45 block entries
    // and 9 RHS sums)
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const AccT v = wave_sum(acc[k]);
        if (lane_id() == 0) red[w][k] = (double)v;
    }
    if (kMode == kPrecondRhs) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const double v = wave_sum((double)y[k]);
            if (lane_id() == 0) red[w][45 + k] = v;
        }
    }
    if (kMode == kAssemble) {
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const double v = wave_sum(gb[k]);
            if (lane_id() == 0) red[w][45 + k] = v;
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 54; k += blockDim.x) {
        const int nw = blockDim.x >> 6;
        double s = 0.0;
        for (int q = 0; q < nw; ++q) s += red[q][k];
        g.chunk_partial[chunk * 54 + k] = s;
    }
}

// One workgroup per camera: sum the chunk partials of the camera.
// kAssemble stores Hcc and bc.  kPrecond forms M_i = Hcc_lambda,i -
// sum W Hpp^-1 W^T and stores M_i^{-1} (FP64 Cholesky); the identity
// preconditioner stores I; fixed cameras store 0.  with_rhs (the pass ran as
// kPrecondRhs): also the reduced RHS r_i = -bc_i + the chunks' RHS sums.
template <typename T, int kMode>
__global__ __launch_bounds__(64) void k_cam_finalize(DeviceGraph g, double min_diag, double max_diag,
                                                     int block_jacobi, int with_rhs, int jacobi_scaling,
                                                     int full) {
    if (!vec_type_ok<T>(g)) return;   // instantiated for another mode
    __shared__ double Ms[54];
    const int i = blockIdx.x;
    const double lambda = kMode == kPrecond ? fabs(g.lam[g.cam_prob[i]]) : 0.0;
    const int k = threadIdx.x;
    const int c0 = g.cam_chunk_off[i], c1 = g.cam_chunk_off[i + 1];
    T* Hcc = (T*)g.hcc;
    if (kMode == kAssemble) {
        if (k < 54) {
            double s = 0.0;
            for (int c = c0; c < c1; ++c) s += g.chunk_partial[c * 54 + k];
            if (k < 45)
                Hcc[i * 45 + k] = (T)s;
            else
                ((T*)g.bc)[i * 9 + (k - 45)] = (T)s;
        }
        return;
    }
    if (kMode == kPrecond && with_rhs && k >= 45 && k < 54) {
        // reduced RHS r = -bc + the camera's chunk sums (from the same pass)
        double sr = 0.0;
        for (int q = c0; q < c1; ++q) sr += g.chunk_partial[q * 54 + k];
        ((T*)g.v_r)[i * 9 + (k - 45)] = (T)(-(double)((const T*)g.bc)[i * 9 + (k - 45)] + sr);
    }
    T* Minv = (T*)g.minv;
    const bool fixed = g.cam_fixed[i] != 0;
    if (fixed || !block_jacobi) {
        // identity, or with column scaling s_k = 1 / (1 + sqrt(H_kk)) the
        // preconditioner diag(s)^2 (PCG on the column-scaled system)
        if (k < 45) {
            int r = 0;
            while (k >= sym9(r, 8) + 1) ++r;
            const int c = k - sym9(r, r) + r;
            double m = 1.0;
            if (jacobi_scaling && r == c) {
                const double sk = 1.0 / (1.0 + sqrt(fmax((double)Hcc[i * 45 + k], 0.0)));
                m = sk * sk;
            }
            Minv[i * 45 + k] = (T)((!fixed && r == c) ? m : 0.0);
        }
        return;
    }
    if (k < 45) {
        int r = 0;
        while (k >= sym9(r, 8) + 1) ++r;
        const int c = k - sym9(r, r) + r;
        double h = (double)Hcc[i * 45 + k];
        if (r == c) h += lambda * fmin(fmax(h, min_diag), max_diag);
        // the Schur form subtracts the point-elimination term; the full
        // system's block is Hcc_lambda itself
        double s = 0.0;
        if (!full)
            for (int q = c0; q < c1; ++q) s += g.chunk_partial[q * 54 + k];
        Ms[k] = h - s;
    }
    // In-place Gauss-Jordan inversion of the SPD block over the workgroup:
    // 81 entries, thread k owns k and k + 64; pivot q replaces A by
    //   a_qq = 1/p, a_qj = a_qj/p, a_iq = -a_iq/p, a_ij -= a_iq a_qj / p
    // (p = a_qq; all from the values before the step).  The pivots are the
    // successive Schur complements, positive exactly when the block is
    // positive definite (the Cholesky condition).
    __shared__ double A[81];
    __shared__ int s_bad;
    const int e0 = k, e1 = k + 64;
    if (e0 < 81) A[e0] = Ms[sym9(e0 / 9, e0 % 9)];
    if (e1 < 81) A[e1] = Ms[sym9(e1 / 9, e1 % 9)];
    if (k == 0) s_bad = 0;
    __syncthreads();
    for (int q = 0; q < 9; ++q) {
        const double piv = A[q * 9 + q];
        if (!(piv > 0.0) || !isfinite(piv)) {   // uniform: every thread reads the same pivot
            if (k == 0) s_bad = 1;
            break;
        }
        const double ip = 1.0 / piv;
        double v0 = 0.0, v1 = 0.0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int e = h ? e1 : e0;
            if (e >= 81) continue;
            const int r = e / 9, c = e % 9;
            double v;
            if (r == q && c == q)
                v = ip;
            else if (r == q)
                v = A[e] * ip;
            else if (c == q)
                v = -A[e] * ip;
            else
                v = A[e] - A[r * 9 + q] * A[q * 9 + c] * ip;
            if (h) v1 = v; else v0 = v;
        }
        __syncthreads();
        if (e0 < 81) A[e0] = v0;
        if (e1 < 81) A[e1] = v1;
        __syncthreads();
    }
    __syncthreads();
    if (s_bad) {
        // rounding left the block indefinite: fall back to the damped diagonal
        if (k < 45) {
            int r = 0;
            while (k >= sym9(r, 8) + 1) ++r;
            const int c = k - sym9(r, r) + r;
            double h = (double)Hcc[i * 45 + sym9(r, r)];
            h += lambda * fmin(fmax(h, min_diag), max_diag);
            Minv[i * 45 + k] = (T)(r == c ? 1.0 / h : 0.0);
        }
        return;
    }
    if (k < 45) {
        int r = 0;
        while (k >= sym9(r, 8) + 1) ++r;
        const int c = k - sym9(r, r) + r;
        Minv[i * 45 + k] = (T)(0.5 * (A[r * 9 + c] + A[c * 9 + r]));
    }
}

// Sum of part[stride * q + off] over the workgroups q of a problem, by one
// wavefront (every lane gets the result).
__device__ __forceinline__ double wave_sum_blocks(const double* part, int stride, int off, int q0,
                                                  int q1, int sub = 0, int parts = 1) {
    // this wavefront is number `sub` of `parts` sharing the range; four
    // independent partial sums keep four loads in flight per lane
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    const int step = kWave * parts;
    int q = q0 + sub * kWave + lane_id();
    for (; q + 3 * step < q1; q += 4 * step) {
        s0 += part[stride * q + off];
        s1 += part[stride * (q + step) + off];
        s2 += part[stride * (q + 2 * step) + off];
        s3 += part[stride * (q + 3 * step) + off];
    }
    for (; q < q1; q += step) s0 += part[stride * q + off];
    return wave_sum((s0 + s1) + (s2 + s3));
}

// ==========================================================================
// PCG decisions.  The step taken by iteration i of the PCG is decided at its
// start, from the state (g.pcg) and the dot products r^T z, r^T r left by
// iteration i-1 (per camera-aligned workgroup in dot_partial): convergence,
// iteration limit, rejection ratio, beta = r^T z / (r^T z)_old.  The product
// kernel takes the decision (every workgroup from the same sums, so all agree;
// the problem's first workgroup stores it in g.pcg_dec for the later kernels
// of the iteration) and multiplies z, not the direction: by linearity
// S p = S z + beta S p_old, so the q reduction forms q = S z + beta q_old and
// p = z + beta p_old itself, and the apply kernel stores the state.  An
// iteration is three kernels with no separate scalar pass, and the product
// gathers one vector.
// ==========================================================================
__device__ __forceinline__ PcgState pcg_decision(const DeviceGraph& g, int prob) {
    PcgState st = g.pcg[prob];
    const int q0 = g.dc_cam.prob_blk[prob], q1 = g.dc_cam.prob_blk[prob + 1];
    double rz = wave_sum_blocks(g.dot_partial, 2, 0, q0, q1);
    double rr = wave_sum_blocks(g.dot_partial, 2, 1, q0, q1);
    if (g.full) {   // the point parts of the full system's vectors
        const int p0 = g.dc_pts.prob_blk[prob], p1 = g.dc_pts.prob_blk[prob + 1];
        rz += wave_sum_blocks(g.pdot_partial, 2, 0, p0, p1);
        rr += wave_sum_blocks(g.pdot_partial, 2, 1, p0, p1);
    }
    if (st.done) {   // stopped earlier: nothing to do
        st.act = 0;
        return st;
    }
    if (st.fresh) {  // first step: p = z, r^T z from the start
        st.fresh = 0;
        st.beta = 0.0;
        st.act = kActFresh | kActState;
        return st;
    }
    int done = 0, keep_best = 0;
    st.iters += 1;
    st.rr = rr;
    const double ratio = g.pcg_ratio;
    const bool track = ratio > 0.0 && isfinite(ratio);
    if (track && rr < st.min_rr) {
        st.min_rr = rr;
        keep_best = 1;
    } else if (track && rr > ratio * ratio * st.min_rr) {
        done = 4;
    }
    if (!done && rr <= st.thresh) done = 1;
    if (!done && st.iters >= g.pcg_max_iters) done = 2;
    st.beta = st.rz > 0.0 ? rz / st.rz : 0.0;
    st.rz = rz;
    st.done = done;
    if (keep_best) st.use_best = 1;
    st.act = kActState | (done ? 0 : kActRun) | (keep_best ? kActKeepBest : 0) |
             (done == 4 ? kActRestore : 0);
    return st;
}

// One entry of the direction: z + beta p_old rounded to the vector type, or z
// on the first step.
template <typename VT>
__device__ __forceinline__ VT dir_entry(VT z, VT pold, int act, VT beta) {
    return (act & kActRun) ? fma(beta, pold, z) : z;
}

// ==========================================================================
// Point passes over the stored weighted Jacobians, one wavefront per tile of
// whole points, camera-side sums privatised in LDS per workgroup and flushed
// as one partial camera vector per workgroup (no global atomics):
//   kRhs:     sum_e J_c^T J_p (Hpp^-1 bp_j)                       (reduced RHS)
//   kMatvec:  sum_e J_c^T J_p Hpp^-1 sum_e' J_p^T J_c' v_i'       (Schur product;
//             v = the PCG vector z, after the iteration's decision)
//   kBacksub: dp_j = -Hpp^-1 (bp_j + sum_e J_p^T J_c dc_i), candidate points,
//             model terms sum |J_e dx_e|^2, bp^T dp, |dp|^2
// ==========================================================================
enum { kRhs = 0, kMatvec = 1, kBacksub = 2 };

// One workgroup's share (decomposition block `bid`) of a point pass; the
// kernels below run one block per workgroup, the persistent PCG kernel loops
// over blocks.
template <typename VT, typename JS, typename AT, int kMode>
__device__ __forceinline__ void pp_body(const DeviceGraph& g, const int bid, const void* __restrict__ J,
                                        const VT* __restrict__ vin, AT* __restrict__ out) {
    if (!vec_type_ok<VT>(g) || !jac_type_ok<JS>(g)) return;   // instantiated for another mode
    // Arithmetic in the vector type (FP32 in the mixed modes); the camera sums
    // in LDS are AT = FP64 in every mode (ds_add_f64: FP32 LDS atomics
    // measured 2.4x slower for this pattern); the back-substitution's model
    // terms are summed in FP64 (gain ratio).
    using T = VT;
    T* zbuf = (T*)g.zbuf;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    AT* acc_lds = (AT*)smem_raw;
    __shared__ double red[16];
    __shared__ int s_act;
    int tb, te;
    const int prob = decomp_block(g.dc_pp, bid, tb, te);
    const int l = lane_id();
    const int c0 = g.prob_cam_off[prob];
    const int nc9 = 9 * (g.prob_cam_off[prob + 1] - c0);   // this problem's camera components
    // two-pass scheme: this pass only produces z_j (camera sums in k_cam_pass)
    const bool cpass = g.cam_pass != 0;
    // the product: this PCG iteration's decision, by the first wavefront
    // while the others clear the partials and request their first tile (edge
    // range, indices, Jacobian), whose loads so overlap the decision's two
    // dependent reads (about a microsecond at bal1m).  Only FP32 Jacobians
    // are requested ahead (FP64: 48 registers; BF16 measured slower with).
    constexpr bool kPreJ = std::is_same<JS, float>::value;
    const int w = threadIdx.x >> 6;
    const bool pre = kMode == kMatvec && w > 0 && tb + w < te;   // uniform per wavefront
    int f_e0 = 0, f_e1 = 0, f_j = 0, f_i = 0;
    T f_jc[2][9], f_jp[2][3];
    if (pre) {
        f_e0 = g.tile_off[tb + w];
        f_e1 = g.tile_off[tb + w + 1];
        if (f_e1 - f_e0 <= kWave) {
            const int e = f_e0 + (l < f_e1 - f_e0 ? l : 0);
            f_j = g.e_pt[e];
            f_i = g.e_cam[e];
            if constexpr (kPreJ) jac_load<JS>(J, e, f_jc, f_jp);
        }
    }
    if (kMode == kMatvec && threadIdx.x < kWave) {
        const PcgState d = pcg_decision(g, prob);
        if (threadIdx.x == 0) {
            s_act = d.act;
            if ((int)bid == g.dc_pp.prob_blk[prob]) g.pcg_dec[prob] = d;
        }
    }
    if (kMode != kBacksub && !cpass)
        for (int k = threadIdx.x; k < nc9; k += blockDim.x) acc_lds[k] = 0;
    if (kMode == kMatvec || (kMode == kRhs && !cpass)) __syncthreads();
    if (kMode == kMatvec && !(s_act & kActStep)) return;   // this problem's PCG has stopped
    const int nw = blockDim.x >> 6;
    const VT* bp = (const VT*)g.bp;
    double red_m = 0.0, red_b = 0.0, red_s = 0.0;
    for (int t = tb + w; t < te; t += nw) {
        const bool first = pre && t == tb + w;
        const int e0 = first ? f_e0 : g.tile_off[t];
        const int e1 = first ? f_e1 : g.tile_off[t + 1];
        const int n = e1 - e0;
        if (n <= kWave) {
            const bool valid = l < n;
            const int e = e0 + (valid ? l : 0);
            const int j = first ? f_j : g.e_pt[e];
            const int i = first ? f_i : g.e_cam[e];
            const int jprev = __shfl_up(j, 1);   // the previous edge of the tile
            const bool st = !valid || l == 0 || jprev != j;
            const uint64_t starts = __ballot(st);
            int head, end;
            segment_of(starts, l, head, end);
            T jc[2][9], jp[2][3];
            if (kPreJ && first) {
#pragma unroll
                for (int a = 0; a < 2; ++a) {
#pragma unroll
                    for (int k = 0; k < 9; ++k) jc[a][k] = f_jc[a][k];
#pragma unroll
                    for (int k = 0; k < 3; ++k) jp[a][k] = f_jp[a][k];
                }
            } else {
                jac_load<JS>(J, e, jc, jp);
            }
            T z[3];
            T pc[9];
            if (kMode == kRhs) {
                const T b0 = (T)bp[j], b1 = (T)bp[g.np + j], b2 = (T)bp[2 * g.np + j];
                const VT* H = (const VT*)g.hpp_inv + kHinvStride * j;
                const T h00 = H[0], h01 = H[1], h02 = H[2], h11 = H[3], h12 = H[4], h22 = H[5];
                z[0] = h00 * b0 + h01 * b1 + h02 * b2;
                z[1] = h01 * b0 + h11 * b1 + h12 * b2;
                z[2] = h02 * b0 + h12 * b1 + h22 * b2;
            } else {
                // the point block is loaded by every lane of the point at the
                // start (its last lane applies it), next to the camera gather
                const VT* H = (const VT*)g.hpp_inv + kHinvStride * j;
                const T h00 = H[0], h01 = H[1], h02 = H[2], h11 = H[3], h12 = H[4], h22 = H[5];
                if constexpr (sizeof(VT) == 8) {
                    gather9(vin, i, pc);   // 5 aligned 16-byte loads instead of 9 scalar ones
                } else {
#pragma unroll
                    for (int k = 0; k < 9; ++k) pc[k] = (T)vin[9 * i + k];
                }
                T a0 = 0, a1 = 0;
#pragma unroll
                for (int k = 0; k < 9; ++k) {
                    a0 += jc[0][k] * pc[k];
                    a1 += jc[1][k] * pc[k];
                }
                T tt[3];
                const SegScan seg(st);
#pragma unroll
                for (int k = 0; k < 3; ++k) tt[k] = seg.sum(valid ? jp[0][k] * a0 + jp[1][k] * a1 : (T)0);
                // the point's last lane (which holds the sums) applies the point block
                T zz[3] = {0, 0, 0};
                if (valid && end == l) {
                    T v0 = tt[0], v1 = tt[1], v2 = tt[2];
                    if (kMode == kBacksub) {
                        v0 += bp[j];
                        v1 += bp[g.np + j];
                        v2 += bp[2 * g.np + j];
                    }
                    zz[0] = h00 * v0 + h01 * v1 + h02 * v2;
                    zz[1] = h01 * v0 + h11 * v1 + h12 * v2;
                    zz[2] = h02 * v0 + h12 * v1 + h22 * v2;
                    if (kMode == kMatvec && cpass) {
                        zbuf[4 * j] = zz[0];
                        zbuf[4 * j + 1] = zz[1];
                        zbuf[4 * j + 2] = zz[2];
                    }
                    if (kMode == kBacksub) {
                        zz[0] = -zz[0];
                        zz[1] = -zz[1];
                        zz[2] = -zz[2];
                        const double d0 = zz[0], d1 = zz[1], d2 = zz[2];
                        g.dpt[3 * j] = d0;
                        g.dpt[3 * j + 1] = d1;
                        g.dpt[3 * j + 2] = d2;
                        g.pt_c[3 * j] = g.pt[3 * j] + d0;
                        g.pt_c[3 * j + 1] = g.pt[3 * j + 1] + d1;
                        g.pt_c[3 * j + 2] = g.pt[3 * j + 2] + d2;
                        red_b += (double)bp[j] * d0 + (double)bp[g.np + j] * d1 +
                                 (double)bp[2 * g.np + j] * d2;
                        red_s += d0 * d0 + d1 * d1 + d2 * d2;
                    }
                }
                if (kMode == kMatvec && cpass) continue;   // uniform: the whole wave
#pragma unroll
                for (int k = 0; k < 3; ++k) z[k] = shfl64(zz[k], end);
            }
            if (kMode == kBacksub) {
                if (valid) {
                    T y0 = jp[0][0] * z[0] + jp[0][1] * z[1] + jp[0][2] * z[2];
                    T y1 = jp[1][0] * z[0] + jp[1][1] * z[1] + jp[1][2] * z[2];
#pragma unroll
                    for (int k = 0; k < 9; ++k) {
                        y0 += jc[0][k] * pc[k];
                        y1 += jc[1][k] * pc[k];
                    }
                    red_m += (double)y0 * (double)y0 + (double)y1 * (double)y1;
                }
            } else if (valid) {
                const T u0 = jp[0][0] * z[0] + jp[0][1] * z[1] + jp[0][2] * z[2];
                const T u1 = jp[1][0] * z[0] + jp[1][1] * z[1] + jp[1][2] * z[2];
#pragma unroll
                for (int k = 0; k < 9; ++k)
                    atomicAdd(&acc_lds[9 * (i - c0) + k], (AT)(jc[0][k] * u0 + jc[1][k] * u1));
            }
        } else {
            // a single point with more than 64 edges: two sweeps over chunks
            const int j = g.e_pt[e0];
            T z[3];
            if (kMode == kRhs) {
                const T b0 = (T)bp[j], b1 = (T)bp[g.np + j], b2 = (T)bp[2 * g.np + j];
                const VT* H = (const VT*)g.hpp_inv + kHinvStride * j;
                z[0] = H[0] * b0 + H[1] * b1 + H[2] * b2;
                z[1] = H[1] * b0 + H[3] * b1 + H[4] * b2;
                z[2] = H[2] * b0 + H[4] * b1 + H[5] * b2;
            } else {
                T tt[3] = {0, 0, 0};
                for (int ch = 0; ch < n; ch += kWave) {
                    if (ch + l < n) {
                        const int e = e0 + ch + l;
                        const int i = g.e_cam[e];
                        T jc[2][9], jp[2][3];
                        jac_load<JS>(J, e, jc, jp);
                        T a0 = 0, a1 = 0;
#pragma unroll
                        for (int k = 0; k < 9; ++k) {
                            const T pk = (T)vin[9 * i + k];
                            a0 += jc[0][k] * pk;
                            a1 += jc[1][k] * pk;
                        }
#pragma unroll
                        for (int k = 0; k < 3; ++k) tt[k] += jp[0][k] * a0 + jp[1][k] * a1;
                    }
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) tt[k] = wave_sum(tt[k]);
                if (kMode == kBacksub) {
                    tt[0] += bp[j];
                    tt[1] += bp[g.np + j];
                    tt[2] += bp[2 * g.np + j];
                }
                const VT* H = (const VT*)g.hpp_inv + kHinvStride * j;
                z[0] = H[0] * tt[0] + H[1] * tt[1] + H[2] * tt[2];
                z[1] = H[1] * tt[0] + H[3] * tt[1] + H[4] * tt[2];
                z[2] = H[2] * tt[0] + H[4] * tt[1] + H[5] * tt[2];
                if (kMode == kMatvec && cpass) {
                    if (l == 0) {
                        zbuf[4 * j] = z[0];
                        zbuf[4 * j + 1] = z[1];
                        zbuf[4 * j + 2] = z[2];
                    }
                    continue;   // uniform: the whole wave
                }
                if (kMode == kBacksub) {
                    z[0] = -z[0];
                    z[1] = -z[1];
                    z[2] = -z[2];
                    if (l == 0) {
                        const double d0 = z[0], d1 = z[1], d2 = z[2];
                        g.dpt[3 * j] = d0;
                        g.dpt[3 * j + 1] = d1;
                        g.dpt[3 * j + 2] = d2;
                        g.pt_c[3 * j] = g.pt[3 * j] + d0;
                        g.pt_c[3 * j + 1] = g.pt[3 * j + 1] + d1;
                        g.pt_c[3 * j + 2] = g.pt[3 * j + 2] + d2;
                        red_b += (double)bp[j] * d0 + (double)bp[g.np + j] * d1 +
                                 (double)bp[2 * g.np + j] * d2;
                        red_s += d0 * d0 + d1 * d1 + d2 * d2;
                    }
                }
            }
            for (int ch = 0; ch < n; ch += kWave) {
                if (ch + l < n) {
                    const int e = e0 + ch + l;
                    const int i = g.e_cam[e];
                    T jc[2][9], jp[2][3];
                    jac_load<JS>(J, e, jc, jp);
                    T u0 = 0, u1 = 0;
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        u0 += jp[0][k] * z[k];
                        u1 += jp[1][k] * z[k];
                    }
                    if (kMode == kBacksub) {
#pragma unroll
                        for (int k = 0; k < 9; ++k) {
                            const T pk = (T)vin[9 * i + k];
                            u0 += jc[0][k] * pk;
                            u1 += jc[1][k] * pk;
                        }
                        red_m += (double)u0 * (double)u0 + (double)u1 * (double)u1;
                    } else {
#pragma unroll
                        for (int k = 0; k < 9; ++k)
                            atomicAdd(&acc_lds[9 * (i - c0) + k], (AT)(jc[0][k] * u0 + jc[1][k] * u1));
                    }
                }
            }
        }
    }
    if (kMode == kBacksub) {
        red_m = block_sum(red_m, red);
        red_b = block_sum(red_b, red);
        red_s = block_sum(red_s, red);
        if (threadIdx.x == 0) {
            g.red_partial[4 * bid + 0] = red_m;
            g.red_partial[4 * bid + 1] = red_b;
            g.red_partial[4 * bid + 2] = red_s;
            g.red_partial[4 * bid + 3] = 0.0;
        }
        return;
    }
    if (cpass) return;
    __syncthreads();
    // the flushed partial vector in the storage type of the PCG vectors: the
    // LDS sums are FP64, each partial is rounded once (FP32 in the mixed
    // modes halves the flush and the reduction's reads)
    VT* dst = (VT*)out + g.pp_part_off[bid];
    for (int k = threadIdx.x; k < nc9; k += blockDim.x) dst[k] = (VT)acc_lds[k];
}

template <typename VT, typename JS, typename AT, int kMode>
__global__ __launch_bounds__(kPointPassBlock) void k_point_pass(DeviceGraph g, const void* __restrict__ J,
                                                     const VT* __restrict__ vin, AT* __restrict__ out) {
    pp_body<VT, JS, AT, kMode>(g, (int)blockIdx.x, J, vin, out);
}

// ==========================================================================
// Full-Hessian PCG (the solver form without point elimination, Sec. IV-D):
// the product H_lambda v over cameras and points together.  Per edge
// u = J_c v_c + J_p v_p; the camera rows J_c^T u are privatised in LDS and
// flushed per workgroup (k_reduce adds the damping), the point rows J_p^T u
// are segmented wavefront sums over the point's edges, finished by the last
// lane with the point's damping.  kMatvec multiplies z after the iteration's
// decision and forms the point parts of q = H z + beta q_old and
// p = z + beta p_old (and p^T q); kBacksub multiplies the step x and gives
// the candidate points and the model terms.  kDyn: the Jacobian is
// recomputed from the parameters in every pass (no stored copy), rounded to
// the storage type so that it equals what would have been stored.
// ==========================================================================
template <typename T, typename JS, bool kDyn>
__device__ __forceinline__ void edge_jacobian(const DeviceGraph& g, int e, int i, int j,
                                              T (&jc)[2][9], T (&jp)[2][3]) {
    if constexpr (kDyn) {
        EdgeEval<double> ev;
        bal_eval<double, true>(g.cam + 9 * i, g.pt + 3 * j, g.obs[e], g.obs[g.ne + e], ev);
        double s, rho, w;
        whiten<double, true>(ev, g.sinfo, g.ne, e, g.loss, g.delta, g.cam_fixed[i] != 0,
                             g.pt_fixed[j] != 0, s, rho, w);
#pragma unroll
        for (int a = 0; a < 2; ++a) {
#pragma unroll
            for (int k = 0; k < 9; ++k) jc[a][k] = (T)jac_round<JS>(ev.jc[a][k]);
#pragma unroll
            for (int k = 0; k < 3; ++k) jp[a][k] = (T)jac_round<JS>(ev.jp[a][k]);
        }
    } else {
        jac_load<JS>(g.jst, e, jc, jp);
    }
}

template <typename VT, typename JS, bool kDyn, int kMode>
__device__ __forceinline__ void full_pp_body(const DeviceGraph& g, const int bid) {
    if (!vec_type_ok<VT>(g) || !jac_type_ok<JS>(g)) return;   // instantiated for another mode
    using T = VT;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    double* acc_lds = (double*)smem_raw;
    __shared__ double red[16];
    __shared__ int s_act;
    __shared__ double s_beta;
    int tb, te;
    const int prob = decomp_block(g.dc_pp, bid, tb, te);
    const int l = lane_id();
    const int c0 = g.prob_cam_off[prob];
    const int nc9 = 9 * (g.prob_cam_off[prob + 1] - c0);
    // the vector multiplied: z of the PCG, or the step x
    const T* vc = (const T*)(kMode == kMatvec ? g.v_z : g.v_x);
    const T* vp = (const T*)(kMode == kMatvec ? g.w_z : g.w_x);
    if (kMode == kMatvec) {
        if (threadIdx.x < kWave) {
            const PcgState d = pcg_decision(g, prob);
            if (threadIdx.x == 0) {
                s_act = d.act;
                s_beta = d.beta;
                if (bid == g.dc_pp.prob_blk[prob]) g.pcg_dec[prob] = d;
            }
        }
        for (int k = threadIdx.x; k < nc9; k += blockDim.x) acc_lds[k] = 0;
        __syncthreads();
        if (!(s_act & kActStep)) return;   // this problem's PCG has stopped
    }
    const int act = kMode == kMatvec ? s_act : 0;
    const T beta = kMode == kMatvec ? (T)s_beta : (T)0;
    const T lambda = (T)fabs(g.lam[prob]);
    const T* Hpp = (const T*)g.hpp;
    const T* bp = (const T*)g.bp;
    const T lo = (T)g.min_diag, hi = (T)g.max_diag;
    const int nw = blockDim.x >> 6;
    double red_q = 0.0, red_m = 0.0, red_b = 0.0, red_s = 0.0;
    // the point rows of one point j (one lane of it): H_lambda v_p finished, then
    // q, p and p^T q (kMatvec), or the candidate point (kBacksub)
    auto point_rows = [&](int j, const T (&tt)[3], const T (&zp)[3]) {
        if (kMode == kMatvec) {
            T q[3], p[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T d = fmin(fmax(Hpp[sym3(c, c) * g.np + j], lo), hi);
                const T hz = tt[c] + lambda * d * zp[c];
                q[c] = (act & kActRun) ? fma(beta, ((const T*)g.w_q)[3 * j + c], hz) : hz;
                p[c] = dir_entry<T>(zp[c], ((const T*)g.w_p)[3 * j + c], act, beta);
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                ((T*)g.w_q)[3 * j + c] = q[c];
                ((T*)g.w_p)[3 * j + c] = p[c];
                red_q += (double)p[c] * (double)q[c];
            }
        } else {
            const double d0 = zp[0], d1 = zp[1], d2 = zp[2];
            g.dpt[3 * j] = d0;
            g.dpt[3 * j + 1] = d1;
            g.dpt[3 * j + 2] = d2;
            g.pt_c[3 * j] = g.pt[3 * j] + d0;
            g.pt_c[3 * j + 1] = g.pt[3 * j + 1] + d1;
            g.pt_c[3 * j + 2] = g.pt[3 * j + 2] + d2;
            red_b += (double)bp[j] * d0 + (double)bp[g.np + j] * d1 + (double)bp[2 * g.np + j] * d2;
            red_s += d0 * d0 + d1 * d1 + d2 * d2;
        }
    };
    for (int t = tb + (int)(threadIdx.x >> 6); t < te; t += nw) {
        const int e0 = g.tile_off[t], e1 = g.tile_off[t + 1];
        const int n = e1 - e0;
        if (n <= kWave) {
            const bool valid = l < n;
            const int e = e0 + (valid ? l : 0);
            const int j = g.e_pt[e];
            const int i = g.e_cam[e];
            const int jprev = __shfl_up(j, 1);
            const bool st = !valid || l == 0 || jprev != j;
            const uint64_t starts = __ballot(st);
            int head, end;
            segment_of(starts, l, head, end);
            T jc[2][9], jp[2][3];
            edge_jacobian<T, JS, kDyn>(g, e, i, j, jc, jp);
            T zp[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) zp[k] = vp[3 * j + k];
            T u0 = 0, u1 = 0;
#pragma unroll
            for (int k = 0; k < 9; ++k) {
                const T pk = vc[9 * i + k];
                u0 += jc[0][k] * pk;
                u1 += jc[1][k] * pk;
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                u0 += jp[0][k] * zp[k];
                u1 += jp[1][k] * zp[k];
            }
            if (kMode == kBacksub) {
                if (valid) red_m += (double)u0 * (double)u0 + (double)u1 * (double)u1;
                if (valid && head == l) {
                    const T none[3] = {0, 0, 0};
                    point_rows(j, none, zp);
                }
                continue;
            }
            T tt[3];
            const SegScan seg(st);
#pragma unroll
            for (int k = 0; k < 3; ++k) tt[k] = seg.sum(valid ? jp[0][k] * u0 + jp[1][k] * u1 : (T)0);
            if (valid && end == l) point_rows(j, tt, zp);   // the last lane holds the sums
            if (valid) {
#pragma unroll
                for (int k = 0; k < 9; ++k)
                    atomicAdd(&acc_lds[9 * (i - c0) + k], (double)(jc[0][k] * u0 + jc[1][k] * u1));
            }
        } else {
            // one point with more than 64 edges: chunks of a wavefront
            const int j = g.e_pt[e0];
            T zp[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) zp[k] = vp[3 * j + k];
            T tt[3] = {0, 0, 0};
            for (int ch = 0; ch < n; ch += kWave) {
                if (ch + l < n) {
                    const int e = e0 + ch + l;
                    const int i = g.e_cam[e];
                    T jc[2][9], jp[2][3];
                    edge_jacobian<T, JS, kDyn>(g, e, i, j, jc, jp);
                    T u0 = 0, u1 = 0;
#pragma unroll
                    for (int k = 0; k < 9; ++k) {
                        const T pk = vc[9 * i + k];
                        u0 += jc[0][k] * pk;
                        u1 += jc[1][k] * pk;
                    }
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        u0 += jp[0][k] * zp[k];
                        u1 += jp[1][k] * zp[k];
                    }
                    if (kMode == kBacksub) {
                        red_m += (double)u0 * (double)u0 + (double)u1 * (double)u1;
                    } else {
#pragma unroll
                        for (int k = 0; k < 3; ++k) tt[k] += jp[0][k] * u0 + jp[1][k] * u1;
#pragma unroll
                        for (int k = 0; k < 9; ++k)
                            atomicAdd(&acc_lds[9 * (i - c0) + k], (double)(jc[0][k] * u0 + jc[1][k] * u1));
                    }
                }
            }
            if (kMode == kMatvec) {
#pragma unroll
                for (int k = 0; k < 3; ++k) tt[k] = wave_sum(tt[k]);
            }
            if (l == 0) point_rows(j, tt, zp);
        }
    }
    if (kMode == kBacksub) {
        red_m = block_sum(red_m, red);
        red_b = block_sum(red_b, red);
        red_s = block_sum(red_s, red);
        if (threadIdx.x == 0) {
            g.red_partial[4 * bid + 0] = red_m;
            g.red_partial[4 * bid + 1] = red_b;
            g.red_partial[4 * bid + 2] = red_s;
            g.red_partial[4 * bid + 3] = 0.0;
        }
        return;
    }
    red_q = block_sum(red_q, red);
    if (threadIdx.x == 0) g.ppq_partial[bid] = red_q;
    // block_sum ends with a barrier: the LDS camera rows are complete
    VT* dst = (VT*)g.cam_partial + g.pp_part_off[bid];
    for (int k = threadIdx.x; k < nc9; k += blockDim.x) dst[k] = (VT)acc_lds[k];
}

template <typename VT, typename JS, bool kDyn, int kMode>
__global__ __launch_bounds__(kPointPassBlock) void k_full_point_pass(DeviceGraph g) {
    full_pp_body<VT, JS, kDyn, kMode>(g, (int)blockIdx.x);
}

// ==========================================================================
// Sum of the per-workgroup camera partials of each problem.
//   kRhs:    r = -bc + sum                              (reduced RHS)
//   kMatvec: S z = Hcc_lambda z - sum; the direction p = z + beta p and
//            q = S p = S z + beta q (FP64); partial dots p^T q (FP64)
// Workgroup: up to 64 components of one problem x 16 partial groups.
// ==========================================================================
template <typename T, int kSubs>
__device__ __forceinline__ void apply_body(const DeviceGraph& g, const int bid0, const int bid_end);

// Every vector-memory access of this wavefront has completed: its stores are
// in the L2 (s_waitcnt vmcnt(0); the workgroup barrier does not wait for them).
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// The fused update: each reduction workgroup of a problem arrives after its
// q, p and p^T q partial are written; the problem's last arrival acquires
// them all and runs the problem's update as kBlock / kPcgBlock camera-aligned
// update workgroups side by side (the arithmetic of the update kernel).  The
// arrival is a device-scope release by one thread after every wavefront's
// stores have reached the L2.
template <typename T, int kBlock>
__device__ __forceinline__ void fused_update(const DeviceGraph& g, const int prob) {
    __shared__ int s_last;
    wait_vmem();
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned int n = (unsigned int)(g.dc_red.prob_blk[prob + 1] - g.dc_red.prob_blk[prob]);
        const unsigned int old =
            __hip_atomic_fetch_add(g.red_count + prob, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        s_last = old == n - 1;
        if (s_last) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // every arrival's writes
            g.red_count[prob] = 0;                               // ready for the next iteration
        }
    }
    __syncthreads();
    if (!s_last) return;
    constexpr int kSubs = kBlock / kPcgBlock;
    const int b1 = g.dc_cam.prob_blk[prob + 1];
    for (int b = g.dc_cam.prob_blk[prob]; b < b1; b += kSubs) {
        apply_body<T, kSubs>(g, b, b1);
        __syncthreads();
    }
}

template <typename T, int kMode, int kBlock>
__device__ __forceinline__ void reduce_body(const DeviceGraph& g, const int bid, double min_diag,
                                            double max_diag) {
    if (!vec_type_ok<T>(g)) return;   // instantiated for another mode
    // The partial vectors are read with one 16-byte load per lane: a row of
    // kRedComps components is kCols lanes, and kGroups rows are summed at once
    // (each partial vector starts on a 16-byte boundary, padded to 4 entries).
    constexpr int kCpl = 16 / (int)sizeof(T);
    constexpr int kCols = kRedComps / kCpl;
    constexpr int kGroups = kBlock / kCols;
    __shared__ T red[kGroups][kRedComps];
    __shared__ double dred[16];
    int kb, ke;
    const int prob = decomp_block(g.dc_red, bid, kb, ke);
    // the decision is read here but tested after every load of the
    // workgroup has been issued (the test would otherwise hold them behind
    // its load); a stopped problem's workgroup only wastes those reads.  A
    // problem whose PCG stopped at this iteration's decision still passes
    // the fused update (which stores the state).
    int act = 0;
    T beta = 0;
    if (kMode == kMatvec) {
        const PcgState* dp = g.pcg_dec + prob;
        act = dp->act;
        beta = (T)dp->beta;
    }
    const bool fuse = kMode == kMatvec && g.fuse_apply;
    const int tid = threadIdx.x;
    const int k = kb + tid;                               // component (threads < kRedComps)
    const bool own = tid < kRedComps && k < ke;
    // the damped diagonal block row, z, p and q (or bc) of this component are
    // loaded before the partial sums, so their latency overlaps
    const int i = k / 9, r = k % 9;
    // arithmetic in the vector type (FP32 in the mixed modes); the dot
    // partials p^T q in FP64
    T h[9], pv[9], lambda = 0, bk = 0, qold = 0;
    T pold = 0;
    if (own) {
        if (kMode == kRhs) {
            bk = ((const T*)g.bc)[k];
        } else {
            lambda = (T)fabs(g.lam[prob]);   // negative: problem idle this trial
            const T* Hcc = (const T*)g.hcc;
            const T* z = (const T*)g.v_z;
#pragma unroll
            for (int c = 0; c < 9; ++c) {
                h[c] = Hcc[i * 45 + sym9(r, c)];
                pv[c] = z[9 * i + c];
            }
            pold = ((const T*)g.v_p)[k];
            qold = ((const T*)g.v_q)[k];
        }
    }
    T tot = 0;
    if (g.cam_pass && kMode == kMatvec && g.bo_chunks > 0) {
        // camera-blocked product pass: the chunk sums of the camera's block
        if (own) {
            // eight independent sums keep eight loads in flight per lane
            const int b = i / kCamBlock, il = i - b * kCamBlock;
            const T* part = (const T*)g.bo_partial + 9 * il + r;
            const int c1 = g.bo_blk_chunk[b + 1];
            int c = g.bo_blk_chunk[b];
            T t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (; c + 8 <= c1; c += 8) {
#pragma unroll
                for (int u = 0; u < 8; ++u) t[u] += part[(size_t)(c + u) * (kCamBlock * 9)];
            }
            for (int u = 0; c < c1; ++c, ++u) t[u] += part[(size_t)c * (kCamBlock * 9)];
            tot = ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
        }
    } else if (g.cam_pass) {
        // two-pass scheme: the camera's chunk sums from k_cam_pass
        if (own)
            for (int c = g.cam_chunk_off[i]; c < g.cam_chunk_off[i + 1]; ++c)
                tot += (T)g.chunk_partial[54 * c + r];
    } else {
        const int col = tid % kCols, grp = tid / kCols;
        const int c0 = kCpl * col;                        // first component of this lane
        const int kl = kb - 9 * g.prob_cam_off[prob] + c0;   // within the problem
        const int q0 = g.dc_pp.prob_blk[prob], q1 = g.dc_pp.prob_blk[prob + 1];
        // a problem's partial vectors are consecutive, each padded to a
        // multiple of 4 entries (the point-pass decomposition's layout), so
        // their addresses need no per-vector offset load; four loads per
        // lane are in flight at once
        const size_t stride = (size_t)(9 * (g.prob_cam_off[prob + 1] - g.prob_cam_off[prob]) + 3) / 4 * 4;
        const T* base = (const T*)g.cam_partial + g.pp_part_off[q0] + kl;   // vector type
        const int nq = q1 - q0;
        T a[4][kCpl];
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int u = 0; u < kCpl; ++u) a[v][u] = 0;
        if (kb + c0 < ke) {
            for (int q = grp; q < nq; q += 4 * kGroups) {
                Chunk16 x[4];
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (q + v * kGroups < nq) x[v].u = *(const uint4*)(base + (size_t)(q + v * kGroups) * stride);
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (q + v * kGroups < nq)
#pragma unroll
                        for (int u = 0; u < kCpl; ++u) a[v][u] += chunk_get<T, T>(x[v], u);
            }
        }
        if (kMode == kMatvec && !(act & kActStep)) {   // this problem's PCG has stopped
            if (fuse && (act & kActState)) fused_update<T, kBlock>(g, prob);
            return;
        }
#pragma unroll
        for (int u = 0; u < kCpl; ++u) red[grp][c0 + u] = (a[0][u] + a[1][u]) + (a[2][u] + a[3][u]);
        __syncthreads();
        // the kGroups rows in two stages over the whole workgroup: kParts
        // partial rows of kGroups / kParts, then their sum by the owners
        constexpr int kParts = kBlock / kRedComps;
        static_assert(kGroups % kParts == 0 && kParts <= kGroups, "row split of the partial sums");
        constexpr int kRows = kGroups / kParts;
        {
            const int c = tid % kRedComps, part = tid / kRedComps;
            T t = 0;
#pragma unroll
            for (int q = 0; q < kRows; ++q) t += red[part * kRows + q][c];
            __syncthreads();
            red[part][c] = t;
        }
        __syncthreads();
        if (own) {
            T t0 = 0, t1 = 0;
#pragma unroll
            for (int q = 0; q < kParts; q += 2) {
                t0 += red[q][tid];
                t1 += red[q + 1][tid];
            }
            tot = t0 + t1;
        }
    }
    if (kMode == kMatvec && !(act & kActStep)) {   // (the two-pass scheme's test)
        if (fuse && (act & kActState)) fused_update<T, kBlock>(g, prob);
        return;
    }
    double dot = 0.0;
    if (own) {
        if (kMode == kRhs) {
            ((T*)g.v_r)[k] = (T)(-bk + tot);
        } else {
            T hp = 0, hd = 0;
#pragma unroll
            for (int c = 0; c < 9; ++c) {
                T hc = h[c];
                const T dmp = c == r ? lambda * fmin(fmax(hc, (T)min_diag), (T)max_diag) : (T)0;
                hd += dmp * pv[c];
                hp += (hc + dmp) * pv[c];
            }
            // S z (Schur form: Hcc_lambda z minus the point elimination), or
            // the full system's camera rows (the edge sums already hold
            // J_c^T J z, so only the damping is added); then
            // q = S p = S z + beta q_old and p = z + beta p_old
            const T sz = g.full ? tot + hd : hp - tot;
            const T q = (act & kActRun) ? fma(beta, qold, sz) : sz;
            T zk = pv[0];
#pragma unroll
            for (int c = 1; c < 9; ++c) zk = c == r ? pv[c] : zk;
            const T pk = dir_entry<T>(zk, pold, act, beta);
            ((T*)g.v_q)[k] = q;
            ((T*)g.v_p)[k] = pk;
            dot = (double)pk * (double)q;
        }
    }
    if (kMode == kMatvec) {
        dot = block_sum(dot, dred);
        if (threadIdx.x == 0) g.pq_partial[bid] = dot;
        if (fuse) fused_update<T, kBlock>(g, prob);
    }
}

template <typename T, int kMode>
__global__ __launch_bounds__(1024) void k_reduce(DeviceGraph g, double min_diag, double max_diag) {
    reduce_body<T, kMode, 1024>(g, (int)blockIdx.x, min_diag, max_diag);
}

// ==========================================================================
// PCG on the reduced camera system of every problem, dots in FP64, scalar
// state per problem in PcgState.  The vector kernels use camera-aligned
// workgroups inside one problem (coalesced accesses; the 9x9 preconditioner
// block is applied from LDS); the scalar kernels are single-workgroup, one
// wavefront per problem at a time.
// ==========================================================================

// z = M^{-1} r for this workgroup's cameras; r_lds holds r of those cameras.
template <typename T>
__device__ __forceinline__ T minv_row(const T* __restrict__ Minv, const T* r_lds, int i, int a,
                                      int base) {
    T s = 0;
#pragma unroll
    for (int b = 0; b < 9; ++b) s += Minv[i * 45 + sym9(a, b)] * r_lds[base + b];
    return s;
}

// PCG start, vectors: x = 0 and the best iterate of the rejection ratio
// x_best = x = 0 (the start is the first candidate), z = M^{-1} r, partial
// (r^T z, r^T r) per workgroup.
template <typename T>
__global__ __launch_bounds__(kPcgBlock) void k_pcg_start(DeviceGraph g) {
    if (!vec_type_ok<T>(g)) return;   // instantiated for another mode
    __shared__ T r_lds[kPcgBlock];
    __shared__ double red[16];
    int cb, ce;
    decomp_block(g.dc_cam, blockIdx.x, cb, ce);
    const int tid = threadIdx.x;
    const int k = 9 * cb + tid;
    const bool valid = tid < 9 * (ce - cb);
    const T* __restrict__ r = (const T*)g.v_r;
    // the reduced right-hand side, or the full system's -b_c
    T rv = valid ? (g.full ? -((const T*)g.bc)[k] : r[k]) : (T)0;
    if (valid && g.full) ((T*)g.v_r)[k] = rv;
    r_lds[tid] = rv;
    __syncthreads();
    double rz = 0.0, rr = 0.0;
    if (valid) {
        const int i = k / 9, a = k % 9;
        const T zv = minv_row((const T*)g.minv, r_lds, i, a, tid - a);
        ((T*)g.v_z)[k] = zv;
        ((T*)g.v_x)[k] = 0;
        ((T*)g.v_best)[k] = 0;
        rz = (double)rv * (double)zv;
        rr = (double)rv * (double)rv;
    }
    rz = block_sum(rz, red);
    rr = block_sum(rr, red);
    if (tid == 0) {
        g.dot_partial[2 * blockIdx.x] = rz;
        g.dot_partial[2 * blockIdx.x + 1] = rr;
    }
}

// PCG start, scalars: rz0, rr0, threshold per problem (the first direction
// p = z is formed by the first iteration).
__global__ __launch_bounds__(1024) void k_pcg_start_finish(DeviceGraph g, double tol, int relative) {
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    for (int prob = w; prob < g.n_probs; prob += nw) {
        const int q0 = g.dc_cam.prob_blk[prob], q1 = g.dc_cam.prob_blk[prob + 1];
        double rz = wave_sum_blocks(g.dot_partial, 2, 0, q0, q1);
        double rr = wave_sum_blocks(g.dot_partial, 2, 1, q0, q1);
        if (g.full) {
            const int p0 = g.dc_pts.prob_blk[prob], p1 = g.dc_pts.prob_blk[prob + 1];
            rz += wave_sum_blocks(g.pdot_partial, 2, 0, p0, p1);
            rr += wave_sum_blocks(g.pdot_partial, 2, 1, p0, p1);
        }
        if (lane_id() == 0) {
            PcgState st;
            st.rz = rz;
            st.rr = rr;
            st.rr0 = rr;
            st.min_rr = rr;
            st.thresh = relative ? tol * tol * rr : tol * tol;
            st.iters = 0;
            st.use_best = 0;
            st.act = 0;
            st.beta = 0.0;
            st.fresh = 1;
            st.pad_ = 0;
            st.done = g.lam[prob] < 0.0 ? 5 : ((rr <= st.thresh || !(rz > 0.0)) ? 1 : 0);
            g.pcg[prob] = st;
            if (g.red_count) g.red_count[prob] = 0;
            // a problem without point-pass workgroups never takes a decision:
            // its slot says stopped (such a problem has r = 0 and stops here)
            g.pcg_dec[prob] = st;
            if (g.pcg_host) g.pcg_host[prob] = st;
        }
    }
}

// PCG step, vectors (camera-aligned workgroups), as decided at the start of
// the iteration (g.pcg_dec): alpha = r^T z / p^T q; x += alpha p; r -= alpha q;
// z = M^{-1} r; partial (r^T z, r^T r) per workgroup for the next decision;
// the best-iterate copy / restore of the rejection ratio.  The problem's first
// workgroup stores the state (the decision, or a breakdown when p^T q <= 0),
// and its host mirror once the PCG stops; no other workgroup reads the state.
// kSubs > 1: a workgroup of kSubs x kPcgBlock threads runs camera workgroups
// bid0 .. bid0 + kSubs - 1 side by side (the persistent kernel), each with
// the arithmetic of a launched one; every thread then passes every barrier.
template <typename T, int kSubs>
__device__ __forceinline__ void apply_body(const DeviceGraph& g, const int bid0, const int bid_end) {
    if (!vec_type_ok<T>(g)) return;   // instantiated for another mode
    __shared__ T r_lds[kSubs * kPcgBlock];
    __shared__ double red[16];
    const int sub = kSubs > 1 ? (int)threadIdx.x / kPcgBlock : 0;
    const int tid = (int)threadIdx.x - sub * kPcgBlock;
    const int bid = bid0 + sub;
    int cb = 0, ce = 0, prob = 0;
    const bool blk = kSubs == 1 || bid < bid_end;
    if (blk) prob = decomp_block(g.dc_cam, bid, cb, ce);
    const int k = 9 * cb + tid;
    const bool valid = tid < 9 * (ce - cb);
    // T PCG stopped before this iteration (the rest of a replayed chunk of
    // iterations) exits after one load.  Otherwise every load of the step is
    // issued before the next wait (the dot, alpha).
    // the decision is read with the rest and tested once every load is
    // issued (a stopped problem's workgroup only wastes those reads)
    const PcgState* dp = g.pcg_dec + prob;
    const int act = blk ? dp->act : 0;
    const double rz_dec = blk ? dp->rz : 0.0;
    // the lead thread loads the decision it stores as the state now, so that
    // the store at the end waits for nothing
    const bool lead0 = blk && tid == 0 && bid == g.dc_cam.prob_blk[prob];
    constexpr int kWords = (int)(sizeof(PcgState) / 8);   // copied as 8-byte words
    static_assert(sizeof(PcgState) % 8 == 0, "PcgState is a whole number of 8-byte words");
    uint2 dq[kWords];
    if (lead0) {
#pragma unroll
        for (int u = 0; u < kWords; ++u) dq[u] = ((const uint2*)dp)[u];
    }
    T* __restrict__ x = (T*)g.v_x;
    T* __restrict__ r = (T*)g.v_r;
    double pq = 0.0;
    if (blk) {
        for (int b = g.dc_red.prob_blk[prob] + tid; b < g.dc_red.prob_blk[prob + 1]; b += kPcgBlock)
            pq += g.pq_partial[b];
        if (g.full)   // the point part of p^T q, from the product's workgroups
            for (int b = g.dc_pp.prob_blk[prob] + tid; b < g.dc_pp.prob_blk[prob + 1]; b += kPcgBlock)
                pq += g.ppq_partial[b];
    }
    // vector arithmetic in the vector type; dots (and alpha) in FP64
    T xk = 0, pk = 0, qk = 0, rk = 0;
    T m[9];
    const int i = k / 9, a = k % 9;
    if (valid) {
        xk = x[k];
        pk = ((const T*)g.v_p)[k];
        qk = ((const T*)g.v_q)[k];
        rk = r[k];
        const T* __restrict__ Minv = (const T*)g.minv;
#pragma unroll
        for (int b = 0; b < 9; ++b) m[b] = Minv[i * 45 + sym9(a, b)];
    }
    const bool live = (act & kActState) != 0;
    if (kSubs == 1 && !live) return;
    const bool lead = lead0 && live;
    // every workgroup of the problem sums the same partials in the same
    // order, so all of them take the same branch
    pq = sub_sum<kPcgBlock>(pq, red);
    if (live && (act & (kActKeepBest | kActRestore))) {   // rejection ratio
        T* __restrict__ best = (T*)g.v_best;
        if (valid && (act & kActKeepBest)) best[k] = (T)xk;
        if (valid && (act & kActRestore)) x[k] = best[k];
    }
    const bool ok = pq > 0.0 && isfinite(pq);
    const bool step = live && (act & kActStep) && ok;
    if (kSubs > 1 || step) {
        const T alpha = step ? (T)(rz_dec / pq) : (T)0;
        T rv = 0;
        if (step && valid) {
            x[k] = (T)fma(alpha, pk, xk);
            rv = (T)fma(-alpha, qk, rk);
            r[k] = rv;
        }
        r_lds[sub * kPcgBlock + tid] = rv;
        __syncthreads();
        double rz = 0.0, rr = 0.0;
        if (step && valid) {
            const int base = sub * kPcgBlock + tid - a;
            T sz = 0;
#pragma unroll
            for (int b = 0; b < 9; ++b) sz += (T)m[b] * (T)r_lds[base + b];
            const T zv = (T)sz;
            ((T*)g.v_z)[k] = zv;
            rz = (double)rv * (double)zv;
            rr = (double)rv * (double)rv;
        }
        rz = sub_sum<kPcgBlock>(rz, red);
        rr = sub_sum<kPcgBlock>(rr, red);
        if (step && tid == 0) {
            g.dot_partial[2 * bid] = rz;
            g.dot_partial[2 * bid + 1] = rr;
        }
    }
    if (lead) {
        // the decision becomes the state (act cleared; done = 3 on a
        // breakdown, x then stays the last iterate)
        static_assert(offsetof(PcgState, done) == 44 && offsetof(PcgState, act) == 52,
                      "field offsets of the state copy");
        if ((act & kActStep) && !ok) dq[5].y = 3;   // done (bytes 44..47)
        dq[6].y = 0;                                // act (bytes 52..55)
#pragma unroll
        for (int u = 0; u < kWords; ++u) ((uint2*)(g.pcg + prob))[u] = dq[u];
        // the host mirror only when the PCG stops (the host waits for every
        // PCG to stop; a store to host memory delays the kernel's end by a
        // bus round trip)
        if (g.pcg_host && dq[5].y != 0) {
#pragma unroll
            for (int u = 0; u < kWords; ++u) ((uint2*)(g.pcg_host + prob))[u] = dq[u];
        }
    }
}

// The point part of the full system's PCG update (workgroup `bid` of the
// point decomposition), as decided for its problem: x += alpha p,
// r -= alpha q, z = Hpp_lambda^-1 r, partial (r^T z, r^T r) of the points;
// the best-iterate copy / restore of the rejection ratio.  alpha from the
// same sums, in the same order, as the camera part.  kSubs as in apply_body.
template <typename T, int kSubs>
__device__ __forceinline__ void apply_pts_body(const DeviceGraph& g, const int bid0) {
    __shared__ double red[16];
    const int sub = kSubs > 1 ? (int)threadIdx.x / kPcgBlock : 0;
    const int tid = (int)threadIdx.x - sub * kPcgBlock;
    const int bid = bid0 + sub;
    int pb = 0, pe = 0, prob = 0;
    const bool blk = kSubs == 1 || bid < g.dc_pts.nblk;
    if (blk) prob = decomp_block(g.dc_pts, bid, pb, pe);
    const PcgState* dp = g.pcg_dec + prob;
    const int act = blk ? dp->act : 0;
    const double rz_dec = blk ? dp->rz : 0.0;
    const bool live = (act & kActState) != 0;
    if (kSubs == 1 && !live) return;
    double pq = 0.0;
    if (live) {
        for (int b = g.dc_red.prob_blk[prob] + tid; b < g.dc_red.prob_blk[prob + 1]; b += kPcgBlock)
            pq += g.pq_partial[b];
        for (int b = g.dc_pp.prob_blk[prob] + tid; b < g.dc_pp.prob_blk[prob + 1]; b += kPcgBlock)
            pq += g.ppq_partial[b];
    }
    pq = sub_sum<kPcgBlock>(pq, red);
    T* __restrict__ x = (T*)g.w_x;
    T* __restrict__ r = (T*)g.w_r;
    T* __restrict__ best = (T*)g.w_best;
    if (live && (act & (kActKeepBest | kActRestore)))
        for (int k = 3 * pb + tid; k < 3 * pe; k += kPcgBlock) {
            if (act & kActKeepBest) best[k] = x[k];
            if (act & kActRestore) x[k] = best[k];
        }
    const bool ok = pq > 0.0 && isfinite(pq);
    const bool step = live && (act & kActStep) && ok;
    if (kSubs == 1 && !step) return;
    const T alpha = step ? (T)(rz_dec / pq) : (T)0;
    const T* __restrict__ p = (const T*)g.w_p;
    const T* __restrict__ q = (const T*)g.w_q;
    double rz = 0.0, rr = 0.0;
    for (int j = pb + tid; step && j < pe; j += kPcgBlock) {
        const T* H = (const T*)g.hpp_inv + kHinvStride * j;
        T rv[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            x[3 * j + c] = fma(alpha, p[3 * j + c], x[3 * j + c]);
            rv[c] = fma(-alpha, q[3 * j + c], r[3 * j + c]);
            r[3 * j + c] = rv[c];
        }
        T zv[3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
            zv[a] = H[sym3(a, 0)] * rv[0] + H[sym3(a, 1)] * rv[1] + H[sym3(a, 2)] * rv[2];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            ((T*)g.w_z)[3 * j + c] = zv[c];
            rz += (double)rv[c] * (double)zv[c];
            rr += (double)rv[c] * (double)rv[c];
        }
    }
    rz = sub_sum<kPcgBlock>(rz, red);
    rr = sub_sum<kPcgBlock>(rr, red);
    if (step && tid == 0) {
        g.pdot_partial[2 * bid] = rz;
        g.pdot_partial[2 * bid + 1] = rr;
    }
}

// PCG start, the full system's point part: r = -b_p, z = Hpp_lambda^-1 r,
// x = best = p = q = 0, partial (r^T z, r^T r) per point workgroup.
template <typename T>
__global__ __launch_bounds__(kPcgBlock) void k_pcg_start_pts(DeviceGraph g) {
    if (!vec_type_ok<T>(g)) return;   // instantiated for another mode
    __shared__ double red[16];
    int pb, pe;
    decomp_block(g.dc_pts, blockIdx.x, pb, pe);
    const T* bp = (const T*)g.bp;
    double rz = 0.0, rr = 0.0;
    for (int j = pb + (int)threadIdx.x; j < pe; j += blockDim.x) {
        const T* H = (const T*)g.hpp_inv + kHinvStride * j;
        T rv[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) rv[c] = -bp[c * g.np + j];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const T zv = H[sym3(a, 0)] * rv[0] + H[sym3(a, 1)] * rv[1] + H[sym3(a, 2)] * rv[2];
            ((T*)g.w_r)[3 * j + a] = rv[a];
            ((T*)g.w_z)[3 * j + a] = zv;
            ((T*)g.w_x)[3 * j + a] = 0;
            ((T*)g.w_best)[3 * j + a] = 0;
            ((T*)g.w_p)[3 * j + a] = 0;
            ((T*)g.w_q)[3 * j + a] = 0;
            rz += (double)rv[a] * (double)zv;
            rr += (double)rv[a] * (double)rv[a];
        }
    }
    rz = block_sum(rz, red);
    rr = block_sum(rr, red);
    if (threadIdx.x == 0) {
        g.pdot_partial[2 * blockIdx.x] = rz;
        g.pdot_partial[2 * blockIdx.x + 1] = rr;
    }
}

// The update of one PCG iteration: camera workgroups first, then (full
// system) the point workgroups.
template <typename T>
__global__ __launch_bounds__(kPcgBlock) void k_pcg_apply(DeviceGraph g) {
    const int b = (int)blockIdx.x;
    if (b < g.dc_cam.nblk)
        apply_body<T, 1>(g, b, g.dc_cam.nblk);
    else if (g.full && vec_type_ok<T>(g))
        apply_pts_body<T, 1>(g, b - g.dc_cam.nblk);
}

// ==========================================================================
// Cameras after PCG: dc = x, candidate cameras; partial b^T dc, |dc|^2 and
// |c|^2 over free cameras per camera-aligned workgroup.
// ==========================================================================
template <typename T>
__global__ __launch_bounds__(kPcgBlock) void k_cam_update(DeviceGraph g) {
    if (!vec_type_ok<T>(g)) return;   // instantiated for another mode
    __shared__ double red[16];
    int cb, ce;
    decomp_block(g.dc_cam, blockIdx.x, cb, ce);
    const T* x = (const T*)g.v_x;
    const T* bc = (const T*)g.bc;
    double bdx = 0.0, s2 = 0.0, x2 = 0.0;
    const int tid = threadIdx.x;
    if (tid < 9 * (ce - cb)) {
        const int k = 9 * cb + tid;
        const int i = k / 9;
        const bool fixed = g.cam_fixed[i] != 0;
        const double d = fixed ? 0.0 : (double)x[k];
        const double c = g.cam[k];
        g.cam_c[k] = c + d;
        bdx = (double)bc[k] * d;
        s2 = d * d;
        if (!fixed) x2 = c * c;
    }
    bdx = block_sum(bdx, red);
    s2 = block_sum(s2, red);
    x2 = block_sum(x2, red);
    if (tid == 0) {
        g.camupd_partial[3 * blockIdx.x] = bdx;
        g.camupd_partial[3 * blockIdx.x + 1] = s2;
        g.camupd_partial[3 * blockIdx.x + 2] = x2;
    }
}

// Combine the per-workgroup partial sums of the trial, per problem (single
// workgroup; with fewer problems than wavefronts several wavefronts share a
// problem's sums).
__global__ __launch_bounds__(1024) void k_finish(DeviceGraph g) {
    __shared__ double part[16][8];
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    // wavefronts per problem: with fixed-order sums one, so that a problem's
    // sums do not depend on how many problems share the batch
    const int wpp = (g.deterministic || g.n_probs >= nw) ? 1 : nw / g.n_probs;
    const int groups = nw / wpp, gw = w / wpp, sub = w % wpp;
    for (int base = 0; base < g.n_probs; base += groups) {
        const int prob = base + gw;
        const bool mine = gw < groups && prob < g.n_probs;
        double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (mine) {
            const int e0 = g.dc_edges.prob_blk[prob], e1 = g.dc_edges.prob_blk[prob + 1];
            const int p0 = g.dc_pp.prob_blk[prob], p1 = g.dc_pp.prob_blk[prob + 1];
            const int t0 = g.dc_pts.prob_blk[prob], t1 = g.dc_pts.prob_blk[prob + 1];
            const int c0 = g.dc_cam.prob_blk[prob], c1 = g.dc_cam.prob_blk[prob + 1];
            v[0] = wave_sum_blocks(g.cost_partial, 1, 0, e0, e1, sub, wpp);
            v[1] = wave_sum_blocks(g.red_partial, 4, 0, p0, p1, sub, wpp);
            v[2] = wave_sum_blocks(g.red_partial, 4, 1, p0, p1, sub, wpp);
            v[3] = wave_sum_blocks(g.red_partial, 4, 2, p0, p1, sub, wpp);
            v[4] = wave_sum_blocks(g.damp_partial, 1, 0, t0, t1, sub, wpp);
            v[5] = wave_sum_blocks(g.camupd_partial, 3, 0, c0, c1, sub, wpp);
            v[6] = wave_sum_blocks(g.camupd_partial, 3, 1, c0, c1, sub, wpp);
            v[7] = wave_sum_blocks(g.camupd_partial, 3, 2, c0, c1, sub, wpp);
        }
        if (lane_id() == 0)
            for (int k = 0; k < 8; ++k) part[w][k] = v[k];
        __syncthreads();
        if (mine && sub == 0 && lane_id() == 0) {
            double t[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            for (int s2 = 0; s2 < wpp; ++s2)
                for (int k = 0; k < 8; ++k) t[k] += part[w + s2][k];
            TrialScalars* ts = g.scal + prob;
            ts->cost = t[0];
            ts->quad = t[1];
            ts->b_dot_dx = t[5] + t[2];
            ts->step2 = t[6] + t[3];
            ts->x2 = t[7] + t[4];
            ts->pcg_iters = g.pcg[prob].iters;
            ts->pcg_reason = g.pcg[prob].done;
            ts->barrier_err = g.gbar ? (int)g.gbar[2] : 0;
            ts->pad_ = 0;
            if (g.scal_host) g.scal_host[prob] = *ts;
        }
        __syncthreads();
    }
}

// Cost only: combine the cost partials per problem (as k_finish).
__global__ __launch_bounds__(1024) void k_cost_finish(DeviceGraph g) {
    __shared__ double part[16];
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const int wpp = (g.deterministic || g.n_probs >= nw) ? 1 : nw / g.n_probs;
    const int groups = nw / wpp, gw = w / wpp, sub = w % wpp;
    for (int base = 0; base < g.n_probs; base += groups) {
        const int prob = base + gw;
        const bool mine = gw < groups && prob < g.n_probs;
        double v = 0.0;
        if (mine)
            v = wave_sum_blocks(g.cost_partial, 1, 0, g.dc_edges.prob_blk[prob],
                                g.dc_edges.prob_blk[prob + 1], sub, wpp);
        if (lane_id() == 0) part[w] = v;
        __syncthreads();
        if (mine && sub == 0 && lane_id() == 0) {
            double t = 0.0;
            for (int s2 = 0; s2 < wpp; ++s2) t += part[w + s2];
            g.scal[prob].cost = t;
            if (g.scal_host) g.scal_host[prob].cost = t;
        }
        __syncthreads();
    }
}

// Accepted problems: the candidate parameters become the current ones.
__global__ __launch_bounds__(256) void k_commit(DeviceGraph g) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < 9 * (size_t)g.nc; k += stride)
        if (g.accept[g.cam_prob[k / 9]]) g.cam[k] = g.cam_c[k];
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < 3 * (size_t)g.np; k += stride)
        if (g.accept[g.pt_prob[k / 3]]) g.pt[k] = g.pt_c[k];
}

// ==========================================================================
// Two-pass scheme (a problem's camera vector exceeds LDS), second pass:
// camera-major over the stored Jacobian's camera-major copy, one workgroup
// per chunk of one camera's runs:
//   sum_e J_c^T (J_p z_j)   with z_j from the first pass (zbuf)
// into chunk_partial[chunk][0..8]; k_reduce adds a camera's chunks.
//   kRhs: z_j = Hpp_lambda^-1 bp_j;  kMatvec: z_j = Hpp_lambda^-1 sum J_p^T J_c v
//   (v the product's camera vector).
// ==========================================================================
template <typename VT, typename JS, int kMode, int kSubs>
__device__ __forceinline__ void cam_pass_body(const DeviceGraph& g, const int chunk0) {
    if (!vec_type_ok<VT>(g) || !jac_type_ok<JS>(g)) return;   // instantiated for another mode
    // arithmetic and sums in the vector type (FP32 in the mixed modes)
    using T = VT;
    constexpr int kWaves = kCamPassBlock / kWave;
    __shared__ T red[kSubs * kWaves][9];
    // kSubs > 1: chunks chunk0 .. chunk0 + kSubs - 1 side by side in one
    // workgroup of kSubs x kCamPassBlock threads (the persistent kernel)
    const int sub = kSubs > 1 ? (int)threadIdx.x / kCamPassBlock : 0;
    const int tid = (int)threadIdx.x - sub * kCamPassBlock;
    const int chunk = chunk0 + sub;
    bool live = kSubs == 1 || chunk < g.n_chunks;
    const int cam = live ? g.chunk_cam[chunk] : 0;
    if (kMode == kMatvec && live && !(g.pcg_dec[g.cam_prob[cam]].act & kActStep)) live = false;   // stopped
    if (kSubs == 1 && !live) return;
    const int rb = live ? g.chunk_run_off[chunk] : 0, re = live ? g.chunk_run_off[chunk + 1] : 0;
    const T* __restrict__ zbuf = (const T*)g.zbuf;
    T y[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) y[k] = (T)0;
    for (int run = rb + tid; run < re; run += kCamPassBlock) {
        const int q0 = g.cm_run_off[run], q1 = g.cm_run_off[run + 1];
        const int j = g.cm_pt[q0];
        const T z0 = zbuf[4 * j], z1 = zbuf[4 * j + 1], z2 = zbuf[4 * j + 2];
        for (int q = q0; q < q1; ++q) {
            T jc[2][9], jp[2][3];
            jac_load<JS>(g.jst_cm, q, jc, jp);
            const T u0 = jp[0][0] * z0 + jp[0][1] * z1 + jp[0][2] * z2;
            const T u1 = jp[1][0] * z0 + jp[1][1] * z1 + jp[1][2] * z2;
#pragma unroll
            for (int k = 0; k < 9; ++k) y[k] += jc[0][k] * u0 + jc[1][k] * u1;
        }
    }
    const int w = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const T v = wave_sum(y[k]);
        if (lane_id() == 0) red[w][k] = v;
    }
    __syncthreads();
    if (live && tid < 9) {
        T s = 0;
        for (int q = 0; q < kWaves; ++q) s += red[sub * kWaves + q][tid];
        g.chunk_partial[54 * chunk + tid] = (double)s;
    }
}

template <typename VT, typename JS, int kMode>
__global__ __launch_bounds__(kCamPassBlock) void k_cam_pass(DeviceGraph g) {
    cam_pass_body<VT, JS, kMode, 1>(g, (int)blockIdx.x);
}

// Two-pass scheme, RHS first pass: z_j = Hpp_lambda^-1 bp_j for every point.
template <typename T>
__global__ __launch_bounds__(256) void k_rhs_z(DeviceGraph g) {
    if (!vec_type_ok<T>(g)) return;   // instantiated for another mode
    using PT = T;
    const T* bp = (const T*)g.bp;
    PT* zbuf = (PT*)g.zbuf;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < g.np; j += gridDim.x * blockDim.x) {
        const PT b0 = bp[j], b1 = bp[g.np + j], b2 = bp[2 * g.np + j];
        const T* H = (const T*)g.hpp_inv + kHinvStride * j;
        zbuf[4 * j] = H[0] * b0 + H[1] * b1 + H[2] * b2;
        zbuf[4 * j + 1] = H[1] * b0 + H[3] * b1 + H[4] * b2;
        zbuf[4 * j + 2] = H[2] * b0 + H[4] * b1 + H[5] * b2;
    }
}

// ==========================================================================
// Camera-blocked camera pass of the Schur product (two-pass form, one
// problem): the camera pass with its edges grouped by block of kCamBlock
// cameras and in point order inside a block, so a workgroup reads z_j of
// nearby points in ascending order instead of one random point per edge.
// One workgroup per chunk (within one block) sums J_c^T J_p z_j per camera of
// the block in LDS (FP64) and writes the block's partial vector (vector type);
// k_reduce adds the block's chunks.  The Jacobian is a copy in block order
// (k_copy_jac_bo, after each linearisation).
// ==========================================================================
template <typename JS>
__global__ __launch_bounds__(256) void k_copy_jac_bo(DeviceGraph g) {
    if (!jac_type_ok<JS>(g)) return;   // instantiated for another mode
    using A = typename std::conditional<std::is_same<JS, double>::value, double, float>::type;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < g.ne;
         e += (long long)gridDim.x * blockDim.x) {
        A jc[2][9], jp[2][3];
        jac_load<JS>(g.jst, g.bo_perm[e], jc, jp);
        jac_save<JS>(g.jst_bo, (int)e, jc, jp);
    }
}

template <typename VT, typename JS>
__global__ __launch_bounds__(kCamBlockThreads) void k_cam_block_pass(DeviceGraph g) {
    if (!vec_type_ok<VT>(g) || !jac_type_ok<JS>(g)) return;   // instantiated for another mode
    using T = VT;
    // the sums in LDS are FP64 in every mode (FP32 LDS atomics are slower)
    extern __shared__ __align__(16) unsigned char bo_lds[];
    double* y = (double*)bo_lds;
    if (!(g.pcg_dec[0].act & kActStep)) return;   // the PCG has stopped (uniform)
    const int ch = blockIdx.x;
    const int b = g.bo_blk[ch], cb0 = b * kCamBlock;
    const int e0 = g.bo_off[ch], e1 = g.bo_off[ch + 1];
    for (int k = threadIdx.x; k < kCamBlock * 9; k += blockDim.x) y[k] = 0.0;
    __syncthreads();
    const T* __restrict__ zbuf = (const T*)g.zbuf;
    for (int e = e0 + (int)threadIdx.x; e < e1; e += blockDim.x) {
        const int j = g.bo_pt[e], il = g.bo_cam[e] - cb0;
        const T z0 = zbuf[4 * j], z1 = zbuf[4 * j + 1], z2 = zbuf[4 * j + 2];
        T jc[2][9], jp[2][3];
        jac_load<JS>(g.jst_bo, e, jc, jp);
        const T u0 = jp[0][0] * z0 + jp[0][1] * z1 + jp[0][2] * z2;
        const T u1 = jp[1][0] * z0 + jp[1][1] * z1 + jp[1][2] * z2;
#pragma unroll
        for (int k = 0; k < 9; ++k) atomicAdd(&y[9 * il + k], (double)(jc[0][k] * u0 + jc[1][k] * u1));
    }
    __syncthreads();
    const int ncb = min(kCamBlock, g.nc - cb0) * 9;
    T* dst = (T*)g.bo_partial + (size_t)ch * (kCamBlock * 9);
    for (int k = threadIdx.x; k < ncb; k += blockDim.x) dst[k] = (T)y[k];
}

// ==========================================================================
// Persistent PCG: one cooperative launch runs every iteration of every
// problem of the batch.  An iteration is the three phases of the launched
// form (the product with its decision, the partial reduction with q and p,
// the update with the next dots; the camera-major pass of the two-pass
// scheme as a fourth), each a loop over its decomposition blocks, separated
// by grid barriers.  Each problem stops on its own decision as in the
// launched form; the loop ends when every problem has stopped, after at most
// max_iters + 1 iterations.
// ==========================================================================
constexpr unsigned int kBarrierSpin = 1u << 21;   // sleeps before a barrier gives up

// Grid barrier over the co-resident workgroups of a cooperative launch:
// bar[0] group arrivals, bar[1] generation, bar[2] error, and the arrival
// counter of workgroup group k (index modulo kGbarGroups) at
// bar[kGbarLine * (1 + k)].  One thread per workgroup takes part.  Its
// arrival at its group is a release at device scope (the workgroup's writes,
// in the L2 once every wavefront has waited for its stores, reach the point
// of coherence of the eight XCDs); a group's last arrival acquires them and arrives at the
// top (release), and the top's last arrival resets the count and opens the
// next generation (release).  The others poll the generation with relaxed
// loads, which read the coherent copy and leave the caches alone, and
// acquire once after the wait.  So each workgroup pays one L2 write-back and
// one or two invalidations per barrier (an acquiring poll would invalidate
// its XCD's L2 on every probe while other workgroups still compute), and no
// counter takes more than about nblocks / kGbarGroups atomics.  The other
// threads are ordered after the acquire by the closing workgroup barrier.  A
// wait longer than kBarrierSpin sleeps sets the error flag and returns, and
// every later barrier returns at once, so the kernel ends whatever happens
// (the host reports the flag).
__device__ __forceinline__ void grid_barrier(unsigned int* bar, unsigned int nblocks, unsigned int& gen) {
    wait_vmem();   // every wavefront's stores are in the L2 before the release
    __syncthreads();
    if (threadIdx.x == 0) {
        constexpr unsigned int G = kGbarGroups;
        const unsigned int grp = blockIdx.x % G;
        const unsigned int groups = nblocks < G ? nblocks : G;
        const unsigned int members = (nblocks - grp + G - 1) / G;
        unsigned int* cnt = bar + kGbarLine * (1 + grp);
        bool open = false;
        if (__hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) == members - 1) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // the group's writes
            __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (__hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) ==
                groups - 1) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // every group's writes
                __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                open = true;
            }
        }
        if (!open) {
            unsigned int spins = 0;
            while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                if (__hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
                __builtin_amdgcn_s_sleep(2);
                if (++spins > kBarrierSpin) {
                    __hip_atomic_fetch_or(&bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // the generation's writes
        }
    }
    ++gen;
    __syncthreads();
}

// kForm: 0 the Schur form, 1 the full system, 2 the full system with
// dynamic Jacobians
template <typename VT, typename JS, int kForm>
__global__ __launch_bounds__(kPersistentBlock) void k_pcg_persistent(DeviceGraph g, double min_diag,
                                                                    double max_diag, int max_launch) {
    // every workgroup runs the same loop (uniform trip count), so each
    // arrives at every barrier; the type check is uniform too
    if (!vec_type_ok<VT>(g) || !jac_type_ok<JS>(g)) return;
    static_assert(kPersistentBlock == kPointPassBlock, "the product runs as launched");
    constexpr int kSubsV = kPersistentBlock / kPcgBlock;        // vector workgroups side by side
    constexpr int kSubsC = kPersistentBlock / kCamPassBlock;    // camera-pass workgroups
    __shared__ int s_more;
    unsigned int gen = 0;
    const unsigned int nb = gridDim.x;
    const bool cpass = g.cam_pass != 0;
    for (int it = 0; it < max_launch; ++it) {
        for (int b = blockIdx.x; b < g.dc_pp.nblk; b += gridDim.x) {
            if constexpr (kForm == 0)
                pp_body<VT, JS, double, kMatvec>(g, b, g.jst, (const VT*)g.v_z, (double*)g.cam_partial);
            else
                full_pp_body<VT, JS, kForm == 2, kMatvec>(g, b);
            __syncthreads();   // the block's shared state is reused by the next one
        }
        if (cpass) {
            grid_barrier(g.gbar, nb, gen);
            for (int c = blockIdx.x * kSubsC; c < g.n_chunks; c += gridDim.x * kSubsC) {
                cam_pass_body<VT, JS, kMatvec, kSubsC>(g, c);
                __syncthreads();
            }
        }
        grid_barrier(g.gbar, nb, gen);
        for (int b = blockIdx.x; b < g.dc_red.nblk; b += gridDim.x) {
            reduce_body<VT, kMatvec, kPersistentBlock>(g, b, min_diag, max_diag);
            __syncthreads();
        }
        grid_barrier(g.gbar, nb, gen);
        // the camera and the point updates are independent (separate vectors
        // and partials), one after the other without a barrier
        for (int b = blockIdx.x * kSubsV; b < g.dc_cam.nblk; b += gridDim.x * kSubsV) {
            apply_body<VT, kSubsV>(g, b, g.dc_cam.nblk);
            __syncthreads();
        }
        if constexpr (kForm != 0) {
            for (int b = blockIdx.x * kSubsV; b < g.dc_pts.nblk; b += gridDim.x * kSubsV) {
                apply_pts_body<VT, kSubsV>(g, b);
                __syncthreads();
            }
        }
        grid_barrier(g.gbar, nb, gen);
        // every workgroup reads the same states after the barrier
        if (threadIdx.x == 0) {
            int more = 0;
            for (int p = 0; p < g.n_probs && !more; ++p) more = g.pcg[p].done == 0;
            if (g.gbar[2] != 0u) more = 0;
            s_more = more;
        }
        __syncthreads();
        if (!s_more) break;
    }
}

// Batch assembly: one workgroup per chunk of one descriptor.
__global__ __launch_bounds__(256) void k_pack(const PackDesc* __restrict__ desc,
                                              const PackChunk* __restrict__ chunks) {
    const PackChunk c = chunks[blockIdx.x];
    const PackDesc d = desc[c.desc];
    const long long end = d.n < (long long)c.begin + kPackChunk ? d.n : (long long)c.begin + kPackChunk;
    for (long long k = c.begin + threadIdx.x; k < end; k += blockDim.x) {
        switch (d.kind) {
            case kPackI32: ((int*)d.dst)[k] = ((const int*)d.src)[k] + d.add; break;
            case kPackF64: ((double*)d.dst)[k] = ((const double*)d.src)[k]; break;
            case kPackU8: ((unsigned char*)d.dst)[k] = ((const unsigned char*)d.src)[k]; break;
            case kPackFillI32: ((int*)d.dst)[k] = d.add; break;
            default: ((double*)d.dst)[k] = d.fval; break;
        }
    }
}

// Streaming read of n 16-byte words, four loads in flight per thread; the
// XOR of the words keeps the loads live; one word per workgroup.
__global__ __launch_bounds__(256) void k_hbm_probe(const uint4* __restrict__ buf, size_t n,
                                                   double* __restrict__ sink) {
    __shared__ uint32_t red[4];
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    uint32_t x = 0;
    for (; k + 3 * stride < n; k += 4 * stride) {
        const uint4 a = buf[k], b = buf[k + stride], c = buf[k + 2 * stride], d = buf[k + 3 * stride];
        x ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^ d.z ^ d.w;
    }
    for (; k < n; k += stride) {
        const uint4 a = buf[k];
        x ^= a.x ^ a.y ^ a.z ^ a.w;
    }
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) x ^= (uint32_t)__shfl_xor((int)x, off, kWave);
    if (lane_id() == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) sink[blockIdx.x] = (double)(red[0] ^ red[1] ^ red[2] ^ red[3]);
}

template <typename T>
__global__ void k_fill(T* p, T v, size_t n) {
    for (size_t k = blockIdx.x * (size_t)blockDim.x + threadIdx.x; k < n;
         k += (size_t)gridDim.x * blockDim.x)
        p[k] = v;
}

// ==========================================================================
// launchers
// ==========================================================================
#define GBA_CHECK_LAUNCH()                 \
    do {                                   \
        hipError_t e_ = hipGetLastError(); \
        if (e_ != hipSuccess) return e_;   \
    } while (0)

template <typename T, typename JS>
static void linearize_kernels(const DeviceGraph& g, hipStream_t s, const RawOut& r, int grid) {
    const bool ad = g.jacobian == GBA_JACOBIAN_AUTODIFF;
    if (r.pos && !ad)
        hipLaunchKernelGGL((k_linearize<T, JS, true, false>), dim3(grid), dim3(256), 0, s, g, r);
    else if (ad)
        hipLaunchKernelGGL((k_linearize<T, JS, false, true>), dim3(grid), dim3(256), 0, s, g, r);
    else
        hipLaunchKernelGGL((k_linearize<T, JS, false, false>), dim3(grid), dim3(256), 0, s, g, r);
    if (r.pos && ad && g.ne > 0) {
        // the caller's layout from the one-lane-per-column kernel
        const size_t lanes = 12 * (size_t)g.ne;
        const int ag = (int)std::min<size_t>((lanes + 255) / 256, 65535);
        hipLaunchKernelGGL(k_jacobian_autodiff, dim3(ag), dim3(256), 0, s, g, r);
    }
}

hipError_t launch_linearize(const DeviceGraph& g, hipStream_t s, const RawOut* raw, bool zero_blocks) {
    RawOut r = raw ? *raw : RawOut{nullptr, nullptr, nullptr, nullptr, nullptr};
    const int blocks = (g.n_tiles * kWave + 255) / 256;
    const int grid = blocks < 1 ? 1 : blocks;
    if (g.mode == kModeFP64) {
        if (zero_blocks) hipLaunchKernelGGL(k_fill<double>, dim3(256), dim3(256), 0, s, (double*)g.hpp, 0.0, (size_t)6 * g.np);
        if (zero_blocks) hipLaunchKernelGGL(k_fill<double>, dim3(256), dim3(256), 0, s, (double*)g.bp, 0.0, (size_t)3 * g.np);
        linearize_kernels<double, double>(g, s, r, grid);
    } else if (g.mode == kModeFP32) {
        if (zero_blocks) hipLaunchKernelGGL(k_fill<float>, dim3(256), dim3(256), 0, s, (float*)g.hpp, 0.f, (size_t)6 * g.np);
        if (zero_blocks) hipLaunchKernelGGL(k_fill<float>, dim3(256), dim3(256), 0, s, (float*)g.bp, 0.f, (size_t)3 * g.np);
        linearize_kernels<float, float>(g, s, r, grid);
    } else {  // FP32 blocks, BF16 Jacobian
        if (zero_blocks) hipLaunchKernelGGL(k_fill<float>, dim3(256), dim3(256), 0, s, (float*)g.hpp, 0.f, (size_t)6 * g.np);
        if (zero_blocks) hipLaunchKernelGGL(k_fill<float>, dim3(256), dim3(256), 0, s, (float*)g.bp, 0.f, (size_t)3 * g.np);
        linearize_kernels<float, bf16>(g, s, r, grid);
    }
    GBA_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_assemble(const DeviceGraph& g, hipStream_t s) {
    if (g.nc == 0) return hipSuccess;
    if (g.n_chunks > 0) {
        const dim3 grid(g.n_chunks), block(256);
        if (g.jacobian == GBA_JACOBIAN_AUTODIFF) {
            if (g.mode == kModeFP64)
                hipLaunchKernelGGL((k_cam_accumulate<double, double, kAssemble, true>), grid, block, 0, s, g);
            else if (g.mode == kModeFP32)
                hipLaunchKernelGGL((k_cam_accumulate<float, float, kAssemble, true>), grid, block, 0, s, g);
            else
                hipLaunchKernelGGL((k_cam_accumulate<float, bf16, kAssemble, true>), grid, block, 0, s, g);
        } else {
            if (g.mode == kModeFP64)
                hipLaunchKernelGGL((k_cam_accumulate<double, double, kAssemble>), grid, block, 0, s, g);
            else if (g.mode == kModeFP32)
                hipLaunchKernelGGL((k_cam_accumulate<float, float, kAssemble>), grid, block, 0, s, g);
            else
                hipLaunchKernelGGL((k_cam_accumulate<float, bf16, kAssemble>), grid, block, 0, s, g);
        }
        GBA_CHECK_LAUNCH();
    }
    if (g.mode == kModeFP64)
        hipLaunchKernelGGL((k_cam_finalize<double, kAssemble>), dim3(g.nc), dim3(64), 0, s, g, 0.0, 0.0, 0, 0, 0, 0);
    else
        hipLaunchKernelGGL((k_cam_finalize<float, kAssemble>), dim3(g.nc), dim3(64), 0, s, g, 0.0, 0.0, 0, 0, 0, 0);
    if (g.bo_chunks > 0) {   // the Jacobian copy of the camera-blocked product pass
        const int grid = (int)std::min<long long>(4096, ((long long)g.ne + 255) / 256);
        if (g.mode == kModeFP64) hipLaunchKernelGGL(k_copy_jac_bo<double>, dim3(grid), dim3(256), 0, s, g);
        else if (g.mode == kModeFP32) hipLaunchKernelGGL(k_copy_jac_bo<float>, dim3(grid), dim3(256), 0, s, g);
        else hipLaunchKernelGGL(k_copy_jac_bo<bf16>, dim3(grid), dim3(256), 0, s, g);
    }
    GBA_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_cost(const DeviceGraph& g, hipStream_t s, const double* cam, const double* pt) {
    if (g.dc_edges.nblk == 0) return hipSuccess;
    hipLaunchKernelGGL(k_cost, dim3(g.dc_edges.nblk), dim3(256), 0, s, g, cam, pt);
    GBA_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_cost_finish(const DeviceGraph& g, hipStream_t s) {
    hipLaunchKernelGGL(k_cost_finish, dim3(1), dim3(1024), 0, s, g);
    GBA_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_damp(const DeviceGraph& g, hipStream_t s, double min_diag, double max_diag) {
    if (g.dc_pts.nblk == 0) return hipSuccess;
    if (g.mode == kModeFP64)
        hipLaunchKernelGGL(k_damp_points<double>, dim3(g.dc_pts.nblk), dim3(256), 0, s, g, min_diag, max_diag);
    else
        hipLaunchKernelGGL(k_damp_points<float>, dim3(g.dc_pts.nblk), dim3(256), 0, s, g, min_diag, max_diag);
    GBA_CHECK_LAUNCH();
    return hipSuccess;
}

// The block-Jacobi pass forms the reduced RHS too in the one-pass scheme;
// with the two-pass scheme (large camera sets) the separate RHS passes are
// cheaper than the extra registers the fused form costs there.
bool precond_forms_rhs(const DeviceGraph& g, int block_jacobi) {
    return block_jacobi != 0 && !g.cam_pass && !g.full;
}

hipError_t launch_precond(const DeviceGraph& g, hipStream_t s, double min_diag, double max_diag,
                          int block_jacobi, int jacobi_scaling) {
    if (g.nc == 0) return hipSuccess;
    const int rhs = precond_forms_rhs(g, block_jacobi) ? 1 : 0;
    // the full system's camera blocks have no point-elimination term
    if (block_jacobi && g.n_chunks > 0 && !g.full) {
        // the pass reads jst_cm: its storage type must be the mode's
        if (g.mode == kModeFP64) {
            if (rhs)
                hipLaunchKernelGGL((k_cam_accumulate<double, double, kPrecondRhs>), dim3(g.n_chunks), dim3(256), 0, s, g);
            else
                hipLaunchKernelGGL((k_cam_accumulate<double, double, kPrecond>), dim3(g.n_chunks), dim3(256), 0, s, g);
        } else if (g.mode == kModeFP32) {
            if (rhs)
                hipLaunchKernelGGL((k_cam_accumulate<float, float, kPrecondRhs>), dim3(g.n_chunks), dim3(256), 0, s, g);
            else
                hipLaunchKernelGGL((k_cam_accumulate<float, float, kPrecond>), dim3(g.n_chunks), dim3(256), 0, s, g);
        } else {
            if (rhs)
                hipLaunchKernelGGL((k_cam_accumulate<float, bf16, kPrecondRhs>), dim3(g.n_chunks), dim3(256), 0, s, g);
            else
                hipLaunchKernelGGL((k_cam_accumulate<float, bf16, kPrecond>), dim3(g.n_chunks), dim3(256), 0, s, g);
        }
        GBA_CHECK_LAUNCH();
    }
    if (g.mode == kModeFP64)
        hipLaunchKernelGGL((k_cam_finalize<double, kPrecond>), dim3(g.nc), dim3(64), 0, s, g, min_diag, max_diag, block_jacobi, rhs, jacobi_scaling, g.full);
    else
        hipLaunchKernelGGL((k_cam_finalize<float, kPrecond>), dim3(g.nc), dim3(64), 0, s, g, min_diag, max_diag, block_jacobi, rhs, jacobi_scaling, g.full);
    GBA_CHECK_LAUNCH();
    return hipSuccess;
}

// Raise a kernel's dynamic LDS limit to `lds` bytes on the current device
// (once per kernel and device; the attribute only grows).  Graph handles and
// the server thread may launch concurrently, so the check and the raise are
// one critical section.
static void ensure_lds(const void* fn, int lds, int* set /* [kMaxDevices] */) {
    static std::mutex mu;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(mu);
    int& cur = set[dev >= 0 && dev < kMaxDevices ? dev : 0];
    if (cur < lds) {
        (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        cur = lds;
    }
}

template <typename VT, typename JS, bool kDyn, int kMode>
static void full_point_pass(const DeviceGraph& g, hipStream_t s) {
    if (g.dc_pp.nblk == 0) return;
    const int lds = kMode == kBacksub ? 0 : g.lds_pp;
    static int lds_set[kMaxDevices] = {};
    if (lds > 0) ensure_lds((const void*)k_full_point_pass<VT, JS, kDyn, kMode>, lds, lds_set);
    hipLaunchKernelGGL((k_full_point_pass<VT, JS, kDyn, kMode>), dim3(g.dc_pp.nblk), dim3(g.block_pp),
                       lds, s, g);
}

template <int kMode>
static void full_pass(const DeviceGraph& g, hipStream_t s) {
    if (g.mode == kModeFP64) {
        if (g.dynamic) full_point_pass<double, double, true, kMode>(g, s);
        else full_point_pass<double, double, false, kMode>(g, s);
    } else if (g.mode == kModeFP32) {
        if (g.dynamic) full_point_pass<float, float, true, kMode>(g, s);
        else full_point_pass<float, float, false, kMode>(g, s);
    } else {
        if (g.dynamic) full_point_pass<float, bf16, true, kMode>(g, s);
        else full_point_pass<float, bf16, false, kMode>(g, s);
    }
}

template <typename VT, typename JS, typename AT, int kMode>
static void point_pass(const DeviceGraph& g, hipStream_t s, const void* vin, void* out) {
    if (g.dc_pp.nblk == 0) return;
    // dynamic LDS: the FP64 camera partials of the product and the RHS, beyond
    // the 64 KiB default (gfx950 has 160 KiB per CU)
    const int lds = kMode == kBacksub ? 0 : g.lds_pp;
    if (lds > 0) {
        // the attribute only grows, per device; graph handles and the server
        // thread may launch concurrently, so the check and the raise are one
        // critical section
        static std::mutex mu;
        static int lds_set[kMaxDevices] = {};
        int dev = 0;
        (void)hipGetDevice(&dev);
        std::lock_guard<std::mutex> lk(mu);
        int& cur = lds_set[dev >= 0 && dev < kMaxDevices ? dev : 0];
        if (cur < lds) {
            (void)hipFuncSetAttribute((const void*)k_point_pass<VT, JS, AT, kMode>,
                                      hipFuncAttributeMaxDynamicSharedMemorySize, lds);
            cur = lds;
        }
    }
    hipLaunchKernelGGL((k_point_pass<VT, JS, AT, kMode>), dim3(g.dc_pp.nblk), dim3(g.block_pp),
                       lds, s, g, (const void*)g.jst, (const VT*)vin, (AT*)out);
}

// Two-pass scheme, camera-major pass of the RHS or of the Schur product.
template <int kMode>
static void cam_pass(const DeviceGraph& g, hipStream_t s) {
    if (g.n_chunks == 0) return;
    if (g.mode == kModeFP64)
        hipLaunchKernelGGL((k_cam_pass<double, double, kMode>), dim3(g.n_chunks), dim3(kCamPassBlock), 0, s, g);
    else if (g.mode == kModeFP32)
        hipLaunchKernelGGL((k_cam_pass<float, float, kMode>), dim3(g.n_chunks), dim3(kCamPassBlock), 0, s, g);
    else
        hipLaunchKernelGGL((k_cam_pass<float, bf16, kMode>), dim3(g.n_chunks), dim3(kCamPassBlock), 0, s, g);
}

template <typename VT, typename JS>
static void cam_block_pass_t(const DeviceGraph& g, hipStream_t s) {
    const int lds = kCamBlock * 9 * (int)sizeof(double);
    static int lds_set[kMaxDevices] = {};
    ensure_lds((const void*)k_cam_block_pass<VT, JS>, lds, lds_set);
    hipLaunchKernelGGL((k_cam_block_pass<VT, JS>), dim3(g.bo_chunks), dim3(kCamBlockThreads), lds, s, g);
}

static void cam_block_pass(const DeviceGraph& g, hipStream_t s) {
    if (g.mode == kModeFP64) cam_block_pass_t<double, double>(g, s);
    else if (g.mode == kModeFP32) cam_block_pass_t<float, float>(g, s);
    else cam_block_pass_t<float, bf16>(g, s);
}

hipError_t launch_rhs(const DeviceGraph& g, hipStream_t s) {
    if (g.nc == 0) return hipSuccess;   // no cameras, hence no edges
    if (g.cam_pass) {
        const int grid = g.np > 0 ? (g.np + 255) / 256 < 4096 ? (g.np + 255) / 256 : 4096 : 1;
        if (g.mode == kModeFP64) {
            hipLaunchKernelGGL(k_rhs_z<double>, dim3(grid), dim3(256), 0, s, g);
            cam_pass<kRhs>(g, s);
            hipLaunchKernelGGL((k_reduce<double, kRhs>), dim3(g.dc_red.nblk), dim3(1024), 0, s, g, 0.0, 0.0);
        } else {
            hipLaunchKernelGGL(k_rhs_z<float>, dim3(grid), dim3(256), 0, s, g);
            cam_pass<kRhs>(g, s);
            hipLaunchKernelGGL((k_reduce<float, kRhs>), dim3(g.dc_red.nblk), dim3(1024), 0, s, g, 0.0, 0.0);
        }
        GBA_CHECK_LAUNCH();
        return hipSuccess;
    }
    if (g.mode == kModeFP64) {
        point_pass<double, double, double, kRhs>(g, s, nullptr, g.cam_partial);
        hipLaunchKernelGGL((k_reduce<double, kRhs>), dim3(g.dc_red.nblk), dim3(1024), 0, s, g, 0.0, 0.0);
    } else {
        if (g.mode == kModeFP32)
            point_pass<float, float, double, kRhs>(g, s, nullptr, g.cam_partial);
        else
            point_pass<float, bf16, double, kRhs>(g, s, nullptr, g.cam_partial);
        hipLaunchKernelGGL((k_reduce<float, kRhs>), dim3(g.dc_red.nblk), dim3(1024), 0, s, g, 0.0, 0.0);
    }
    GBA_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_pcg_init(const DeviceGraph& g, hipStream_t s, double tol, int relative) {
    if (g.nc == 0) return hipSuccess;
    if (g.mode == kModeFP64) {
        hipLaunchKernelGGL(k_pcg_start<double>, dim3(g.dc_cam.nblk), dim3(kPcgBlock), 0, s, g);
        if (g.full && g.dc_pts.nblk > 0)
            hipLaunchKernelGGL(k_pcg_start_pts<double>, dim3(g.dc_pts.nblk), dim3(kPcgBlock), 0, s, g);
        hipLaunchKernelGGL(k_pcg_start_finish, dim3(1), dim3(1024), 0, s, g, tol, relative);
    } else {
        hipLaunchKernelGGL(k_pcg_start<float>, dim3(g.dc_cam.nblk), dim3(kPcgBlock), 0, s, g);
        if (g.full && g.dc_pts.nblk > 0)
            hipLaunchKernelGGL(k_pcg_start_pts<float>, dim3(g.dc_pts.nblk), dim3(kPcgBlock), 0, s, g);
        hipLaunchKernelGGL(k_pcg_start_finish, dim3(1), dim3(1024), 0, s, g, tol, relative);
    }
    GBA_CHECK_LAUNCH();
    return hipSuccess;
}

// The product of one PCG iteration (with its decision): the Schur product of
// z; q = S p follows from it by linearity in the reduction.
hipError_t launch_matvec(const DeviceGraph& g0, hipStream_t s, int max_iters, double ratio) {
    if (g0.nc == 0) return hipSuccess;
    DeviceGraph g = g0;
    g.pcg_max_iters = max_iters;
    g.pcg_ratio = ratio;
    if (g.full) {
        full_pass<kMatvec>(g, s);
        GBA_CHECK_LAUNCH();
        return hipSuccess;
    }
    if (g.mode == kModeFP64) {
        point_pass<double, double, double, kMatvec>(g, s, g.v_z, g.cam_partial);
    } else if (g.mode == kModeFP32) {
        point_pass<float, float, double, kMatvec>(g, s, g.v_z, g.cam_partial);
    } else {
        point_pass<float, bf16, double, kMatvec>(g, s, g.v_z, g.cam_partial);
    }
    if (g.cam_pass && g.bo_chunks > 0) cam_block_pass(g, s);
    else if (g.cam_pass) cam_pass<kMatvec>(g, s);
    GBA_CHECK_LAUNCH();
    return hipSuccess;
}

// One PCG iteration: the product (which takes the step's decision), the q
// reduction and the vector update.
hipError_t launch_pcg_iter(const DeviceGraph& g, hipStream_t s, double min_diag, double max_diag,
                           int max_iters, double ratio, hipEvent_t ev0, hipEvent_t ev1) {
    if (g.nc == 0) return hipSuccess;
    if (ev0) (void)hipEventRecord(ev0, s);
    hipError_t e = launch_matvec(g, s, max_iters, ratio);
    if (e != hipSuccess) return e;
    if (ev1) (void)hipEventRecord(ev1, s);
    const int apply_blocks = g.dc_cam.nblk + (g.full ? g.dc_pts.nblk : 0);
    // small problems: the reduction's last workgroup per problem runs the update
    if (g.mode == kModeFP64) {
        hipLaunchKernelGGL((k_reduce<double, kMatvec>), dim3(g.dc_red.nblk), dim3(1024), 0, s, g, min_diag, max_diag);
        if (!g.fuse_apply)
            hipLaunchKernelGGL(k_pcg_apply<double>, dim3(apply_blocks), dim3(kPcgBlock), 0, s, g);
    } else {
        hipLaunchKernelGGL((k_reduce<float, kMatvec>), dim3(g.dc_red.nblk), dim3(1024), 0, s, g, min_diag, max_diag);
        if (!g.fuse_apply)
            hipLaunchKernelGGL(k_pcg_apply<float>, dim3(apply_blocks), dim3(kPcgBlock), 0, s, g);
    }
    GBA_CHECK_LAUNCH();
    return hipSuccess;
}

template <typename VT, typename JS, int kForm>
static hipError_t persistent_launch(const DeviceGraph& g, hipStream_t s, double min_diag,
                                    double max_diag, int max_launch, bool check_only) {
    const void* fn = (const void*)k_pcg_persistent<VT, JS, kForm>;
    const int lds = g.cam_pass ? 0 : g.lds_pp;
    int dev = 0, coop = 0, n_cu = 0, max_lds = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess)
        e = hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
    if (e != hipSuccess) return e;
    if (!coop || lds + 4096 > max_lds) return hipErrorNotSupported;
    if (lds > 0) {
        e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
        if (e != hipSuccess) return e;
    }
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kPersistentBlock, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorNotSupported;
    if (check_only) return hipSuccess;
    // one workgroup per product and reduction workgroup, or per kSubs vector
    // (camera-pass) workgroups, up to a co-resident grid
    constexpr int kSubsV = kPersistentBlock / kPcgBlock, kSubsC = kPersistentBlock / kCamPassBlock;
    int want = std::max(std::max(g.dc_pp.nblk, g.dc_red.nblk),
                        std::max((g.dc_cam.nblk + kSubsV - 1) / kSubsV,
                                 g.full ? (g.dc_pts.nblk + kSubsV - 1) / kSubsV : 0));
    if (g.cam_pass) want = std::max(want, (g.n_chunks + kSubsC - 1) / kSubsC);
    const int grid = std::max(1, std::min(want, per_cu * n_cu));
    // a fresh barrier: arrivals, generation and error flag cleared by a fill
    // kernel (no memset node, so the launch may be captured)
    hipLaunchKernelGGL(k_fill<unsigned int>, dim3(1), dim3(256), 0, s, g.gbar, 0u, (size_t)kGbarWords);
    GBA_CHECK_LAUNCH();
    DeviceGraph ga = g;
    ga.fuse_apply = 0;   // the update is a phase of its own here
    void* args[] = {(void*)&ga, (void*)&min_diag, (void*)&max_diag, (void*)&max_launch};
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kPersistentBlock), args, (unsigned)lds, s);
}

template <bool kCheck, int kForm>
static hipError_t persistent_form(const DeviceGraph& g, hipStream_t s, double min_diag,
                                  double max_diag, int max_launch) {
    if (g.mode == kModeFP64)
        return persistent_launch<double, double, kForm>(g, s, min_diag, max_diag, max_launch, kCheck);
    if (g.mode == kModeFP32)
        return persistent_launch<float, float, kForm>(g, s, min_diag, max_diag, max_launch, kCheck);
    return persistent_launch<float, bf16, kForm>(g, s, min_diag, max_diag, max_launch, kCheck);
}

template <bool kCheck>
static hipError_t persistent_dispatch(const DeviceGraph& g, hipStream_t s, double min_diag,
                                      double max_diag, int max_launch) {
    if (!g.full) return persistent_form<kCheck, 0>(g, s, min_diag, max_diag, max_launch);
    if (!g.dynamic) return persistent_form<kCheck, 1>(g, s, min_diag, max_diag, max_launch);
    return persistent_form<kCheck, 2>(g, s, min_diag, max_diag, max_launch);
}

bool pcg_persistent_ok(const DeviceGraph& g) {
    return persistent_dispatch<true>(g, nullptr, 0.0, 0.0, 1) == hipSuccess;
}

hipError_t launch_pcg_persistent(const DeviceGraph& g0, hipStream_t s, double min_diag, double max_diag,
                                 int max_iters, double ratio) {
    if (g0.nc == 0) return hipSuccess;
    DeviceGraph g = g0;
    g.bo_chunks = 0;   // the persistent kernel takes the camera-major pass (its structures are always built)
    g.pcg_max_iters = max_iters;
    g.pcg_ratio = ratio;
    // a PCG of k steps takes k + 1 iterations (the last finds the stop)
    return persistent_dispatch<false>(g, s, min_diag, max_diag, max_iters + 1);
}

hipError_t launch_backsub(const DeviceGraph& g, hipStream_t s) {
    if (g.nc == 0) return hipSuccess;
    if (g.full) {
        // the point step is the PCG's point part: candidates and model terms
        if (g.mode == kModeFP64)
            hipLaunchKernelGGL(k_cam_update<double>, dim3(g.dc_cam.nblk), dim3(kPcgBlock), 0, s, g);
        else
            hipLaunchKernelGGL(k_cam_update<float>, dim3(g.dc_cam.nblk), dim3(kPcgBlock), 0, s, g);
        full_pass<kBacksub>(g, s);
        GBA_CHECK_LAUNCH();
        return hipSuccess;
    }
    if (g.mode == kModeFP64) {
        hipLaunchKernelGGL(k_cam_update<double>, dim3(g.dc_cam.nblk), dim3(kPcgBlock), 0, s, g);
        point_pass<double, double, double, kBacksub>(g, s, g.v_x, nullptr);
    } else {
        hipLaunchKernelGGL(k_cam_update<float>, dim3(g.dc_cam.nblk), dim3(kPcgBlock), 0, s, g);
        if (g.mode == kModeFP32)
            point_pass<float, float, double, kBacksub>(g, s, g.v_x, nullptr);
        else
            point_pass<float, bf16, double, kBacksub>(g, s, g.v_x, nullptr);
    }
    GBA_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_finish(const DeviceGraph& g, hipStream_t s) {
    hipLaunchKernelGGL(k_finish, dim3(1), dim3(1024), 0, s, g);
    GBA_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_pack(const PackDesc* desc, const PackChunk* chunks, int n_chunks, hipStream_t s) {
    if (n_chunks <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pack, dim3(n_chunks), dim3(256), 0, s, desc, chunks);
    GBA_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_fill_f64(double* p, double v, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t grid = (n + 255) / 256;
    grid = grid > 4096 ? 4096 : grid;
    hipLaunchKernelGGL(k_fill<double>, dim3((unsigned)grid), dim3(256), 0, s, p, v, n);
    GBA_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_hbm_probe(const void* buf, size_t n16, double* sink, hipStream_t s) {
    hipLaunchKernelGGL(k_hbm_probe, dim3(kProbeBlocks), dim3(256), 0, s, (const uint4*)buf, n16, sink);
    GBA_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_commit(const DeviceGraph& g, hipStream_t s) {
    size_t n = 9 * (size_t)g.nc > 3 * (size_t)g.np ? 9 * (size_t)g.nc : 3 * (size_t)g.np;
    int grid = (int)((n + 255) / 256);
    grid = grid < 1 ? 1 : (grid > 2048 ? 2048 : grid);
    hipLaunchKernelGGL(k_commit, dim3(grid), dim3(256), 0, s, g);
    GBA_CHECK_LAUNCH();
    return hipSuccess;
}

}  // namespace gba
