// Device helpers of the gfx950 bundle-adjustment kernels: wavefront
// segmented reductions, the closed-form BAL residual and Jacobian, robust
// weighting, BF16 storage and small symmetric-block algebra.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gba_internal.h"

namespace gba {

// ------------------------------------------------------------ bf16 storage
struct bf16 {
    uint16_t v;
};

__device__ __forceinline__ float to_float(bf16 x) {
    return __uint_as_float(((uint32_t)x.v) << 16);
}
__device__ __forceinline__ float to_float(float x) { return x; }
__device__ __forceinline__ double to_float(double x) { return x; }

// round-to-nearest-even FP32 -> BF16 (finite inputs)
__device__ __forceinline__ bf16 to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return bf16{(uint16_t)(u >> 16)};
}

template <typename S, typename T>
__device__ __forceinline__ S store_as(T x) { return (S)x; }
template <>
__device__ __forceinline__ bf16 store_as<bf16, float>(float x) { return to_bf16(x); }

template <typename T, typename S>
__device__ __forceinline__ T load_as(S x) { return (T)to_float(x); }

// Storage of a Jacobian entry computed in the arithmetic type A, and the
// value the stored entry represents (the linear system is built from what is
// stored).
template <typename JS, typename A>
__device__ __forceinline__ JS jac_store(A x) { return (JS)x; }
template <>
__device__ __forceinline__ bf16 jac_store<bf16, double>(double x) { return to_bf16((float)x); }
template <>
__device__ __forceinline__ bf16 jac_store<bf16, float>(float x) { return to_bf16(x); }
template <typename JS, typename A>
__device__ __forceinline__ A jac_round(A x) { return (A)to_float(jac_store<JS, A>(x)); }

// ------------------------------------------------ stored Jacobian layout
// 24 entries per edge, in the order jc[0][0..8], jc[1][0..8], jp[0][0..2],
// jp[1][0..2], packed into 16-byte chunks of 2 (FP64), 4 (FP32) or 8 (BF16)
// entries.  Chunk c of edge e is 16-byte element ((e / 64) * n + c) * 64 +
// e % 64 (n chunks per edge): a wavefront reading chunk c of 64 consecutive
// edges reads one contiguous KiB with one 16-byte load per lane.
union Chunk16 {
    uint4 u;
    double d[2];
    float f[4];
    uint16_t h[8];
};

template <typename JS> struct JacPack;
template <> struct JacPack<double> { static constexpr int kPer = 2; };
template <> struct JacPack<float> { static constexpr int kPer = 4; };
template <> struct JacPack<bf16> { static constexpr int kPer = 8; };

__host__ __device__ __forceinline__ size_t jac_chunk(int e, int c, int n) {
    return ((size_t)(e >> 6) * n + c) * 64 + (e & 63);
}

// entry s of a 16-byte chunk of storage type JS, in the arithmetic type A
__device__ __forceinline__ double chunk_raw(const Chunk16& q, int s, double*) { return q.d[s]; }
__device__ __forceinline__ float chunk_raw(const Chunk16& q, int s, float*) { return q.f[s]; }
__device__ __forceinline__ float chunk_raw(const Chunk16& q, int s, bf16*) {
    return __uint_as_float(((uint32_t)q.h[s]) << 16);
}
template <typename A, typename JS>
__device__ __forceinline__ A chunk_get(const Chunk16& q, int s) {
    return (A)chunk_raw(q, s, (JS*)nullptr);
}
// kept for the FP64 sums of stored entries
__device__ __forceinline__ double chunk_get(const Chunk16& q, int s, double*) { return q.d[s]; }
__device__ __forceinline__ double chunk_get(const Chunk16& q, int s, float*) { return (double)q.f[s]; }
__device__ __forceinline__ double chunk_get(const Chunk16& q, int s, bf16*) {
    return (double)__uint_as_float(((uint32_t)q.h[s]) << 16);
}
template <typename A>
__device__ __forceinline__ void chunk_put(Chunk16& q, int s, A x, double*) { q.d[s] = (double)x; }
template <typename A>
__device__ __forceinline__ void chunk_put(Chunk16& q, int s, A x, float*) { q.f[s] = (float)x; }
template <typename A>
__device__ __forceinline__ void chunk_put(Chunk16& q, int s, A x, bf16*) {
    q.h[s] = to_bf16((float)x).v;
}

// the 24 stored entries of edge e, in the arithmetic type A
template <typename JS, typename A>
__device__ __forceinline__ void jac_load(const void* __restrict__ J, int e, A (&jc)[2][9],
                                         A (&jp)[2][3]) {
    constexpr int kPer = JacPack<JS>::kPer, kCh = 24 / kPer;
    const uint4* __restrict__ src = (const uint4*)J;
    A v[24];
#pragma unroll
    for (int c = 0; c < kCh; ++c) {
        Chunk16 q;
        q.u = src[jac_chunk(e, c, kCh)];
#pragma unroll
        for (int s = 0; s < kPer; ++s) v[c * kPer + s] = chunk_get<A, JS>(q, s);
    }
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        jc[0][a] = v[a];
        jc[1][a] = v[9 + a];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        jp[0][a] = v[18 + a];
        jp[1][a] = v[21 + a];
    }
}

// store the 24 entries of edge e, rounded to JS as jac_store<JS> does
template <typename JS, typename A>
__device__ __forceinline__ void jac_save(void* __restrict__ J, int e, const A (&jc)[2][9],
                                         const A (&jp)[2][3]) {
    constexpr int kPer = JacPack<JS>::kPer, kCh = 24 / kPer;
    A v[24];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        v[a] = jc[0][a];
        v[9 + a] = jc[1][a];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        v[18 + a] = jp[0][a];
        v[21 + a] = jp[1][a];
    }
    uint4* __restrict__ dst = (uint4*)J;
#pragma unroll
    for (int c = 0; c < kCh; ++c) {
        Chunk16 q;
#pragma unroll
        for (int s = 0; s < kPer; ++s) chunk_put<A>(q, s, v[c * kPer + s], (JS*)nullptr);
        dst[jac_chunk(e, c, kCh)] = q.u;
    }
}

// ------------------------------------------------------------ wave helpers
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

// For a 64-bit mask of segment starts, the first lane (head) and the last
// lane (end) of the segment holding lane l.
__device__ __forceinline__ void segment_of(uint64_t starts, int l, int& head, int& end) {
    const uint64_t upto = (l == 63) ? ~0ull : ((2ull << l) - 1ull);
    const uint64_t le = starts & upto;
    head = 63 - __clzll((long long)le);
    const uint64_t after = starts & ~upto;
    end = after ? (__ffsll((long long)after) - 2) : 63;
}

template <typename T>
__device__ __forceinline__ T shfl_down64(T v, int off) {
    return __shfl_down(v, off, kWave);
}
template <typename T>
__device__ __forceinline__ T shfl64(T v, int src) {
    return __shfl(v, src, kWave);
}

// Segmented inclusive prefix sums across a wavefront by DPP lane moves, with
// no LDS traffic (a ds_bpermute shuffle goes through the LDS crossbar and
// waits for it): Hillis-Steele steps of 1, 2, 4 and 8 lanes inside each row
// of 16, then the broadcasts of lane 15 into rows 1 and 3 and of lane 31
// into rows 2 and 3.  `start` marks the first lane of a segment.  After
// sum(v) the last lane of each segment holds the segment's total (the order
// of the additions depends only on the segmentation).  The closing flags of
// the six steps are computed once per segmentation and shared by its sums.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ int dpp_move(int v) {
    // lanes outside the row mask, or without a source lane, read 0
    return __builtin_amdgcn_update_dpp(0, v, kCtrl, kRowMask, 0xF, false);
}

struct SegScan {
    bool closed[6];   // before step s the lane's prefix already starts a segment

    __device__ __forceinline__ explicit SegScan(bool start) {
        int f = start ? 1 : 0;
        closed[0] = f != 0;
        f |= dpp_move<0x111, 0xF>(f);   // row_shr:1
        closed[1] = f != 0;
        f |= dpp_move<0x112, 0xF>(f);   // row_shr:2
        closed[2] = f != 0;
        f |= dpp_move<0x114, 0xF>(f);   // row_shr:4
        closed[3] = f != 0;
        f |= dpp_move<0x118, 0xF>(f);   // row_shr:8
        closed[4] = f != 0;
        f |= dpp_move<0x142, 0xA>(f);   // row_bcast:15
        closed[5] = f != 0;
    }

    template <int kCtrl, int kRowMask>
    __device__ __forceinline__ static float move(float v) {
        return __int_as_float(dpp_move<kCtrl, kRowMask>(__float_as_int(v)));
    }
    template <int kCtrl, int kRowMask>
    __device__ __forceinline__ static double move(double v) {
        const int lo = dpp_move<kCtrl, kRowMask>(__double2loint(v));
        const int hi = dpp_move<kCtrl, kRowMask>(__double2hiint(v));
        return __hiloint2double(hi, lo);
    }

    template <typename T>
    __device__ __forceinline__ T sum(T v) const {
        T m;
        m = move<0x111, 0xF>(v);
        v = closed[0] ? v : v + m;
        m = move<0x112, 0xF>(v);
        v = closed[1] ? v : v + m;
        m = move<0x114, 0xF>(v);
        v = closed[2] ? v : v + m;
        m = move<0x118, 0xF>(v);
        v = closed[3] ? v : v + m;
        m = move<0x142, 0xA>(v);
        v = closed[4] ? v : v + m;
        m = move<0x143, 0xC>(v);
        v = closed[5] ? v : v + m;
        return v;
    }
};

// Sum over the 64 lanes of a wavefront (every lane active), returned to
// every lane: the inclusive-scan steps of SegScan without segments (DPP lane
// moves, no LDS round trips), then lane 63's total read into a scalar
// register.  The order of the additions is fixed.
__device__ __forceinline__ float lane63(float v) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ double lane63(double v) {
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), 63);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), 63);
    return __hiloint2double(hi, lo);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    v += SegScan::move<0x111, 0xF>(v);
    v += SegScan::move<0x112, 0xF>(v);
    v += SegScan::move<0x114, 0xF>(v);
    v += SegScan::move<0x118, 0xF>(v);
    v += SegScan::move<0x142, 0xA>(v);
    v += SegScan::move<0x143, 0xC>(v);
    return lane63(v);
}

// Block-wide sum; every thread gets the result.  `red` holds >= 16 values.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T* red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    const int nw = (blockDim.x + kWave - 1) >> 6;
    __syncthreads();
    if (lane_id() == 0) red[w] = v;
    __syncthreads();
    T s = 0;
    for (int k = 0; k < nw; ++k) s += red[k];
    __syncthreads();
    return s;
}

// Sum over a sub-block of kSub consecutive threads (a whole number of waves
// that divides the workgroup); every thread gets its sub-block's sum.  Every
// thread of the workgroup calls it (it holds the workgroup's barriers).  With
// kSub == blockDim.x it is block_sum, in the same order.  `red` holds one
// value per wave of the workgroup (>= 16).
template <int kSub, typename T>
__device__ __forceinline__ T sub_sum(T v, T* red) {
    static_assert(kSub % kWave == 0, "a sub-block is whole waves");
    constexpr int nw = kSub / kWave;
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    const int w0 = w - w % nw;
    __syncthreads();
    if (lane_id() == 0) red[w] = v;
    __syncthreads();
    T s = 0;
    for (int k = 0; k < nw; ++k) s += red[w0 + k];
    __syncthreads();
    return s;
}

// ------------------------------------------- camera-vector gathers
// The 9 entries of camera i of a [nc][9] vector with 16-byte loads: the
// aligned chunks covering them (3 for FP32, 5 for FP64) and a select of the
// start.  May read up to 12 (FP32) / 8 (FP64) bytes past the last camera;
// the vectors are allocated with that slack.
__device__ __forceinline__ uint32_t pick32(uint32_t a, uint32_t b, uint32_t m) {
    return (a & ~m) | (b & m);   // m = 0: a, m = ~0: b (bitwise, no memory select)
}

template <typename A>
__device__ __forceinline__ void gather9(const float* __restrict__ v, int i, A (&out)[9]) {
    const size_t w = 9 * (size_t)i;
    const uint4* b = (const uint4*)(v + (w & ~(size_t)3));
    const uint32_t m1 = (w & 1) ? ~0u : 0u, m2 = (w & 2) ? ~0u : 0u;
    const uint4 c0 = b[0], c1 = b[1], c2 = b[2];
    const uint32_t q[12] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w, c2.x, c2.y, c2.z, c2.w};
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const uint32_t lo = pick32(q[k], q[k + 1], m1);
        const uint32_t hi = pick32(q[k + 2], q[k + 3], m1);
        out[k] = (A)__uint_as_float(pick32(lo, hi, m2));
    }
}

__device__ __forceinline__ void gather9(const double* __restrict__ v, int i, double (&out)[9]) {
    const size_t w = 9 * (size_t)i;
    const uint4* b = (const uint4*)(v + (w & ~(size_t)1));
    const uint32_t m = (w & 1) ? ~0u : 0u;
    const uint4 c0 = b[0], c1 = b[1], c2 = b[2], c3 = b[3], c4 = b[4];
    const uint32_t q[20] = {c0.x, c0.y, c0.z, c0.w, c1.x, c1.y, c1.z, c1.w, c2.x, c2.y,
                            c2.z, c2.w, c3.x, c3.y, c3.z, c3.w, c4.x, c4.y, c4.z, c4.w};
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const uint32_t lo = pick32(q[2 * k], q[2 * k + 2], m);
        const uint32_t hi = pick32(q[2 * k + 1], q[2 * k + 3], m);
        out[k] = __hiloint2double((int)hi, (int)lo);
    }
}

// ------------------------------------------------------ BAL camera model
// r = f (1 + k1 |p|^2 + k2 |p|^4) p - obs with p = -(P_x, P_y) / P_z and
// P = R(w) X + t; jc = dr/d(w, t, f, k1, k2), jp = dr/dX.
// Rotation: R = I + a W + b W^2 with W = [w]x, a = sin(th)/th,
// b = (1 - cos th)/th^2 (Rodrigues); derivative w.r.t. the angle-axis vector
// dP/dw = -R [X]x Jr(w) with the right Jacobian Jr = I - b W + c W^2,
// c = (th - sin th)/th^3.  For th^2 <= 1e-16 the rotation is taken to first
// order, R X = X + w x X, whose derivative is dP/dw = -[X]x.
template <typename T>
struct EdgeEval {
    T r[2];
    T jc[2][9];
    T jp[2][3];
};

template <typename T, bool kJac>
__device__ __forceinline__ void bal_eval(const double* __restrict__ cam,
                                         const double* __restrict__ X, double ou, double ov,
                                         EdgeEval<T>& e) {
    const T w0 = (T)cam[0], w1 = (T)cam[1], w2 = (T)cam[2];
    const T x0 = (T)X[0], x1 = (T)X[1], x2 = (T)X[2];
    const T th2 = w0 * w0 + w1 * w1 + w2 * w2;
    T R[3][3], M[3][3];
    if (th2 > (T)1e-16) {
        const T th = sqrt(th2);
        const T s = sin(th);
        const T hs = sin((T)0.5 * th);
        const T a = s / th;
        const T b = (T)2 * hs * hs / th2;
        R[0][0] = (T)1 + b * (w0 * w0 - th2);
        R[0][1] = -a * w2 + b * w0 * w1;
        R[0][2] = a * w1 + b * w0 * w2;
        R[1][0] = a * w2 + b * w1 * w0;
        R[1][1] = (T)1 + b * (w1 * w1 - th2);
        R[1][2] = -a * w0 + b * w1 * w2;
        R[2][0] = -a * w1 + b * w2 * w0;
        R[2][1] = a * w0 + b * w2 * w1;
        R[2][2] = (T)1 + b * (w2 * w2 - th2);
        if (kJac) {
            const T c = th < (T)1e-2
                            ? ((T)1 / (T)6 - th2 * ((T)1 / (T)120 - th2 * ((T)1 / (T)5040)))
                            : (th - s) / (th2 * th);
            T Jr[3][3];
            Jr[0][0] = (T)1 + c * (w0 * w0 - th2);
            Jr[0][1] = b * w2 + c * w0 * w1;
            Jr[0][2] = -b * w1 + c * w0 * w2;
            Jr[1][0] = -b * w2 + c * w1 * w0;
            Jr[1][1] = (T)1 + c * (w1 * w1 - th2);
            Jr[1][2] = b * w0 + c * w1 * w2;
            Jr[2][0] = b * w1 + c * w2 * w0;
            Jr[2][1] = -b * w0 + c * w2 * w1;
            Jr[2][2] = (T)1 + c * (w2 * w2 - th2);
            // K = R [X]x,  [X]x = [[0,-x2,x1],[x2,0,-x0],[-x1,x0,0]]
            T K[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                K[i][0] = R[i][1] * x2 - R[i][2] * x1;
                K[i][1] = -R[i][0] * x2 + R[i][2] * x0;
                K[i][2] = R[i][0] * x1 - R[i][1] * x0;
            }
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    M[i][j] = -(K[i][0] * Jr[0][j] + K[i][1] * Jr[1][j] + K[i][2] * Jr[2][j]);
        }
    } else {
        R[0][0] = (T)1;
        R[0][1] = -w2;
        R[0][2] = w1;
        R[1][0] = w2;
        R[1][1] = (T)1;
        R[1][2] = -w0;
        R[2][0] = -w1;
        R[2][1] = w0;
        R[2][2] = (T)1;
        if (kJac) {
            M[0][0] = 0;
            M[0][1] = x2;
            M[0][2] = -x1;
            M[1][0] = -x2;
            M[1][1] = 0;
            M[1][2] = x0;
            M[2][0] = x1;
            M[2][1] = -x0;
            M[2][2] = 0;
        }
    }
    const T P0 = R[0][0] * x0 + R[0][1] * x1 + R[0][2] * x2 + (T)cam[3];
    const T P1 = R[1][0] * x0 + R[1][1] * x1 + R[1][2] * x2 + (T)cam[4];
    const T P2 = R[2][0] * x0 + R[2][1] * x1 + R[2][2] * x2 + (T)cam[5];
    const T f = (T)cam[6], k1 = (T)cam[7], k2 = (T)cam[8];
    const T inv = (T)1 / P2;
    const T px = -P0 * inv, py = -P1 * inv;
    const T n = px * px + py * py;
    const T d = (T)1 + k1 * n + k2 * n * n;
    const T fd = f * d;
    e.r[0] = fd * px - (T)ou;
    e.r[1] = fd * py - (T)ov;
    if (!kJac) return;
    const T g = (T)2 * f * (k1 + (T)2 * k2 * n);
    const T A00 = fd + g * px * px, A01 = g * px * py, A11 = fd + g * py * py;
    T G[2][3];
    G[0][0] = -inv * A00;
    G[0][1] = -inv * A01;
    G[0][2] = -inv * (A00 * px + A01 * py);
    G[1][0] = -inv * A01;
    G[1][1] = -inv * A11;
    G[1][2] = -inv * (A01 * px + A11 * py);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            e.jp[a][j] = G[a][0] * R[0][j] + G[a][1] * R[1][j] + G[a][2] * R[2][j];
            e.jc[a][j] = G[a][0] * M[0][j] + G[a][1] * M[1][j] + G[a][2] * M[2][j];
            e.jc[a][3 + j] = G[a][j];
        }
    }
    e.jc[0][6] = d * px;
    e.jc[1][6] = d * py;
    e.jc[0][7] = f * n * px;
    e.jc[1][7] = f * n * py;
    e.jc[0][8] = f * n * n * px;
    e.jc[1][8] = f * n * n * py;
}

// Robust kernel on s (squared Mahalanobis norm): rho(s) and the IRLS weight
// rho'(s).  Huber: rho = s (s <= d^2), 2 d sqrt(s) - d^2 otherwise.
template <typename T>
__device__ __forceinline__ void robust(int loss, double delta, T s, T& rho, T& w) {
    const T d = (T)delta;
    if (loss == 1 && s > d * d) {
        const T q = sqrt(s);
        rho = (T)2 * d * q - d * d;
        w = d / q;
    } else {
        rho = s;
        w = (T)1;
    }
}

// Whiten one edge: with Omega = A^T A (A upper triangular, rows (a00 a01),
// (0 a11)), r~ = sqrt(w) A r and J~ = sqrt(w) A J.  Returns s = |A r|^2 and
// rho(s).  Jacobian blocks of fixed vertices are zeroed.
template <typename T, bool kJac>
__device__ __forceinline__ void whiten(EdgeEval<T>& e, const double* sinfo, int stride, int idx,
                                       int loss, double delta, bool cam_fixed, bool pt_fixed,
                                       T& s_out, T& rho_out, T& w_out) {
    T a00 = 1, a01 = 0, a11 = 1;
    if (sinfo) {
        a00 = (T)sinfo[idx];
        a01 = (T)sinfo[stride + idx];
        a11 = (T)sinfo[2 * stride + idx];
    }
    const T ar0 = a00 * e.r[0] + a01 * e.r[1];
    const T ar1 = a11 * e.r[1];
    const T s = ar0 * ar0 + ar1 * ar1;
    T rho, w;
    robust<T>(loss, delta, s, rho, w);
    const T sw = sqrt(w);
    e.r[0] = sw * ar0;
    e.r[1] = sw * ar1;
    s_out = s;
    rho_out = rho;
    w_out = w;
    if (!kJac) return;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const T j0 = e.jc[0][k], j1 = e.jc[1][k];
        e.jc[0][k] = cam_fixed ? (T)0 : sw * (a00 * j0 + a01 * j1);
        e.jc[1][k] = cam_fixed ? (T)0 : sw * (a11 * j1);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const T j0 = e.jp[0][k], j1 = e.jp[1][k];
        e.jp[0][k] = pt_fixed ? (T)0 : sw * (a00 * j0 + a01 * j1);
        e.jp[1][k] = pt_fixed ? (T)0 : sw * (a11 * j1);
    }
}

// ------------------------------------------------ small symmetric algebra
// In-place inverse of a symmetric positive definite n x n matrix given as a
// full row-major array, via Cholesky.  Returns false if not positive definite.
template <int N>
__device__ inline bool spd_inverse(double (&A)[N][N]) {
    double L[N][N];
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j) L[i][j] = 0.0;
    for (int j = 0; j < N; ++j) {
        double s = A[j][j];
        for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
        if (!(s > 0.0)) return false;
        const double ljj = sqrt(s);
        L[j][j] = ljj;
        const double il = 1.0 / ljj;
        for (int i = j + 1; i < N; ++i) {
            double t = A[i][j];
            for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
            L[i][j] = t * il;
        }
    }
    // Linv lower triangular
    double Li[N][N];
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) Li[i][j] = 0.0;
    for (int i = 0; i < N; ++i) {
        Li[i][i] = 1.0 / L[i][i];
        for (int j = 0; j < i; ++j) {
            double t = 0.0;
            for (int k = j; k < i; ++k) t -= L[i][k] * Li[k][j];
            Li[i][j] = t / L[i][i];
        }
    }
    // A^{-1} = Linv^T Linv
    for (int i = 0; i < N; ++i)
        for (int j = i; j < N; ++j) {
            double t = 0.0;
            for (int k = j; k < N; ++k) t += Li[k][i] * Li[k][j];
            A[i][j] = t;
            A[j][i] = t;
        }
    return true;
}

}  // namespace gba
