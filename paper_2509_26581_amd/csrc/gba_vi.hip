// Visual-inertial factors on the GPU (Background Eq. 8; Sec. V-C): IMU
// preintegration between consecutive keyframes, the inertial residual with
// first-order bias correction, and rectified stereo reprojection.  Residuals
// are written once over a generic scalar; their Jacobians come from forward-
// mode automatic differentiation (Sec. IV-C), one lane per (factor, column)
// with the column's local perturbation seeded.  Keyframe state: rotation
// R (world <- body, passed as an angle-axis vector), position p, velocity v,
// gyroscope bias b_g, accelerometer bias b_a; Jacobian columns are the right
// perturbation R Exp(dtheta) and additive p, v, b.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <vector>

#include "gba.h"
#include "gba_autodiff.h"
#include "gba_device.h"

namespace gba {
namespace vi {

constexpr double kSmall = 1e-8;   // |phi|^2 below which Exp / Log use their series
constexpr double kGravity[3] = {0.0, 0.0, -9.81};

// layout of one preintegrated interval (doubles)
enum {
    kDt = 0, kDR = 1, kDV = 10, kDP = 13, kJRg = 16, kJvg = 25, kJva = 34, kJpg = 43, kJpa = 52,
    kBg0 = 61, kBa0 = 64, kCov = 67, kPreStride = 148
};

template <typename S>
__device__ __forceinline__ void skew(const S (&v)[3], S (&K)[3][3]) {
    const S z = v[0] * 0.0;
    K[0][0] = z;     K[0][1] = -v[2]; K[0][2] = v[1];
    K[1][0] = v[2];  K[1][1] = z;     K[1][2] = -v[0];
    K[2][0] = -v[1]; K[2][1] = v[0];  K[2][2] = z;
}

template <typename A, typename B, typename C>
__device__ __forceinline__ void mm(const A (&a)[3][3], const B (&b)[3][3], C (&c)[3][3]) {
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) c[r][k] = a[r][0] * b[0][k] + a[r][1] * b[1][k] + a[r][2] * b[2][k];
}

template <typename A, typename B, typename C>
__device__ __forceinline__ void mtm(const A (&a)[3][3], const B (&b)[3][3], C (&c)[3][3]) {
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int k = 0; k < 3; ++k) c[r][k] = a[0][r] * b[0][k] + a[1][r] * b[1][k] + a[2][r] * b[2][k];
}

// Exp of a 3-vector: I + a K + b K^2, a = sin t / t, b = (1 - cos t) / t^2
// (series below |phi|^2 = kSmall); generic over double and Dual<double>.
template <typename S>
__device__ __forceinline__ void so3_exp(const S (&phi)[3], S (&R)[3][3]) {
    const S t2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
    S a, b;
    if (ad_value(t2) < kSmall) {
        a = 1.0 - t2 / 6.0;
        b = 0.5 - t2 / 24.0;
    } else {
        const S t = ad_sqrt(t2);
        a = ad_sin(t) / t;
        b = (1.0 - ad_cos(t)) / t2;
    }
    S K[3][3], K2[3][3];
    skew(phi, K);
    mm(K, K, K2);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) R[r][c] = a * K[r][c] + b * K2[r][c] + (r == c ? 1.0 : 0.0);
}

// Log of a rotation matrix: theta = atan2(|v|, (tr R - 1) / 2) with v the
// axial part; theta / sin theta by its series below |v|^2 = kSmall.
template <typename S>
__device__ __forceinline__ void so3_log(const S (&R)[3][3], S (&phi)[3]) {
    const S c = 0.5 * (R[0][0] + R[1][1] + R[2][2] - 1.0);
    const S v[3] = {0.5 * (R[2][1] - R[1][2]), 0.5 * (R[0][2] - R[2][0]), 0.5 * (R[1][0] - R[0][1])};
    const S s2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    S f;
    if (ad_value(s2) < kSmall) {
        f = 1.0 + s2 / 6.0 + 0.075 * s2 * s2;
    } else {
        const S s = ad_sqrt(s2);
        f = ad_atan2(s, c) / s;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) phi[k] = v[k] * f;
}

__device__ inline void right_jacobian(const double (&phi)[3], double (&J)[3][3]) {
    const double t2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2];
    double a, b;
    if (t2 < kSmall) {
        a = 0.5;
        b = 1.0 / 6.0;
    } else {
        const double t = sqrt(t2);
        a = (1.0 - cos(t)) / t2;
        b = (t - sin(t)) / (t2 * t);
    }
    double K[3][3], K2[3][3];
    skew(phi, K);
    mm(K, K, K2);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) J[r][c] = (r == c ? 1.0 : 0.0) - a * K[r][c] + b * K2[r][c];
}

// ---------------------------------------------------------- preintegration
// One lane per interval: the samples [off[f], off[f+1]) with the interval's
// bias estimates; deltas, bias Jacobians and the covariance (continuous noise
// densities sg, sa) are propagated with the values before each step.
__global__ __launch_bounds__(64) void k_preintegrate(int n, const long long* __restrict__ off,
                                                    const double* __restrict__ gyro,
                                                    const double* __restrict__ acc, double dt,
                                                    const double* __restrict__ bias0, double sg,
                                                    double sa, double* __restrict__ out) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n) return;
    double dR[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}}, dv[3] = {0, 0, 0}, dp[3] = {0, 0, 0};
    double JRg[3][3] = {}, Jvg[3][3] = {}, Jva[3][3] = {}, Jpg[3][3] = {}, Jpa[3][3] = {};
    double cov[9][9] = {};
    const double qg = sg * sg / dt, qa = sa * sa / dt;
    const double* b0 = bias0 + 6 * f;
    for (long long s = off[f]; s < off[f + 1]; ++s) {
        double w[3], a[3];
        for (int k = 0; k < 3; ++k) {
            w[k] = (gyro[3 * s + k] - b0[k]) * dt;
            a[k] = acc[3 * s + k] - b0[3 + k];
        }
        double Ra[3], ax[3][3], Rax[3][3], dRk[3][3], Jrk[3][3];
        for (int r = 0; r < 3; ++r) Ra[r] = dR[r][0] * a[0] + dR[r][1] * a[1] + dR[r][2] * a[2];
        skew(a, ax);
        mm(dR, ax, Rax);
        so3_exp(w, dRk);
        right_jacobian(w, Jrk);
        // covariance: A cov A^T + B_g qg B_g^T + B_a qa B_a^T over [dphi, dv, dp]
        double A[9][9] = {};
        for (int k = 0; k < 9; ++k) A[k][k] = 1.0;
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                A[r][c] = dRk[c][r];
                A[3 + r][c] = -Rax[r][c] * dt;
                A[6 + r][c] = -0.5 * Rax[r][c] * dt * dt;
            }
        for (int r = 0; r < 3; ++r) A[6 + r][3 + r] = dt;
        double AC[9][9];
        for (int r = 0; r < 9; ++r)
            for (int c = 0; c < 9; ++c) {
                double t = 0.0;
                for (int k = 0; k < 9; ++k) t += A[r][k] * cov[k][c];
                AC[r][c] = t;
            }
        double Bg[9][3] = {}, Ba[9][3] = {};
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                Bg[r][c] = Jrk[r][c] * dt;
                Ba[3 + r][c] = dR[r][c] * dt;
                Ba[6 + r][c] = 0.5 * dR[r][c] * dt * dt;
            }
        for (int r = 0; r < 9; ++r)
            for (int c = 0; c < 9; ++c) {
                double t = 0.0, ng = 0.0, na = 0.0;
                for (int k = 0; k < 9; ++k) t += AC[r][k] * A[c][k];
                for (int k = 0; k < 3; ++k) {
                    ng += Bg[r][k] * Bg[c][k];
                    na += Ba[r][k] * Ba[c][k];
                }
                cov[r][c] = t + qg * ng + qa * na;
            }
        // bias Jacobians: position, velocity, then rotation
        double RaxJ[3][3];
        mm(Rax, JRg, RaxJ);
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                Jpa[r][c] = Jpa[r][c] + Jva[r][c] * dt - 0.5 * dR[r][c] * dt * dt;
                Jpg[r][c] = Jpg[r][c] + Jvg[r][c] * dt - 0.5 * RaxJ[r][c] * dt * dt;
                Jva[r][c] = Jva[r][c] - dR[r][c] * dt;
                Jvg[r][c] = Jvg[r][c] - RaxJ[r][c] * dt;
            }
        double JR2[3][3];
        mtm(dRk, JRg, JR2);
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) JRg[r][c] = JR2[r][c] - Jrk[r][c] * dt;
        // deltas
        for (int r = 0; r < 3; ++r) {
            dp[r] = dp[r] + dv[r] * dt + 0.5 * Ra[r] * dt * dt;
            dv[r] = dv[r] + Ra[r] * dt;
        }
        double R2[3][3];
        mm(dR, dRk, R2);
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) dR[r][c] = R2[r][c];
    }
    double* o = out + (size_t)kPreStride * f;
    o[kDt] = dt * (double)(off[f + 1] - off[f]);
    for (int r = 0; r < 3; ++r) {
        o[kDV + r] = dv[r];
        o[kDP + r] = dp[r];
        o[kBg0 + r] = b0[r];
        o[kBa0 + r] = b0[3 + r];
        for (int c = 0; c < 3; ++c) {
            o[kDR + 3 * r + c] = dR[r][c];
            o[kJRg + 3 * r + c] = JRg[r][c];
            o[kJvg + 3 * r + c] = Jvg[r][c];
            o[kJva + 3 * r + c] = Jva[r][c];
            o[kJpg + 3 * r + c] = Jpg[r][c];
            o[kJpa + 3 * r + c] = Jpa[r][c];
        }
    }
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c) o[kCov + 9 * r + c] = 0.5 * (cov[r][c] + cov[c][r]);
}

// ------------------------------------------------------------ residuals
// r = (Log((dR Exp(JRg dbg))^T Ri^T Rj),
//      Ri^T (vj - vi - g dt) - (dv + Jvg dbg + Jva dba),
//      Ri^T (pj - pi - vi dt - 1/2 g dt^2) - (dp + Jpg dbg + Jpa dba))
template <typename S>
__device__ __forceinline__ void inertial_residual(const S (&Ri)[3][3], const S (&pi)[3],
                                                  const S (&vi)[3], const S (&bgi)[3],
                                                  const S (&bai)[3], const S (&Rj)[3][3],
                                                  const S (&pj)[3], const S (&vj)[3],
                                                  const double* __restrict__ pre, S (&r)[9]) {
    const double dt = pre[kDt];
    S dbg[3], dba[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        dbg[k] = bgi[k] - pre[kBg0 + k];
        dba[k] = bai[k] - pre[kBa0 + k];
    }
    S corr[3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
        corr[k] = pre[kJRg + 3 * k] * dbg[0] + pre[kJRg + 3 * k + 1] * dbg[1] + pre[kJRg + 3 * k + 2] * dbg[2];
    S Ec[3][3], dRc[3][3], RiRj[3][3], E[3][3];
    so3_exp(corr, Ec);
    double dR[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) dR[a][b] = pre[kDR + 3 * a + b];
    mm(dR, Ec, dRc);
    mtm(Ri, Rj, RiRj);
    mtm(dRc, RiRj, E);
    S rR[3];
    so3_log(E, rR);
    S wv[3], wp[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        wv[k] = vj[k] - vi[k] - kGravity[k] * dt;
        wp[k] = pj[k] - pi[k] - vi[k] * dt - 0.5 * kGravity[k] * dt * dt;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        r[k] = rR[k];
        const S dvc = pre[kDV + k] + (pre[kJvg + 3 * k] * dbg[0] + pre[kJvg + 3 * k + 1] * dbg[1] +
                                      pre[kJvg + 3 * k + 2] * dbg[2]) +
                      (pre[kJva + 3 * k] * dba[0] + pre[kJva + 3 * k + 1] * dba[1] + pre[kJva + 3 * k + 2] * dba[2]);
        const S dpc = pre[kDP + k] + (pre[kJpg + 3 * k] * dbg[0] + pre[kJpg + 3 * k + 1] * dbg[1] +
                                      pre[kJpg + 3 * k + 2] * dbg[2]) +
                      (pre[kJpa + 3 * k] * dba[0] + pre[kJpa + 3 * k + 1] * dba[1] + pre[kJpa + 3 * k + 2] * dba[2]);
        r[3 + k] = Ri[0][k] * wv[0] + Ri[1][k] * wv[1] + Ri[2][k] * wv[2] - dvc;
        r[6 + k] = Ri[0][k] * wp[0] + Ri[1][k] * wp[1] + Ri[2][k] * wp[2] - dpc;
    }
}

// R (I + [d]x): the right perturbation R Exp(d) to first order at d = 0
template <typename S>
__device__ __forceinline__ void perturb_rot(const double (&R)[3][3], const S (&d)[3], S (&Rp)[3][3]) {
    S K[3][3];
    skew(d, K);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            Rp[r][c] = R[r][0] * K[0][c] + R[r][1] * K[1][c] + R[r][2] * K[2][c] + R[r][c];
}

__device__ __forceinline__ void state_rotation(const double* __restrict__ s, double (&R)[3][3]) {
    const double w[3] = {s[0], s[1], s[2]};
    so3_exp(w, R);
}

// One lane per (factor, column): factor f joins keyframes f and f + 1;
// columns dtheta_i, dp_i, dv_i, dbg_i, dba_i, dtheta_j, dp_j, dv_j (3 each).
__global__ __launch_bounds__(256) void k_inertial_eval(int n, const double* __restrict__ st,
                                                       const double* __restrict__ pre,
                                                       double* __restrict__ r_out,
                                                       double* __restrict__ j_out) {
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= 24LL * n) return;
    const int f = (int)(t / 24), col = (int)(t % 24);
    using S = Dual<double>;
    const double* si = st + 15 * (size_t)f;
    const double* sj = st + 15 * (size_t)(f + 1);
    double Ri0[3][3], Rj0[3][3];
    state_rotation(si, Ri0);
    state_rotation(sj, Rj0);
    S z[24];
#pragma unroll
    for (int k = 0; k < 24; ++k) z[k] = {0.0, k == col ? 1.0 : 0.0};
    S di[3] = {z[0], z[1], z[2]}, dj[3] = {z[15], z[16], z[17]};
    S Ri[3][3], Rj[3][3];
    perturb_rot(Ri0, di, Ri);
    perturb_rot(Rj0, dj, Rj);
    S pi[3], vi[3], bg[3], ba[3], pj[3], vj[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        pi[k] = si[3 + k] + z[3 + k];
        vi[k] = si[6 + k] + z[6 + k];
        bg[k] = si[9 + k] + z[9 + k];
        ba[k] = si[12 + k] + z[12 + k];
        pj[k] = sj[3 + k] + z[18 + k];
        vj[k] = sj[6 + k] + z[21 + k];
    }
    S r[9];
    inertial_residual(Ri, pi, vi, bg, ba, Rj, pj, vj, pre + (size_t)kPreStride * f, r);
#pragma unroll
    for (int k = 0; k < 9; ++k) j_out[(size_t)216 * f + 24 * k + col] = r[k].d;
    if (col == 0)
#pragma unroll
        for (int k = 0; k < 9; ++k) r_out[9 * (size_t)f + k] = r[k].v;
}

// One lane per (observation, column): columns dtheta, dp of the keyframe and
// dX of the point.  Xc = R^T (X - p); u_l = fx Xc_x / Xc_z + cx,
// v_l = fy Xc_y / Xc_z + cy, u_r = u_l - fx b / Xc_z; minus the observation.
__global__ __launch_bounds__(256) void k_stereo_eval(long long n, const double* __restrict__ st,
                                                     const double* __restrict__ pts,
                                                     const long long* __restrict__ kf,
                                                     const long long* __restrict__ pt,
                                                     const double* __restrict__ obs, double fx,
                                                     double fy, double cx, double cy, double base,
                                                     double* __restrict__ r_out,
                                                     double* __restrict__ j_out) {
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= 9LL * n) return;
    const long long e = t / 9;
    const int col = (int)(t % 9);
    using S = Dual<double>;
    const double* s = st + 15 * (size_t)kf[e];
    const double* X = pts + 3 * (size_t)pt[e];
    double R0[3][3];
    state_rotation(s, R0);
    S d[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = {0.0, k == col ? 1.0 : 0.0};
    S R[3][3];
    perturb_rot(R0, d, R);
    S q[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const S pk = S{s[3 + k], 3 + k == col ? 1.0 : 0.0};
        const S xk = S{X[k], 6 + k == col ? 1.0 : 0.0};
        q[k] = xk - pk;
    }
    S Xc[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) Xc[k] = R[0][k] * q[0] + R[1][k] * q[1] + R[2][k] * q[2];
    const S inv = 1.0 / Xc[2];
    const S ul = fx * Xc[0] * inv + cx;
    const S vl = fy * Xc[1] * inv + cy;
    const S ur = ul - fx * base * inv;
    const S r[3] = {ul - obs[3 * e], vl - obs[3 * e + 1], ur - obs[3 * e + 2]};
#pragma unroll
    for (int k = 0; k < 3; ++k) j_out[(size_t)27 * e + 9 * k + col] = r[k].d;
    if (col == 0)
#pragma unroll
        for (int k = 0; k < 3; ++k) r_out[3 * (size_t)e + k] = r[k].v;
}

// block-wide sum of a double over a 256-thread workgroup (lane 0 of the
// first wavefront holds the result)
__device__ __forceinline__ double block_sum_vi(double v, double* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x == 0)
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += red[k];
    return s;
}

// ==========================================================================
// The visual-inertial LM solve (Background Eq. 8; Sec. V-C), FP64
// arithmetic, in two forms of the damped step: the points eliminated (Eq.
// 5-6 on the keyframe / point partition) and PCG on the keyframe Schur
// complement, or the paper's form for its VI runs, PCG on the whole damped
// system over keyframe states and points; block-Jacobi preconditioned
// (15 x 15 keyframe blocks; 3 x 3 point blocks in the whole-system form).
// Unknowns per keyframe: dtheta, dp, dv, dbg, dba (the rotation updated on
// the right); per point: dX.  The first keyframe is held fixed (its columns
// are zero).  Terms:
//   stereo   1/2 rho(|r|^2 / sigma^2), Huber on the squared norm, IRLS
//            whitening sqrt(w) / sigma;
//   inertial 1/2 r^T Omega r, Omega the inverse preintegrated covariance;
//   bias     1/2 r^T Omega_b r, r = b_j - b_i, Omega_b from the random-walk
//            densities and the interval length.
// ==========================================================================
constexpr int kSt = 21;   // device keyframe state: R (row-major), p, v, bg, ba

struct VIDev {
    int K;                 // keyframes
    long long N, M;        // points, stereo observations
    double* st;            // [K kSt] current
    double* st_c;          // [K kSt] candidate
    double* X;             // [3 N]
    double* X_c;
    const int* kf;         // [M]
    const int* pt;
    const double* obs;     // [3 M]
    const double* pre;     // [kPreStride (K - 1)]
    double* info;          // [81 (K - 1)] Omega of the inertial terms
    void* jsp;             // whole-system form: whitened stereo J (dtheta, dp | dX), padded
                           // point-order tiles (js_at), double or float when w32; null in
                           // the Schur form
    double* ji;            // [216 (K - 1)] inertial Jacobians
    double* ri;            // [9 (K - 1)]
    double* b;             // [n] gradient J^T Omega r
    double* hk;            // [225 K] keyframe diagonal blocks
    double* hp;            // [9 N] point diagonal blocks
    double* dg;            // [n] clipped diagonal (damping)
    double* mki;           // [225 K] inverses of the damped keyframe blocks (of S in the Schur form)
    double* mp;            // [9 N] inverses of the damped point blocks
    double* scal;          // [8 + kPcgScalars] reductions
    // Schur form (null in the whole-system form): W_e = J_k^T J_p (6 x 3)
    // per observation, in keyframe order (wk) and in padded point order
    // (wp), each in tiles of 64 observations x 18 entries in 16-byte lane
    // groups (w_at)
    void* wk;              // double, or float when w32
    void* wp;
    int w32;
    const int* qkf;        // [Mp] keyframe of the i-th observation in padded point order
    const int* qpt;        // [Mp] its point, -1 in a pad slot
    const double* qobs;    // [3 Mp] the observed pixels in point order
    long long Mp;          // padded point-order length (a multiple of 64)
    const int* longp;      // [nlong] the points with more than 64 observations
    int nlong;
    double* tb;            // [3 N] their partial sums (zero between passes)
    const int* lslot;      // [nlslot] the point-order slots of their observations
    long long nlslot;
    double* sm;            // [36 K] sum over a keyframe's observations of W C^-1 W^T
    double* icx;           // [135 (K - 1)] inertial cross blocks J_i^T Omega J_j (15 x 9)
    double fx, fy, cx, cy, base, inv_sigma, delta2, wg, wa;   // wg, wa: 1 / sigma_w^2
    long long n() const { return 15LL * K + 3 * N; }
};

// PCG scalars on the device: three slots of dot accumulators {p.q parts,
// r.r, r.z, ...}, used round robin (step s accumulates into slot s % 3,
// takes the previous step's values from slot (s + 2) % 3 and clears slot
// (s + 1) % 3 for the next step, so no kernel reads a value another
// workgroup of it resets), then the stop threshold, the stop flag, the step
// count and the squared rejection ratio
// p.q is summed in kPqParts parts (a workgroup adds to part blockIdx %
// kPqParts: thousands of workgroups adding to one address serialise)
constexpr int kPqParts = 256;
// per slot also: the least r.r so far (the rejection test), a breakdown flag
// set by the update kernel and the stop decision of the direction kernel
enum { kAccPq = 0, kAccRr = kPqParts, kAccRz, kAccMin, kAccBreak, kAccStop, kAccRrP,
       kAccRzP = kAccRrP + kPqParts, kAccN = kAccRzP + kPqParts };
constexpr int kSlots = 3;
enum { kThr = kSlots * kAccN, kDone, kSteps, kRatio2, kPcgScalars };
// the cost, |x| and model-decrease sums: kRedSlots sums of kPqParts parts
// each, after the PCG scalars (scal = 8 unused, the PCG scalars, the parts)
constexpr int kRedSlots = 8;
constexpr long long kRedOff = 8 + kPcgScalars;
constexpr long long kScalN = kRedOff + (long long)kRedSlots * kPqParts;

__device__ __forceinline__ bool pcg_done(const double* ps) { return ps && ps[kDone] != 0.0; }

// the keyframe window of the LDS partials of the point-order products, and
// their workgroup size
constexpr int kKfWin = 64;
constexpr int kFuseBlock = 512;

// W tiles: 64 observations x 18 entries, in 16-byte groups so that a lane
// loads its entries as float4 / double2 and one load instruction of a
// wavefront reads 1 KiB contiguous: group g (V = 16 / sizeof(WT) entries,
// the last one of FP32 two wide) of lane l at tile + 64 V g + width l
template <typename WT>
__device__ __forceinline__ size_t w_at(long long e, int c) {
    constexpr int V = 16 / (int)sizeof(WT);
    const int g = c / V;
    const int width = (18 - g * V) < V ? (18 - g * V) : V;
    return (size_t)(e >> 6) * (18 * 64) + (size_t)g * V * 64 + (size_t)(e & 63) * width + (c - g * V);
}

template <typename WT>
__device__ __forceinline__ void load_w(const void* w, long long e, double (&out)[18]);

template <>
__device__ __forceinline__ void load_w<float>(const void* w, long long e, double (&out)[18]) {
    const float* t = (const float*)w + (size_t)(e >> 6) * (18 * 64);
    const int l = (int)(e & 63);
    for (int g = 0; g < 4; ++g) {
        const float4 v = ((const float4*)t)[g * 64 + l];
        out[4 * g] = v.x;
        out[4 * g + 1] = v.y;
        out[4 * g + 2] = v.z;
        out[4 * g + 3] = v.w;
    }
    const float2 v = ((const float2*)(t + 1024))[l];
    out[16] = v.x;
    out[17] = v.y;
}

template <>
__device__ __forceinline__ void load_w<double>(const void* w, long long e, double (&out)[18]) {
    const double* t = (const double*)w + (size_t)(e >> 6) * (18 * 64);
    const int l = (int)(e & 63);
    for (int g = 0; g < 9; ++g) {
        const double2 v = ((const double2*)t)[g * 64 + l];
        out[2 * g] = v.x;
        out[2 * g + 1] = v.y;
    }
}

__device__ __forceinline__ void atomic_add(double* a, double v) { unsafeAtomicAdd(a, v); }

__global__ void k_vi_states_in(int K, const double* __restrict__ s15, double* __restrict__ s21) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    const double w[3] = {s15[15 * k], s15[15 * k + 1], s15[15 * k + 2]};
    double R[3][3];
    so3_exp(w, R);
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) s21[kSt * k + 3 * r + c] = R[r][c];
    for (int j = 0; j < 12; ++j) s21[kSt * k + 9 + j] = s15[15 * k + 3 + j];
}

__global__ void k_vi_states_out(int K, const double* __restrict__ s21, double* __restrict__ s15) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= K) return;
    double R[3][3], w[3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) R[r][c] = s21[kSt * k + 3 * r + c];
    so3_log(R, w);
    for (int j = 0; j < 3; ++j) s15[15 * k + j] = w[j];
    for (int j = 0; j < 12; ++j) s15[15 * k + 3 + j] = s21[kSt * k + 9 + j];
}

// Omega = cov^-1 per interval by Cholesky (cov = L L^T): Omega = L^-T L^-1.
__global__ void k_vi_info(int n, const double* __restrict__ pre, double* __restrict__ info) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= n) return;
    const double* C = pre + (size_t)kPreStride * f + kCov;
    double L[9][9] = {};
    for (int j = 0; j < 9; ++j) {
        double d = C[9 * j + j];
        for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
        L[j][j] = sqrt(d);
        for (int i = j + 1; i < 9; ++i) {
            double t = C[9 * i + j];
            for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
            L[i][j] = t / L[j][j];
        }
    }
    double Li[9][9] = {};   // L^-1 (lower)
    for (int c = 0; c < 9; ++c) {
        for (int r = c; r < 9; ++r) {
            double t = r == c ? 1.0 : 0.0;
            for (int k = c; k < r; ++k) t -= L[r][k] * Li[k][c];
            Li[r][c] = t / L[r][r];
        }
    }
    double* O = info + 81 * (size_t)f;
    for (int r = 0; r < 9; ++r)
        for (int c = 0; c < 9; ++c) {
            double t = 0.0;
            for (int k = (r > c ? r : c); k < 9; ++k) t += Li[k][r] * Li[k][c];
            O[9 * r + c] = t;
        }
}

// Stereo projection of observation e at (R, p) and X: Xc, the prediction and
// (with kJac) the 3 x 9 Jacobian over dtheta, dp, dX.
template <bool kJac>
__device__ __forceinline__ void vi_stereo(const VIDev& d, const double* __restrict__ s,
                                          const double* __restrict__ X, long long e, double (&r)[3],
                                          double (&J)[3][9]) {
    double q[3], Xc[3];
    for (int k = 0; k < 3; ++k) q[k] = X[k] - s[9 + k];
    for (int k = 0; k < 3; ++k) Xc[k] = s[k] * q[0] + s[3 + k] * q[1] + s[6 + k] * q[2];
    const double iz = 1.0 / Xc[2];
    const double ul = d.fx * Xc[0] * iz + d.cx;
    r[0] = ul - d.obs[3 * e];
    r[1] = d.fy * Xc[1] * iz + d.cy - d.obs[3 * e + 1];
    r[2] = ul - d.fx * d.base * iz - d.obs[3 * e + 2];
    if (!kJac) return;
    double P[3][3] = {{d.fx * iz, 0.0, -d.fx * Xc[0] * iz * iz},
                      {0.0, d.fy * iz, -d.fy * Xc[1] * iz * iz},
                      {d.fx * iz, 0.0, -d.fx * (Xc[0] - d.base) * iz * iz}};
    const double Kx[3][3] = {{0.0, -Xc[2], Xc[1]}, {Xc[2], 0.0, -Xc[0]}, {-Xc[1], Xc[0], 0.0}};
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) {
            J[a][c] = P[a][0] * Kx[0][c] + P[a][1] * Kx[1][c] + P[a][2] * Kx[2][c];
            // P R^T: (R^T)[k][c] = R[c][k]
            const double PRt = P[a][0] * s[3 * c] + P[a][1] * s[3 * c + 1] + P[a][2] * s[3 * c + 2];
            J[a][3 + c] = -PRt;
            J[a][6 + c] = PRt;
        }
}

__device__ __forceinline__ void vi_huber(double s, double delta2, double& rho, double& w) {
    if (delta2 > 0.0 && s > delta2) {
        const double q = sqrt(s);
        rho = 2.0 * sqrt(delta2) * q - delta2;
        w = sqrt(delta2) / q;
    } else {
        rho = s;
        w = 1.0;
    }
}

// whitened residual and Jacobian of observation (k, j) with the observed
// pixels ob (zero when !valid; the first keyframe's columns zero)
__device__ __forceinline__ void vi_stereo_whitened(const VIDev& d, const double* __restrict__ ob, int k, int j,
                                                   bool valid, double (&r)[3], double (&J)[3][9]) {
    VIDev dd = d;
    dd.obs = ob;
    vi_stereo<true>(dd, d.st + (size_t)kSt * k, d.X + 3 * (size_t)j, 0, r, J);
    const double s = (r[0] * r[0] + r[1] * r[1] + r[2] * r[2]) * d.inv_sigma * d.inv_sigma;
    double rho, w;
    vi_huber(s, d.delta2, rho, w);
    const double sc = valid ? sqrt(w) * d.inv_sigma : 0.0;
    for (int a = 0; a < 3; ++a) {
        r[a] *= sc;
        for (int c = 0; c < 9; ++c) J[a][c] = (k == 0 && c < 6) ? 0.0 : J[a][c] * sc;
    }
}

// linearisation of the stereo terms in keyframe order: the keyframe's
// gradient and 6 x 6 block terms summed across its run of the wavefront
// (SegScan) and added once per run; in the Schur form W = J_k^T J_p is
// stored (keyframe-order tiles).  The point terms come from the point-order
// pass below.
__global__ void k_vi_lin_stereo(VIDev d) {
    const long long e0 = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const bool valid = e0 < d.M;
    const long long e = valid ? e0 : d.M - 1;
    const int k = d.kf[e], j = d.pt[e];
    const int l = (int)(threadIdx.x & 63);
    const int kprev = __shfl_up(k, 1, 64);
    const bool start = !valid || l == 0 || kprev != k;
    const SegScan seg(start);
    int head, end;
    segment_of(__ballot(start), l, head, end);
    double r[3], J[3][9];
    vi_stereo_whitened(d, d.obs + 3 * e, k, j, valid, r, J);
    if (valid && d.wk)
        for (int a = 0; a < 6; ++a)
            for (int c = 0; c < 3; ++c) {
                const double w = J[0][a] * J[0][6 + c] + J[1][a] * J[1][6 + c] + J[2][a] * J[2][6 + c];
                if (d.w32) ((float*)d.wk)[w_at<float>(e, 3 * a + c)] = (float)w;
                else ((double*)d.wk)[w_at<double>(e, 3 * a + c)] = w;
            }
    const bool last = valid && l == end;
    double* bk = d.b + 15 * (size_t)k;
    for (int c = 0; c < 6; ++c) {
        const double sg = seg.sum(J[0][c] * r[0] + J[1][c] * r[1] + J[2][c] * r[2]);
        if (last) atomic_add(bk + c, sg);
    }
    for (int a = 0; a < 6; ++a)
        for (int c = 0; c < 6; ++c) {
            const double h = seg.sum(J[0][a] * J[0][c] + J[1][a] * J[1][c] + J[2][a] * J[2][c]);
            if (last && k != 0) atomic_add(d.hk + 225 * (size_t)k + 15 * a + c, h);
        }
}

// whitened J (3 x 9) of the whole-system form in padded point-order tiles:
// entry c of slot i at (27 tile + c) 64 + lane
__device__ __forceinline__ size_t js_at(long long i, int c) {
    return ((size_t)(i >> 6) * 27 + c) * 64 + (size_t)(i & 63);
}

// the same terms in point order: W (Schur form) or the whitened J
// (whole-system form) stored in point-order tiles,
// the point's gradient b_p and block H_pp summed across its run of the
// wavefront; a point whose observations all sit in one wavefront is stored,
// one split across wavefronts is added in parts (b and hp are zero before)
template <typename WT>
__global__ void k_vi_lin_stereo_pts(VIDev d) {
    const long long i0 = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long i = i0 < d.Mp ? i0 : d.Mp - 1;
    const int jq = d.qpt[i];
    const bool valid = i0 < d.Mp && jq >= 0;
    const int j = valid ? jq : 0, k = valid ? d.qkf[i] : 0;
    const int l = (int)(threadIdx.x & 63);
    const int jprev = __shfl_up(jq, 1, 64);
    const bool start = !valid || l == 0 || jprev != jq;
    const SegScan seg(start);
    int head, end;
    segment_of(__ballot(start), l, head, end);
    const bool first = i == 0 || d.qpt[i - 1] != jq;
    const bool lastp = i == d.Mp - 1 || d.qpt[i + 1] != jq;
    const bool whole = (__shfl(first ? 1 : 0, head, 64) != 0) && lastp;
    double r[3], J[3][9];
    vi_stereo_whitened(d, d.qobs + 3 * i, k, j, valid, r, J);
    if (valid && d.wp)
        for (int a = 0; a < 6; ++a)
            for (int c = 0; c < 3; ++c)
                ((WT*)d.wp)[w_at<WT>(i, 3 * a + c)] =
                    (WT)(J[0][a] * J[0][6 + c] + J[1][a] * J[1][6 + c] + J[2][a] * J[2][6 + c]);
    if (valid && d.jsp)
        for (int a = 0; a < 3; ++a)
            for (int c = 0; c < 9; ++c) ((WT*)d.jsp)[js_at(i, 9 * a + c)] = (WT)J[a][c];
    const bool out = valid && l == end;
    double* bp = d.b + 15 * (size_t)d.K + 3 * (size_t)j;
    for (int c = 0; c < 3; ++c) {
        const double g = seg.sum(J[0][6 + c] * r[0] + J[1][6 + c] * r[1] + J[2][6 + c] * r[2]);
        if (out) {
            if (whole) bp[c] = g;
            else atomic_add(bp + c, g);
        }
    }
    double* hp = d.hp + 9 * (size_t)j;
    for (int a = 0; a < 3; ++a)
        for (int c = 0; c < 3; ++c) {
            const double h = seg.sum(J[0][6 + a] * J[0][6 + c] + J[1][6 + a] * J[1][6 + c] +
                                     J[2][6 + a] * J[2][6 + c]);
            if (out) {
                if (whole) hp[3 * a + c] = h;
                else atomic_add(hp + 3 * a + c, h);
            }
        }
}

// inertial Jacobians by forward-mode AD, one lane per (term, column), at the
// device states (rotation matrices); columns of a fixed first keyframe zero
__global__ __launch_bounds__(256) void k_vi_lin_inertial(VIDev d) {
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const int n = d.K - 1;
    if (t >= 24LL * n) return;
    const int f = (int)(t / 24), col = (int)(t % 24);
    using S = Dual<double>;
    const double* si = d.st + (size_t)kSt * f;
    const double* sj = d.st + (size_t)kSt * (f + 1);
    double Ri0[3][3], Rj0[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            Ri0[r][c] = si[3 * r + c];
            Rj0[r][c] = sj[3 * r + c];
        }
    S z[24];
    for (int k = 0; k < 24; ++k) z[k] = {0.0, k == col ? 1.0 : 0.0};
    S di[3] = {z[0], z[1], z[2]}, dj[3] = {z[15], z[16], z[17]};
    S Ri[3][3], Rj[3][3];
    perturb_rot(Ri0, di, Ri);
    perturb_rot(Rj0, dj, Rj);
    S pi[3], vi_[3], bg[3], ba[3], pj[3], vj[3];
    for (int k = 0; k < 3; ++k) {
        pi[k] = si[9 + k] + z[3 + k];
        vi_[k] = si[12 + k] + z[6 + k];
        bg[k] = si[15 + k] + z[9 + k];
        ba[k] = si[18 + k] + z[12 + k];
        pj[k] = sj[9 + k] + z[18 + k];
        vj[k] = sj[12 + k] + z[21 + k];
    }
    S r[9];
    inertial_residual(Ri, pi, vi_, bg, ba, Rj, pj, vj, d.pre + (size_t)kPreStride * f, r);
    const bool zero = f == 0 && col < 15;
    for (int k = 0; k < 9; ++k) d.ji[(size_t)216 * f + 24 * k + col] = zero ? 0.0 : r[k].d;
    if (col == 0)
        for (int k = 0; k < 9; ++k) d.ri[9 * (size_t)f + k] = r[k].v;
}

// inertial and bias terms: gradient and diagonal blocks, one wavefront per
// term, lane c < 24 for column c (keyframe i's 15, then keyframe j's first 9)
__global__ __launch_bounds__(256) void k_vi_acc_inertial(VIDev d) {
    const int f = (int)((blockIdx.x * (long long)blockDim.x + threadIdx.x) >> 6);
    const int l = (int)(threadIdx.x & 63);
    if (f >= d.K - 1) return;   // whole wavefronts
    const double* J = d.ji + (size_t)216 * f;
    const double* O = d.info + 81 * (size_t)f;
    const double* r = d.ri + 9 * (size_t)f;
    double* bi = d.b + 15 * (size_t)f;
    double* bj = d.b + 15 * (size_t)(f + 1);
    double* hi = d.hk + 225 * (size_t)f;
    double* hj = d.hk + 225 * (size_t)(f + 1);
    if (l < 24) {
        double Or[9], OJ[9];   // Omega r, and column l of Omega J
        for (int a = 0; a < 9; ++a) {
            double t = 0.0, u = 0.0;
            for (int c = 0; c < 9; ++c) {
                t += O[9 * a + c] * r[c];
                u += O[9 * a + c] * J[24 * c + l];
            }
            Or[a] = t;
            OJ[a] = u;
        }
        double g = 0.0;
        for (int a = 0; a < 9; ++a) g += J[24 * a + l] * Or[a];
        atomic_add(l < 15 ? bi + l : bj + (l - 15), g);
        // column l of J^T Omega J within its keyframe's block
        const int c0 = l < 15 ? 0 : 15, c1 = l < 15 ? 15 : 24;
        for (int c = c0; c < c1; ++c) {
            double t = 0.0;
            for (int a = 0; a < 9; ++a) t += J[24 * a + c] * OJ[a];
            if (l < 15) atomic_add(hi + 15 * c + l, t);
            else atomic_add(hj + 15 * (c - 15) + (l - 15), t);
        }
    } else if (l < 30) {
        // bias random walk: r = b_j - b_i (6), Omega_b = diag(wg I3, wa I3) / dt
        const int k = l - 24;
        const double dt = d.pre[(size_t)kPreStride * f + kDt];
        const double* si = d.st + (size_t)kSt * f;
        const double* sj = d.st + (size_t)kSt * (f + 1);
        const double w = (k < 3 ? d.wg : d.wa) / dt;
        const double rb = sj[15 + k] - si[15 + k];
        atomic_add(bj + 9 + k, w * rb);
        atomic_add(hj + 15 * (9 + k) + 9 + k, w);
        if (f != 0) {
            atomic_add(bi + 9 + k, -w * rb);
            atomic_add(hi + 15 * (9 + k) + 9 + k, w);
        }
    }
}

// cost at (st, X): 1/2 sum rho over stereo, 1/2 r^T Omega r over inertial,
// 1/2 r^T Omega_b r over bias; into the parts of reduction slot `slot`
__global__ void k_vi_cost(VIDev d, const double* __restrict__ st, const double* __restrict__ X,
                          int slot) {
    __shared__ double red[16];
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    double c = 0.0;
    if (t < d.M) {
        double r[3], J[3][9];
        vi_stereo<false>(d, st + (size_t)kSt * d.kf[t], X + 3 * (size_t)d.pt[t], t, r, J);
        double rho, w;
        vi_huber((r[0] * r[0] + r[1] * r[1] + r[2] * r[2]) * d.inv_sigma * d.inv_sigma, d.delta2, rho, w);
        c = 0.5 * rho;
    } else if (t < d.M + d.K - 1) {
        const int f = (int)(t - d.M);
        const double* si = st + (size_t)kSt * f;
        const double* sj = st + (size_t)kSt * (f + 1);
        double Ri[3][3], Rj[3][3], pi[3], vi_[3], bg[3], ba[3], pj[3], vj[3];
        for (int a = 0; a < 3; ++a) {
            for (int b = 0; b < 3; ++b) {
                Ri[a][b] = si[3 * a + b];
                Rj[a][b] = sj[3 * a + b];
            }
            pi[a] = si[9 + a];
            vi_[a] = si[12 + a];
            bg[a] = si[15 + a];
            ba[a] = si[18 + a];
            pj[a] = sj[9 + a];
            vj[a] = sj[12 + a];
        }
        double r[9];
        inertial_residual(Ri, pi, vi_, bg, ba, Rj, pj, vj, d.pre + (size_t)kPreStride * f, r);
        const double* O = d.info + 81 * (size_t)f;
        for (int a = 0; a < 9; ++a)
            for (int b = 0; b < 9; ++b) c += 0.5 * r[a] * O[9 * a + b] * r[b];
        const double dt = d.pre[(size_t)kPreStride * f + kDt];
        for (int k = 0; k < 6; ++k) {
            const double rb = sj[15 + k] - si[15 + k];
            c += 0.5 * ((k < 3 ? d.wg : d.wa) / dt) * rb * rb;
        }
    }
    c = block_sum_vi(c, red);
    if (threadIdx.x == 0) atomic_add(d.scal + kRedOff + slot * kPqParts + blockIdx.x % kPqParts, c);
}

// the point blocks of the preconditioner (and, in the Schur form, C^-1):
// D = clip(diag H_pp), the damped 3 x 3 block inverted by cofactors; one
// lane per point
__global__ void k_vi_precond_pts(VIDev d, double lam, double lo, double hi) {
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t < d.N) {
        const long long j = t;
        const double* H = d.hp + 9 * j;
        double A[3][3];
        for (int a = 0; a < 3; ++a) {
            const double dd = fmin(fmax(H[4 * a], lo), hi);
            d.dg[15 * (size_t)d.K + 3 * j + a] = dd;
            for (int c = 0; c < 3; ++c) A[a][c] = H[3 * a + c] + (a == c ? lam * dd : 0.0);
        }
        const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
        const double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
        const double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
        const double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
        const double id = 1.0 / det;
        double* M = d.mp + 9 * j;
        M[0] = c00 * id;
        M[1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) * id;
        M[2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) * id;
        M[3] = c01 * id;
        M[4] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) * id;
        M[5] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) * id;
        M[6] = c02 * id;
        M[7] = (A[0][1] * A[2][0] - A[0][0] * A[2][1]) * id;
        M[8] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) * id;
    }
}

// the keyframe blocks of the preconditioner, one wavefront per keyframe:
// D = clip(diag H), A = H + lambda diag(D) (less sm in the Schur form),
// factored A = L L^T in LDS (right-looking, the trailing update spread over
// the lanes), then A^-1 column by column (lane c < 15 solves L L^T x = e_c)
__global__ __launch_bounds__(256) void k_vi_precond_kf(VIDev d, double lam, double lo, double hi) {
    __shared__ double La[4][225];
    const int w = (int)(threadIdx.x >> 6), l = (int)(threadIdx.x & 63);
    const long long k = blockIdx.x * 4LL + w;
    if (k >= d.K) return;   // whole wavefronts; no workgroup barrier below
    double* A = La[w];
    const double* H = d.hk + 225 * (size_t)k;
    for (int e = l; e < 225; e += 64) {
        const int a = e / 15, c = e % 15;
        double v = H[e];
        if (a == c) {
            const double dd = fmin(fmax(v, lo), hi);
            d.dg[15 * (size_t)k + a] = dd;
            v += lam * dd;
        }
        if (d.sm && a < 6 && c < 6) v -= d.sm[36 * (size_t)k + 6 * a + c];
        A[e] = v;
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    for (int j = 0; j < 15; ++j) {
        const double ljj = sqrt(fmax(A[16 * j], 1e-300));
        if (l > j && l < 15) A[15 * l + j] /= ljj;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (l == 0) A[16 * j] = ljj;
        // trailing update of the lower triangle: (a, c), j < c <= a < 15
        for (int e = l; e < 225; e += 64) {
            const int a = e / 15, c = e % 15;
            if (c > j && c <= a) A[e] -= A[15 * a + j] * A[15 * c + j];
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    }
    if (l < 15) {
        double y[15];
        for (int i = 0; i < 15; ++i) {
            double u = i == l ? 1.0 : 0.0;
            for (int q = 0; q < i; ++q) u -= A[15 * i + q] * y[q];
            y[i] = u / A[16 * i];
        }
        for (int i = 14; i >= 0; --i) {
            double u = y[i];
            for (int q = i + 1; q < 15; ++q) u -= A[15 * q + i] * y[q];
            y[i] = u / A[16 * i];
        }
        double* Mi = d.mki + 225 * (size_t)k;
        for (int i = 0; i < 15; ++i) Mi[15 * i + l] = y[i];
    }
}

// z = M^-1 r: one lane per keyframe row (the block inverse's row times the
// keyframe's residual), one per point
__global__ void k_vi_apply_m(VIDev d, const double* __restrict__ r, double* __restrict__ z,
                             const double* __restrict__ ps) {
    if (pcg_done(ps)) return;
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t < 15LL * d.K) {
        const long long k = t / 15;
        const int row = (int)(t % 15);
        const double* Mi = d.mki + 225 * (size_t)k + 15 * row;
        const double* rk = r + 15 * (size_t)k;
        double u = 0.0;
        for (int c = 0; c < 15; ++c) u += Mi[c] * rk[c];
        z[t] = u;
    } else if (t < 15LL * d.K + d.N) {
        const long long j = t - 15LL * d.K;
        const size_t o = 15 * (size_t)d.K + 3 * j;
        const double* M = d.mp + 9 * j;
        const double a = r[o], b = r[o + 1], c = r[o + 2];
        for (int i = 0; i < 3; ++i) z[o + i] = M[3 * i] * a + M[3 * i + 1] * b + M[3 * i + 2] * c;
    }
}

// q += (stereo part of H) v, whole-system form: one pass over the padded
// point-order J.  Per observation u = J_k v_k + J_p v_j; the point rows
// J_p^T u are summed across the point's run of the wavefront (added by its
// last lane: whole runs own the point's rows, parts of a point split across
// wavefronts add atomically), the keyframe rows J_k^T u go to the
// workgroup's LDS partials of its keyframe window (as in k_vi_schur_pts) and
// to q with one atomic add per entry.  q holds lambda D v on entry.
template <typename JT>
__global__ __launch_bounds__(512) void k_vi_prod_stereo(VIDev d, const double* __restrict__ v,
                                                       double* __restrict__ q, const double* __restrict__ ps) {
    if (pcg_done(ps)) return;
    __shared__ double part[kKfWin * 6];
    __shared__ int kmin_w[16];
    const long long i0 = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long i = i0 < d.Mp ? i0 : d.Mp - 1;
    const int jq = d.qpt[i];
    const bool valid = i0 < d.Mp && jq >= 0;
    const int j = valid ? jq : 0, k = valid ? d.qkf[i] : 0;
    const int l = (int)(threadIdx.x & 63);
    const int jprev = __shfl_up(jq, 1, 64);
    const bool start = !valid || l == 0 || jprev != jq;
    const SegScan seg(start);
    int head, end;
    segment_of(__ballot(start), l, head, end);
    const bool first = i == 0 || d.qpt[i - 1] != jq;
    const bool lastp = i == d.Mp - 1 || d.qpt[i + 1] != jq;
    const bool whole = (__shfl(first ? 1 : 0, head, 64) != 0) && lastp;   // at the run's last lane
    const size_t ok = 15 * (size_t)k, op = 15 * (size_t)d.K + 3 * (size_t)j;
    double in[9];
    for (int c = 0; c < 6; ++c) in[c] = v[ok + c];
    for (int c = 0; c < 3; ++c) in[6 + c] = v[op + c];
    double J[27];
    for (int c = 0; c < 27; ++c) J[c] = (double)((const JT*)d.jsp)[js_at(i, c)];
    double u[3];
    for (int a = 0; a < 3; ++a) {
        double t = 0.0;
        for (int c = 0; c < 9; ++c) t += J[9 * a + c] * in[c];
        u[a] = valid ? t : 0.0;
    }
    for (int c = 0; c < 3; ++c) {
        const double sy = seg.sum(J[6 + c] * u[0] + J[15 + c] * u[1] + J[24 + c] * u[2]);
        if (valid && l == end) {
            if (whole) q[op + c] += sy;
            else atomic_add(q + op + c, sy);
        }
    }
    int km = valid ? k : 0x7fffffff;
    for (int off = 32; off > 0; off >>= 1) km = min(km, __shfl_xor(km, off, 64));
    if (l == 0) kmin_w[threadIdx.x >> 6] = km;
    for (int e = threadIdx.x; e < kKfWin * 6; e += blockDim.x) part[e] = 0.0;
    __syncthreads();
    int kbase = 0x7fffffff;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) kbase = min(kbase, kmin_w[w]);
    if (valid && k != 0) {
        const int kk = k - kbase;
        for (int c = 0; c < 6; ++c) {
            const double y = J[c] * u[0] + J[9 + c] * u[1] + J[18 + c] * u[2];
            if (kk < kKfWin) atomicAdd(part + 6 * kk + c, y);
            else atomic_add(q + ok + c, y);
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; kbase != 0x7fffffff && e < kKfWin * 6; e += blockDim.x) {
        const int kf = kbase + e / 6;
        const double val = part[e];
        if (val != 0.0 && kf < d.K && kf != 0) atomic_add(q + 15 * (size_t)kf + e % 6, val);
    }
}

// q += (inertial and bias parts of H) v: one wavefront per term; lane c < 24
// holds column c (keyframe i's 15 entries, then keyframe j's first 9)
__global__ __launch_bounds__(256) void k_vi_prod_inertial(VIDev d, const double* __restrict__ v,
                                                          double* __restrict__ q,
                                                          const double* __restrict__ ps) {
    if (pcg_done(ps)) return;
    const int f = (int)((blockIdx.x * (long long)blockDim.x + threadIdx.x) >> 6);
    const int l = (int)(threadIdx.x & 63);
    if (f >= d.K - 1) return;   // whole wavefronts
    const size_t oi = 15 * (size_t)f, oj = 15 * (size_t)(f + 1);
    const double* J = d.ji + (size_t)216 * f;
    const double* O = d.info + 81 * (size_t)f;
    const bool col = l < 24;
    const double vc = col ? v[l < 15 ? oi + l : oj + (l - 15)] : 0.0;
    double jc[9];
    for (int a = 0; a < 9; ++a) jc[a] = col ? J[24 * a + l] : 0.0;
    // u = J v (sums over the 24 columns), w = Omega u, y_c = sum_a J[a][c] w[a]
    double u[9];
    for (int a = 0; a < 9; ++a) u[a] = wave_sum(jc[a] * vc);
    double y = 0.0;
    for (int a = 0; a < 9; ++a) {
        double w = 0.0;
        for (int b = 0; b < 9; ++b) w += O[9 * a + b] * u[b];
        y += jc[a] * w;
    }
    if (col) atomic_add(q + (l < 15 ? oi + l : oj + (l - 15)), y);
    if (l < 6) {
        const double dt = d.pre[(size_t)kPreStride * f + kDt];
        const double wb = (l < 3 ? d.wg : d.wa) / dt;
        const double vi_k = f != 0 ? v[oi + 9 + l] : 0.0;
        const double yb = wb * (v[oj + 9 + l] - vi_k);
        atomic_add(q + oj + 9 + l, yb);
        if (f != 0) atomic_add(q + oi + 9 + l, -yb);
    }
}

// ---- Schur form: the points eliminated (Eq. 5-6 on the keyframe / point
// partition).  With the damped blocks A (keyframes), B (keyframe-point,
// B_kj = W_e for the observation e of point j in keyframe k) and C (points):
//   S p = A p - B C^-1 B^T p,  v = -b_k + B C^-1 b_p,
//   x_p = C^-1 (-b_p - B^T x_k).
// A p is the keyframe diagonal blocks (hk + lambda D) plus the inertial and
// bias cross terms between consecutive keyframes.

// row t of A v: the keyframe diagonal block (damped) and the cross blocks to
// keyframes k - 1 and k + 1 (inertial, and the bias random walk's -Omega_b)
__device__ __forceinline__ double vi_ap_row(const VIDev& d, double lam, const double* __restrict__ v, long long t) {
    const long long k = t / 15;
    const int row = (int)(t % 15);
    const double* H = d.hk + 225 * (size_t)k + 15 * row;
    const double* vk = v + 15 * (size_t)k;
    double u = lam * d.dg[t] * vk[row];
    for (int c = 0; c < 15; ++c) u += H[c] * vk[c];
    if (k + 1 < d.K) {   // keyframe k as i of the term k: row of icx_k
        const double* C = d.icx + 135 * (size_t)k + 9 * row;
        const double* vj = v + 15 * (size_t)(k + 1);
        for (int c = 0; c < 9; ++c) u += C[c] * vj[c];
        if (row >= 9 && k != 0) {
            const double dt = d.pre[(size_t)kPreStride * k + kDt];
            u -= ((row < 12 ? d.wg : d.wa) / dt) * vj[row];
        }
    }
    if (k > 0) {         // keyframe k as j of the term k - 1: column of icx_{k-1}
        const double* vi = v + 15 * (size_t)(k - 1);
        if (row < 9) {
            const double* C = d.icx + 135 * (size_t)(k - 1) + row;
            for (int c = 0; c < 15; ++c) u += C[9 * c] * vi[c];
        } else if (k - 1 != 0) {
            const double dt = d.pre[(size_t)kPreStride * (k - 1) + kDt];
            u -= ((row < 12 ? d.wg : d.wa) / dt) * vi[row];
        }
    }
    return u;
}

// z_j = sign C_j^-1 (sum_{e of j} W_e^T v_k(e) + add_j): observations in
// padded point order (a point's observations within one wavefront unless it
// has more than 64; pad slots have point -1), a point's sum across its run of
// the wavefront.  A whole run stores z_j and, with acc, adds -t_j . z_j to
// acc (the point part of p . S p = p . A p - sum_j t_j . C_j^-1 t_j); a run
// of a point split across wavefronts adds its part of t_j to tb for
// k_vi_long_pts
//
// kFuse (the PCG product, sign 1, no add): the keyframe side too, q_k -=
// sum_{e of k} W_e z_j(e), in the same pass: z_j goes from the run's last
// lane to the run, each observation's W_e z_j is added to the workgroup's
// LDS partials of the keyframes kbase .. kbase + kKfWin - 1 (kbase the least
// keyframe the workgroup sees; points are numbered by first observing
// keyframe, so a workgroup's keyframes lie close together; one further out
// is added to q directly), and the partials go to q with one atomic add
// each.  Split points take this step in k_vi_long_kf.  The workgroups after
// the point ones add q += A v (one lane per keyframe row, vi_ap_row; q is
// zero beforehand) and v . A v: the whole product S v in one launch.

template <typename WT, bool kFuse>
__global__ __launch_bounds__(1024) void k_vi_schur_pts(VIDev d, const double* __restrict__ v,
                                                      const double* __restrict__ add, double sign,
                                                      double* __restrict__ z, const double* __restrict__ ps,
                                                      double* __restrict__ acc, double* __restrict__ q,
                                                      double lam) {
    if (pcg_done(ps)) return;
    __shared__ double red[16];
    __shared__ double part[kFuse ? kKfWin * 6 : 1];
    __shared__ int kmin_w[16];
    if (kFuse) {
        const long long pt_blocks = (d.Mp + blockDim.x - 1) / blockDim.x;
        if (blockIdx.x >= pt_blocks) {   // the keyframe rows (uniform per workgroup)
            const long long t0 = (blockIdx.x - pt_blocks) * (long long)blockDim.x + threadIdx.x;
            const bool act = t0 < 15LL * d.K;
            const long long t = act ? t0 : 0;
            const double u = vi_ap_row(d, lam, v, t);
            if (act) atomic_add(q + t, u);
            const double sa = block_sum_vi(act ? v[t] * u : 0.0, red);
            if (threadIdx.x == 0) atomic_add(acc + blockIdx.x % kPqParts, sa);
            return;
        }
    }
    const long long i0 = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const long long i = i0 < d.Mp ? i0 : d.Mp - 1;
    const int j = d.qpt[i];
    const bool valid = i0 < d.Mp && j >= 0;
    const int jj = valid ? j : 0, k = valid ? d.qkf[i] : 0;
    const int l = (int)(threadIdx.x & 63);
    const int jprev = __shfl_up(j, 1, 64);
    const bool start = !valid || l == 0 || jprev != j;
    const SegScan seg(start);
    int head, end;
    segment_of(__ballot(start), l, head, end);
    // the point's first and last observations in the whole order
    const bool first = i == 0 || d.qpt[i - 1] != j;
    const bool last = i == d.Mp - 1 || d.qpt[i + 1] != j;
    // (the run is the point's every observation; meaningful at the run's last lane)
    const bool whole = (__shfl(first ? 1 : 0, head, 64) != 0) && last;
    const double* Mi = d.mp + 9 * (size_t)jj;
    double M[9];
    for (int c = 0; c < 9; ++c) M[c] = Mi[c];
    const double* vk = v + 15 * (size_t)k;
    double W[18];
    load_w<WT>(d.wp, i, W);
    double t[3];
    for (int c = 0; c < 3; ++c) {
        double u = 0.0;
        for (int a = 0; a < 6; ++a) u += W[3 * a + c] * vk[a];
        t[c] = seg.sum(valid ? u : 0.0);
    }
    double tz = 0.0, o[3] = {0.0, 0.0, 0.0};
    if (valid && l == end) {
        if (whole) {
            if (add)
                for (int c = 0; c < 3; ++c) t[c] += add[3 * (size_t)j + c];
            for (int a = 0; a < 3; ++a) {
                o[a] = sign * (M[3 * a] * t[0] + M[3 * a + 1] * t[1] + M[3 * a + 2] * t[2]);
                z[3 * (size_t)j + a] = o[a];
                tz += t[a] * o[a];
            }
        } else {
            for (int a = 0; a < 3; ++a) atomic_add(d.tb + 3 * (size_t)j + a, t[a]);
        }
    }
    if (kFuse) {
        // the least keyframe of the workgroup's observations
        int km = valid ? k : 0x7fffffff;
        for (int off = 32; off > 0; off >>= 1) km = min(km, __shfl_xor(km, off, 64));
        if (l == 0) kmin_w[threadIdx.x >> 6] = km;
        for (int e = threadIdx.x; e < kKfWin * 6; e += blockDim.x) part[e] = 0.0;
        __syncthreads();
        int kbase = 0x7fffffff;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) kbase = min(kbase, kmin_w[w]);
        // z_j and the run's wholeness from its last lane (`whole` holds
        // there only)
        double zj[3];
        for (int a = 0; a < 3; ++a) zj[a] = __shfl(o[a], end, 64);
        const bool run_whole = __shfl(whole ? 1 : 0, end, 64) != 0;
        if (valid && run_whole) {
            const int kk = k - kbase;
            for (int a = 0; a < 6; ++a) {
                const double y = W[3 * a] * zj[0] + W[3 * a + 1] * zj[1] + W[3 * a + 2] * zj[2];
                if (kk < kKfWin) atomicAdd(part + 6 * kk + a, -y);
                else if (k != 0) atomic_add(q + 15 * (size_t)k + a, -y);
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; kbase != 0x7fffffff && e < kKfWin * 6; e += blockDim.x) {
            const int kf = kbase + e / 6;
            const double val = part[e];
            if (val != 0.0 && kf < d.K && kf != 0) atomic_add(q + 15 * (size_t)kf + e % 6, val);
        }
    }
    if (acc) {
        tz = block_sum_vi(tz, red);
        if (threadIdx.x == 0) atomic_add(acc + blockIdx.x % kPqParts, -tz);
    }
}

// the keyframe side of the product for the observations of split points:
// q_k -= W_e z_j, one lane per such observation (their slots in lslot)
template <typename WT>
__global__ void k_vi_long_kf(VIDev d, const double* __restrict__ z, double* __restrict__ q,
                             const double* __restrict__ ps) {
    if (pcg_done(ps)) return;
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= d.nlslot) return;
    const long long i = d.lslot[t];
    const int j = d.qpt[i], k = d.qkf[i];
    if (k == 0) return;
    double W[18];
    load_w<WT>(d.wp, i, W);
    const double zj[3] = {z[3 * (size_t)j], z[3 * (size_t)j + 1], z[3 * (size_t)j + 2]};
    for (int a = 0; a < 6; ++a)
        atomic_add(q + 15 * (size_t)k + a, -(W[3 * a] * zj[0] + W[3 * a + 1] * zj[1] + W[3 * a + 2] * zj[2]));
}

// the points split across wavefronts (more than 64 observations): z_j =
// sign C_j^-1 (t_j + add_j) from the parts in tb, -t_j . z_j into acc, tb
// cleared for the next pass; one lane per such point
__global__ void k_vi_long_pts(VIDev d, const double* __restrict__ add, double sign, double* __restrict__ z,
                              const double* __restrict__ ps, double* __restrict__ acc) {
    if (pcg_done(ps)) return;
    __shared__ double red[16];
    const int q = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    double tz = 0.0;
    if (q < d.nlong) {
        const int j = d.longp[q];
        double t[3];
        for (int c = 0; c < 3; ++c) {
            t[c] = d.tb[3 * (size_t)j + c] + (add ? add[3 * (size_t)j + c] : 0.0);
            d.tb[3 * (size_t)j + c] = 0.0;
        }
        const double* Mi = d.mp + 9 * (size_t)j;
        for (int a = 0; a < 3; ++a) {
            const double o = sign * (Mi[3 * a] * t[0] + Mi[3 * a + 1] * t[1] + Mi[3 * a + 2] * t[2]);
            z[3 * (size_t)j + a] = o;
            tz += t[a] * o;
        }
    }
    if (acc) {
        tz = block_sum_vi(tz, red);
        if (threadIdx.x == 0) atomic_add(acc + blockIdx.x % kPqParts, -tz);
    }
}

// out_j = sign C_j^-1 in_j, one lane per point
__global__ void k_vi_pt_apply(VIDev d, const double* __restrict__ in, double sign, double* __restrict__ out) {
    const long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (j >= d.N) return;
    const double* Mi = d.mp + 9 * j;
    const double a = in[3 * j], b = in[3 * j + 1], c = in[3 * j + 2];
    for (int r = 0; r < 3; ++r) out[3 * j + r] = sign * (Mi[3 * r] * a + Mi[3 * r + 1] * b + Mi[3 * r + 2] * c);
}

// sum over the points of x_j^T H_pp,j x_j (the undamped point blocks) into *out
__global__ void k_vi_pt_quad(VIDev d, const double* __restrict__ x, double* __restrict__ out) {
    __shared__ double red[16];
    const long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    double s = 0.0;
    if (j < d.N) {
        const double* H = d.hp + 9 * j;
        const double a = x[3 * j], b = x[3 * j + 1], c = x[3 * j + 2];
        s = a * (H[0] * a + H[1] * b + H[2] * c) + b * (H[3] * a + H[4] * b + H[5] * c) +
            c * (H[6] * a + H[7] * b + H[8] * c);
    }
    s = block_sum_vi(s, red);
    if (threadIdx.x == 0) atomic_add(out + blockIdx.x % kPqParts, s);   // out: kPqParts parts
}

// q_k -= sum_{e of k} W_e z_j(e): observations in keyframe order, the
// keyframe's sum across its run of the wavefront, one atomic add per run
template <typename WT>
__global__ void k_vi_schur_kf(VIDev d, const double* __restrict__ z, double* __restrict__ q,
                              const double* __restrict__ ps) {
    if (pcg_done(ps)) return;
    const long long e0 = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const bool valid = e0 < d.M;
    const long long e = valid ? e0 : d.M - 1;
    const int k = d.kf[e], j = d.pt[e];
    const int l = (int)(threadIdx.x & 63);
    const int kprev = __shfl_up(k, 1, 64);
    const bool start = !valid || l == 0 || kprev != k;
    const SegScan seg(start);
    int head, end;
    segment_of(__ballot(start), l, head, end);
    const double zj[3] = {z[3 * (size_t)j], z[3 * (size_t)j + 1], z[3 * (size_t)j + 2]};
    double W[18];
    load_w<WT>(d.wk, e, W);
    double y[6];
    for (int a = 0; a < 6; ++a) {
        double u = 0.0;
        for (int c = 0; c < 3; ++c) u += W[3 * a + c] * zj[c];
        y[a] = seg.sum(valid ? u : 0.0);
    }
    if (valid && l == end && k != 0)
        for (int a = 0; a < 6; ++a) atomic_add(q + 15 * (size_t)k + a, -y[a]);
}

// sm_k = sum_{e of k} W_e C_j^-1 W_e^T (the pose block's Schur term for the
// preconditioner: the diagonal block of S when each keyframe sees a point at
// most once), summed across the keyframe's run of the wavefront
template <typename WT>
__global__ void k_vi_schur_blocks(VIDev d) {
    const long long e0 = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const bool valid = e0 < d.M;
    const long long e = valid ? e0 : d.M - 1;
    const int k = d.kf[e], j = d.pt[e];
    const int l = (int)(threadIdx.x & 63);
    const int kprev = __shfl_up(k, 1, 64);
    const bool start = !valid || l == 0 || kprev != k;
    const SegScan seg(start);
    int head, end;
    segment_of(__ballot(start), l, head, end);
    const double* Mi = d.mp + 9 * (size_t)j;
    double W[6][3], G[6][3], Wf[18];
    load_w<WT>(d.wk, e, Wf);
    for (int a = 0; a < 6; ++a)
        for (int c = 0; c < 3; ++c) W[a][c] = valid ? Wf[3 * a + c] : 0.0;
    for (int a = 0; a < 6; ++a)
        for (int c = 0; c < 3; ++c) G[a][c] = W[a][0] * Mi[c] + W[a][1] * Mi[3 + c] + W[a][2] * Mi[6 + c];
    const bool out = valid && l == end && k != 0;
    double* S = d.sm + 36 * (size_t)k;
    for (int a = 0; a < 6; ++a)
        for (int c = a; c < 6; ++c) {
            const double h = seg.sum(G[a][0] * W[c][0] + G[a][1] * W[c][1] + G[a][2] * W[c][2]);
            if (out) {
                atomic_add(S + 6 * a + c, h);
                if (c != a) atomic_add(S + 6 * c + a, h);
            }
        }
}

// the inertial cross blocks of the damped system, once per linearisation:
// icx_f = J_i^T Omega J_j over keyframe i's 15 columns and keyframe j's first
// 9 (one lane per entry)
__global__ void k_vi_cross(VIDev d) {
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t >= 135LL * (d.K - 1)) return;
    const long long f = t / 135;
    const int a = (int)(t % 135) / 9, c = (int)(t % 9);
    const double* J = d.ji + (size_t)216 * f;
    const double* O = d.info + 81 * (size_t)f;
    double u = 0.0;
    for (int m = 0; m < 9; ++m) {
        double w = 0.0;
        for (int k = 0; k < 9; ++k) w += O[9 * m + k] * J[24 * k + 15 + c];
        u += J[24 * m + a] * w;
    }
    d.icx[t] = u;
}

// q_k = A_k v: (hk_k + lambda diag(D_k)) v_k plus the cross blocks to
// keyframes k - 1 and k + 1 (inertial, and the bias random walk's -Omega_b);
// one lane per keyframe row, no atomics
__global__ void k_vi_schur_ap(VIDev d, double lam, const double* __restrict__ v, double* __restrict__ q,
                              const double* __restrict__ ps, double* __restrict__ acc) {
    if (pcg_done(ps)) return;
    __shared__ double red[16];
    const long long t0 = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    const bool act = t0 < 15LL * d.K;
    const long long t = act ? t0 : 0;
    const double u = vi_ap_row(d, lam, v, t);
    if (act) q[t] = u;
    if (acc) {   // with acc: v . A v (the keyframe part of p . S p)
        const double s = block_sum_vi(act ? v[t] * u : 0.0, red);
        if (threadIdx.x == 0) atomic_add(acc + blockIdx.x % kPqParts, s);
    }
}

// q = lambda diag(D) v (the first term of the product; the others add)
__global__ void k_vi_prod_damp(long long n, double lam, const double* __restrict__ dg,
                               const double* __restrict__ v, double* __restrict__ q,
                               const double* __restrict__ ps) {
    if (pcg_done(ps)) return;
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) q[i] = lam * dg[i] * v[i];
}

// r.r and r.z into the accumulators acc (the start of the PCG)
__global__ void k_vi_dot2(long long n, const double* __restrict__ r, const double* __restrict__ z,
                          double* __restrict__ acc) {
    __shared__ double red[16];
    double a = 0.0, b = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        a += r[i] * r[i];
        b += r[i] * z[i];
    }
    a = block_sum_vi(a, red);
    __syncthreads();
    b = block_sum_vi(b, red);
    if (threadIdx.x == 0) {
        atomic_add(acc + kAccRr, a);
        atomic_add(acc + kAccRz, b);
    }
}

// the start: threshold tol^2 r0.r0 (r0.r0 and r0.z0 in the last slot);
// nothing to do when r0 is already below it or r0.z0 <= 0.  ratio2: the
// squared rejection ratio (0: no rejection test)
__global__ void k_vi_pcg_init(double* __restrict__ ps, double tol, double ratio2) {
    double* a = ps + kAccN * (kSlots - 1);
    const double thr = tol * tol * a[kAccRr];
    ps[kThr] = thr;
    ps[kDone] = (a[kAccRr] > thr && a[kAccRz] > 0.0) ? 0.0 : 1.0;
    ps[kSteps] = 0.0;
    ps[kRatio2] = ratio2;
    a[kAccMin] = a[kAccRr];
    a[kAccStop] = ps[kDone];
}

// step `slot`: alpha = r.z / p.q (a step with p.q <= 0 ends the iteration at
// the current iterate), x += alpha p, r -= alpha q, z = M^-1 r and the new
// r.r, r.z.  Keyframe rows: 16 lanes per keyframe (15 used), the residual
// block through LDS for the 15 x 15 inverse; point rows (the whole-system
// form): three lanes per point in the workgroups after the keyframe ones.
constexpr int kUpdPts = 85;   // points per 256-lane workgroup of the update
__global__ __launch_bounds__(256) void k_vi_pcg_update(VIDev d, long long npt, double* __restrict__ ps,
                                                      int slot, const double* __restrict__ p,
                                                      const double* __restrict__ q, double* __restrict__ x,
                                                      double* __restrict__ r, double* __restrict__ z) {
    __shared__ double rs[256];
    __shared__ double red[16];
    if (ps[kDone] != 0.0) return;
    double* acc = ps + kAccN * slot;
    __shared__ double pq_s;
    {
        const double part = block_sum_vi(threadIdx.x < kPqParts ? acc[kAccPq + threadIdx.x] : 0.0, red);
        if (threadIdx.x == 0) pq_s = part;
        __syncthreads();
    }
    const double pq = pq_s;
    if (!(pq > 0.0)) {   // breakdown: decided by every workgroup alike
        if (blockIdx.x == 0 && threadIdx.x == 0) acc[kAccBreak] = 1.0;
        return;
    }
    const double alpha = ps[kAccN * ((slot + kSlots - 1) % kSlots) + kAccRz] / pq;
    const long long kf_blocks = (d.K + 15) / 16;
    double rr = 0.0, rz = 0.0;
    if (blockIdx.x < kf_blocks) {
        const long long k = blockIdx.x * 16LL + (threadIdx.x >> 4);
        const int row = (int)(threadIdx.x & 15);
        const bool act = k < d.K && row < 15;
        const size_t i = 15 * (size_t)k + row;
        double rn = 0.0;
        if (act) {
            x[i] += alpha * p[i];
            rn = r[i] - alpha * q[i];
            r[i] = rn;
        }
        rs[threadIdx.x] = rn;
        __syncthreads();
        if (act) {
            const double* Mi = d.mki + 225 * (size_t)k + 15 * row;
            const double* rk = rs + (threadIdx.x & ~15u);
            double u = 0.0;
            for (int c = 0; c < 15; ++c) u += Mi[c] * rk[c];
            z[i] = u;
            rr = rn * rn;
            rz = rn * u;
        }
    } else {
        // point rows: three lanes per point (kUpdPts points per workgroup),
        // so consecutive lanes take consecutive rows; the point's residual
        // through LDS for its 3 x 3 inverse
        const int pl = (int)threadIdx.x / 3, a = (int)threadIdx.x - 3 * pl;
        const long long j = (blockIdx.x - kf_blocks) * (long long)kUpdPts + pl;
        const bool act = pl < kUpdPts && j < npt;
        const size_t i = 15 * (size_t)d.K + 3 * (size_t)j + a;
        double rn = 0.0;
        if (act) {
            x[i] += alpha * p[i];
            rn = r[i] - alpha * q[i];
            r[i] = rn;
        }
        rs[threadIdx.x] = rn;
        __syncthreads();
        if (act) {
            const double* M = d.mp + 9 * (size_t)j + 3 * a;
            const double* rk = rs + 3 * pl;
            const double u = M[0] * rk[0] + M[1] * rk[1] + M[2] * rk[2];
            z[i] = u;
            rr = rn * rn;
            rz = rn * u;
        }
    }
    rr = block_sum_vi(rr, red);
    __syncthreads();
    rz = block_sum_vi(rz, red);
    if (threadIdx.x == 0) {
        atomic_add(acc + kAccRrP + blockIdx.x % kPqParts, rr);   // summed by k_vi_pcg_dir
        atomic_add(acc + kAccRzP + blockIdx.x % kPqParts, rz);
        if (blockIdx.x == 0) ps[kSteps] += 1.0;
    }
}

// step `slot`, continued, with the decisions of the PCG rules: a breakdown
// ends at the current iterate; with the rejection test, a new least r.r
// saves x in xb, and r.r > ratio^2 times the least ends the iteration with
// xb restored; r.r <= the threshold ends it; otherwise p = z + beta p with
// beta = r.z / previous r.z.  Every workgroup takes the same decisions from
// this slot's and the previous slot's values (which no workgroup of this
// kernel writes); workgroup 0 records them (this slot's least r.r and stop
// flag, the stop flag the later kernels read) and clears the next slot; qz
// (when given) is cleared for the next product.
__global__ void k_vi_pcg_dir(long long n, double* __restrict__ ps, int slot, const double* __restrict__ z,
                             double* __restrict__ p, double* __restrict__ x, double* __restrict__ xb,
                             double* __restrict__ qz) {
    double* acc = ps + kAccN * slot;
    const double* prev = ps + kAccN * ((slot + kSlots - 1) % kSlots);
    const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
    const long long st = (long long)gridDim.x * blockDim.x;
    const long long i0 = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    // this step's r.r and r.z from their parts (the same sums, in the same
    // order, in every workgroup); workgroup 0 keeps them in the slot
    __shared__ double red[16];
    __shared__ double sums[2];
    {
        const double a = block_sum_vi(threadIdx.x < kPqParts ? acc[kAccRrP + threadIdx.x] : 0.0, red);
        __syncthreads();
        const double b = block_sum_vi(threadIdx.x < kPqParts ? acc[kAccRzP + threadIdx.x] : 0.0, red);
        if (threadIdx.x == 0) {
            sums[0] = a;
            sums[1] = b;
        }
        __syncthreads();
    }
    if (lead) {
        acc[kAccRr] = sums[0];
        acc[kAccRz] = sums[1];
    }
    if (blockIdx.x == 0)
        for (int e = threadIdx.x; e < kAccN; e += blockDim.x) ps[kAccN * ((slot + 1) % kSlots) + e] = 0.0;
    if (prev[kAccStop] != 0.0 || acc[kAccBreak] != 0.0) {
        if (lead) {
            acc[kAccStop] = 1.0;
            acc[kAccMin] = prev[kAccMin];
            ps[kDone] = 1.0;
        }
        return;
    }
    const double rr = sums[0], least = prev[kAccMin], ratio2 = ps[kRatio2];
    double nmin = least;
    if (ratio2 > 0.0) {
        if (rr < least) {
            nmin = rr;
            for (long long i = i0; i < n; i += st) xb[i] = x[i];
        } else if (rr > ratio2 * least) {
            for (long long i = i0; i < n; i += st) x[i] = xb[i];
            if (lead) {
                acc[kAccStop] = 1.0;
                acc[kAccMin] = least;
                ps[kDone] = 1.0;
            }
            return;
        }
    }
    if (rr <= ps[kThr]) {
        if (lead) {
            acc[kAccStop] = 1.0;
            acc[kAccMin] = nmin;
            ps[kDone] = 1.0;
        }
        return;
    }
    const double beta = sums[1] / prev[kAccRz];
    for (long long i = i0; i < n; i += st) {
        p[i] = z[i] + beta * p[i];
        if (qz) qz[i] = 0.0;   // the next product adds into q
    }
    if (lead) acc[kAccMin] = nmin;
}

// out[blockIdx % parts] += the workgroup's part of a . b (parts > 1 spreads
// the additions over addresses that the reader sums)
__global__ void k_vi_dot(long long n, const double* __restrict__ a, const double* __restrict__ b,
                         double* __restrict__ out, const double* __restrict__ ps = nullptr, int parts = 1) {
    if (pcg_done(ps)) return;
    __shared__ double red[16];
    double s = 0.0;
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        s += a[i] * b[i];
    s = block_sum_vi(s, red);
    if (threadIdx.x == 0) atomic_add(out + blockIdx.x % parts, s);
}

// p = z (the first direction)
__global__ void k_vi_copy(long long n, const double* __restrict__ z, double* __restrict__ p) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) p[i] = z[i];
}

__global__ void k_vi_neg(long long n, const double* __restrict__ b, double* __restrict__ r,
                         double* __restrict__ x) {
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) {
        r[i] = -b[i];
        x[i] = 0.0;
    }
}

__global__ void k_vi_fill(long long n, double* __restrict__ a, const double* __restrict__ ps = nullptr) {
    if (pcg_done(ps)) return;
    const long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0.0;
}

// candidate: R Exp(dtheta), p + dp, v + dv, b + db; X + dX
__global__ void k_vi_step(VIDev d, const double* __restrict__ dx) {
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (t < d.K) {
        const double* s = d.st + (size_t)kSt * t;
        double* c = d.st_c + (size_t)kSt * t;
        const double* u = dx + 15 * (size_t)t;
        const double w[3] = {u[0], u[1], u[2]};
        double E[3][3];
        so3_exp(w, E);
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                c[3 * a + b] = s[3 * a] * E[0][b] + s[3 * a + 1] * E[1][b] + s[3 * a + 2] * E[2][b];
        for (int k = 0; k < 12; ++k) c[9 + k] = s[9 + k] + u[3 + k];
    } else if (t < d.K + d.N) {
        const long long j = t - d.K;
        for (int k = 0; k < 3; ++k) d.X_c[3 * j + k] = d.X[3 * j + k] + dx[15 * (size_t)d.K + 3 * j + k];
    }
}

// |x|^2 over the free parameters: |Log R|^2 and the other state entries of
// keyframes 1.., and the points
__global__ void k_vi_xnorm(VIDev d, const double* __restrict__ st, const double* __restrict__ X, int slot) {
    __shared__ double red[16];
    const long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    double s = 0.0;
    if (t >= 1 && t < d.K) {
        const double* q = st + (size_t)kSt * t;
        double R[3][3], w[3];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) R[a][b] = q[3 * a + b];
        so3_log(R, w);
        for (int k = 0; k < 3; ++k) s += w[k] * w[k];
        for (int k = 9; k < kSt; ++k) s += q[k] * q[k];
    } else if (t >= d.K && t < d.K + d.N) {
        const long long j = t - d.K;
        for (int k = 0; k < 3; ++k) s += X[3 * j + k] * X[3 * j + k];
    }
    s = block_sum_vi(s, red);
    if (threadIdx.x == 0) atomic_add(d.scal + kRedOff + slot * kPqParts + blockIdx.x % kPqParts, s);
}

}  // namespace vi
}  // namespace gba

// ------------------------------------------------------------------ C ABI
namespace {

// Device buffers of one call, released on every return path.
struct DevBufs {
    std::vector<void*> p;
    size_t bytes = 0;
    ~DevBufs() {
        for (void* q : p) (void)hipFree(q);
    }
    template <typename T>
    bool up(T** dst, const T* src, size_t n) {
        void* q = nullptr;
        if (hipMalloc(&q, n * sizeof(T) + 16) != hipSuccess) return false;
        p.push_back(q);
        bytes += n * sizeof(T) + 16;
        *dst = (T*)q;
        return !src || hipMemcpy(q, src, n * sizeof(T), hipMemcpyHostToDevice) == hipSuccess;
    }
};

}  // namespace

extern "C" {

gba_status gba_vi_preintegrate(int device, int n, const int64_t* sample_off, const double* gyro,
                               const double* acc, double dt, const double* bias0, double sigma_g,
                               double sigma_a, double* out) {
    if (n < 0 || !sample_off || !bias0 || !out || !(dt > 0.0) || !(sigma_g >= 0.0) || !(sigma_a >= 0.0))
        return GBA_ERR_INVALID_ARG;
    if (n == 0) return GBA_OK;
    for (int f = 0; f < n; ++f)
        if (sample_off[f + 1] < sample_off[f] || sample_off[0] != 0) return GBA_ERR_INVALID_ARG;
    const size_t ns = (size_t)sample_off[n];
    if (ns > 0 && (!gyro || !acc)) return GBA_ERR_INVALID_ARG;
    if (hipSetDevice(device) != hipSuccess) return GBA_ERR_HIP;
    DevBufs b;
    long long* doff = nullptr;
    double *dg = nullptr, *da = nullptr, *db = nullptr, *dout = nullptr;
    if (!b.up(&doff, (const long long*)sample_off, (size_t)n + 1) || !b.up(&dg, gyro, 3 * ns + 3) ||
        !b.up(&da, acc, 3 * ns + 3) || !b.up(&db, bias0, 6 * (size_t)n) ||
        !b.up(&dout, (const double*)nullptr, (size_t)gba::vi::kPreStride * n))
        return GBA_ERR_HIP;
    hipLaunchKernelGGL(gba::vi::k_preintegrate, dim3((n + 63) / 64), dim3(64), 0, nullptr, n, doff, dg,
                       da, dt, db, sigma_g, sigma_a, dout);
    if (hipGetLastError() != hipSuccess) return GBA_ERR_HIP;
    if (hipMemcpy(out, dout, sizeof(double) * gba::vi::kPreStride * n, hipMemcpyDeviceToHost) != hipSuccess)
        return GBA_ERR_HIP;
    return GBA_OK;
}

gba_status gba_vi_eval_inertial(int device, int n_kf, const double* states, const double* pre,
                                double* r, double* J) {
    if (n_kf < 0 || (n_kf > 1 && (!states || !pre || !r || !J))) return GBA_ERR_INVALID_ARG;
    const int n = n_kf > 1 ? n_kf - 1 : 0;
    if (n == 0) return GBA_OK;
    if (hipSetDevice(device) != hipSuccess) return GBA_ERR_HIP;
    DevBufs b;
    double *ds = nullptr, *dp = nullptr, *dr = nullptr, *dj = nullptr;
    if (!b.up(&ds, states, 15 * (size_t)n_kf) || !b.up(&dp, pre, (size_t)gba::vi::kPreStride * n) ||
        !b.up(&dr, (const double*)nullptr, 9 * (size_t)n) || !b.up(&dj, (const double*)nullptr, 216 * (size_t)n))
        return GBA_ERR_HIP;
    const long long lanes = 24LL * n;
    hipLaunchKernelGGL(gba::vi::k_inertial_eval, dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0,
                       nullptr, n, ds, dp, dr, dj);
    if (hipGetLastError() != hipSuccess) return GBA_ERR_HIP;
    if (hipMemcpy(r, dr, sizeof(double) * 9 * n, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(J, dj, sizeof(double) * 216 * n, hipMemcpyDeviceToHost) != hipSuccess)
        return GBA_ERR_HIP;
    return GBA_OK;
}

gba_status gba_vi_eval_stereo(int device, int n_kf, const double* states, int64_t n_pts,
                              const double* pts, int64_t n_obs, const int64_t* kf, const int64_t* pt,
                              const double* obs, const double* intr, double* r, double* J) {
    if (n_kf < 0 || n_pts < 0 || n_obs < 0 || !intr) return GBA_ERR_INVALID_ARG;
    if (n_obs == 0) return GBA_OK;
    if (!states || !pts || !kf || !pt || !obs || !r || !J) return GBA_ERR_INVALID_ARG;
    for (int64_t e = 0; e < n_obs; ++e)
        if (kf[e] < 0 || kf[e] >= n_kf || pt[e] < 0 || pt[e] >= n_pts) return GBA_ERR_UNKNOWN_ID;
    if (hipSetDevice(device) != hipSuccess) return GBA_ERR_HIP;
    DevBufs b;
    double *ds = nullptr, *dpts = nullptr, *dobs = nullptr, *dr = nullptr, *dj = nullptr;
    long long *dkf = nullptr, *dpt = nullptr;
    if (!b.up(&ds, states, 15 * (size_t)n_kf) || !b.up(&dpts, pts, 3 * (size_t)n_pts) ||
        !b.up(&dkf, (const long long*)kf, (size_t)n_obs) || !b.up(&dpt, (const long long*)pt, (size_t)n_obs) ||
        !b.up(&dobs, obs, 3 * (size_t)n_obs) || !b.up(&dr, (const double*)nullptr, 3 * (size_t)n_obs) ||
        !b.up(&dj, (const double*)nullptr, 27 * (size_t)n_obs))
        return GBA_ERR_HIP;
    const long long lanes = 9LL * n_obs;
    hipLaunchKernelGGL(gba::vi::k_stereo_eval, dim3((unsigned)((lanes + 255) / 256)), dim3(256), 0,
                       nullptr, (long long)n_obs, ds, dpts, dkf, dpt, dobs, intr[0], intr[1], intr[2],
                       intr[3], intr[4], dr, dj);
    if (hipGetLastError() != hipSuccess) return GBA_ERR_HIP;
    if (hipMemcpy(r, dr, sizeof(double) * 3 * n_obs, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(J, dj, sizeof(double) * 27 * n_obs, hipMemcpyDeviceToHost) != hipSuccess)
        return GBA_ERR_HIP;
    return GBA_OK;
}

void gba_vi_default_options(gba_vi_options* o) {
    if (!o) return;
    o->pcg_max_iters = 100;
    o->solver = GBA_SOLVER_SCHUR;
    o->precision = GBA_FP64;
    o->reserved1 = 0;
    o->pcg_rejection_ratio = 0.0;
    o->pcg_tol = 1e-8;
    o->initial_lambda = 1e-4;
    o->min_diag = 1e-6;
    o->max_diag = 1e32;
}

gba_status gba_vi_solve(int device, const gba_vi_problem* prob, int max_iters, double tol,
                        const gba_vi_options* opts, gba_report* report, gba_trial* log, int max_log,
                        int* n_log) {
    using namespace gba::vi;
    const auto t_start = std::chrono::steady_clock::now();
    if (n_log) *n_log = 0;
    if (!prob || max_iters < 0 || !(tol >= 0.0) || (max_log > 0 && !log)) return GBA_ERR_INVALID_ARG;
    const gba_vi_problem& P = *prob;
    if (P.n_kf < 2 || P.n_pts < 0 || P.n_obs < 0 || !P.states || !P.intr || !P.pre ||
        (P.n_pts > 0 && !P.pts) || (P.n_obs > 0 && (!P.kf || !P.pt || !P.obs)) ||
        !(P.sigma_px > 0.0) || !(P.huber_delta2 >= 0.0) || !(P.sigma_gw > 0.0) || !(P.sigma_aw > 0.0))
        return GBA_ERR_INVALID_ARG;
    if (P.n_obs > INT32_MAX / 27 || P.n_pts > INT32_MAX || P.n_kf > INT32_MAX / 225)
        return GBA_ERR_UNSUPPORTED;
    gba_vi_options o;
    gba_vi_default_options(&o);
    if (opts) o = *opts;
    if (o.pcg_max_iters < 1 || !(o.pcg_tol >= 0.0) || !(o.initial_lambda > 0.0) ||
        (o.solver != GBA_SOLVER_SCHUR && o.solver != GBA_SOLVER_FULL) ||
        (o.precision != GBA_FP64 && o.precision != GBA_MIXED_FP32) ||

        !(o.min_diag > 0.0) || !(o.max_diag >= o.min_diag))
        return GBA_ERR_INVALID_ARG;
    // observations in keyframe order (a stable counting sort), so that the
    // keyframe terms of a wavefront sum across it before their atomic add
    std::vector<int> hkf((size_t)P.n_obs + 1, 0), hpt((size_t)P.n_obs + 1, 0);   // + 1: uploaded with a pad
    std::vector<double> hobs(3 * (size_t)P.n_obs + 1, 0.0);
    {
        std::vector<int64_t> cnt((size_t)P.n_kf + 1, 0);
        for (int64_t e = 0; e < P.n_obs; ++e) {
            if (P.kf[e] < 0 || P.kf[e] >= P.n_kf || P.pt[e] < 0 || P.pt[e] >= P.n_pts)
                return GBA_ERR_UNKNOWN_ID;
            ++cnt[(size_t)P.kf[e] + 1];
        }
        for (int k = 0; k < P.n_kf; ++k) cnt[(size_t)k + 1] += cnt[(size_t)k];
        for (int64_t e = 0; e < P.n_obs; ++e) {
            const size_t q = (size_t)cnt[(size_t)P.kf[e]]++;
            hkf[q] = (int)P.kf[e];
            hpt[q] = (int)P.pt[e];
            for (int c = 0; c < 3; ++c) hobs[3 * q + c] = P.obs[3 * e + c];
        }
    }
    // points renumbered by the first keyframe that observes them (stable;
    // unobserved points last), so that a keyframe's observations and a run
    // of consecutive points touch nearby points and keyframes: the point
    // and keyframe gathers of the products stay within a narrow window
    std::vector<int> pt_new((size_t)P.n_pts), pt_old((size_t)P.n_pts);
    {
        std::vector<int> first((size_t)P.n_pts, P.n_kf);
        for (int64_t e = 0; e < P.n_obs; ++e) first[hpt[e]] = std::min(first[hpt[e]], hkf[e]);
        std::vector<int64_t> cnt((size_t)P.n_kf + 2, 0);
        for (int64_t j = 0; j < P.n_pts; ++j) ++cnt[(size_t)first[j] + 1];
        for (int k = 0; k <= P.n_kf; ++k) cnt[(size_t)k + 1] += cnt[(size_t)k];
        for (int64_t j = 0; j < P.n_pts; ++j) {
            const int q = (int)cnt[(size_t)first[j]]++;
            pt_new[j] = q;
            pt_old[q] = (int)j;
        }
        for (int64_t e = 0; e < P.n_obs; ++e) hpt[e] = pt_new[hpt[e]];
    }
    std::vector<double> hX(3 * (size_t)P.n_pts + 1, 0.0);
    for (int64_t q = 0; q < P.n_pts; ++q)
        for (int c = 0; c < 3; ++c) hX[3 * q + c] = P.pts[3 * (size_t)pt_old[q] + c];
    const bool schur = o.solver == GBA_SOLVER_SCHUR;
    // the same observations in point order (stable in the keyframe order),
    // padded so that a point's observations sit in one wavefront (64 slots)
    // unless it has more than 64 of them
    std::vector<int> hqkf, hqpt, hlong, hlslot;
    std::vector<double> hqobs;
    long long Mp = 0;
    {
        std::vector<int64_t> cnt((size_t)P.n_pts, 0), at((size_t)P.n_pts, 0);
        for (int64_t e = 0; e < P.n_obs; ++e) ++cnt[(size_t)hpt[e]];
        for (int64_t j = 0; j < P.n_pts; ++j) {
            const int64_t c = cnt[(size_t)j];
            if (c == 0) continue;
            if (c > 64) hlong.push_back((int)j);
            else if (Mp % 64 + c > 64) Mp = (Mp + 63) / 64 * 64;
            at[(size_t)j] = Mp;
            Mp += c;
        }
        Mp = (Mp + 63) / 64 * 64;
        if (Mp > INT32_MAX / 18) return GBA_ERR_UNSUPPORTED;
        hqkf.assign((size_t)Mp + 1, 0);
        hqpt.assign((size_t)Mp + 1, -1);
        hqobs.assign(3 * (size_t)Mp + 1, 0.0);
        for (int64_t e = 0; e < P.n_obs; ++e) {
            const size_t q = (size_t)at[(size_t)hpt[e]]++;
            hqkf[q] = hkf[e];
            hqpt[q] = hpt[e];
            for (int c = 0; c < 3; ++c) hqobs[3 * q + c] = hobs[3 * e + c];
        }
        for (const int j : hlong)
            for (int64_t q = at[(size_t)j] - cnt[(size_t)j]; q < at[(size_t)j]; ++q) hlslot.push_back((int)q);
    }
    if (hipSetDevice(device) != hipSuccess) return GBA_ERR_HIP;
    const int K = P.n_kf;
    const long long N = P.n_pts, M = P.n_obs, n = 15LL * K + 3 * N;
    DevBufs B;
    VIDev d{};
    d.K = K;
    d.N = N;
    d.M = M;
    double *s15 = nullptr, *pre = nullptr, *x = nullptr, *r = nullptr, *z = nullptr, *pv = nullptr,
           *q = nullptr, *xb = nullptr;
    int *dkf = nullptr, *dpt = nullptr;
    double* obs = nullptr;
    if (!B.up(&s15, P.states, 15 * (size_t)K) || !B.up(&d.st, (const double*)nullptr, kSt * (size_t)K) ||
        !B.up(&d.st_c, (const double*)nullptr, kSt * (size_t)K) ||
        !B.up(&d.X, (const double*)hX.data(), 3 * (size_t)N) || !B.up(&d.X_c, (const double*)nullptr, 3 * (size_t)N + 1) ||
        !B.up(&dkf, hkf.data(), (size_t)M + 1) || !B.up(&dpt, hpt.data(), (size_t)M + 1) ||
        !B.up(&obs, hobs.data(), 3 * (size_t)M + 1) ||
        !B.up(&pre, P.pre, (size_t)kPreStride * (K - 1)) ||
        !B.up(&d.info, (const double*)nullptr, 81 * (size_t)(K - 1)) ||
        !B.up(&d.ji, (const double*)nullptr, 216 * (size_t)(K - 1)) ||
        !B.up(&d.ri, (const double*)nullptr, 9 * (size_t)(K - 1)) ||
        !B.up(&d.b, (const double*)nullptr, (size_t)n) || !B.up(&d.hk, (const double*)nullptr, 225 * (size_t)K) ||
        !B.up(&d.hp, (const double*)nullptr, 9 * (size_t)N + 1) || !B.up(&d.dg, (const double*)nullptr, (size_t)n) ||
        !B.up(&d.mki, (const double*)nullptr, 225 * (size_t)K) || !B.up(&d.mp, (const double*)nullptr, 9 * (size_t)N + 1) ||
        !B.up(&d.scal, (const double*)nullptr, (size_t)kScalN) || !B.up(&x, (const double*)nullptr, (size_t)n) ||
        !B.up(&r, (const double*)nullptr, (size_t)n) || !B.up(&z, (const double*)nullptr, (size_t)n) ||
        !B.up(&pv, (const double*)nullptr, (size_t)n) || !B.up(&q, (const double*)nullptr, (size_t)n) ||
        !B.up(&xb, (const double*)nullptr, (size_t)n))
        return GBA_ERR_OOM;
    {   // the padded point order (both forms)
        int *qkf = nullptr, *qpt = nullptr;
        double* qobs = nullptr;
        if (!B.up(&qkf, hqkf.data(), (size_t)Mp + 1) || !B.up(&qpt, hqpt.data(), (size_t)Mp + 1) ||
            !B.up(&qobs, hqobs.data(), 3 * (size_t)Mp + 1))
            return GBA_ERR_OOM;
        d.qkf = qkf;
        d.qpt = qpt;
        d.qobs = qobs;
        d.Mp = Mp;
    }
    if (!schur) {   // the point-order J (FP32: half the doubles, rounded up)
        d.w32 = o.precision == GBA_MIXED_FP32 ? 1 : 0;
        double* jp = nullptr;
        if (!B.up(&jp, (const double*)nullptr, (27 * 64 * (size_t)(Mp / 64) + 2) / (d.w32 ? 2 : 1))) return GBA_ERR_OOM;
        d.jsp = jp;
    }
    double* zb = nullptr;   // Schur form: the point vector of a product
    if (schur) {
        // W in FP32 takes half the doubles of FP64 (rounded up)
        d.w32 = o.precision == GBA_MIXED_FP32 ? 1 : 0;
        const size_t wn = (18 * 64 * (size_t)((M + 63) / 64) + 2) / (d.w32 ? 2 : 1);
        const size_t wpn = (18 * 64 * (size_t)(Mp / 64) + 2) / (d.w32 ? 2 : 1);
        int *lp = nullptr, *ls = nullptr;
        double *wk = nullptr, *wp = nullptr;
        if (!B.up(&wk, (const double*)nullptr, wn) || !B.up(&wp, (const double*)nullptr, wpn) ||
            !B.up(&d.icx, (const double*)nullptr, 135 * (size_t)(K - 1)) ||
            !B.up(&d.sm, (const double*)nullptr, 36 * (size_t)K) ||
            !B.up(&zb, (const double*)nullptr, 3 * (size_t)N + 1) ||
            !B.up(&lp, hlong.empty() ? (const int*)nullptr : hlong.data(), hlong.size() + 1) ||
            !B.up(&ls, hlslot.empty() ? (const int*)nullptr : hlslot.data(), hlslot.size() + 1) ||
            !B.up(&d.tb, (const double*)nullptr, 3 * (size_t)N + 1))
            return GBA_ERR_OOM;
        if (hipMemset(d.tb, 0, sizeof(double) * (3 * (size_t)N + 1)) != hipSuccess) return GBA_ERR_HIP;
        d.wk = wk;
        d.wp = wp;
        d.longp = lp;
        d.nlong = (int)hlong.size();
        d.lslot = ls;
        d.nlslot = (long long)hlslot.size();
    }
    d.kf = dkf;
    d.pt = dpt;
    d.obs = obs;
    d.pre = pre;
    d.fx = P.intr[0];
    d.fy = P.intr[1];
    d.cx = P.intr[2];
    d.cy = P.intr[3];
    d.base = P.intr[4];
    d.inv_sigma = 1.0 / P.sigma_px;
    d.delta2 = P.huber_delta2;
    d.wg = 1.0 / (P.sigma_gw * P.sigma_gw);
    d.wa = 1.0 / (P.sigma_aw * P.sigma_aw);
    auto grid = [](long long cnt) { return dim3((unsigned)std::max(1LL, (cnt + 255) / 256)); };
    const dim3 blk(256);
    hipError_t err = hipSuccess;
    auto chk = [&]() {
        if (err == hipSuccess) err = hipGetLastError();
        return err == hipSuccess;
    };
    hipLaunchKernelGGL(k_vi_states_in, grid(K), blk, 0, nullptr, K, s15, d.st);
    hipLaunchKernelGGL(k_vi_info, grid(K - 1), blk, 0, nullptr, K - 1, pre, d.info);
    if (!chk()) return GBA_ERR_HIP;
    double hs[8 + kPcgScalars];
    auto read_scal = [&]() {
        if (err == hipSuccess) err = hipMemcpy(hs, d.scal, sizeof(hs), hipMemcpyDeviceToHost);
        return err == hipSuccess;
    };
    // the reduction slots' parts (each slot's parts summed in index order)
    std::vector<double> hr((size_t)kRedSlots * kPqParts);
    auto read_red = [&]() {
        if (err == hipSuccess)
            err = hipMemcpy(hr.data(), d.scal + kRedOff, hr.size() * sizeof(double), hipMemcpyDeviceToHost);
        return err == hipSuccess;
    };
    auto red_sum = [&](int slot) {
        double t = 0.0;
        for (int i = 0; i < kPqParts; ++i) t += hr[(size_t)slot * kPqParts + i];
        return t;
    };
    auto red_parts = [&](int slot) { return d.scal + kRedOff + (long long)slot * kPqParts; };
    const long long n_scal = kScalN;
    double* ps = d.scal + 8;   // PCG scalars
    auto zero_scal = [&]() {
        hipLaunchKernelGGL(k_vi_fill, grid(n_scal), blk, 0, nullptr, n_scal, d.scal, (const double*)nullptr);
    };
    // cost of (st, X) into slot 0, and |x|^2 into slot 1 when asked
    // cost of (st, X) into slot 0 and, with nst, |x| of (nst, nX) into slot
    // 1, one readback
    auto cost_of = [&](const double* st, const double* X, const double* nst, const double* nX, double& F,
                       double& xn) {
        zero_scal();
        hipLaunchKernelGGL(k_vi_cost, grid(M + K - 1), blk, 0, nullptr, d, st, X, 0);
        if (nst) hipLaunchKernelGGL(k_vi_xnorm, grid(K + N), blk, 0, nullptr, d, nst, nX, 1);
        if (!chk() || !read_red()) return false;
        F = red_sum(0);
        xn = std::sqrt(red_sum(1));
        return true;
    };
    auto linearize = [&]() {
        const double* none = nullptr;
        hipLaunchKernelGGL(k_vi_fill, grid(n), blk, 0, nullptr, n, d.b, none);
        hipLaunchKernelGGL(k_vi_fill, grid(225LL * K), blk, 0, nullptr, 225LL * K, d.hk, none);
        hipLaunchKernelGGL(k_vi_fill, grid(9 * N + 1), blk, 0, nullptr, 9 * N + 1, d.hp, none);
        if (M > 0) hipLaunchKernelGGL(k_vi_lin_stereo, grid(M), blk, 0, nullptr, d);
        if (M > 0) {
            if (d.w32) hipLaunchKernelGGL(k_vi_lin_stereo_pts<float>, grid(Mp), blk, 0, nullptr, d);
            else hipLaunchKernelGGL(k_vi_lin_stereo_pts<double>, grid(Mp), blk, 0, nullptr, d);
        }
        hipLaunchKernelGGL(k_vi_lin_inertial, grid(24LL * (K - 1)), blk, 0, nullptr, d);
        hipLaunchKernelGGL(k_vi_acc_inertial, grid(64LL * (K - 1)), blk, 0, nullptr, d);
        if (schur) hipLaunchKernelGGL(k_vi_cross, grid(135LL * (K - 1)), blk, 0, nullptr, d);
        return chk();
    };
    auto schur_kf = [&](const double* zz, double* out, const double* g) {
        if (M == 0) return;
        if (d.w32) hipLaunchKernelGGL(k_vi_schur_kf<float>, grid(M), blk, 0, nullptr, d, zz, out, g);
        else hipLaunchKernelGGL(k_vi_schur_kf<double>, grid(M), blk, 0, nullptr, d, zz, out, g);
    };
    // q = (H + lam diag(D)) v, the whole system (nothing once g's stop flag is set)
    auto product = [&](const double* v, double* out, double lam, const double* g) {
        hipLaunchKernelGGL(k_vi_prod_damp, grid(n), blk, 0, nullptr, n, lam, d.dg, v, out, g);
        if (M > 0) {
            const dim3 pg((unsigned)((Mp + kFuseBlock - 1) / kFuseBlock));
            if (d.w32) hipLaunchKernelGGL(k_vi_prod_stereo<float>, pg, dim3(kFuseBlock), 0, nullptr, d, v, out, g);
            else hipLaunchKernelGGL(k_vi_prod_stereo<double>, pg, dim3(kFuseBlock), 0, nullptr, d, v, out, g);
        }
        hipLaunchKernelGGL(k_vi_prod_inertial, grid(64LL * (K - 1)), blk, 0, nullptr, d, v, out, g);
    };
    // z = sign C^-1 (B^T v + add) over the points (acc: -t . z added)
    auto schur_pts = [&](const double* v, const double* add, double sign, double* out, const double* g,
                         double* acc) {
        if (M == 0) return;
        double* none_q = nullptr;
        if (d.w32)
            hipLaunchKernelGGL((k_vi_schur_pts<float, false>), grid(Mp), blk, 0, nullptr, d, v, add, sign, out, g,
                               acc, none_q, 0.0);
        else
            hipLaunchKernelGGL((k_vi_schur_pts<double, false>), grid(Mp), blk, 0, nullptr, d, v, add, sign, out, g,
                               acc, none_q, 0.0);
        if (d.nlong > 0)
            hipLaunchKernelGGL(k_vi_long_pts, grid(d.nlong), blk, 0, nullptr, d, add, sign, out, g, acc);
    };
    // q = S v over the keyframes in one pass over the point-order W (the
    // point vector through zb): A v first, then the fused point pass adds
    // -B C^-1 B^T v; acc: v . S v
    // (out is zero on entry: cleared before the PCG and by each direction step)
    const dim3 fuse_grid((unsigned)((Mp + kFuseBlock - 1) / kFuseBlock + (15LL * K + kFuseBlock - 1) / kFuseBlock));
    auto schur_product = [&](const double* v, double* out, double lam, const double* g, double* acc) {
        const double* no_add = nullptr;
        if (d.w32)
            hipLaunchKernelGGL((k_vi_schur_pts<float, true>), fuse_grid, dim3(kFuseBlock), 0, nullptr, d, v, no_add,
                               1.0, zb, g, acc, out, lam);
        else
            hipLaunchKernelGGL((k_vi_schur_pts<double, true>), fuse_grid, dim3(kFuseBlock), 0, nullptr, d, v, no_add,
                               1.0, zb, g, acc, out, lam);
        if (d.nlong > 0) {
            hipLaunchKernelGGL(k_vi_long_pts, grid(d.nlong), blk, 0, nullptr, d, no_add, 1.0, zb, g, acc);
            if (d.w32) hipLaunchKernelGGL(k_vi_long_kf<float>, grid(d.nlslot), blk, 0, nullptr, d, (const double*)zb, out, g);
            else hipLaunchKernelGGL(k_vi_long_kf<double>, grid(d.nlslot), blk, 0, nullptr, d, (const double*)zb, out, g);
        }
    };
    auto dot_blocks = [](long long len) { return dim3((unsigned)std::min<long long>(1024, (len + 255) / 256)); };
    // PCG from 0 to |r| <= pcg_tol |r0|: on (H + lam D) x = -b (full form),
    // or on S x_k = v followed by the point back-substitution (Schur form)
    const long long nn = schur ? 15LL * K : n;          // PCG unknowns
    const long long nm = schur ? 15LL * K : 15LL * K + N;   // preconditioner lanes
    // the PCG runs from its device scalars: its kernels are queued without
    // host round trips, and the stop flag is read every kPcgSync steps (a
    // read drains the queue); the first read comes kPcgSync steps before the
    // previous solve's count, as the next solve usually takes about as many
    constexpr int kPcgSync = 8;
    int prev_iters = 0;
    auto pcg = [&](double lam, int& iters) {
        iters = 0;
        const double* none = nullptr;
        if (schur) {
            hipLaunchKernelGGL(k_vi_precond_pts, grid(N), blk, 0, nullptr, d, lam, o.min_diag, o.max_diag);
            hipLaunchKernelGGL(k_vi_fill, grid(36LL * K), blk, 0, nullptr, 36LL * K, d.sm, none);
            if (M > 0) {
                if (d.w32) hipLaunchKernelGGL(k_vi_schur_blocks<float>, grid(M), blk, 0, nullptr, d);
                else hipLaunchKernelGGL(k_vi_schur_blocks<double>, grid(M), blk, 0, nullptr, d);
            }
            hipLaunchKernelGGL(k_vi_precond_kf, dim3((unsigned)((K + 3) / 4)), blk, 0, nullptr, d, lam, o.min_diag,
                               o.max_diag);
            // r = -b_k + B C^-1 b_p
            hipLaunchKernelGGL(k_vi_pt_apply, grid(N), blk, 0, nullptr, d, (const double*)(d.b + 15 * (size_t)K),
                               -1.0, zb);
            hipLaunchKernelGGL(k_vi_neg, grid(nn), blk, 0, nullptr, nn, d.b, r, x);
            schur_kf(zb, r, none);
        } else {
            hipLaunchKernelGGL(k_vi_precond_pts, grid(N), blk, 0, nullptr, d, lam, o.min_diag, o.max_diag);
            hipLaunchKernelGGL(k_vi_precond_kf, dim3((unsigned)((K + 3) / 4)), blk, 0, nullptr, d, lam, o.min_diag,
                               o.max_diag);
            hipLaunchKernelGGL(k_vi_neg, grid(n), blk, 0, nullptr, n, d.b, r, x);
        }
        zero_scal();
        hipLaunchKernelGGL(k_vi_apply_m, grid(nm), blk, 0, nullptr, d, r, z, none);
        hipLaunchKernelGGL(k_vi_copy, grid(nn), blk, 0, nullptr, nn, (const double*)z, pv);
        hipLaunchKernelGGL(k_vi_dot2, dot_blocks(nn), blk, 0, nullptr, nn, r, z, ps + kAccN * (kSlots - 1));
        const double ratio2 = (o.pcg_rejection_ratio > 0.0 && std::isfinite(o.pcg_rejection_ratio))
                                  ? o.pcg_rejection_ratio * o.pcg_rejection_ratio : 0.0;
        hipLaunchKernelGGL(k_vi_fill, grid(nn), blk, 0, nullptr, nn, xb, none);   // the best iterate: x0 = 0
        if (schur) hipLaunchKernelGGL(k_vi_fill, grid(nn), blk, 0, nullptr, nn, q, none);   // the products add into q
        hipLaunchKernelGGL(k_vi_pcg_init, dim3(1), dim3(1), 0, nullptr, ps, o.pcg_tol, ratio2);
        const long long npt = schur ? 0 : N;
        const dim3 upd((unsigned)((K + 15) / 16 + (npt + kUpdPts - 1) / kUpdPts));
        const dim3 dirg((unsigned)std::max(1LL, std::min<long long>(1024, (nn + 255) / 256)));
        for (int it = 0; it < o.pcg_max_iters; ++it) {
            const int slot = it % kSlots;
            if (schur) {
                schur_product(pv, q, lam, ps, ps + kAccN * slot + kAccPq);   // p . q summed inside
            } else {
                product(pv, q, lam, ps);
                hipLaunchKernelGGL(k_vi_dot, dot_blocks(nn), blk, 0, nullptr, nn, (const double*)pv,
                                   (const double*)q, ps + kAccN * slot + kAccPq, (const double*)ps, kPqParts);
            }
            hipLaunchKernelGGL(k_vi_pcg_update, upd, blk, 0, nullptr, d, npt, ps, slot, (const double*)pv,
                               (const double*)q, x, r, z);
            hipLaunchKernelGGL(k_vi_pcg_dir, dirg, blk, 0, nullptr, nn, ps, slot, (const double*)z, pv, x, xb,
                               schur ? q : nullptr);
            const int first_read = std::max(kPcgSync, prev_iters - kPcgSync);
            if (it + 1 >= first_read && (it + 1 - first_read) % kPcgSync == 0 && it + 1 < o.pcg_max_iters) {
                if (!chk() || !read_scal()) return false;
                if (hs[8 + kDone] != 0.0) break;
            }
        }
        if (schur) {
            // x_p = -C^-1 (b_p + B^T x_k)
            double* xp = x + 15 * (size_t)K;
            hipLaunchKernelGGL(k_vi_fill, grid(3 * N), blk, 0, nullptr, 3 * N, xp, none);
            schur_pts(x, d.b + 15 * (size_t)K, -1.0, xp, none, nullptr);
        }
        if (!chk() || !read_scal()) return false;
        iters = (int)hs[8 + kSteps];
        prev_iters = iters;
        return true;
    };
    gba_report rep{};
    if (hipDeviceSynchronize() != hipSuccess) return GBA_ERR_HIP;
    rep.ms_other = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    rep.workspace_bytes = B.bytes;
    double F = 0.0, xn = 0.0;
    if (!cost_of(d.st, d.X, nullptr, nullptr, F, xn)) return GBA_ERR_HIP;
    rep.initial_cost = F;
    rep.termination = GBA_TERM_MAX_ITERS;
    int nl = 0;
    double lam = o.initial_lambda, nu = 2.0;
    if (!std::isfinite(F)) {
        rep.termination = GBA_TERM_NUMERICAL_FAILURE;
    } else if (max_iters > 0) {
        if (!linearize()) return GBA_ERR_HIP;
        for (int it = 0; it < max_iters; ++it) {
            int iters = 0;
            if (!pcg(lam, iters)) return GBA_ERR_HIP;
            rep.pcg_iters_total += iters;
            // model decrease -(b.dx + 1/2 dx^T H dx) with the undamped H; in
            // the Schur form dx^T H dx = dx_k^T A dx_k + 2 dx_k^T B dx_p
            // + sum_j dx_j^T H_pp,j dx_j from the blocks
            // (the sums into scal slots 0..4, one readback)
            double bdx = 0.0, dHd = 0.0, dd = 0.0;
            const double* cnone = nullptr;
            zero_scal();
            if (schur) {
                const double* xp = x + 15 * (size_t)K;
                hipLaunchKernelGGL(k_vi_schur_ap, grid(15LL * K), blk, 0, nullptr, d, 0.0, (const double*)x, q,
                                   cnone, (double*)nullptr);
                hipLaunchKernelGGL(k_vi_fill, grid(15LL * K), blk, 0, nullptr, 15LL * K, z, cnone);
                schur_kf(xp, z, nullptr);   // z = -B dx_p
                hipLaunchKernelGGL(k_vi_pt_quad, grid(N), blk, 0, nullptr, d, xp, red_parts(2));
                hipLaunchKernelGGL(k_vi_dot, dot_blocks(15LL * K), blk, 0, nullptr, 15LL * K, (const double*)x,
                                   (const double*)q, red_parts(0), cnone, kPqParts);
                hipLaunchKernelGGL(k_vi_dot, dot_blocks(15LL * K), blk, 0, nullptr, 15LL * K, (const double*)x,
                                   (const double*)z, red_parts(1), cnone, kPqParts);
            } else {
                product(x, q, 0.0, nullptr);
                hipLaunchKernelGGL(k_vi_dot, dot_blocks(n), blk, 0, nullptr, n, (const double*)x, (const double*)q,
                                   red_parts(0), cnone, kPqParts);
            }
            hipLaunchKernelGGL(k_vi_dot, dot_blocks(n), blk, 0, nullptr, n, (const double*)d.b, (const double*)x,
                               red_parts(3), cnone, kPqParts);
            hipLaunchKernelGGL(k_vi_dot, dot_blocks(n), blk, 0, nullptr, n, (const double*)x, (const double*)x,
                               red_parts(4), cnone, kPqParts);
            if (!chk() || !read_red()) return GBA_ERR_HIP;
            dHd = schur ? red_sum(0) - 2.0 * red_sum(1) + red_sum(2) : red_sum(0);
            bdx = red_sum(3);
            dd = red_sum(4);
            const double L = -(bdx + 0.5 * dHd);
            hipLaunchKernelGGL(k_vi_step, grid(K + N), blk, 0, nullptr, d, x);
            double Fn = 0.0, xnorm = 0.0;
            if (!cost_of(d.st_c, d.X_c, d.st, d.X, Fn, xnorm))   // candidate cost, current |x|
                return GBA_ERR_HIP;
            const double dnorm = std::sqrt(dd);
            const bool accepted = L > 0.0 && Fn < F;
            const double gain = L != 0.0 ? (F - Fn) / L : NAN;
            if (nl < max_log) log[nl++] = gba_trial{F, Fn, lam, L, dnorm, accepted ? 1 : 0, iters};
            rep.trials += 1;
            int stop = 0;
            if (accepted) {
                rep.accepted += 1;
                const double rel = (F - Fn) / F;
                std::swap(d.st, d.st_c);
                std::swap(d.X, d.X_c);
                F = Fn;
                lam *= std::max(1.0 / 3.0, 1.0 - std::pow(2.0 * gain - 1.0, 3));
                nu = 2.0;
                if (rel < tol) stop = GBA_TERM_COST_TOL;
            } else {
                lam *= nu;
                nu *= 2.0;
            }
            if (!stop && dnorm <= tol * (xnorm + tol)) stop = GBA_TERM_STEP_TOL;
            if (!stop && lam > 1e32) stop = GBA_TERM_LAMBDA_OVERFLOW;
            if (stop) {
                rep.termination = stop;
                break;
            }
            if (accepted && !linearize()) return GBA_ERR_HIP;
        }
    }
    rep.final_cost = F;
    rep.final_lambda = lam;
    hipLaunchKernelGGL(k_vi_states_out, grid(K), blk, 0, nullptr, K, d.st, s15);
    if (!chk()) return GBA_ERR_HIP;
    if (hipMemcpy(P.states, s15, sizeof(double) * 15 * K, hipMemcpyDeviceToHost) != hipSuccess ||
        (N > 0 && hipMemcpy(hX.data(), d.X, sizeof(double) * 3 * N, hipMemcpyDeviceToHost) != hipSuccess))
        return GBA_ERR_HIP;
    for (int64_t q = 0; q < N; ++q)
        for (int c = 0; c < 3; ++c) P.pts[3 * (size_t)pt_old[q] + c] = hX[3 * q + c];
    rep.ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    if (report) *report = rep;
    if (n_log) *n_log = nl;
    return GBA_OK;
}

}  // extern "C"
