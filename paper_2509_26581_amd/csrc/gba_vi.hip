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

#include <cmath>
#include <vector>

#include "gba.h"
#include "gba_autodiff.h"

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

}  // namespace vi
}  // namespace gba

// ------------------------------------------------------------------ C ABI
namespace {

// Device buffers of one call, released on every return path.
struct DevBufs {
    std::vector<void*> p;
    ~DevBufs() {
        for (void* q : p) (void)hipFree(q);
    }
    template <typename T>
    bool up(T** dst, const T* src, size_t n) {
        void* q = nullptr;
        if (hipMalloc(&q, n * sizeof(T) + 16) != hipSuccess) return false;
        p.push_back(q);
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

}  // extern "C"
