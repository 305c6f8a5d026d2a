// Forward-mode automatic differentiation of the bundle-adjustment residual
// (Sec. IV-C): the residual is written once, generically over its scalar
// type; evaluated on dual numbers a + b eps (eps^2 = 0) whose infinitesimal
// part seeds one input parameter, it yields one column of the edge's
// Jacobian.  No dual-number storage is allocated: the duals live in
// registers for one evaluation.
#pragma once

#include <hip/hip_runtime.h>

namespace gba {

template <typename T>
struct Dual {
    T v;   // value
    T d;   // derivative along the seeded input
};

template <typename T>
__device__ __forceinline__ Dual<T> operator+(Dual<T> a, Dual<T> b) { return {a.v + b.v, a.d + b.d}; }
template <typename T>
__device__ __forceinline__ Dual<T> operator-(Dual<T> a, Dual<T> b) { return {a.v - b.v, a.d - b.d}; }
template <typename T>
__device__ __forceinline__ Dual<T> operator-(Dual<T> a) { return {-a.v, -a.d}; }
template <typename T>
__device__ __forceinline__ Dual<T> operator*(Dual<T> a, Dual<T> b) {
    return {a.v * b.v, a.d * b.v + a.v * b.d};
}
template <typename T>
__device__ __forceinline__ Dual<T> operator/(Dual<T> a, Dual<T> b) {
    const T q = a.v / b.v;
    return {q, (a.d - q * b.d) / b.v};
}
template <typename T>
__device__ __forceinline__ Dual<T> operator+(Dual<T> a, T b) { return {a.v + b, a.d}; }
template <typename T>
__device__ __forceinline__ Dual<T> operator+(T a, Dual<T> b) { return {a + b.v, b.d}; }
template <typename T>
__device__ __forceinline__ Dual<T> operator-(Dual<T> a, T b) { return {a.v - b, a.d}; }
template <typename T>
__device__ __forceinline__ Dual<T> operator-(T a, Dual<T> b) { return {a - b.v, -b.d}; }
template <typename T>
__device__ __forceinline__ Dual<T> operator*(Dual<T> a, T b) { return {a.v * b, a.d * b}; }
template <typename T>
__device__ __forceinline__ Dual<T> operator*(T a, Dual<T> b) { return {a * b.v, a * b.d}; }
template <typename T>
__device__ __forceinline__ Dual<T> operator/(Dual<T> a, T b) { return {a.v / b, a.d / b}; }
template <typename T>
__device__ __forceinline__ Dual<T> operator/(T a, Dual<T> b) {
    const T q = a / b.v;
    return {q, -q * b.d / b.v};
}

template <typename T>
__device__ __forceinline__ Dual<T> ad_sqrt(Dual<T> a) {
    const T s = sqrt(a.v);
    return {s, a.d / (T(2) * s)};
}
template <typename T>
__device__ __forceinline__ Dual<T> ad_sin(Dual<T> a) { return {sin(a.v), cos(a.v) * a.d}; }
template <typename T>
__device__ __forceinline__ Dual<T> ad_cos(Dual<T> a) { return {cos(a.v), -sin(a.v) * a.d}; }
template <typename T>
__device__ __forceinline__ Dual<T> ad_atan2(Dual<T> y, Dual<T> x) {
    const T den = x.v * x.v + y.v * y.v;
    return {atan2(y.v, x.v), (x.v * y.d - y.v * x.d) / den};
}
template <typename T>
__device__ __forceinline__ T ad_sqrt(T a) { return sqrt(a); }
template <typename T>
__device__ __forceinline__ T ad_sin(T a) { return sin(a); }
template <typename T>
__device__ __forceinline__ T ad_cos(T a) { return cos(a); }
template <typename T>
__device__ __forceinline__ T ad_atan2(T y, T x) { return atan2(y, x); }

template <typename T>
__device__ __forceinline__ T ad_value(Dual<T> a) { return a.v; }
template <typename T>
__device__ __forceinline__ T ad_value(T a) { return a; }

// The BAL residual r = f d p - u of camera c = (w, t, f, k1, k2) and point
// X, generic over the scalar type S (T or Dual<T>).  R(w) X = X + a (w x X)
// + b w x (w x X) with a = sin(th)/th and b = (1 - cos th)/th^2 as functions
// of t = th^2: below th = 1e-2 by their Taylor series in t (so that their
// derivatives carry no cancellation), and for t <= 1e-16 the first-order
// rotation X + w x X (the same branches as the closed form).  The branch is
// chosen on the value part.
template <typename T, typename S>
__device__ __forceinline__ void bal_residual_generic(const S (&c)[9], const S (&X)[3], double ou,
                                                     double ov, S (&r)[2]) {
    const S t = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
    const T tv = ad_value(t);
    const S wx0 = c[1] * X[2] - c[2] * X[1];
    const S wx1 = c[2] * X[0] - c[0] * X[2];
    const S wx2 = c[0] * X[1] - c[1] * X[0];
    S P0, P1, P2;
    if (tv > T(1e-16)) {
        S a, b;
        if (tv < T(1e-4)) {
            // a = sum (-t)^k / (2k+1)!,  b = sum (-t)^k / (2k+2)!
            a = T(1) - t * (T(1) / T(6) - t * (T(1) / T(120) - t * (T(1) / T(5040))));
            b = T(0.5) - t * (T(1) / T(24) - t * (T(1) / T(720) - t * (T(1) / T(40320))));
        } else {
            const S th = ad_sqrt(t);
            const S hs = ad_sin(th * T(0.5));
            a = ad_sin(th) / th;
            b = T(2) * hs * hs / t;
        }
        const S ww0 = c[1] * wx2 - c[2] * wx1;
        const S ww1 = c[2] * wx0 - c[0] * wx2;
        const S ww2 = c[0] * wx1 - c[1] * wx0;
        P0 = X[0] + a * wx0 + b * ww0 + c[3];
        P1 = X[1] + a * wx1 + b * ww1 + c[4];
        P2 = X[2] + a * wx2 + b * ww2 + c[5];
    } else {
        P0 = X[0] + wx0 + c[3];
        P1 = X[1] + wx1 + c[4];
        P2 = X[2] + wx2 + c[5];
    }
    const S px = -(P0 / P2), py = -(P1 / P2);
    const S n = px * px + py * py;
    const S d = T(1) + c[7] * n + c[8] * n * n;
    const S fd = c[6] * d;
    r[0] = fd * px - T(ou);
    r[1] = fd * py - T(ov);
}

// One Jacobian column of an edge: column k of (dr/dc | dr/dX) (k < 9: camera
// parameter k, else point coordinate k - 9), and the residual value.
template <typename T>
__device__ __forceinline__ void bal_jacobian_column(const double* __restrict__ cam,
                                                    const double* __restrict__ pt, double ou,
                                                    double ov, int k, T (&r)[2], T (&col)[2]) {
    Dual<T> c[9], X[3], rr[2];
#pragma unroll
    for (int i = 0; i < 9; ++i) c[i] = {T(cam[i]), T(i == k ? 1 : 0)};
#pragma unroll
    for (int i = 0; i < 3; ++i) X[i] = {T(pt[i]), T(9 + i == k ? 1 : 0)};
    bal_residual_generic<T>(c, X, ou, ov, rr);
    r[0] = rr[0].v;
    r[1] = rr[1].v;
    col[0] = rr[0].d;
    col[1] = rr[1].d;
}

}  // namespace gba
