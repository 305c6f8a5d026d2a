"""BAL camera model, written plainly (test infrastructure, FP64).

The paper benchmarks on BAL problems (Sec. V, Table I) but never writes the
camera model out; the reading used throughout this project is the BAL one:

  camera c = (w in R^3 angle-axis, t in R^3, f, k1, k2)
  P = R(w) X + t                     R(w) by the Rodrigues formula
  p = -(P_x / P_z, P_y / P_z)        BAL looks down -z
  d = 1 + k1 |p|^2 + k2 |p|^4        radial distortion
  proj = f d p                       pixels
  r = proj - u                       residual = prediction minus measurement
                                     (Background: projection minus observation)

Small rotations: when |w|^2 <= THETA2_MIN the rotation is taken to first order,
R(w) X = X + w x X, and its derivative is that of the first-order form.

All functions accept plain float arrays or oracle.dual.Dual objects, so the
same code yields values and (through dual numbers) exact Jacobians.
"""
import numpy as np

from . import dual as D

THETA2_MIN = 1e-16


def _cross(a, b):
    return [a[1] * b[2] - a[2] * b[1],
            a[2] * b[0] - a[0] * b[2],
            a[0] * b[1] - a[1] * b[0]]


def rotate(w, X):
    """R(w) X for angle-axis w (3 components) and point X (3 components)."""
    th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2]
    big = D.value(th2) > THETA2_MIN
    th = D.sqrt(D.where(big, th2, 1.0))
    c = D.cos(th)
    s = D.sin(th)
    k = [w[i] / th for i in range(3)]
    kx = _cross(k, X)
    kd = k[0] * X[0] + k[1] * X[1] + k[2] * X[2]
    one_c = 1.0 - c
    full = [X[i] * c + kx[i] * s + k[i] * kd * one_c for i in range(3)]
    wx = _cross(w, X)
    first = [X[i] + wx[i] for i in range(3)]
    return [D.where(big, full[i], first[i]) for i in range(3)]


def project(cam, X):
    """BAL projection of point X (3 comps) by camera cam (9 comps) -> 2 comps."""
    P = rotate(cam[0:3], X)
    P = [P[i] + cam[3 + i] for i in range(3)]
    px = -(P[0] / P[2])
    py = -(P[1] / P[2])
    n = px * px + py * py
    d = 1.0 + cam[7] * n + cam[8] * n * n
    fd = cam[6] * d
    return [fd * px, fd * py]


def residuals(cams, pts, cam_idx, pt_idx, obs):
    """Residuals r_e = proj(cam[cam_idx[e]], pts[pt_idx[e]]) - obs[e]; (N, 2)."""
    c = cams[cam_idx]
    x = pts[pt_idx]
    pr = project([c[:, k] for k in range(9)], [x[:, k] for k in range(3)])
    return np.stack([pr[0] - obs[:, 0], pr[1] - obs[:, 1]], axis=1)


def residuals_and_jacobians(cams, pts, cam_idx, pt_idx, obs):
    """Residuals (N,2) and their Jacobians w.r.t. the 9 camera parameters
    (N,2,9) and the 3 point coordinates (N,2,3), by forward-mode dual numbers."""
    params = np.concatenate([cams[cam_idx], pts[pt_idx]], axis=1)   # (N, 12)
    v = D.seed(params)
    pr = project(v[0:9], v[9:12])
    r = np.stack([pr[0].v - obs[:, 0], pr[1].v - obs[:, 1]], axis=1)
    J = np.stack([pr[0].d, pr[1].d], axis=1)                          # (N, 2, 12)
    return r, J[:, :, :9].copy(), J[:, :, 9:].copy()
