"""Visual-inertial factors (test infrastructure, FP64, plain numpy).

The paper's visual-inertial bundle adjustment (Background, Eq. 8; Sec. V-C)
adds to the reprojection terms an inertial residual between consecutive
keyframes (the preintegrated IMU measurements against the change of rotation,
velocity and position computed from the keyframe states) and a bias residual
(gyroscope and accelerometer random walk), and uses stereo reprojection.  The
paper takes these definitions from the SLAM system it is embedded in; they are
restated here from the published on-manifold preintegration method (discrete
propagation of the rotation, velocity and position deltas, their first-order
bias Jacobians and the noise covariance, Forster et al.).

Readings (listed in the design notes):
  * keyframe state: rotation R (world <- body), position p, velocity v (world
    frame), gyroscope bias b_g, accelerometer bias b_a;
  * perturbation for Jacobians: R <- R Exp(dtheta) (right), p, v, b additive;
  * gravity g = (0, 0, -9.81) in the world frame;
  * stereo: rectified pinhole pair, camera frame = body frame, right camera
    shifted by the baseline along +x: residual (u_l, v_l, u_r) - observation.

Generic over oracle.dual.Dual so that the same code gives exact Jacobians.
"""
import numpy as np

from . import dual as D

GRAVITY = np.array([0.0, 0.0, -9.81])
SMALL = 1e-8     # |phi|^2 below which Exp / Log use their series


# ------------------------------------------------------------ SO(3), plain
def skew(v):
    return np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])


def so3_exp(phi):
    phi = np.asarray(phi, float)
    t2 = float(phi @ phi)
    K = skew(phi)
    if t2 < SMALL:
        a, b = 1.0 - t2 / 6.0, 0.5 - t2 / 24.0
    else:
        t = np.sqrt(t2)
        a, b = np.sin(t) / t, (1.0 - np.cos(t)) / t2
    return np.eye(3) + a * K + b * (K @ K)


def so3_log(R):
    c = np.clip(0.5 * (np.trace(R) - 1.0), -1.0, 1.0)
    v = 0.5 * np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
    s = np.linalg.norm(v)
    t = np.arctan2(s, c)
    return v * (1.0 + s * s / 6.0) if s < 1e-8 else v * (t / s)


def right_jacobian(phi):
    phi = np.asarray(phi, float)
    t2 = float(phi @ phi)
    K = skew(phi)
    if t2 < SMALL:
        return np.eye(3) - 0.5 * K + (K @ K) / 6.0
    t = np.sqrt(t2)
    return np.eye(3) - (1.0 - np.cos(t)) / t2 * K + (t - np.sin(t)) / (t2 * t) * (K @ K)


# ------------------------------------------------------------ preintegration
class Preintegrated:
    """Deltas between two keyframes: dt, dR, dv, dp; bias Jacobians JRg, Jvg,
    Jva, Jpg, Jpa; covariance cov (9 x 9 over [dphi, dv, dp]); the biases the
    measurements were integrated with (bg0, ba0)."""
    pass


def preintegrate(gyro, acc, dt, bg0, ba0, sigma_g=0.0, sigma_a=0.0):
    """Integrate n IMU samples (gyro, acc: (n, 3), one every dt seconds) with
    the bias estimates bg0, ba0.  Each step uses the deltas before it:
        dp += dv dt + 1/2 dR a dt^2,  dv += dR a dt,  dR = dR Exp(w dt)
    with w = gyro - bg0, a = acc - ba0; the bias Jacobians and the covariance
    (continuous noise densities sigma_g, sigma_a) are propagated alongside."""
    P = Preintegrated()
    dR, dv, dp = np.eye(3), np.zeros(3), np.zeros(3)
    JRg = np.zeros((3, 3))
    Jvg, Jva, Jpg, Jpa = (np.zeros((3, 3)) for _ in range(4))
    cov = np.zeros((9, 9))
    qg, qa = sigma_g ** 2 / dt, sigma_a ** 2 / dt
    for w_m, a_m in zip(np.asarray(gyro, float), np.asarray(acc, float)):
        w = w_m - bg0
        a = a_m - ba0
        Ra = dR @ a
        Rax = dR @ skew(a)
        dRk = so3_exp(w * dt)
        Jrk = right_jacobian(w * dt)
        # covariance over [dphi, dv, dp] with the deltas before the step
        A = np.eye(9)
        A[0:3, 0:3] = dRk.T
        A[3:6, 0:3] = -Rax * dt
        A[6:9, 0:3] = -0.5 * Rax * dt * dt
        A[6:9, 3:6] = np.eye(3) * dt
        Bg = np.zeros((9, 3))
        Bg[0:3] = Jrk * dt
        Ba = np.zeros((9, 3))
        Ba[3:6] = dR * dt
        Ba[6:9] = 0.5 * dR * dt * dt
        cov = A @ cov @ A.T + qg * (Bg @ Bg.T) + qa * (Ba @ Ba.T)
        # bias Jacobians (position, velocity, then rotation)
        Jpa = Jpa + Jva * dt - 0.5 * dR * dt * dt
        Jpg = Jpg + Jvg * dt - 0.5 * Rax @ JRg * dt * dt
        Jva = Jva - dR * dt
        Jvg = Jvg - Rax @ JRg * dt
        JRg = dRk.T @ JRg - Jrk * dt
        # deltas
        dp = dp + dv * dt + 0.5 * Ra * dt * dt
        dv = dv + Ra * dt
        dR = dR @ dRk
    P.dt = dt * len(gyro)
    P.dR, P.dv, P.dp = dR, dv, dp
    P.JRg, P.Jvg, P.Jva, P.Jpg, P.Jpa = JRg, Jvg, Jva, Jpg, Jpa
    P.cov = 0.5 * (cov + cov.T)
    P.bg0, P.ba0 = np.asarray(bg0, float), np.asarray(ba0, float)
    return P


# ------------------------------------------------------ generic 3x3 algebra
def _s(x):
    """numpy scalars as Python floats (so that they combine with Duals)."""
    return float(x) if isinstance(x, (np.floating, np.integer, float, int)) else x


def _vec(v):
    return [_s(v[k]) for k in range(3)]


def _mat(M):
    return [[_s(M[r][c]) for c in range(3)] for r in range(3)]


def _mm(A, B):
    return [[A[r][0] * B[0][c] + A[r][1] * B[1][c] + A[r][2] * B[2][c] for c in range(3)]
            for r in range(3)]


def _mtm(A, B):
    """A^T B"""
    return [[A[0][r] * B[0][c] + A[1][r] * B[1][c] + A[2][r] * B[2][c] for c in range(3)]
            for r in range(3)]


def _mv(A, v):
    return [A[r][0] * v[0] + A[r][1] * v[1] + A[r][2] * v[2] for r in range(3)]


def _mtv(A, v):
    return [A[0][r] * v[0] + A[1][r] * v[1] + A[2][r] * v[2] for r in range(3)]


def _skew_g(v):
    z = 0.0 * v[0]
    return [[z, -v[2], v[1]], [v[2], z, -v[0]], [-v[1], v[0], z]]


def _exp_g(phi):
    """Exp of a generic 3-vector (elements Dual or float, vectorised)."""
    t2 = phi[0] * phi[0] + phi[1] * phi[1] + phi[2] * phi[2]
    small = D.value(t2) < SMALL
    t = D.sqrt(D.where(small, 1.0 + 0.0 * D.value(t2), t2))
    a = D.where(small, 1.0 - t2 / 6.0, D.sin(t) / t)
    b = D.where(small, 0.5 - t2 / 24.0, (1.0 - D.cos(t)) / (t * t))
    K = _skew_g(phi)
    K2 = _mm(K, K)
    return [[(1.0 if r == c else 0.0) + a * K[r][c] + b * K2[r][c] for c in range(3)]
            for r in range(3)]


def _atan2(y, x):
    if not isinstance(y, D.Dual) and not isinstance(x, D.Dual):
        return np.arctan2(y, x)
    yv, yd = D.Dual._split(y)
    xv, xd = D.Dual._split(x)
    den = xv * xv + yv * yv
    k = (yd if yd is not None else xd).shape[-1]
    n = yv.shape[0]
    yd = np.zeros((n, k)) if yd is None else yd
    xd = np.zeros((n, k)) if xd is None else xd
    return D.Dual(np.arctan2(yv, xv), (xv[..., None] * yd - yv[..., None] * xd) / den[..., None])


def _log_g(R):
    """Log of a generic rotation matrix: theta = atan2(|v|, (tr R - 1)/2) with
    v the axial part; theta / sin(theta) by its series near 0."""
    c = 0.5 * (R[0][0] + R[1][1] + R[2][2] - 1.0)
    v = [0.5 * (R[2][1] - R[1][2]), 0.5 * (R[0][2] - R[2][0]), 0.5 * (R[1][0] - R[0][1])]
    s2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2]
    small = D.value(s2) < SMALL
    s = D.sqrt(D.where(small, 1.0 + 0.0 * D.value(s2), s2))
    f = D.where(small, 1.0 + s2 / 6.0 + 0.075 * s2 * s2, _atan2(s, c) / s)
    return [v[k] * f for k in range(3)]


# ------------------------------------------------------------ residuals
def inertial_residual(Ri, pi, vi, bgi, bai, Rj, pj, vj, pre, g=GRAVITY):
    """r = (r_R, r_v, r_p), 9 components (generic):
        r_R = Log((dR Exp(JRg dbg))^T Ri^T Rj)
        r_v = Ri^T (vj - vi - g dt) - (dv + Jvg dbg + Jva dba)
        r_p = Ri^T (pj - pi - vi dt - 1/2 g dt^2) - (dp + Jpg dbg + Jpa dba)
    with dbg = bgi - bg0, dba = bai - ba0 (first-order bias correction)."""
    dt = float(pre.dt)
    Ri, Rj = _mat(Ri), _mat(Rj)
    pi, vi, bgi, bai, pj, vj = (_vec(x) for x in (pi, vi, bgi, bai, pj, vj))
    g = _vec(g)
    dbg = [bgi[k] - float(pre.bg0[k]) for k in range(3)]
    dba = [bai[k] - float(pre.ba0[k]) for k in range(3)]
    corr = _mv(_mat(pre.JRg), dbg)
    dRc = _mm(_mat(pre.dR), _exp_g(corr))
    E = _mtm(dRc, _mtm(Ri, Rj))           # dRc^T Ri^T Rj
    rR = _log_g(E)
    dvc = [float(pre.dv[k]) + _mv(_mat(pre.Jvg), dbg)[k] + _mv(_mat(pre.Jva), dba)[k] for k in range(3)]
    dpc = [float(pre.dp[k]) + _mv(_mat(pre.Jpg), dbg)[k] + _mv(_mat(pre.Jpa), dba)[k] for k in range(3)]
    wv = [vj[k] - vi[k] - g[k] * dt for k in range(3)]
    wp = [pj[k] - pi[k] - vi[k] * dt - 0.5 * g[k] * dt * dt for k in range(3)]
    rv = [x - y for x, y in zip(_mtv(Ri, wv), dvc)]
    rp = [x - y for x, y in zip(_mtv(Ri, wp), dpc)]
    return rR + rv + rp


def bias_residual(bgi, bai, bgj, baj):
    """Random walk of the biases between consecutive keyframes (6 comps)."""
    return [bgj[k] - bgi[k] for k in range(3)] + [baj[k] - bai[k] for k in range(3)]


def stereo_residual(R, p, X, fx, fy, cx, cy, base, obs):
    """Rectified stereo reprojection of world point X by the keyframe (R, p)
    (world <- body = camera): Xc = R^T (X - p); u_l = fx Xc_x / Xc_z + cx,
    v_l = fy Xc_y / Xc_z + cy, u_r = u_l - fx base / Xc_z; minus obs (3)."""
    R, p, X = _mat(R), _vec(p), _vec(X)
    fx, fy, cx, cy, base = (float(x) for x in (fx, fy, cx, cy, base))
    Xc = _mtv(R, [X[k] - p[k] for k in range(3)])
    inv = 1.0 / Xc[2]
    ul = fx * Xc[0] * inv + cx
    vl = fy * Xc[1] * inv + cy
    ur = ul - fx * base * inv
    return [ul - float(obs[0]), vl - float(obs[1]), ur - float(obs[2])]


# ----------------------------------------------------- Jacobians by duals
STATE_COLS = ("dtheta_i", "dp_i", "dv_i", "dbg_i", "dba_i", "dtheta_j", "dp_j", "dv_j")


def _perturbed_rot(R, d):
    """R (I + [d]x): the first-order right perturbation R Exp(d) at d = 0."""
    K = _skew_g(d)
    return [[R[r][0] * ((1.0 if c == 0 else 0.0) + K[0][c]) +
             R[r][1] * ((1.0 if c == 1 else 0.0) + K[1][c]) +
             R[r][2] * ((1.0 if c == 2 else 0.0) + K[2][c]) for c in range(3)] for r in range(3)]


def inertial_residual_and_jacobian(Ri, pi, vi, bgi, bai, Rj, pj, vj, pre, g=GRAVITY):
    """Residual (9,) and Jacobian (9, 24) of one inertial factor with respect
    to the local perturbations in STATE_COLS order (3 columns each)."""
    z = D.seed(np.zeros((1, 24)))
    Ri_ = _perturbed_rot(_mat(Ri), z[0:3])
    Rj_ = _perturbed_rot(_mat(Rj), z[15:18])
    pi_ = [float(pi[k]) + z[3 + k] for k in range(3)]
    vi_ = [float(vi[k]) + z[6 + k] for k in range(3)]
    bg_ = [float(bgi[k]) + z[9 + k] for k in range(3)]
    ba_ = [float(bai[k]) + z[12 + k] for k in range(3)]
    pj_ = [float(pj[k]) + z[18 + k] for k in range(3)]
    vj_ = [float(vj[k]) + z[21 + k] for k in range(3)]
    r = inertial_residual(Ri_, pi_, vi_, bg_, ba_, Rj_, pj_, vj_, pre, g)
    return (np.array([float(x.v[0]) for x in r]),
            np.stack([x.d[0] for x in r]))


def stereo_residual_and_jacobian(R, p, X, fx, fy, cx, cy, base, obs):
    """Residual (3,) and Jacobian (3, 9): columns dtheta, dp of the keyframe,
    then dX of the point."""
    z = D.seed(np.zeros((1, 9)))
    R_ = _perturbed_rot(_mat(R), z[0:3])
    p_ = [float(p[k]) + z[3 + k] for k in range(3)]
    X_ = [float(X[k]) + z[6 + k] for k in range(3)]
    r = stereo_residual(R_, p_, X_, fx, fy, cx, cy, base, obs)
    return np.array([float(x.v[0]) for x in r]), np.stack([x.d[0] for x in r])
