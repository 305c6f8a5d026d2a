"""Seeded synthetic visual-inertial inputs (the stereo-inertial configuration:
keyframes along a smooth trajectory, a 200 Hz IMU between them, map points
seen by a rectified stereo pair).

Like synth.py this module only draws inputs: a true trajectory, IMU samples
synthesised from its analytic derivatives plus white noise and a bias random
walk, points near the path, and stereo pixel measurements of the true scene.
It holds none of the method's arithmetic (no preintegration, residual or
derivative) and imports nothing from the solver or the CPU checker.

Trajectory: position a sum of sinusoids (about 1.5 m/s), orientation
ZYX angles that follow the heading with small roll and pitch oscillations;
body angular velocity from the rotation's time derivative (central
difference at 1e-6 s), specific force = R^T (acceleration - g).
"""
from dataclasses import dataclass

import numpy as np
from scipy.spatial.transform import Rotation

G_WORLD = np.array([0.0, 0.0, -9.81])


@dataclass
class VIScene:
    n_kf: int
    kf_dt: float
    imu_dt: float
    R_true: np.ndarray       # (n_kf, 3, 3) world <- body
    p_true: np.ndarray       # (n_kf, 3)
    v_true: np.ndarray       # (n_kf, 3)
    bg_true: np.ndarray      # (n_kf, 3)
    ba_true: np.ndarray      # (n_kf, 3)
    gyro: np.ndarray         # (n_kf - 1, m, 3) samples of each interval
    acc: np.ndarray          # (n_kf - 1, m, 3)
    pts: np.ndarray          # (n_pts, 3)
    st_kf: np.ndarray        # (n_obs,) keyframe of each stereo observation
    st_pt: np.ndarray        # (n_obs,) point
    st_obs: np.ndarray       # (n_obs, 3) u_l, v_l, u_r
    intr: tuple              # fx, fy, cx, cy, baseline


def _traj(t, rng_par):
    amp, freq, phase = rng_par
    p = (amp[:, None] * np.sin(freq[:, None] * t[None, :] + phase[:, None])).sum(axis=0)
    return p


def _pose(t, par):
    """Position (3,) and rotation of the body at time t."""
    px = _traj(np.atleast_1d(t), par[0])[0]
    py = _traj(np.atleast_1d(t), par[1])[0]
    pz = _traj(np.atleast_1d(t), par[2])[0]
    yaw = 0.4 * np.sin(0.3 * t) + 0.1 * t
    pitch = 0.05 * np.sin(0.9 * t + 0.3)
    roll = 0.05 * np.sin(1.1 * t + 1.0)
    R = Rotation.from_euler("ZYX", [yaw, pitch, roll]).as_matrix()
    return np.array([px, py, pz]), R


def make_vi_scene(seed=0, n_kf=20, kf_dt=0.25, rate=200, n_pts=400, gyro_noise=1.7e-4,
                  acc_noise=2e-3, gyro_walk=2e-5, acc_walk=3e-3, pixel_noise=1.0,
                  intr=(380.0, 380.0, 320.0, 240.0, 0.11), max_depth=20.0):
    rng = np.random.default_rng(seed)
    # position: three sinusoids per axis, amplitudes scaled for ~1.5 m/s
    par = [(rng.uniform(1.0, 4.0, 3), rng.uniform(0.05, 0.4, 3), rng.uniform(0, 2 * np.pi, 3))
           for _ in range(3)]
    imu_dt = 1.0 / rate
    m = int(round(kf_dt * rate))
    h = 1e-6

    def state(t):
        p, R = _pose(t, par)
        p1, R1 = _pose(t + h, par)
        p0, R0 = _pose(t - h, par)
        v = (p1 - p0) / (2 * h)
        a = (p1 - 2 * p + p0) / (h * h)
        Rdot = (R1 - R0) / (2 * h)
        W = R.T @ Rdot
        w = 0.5 * np.array([W[2, 1] - W[1, 2], W[0, 2] - W[2, 0], W[1, 0] - W[0, 1]])
        return p, R, v, a, w

    n_int = n_kf - 1
    gyro = np.zeros((n_int, m, 3))
    acc = np.zeros((n_int, m, 3))
    bg = np.zeros((n_kf, 3))
    ba = np.zeros((n_kf, 3))
    bg[0] = rng.normal(scale=0.01, size=3)
    ba[0] = rng.normal(scale=0.05, size=3)
    Rk, pk, vk = [], [], []
    for k in range(n_kf):
        p, R, v, _, _ = state(k * kf_dt)
        Rk.append(R)
        pk.append(p)
        vk.append(v)
    for i in range(n_int):
        # biases held per interval, random walk between keyframes
        bg[i + 1] = bg[i] + rng.normal(scale=gyro_walk * np.sqrt(kf_dt), size=3)
        ba[i + 1] = ba[i] + rng.normal(scale=acc_walk * np.sqrt(kf_dt), size=3)
        for s in range(m):
            t = i * kf_dt + (s + 0.5) * imu_dt
            _, R, _, a, w = state(t)
            gyro[i, s] = w + bg[i] + rng.normal(scale=gyro_noise / np.sqrt(imu_dt), size=3)
            acc[i, s] = R.T @ (a - G_WORLD) + ba[i] + rng.normal(scale=acc_noise / np.sqrt(imu_dt),
                                                                 size=3)
    Rk, pk, vk = np.array(Rk), np.array(pk), np.array(vk)
    # points: near the path, seen by the keyframes that have them in front
    # at depth 2..max_depth and inside the image
    fx, fy, cx, cy, base = intr
    anchor = rng.integers(0, n_kf, size=n_pts)
    pts = np.zeros((n_pts, 3))
    for q in range(n_pts):
        dirc = np.array([rng.uniform(-0.5, 0.5), rng.uniform(-0.4, 0.4), 1.0])
        pts[q] = pk[anchor[q]] + Rk[anchor[q]] @ (dirc * rng.uniform(2.0, max_depth))
    kf_l, pt_l, ob_l = [], [], []
    for k in range(n_kf):
        Xc = (pts - pk[k]) @ Rk[k]            # R^T (X - p), row-wise
        z = Xc[:, 2]
        ok = (z > 2.0) & (z < max_depth)
        u = fx * Xc[:, 0] / np.where(ok, z, 1.0) + cx
        v = fy * Xc[:, 1] / np.where(ok, z, 1.0) + cy
        ok &= (u > 0) & (u < 2 * cx) & (v > 0) & (v < 2 * cy)
        for q in np.flatnonzero(ok):
            ur = u[q] - fx * base / z[q]
            kf_l.append(k)
            pt_l.append(q)
            ob_l.append([u[q], v[q], ur] + rng.normal(scale=pixel_noise, size=3))
    return VIScene(n_kf=n_kf, kf_dt=kf_dt, imu_dt=imu_dt, R_true=Rk, p_true=pk, v_true=vk,
                   bg_true=bg, ba_true=ba, gyro=gyro, acc=acc, pts=pts,
                   st_kf=np.array(kf_l, np.int64), st_pt=np.array(pt_l, np.int64),
                   st_obs=np.array(ob_l, float), intr=intr)
