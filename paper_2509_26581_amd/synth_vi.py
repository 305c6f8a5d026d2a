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
difference at 1e-6 s), specific force = R^T (acceleration - g).  With
`window`, a point is seen only by keyframes within that many of its anchor
keyframe (the sliding-window visibility of a long trajectory: about 2M
observations for 2,000 keyframes and 300k points at window 3).
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
    return (amp[:, None] * np.sin(freq[:, None] * t[None, :] + phase[:, None])).sum(axis=0)


def _poses(t, par):
    """Positions (n, 3) and rotations (n, 3, 3) of the body at times t (n,)."""
    t = np.atleast_1d(np.asarray(t, float))
    p = np.stack([_traj(t, par[0]), _traj(t, par[1]), _traj(t, par[2])], axis=1)
    yaw = 0.4 * np.sin(0.3 * t) + 0.1 * t
    pitch = 0.05 * np.sin(0.9 * t + 0.3)
    roll = 0.05 * np.sin(1.1 * t + 1.0)
    R = Rotation.from_euler("ZYX", np.stack([yaw, pitch, roll], axis=1)).as_matrix()
    return p, R


def make_vi_scene(seed=0, n_kf=20, kf_dt=0.25, rate=200, n_pts=400, gyro_noise=1.7e-4,
                  acc_noise=2e-3, gyro_walk=2e-5, acc_walk=3e-3, pixel_noise=1.0,
                  intr=(380.0, 380.0, 320.0, 240.0, 0.11), max_depth=20.0, window=None):
    """window: a point is observed only by keyframes within this many of
    the keyframe it was placed in front of (None: by every keyframe that sees
    it); the sliding-window visibility of a long trajectory."""
    rng = np.random.default_rng(seed)
    # position: three sinusoids per axis, amplitudes scaled for ~1.5 m/s
    par = [(rng.uniform(1.0, 4.0, 3), rng.uniform(0.05, 0.4, 3), rng.uniform(0, 2 * np.pi, 3))
           for _ in range(3)]
    imu_dt = 1.0 / rate
    m = int(round(kf_dt * rate))
    h = 1e-6

    def states(t):
        """p, R, v, a (world) and the body angular velocity at times t."""
        p, R = _poses(t, par)
        p1, R1 = _poses(t + h, par)
        p0, R0 = _poses(t - h, par)
        v = (p1 - p0) / (2 * h)
        a = (p1 - 2 * p + p0) / (h * h)
        W = np.einsum("nji,njk->nik", R, (R1 - R0) / (2 * h))     # R^T Rdot
        w = 0.5 * np.stack([W[:, 2, 1] - W[:, 1, 2], W[:, 0, 2] - W[:, 2, 0],
                            W[:, 1, 0] - W[:, 0, 1]], axis=1)
        return p, R, v, a, w

    n_int = n_kf - 1
    # biases held per interval, random walk between keyframes
    bg = np.zeros((n_kf, 3))
    ba = np.zeros((n_kf, 3))
    bg[0] = rng.normal(scale=0.01, size=3)
    ba[0] = rng.normal(scale=0.05, size=3)
    steps_g = rng.normal(scale=gyro_walk * np.sqrt(kf_dt), size=(n_int, 3))
    steps_a = rng.normal(scale=acc_walk * np.sqrt(kf_dt), size=(n_int, 3))
    bg[1:] = bg[0] + np.cumsum(steps_g, axis=0)
    ba[1:] = ba[0] + np.cumsum(steps_a, axis=0)
    pk, Rk, vk, _, _ = states(np.arange(n_kf) * kf_dt)
    # IMU samples at the middle of each sample period
    ts = (np.arange(n_int)[:, None] * kf_dt + (np.arange(m)[None, :] + 0.5) * imu_dt).ravel()
    _, Rs, _, a_s, w_s = states(ts)
    f_body = np.einsum("nji,nj->ni", Rs, a_s - G_WORLD)
    gyro = (w_s.reshape(n_int, m, 3) + bg[:-1, None, :] +
            rng.normal(scale=gyro_noise / np.sqrt(imu_dt), size=(n_int, m, 3)))
    acc = (f_body.reshape(n_int, m, 3) + ba[:-1, None, :] +
           rng.normal(scale=acc_noise / np.sqrt(imu_dt), size=(n_int, m, 3)))
    # points: near the path, seen by the keyframes that have them in front
    # at depth 2..max_depth and inside the image
    fx, fy, cx, cy, base = intr
    anchor = rng.integers(0, n_kf, size=n_pts)
    dirc = np.stack([rng.uniform(-0.5, 0.5, n_pts), rng.uniform(-0.4, 0.4, n_pts),
                     np.ones(n_pts)], axis=1)
    depth = rng.uniform(2.0, max_depth, n_pts)
    pts = pk[anchor] + np.einsum("nij,nj->ni", Rk[anchor], dirc * depth[:, None])
    kf_l, pt_l = [], []
    for k in range(n_kf):
        if window is None:
            cand = np.arange(n_pts)
        else:
            cand = np.flatnonzero(np.abs(anchor - k) <= window)
        Xc = (pts[cand] - pk[k]) @ Rk[k]            # R^T (X - p), row-wise
        z = Xc[:, 2]
        ok = (z > 2.0) & (z < max_depth)
        zs = np.where(ok, z, 1.0)
        u = fx * Xc[:, 0] / zs + cx
        v = fy * Xc[:, 1] / zs + cy
        ok &= (u > 0) & (u < 2 * cx) & (v > 0) & (v < 2 * cy)
        sel = cand[ok]
        kf_l.append(np.full(len(sel), k, np.int64))
        pt_l.append(sel)
    st_kf = np.concatenate(kf_l)
    st_pt = np.concatenate(pt_l)
    Xc = np.einsum("nji,nj->ni", Rk[st_kf], pts[st_pt] - pk[st_kf])
    ul = fx * Xc[:, 0] / Xc[:, 2] + cx
    vl = fy * Xc[:, 1] / Xc[:, 2] + cy
    ur = ul - fx * base / Xc[:, 2]
    obs = np.stack([ul, vl, ur], axis=1) + rng.normal(scale=pixel_noise, size=(len(st_kf), 3))
    return VIScene(n_kf=n_kf, kf_dt=kf_dt, imu_dt=imu_dt, R_true=Rk, p_true=pk, v_true=vk,
                   bg_true=bg, ba_true=ba, gyro=gyro, acc=acc, pts=pts,
                   st_kf=st_kf, st_pt=st_pt, st_obs=obs, intr=intr)
