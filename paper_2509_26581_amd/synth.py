"""Seeded synthetic bundle-adjustment inputs with BAL-like shapes.

This module only draws inputs: a true scene, which cameras see which points,
pixel measurements of that scene, and a perturbed starting point.  It holds
none of the solver's arithmetic (no residual, derivative, robust kernel or
linear algebra of the method) and imports nothing from the solver or from the
CPU checker, so both consume the same inputs without sharing code.

The measurements are drawn from the true scene through the BAL camera
(P = R X + t, p = -P_xy / P_z, pixel = f (1 + k1 |p|^2 + k2 |p|^4) p, plus
Gaussian pixel noise).  The scene is built from look-at rotation matrices;
angle-axis parameters are obtained from them with scipy's rotation routines.

Workloads (sizes as in the benchmark configurations):
  small   10 cameras on a ring, 500 points, tracks U{3..8}      (~2.75k obs)
  bal1m   1,000 cameras on a sphere, 200k points, tracks 2+Geom(1/4)  (~1.0M)
  bal8m   10,000 cameras, 1M points, tracks 2+Geom(1/7)          (~8M obs)
  bal8m_proxy  1,000 cameras, 100k points, tracks 2+Geom(1/7)    (~0.8M obs)
Points are uniform in the box [-5, 5]^3; cameras sit at distance 20-30
(sphere) or 25 (ring) looking at the origin, so every point is in front of
every camera at depth >= 10 and random visibility is geometrically valid.
"""
from dataclasses import dataclass, field

import numpy as np
from scipy.spatial.transform import Rotation

SQUARED = 0
HUBER = 1

WORKLOADS = {
    "small": dict(n_cams=10, n_pts=500, layout="ring", track=("uniform", 3, 8),
                  loss=SQUARED, delta=1.0, trials=10, pcg_max_iters=90,
                  pcg_tol=1e-14),
    "bal1m": dict(n_cams=1000, n_pts=200_000, layout="sphere",
                  track=("geometric", 0.25), loss=HUBER, delta=1.0, trials=20,
                  pcg_max_iters=100, pcg_tol=1e-6),
    "bal8m": dict(n_cams=10_000, n_pts=1_000_000, layout="sphere",
                  track=("geometric", 1.0 / 7.0), loss=HUBER, delta=1.0,
                  trials=15, pcg_max_iters=100, pcg_tol=1e-6),
    # one tenth of bal8m in cameras and points (same track law): the size at
    # which the CPU checker can still solve the at-scale configuration
    "bal8m_proxy": dict(n_cams=1_000, n_pts=100_000, layout="sphere",
                        track=("geometric", 1.0 / 7.0), loss=HUBER, delta=1.0,
                        trials=15, pcg_max_iters=100, pcg_tol=1e-6),
}


@dataclass
class Scene:
    n_cams: int
    n_pts: int
    cams_true: np.ndarray      # (Nc, 9)  w, t, f, k1, k2
    pts_true: np.ndarray       # (Np, 3)
    cams0: np.ndarray          # perturbed start
    pts0: np.ndarray
    cam_idx: np.ndarray        # (No,) int64, shuffled edge order
    pt_idx: np.ndarray         # (No,) int64
    obs: np.ndarray            # (No, 2) pixels
    loss: int = SQUARED
    delta: float = 1.0
    trials: int = 10
    pcg_max_iters: int = 100
    pcg_tol: float = 1e-6
    meta: dict = field(default_factory=dict)

    @property
    def n_obs(self):
        return len(self.cam_idx)


def _look_at(centers, roll):
    """World->camera rotation matrices for cameras at `centers` looking at the
    origin along their -z axis, rotated by `roll` about that axis."""
    z = centers / np.linalg.norm(centers, axis=1, keepdims=True)
    up = np.tile(np.array([0.0, 0.0, 1.0]), (len(z), 1))
    para = np.abs(z[:, 2]) > 0.99
    up[para] = np.array([0.0, 1.0, 0.0])
    x = np.cross(up, z)
    x /= np.linalg.norm(x, axis=1, keepdims=True)
    y = np.cross(z, x)
    R = np.stack([x, y, z], axis=1)                       # rows = camera axes
    c, s = np.cos(roll), np.sin(roll)
    Rz = np.zeros((len(z), 3, 3))
    Rz[:, 0, 0] = c
    Rz[:, 0, 1] = -s
    Rz[:, 1, 0] = s
    Rz[:, 1, 1] = c
    Rz[:, 2, 2] = 1.0
    return Rz @ R


def _distinct_cameras(rng, n_cams, lengths):
    """For each point, `lengths[j]` distinct cameras drawn uniformly."""
    n = len(lengths)
    lmax = int(lengths.max())
    sel = np.full((n, lmax), -1, np.int64)
    for k in range(lmax):
        rows = np.flatnonzero(lengths > k)
        cand = rng.integers(0, n_cams, size=len(rows))
        while True:
            clash = np.zeros(len(rows), bool)
            for q in range(k):
                clash |= sel[rows, q] == cand
            if not clash.any():
                break
            cand[clash] = rng.integers(0, n_cams, size=int(clash.sum()))
        sel[rows, k] = cand
    return sel


def _measure(R, t, f, k1, k2, X):
    P = np.einsum("nij,nj->ni", R, X) + t
    p = -P[:, :2] / P[:, 2:3]
    n2 = (p * p).sum(1)
    g = f * (1.0 + k1 * n2 + k2 * n2 * n2)
    return g[:, None] * p, P[:, 2]


def make_scene(workload="small", seed=0, noise_px=1.0, perturb=True, **over):
    """Draw one seeded problem.  `over` overrides workload fields (n_cams,
    n_pts, track, layout, loss, delta, trials, ...)."""
    cfg = dict(WORKLOADS[workload]) if isinstance(workload, str) else dict(workload)
    cfg.update(over)
    rng = np.random.default_rng(seed)
    nc, npt = int(cfg["n_cams"]), int(cfg["n_pts"])

    pts = rng.uniform(-5.0, 5.0, size=(npt, 3))
    if cfg["layout"] == "ring":
        ang = 2 * np.pi * (np.arange(nc) + rng.uniform(-0.2, 0.2, nc)) / nc
        centers = np.stack([25 * np.cos(ang), 25 * np.sin(ang),
                            rng.uniform(-2, 2, nc)], axis=1)
    else:
        d = rng.normal(size=(nc, 3))
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        centers = d * rng.uniform(20.0, 30.0, size=(nc, 1))
    roll = rng.uniform(-0.1, 0.1, nc)
    R = _look_at(centers, roll)
    t = -np.einsum("nij,nj->ni", R, centers)
    f = rng.uniform(400.0, 600.0, nc)
    k1 = rng.uniform(-0.05, 0.05, nc)
    k2 = rng.uniform(-0.005, 0.005, nc)
    cams = np.concatenate([Rotation.from_matrix(R).as_rotvec(), t,
                           f[:, None], k1[:, None], k2[:, None]], axis=1)

    tr = cfg["track"]
    if tr[0] == "uniform":
        lengths = rng.integers(tr[1], tr[2] + 1, size=npt)
    else:
        lengths = 1 + rng.geometric(tr[1], size=npt)          # 2 + Geom0(p)
    lengths = np.minimum(lengths, nc)
    sel = _distinct_cameras(rng, nc, lengths)
    pt_idx = np.repeat(np.arange(npt), lengths)
    mask = sel >= 0
    cam_idx = sel[mask]
    obs, depth = _measure(R[cam_idx], t[cam_idx], f[cam_idx], k1[cam_idx],
                          k2[cam_idx], pts[pt_idx])
    if noise_px:
        obs = obs + rng.normal(0.0, noise_px, size=obs.shape)
    perm = rng.permutation(len(cam_idx))
    cam_idx, pt_idx, obs = cam_idx[perm], pt_idx[perm], obs[perm]

    cams0 = cams.copy()
    pts0 = pts.copy()
    if perturb:
        cams0[:, 0:3] += rng.normal(0.0, 0.05, size=(nc, 3))
        cams0[:, 3:6] += rng.normal(0.0, 0.1, size=(nc, 3))
        pts0 += rng.normal(0.0, 0.1, size=pts.shape)
    return Scene(nc, npt, cams, pts, cams0, pts0, cam_idx.astype(np.int64),
                 pt_idx.astype(np.int64), obs, int(cfg["loss"]),
                 float(cfg["delta"]), int(cfg["trials"]),
                 int(cfg["pcg_max_iters"]), float(cfg["pcg_tol"]),
                 dict(workload=workload if isinstance(workload, str) else "custom",
                      seed=seed, min_depth=float(-depth.max()) if len(depth) else 0.0,
                      noise_px=noise_px))


# ------------------------------------------------------------ local-BA stream
LOCAL = dict(k_range=(5, 40), np_range=(500, 20_000), track_max=10, window_extra=4,
             arc_per_keyframe=0.03, trials=10)


def make_local_request(seed, noise_px=1.0, perturb=True, **over):
    """One local bundle-adjustment request (a sliding-window problem):
    K = round(logU[5, 40]) keyframes along an arc of radius 25 around the
    point box, Np = round(logU[500, 20k]) points, each seen by
    L ~ U{2..min(10, K)} distinct keyframes inside a window of L + 4
    consecutive keyframes; the first two keyframes are fixed (gauge).
    Returns a dict of request arrays (dense indices, shuffled edges)."""
    cfg = dict(LOCAL)
    cfg.update(over)
    rng = np.random.default_rng(seed)
    lo, hi = cfg["k_range"]
    K = int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
    lo, hi = cfg["np_range"]
    npt = int(round(np.exp(rng.uniform(np.log(lo), np.log(hi)))))
    pts = rng.uniform(-5.0, 5.0, size=(npt, 3))
    ang0 = rng.uniform(0, 2 * np.pi)
    ang = ang0 + cfg["arc_per_keyframe"] * np.arange(K) + rng.uniform(-0.005, 0.005, K)
    centers = np.stack([25 * np.cos(ang), 25 * np.sin(ang), rng.uniform(-2, 2, K)], axis=1)
    R = _look_at(centers, rng.uniform(-0.1, 0.1, K))
    t = -np.einsum("nij,nj->ni", R, centers)
    f = rng.uniform(400.0, 600.0, K)
    k1 = rng.uniform(-0.05, 0.05, K)
    k2 = rng.uniform(-0.005, 0.005, K)
    cams = np.concatenate([Rotation.from_matrix(R).as_rotvec(), t,
                           f[:, None], k1[:, None], k2[:, None]], axis=1)
    lengths = rng.integers(2, min(cfg["track_max"], K) + 1, size=npt)
    width = np.minimum(lengths + cfg["window_extra"], K)
    start = (rng.uniform(size=npt) * (K - width + 1)).astype(np.int64)
    # L distinct window positions per point: the L smallest of random keys
    # over the point's window
    wmax = int(width.max())
    keys = rng.uniform(size=(npt, wmax))
    keys[np.arange(wmax)[None, :] >= width[:, None]] = np.inf
    sel = np.argsort(keys, axis=1)[:, :int(lengths.max())]
    mask = np.arange(sel.shape[1])[None, :] < lengths[:, None]
    pt_idx = np.repeat(np.arange(npt), lengths)
    cam_idx = (sel + start[:, None])[mask]
    obs, _ = _measure(R[cam_idx], t[cam_idx], f[cam_idx], k1[cam_idx], k2[cam_idx],
                      pts[pt_idx])
    if noise_px:
        obs = obs + rng.normal(0.0, noise_px, size=obs.shape)
    perm = rng.permutation(len(cam_idx))
    cam_idx, pt_idx, obs = cam_idx[perm], pt_idx[perm], obs[perm]
    cams0, pts0 = cams.copy(), pts.copy()
    fixed = np.zeros(K, bool)
    fixed[:2] = True
    if perturb:
        free = ~fixed
        cams0[free, 0:3] += rng.normal(0.0, 0.05, size=(int(free.sum()), 3))
        cams0[free, 3:6] += rng.normal(0.0, 0.1, size=(int(free.sum()), 3))
        pts0 += rng.normal(0.0, 0.1, size=pts.shape)
    return {"cams": cams0, "pts": pts0, "cam_idx": cam_idx.astype(np.int32),
            "pt_idx": pt_idx.astype(np.int32), "uv": obs, "cam_fixed": fixed,
            "max_iters": int(cfg["trials"]), "tol": 0.0,
            "cams_true": cams, "pts_true": pts, "seed": seed}


def poisson_arrivals(n, rate_per_s, seed):
    """Arrival times (s) of a Poisson stream: cumulative Exp(rate) gaps."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))
