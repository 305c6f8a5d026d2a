"""Similarity (7-DoF gauge) alignment of BA solutions (test infrastructure).

Bundle adjustment without fixed vertices is invariant to a similarity
transform of the scene: X' = s Q X + tau, R' = R Q^T, t' = s t - R Q^T tau
(f, k1, k2 unchanged) leaves every projection unchanged.  Two solutions are
compared after aligning one onto the other with the closed-form least-squares
similarity of Umeyama (1991) over the points.
"""
import numpy as np
from scipy.spatial.transform import Rotation


def umeyama(src, dst):
    """s, Q, tau minimising sum |s Q src_k + tau - dst_k|^2."""
    src = np.asarray(src, np.float64)
    dst = np.asarray(dst, np.float64)
    mu_s = src.mean(0)
    mu_d = dst.mean(0)
    a = src - mu_s
    b = dst - mu_d
    var_s = (a * a).sum() / len(src)
    cov = b.T @ a / len(src)
    U, S, Vt = np.linalg.svd(cov)
    E = np.eye(3)
    if np.linalg.det(U) * np.linalg.det(Vt) < 0:
        E[2, 2] = -1.0
    Q = U @ E @ Vt
    s = float(np.trace(np.diag(S) @ E) / var_s)
    tau = mu_d - s * Q @ mu_s
    return s, Q, tau


def transform_scene(cams, pts, s, Q, tau):
    cams = np.asarray(cams, np.float64)
    R = Rotation.from_rotvec(cams[:, 0:3]).as_matrix()
    R2 = R @ Q.T
    out = cams.copy()
    out[:, 0:3] = Rotation.from_matrix(R2).as_rotvec()
    out[:, 3:6] = s * cams[:, 3:6] - np.einsum("nij,j->ni", R2, tau)
    pts2 = s * (np.asarray(pts, np.float64) @ Q.T) + tau
    return out, pts2


def aligned_errors(cams, pts, ref_cams, ref_pts):
    """Align (cams, pts) onto (ref_cams, ref_pts); return the relative
    parameter error over the stacked (rotation, t, f, k1, k2, X) vector plus
    per-block figures.  An angle-axis vector is not unique (theta about n and
    2 pi - theta about -n give the same rotation), so the rotation part of the
    difference is the angle of R R_ref^{-1} rather than a difference of
    angle-axis vectors."""
    s, Q, tau = umeyama(pts, ref_pts)
    c2, p2 = transform_scene(cams, pts, s, Q, tau)
    ref_cams = np.asarray(ref_cams, np.float64)
    ref_pts = np.asarray(ref_pts, np.float64)
    Ra = Rotation.from_rotvec(c2[:, 0:3])
    Rb = Rotation.from_rotvec(ref_cams[:, 0:3])
    rot_err = (Ra * Rb.inv()).magnitude()
    num = np.sqrt(np.sum(rot_err ** 2) + np.sum((c2[:, 3:] - ref_cams[:, 3:]) ** 2) +
                  np.sum((p2 - ref_pts) ** 2))
    den = np.sqrt(np.sum(ref_cams ** 2) + np.sum(ref_pts ** 2))
    # each parameter block against its own scale, so that the small
    # distortion terms and the rotations are not measured against the focal
    # lengths and the points
    def rel(d, ref):
        return float(np.linalg.norm(d) / max(np.linalg.norm(ref), 1e-300))

    blocks = {"rot": rel(rot_err, ref_cams[:, 0:3]),
              "t": rel(c2[:, 3:6] - ref_cams[:, 3:6], ref_cams[:, 3:6]),
              "f": rel(c2[:, 6] - ref_cams[:, 6], ref_cams[:, 6]),
              "k1": rel(c2[:, 7] - ref_cams[:, 7], ref_cams[:, 7]),
              "k2": rel(c2[:, 8] - ref_cams[:, 8], ref_cams[:, 8]),
              "X": rel(p2 - ref_pts, ref_pts)}
    return dict(rel=float(num / den), scale=s, max_rot=float(rot_err.max()),
                pts_rel=float(np.linalg.norm(p2 - ref_pts) / np.linalg.norm(ref_pts)),
                cams_rel=float(np.linalg.norm(c2[:, 3:] - ref_cams[:, 3:]) /
                               np.linalg.norm(ref_cams[:, 3:])),
                blocks=blocks, max_block=max(blocks.values()))
