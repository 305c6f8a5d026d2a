"""Preconditioned conjugate gradients on the full damped normal equations
(test infrastructure, FP64, dense; small problems only).

The paper's own solver form: PCG over the whole Hessian, camera and point
unknowns together, with block-Jacobi preconditioning (Sec. IV-D; its BAL and
visual-inertial runs solve the full system, Sec. V).  This module states that
system plainly so that the GPU path's full-Hessian PCG can be compared with
it iterate by iterate:

  * unknowns: the free cameras (9 each) then the free points (3 each), in
    index order;
  * H_l = H + lambda diag(clamp(diag H, min_diag, max_diag)) (Eq. 4 with the
    clamped diagonal), H = J^T W J assembled from the blocks Hcc, Hpp and the
    coupling blocks Hcp of the linearisation (Eq. 5);
  * right-hand side -b (Eq. 6);
  * preconditioner: the inverses of the 9x9 camera and 3x3 point diagonal
    blocks of H_l (block Jacobi);
  * the iteration itself is oracle.pcg.pcg (x_0 = 0, the same stopping
    rules).

Independent of the HIP path; pinned in tests/test_oracle_full_pins.py
against the exact block-Cholesky step, the reduced camera system and a
Hessian formed from finite-difference Jacobians.
"""
import numpy as np


def full_system(problem, lin, lam, min_diag, max_diag):
    """(H_l, v = -b, free camera ids, free point ids), dense."""
    dc_diag, dp_diag = problem.damped_diagonal(lin, min_diag, max_diag)
    fc, fp = problem.free_cams, problem.free_pts
    nc, npf = len(fc), len(fp)
    cam_pos = -np.ones(problem.n_cams, np.int64)
    cam_pos[fc] = np.arange(nc)
    pt_pos = -np.ones(problem.n_pts, np.int64)
    pt_pos[fp] = np.arange(npf)
    N = 9 * nc + 3 * npf
    H = np.zeros((N, N))
    for k, i in enumerate(fc):
        H[9 * k:9 * k + 9, 9 * k:9 * k + 9] = lin.Hcc[i] + lam * np.diag(dc_diag[i])
    o = 9 * nc
    for k, j in enumerate(fp):
        H[o + 3 * k:o + 3 * k + 3, o + 3 * k:o + 3 * k + 3] = lin.Hpp[j] + lam * np.diag(dp_diag[j])
    for b in range(len(lin.pair_cam)):
        a, c = cam_pos[lin.pair_cam[b]], pt_pos[lin.pair_pt[b]]
        if a >= 0 and c >= 0:
            H[9 * a:9 * a + 9, o + 3 * c:o + 3 * c + 3] += lin.Hcp[b]
            H[o + 3 * c:o + 3 * c + 3, 9 * a:9 * a + 9] += lin.Hcp[b].T
    v = -np.concatenate([lin.bc[fc].reshape(-1), lin.bp[fp].reshape(-1)])
    return H, v, fc, fp


def block_jacobi_full(H, n_cams):
    """Inverses of the 9x9 camera blocks (the first 9 n_cams unknowns) and of
    the 3x3 point blocks (the rest), as one block-diagonal matrix."""
    M = np.zeros_like(H)
    o = 9 * n_cams
    for a in range(0, o, 9):
        M[a:a + 9, a:a + 9] = np.linalg.inv(H[a:a + 9, a:a + 9])
    for a in range(o, H.shape[0], 3):
        M[a:a + 3, a:a + 3] = np.linalg.inv(H[a:a + 3, a:a + 3])
    return M


def split(x, problem, fc, fp):
    """A full-system vector as (camera steps (n_cams, 9), point steps
    (n_pts, 3)), zero for fixed vertices."""
    dcam = np.zeros((problem.n_cams, 9))
    dpt = np.zeros((problem.n_pts, 3))
    dcam[fc] = x[:9 * len(fc)].reshape(-1, 9)
    dpt[fp] = x[9 * len(fc):].reshape(-1, 3)
    return dcam, dpt
