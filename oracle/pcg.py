"""Preconditioned conjugate gradients on the reduced camera system
(test infrastructure, FP64, dense; small problems only).

The paper solves the damped normal equations with preconditioned conjugate
gradients over the graph structure, with a block-Jacobi preconditioner, a
tolerance, an iteration limit and a rejection ratio (Sec. IV-D).  The GPU
path runs that iteration on the Schur complement of the point blocks (the
reduced camera system of Eq. 6).  This module states the same iteration
plainly, on dense matrices, so that the GPU path's truncated iterates and
stopping decisions can be compared with it:

  * reduced system (Eq. 5-6, points eliminated):
        S  = Hcc_l - Hcp Hpp_l^-1 Hcp^T,
        v  = -bc + Hcp Hpp_l^-1 bp,
    with H_l = H + lambda diag(clamp(diag H)) over the free variables;
  * preconditioner: the exact 9x9 diagonal blocks of S (reading R12);
  * x_0 = 0; stop when r^T r <= tol^2 r_0^T r_0 (relative) or tol^2
    (absolute) (reading R10), after max_iters steps, or when
    r^T r > ratio^2 min_m r_m^T r_m with the iterate of smallest residual
    (x_0 included) returned (reading R11); a step with p^T S p <= 0 ends the
    iteration at the current iterate.

Independent of the HIP path; pinned in tests/test_oracle_pcg_pins.py against
np.linalg.solve, the Krylov-subspace minimisation property of CG and brute
force enumeration of the stopping rule.
"""
import numpy as np

DONE_CONVERGED = 1
DONE_MAX_ITERS = 2
DONE_BREAKDOWN = 3
DONE_REJECTED = 4


def reduced_system(problem, lin, lam, min_diag, max_diag):
    """(S, v, free camera ids) of the damped step at lambda, densely."""
    dc_diag, dp_diag = problem.damped_diagonal(lin, min_diag, max_diag)
    fc, fp = problem.free_cams, problem.free_pts
    nc, npf = len(fc), len(fp)
    cam_pos = -np.ones(problem.n_cams, np.int64)
    cam_pos[fc] = np.arange(nc)
    pt_pos = -np.ones(problem.n_pts, np.int64)
    pt_pos[fp] = np.arange(npf)
    Hcc = np.zeros((9 * nc, 9 * nc))
    for k, i in enumerate(fc):
        Hcc[9 * k:9 * k + 9, 9 * k:9 * k + 9] = lin.Hcc[i] + lam * np.diag(dc_diag[i])
    Hpp = np.zeros((3 * npf, 3 * npf))
    for k, j in enumerate(fp):
        Hpp[3 * k:3 * k + 3, 3 * k:3 * k + 3] = lin.Hpp[j] + lam * np.diag(dp_diag[j])
    Hcp = np.zeros((9 * nc, 3 * npf))
    for b in range(len(lin.pair_cam)):
        a, c = cam_pos[lin.pair_cam[b]], pt_pos[lin.pair_pt[b]]
        if a >= 0 and c >= 0:
            Hcp[9 * a:9 * a + 9, 3 * c:3 * c + 3] += lin.Hcp[b]
    bc = lin.bc[fc].reshape(-1)
    bp = lin.bp[fp].reshape(-1)
    HinvT = np.linalg.solve(Hpp, Hcp.T)             # Hpp_l^-1 Hcp^T
    S = Hcc - Hcp @ HinvT
    v = -bc + HinvT.T @ bp
    return 0.5 * (S + S.T), v, fc


def block_jacobi(S, block=9):
    """Inverses of the diagonal blocks of S, as one block-diagonal matrix."""
    n = S.shape[0]
    M = np.zeros_like(S)
    for a in range(0, n, block):
        M[a:a + block, a:a + block] = np.linalg.inv(S[a:a + block, a:a + block])
    return M


def pcg(S, v, Minv, tol, relative=True, max_iters=100, ratio=np.inf):
    """Returns (x, steps taken, reason) of PCG on S x = v from x = 0.

    Minv applies the preconditioner inverse (a matrix).  The reason is one of
    the DONE_* codes; ratio <= 0 or infinite disables the rejection test.
    """
    x = np.zeros_like(v)
    r = v.copy()
    z = Minv @ r
    rz = r @ z
    rr = r @ r
    thresh = tol * tol * rr if relative else tol * tol
    if rr <= thresh or not rz > 0.0:
        return x, 0, DONE_CONVERGED
    track = ratio > 0.0 and np.isfinite(ratio)
    best, min_rr = x.copy(), rr
    p = z.copy()
    for k in range(1, max_iters + 1):
        q = S @ p
        pq = p @ q
        if not (pq > 0.0 and np.isfinite(pq)):
            return x, k - 1, DONE_BREAKDOWN
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        z = Minv @ r
        rz_new = r @ z
        rr = r @ r
        if track and rr < min_rr:
            min_rr, best = rr, x.copy()
        elif track and rr > ratio * ratio * min_rr:
            return best, k, DONE_REJECTED
        if rr <= thresh:
            return x, k, DONE_CONVERGED
        if k >= max_iters:
            return x, k, DONE_MAX_ITERS
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    return x, max_iters, DONE_MAX_ITERS


def schur_pcg_step(problem, lin, lam, min_diag, max_diag, tol, relative=True,
                   max_iters=100, ratio=np.inf, precond="block_jacobi"):
    """The damped LM step computed as the GPU path does, written plainly and
    densely: PCG on the reduced camera system (steps above), then the point
    steps by back-substitution dp = Hpp_l^-1 (-bp - Hcp^T dc) (the Schur form
    of Eq. 6).  Returns ((dcam, dpt), PCG steps)."""
    S, v, fc = reduced_system(problem, lin, lam, min_diag, max_diag)
    if precond == "block_jacobi":
        M = block_jacobi(S)
    else:
        M = np.eye(len(v))
    x, steps, _ = pcg(S, v, M, tol, relative, max_iters, ratio)
    dc_diag, dp_diag = problem.damped_diagonal(lin, min_diag, max_diag)
    fp = problem.free_pts
    cam_pos = -np.ones(problem.n_cams, np.int64)
    cam_pos[fc] = np.arange(len(fc))
    dcam = np.zeros((problem.n_cams, 9))
    dcam[fc] = x.reshape(-1, 9)
    # t_j = -bp_j - sum over the point's camera pairs of Hcp^T dc
    t = -lin.bp.copy()
    for b in range(len(lin.pair_cam)):
        i, j = lin.pair_cam[b], lin.pair_pt[b]
        if cam_pos[i] >= 0:
            t[j] -= lin.Hcp[b].T @ dcam[i]
    dpt = np.zeros((problem.n_pts, 3))
    for j in fp:
        dpt[j] = np.linalg.solve(lin.Hpp[j] + lam * np.diag(dp_diag[j]), t[j])
    return (dcam, dpt), steps


class SchurPcgProblem:
    """A BA problem whose LM steps are the truncated Schur + PCG steps of
    schur_pcg_step (every other part of the LM problem interface is the
    wrapped problem's)."""

    def __init__(self, problem, tol, relative=True, max_iters=100, ratio=np.inf,
                 precond="block_jacobi"):
        self.p = problem
        self.kw = dict(tol=tol, relative=relative, max_iters=max_iters, ratio=ratio,
                       precond=precond)
        self.steps = []

    def __getattr__(self, name):
        return getattr(self.p, name)

    def solve(self, lin, lam, min_diag, max_diag):
        dx, steps = schur_pcg_step(self.p, lin, lam, min_diag, max_diag, **self.kw)
        self.steps.append(steps)
        return dx
