"""Bundle adjustment as an LM problem: full normal equations and their exact
block Cholesky solve (test infrastructure, FP64).

Variables: cameras (9 parameters each) and points (3 each); fixed vertices
carry no unknowns and inactive edges contribute nothing (Sec. IV-A listing of
set_fixed / set_active; Sec. IV-D: kernels respect fixed vertices and inactive
constraints).  For the active edges e = (i, j) with residual r_e, Jacobian
blocks J_ce (2x9), J_pe (2x3), information Omega_e (identity when not given)
and IRLS weight w_e = rho'(r_e^T Omega_e r_e):

  H = sum_e J_e^T w_e Omega_e J_e,  b = sum_e J_e^T w_e Omega_e r_e   (Eq. 5)

restricted to the free variables.  The damped system (Eq. 4-6) uses
D^T D = clamp(diag H, min_diag, max_diag) (Sec. IV-D clamps the diagonal).

The solve is an exact sparse Cholesky factorisation H_lambda = L L^T of the
full system.  Elimination order: every point block first, then the camera
blocks.  Points are never adjacent to each other, so eliminating them creates
fill only among cameras; this is the order a minimum-degree rule produces on a
bundle-adjustment graph (a point's degree is its track length, a camera's is
the number of points it sees).  The trailing camera block is dense and is
factored by LAPACK.  No reduced-system iteration is involved.
"""
import numpy as np
import scipy.linalg

from . import camera, robust


def _omega(info, n):
    """Per-edge 2x2 information matrices from (n, 3) upper-triangular values."""
    om = np.empty((n, 2, 2))
    if info is None:
        om[:] = np.eye(2)
    else:
        info = np.asarray(info, dtype=np.float64)
        om[:, 0, 0] = info[:, 0]
        om[:, 0, 1] = info[:, 1]
        om[:, 1, 0] = info[:, 1]
        om[:, 1, 1] = info[:, 2]
    return om


def _mat2(A, B):
    """Batched A @ B for A (n,2,2), B (n,2,k)."""
    return np.matmul(A, B)


def _tmul(A, B):
    """Batched A^T B for A (n,m,i), B (n,m,j) -> (n,i,j), summing over m."""
    return np.matmul(A.transpose(0, 2, 1), B)


def _tvec(A, v):
    """Batched A^T v for A (n,m,i), v (n,m) -> (n,i)."""
    return np.matmul(A.transpose(0, 2, 1), v[:, :, None])[:, :, 0]


def _scatter_sum(index, values, n):
    """out[k] = sum of values[e] over e with index[e] == k."""
    shape = values.shape[1:]
    flat = values.reshape(len(values), -1)
    out = np.empty((n, flat.shape[1]))
    for c in range(flat.shape[1]):
        out[:, c] = np.bincount(index, weights=flat[:, c], minlength=n)
    return out.reshape((n,) + shape)


class Linearization:
    pass


class BAProblem:
    """Bundle adjustment over BAL cameras; x = (cams (Nc,9), pts (Np,3))."""

    def __init__(self, n_cams, n_pts, cam_idx, pt_idx, obs, info=None,
                 cam_fixed=None, pt_fixed=None, edge_active=None,
                 loss=robust.SQUARED, delta=1.0, pair_chunk=500_000):
        self.n_cams = int(n_cams)
        self.n_pts = int(n_pts)
        cam_idx = np.asarray(cam_idx, dtype=np.int64)
        pt_idx = np.asarray(pt_idx, dtype=np.int64)
        obs = np.asarray(obs, dtype=np.float64)
        act = (np.ones(len(cam_idx), bool) if edge_active is None
               else np.asarray(edge_active, bool))
        self.cam_idx = cam_idx[act]
        self.pt_idx = pt_idx[act]
        self.obs = obs[act]
        self.omega = _omega(None if info is None else np.asarray(info)[act],
                            len(self.cam_idx))
        self.cam_fixed = (np.zeros(self.n_cams, bool) if cam_fixed is None
                          else np.asarray(cam_fixed, bool))
        self.pt_fixed = (np.zeros(self.n_pts, bool) if pt_fixed is None
                         else np.asarray(pt_fixed, bool))
        self.loss = loss
        self.delta = float(delta)
        self.pair_chunk = pair_chunk
        # touched free vertices define the unknowns (an untouched free vertex
        # still gets an unknown: its row is lambda * min_diag * I, step 0)
        self.free_cams = np.flatnonzero(~self.cam_fixed)
        self.free_pts = np.flatnonzero(~self.pt_fixed)

    # --- LM problem interface -------------------------------------------
    def n_free(self):
        if len(self.cam_idx) == 0:
            return 0
        return 9 * len(self.free_cams) + 3 * len(self.free_pts)

    def _s(self, r):
        return np.einsum("ni,nij,nj->n", r, self.omega, r)

    def cost(self, x):
        cams, pts = x
        r = camera.residuals(cams, pts, self.cam_idx, self.pt_idx, self.obs)
        return 0.5 * float(np.sum(robust.rho(self._s(r), self.loss, self.delta)))

    def residual_stats(self, x):
        """(chi2 = sum rho, mse = sum |r|^2 / n_edges) over active edges."""
        cams, pts = x
        r = camera.residuals(cams, pts, self.cam_idx, self.pt_idx, self.obs)
        s = self._s(r)
        return (float(np.sum(robust.rho(s, self.loss, self.delta))),
                float(np.sum(r * r) / max(len(r), 1)))

    def linearize(self, x):
        cams, pts = x
        r, Jc, Jp = camera.residuals_and_jacobians(
            cams, pts, self.cam_idx, self.pt_idx, self.obs)
        s = self._s(r)
        w = robust.weight(s, self.loss, self.delta)
        Jc = Jc * (~self.cam_fixed[self.cam_idx])[:, None, None]
        Jp = Jp * (~self.pt_fixed[self.pt_idx])[:, None, None]
        WOm = self.omega * w[:, None, None]                  # w Omega  (n,2,2)
        OJc = _mat2(WOm, Jc)                                 # (n,2,9)
        OJp = _mat2(WOm, Jp)                                 # (n,2,3)
        Or = np.matmul(WOm, r[:, :, None])[:, :, 0]
        L = Linearization()
        L.r, L.Jc, L.Jp, L.w = r, Jc, Jp, w
        L.Hcc = _scatter_sum(self.cam_idx, _tmul(Jc, OJc), self.n_cams)
        L.bc = _scatter_sum(self.cam_idx, _tvec(Jc, Or), self.n_cams)
        L.Hpp = _scatter_sum(self.pt_idx, _tmul(Jp, OJp), self.n_pts)
        L.bp = _scatter_sum(self.pt_idx, _tvec(Jp, Or), self.n_pts)
        # camera-point coupling blocks, summed over repeated (i, j) pairs
        key = self.cam_idx * self.n_pts + self.pt_idx
        uk, inv = np.unique(key, return_inverse=True)
        L.pair_cam = uk // self.n_pts
        L.pair_pt = uk % self.n_pts
        L.Hcp = _scatter_sum(inv, _tmul(Jc, OJp), len(uk))
        return L

    def damped_diagonal(self, lin, min_diag, max_diag):
        dc = np.clip(np.einsum("nii->ni", lin.Hcc), min_diag, max_diag)
        dp = np.clip(np.einsum("nii->ni", lin.Hpp), min_diag, max_diag)
        return dc, dp

    def solve(self, lin, lam, min_diag, max_diag):
        """Exact solution of (H + lam D) dx = -b over the free variables."""
        dc_diag, dp_diag = self.damped_diagonal(lin, min_diag, max_diag)
        fc = self.free_cams
        fp = self.free_pts
        nc, npf = len(fc), len(fp)
        cam_pos = -np.ones(self.n_cams, np.int64)
        cam_pos[fc] = np.arange(nc)
        pt_pos = -np.ones(self.n_pts, np.int64)
        pt_pos[fp] = np.arange(npf)

        # point blocks: App_j = Hpp_j + lam diag(Dp_j);  Lpp_j Lpp_j^T = App_j
        App = lin.Hpp[fp] + lam * dp_diag[fp][:, :, None] * np.eye(3)
        Lpp = np.linalg.cholesky(App) if npf else np.zeros((0, 3, 3))
        yp = (np.linalg.solve(Lpp, -lin.bp[fp][:, :, None])[:, :, 0]
              if npf else np.zeros((0, 3)))

        # coupling blocks between free cameras and free points
        keep = (cam_pos[lin.pair_cam] >= 0) & (pt_pos[lin.pair_pt] >= 0)
        pc = cam_pos[lin.pair_cam[keep]]
        pp = pt_pos[lin.pair_pt[keep]]
        Hcp = lin.Hcp[keep]
        # Lcp_(i,j) = Hcp_(i,j) Lpp_j^{-T}  <=>  Lcp^T = Lpp_j^{-1} Hcp^T
        LcpT = (np.linalg.solve(Lpp[pp], Hcp.transpose(0, 2, 1))
                if len(pp) else np.zeros((0, 3, 9)))             # (P,3,9)

        # trailing camera block: Acc = Hcc + lam Dc - Lcp Lcp^T  (dense)
        N = 9 * nc
        Acc = np.zeros((N, N))
        for k, i in enumerate(fc):
            Acc[9 * k:9 * k + 9, 9 * k:9 * k + 9] = (
                lin.Hcc[i] + lam * np.diag(dc_diag[i]))
        order = np.argsort(pp, kind="stable")
        pc_s, pp_s, LcpT_s = pc[order], pp[order], LcpT[order]
        counts = np.bincount(pp_s, minlength=npf) if npf else np.zeros(0, int)
        starts = np.concatenate([[0], np.cumsum(counts)[:-1]]) if npf else counts
        sq = counts * counts
        total = int(sq.sum())
        if total:
            # every ordered pair (a, b) of coupling blocks of one point adds
            # Lcp_a Lcp_b^T at camera block (cam_a, cam_b); the pairs with
            # a > b give the transposes of those with a < b
            pts_rep = np.repeat(np.arange(npf), sq)
            base = np.repeat(np.cumsum(sq) - sq, sq)
            loc = np.arange(total) - base
            m = counts[pts_rep]
            a = starts[pts_rep] + loc // m
            b = starts[pts_rep] + loc % m
            keep = a <= b
            a, b = a[keep], b[keep]
            rr = np.arange(9)
            off81 = (rr[:, None] * N + rr[None, :]).ravel()
            accum = np.zeros(N * N)
            for s0 in range(0, len(a), self.pair_chunk):
                aa = a[s0:s0 + self.pair_chunk]
                bb = b[s0:s0 + self.pair_chunk]
                prod = _tmul(LcpT_s[aa], LcpT_s[bb])               # (n,9,9)
                prod[aa == bb] *= 0.5
                base = 9 * pc_s[aa] * N + 9 * pc_s[bb]
                flat = base[:, None] + off81[None, :]
                accum += np.bincount(flat.ravel(), weights=prod.reshape(-1),
                                     minlength=N * N)
            accum = accum.reshape(N, N)
            accum += accum.T.copy()
            Acc -= accum

        # forward: Lcc y_c = -b_c - Lcp y_p
        rhs_c = -lin.bc[fc].reshape(-1) if nc else np.zeros(0)
        if len(pp):
            contrib = _tvec(LcpT, yp[pp])                           # (P,9)
            idx = (9 * pc[:, None] + np.arange(9)[None, :]).ravel()
            rhs_c = rhs_c - np.bincount(idx, weights=contrib.ravel(),
                                        minlength=N)
        if nc:
            cf = scipy.linalg.cho_factor(Acc, lower=True, check_finite=False)
            dcf = scipy.linalg.cho_solve(cf, rhs_c, check_finite=False)
        else:
            dcf = np.zeros(0)
        dcf = dcf.reshape(nc, 9)

        # back: Lpp^T dp = y_p - Lcp^T dc
        t = yp.copy()
        if len(pp):
            back = np.matmul(LcpT, dcf[pc][:, :, None])[:, :, 0]     # (P,3)
            for k in range(3):
                t[:, k] -= np.bincount(pp, weights=back[:, k], minlength=npf)
        dpf = (np.linalg.solve(Lpp.transpose(0, 2, 1), t[:, :, None])[:, :, 0]
               if npf else np.zeros((0, 3)))

        dcam = np.zeros((self.n_cams, 9))
        dcam[fc] = dcf
        dpt = np.zeros((self.n_pts, 3))
        dpt[fp] = dpf
        return dcam, dpt

    def model_decrease(self, lin, dx):
        dcam, dpt = dx
        b_dx = float(np.sum(lin.bc * dcam) + np.sum(lin.bp * dpt))
        jd = (np.matmul(lin.Jc, dcam[self.cam_idx][:, :, None]) +
              np.matmul(lin.Jp, dpt[self.pt_idx][:, :, None]))[:, :, 0]
        quad = float(np.sum(lin.w * self._s(jd)))
        return -(b_dx + 0.5 * quad)

    def step(self, x, dx):
        cams, pts = x
        dcam, dpt = dx
        return cams + dcam, pts + dpt

    def norm(self, v):
        cams, pts = v
        return float(np.sqrt(np.sum(cams[self.free_cams] ** 2) +
                             np.sum(pts[self.free_pts] ** 2)))


def solve(problem, cams0, pts0, max_iters, tol=0.0, initial_lambda=1e-4,
          min_diag=1e-6, max_diag=1e32):
    from . import lm
    return lm.levenberg_marquardt(problem, (np.array(cams0, np.float64),
                                            np.array(pts0, np.float64)),
                                  max_iters, tol, initial_lambda,
                                  min_diag, max_diag)
