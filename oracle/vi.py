"""Visual-inertial bundle adjustment as a least-squares problem for the LM
loop (test infrastructure, FP64, plain numpy; dense normal equations).

The paper's visual-inertial optimisation (Background, Eq. 8; Sec. V-C)
minimises, over keyframe states and map points, the stereo reprojection
terms plus an inertial term between consecutive keyframes and a bias
random-walk term.  The factor definitions are those of oracle.imu; this
module adds their weights, the robust kernel of the stereo terms, the
manifold update and the damped normal equations:

  F = 1/2 sum_stereo rho(s_e) + 1/2 sum_inertial r^T Omega_I r
      + 1/2 sum_bias r^T Omega_b r,
  s_e = |r_e|^2 / sigma_px^2,   rho = Huber on s with threshold delta2
      (rho(s) = s for s <= delta2, 2 sqrt(delta2 s) - delta2 above; as the BA
      cost, with delta = sqrt(delta2)),
  Omega_I = cov^-1 (the preintegrated covariance),
  Omega_b = diag(1 / (sigma_gw^2 dt) I3, 1 / (sigma_aw^2 dt) I3).

Readings (listed in the design notes):
  * unknowns per keyframe: 15 (dtheta, dp, dv, dbg, dba; the rotation
    updated on the right, R <- R Exp(dtheta)), per point 3;
  * the first keyframe is held fixed (the gauge: its columns are removed);
  * the stereo terms are weighted as the BA edges (IRLS: J~ = sqrt(w) J /
    sigma_px with w = rho'(s));
  * the damped system is H + lambda diag(clip(diag H, min_diag, max_diag)),
    the normal equations of the whole system (no point elimination), as in
    the paper's full-system PCG.

The Schur form of the same step (schur_pcg_step) eliminates the points
(Eq. 5-6 applied to the keyframe / point partition): with the damped
blocks A (keyframes), B (keyframe-point) and C (points, block diagonal),
    S = A - B C^-1 B^T,   v = -b_k + B C^-1 b_p,
PCG on S x_k = v from 0 with the exact 15 x 15 diagonal blocks of S as
the block-Jacobi preconditioner and the stop rules of oracle.pcg.pcg, then
x_p = C^-1 (-b_p - B^T x_k).  S carries the keyframe-keyframe blocks of
the inertial terms and of the points two keyframes share.

The stereo Jacobian is the closed form of the projection chain
(dXc/dtheta = [Xc]x, dXc/dp = -R^T, dXc/dX = R^T); it is pinned against the
dual numbers of oracle.imu.  The inertial Jacobian comes from those dual
numbers.
"""
import numpy as np

from . import imu
from . import pcg as _pcg


class VIState:
    """Keyframe rotations R (K, 3, 3), positions p, velocities v, biases bg,
    ba (K, 3) and points X (N, 3)."""

    def __init__(self, R, p, v, bg, ba, X):
        self.R = np.asarray(R, float)
        self.p = np.asarray(p, float)
        self.v = np.asarray(v, float)
        self.bg = np.asarray(bg, float)
        self.ba = np.asarray(ba, float)
        self.X = np.asarray(X, float)

    @property
    def n_kf(self):
        return len(self.p)

    @property
    def n_pts(self):
        return len(self.X)


def huber(s, delta2):
    """rho(s) and rho'(s) of the Huber kernel on the squared norm s."""
    s = np.asarray(s, float)
    if not delta2 > 0.0:
        return s.copy(), np.ones_like(s)
    lin = s > delta2
    q = np.sqrt(np.where(lin, s, 1.0))
    rho = np.where(lin, 2.0 * np.sqrt(delta2) * q - delta2, s)
    w = np.where(lin, np.sqrt(delta2) / q, 1.0)
    return rho, w


def stereo_project(R, p, X, intr):
    """Xc = R^T (X - p) and (u_l, v_l, u_r) for arrays of observations."""
    fx, fy, cx, cy, base = intr
    Xc = np.einsum("nji,nj->ni", R, X - p)
    z = Xc[:, 2]
    ul = fx * Xc[:, 0] / z + cx
    vl = fy * Xc[:, 1] / z + cy
    ur = ul - fx * base / z
    return Xc, np.stack([ul, vl, ur], axis=1)


def stereo_jacobian(R, Xc, intr):
    """d(u_l, v_l, u_r) / d(dtheta, dp, dX): (n, 3, 9), the chain rule of the
    projection through Xc = R^T (X - p) with the right perturbation."""
    fx, fy, _, _, base = intr
    x, y, z = Xc[:, 0], Xc[:, 1], Xc[:, 2]
    n = len(z)
    P = np.zeros((n, 3, 3))          # d(ul, vl, ur) / dXc
    P[:, 0, 0] = fx / z
    P[:, 0, 2] = -fx * x / z ** 2
    P[:, 1, 1] = fy / z
    P[:, 1, 2] = -fy * y / z ** 2
    P[:, 2, 0] = fx / z
    P[:, 2, 2] = -fx * (x - base) / z ** 2
    K = np.zeros((n, 3, 3))          # [Xc]x = dXc / dtheta
    K[:, 0, 1], K[:, 0, 2] = -z, y
    K[:, 1, 0], K[:, 1, 2] = z, -x
    K[:, 2, 0], K[:, 2, 1] = -y, x
    Rt = np.transpose(R, (0, 2, 1))
    J = np.zeros((n, 3, 9))
    J[:, :, 0:3] = P @ K
    J[:, :, 3:6] = -(P @ Rt)
    J[:, :, 6:9] = P @ Rt
    return J


class VIProblem:
    """The LM problem of oracle.lm over VIState.  pre: a list of K - 1
    imu.Preintegrated intervals (keyframe f to f + 1)."""

    def __init__(self, kf, pt, obs, intr, pre, sigma_px=1.0, delta2=0.0,
                 sigma_gw=1e-4, sigma_aw=1e-3):
        self.kf = np.asarray(kf, np.int64)
        self.pt = np.asarray(pt, np.int64)
        self.obs = np.asarray(obs, float)
        self.intr = tuple(float(v) for v in intr)
        self.pre = list(pre)
        self.sigma_px = float(sigma_px)
        self.delta2 = float(delta2)
        self.info_I = [np.linalg.inv(P.cov) for P in self.pre]
        self.info_b = [np.concatenate([np.full(3, 1.0 / (sigma_gw ** 2 * P.dt)),
                                       np.full(3, 1.0 / (sigma_aw ** 2 * P.dt))])
                       for P in self.pre]
        self.K = len(self.pre) + 1

    # --------------------------------------------------------------- layout
    def n_vars(self, x):
        return 15 * x.n_kf + 3 * x.n_pts

    def free_mask(self, x):
        f = np.ones(self.n_vars(x), bool)
        f[0:15] = False                  # the first keyframe: gauge
        return f

    def n_free(self):
        return 1

    # ----------------------------------------------------------- residuals
    def _stereo(self, x):
        R, p = x.R[self.kf], x.p[self.kf]
        Xc, pred = stereo_project(R, p, x.X[self.pt], self.intr)
        r = pred - self.obs
        return R, Xc, r

    def _inertial(self, x, f):
        return imu.inertial_residual_and_jacobian(
            x.R[f], x.p[f], x.v[f], x.bg[f], x.ba[f], x.R[f + 1], x.p[f + 1], x.v[f + 1],
            self.pre[f])

    def cost(self, x):
        _, _, r = self._stereo(x)
        s = np.sum(r * r, axis=1) / self.sigma_px ** 2
        rho, _ = huber(s, self.delta2)
        F = 0.5 * float(np.sum(rho))
        for f in range(self.K - 1):
            ri = np.array([float(v) for v in imu.inertial_residual(
                x.R[f], x.p[f], x.v[f], x.bg[f], x.ba[f], x.R[f + 1], x.p[f + 1],
                x.v[f + 1], self.pre[f])])
            F += 0.5 * float(ri @ self.info_I[f] @ ri)
            rb = np.concatenate([x.bg[f + 1] - x.bg[f], x.ba[f + 1] - x.ba[f]])
            F += 0.5 * float(rb @ (self.info_b[f] * rb))
        return F

    def linearize(self, x):
        """Dense whitened Jacobian (rows: stereo, inertial, bias; columns: 15
        per keyframe, 3 per point), residual, H = J^T J and b = J^T r."""
        n = self.n_vars(x)
        R, Xc, r = self._stereo(x)
        s = np.sum(r * r, axis=1) / self.sigma_px ** 2
        _, w = huber(s, self.delta2)
        sc = np.sqrt(w) / self.sigma_px
        Js = stereo_jacobian(R, Xc, self.intr) * sc[:, None, None]
        rs = r * sc[:, None]
        m = 3 * len(self.kf) + 15 * (self.K - 1)
        J = np.zeros((m, n))
        res = np.zeros(m)
        for e in range(len(self.kf)):
            c0, c1 = 15 * self.kf[e], 15 * x.n_kf + 3 * self.pt[e]
            J[3 * e:3 * e + 3, c0:c0 + 6] = Js[e, :, 0:6]
            J[3 * e:3 * e + 3, c1:c1 + 3] = Js[e, :, 6:9]
        res[0:3 * len(self.kf)] = rs.ravel()
        row = 3 * len(self.kf)
        for f in range(self.K - 1):
            ri, Ji = self._inertial(x, f)
            L = np.linalg.cholesky(self.info_I[f])      # Omega = L L^T: whitened = L^T r
            ri, Ji = L.T @ ri, L.T @ Ji
            i0, j0 = 15 * f, 15 * (f + 1)
            J[row:row + 9, i0:i0 + 15] = Ji[:, 0:15]
            J[row:row + 9, j0:j0 + 9] = Ji[:, 15:24]
            res[row:row + 9] = ri
            row += 9
            sb = np.sqrt(self.info_b[f])
            for k in range(6):
                J[row + k, i0 + 9 + k] = -sb[k]
                J[row + k, j0 + 9 + k] = sb[k]
            res[row:row + 6] = sb * np.concatenate([x.bg[f + 1] - x.bg[f], x.ba[f + 1] - x.ba[f]])
            row += 6
        J[:, ~self.free_mask(x)] = 0.0
        return dict(J=J, r=res, H=J.T @ J, b=J.T @ res, free=self.free_mask(x))

    # ---------------------------------------------------------- linear step
    def solve(self, lin, lam, min_diag, max_diag):
        f = lin["free"]
        H = lin["H"][np.ix_(f, f)]
        d = np.clip(np.diag(H), min_diag, max_diag)
        dx = np.zeros(len(f))
        dx[f] = np.linalg.solve(H + lam * np.diag(d), -lin["b"][f])
        return dx

    def reduced_system(self, lin, lam, min_diag, max_diag):
        """(S, v, A, B, C, b_k, b_p) of the damped step over the free
        variables, densely: keyframes 1.. first (15 each), then the points."""
        f = lin["free"]
        H = lin["H"][np.ix_(f, f)]
        Hd = H + lam * np.diag(np.clip(np.diag(H), min_diag, max_diag))
        b = lin["b"][f]
        nk = 15 * (self.K - 1)
        A, B, C = Hd[:nk, :nk], Hd[:nk, nk:], Hd[nk:, nk:]
        bk, bp = b[:nk], b[nk:]
        CiBt = np.linalg.solve(C, B.T)               # C^-1 B^T
        S = A - B @ CiBt
        v = -bk + CiBt.T @ bp
        return 0.5 * (S + S.T), v, A, B, C, bk, bp

    def schur_pcg_step(self, lin, lam, min_diag, max_diag, tol, max_iters, ratio=np.inf):
        """The damped step by PCG on the keyframe Schur complement (relative
        tolerance, the rejection test of oracle.pcg.pcg with ratio), then
        point back-substitution.  Returns (dx over all variables, PCG
        steps); the PCG's stop reason is kept in self.last_reason."""
        S, v, A, B, C, bk, bp = self.reduced_system(lin, lam, min_diag, max_diag)
        M = _pcg.block_jacobi(S, 15)
        xk, steps, self.last_reason = _pcg.pcg(S, v, M, tol, True, max_iters, ratio)
        xp = np.linalg.solve(C, -bp - B.T @ xk)
        dx = np.zeros(len(lin["free"]))
        dx[lin["free"]] = np.concatenate([xk, xp])
        return dx, steps

    def model_decrease(self, lin, dx):
        Jd = lin["J"] @ dx
        return -(float(lin["b"] @ dx) + 0.5 * float(Jd @ Jd))

    def step(self, x, dx):
        K = x.n_kf
        d = dx[0:15 * K].reshape(K, 15)
        R = np.stack([x.R[k] @ imu.so3_exp(d[k, 0:3]) for k in range(K)])
        return VIState(R, x.p + d[:, 3:6], x.v + d[:, 6:9], x.bg + d[:, 9:12],
                       x.ba + d[:, 12:15], x.X + dx[15 * K:].reshape(-1, 3))

    def norm(self, v):
        if isinstance(v, VIState):
            parts = [np.array([imu.so3_log(Rk) for Rk in v.R[1:]]).ravel(), v.p[1:].ravel(),
                     v.v[1:].ravel(), v.bg[1:].ravel(), v.ba[1:].ravel(), v.X.ravel()]
            return float(np.linalg.norm(np.concatenate(parts)))
        return float(np.linalg.norm(np.asarray(v)[15:]))
