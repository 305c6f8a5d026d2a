"""Dense generic least-squares problems for the LM loop (test infrastructure).

Used for the paper's running example (Sec. IV: 2-D points pulled onto a circle
by the constraint x^2 + y^2 - r^2, the last point fixed, the third constraint
disabled) and for a linear-residual check of the LM loop.  Jacobians come from
the dual numbers of oracle.dual; the damped system is solved densely.
"""
import numpy as np

from . import dual as D


class DenseProblem:
    """residual_fn maps a length-n list of scalars (floats or Duals) to a
    length-m list of residuals; params listed in `fixed` carry no unknown;
    residuals listed as inactive are dropped."""

    def __init__(self, residual_fn, n, fixed=None, active=None):
        self.fn = residual_fn
        self.n = n
        self.fixed = np.zeros(n, bool) if fixed is None else np.asarray(fixed, bool)
        self.active = active

    def _res(self, x, duals):
        if duals:
            xs = D.seed(np.asarray(x, np.float64)[None, :])
        else:
            xs = [np.array([v], np.float64) for v in x]
        res = self.fn(xs)
        if self.active is not None:
            res = [r for r, a in zip(res, self.active) if a]
        return res

    def n_free(self):
        return int((~self.fixed).sum())

    def cost(self, x):
        r = np.array([D.value(v)[0] for v in self._res(x, False)])
        return 0.5 * float(r @ r)

    def linearize(self, x):
        res = self._res(x, True)
        r = np.array([v.v[0] for v in res])
        J = np.array([v.d[0] for v in res]).reshape(len(res), self.n)
        J[:, self.fixed] = 0.0
        return dict(r=r, J=J, H=J.T @ J, b=J.T @ r)

    def solve(self, lin, lam, min_diag, max_diag):
        f = ~self.fixed
        H = lin["H"][np.ix_(f, f)]
        d = np.clip(np.diag(H), min_diag, max_diag)
        dx = np.zeros(self.n)
        dx[f] = np.linalg.solve(H + lam * np.diag(d), -lin["b"][f])
        return dx

    def model_decrease(self, lin, dx):
        Jd = lin["J"] @ dx
        return -(float(lin["b"] @ dx) + 0.5 * float(Jd @ Jd))

    def step(self, x, dx):
        return np.asarray(x, np.float64) + dx

    def norm(self, v):
        return float(np.linalg.norm(np.asarray(v)[~self.fixed]))


def circle_problem(points, radius, fixed_last=True, disabled=(2,)):
    """The paper's running example: one constraint x^2 + y^2 - r^2 per point."""
    n_pts = len(points)

    def fn(xs):
        return [xs[2 * k] * xs[2 * k] + xs[2 * k + 1] * xs[2 * k + 1]
                - radius * radius for k in range(n_pts)]

    fixed = np.zeros(2 * n_pts, bool)
    if fixed_last:
        fixed[-2:] = True
    active = np.ones(n_pts, bool)
    for k in disabled:
        active[k] = False
    return DenseProblem(fn, 2 * n_pts, fixed, active), np.asarray(points, float).ravel()
