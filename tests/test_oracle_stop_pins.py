"""Pins of the oracle's stop rules and the remaining unpinned pieces
(test infrastructure checks, CPU only).

The paper leaves the LM stop rules unstated; the reading (Background,
Eq. 3-6 loop) stops after max_iters trials, on an accepted step with
(F - F') / F < tol (COST_TOL), on |dx| <= tol (|x| + tol) (STEP_TOL), on
lambda > 1e32 (LAMBDA_OVERFLOW) and on a non-finite starting cost
(NUMERICAL_FAILURE).  Each rule is pinned by a case whose outcome follows
from quantities computed independently of the rule: a least-squares
solution from np.linalg.lstsq, the exact damped step from an augmented
least-squares system, the unstopped trajectory of the same problem, or a
hand-computed damping sequence.
"""
import math

import numpy as np
import pytest

from oracle import ba, dense, lm, pcg, robust
from paper_2509_26581_amd import synth


def _linear(A, y):
    m, n = A.shape

    def fn(xs):
        return [sum(A[i, k] * xs[k] for k in range(n)) - y[i] for i in range(m)]

    return dense.DenseProblem(fn, n)


def _damped_step_lstsq(A, y, x, lam):
    """The damped step of a linear problem as the least-squares solution of
    [A; sqrt(lam D)] dx = [y - A x; 0] with D = diag(A^T A) clamped at 1e-6,
    computed by LAPACK's least-squares routine (not the normal equations)."""
    D = np.clip(np.einsum("ij,ij->j", A, A), 1e-6, 1e32)
    K = np.vstack([A, np.diag(np.sqrt(lam * D))])
    rhs = np.concatenate([y - A @ x, np.zeros(A.shape[1])])
    return np.linalg.lstsq(K, rhs, rcond=None)[0]


def test_cost_tol_stops_at_the_first_small_accepted_decrease():
    # a linear problem started away from its least-squares solution: the first
    # damped step lands next to the solution, the second one only removes the
    # remaining O(lambda) error, so with tol = 1e-6 the loop stops at trial 2
    rng = np.random.default_rng(12)
    A = rng.normal(size=(12, 4))
    y = rng.normal(size=12)
    x0 = rng.normal(size=4) * 3.0
    xs = np.linalg.lstsq(A, y, rcond=None)[0]
    Fmin = 0.5 * float(np.sum((A @ xs - y) ** 2))
    prob = _linear(A, y)
    res = lm.levenberg_marquardt(prob, x0, 20, tol=1e-6)
    assert res.termination == lm.TERM_COST_TOL and res.trials == 2
    assert all(e["accepted"] for e in res.log)
    # trial 1 reaches the damped step of the augmented system
    dx1 = _damped_step_lstsq(A, y, x0, 1e-4)
    F1 = 0.5 * float(np.sum((A @ (x0 + dx1) - y) ** 2))
    assert math.isclose(res.log[0]["candidate_cost"], F1, rel_tol=1e-10)
    assert (res.log[0]["cost"] - F1) / res.log[0]["cost"] > 1e-6
    assert (F1 - res.cost) / F1 < 1e-6
    assert abs(res.cost - Fmin) <= 1e-9 * Fmin


@pytest.mark.parametrize("tol", [1e-3, 3e-5])
def test_cost_tol_against_the_unstopped_trajectory(tol):
    # the rule applied by brute force to the tol = 0 trajectory of a BA
    # problem gives the trial the stopped run ends at
    sc = synth.make_scene("small", seed=40, n_cams=5, n_pts=120, noise_px=1.0)
    prob = ba.BAProblem(sc.n_cams, sc.n_pts, sc.cam_idx, sc.pt_idx, sc.obs)
    full = ba.solve(prob, sc.cams0, sc.pts0, 12)
    assert full.termination == lm.TERM_MAX_ITERS
    stop = None
    for k, e in enumerate(full.log):
        if e["accepted"] and (e["cost"] - e["candidate_cost"]) / e["cost"] < tol:
            stop = k
            break
    assert stop is not None
    res = ba.solve(prob, sc.cams0, sc.pts0, 12, tol=tol)
    assert res.termination == lm.TERM_COST_TOL
    assert res.trials == stop + 1
    assert res.cost == full.log[stop]["candidate_cost"]


def test_step_tol_fires_at_the_threshold_of_the_first_step():
    # far from the origin (|x| ~ 1e6) the first step of unit size is relative
    # 1e-6: STEP_TOL fires at trial 1 exactly when tol (|x0| + tol) >= |dx1|,
    # with |dx1| from the augmented least-squares step
    rng = np.random.default_rng(13)
    A = rng.normal(size=(10, 3))
    xs = 1e6 * np.ones(3)
    y = A @ xs + 0.01 * rng.normal(size=10)
    x0 = xs + rng.normal(size=3)
    dx1 = _damped_step_lstsq(A, y, x0, 1e-4)
    nx, nd = float(np.linalg.norm(x0)), float(np.linalg.norm(dx1))
    t_star = 0.5 * (-nx + math.sqrt(nx * nx + 4.0 * nd))   # t (|x0| + t) = |dx1|
    prob = _linear(A, y)
    above = lm.levenberg_marquardt(prob, x0, 10, tol=1.01 * t_star)
    assert above.termination == lm.TERM_STEP_TOL and above.trials == 1
    assert above.log[0]["accepted"]
    assert math.isclose(above.log[0]["step_norm"], nd, rel_tol=1e-8)
    below = lm.levenberg_marquardt(prob, x0, 10, tol=0.99 * t_star)
    assert below.trials >= 2


def test_step_tol_on_a_zero_step():
    # zero residual at the start: b = 0, the step is exactly zero and not
    # accepted (F' = F); |dx| = 0 <= tol (|x| + tol) holds even for tol = 0
    rng = np.random.default_rng(14)
    A = rng.normal(size=(6, 3))
    x0 = rng.normal(size=3)
    res = lm.levenberg_marquardt(_linear(A, A @ x0), x0, 5, tol=0.0)
    assert res.termination == lm.TERM_STEP_TOL and res.trials == 1
    assert res.log[0]["step_norm"] == 0.0 and not res.log[0]["accepted"]


def test_lambda_overflow_after_three_rejections_from_a_huge_damping():
    # with lambda0 = 1e31 the step is ~1e-31 of the parameters, x + dx == x,
    # F' == F and every trial is rejected: lambda 1e31 -> 2e31 -> 8e31 ->
    # 6.4e32 > 1e32 ends the loop after three trials
    sc = synth.make_scene("small", seed=41, n_cams=4, n_pts=60)
    prob = ba.BAProblem(sc.n_cams, sc.n_pts, sc.cam_idx, sc.pt_idx, sc.obs)
    res = ba.solve(prob, sc.cams0, sc.pts0, 50, initial_lambda=1e31)
    assert res.termination == lm.TERM_LAMBDA_OVERFLOW and res.trials == 3
    assert [e["lam"] for e in res.log] == [1e31, 2e31, 8e31]
    assert not any(e["accepted"] for e in res.log)
    assert all(e["candidate_cost"] == e["cost"] for e in res.log)
    np.testing.assert_array_equal(res.x[0], sc.cams0)


def test_numerical_failure_on_a_point_in_the_camera_plane():
    # a point with P_z = 0 in front of no camera: the projection divides by
    # zero, the starting cost is not finite, no trial runs
    sc = synth.make_scene("small", seed=42, n_cams=3, n_pts=20)
    cams = sc.cams0.copy()
    pts = sc.pts0.copy()
    cams[0, :6] = 0.0                     # R = I, t = 0: P = X
    j = int(sc.pt_idx[sc.cam_idx == 0][0])
    pts[j] = [1.0, 2.0, 0.0]
    prob = ba.BAProblem(sc.n_cams, sc.n_pts, sc.cam_idx, sc.pt_idx, sc.obs)
    with np.errstate(divide="ignore", invalid="ignore"):
        res = ba.solve(prob, cams, pts, 5)
    assert res.termination == lm.TERM_NUMERICAL_FAILURE and res.trials == 0
    assert not math.isfinite(res.cost)


# ------------------------------------------------------------ PCG breakdown
def test_pcg_breakdown_on_the_first_step_returns_the_start():
    # S = diag(1, -1), v = (0, 1), M = I: p = v, p^T S p = -1 <= 0
    S = np.diag([1.0, -1.0])
    x, k, why = pcg.pcg(S, np.array([0.0, 1.0]), np.eye(2), tol=1e-12)
    assert why == pcg.DONE_BREAKDOWN and k == 0
    np.testing.assert_array_equal(x, [0.0, 0.0])


def test_pcg_breakdown_on_the_second_step_keeps_the_first_iterate():
    # S = diag(2, -1), v = (1, 1), M = I, by hand: p1 = v, p1^T S p1 = 1,
    # alpha = 2, x1 = (2, 2), r1 = (-3, 3), beta = 18 / 2 = 9,
    # p2 = (6, 12), p2^T S p2 = 72 - 144 < 0: stop at x1 after one step
    S = np.diag([2.0, -1.0])
    x, k, why = pcg.pcg(S, np.array([1.0, 1.0]), np.eye(2), tol=1e-12)
    assert why == pcg.DONE_BREAKDOWN and k == 1
    np.testing.assert_allclose(x, [2.0, 2.0], rtol=0, atol=1e-15)


def test_pcg_column_scaling_equals_the_diagonal_preconditioner():
    # CG on the column-scaled system (D S D) y = D v, x = D y, iterate by
    # iterate equals PCG on S with M^-1 = D^2 (the Sec. IV-D column rescaling
    # with the identity preconditioner)
    rng = np.random.default_rng(15)
    B = rng.normal(size=(18, 18))
    S = B @ B.T + 18 * np.eye(18)
    S[:9, :9] *= 100.0
    v = rng.normal(size=18)
    s = 1.0 / (1.0 + np.sqrt(np.diag(S)))
    D = np.diag(s)
    for k in (1, 2, 5):
        y, ky, _ = pcg.pcg(D @ S @ D, D @ v, np.eye(18), tol=1e-30, max_iters=k)
        x, kx, _ = pcg.pcg(S, v, D @ D, tol=1e-30, max_iters=k)
        assert kx == ky == k
        np.testing.assert_allclose(D @ y, x, rtol=1e-10, atol=1e-14)
    # and with block-Jacobi blocks the scaling cancels: the same iterates
    Mb = pcg.block_jacobi(S)
    Mbs = pcg.block_jacobi(D @ S @ D)
    for k in (1, 3):
        y, _, _ = pcg.pcg(D @ S @ D, D @ v, Mbs, tol=1e-30, max_iters=k)
        x, _, _ = pcg.pcg(S, v, Mb, tol=1e-30, max_iters=k)
        np.testing.assert_allclose(D @ y, x, rtol=1e-10, atol=1e-14)


# ------------------------------------------------------ residual statistics
def test_residual_statistics_by_hand():
    # one camera at the origin looking down -z (R = I, t = 0, f = 500, no
    # distortion) and two points on its optical axis: both project to (0, 0),
    # so r = -u exactly
    cams = np.array([[0, 0, 0, 0, 0, 0, 500.0, 0, 0]])
    pts = np.array([[0, 0, -10.0], [0, 0, -20.0]])
    uv = np.array([[3.0, 4.0], [0.3, 0.4]])
    for loss, delta, chi2 in [(robust.SQUARED, 1.0, 25.0 + 0.25),
                              (robust.HUBER, 1.0, (2 * 5.0 - 1.0) + 0.25)]:
        prob = ba.BAProblem(1, 2, np.array([0, 0]), np.array([0, 1]), uv, loss=loss,
                            delta=delta)
        c, mse = prob.residual_stats((cams, pts))
        assert math.isclose(c, chi2, rel_tol=1e-15)
        assert math.isclose(mse, (25.0 + 0.25) / 2, rel_tol=1e-15)
        assert math.isclose(prob.cost((cams, pts)), 0.5 * chi2, rel_tol=1e-15)
