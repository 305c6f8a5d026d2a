"""Pins of the visual-inertial LM problem (oracle/vi.py) against what the
mathematics fixes: the closed-form stereo Jacobian against the dual numbers of
the factor definitions, the gradient b = J^T r against central differences
of the cost along manifold directions, zero stereo cost at the truth of
noise-free data, and the LM loop's descent to the noise level."""
import numpy as np

from oracle import imu, lm, vi
from paper_2509_26581_amd import synth_vi


def _scene(seed=0, n_kf=8, n_pts=120, noise=True):
    kw = {} if noise else dict(gyro_noise=0.0, acc_noise=0.0, gyro_walk=0.0, acc_walk=0.0,
                               pixel_noise=0.0)
    return synth_vi.make_vi_scene(seed=seed, n_kf=n_kf, n_pts=n_pts, **kw)


def _problem(sc, delta2=7.815):
    pre = [imu.preintegrate(sc.gyro[f], sc.acc[f], sc.imu_dt, sc.bg_true[f], sc.ba_true[f],
                            1.7e-4, 2e-3) for f in range(sc.n_kf - 1)]
    return vi.VIProblem(sc.st_kf, sc.st_pt, sc.st_obs, sc.intr, pre, sigma_px=1.0,
                        delta2=delta2, sigma_gw=2e-5, sigma_aw=3e-3)


def _truth(sc):
    return vi.VIState(sc.R_true, sc.p_true, sc.v_true, sc.bg_true, sc.ba_true, sc.pts)


def _perturbed(sc, seed=1, rot=0.01, pos=0.05, vel=0.05, pts=0.05):
    rng = np.random.default_rng(seed)
    K = sc.n_kf
    R = np.stack([sc.R_true[k] @ imu.so3_exp(rng.normal(0, rot, 3) if k else np.zeros(3))
                  for k in range(K)])
    dp = rng.normal(0, pos, (K, 3))
    dv = rng.normal(0, vel, (K, 3))
    dp[0] = dv[0] = 0.0
    return vi.VIState(R, sc.p_true + dp, sc.v_true + dv, sc.bg_true.copy(), sc.ba_true.copy(),
                      sc.pts + rng.normal(0, pts, sc.pts.shape))


def test_stereo_jacobian_closed_form_equals_dual_numbers():
    rng = np.random.default_rng(3)
    intr = (380.0, 380.0, 320.0, 240.0, 0.11)
    for _ in range(10):
        R = imu.so3_exp(rng.normal(0, 0.5, 3))
        p = rng.normal(0, 1.0, 3)
        X = p + R @ np.array([rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(3, 10)])
        obs = rng.normal(0, 1.0, 3) + [300.0, 200.0, 290.0]
        r_d, J_d = imu.stereo_residual_and_jacobian(R, p, X, *intr, obs)
        Xc, pred = vi.stereo_project(R[None], p[None], X[None], intr)
        J = vi.stereo_jacobian(R[None], Xc, intr)[0]
        np.testing.assert_allclose(pred[0] - obs, r_d, rtol=0, atol=1e-9)
        np.testing.assert_allclose(J, J_d, rtol=1e-10, atol=1e-8)


def test_gradient_equals_central_differences_of_the_cost():
    sc = _scene(seed=2)
    prob = _problem(sc, delta2=2.0)          # many stereo terms in the linear branch
    x = _perturbed(sc)
    lin = prob.linearize(x)
    rng = np.random.default_rng(4)
    n = prob.n_vars(x)
    for _ in range(3):
        d = rng.normal(size=n)
        d[0:15] = 0.0
        d *= 1e-6 / np.linalg.norm(d)
        g = (prob.cost(prob.step(x, d)) - prob.cost(prob.step(x, -d))) / 2.0
        assert abs(g - lin["b"] @ d) <= 1e-5 * abs(lin["b"] @ d) + 1e-12, (g, lin["b"] @ d)


def test_stereo_cost_vanishes_at_the_truth_of_noise_free_data():
    sc = _scene(seed=5, noise=False)
    prob = _problem(sc)
    x = _truth(sc)
    _, _, r = prob._stereo(x)
    assert np.max(np.abs(r)) < 1e-8


def test_model_decrease_is_the_undamped_quadratic_model():
    # a tiny step: the model decrease predicts the cost decrease to second order
    sc = _scene(seed=6)
    prob = _problem(sc, delta2=0.0)
    x = _perturbed(sc, seed=7)
    lin = prob.linearize(x)
    dx = prob.solve(lin, 1e-4, 1e-6, 1e32) * 1e-3
    L = prob.model_decrease(lin, dx)
    dF = prob.cost(x) - prob.cost(prob.step(x, dx))
    assert L > 0.0
    assert abs(dF - L) <= 1e-3 * L


def test_lm_descends_to_the_noise_level():
    sc = _scene(seed=8, n_kf=8, n_pts=100)
    prob = _problem(sc)
    x0 = _perturbed(sc, seed=9)
    res = lm.levenberg_marquardt(prob, x0, 15)
    costs = [t["cost"] for t in res.log if t["accepted"]] + [res.cost]
    assert all(b <= a for a, b in zip(costs, costs[1:]))
    assert res.cost < 0.05 * res.initial_cost
    # the estimate lies near the truth (keyframe 0 held at it); a point's
    # stereo depth is only known to about z^2 sigma_px / (f b) (metres at
    # 20 m with an 11 cm baseline), so the points are judged by the median
    assert np.max(np.abs(res.x.p - sc.p_true)) < 0.02
    assert np.median(np.linalg.norm(res.x.X - sc.pts, axis=1)) < 0.05
