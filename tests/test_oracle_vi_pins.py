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


def _schur_setup(seed=10, lam=1e-3):
    sc = _scene(seed=seed, n_kf=6, n_pts=60)
    prob = _problem(sc)
    x = _perturbed(sc, seed=seed + 1)
    return prob, prob.linearize(x), lam


def test_schur_step_converged_equals_the_full_solve():
    prob, lin, lam = _schur_setup()
    dx_full = prob.solve(lin, lam, 1e-6, 1e32)
    dx, steps = prob.schur_pcg_step(lin, lam, 1e-6, 1e32, 0.0, 400)
    assert steps > 0
    np.testing.assert_allclose(dx, dx_full, rtol=0, atol=1e-9 * np.max(np.abs(dx_full)))


def test_schur_back_substitution_solves_the_point_rows_exactly():
    # a truncated keyframe step: the point rows of the damped full system
    # still hold exactly, whatever x_k is
    prob, lin, lam = _schur_setup(seed=11)
    dx, _ = prob.schur_pcg_step(lin, lam, 1e-6, 1e32, 0.0, 2)
    f = lin["free"]
    H = lin["H"][np.ix_(f, f)]
    Hd = H + lam * np.diag(np.clip(np.diag(H), 1e-6, 1e32))
    nk = 15 * (prob.K - 1)
    res = Hd @ dx[f] + lin["b"][f]
    assert np.max(np.abs(res[nk:])) <= 1e-9 * np.max(np.abs(lin["b"][f]))
    assert np.max(np.abs(res[:nk])) > 1e-6 * np.max(np.abs(lin["b"][f]))   # truncated


def test_schur_iterates_minimise_the_energy_over_the_preconditioned_krylov_space():
    # CG's k-th iterate is the Galerkin solution on span{z0, (M S) z0, ...,
    # (M S)^(k-1) z0}, z0 = M v, M the inverse diagonal blocks of S
    prob, lin, lam = _schur_setup(seed=12)
    S, v, A, B, C, bk, bp = prob.reduced_system(lin, lam, 1e-6, 1e32)
    Minv = np.zeros_like(S)
    for a in range(0, len(v), 15):
        Minv[a:a + 15, a:a + 15] = np.linalg.inv(S[a:a + 15, a:a + 15])
    nk = len(v)
    for k in (1, 2, 4):
        dx, steps = prob.schur_pcg_step(lin, lam, 1e-6, 1e32, 0.0, k)
        assert steps == k
        xk = dx[lin["free"]][:nk]
        V = [Minv @ v]
        for _ in range(k - 1):
            V.append(Minv @ (S @ V[-1]))
        Q, _ = np.linalg.qr(np.stack(V, axis=1))
        y = np.linalg.solve(Q.T @ S @ Q, Q.T @ v)
        np.testing.assert_allclose(xk, Q @ y, rtol=0, atol=1e-8 * np.max(np.abs(Q @ y)))


def test_schur_diagonal_blocks_are_the_per_observation_sums():
    # each (keyframe, point) pair is observed once in these scenes, so the
    # diagonal block of S at keyframe k is its damped block minus, over its
    # observations e of point j, W_e C_j^-1 W_e^T with W_e = J_k^T J_p
    prob, lin, lam = _schur_setup(seed=13)
    S, v, A, B, C, bk, bp = prob.reduced_system(lin, lam, 1e-6, 1e32)
    J = lin["J"]
    K = prob.K
    assert len(set(zip(prob.kf.tolist(), prob.pt.tolist()))) == len(prob.kf)
    for k in range(1, K):
        blk = A[15 * (k - 1):15 * k, 15 * (k - 1):15 * k].copy()
        for e in np.flatnonzero(prob.kf == k):
            j = prob.pt[e]
            Jk = J[3 * e:3 * e + 3, 15 * k:15 * k + 15]
            Jp = J[3 * e:3 * e + 3, 15 * K + 3 * j:15 * K + 3 * j + 3]
            Cj = C[3 * j:3 * j + 3, 3 * j:3 * j + 3]
            W = Jk.T @ Jp
            blk -= W @ np.linalg.solve(Cj, W.T)
        np.testing.assert_allclose(S[15 * (k - 1):15 * k, 15 * (k - 1):15 * k], blk,
                                   rtol=0, atol=1e-9 * np.max(np.abs(blk)))
