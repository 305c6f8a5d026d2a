"""The visual-inertial LM solve on the GPU (gba_vi_solve, in both forms of
the damped step: PCG on the keyframe Schur complement with point
back-substitution, and PCG on the whole damped system over keyframe states
and points) against the oracle's LM with exact dense solves (oracle/vi.py):
per-trial costs, damping and decisions, the final cost and the final states
and points; and the truncated Schur-form steps against the oracle's Schur
PCG.  The GPU path preintegrates its own IMU intervals
(gba_vi_preintegrate); the oracle uses its own."""
import numpy as np
import pytest

from oracle import imu, lm, vi
from paper_2509_26581_amd import gba, synth_vi

pytestmark = pytest.mark.gpu

SIG_G, SIG_A, SIG_GW, SIG_AW = 1.7e-4, 2e-3, 2e-5, 3e-3


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gba.load()


def _setup(seed, n_kf, n_pts, delta2):
    sc = synth_vi.make_vi_scene(seed=seed, n_kf=n_kf, n_pts=n_pts)
    rng = np.random.default_rng(seed + 100)
    R0 = np.stack([sc.R_true[k] @ imu.so3_exp(rng.normal(0, 0.01, 3) if k else np.zeros(3))
                   for k in range(n_kf)])
    dp = rng.normal(0, 0.05, (n_kf, 3))
    dv = rng.normal(0, 0.05, (n_kf, 3))
    dp[0] = dv[0] = 0.0
    X0 = sc.pts + rng.normal(0, 0.05, sc.pts.shape)
    x0 = vi.VIState(R0, sc.p_true + dp, sc.v_true + dv, sc.bg_true.copy(), sc.ba_true.copy(), X0)
    pre_o = [imu.preintegrate(sc.gyro[f], sc.acc[f], sc.imu_dt, sc.bg_true[f], sc.ba_true[f],
                              SIG_G, SIG_A) for f in range(n_kf - 1)]
    prob = vi.VIProblem(sc.st_kf, sc.st_pt, sc.st_obs, sc.intr, pre_o, sigma_px=1.0,
                        delta2=delta2, sigma_gw=SIG_GW, sigma_aw=SIG_AW)
    m = sc.gyro.shape[1]
    off = np.arange(n_kf, dtype=np.int64) * m
    bias0 = np.concatenate([sc.bg_true[:-1], sc.ba_true[:-1]], axis=1)
    pre_g = gba.gba_vi_preintegrate(0, off, sc.gyro.reshape(-1, 3), sc.acc.reshape(-1, 3),
                                    sc.imu_dt, bias0, SIG_G, SIG_A)
    states = np.concatenate([np.array([imu.so3_log(R) for R in R0]), x0.p, x0.v, x0.bg, x0.ba],
                            axis=1)
    return sc, prob, x0, states, pre_g


def _gpu(sc, states, x0, pre_g, trials, delta2, **opt):
    o = gba.vi_options(**opt)
    return gba.gba_vi_solve(0, states, x0.X, sc.st_kf, sc.st_pt, sc.st_obs, sc.intr, pre_g, trials,
                            sigma_px=1.0, huber_delta2=delta2, sigma_gw=SIG_GW, sigma_aw=SIG_AW,
                            options=o)


@pytest.mark.parametrize("solver", [gba.GBA_SOLVER_SCHUR, gba.GBA_SOLVER_FULL])
@pytest.mark.parametrize("delta2", [0.0, 7.815])
def test_vi_lm_trajectory_matches_the_oracle(delta2, solver):
    sc, prob, x0, states, pre_g = _setup(seed=8, n_kf=8, n_pts=100, delta2=delta2)
    res = lm.levenberg_marquardt(prob, x0, 8)
    st, X, rep, log = _gpu(sc, states, x0, pre_g, 8, delta2, pcg_tol=1e-12, pcg_max_iters=4000,
                           solver=solver)
    assert len(log) == len(res.log)
    assert abs(rep["initial_cost"] - res.initial_cost) <= 1e-9 * res.initial_cost
    for a, b in zip(log, res.log):
        assert abs(a["cost"] - b["cost"]) <= 1e-8 * b["cost"], (a, b)
        if abs(b["cost"] - b["candidate_cost"]) <= 1e-8 * b["cost"]:
            break   # decrease at the rounding level: decisions are rounding noise
        assert a["accepted"] == b["accepted"], (a, b)
        assert abs(a["lam"] - b["lam"]) <= 1e-9 * b["lam"], (a, b)
        assert abs(a["model_decrease"] - b["model_decrease"]) <= 1e-6 * abs(b["model_decrease"]), (a, b)
    assert abs(rep["final_cost"] - res.cost) <= 1e-8 * res.cost
    R = np.stack([imu.so3_exp(w) for w in st[:, 0:3]])
    assert np.max(np.abs(R - res.x.R)) < 1e-7
    np.testing.assert_allclose(st[:, 3:6], res.x.p, rtol=0, atol=1e-7)
    np.testing.assert_allclose(st[:, 6:9], res.x.v, rtol=0, atol=1e-7)
    np.testing.assert_allclose(st[:, 9:15], np.concatenate([res.x.bg, res.x.ba], axis=1),
                               rtol=0, atol=1e-7)
    np.testing.assert_allclose(X, res.x.X, rtol=0, atol=1e-6 * np.max(np.abs(res.x.X)))
    # the first keyframe is the gauge: unchanged (its rotation to the
    # rounding of the angle-axis / matrix round trip at the boundary)
    np.testing.assert_array_equal(st[0, 3:], states[0, 3:])
    np.testing.assert_allclose(st[0, 0:3], states[0, 0:3], rtol=0, atol=1e-14)


@pytest.mark.parametrize("solver", [gba.GBA_SOLVER_SCHUR, gba.GBA_SOLVER_FULL])
def test_vi_two_keyframes_and_unobserved_points(solver):
    # the smallest window (one free keyframe behind the fixed first) with
    # points that no keyframe observes placed between observed points in the
    # caller's order: their rows of the damped system hold only the damping
    # and a zero gradient, so they come back exactly as given, at their own
    # places; everything else follows the oracle
    sc, prob, x0, states, pre_g = _setup(seed=12, n_kf=2, n_pts=60, delta2=7.815)
    N, extra = x0.X.shape[0], 7
    rng = np.random.default_rng(13)
    pos = np.sort(rng.choice(N + extra, extra, replace=False))
    keep = np.setdiff1d(np.arange(N + extra), pos)   # old point j is now keep[j]
    X0 = np.empty((N + extra, 3))
    X0[keep] = x0.X
    X0[pos] = rng.normal(0.0, 3.0, (extra, 3))
    pt = keep[sc.st_pt]
    prob2 = vi.VIProblem(sc.st_kf, pt, sc.st_obs, sc.intr, prob.pre, sigma_px=1.0, delta2=7.815,
                         sigma_gw=SIG_GW, sigma_aw=SIG_AW)
    xs = vi.VIState(x0.R, x0.p, x0.v, x0.bg, x0.ba, X0)
    res = lm.levenberg_marquardt(prob2, xs, 5)
    st, X, rep, log = gba.gba_vi_solve(0, states, X0, sc.st_kf, pt, sc.st_obs, sc.intr, pre_g, 5,
                                       sigma_px=1.0, huber_delta2=7.815, sigma_gw=SIG_GW,
                                       sigma_aw=SIG_AW,
                                       options=gba.vi_options(pcg_tol=1e-12, pcg_max_iters=4000,
                                                              solver=solver))
    assert len(log) == len(res.log)
    assert abs(rep["initial_cost"] - res.initial_cost) <= 1e-9 * res.initial_cost
    for a, b in zip(log, res.log):
        assert abs(a["cost"] - b["cost"]) <= 1e-8 * b["cost"], (a, b)
        if abs(b["cost"] - b["candidate_cost"]) <= 1e-8 * b["cost"]:
            break
        assert a["accepted"] == b["accepted"], (a, b)
    assert abs(rep["final_cost"] - res.cost) <= 1e-8 * res.cost
    np.testing.assert_array_equal(X[pos], X0[pos])
    np.testing.assert_array_equal(res.x.X[pos], X0[pos])
    np.testing.assert_allclose(X[keep], res.x.X[keep], rtol=0, atol=1e-6 * np.max(np.abs(res.x.X)))
    np.testing.assert_allclose(st[:, 3:6], res.x.p, rtol=0, atol=1e-7)
    np.testing.assert_array_equal(st[0, 3:], states[0, 3:])


@pytest.mark.parametrize("k", [1, 3, 7])
def test_vi_truncated_schur_step_matches_the_oracle(k):
    # k PCG steps on S from the first linearisation: the candidate cost, the
    # model decrease and the step norm of the GPU's step against the oracle's
    # Schur PCG step (same preconditioner, same stop rules)
    # (with one more point that no keyframe observes: its step is zero)
    sc, prob, x0, states, pre_g = _setup(seed=5, n_kf=9, n_pts=120, delta2=7.815)
    x0 = vi.VIState(x0.R, x0.p, x0.v, x0.bg, x0.ba, np.vstack([x0.X, [[0.5, -0.2, 7.0]]]))
    st, X, rep, log = _gpu(sc, states, x0, pre_g, 1, 7.815, pcg_tol=0.0, pcg_max_iters=k,
                           solver=gba.GBA_SOLVER_SCHUR)
    lin = prob.linearize(x0)
    dx, steps = prob.schur_pcg_step(lin, 1e-4, 1e-6, 1e32, 0.0, k)
    assert log[0]["pcg_iters"] == steps == k
    F1 = prob.cost(prob.step(x0, dx))
    L = prob.model_decrease(lin, dx)
    t = log[0]
    assert abs(t["candidate_cost"] - F1) <= 1e-9 * F1, (t, F1)
    assert abs(t["model_decrease"] - L) <= 1e-8 * abs(L), (t, L)
    assert abs(t["step_norm"] - np.linalg.norm(dx)) <= 1e-8 * np.linalg.norm(dx)


@pytest.mark.parametrize("solver", [gba.GBA_SOLVER_SCHUR, gba.GBA_SOLVER_FULL])
def test_vi_rejection_ratio(solver):
    # a ratio just above 1 ends the PCG at the first rise of |r| and returns
    # the best iterate; in the Schur form the step matches the oracle's Schur
    # PCG with the same ratio, in both forms an infinite or zero ratio is the
    # plain PCG
    from oracle import pcg as opcg
    sc, prob, x0, states, pre_g = _setup(seed=5, n_kf=9, n_pts=120, delta2=7.815)
    kw = dict(pcg_tol=0.0, pcg_max_iters=60, solver=solver)
    _, _, _, plain = _gpu(sc, states, x0, pre_g, 1, 7.815, **kw)
    _, _, _, off = _gpu(sc, states, x0, pre_g, 1, 7.815, pcg_rejection_ratio=float("inf"), **kw)
    assert off[0]["pcg_iters"] == plain[0]["pcg_iters"] == 60
    # (atomic sums: two runs agree to rounding, not bit for bit)
    assert abs(off[0]["step_norm"] - plain[0]["step_norm"]) <= 1e-10 * plain[0]["step_norm"]
    _, _, _, rej = _gpu(sc, states, x0, pre_g, 1, 7.815, pcg_rejection_ratio=1.001, **kw)
    assert rej[0]["pcg_iters"] < 60
    if solver == gba.GBA_SOLVER_SCHUR:
        lin = prob.linearize(x0)
        dx, steps = prob.schur_pcg_step(lin, 1e-4, 1e-6, 1e32, 0.0, 60, ratio=1.001)
        assert prob.last_reason == opcg.DONE_REJECTED
        assert rej[0]["pcg_iters"] == steps
        L = prob.model_decrease(lin, dx)
        assert abs(rej[0]["model_decrease"] - L) <= 1e-8 * abs(L)
        assert abs(rej[0]["step_norm"] - np.linalg.norm(dx)) <= 1e-8 * np.linalg.norm(dx)


@pytest.mark.parametrize("precision,solver", [(gba.GBA_FP64, gba.GBA_SOLVER_SCHUR),
                                              (gba.GBA_MIXED_FP32, gba.GBA_SOLVER_SCHUR),
                                              (gba.GBA_FP64, gba.GBA_SOLVER_FULL)])
def test_vi_long_tracks_match_the_oracle(precision, solver):
    # 70 keyframes that all see the same 40 points: every point has more
    # than 64 observations, so its sums span wavefronts (the split-point
    # paths of the Schur form); trajectory and one truncated step against
    # the oracle
    sc, prob, x0, states, pre_g = _setup(seed=4, n_kf=70, n_pts=40, delta2=7.815)
    assert np.bincount(sc.st_pt).max() > 64
    res = lm.levenberg_marquardt(prob, x0, 3)
    st, X, rep, log = _gpu(sc, states, x0, pre_g, 3, 7.815, pcg_tol=1e-12, pcg_max_iters=4000,
                           precision=precision, solver=solver)
    tol = 1e-8 if precision == gba.GBA_FP64 else 1e-6
    for a, b in zip(log, res.log):
        assert abs(a["cost"] - b["cost"]) <= tol * b["cost"], (a, b)
        assert a["accepted"] == b["accepted"]
    assert abs(rep["final_cost"] - res.cost) <= tol * res.cost
    np.testing.assert_allclose(X, res.x.X, rtol=0, atol=1e-4 * np.max(np.abs(res.x.X)))
    if precision == gba.GBA_FP64 and solver == gba.GBA_SOLVER_SCHUR:
        st3, X3, rep3, log3 = _gpu(sc, states, x0, pre_g, 1, 7.815, pcg_tol=0.0, pcg_max_iters=3)
        lin = prob.linearize(x0)
        dx, steps = prob.schur_pcg_step(lin, 1e-4, 1e-6, 1e32, 0.0, 3)
        L = prob.model_decrease(lin, dx)
        assert abs(log3[0]["model_decrease"] - L) <= 1e-8 * abs(L)
        assert abs(log3[0]["step_norm"] - np.linalg.norm(dx)) <= 1e-8 * np.linalg.norm(dx)


@pytest.mark.parametrize("solver", [gba.GBA_SOLVER_SCHUR, gba.GBA_SOLVER_FULL])
def test_vi_inertial_only_matches_the_oracle(solver):
    # no points and no stereo observations: the inertial and bias terms
    # alone (the empty-observation paths of every kernel)
    sc = synth_vi.make_vi_scene(seed=6, n_kf=7, n_pts=50)
    K = sc.n_kf
    pre_o = [imu.preintegrate(sc.gyro[f], sc.acc[f], sc.imu_dt, sc.bg_true[f], sc.ba_true[f],
                              SIG_G, SIG_A) for f in range(K - 1)]
    e = np.zeros(0, np.int64)
    prob = vi.VIProblem(e, e, np.zeros((0, 3)), sc.intr, pre_o, sigma_px=1.0, delta2=0.0,
                        sigma_gw=SIG_GW, sigma_aw=SIG_AW)
    rng = np.random.default_rng(1)
    R0 = np.stack([sc.R_true[k] @ imu.so3_exp(rng.normal(0, 0.01, 3) if k else np.zeros(3))
                   for k in range(K)])
    dp = rng.normal(0, 0.05, (K, 3))
    dp[0] = 0.0
    x0 = vi.VIState(R0, sc.p_true + dp, sc.v_true.copy(), sc.bg_true.copy(), sc.ba_true.copy(),
                    np.zeros((0, 3)))
    res = lm.levenberg_marquardt(prob, x0, 4)
    m = sc.gyro.shape[1]
    pre_g = gba.gba_vi_preintegrate(0, np.arange(K, dtype=np.int64) * m, sc.gyro.reshape(-1, 3),
                                    sc.acc.reshape(-1, 3), sc.imu_dt,
                                    np.concatenate([sc.bg_true[:-1], sc.ba_true[:-1]], axis=1),
                                    SIG_G, SIG_A)
    states = np.concatenate([np.array([imu.so3_log(R) for R in R0]), x0.p, x0.v, x0.bg, x0.ba], axis=1)
    st, X, rep, log = gba.gba_vi_solve(0, states, np.zeros((0, 3)), e, e, np.zeros((0, 3)), sc.intr,
                                       pre_g, 4, sigma_px=1.0, sigma_gw=SIG_GW, sigma_aw=SIG_AW,
                                       options=gba.vi_options(pcg_tol=1e-12, pcg_max_iters=4000,
                                                              solver=solver))
    assert X.shape == (0, 3) and len(log) == len(res.log)
    assert abs(rep["initial_cost"] - res.initial_cost) <= 1e-9 * res.initial_cost
    for a, b in zip(log, res.log):
        assert abs(a["cost"] - b["cost"]) <= 1e-8 * b["cost"] + 1e-9, (a, b)
        assert a["accepted"] == b["accepted"]
    np.testing.assert_allclose(st[:, 3:6], res.x.p, rtol=0, atol=1e-7)
    np.testing.assert_allclose(st[:, 6:9], res.x.v, rtol=0, atol=1e-7)


@pytest.mark.parametrize("solver", [gba.GBA_SOLVER_SCHUR, gba.GBA_SOLVER_FULL])
def test_vi_mixed_fp32_within_the_mixed_bounds(solver):
    # W = J_k^T J_p stored in FP32 (Schur form): final cost within 1e-4 and
    # the solution within 1e-3 relative of the oracle's FP64 LM (the mixed
    # bounds), and the first trial's step close to the FP64 path's
    delta2 = 7.815
    sc, prob, x0, states, pre_g = _setup(seed=8, n_kf=8, n_pts=100, delta2=delta2)
    res = lm.levenberg_marquardt(prob, x0, 8)
    st, X, rep, log = _gpu(sc, states, x0, pre_g, 8, delta2, pcg_tol=1e-12, pcg_max_iters=4000,
                           precision=gba.GBA_MIXED_FP32, solver=solver)
    st64, X64, rep64, log64 = _gpu(sc, states, x0, pre_g, 8, delta2, pcg_tol=1e-12,
                                   pcg_max_iters=4000, solver=solver)
    assert abs(rep["final_cost"] - res.cost) <= 1e-4 * res.cost
    b = np.concatenate([res.x.p.ravel(), res.x.v.ravel(), res.x.bg.ravel(), res.x.ba.ravel(),
                        res.x.X.ravel()])
    a = np.concatenate([st[:, 3:6].ravel(), st[:, 6:9].ravel(), st[:, 9:12].ravel(),
                        st[:, 12:15].ravel(), X.ravel()])
    assert np.linalg.norm(a - b) <= 1e-3 * np.linalg.norm(b)
    t, t64 = log[0], log64[0]
    # the FP32 storage moves the step at FP32's rounding level (and so is in use)
    dstep = abs(t["step_norm"] - t64["step_norm"]) / t64["step_norm"]
    assert 1e-12 < dstep < 1e-4, dstep
    assert abs(t["model_decrease"] - t64["model_decrease"]) <= 1e-5 * abs(t64["model_decrease"])
    assert abs(t["candidate_cost"] - t64["candidate_cost"]) <= 1e-5 * t64["candidate_cost"]
    print("mixed fp32: final cost rel", abs(rep["final_cost"] - res.cost) / res.cost,
          "solution rel", np.linalg.norm(a - b) / np.linalg.norm(b),
          "first-trial step norm rel", dstep, "model decrease rel",
          abs(t["model_decrease"] - t64["model_decrease"]) / abs(t64["model_decrease"]))


@pytest.mark.parametrize("solver", [gba.GBA_SOLVER_SCHUR, gba.GBA_SOLVER_FULL])
def test_vi_truncated_pcg_still_descends(solver):
    # a loose PCG: every accepted trial lowers the cost
    sc, prob, x0, states, pre_g = _setup(seed=3, n_kf=10, n_pts=150, delta2=7.815)
    st, X, rep, log = _gpu(sc, states, x0, pre_g, 10, 7.815, pcg_tol=1e-3, pcg_max_iters=30,
                           solver=solver)
    costs = [t["cost"] for t in log] + [rep["final_cost"]]
    assert all(b <= a for a, b in zip(costs, costs[1:]))
    assert rep["final_cost"] < 0.2 * rep["initial_cost"]
    assert rep["pcg_iters_total"] <= 30 * rep["trials"]


def test_vi_solve_errors():
    sc, prob, x0, states, pre_g = _setup(seed=1, n_kf=4, n_pts=30, delta2=0.0)
    with pytest.raises(gba.GbaError) as e:
        gba.gba_vi_solve(0, states[:1], x0.X, sc.st_kf[:0], sc.st_pt[:0], sc.st_obs[:0], sc.intr,
                         pre_g[:0], 3)
    assert e.value.status == -1                      # one keyframe
    bad = sc.st_pt.copy()
    bad[0] = len(x0.X)
    with pytest.raises(gba.GbaError) as e:
        gba.gba_vi_solve(0, states, x0.X, sc.st_kf, bad, sc.st_obs, sc.intr, pre_g, 3)
    assert e.value.status == -2                      # unknown point
    with pytest.raises(gba.GbaError) as e:
        gba.gba_vi_solve(0, states, x0.X, sc.st_kf, sc.st_pt, sc.st_obs, sc.intr, pre_g, 3,
                         sigma_px=0.0)
    assert e.value.status == -1
    with pytest.raises(gba.GbaError) as e:
        _gpu(sc, states, x0, pre_g, 3, 0.0, solver=7)
    assert e.value.status == -1                      # unknown solver form
    with pytest.raises(gba.GbaError) as e:
        _gpu(sc, states, x0, pre_g, 3, 0.0, precision=gba.GBA_MIXED_BF16)
    assert e.value.status == -1


def test_vi_full_size_configuration():
    """The measured configuration (2,000 keyframes 0.25 s apart with a 200 Hz
    IMU, 300k points seen within three keyframes of their anchor, ~2.07M
    stereo observations, Huber, W in FP32, Schur form, PCG tol 1e-6 max 100),
    as bench.py runs it.  The oracle cannot solve it densely, so it checks
    what holds at any size: the reported initial and final costs equal the
    oracle's cost (its own preintegration) at the start and at the returned
    states and points, accepted costs decrease, the solve makes progress and
    the first keyframe stays fixed."""
    from scipy.spatial.transform import Rotation
    sc = synth_vi.make_vi_scene(seed=0, n_kf=2000, n_pts=300000, window=3)
    K = sc.n_kf
    rng = np.random.default_rng(1)
    dth = rng.normal(0, 0.01, (K, 3))
    dth[0] = 0.0
    R0 = (Rotation.from_matrix(sc.R_true) * Rotation.from_rotvec(dth)).as_rotvec()
    dp = rng.normal(0, 0.05, (K, 3))
    dv = rng.normal(0, 0.05, (K, 3))
    dp[0] = dv[0] = 0.0
    states = np.concatenate([R0, sc.p_true + dp, sc.v_true + dv, sc.bg_true, sc.ba_true], axis=1)
    pts0 = sc.pts + rng.normal(0, 0.05, sc.pts.shape)
    m = sc.gyro.shape[1]
    off = np.arange(K, dtype=np.int64) * m
    bias0 = np.concatenate([sc.bg_true[:-1], sc.ba_true[:-1]], axis=1)
    pre_g = gba.gba_vi_preintegrate(0, off, sc.gyro.reshape(-1, 3), sc.acc.reshape(-1, 3), sc.imu_dt,
                                    bias0, SIG_G, SIG_A)
    o = gba.vi_options(pcg_max_iters=100, pcg_tol=1e-6, precision=gba.GBA_MIXED_FP32)
    st, X, rep, log = gba.gba_vi_solve(0, states, pts0, sc.st_kf, sc.st_pt, sc.st_obs, sc.intr, pre_g, 5,
                                       sigma_px=1.0, huber_delta2=7.815, sigma_gw=SIG_GW, sigma_aw=SIG_AW,
                                       options=o)
    pre_o = [imu.preintegrate(sc.gyro[f], sc.acc[f], sc.imu_dt, sc.bg_true[f], sc.ba_true[f], SIG_G, SIG_A)
             for f in range(K - 1)]
    prob = vi.VIProblem(sc.st_kf, sc.st_pt, sc.st_obs, sc.intr, pre_o, sigma_px=1.0, delta2=7.815,
                        sigma_gw=SIG_GW, sigma_aw=SIG_AW)

    def state(s15, P):
        R = Rotation.from_rotvec(s15[:, 0:3]).as_matrix()
        return vi.VIState(R, s15[:, 3:6], s15[:, 6:9], s15[:, 9:12], s15[:, 12:15], P)

    F0 = prob.cost(state(states, pts0))
    assert abs(rep["initial_cost"] - F0) <= 1e-9 * F0
    F = prob.cost(state(st, X))
    assert abs(rep["final_cost"] - F) <= 1e-9 * F
    acc = [t["candidate_cost"] for t in log if t["accepted"]]
    assert len(acc) >= 3 and all(b < a for a, b in zip(acc, acc[1:]))
    assert rep["final_cost"] < 0.01 * rep["initial_cost"]
    assert rep["pcg_iters_total"] <= 100 * rep["trials"]
    np.testing.assert_array_equal(st[0, 3:], states[0, 3:])
    np.testing.assert_allclose(st[0, 0:3], states[0, 0:3], rtol=0, atol=1e-14)
