"""Pins of the oracle's preconditioned conjugate gradients (oracle/pcg.py):
the reduced system against the exact block-Cholesky step, convergence to a
direct solve, the Krylov-subspace minimisation property of the iterates,
termination in as many steps as distinct eigenvalues, and the rejection ratio
against an explicit enumeration of the iterates.
"""
import numpy as np
import pytest

from oracle import ba, pcg, robust
from paper_2509_26581_amd import synth


def _ba_system(seed=34, lam=1e-2, n_cams=6, n_pts=200):
    sc = synth.make_scene("small", seed=seed, n_cams=n_cams, n_pts=n_pts)
    prob = ba.BAProblem(sc.n_cams, sc.n_pts, sc.cam_idx, sc.pt_idx, sc.obs,
                        loss=robust.HUBER, delta=sc.delta)
    lin = prob.linearize((sc.cams0, sc.pts0))
    return prob, lin


def _spd(n, cond, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    ev = np.geomspace(1.0, cond, n)
    return (Q * ev) @ Q.T, rng.normal(size=n)


@pytest.mark.parametrize("lam", [1e-4, 1e-1])
def test_reduced_system_gives_the_exact_step(lam):
    # the Schur complement system solved directly = the camera part of the
    # exact block-Cholesky solve of the full damped system
    prob, lin = _ba_system(lam=lam)
    S, v, fc = pcg.reduced_system(prob, lin, lam, 1e-6, 1e32)
    assert np.allclose(S, S.T, rtol=0, atol=1e-12 * np.abs(S).max())
    assert np.linalg.eigvalsh(S).min() > 0
    dc, _ = prob.solve(lin, lam, 1e-6, 1e32)
    np.testing.assert_allclose(np.linalg.solve(S, v), dc[fc].ravel(), rtol=1e-8,
                               atol=1e-10 * np.abs(dc).max())


def test_block_jacobi_is_the_inverse_of_the_diagonal_blocks():
    S, _ = _spd(27, 1e3, 3)
    M = pcg.block_jacobi(S)
    for a in range(0, 27, 9):
        np.testing.assert_allclose(M[a:a + 9, a:a + 9] @ S[a:a + 9, a:a + 9], np.eye(9),
                                   atol=1e-10)
    assert np.all(M[:9, 9:] == 0)


def test_pcg_converges_to_the_direct_solve():
    prob, lin = _ba_system()
    S, v, _ = pcg.reduced_system(prob, lin, 1e-2, 1e-6, 1e32)
    x, steps, why = pcg.pcg(S, v, pcg.block_jacobi(S), tol=1e-13, max_iters=500)
    assert why == pcg.DONE_CONVERGED and 0 < steps < 500
    want = np.linalg.solve(S, v)
    np.testing.assert_allclose(x, want, rtol=0, atol=1e-9 * np.abs(want).max())


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_pcg_iterates_minimise_the_energy_error_over_the_krylov_space(k):
    # x_k minimises |x - x*|_S over K_k(M S, M v): build that space
    # explicitly and solve the k x k projected system
    S, v = _spd(30, 50.0, 7)
    M = pcg.block_jacobi(S, block=3)
    x, steps, why = pcg.pcg(S, v, M, tol=0.0, max_iters=k)
    assert steps == k and why == pcg.DONE_MAX_ITERS
    cols = [M @ v]
    for _ in range(k - 1):
        cols.append(M @ (S @ cols[-1]))
    Q, _ = np.linalg.qr(np.stack(cols, axis=1))
    want = Q @ np.linalg.solve(Q.T @ S @ Q, Q.T @ v)
    np.testing.assert_allclose(x, want, rtol=0, atol=1e-9 * np.abs(want).max())


def test_pcg_ends_after_as_many_steps_as_distinct_eigenvalues():
    rng = np.random.default_rng(5)
    d = np.repeat([1.0, 3.0, 7.0], [10, 10, 7])
    S = np.diag(d)
    v = rng.normal(size=len(d))
    x, steps, why = pcg.pcg(S, v, np.eye(len(d)), tol=1e-12, max_iters=50)
    assert why == pcg.DONE_CONVERGED and steps == 3
    np.testing.assert_allclose(x, v / d, atol=1e-10)


def _enumerate(S, v, M, kmax):
    """Iterates x_0..x_kmax of the plain iteration and their residuals."""
    xs = [np.zeros_like(v)]
    for k in range(1, kmax + 1):
        x, _, _ = pcg.pcg(S, v, M, tol=0.0, max_iters=k)
        xs.append(x)
    rr = [float((v - S @ x) @ (v - S @ x)) for x in xs]
    return xs, rr


def test_rejection_ratio_returns_the_best_iterate():
    # a BA reduced system whose residual norm rises at step 6 (by a factor
    # 2.3 over the best so far); with ratio 1.5 the iteration stops there
    # and returns the iterate of smallest residual
    prob, lin = _ba_system(seed=34, lam=1e-2)
    S, v, _ = pcg.reduced_system(prob, lin, 1e-2, 1e-6, 1e32)
    M = pcg.block_jacobi(S)
    xs, rr = _enumerate(S, v, M, 8)
    k = next(k for k in range(1, 9) if rr[k] > 1.5 ** 2 * min(rr[:k]))
    assert k == 6
    best = int(np.argmin(rr[:k]))
    x, steps, why = pcg.pcg(S, v, M, tol=1e-30, max_iters=50, ratio=1.5)
    assert why == pcg.DONE_REJECTED and steps == k
    np.testing.assert_allclose(x, xs[best], rtol=0, atol=1e-10 * np.abs(xs[best]).max())


def test_rejection_before_any_improvement_returns_the_start():
    # the first step raises the residual norm (a preconditioner that fits S
    # badly): the best iterate is x_0 = 0
    S = np.diag([1.0, 100.0])
    v = np.array([1.0, 0.1])
    M = np.diag([1.0, 1.0])          # identity: the first step follows v
    # step 1: alpha = v.v / v.Sv = 0.505, r_1 = (0.495, -4.95), |r_1|^2 = 24.747525
    xs, rr = _enumerate(S, v, M, 1)
    assert abs(rr[1] - 24.747525) < 1e-12 and abs(rr[0] - 1.01) < 1e-15
    x, steps, why = pcg.pcg(S, v, M, tol=1e-30, max_iters=10, ratio=1.0)
    assert why == pcg.DONE_REJECTED and steps == 1
    assert np.all(x == 0.0)


def test_schur_pcg_step_converged_equals_the_block_cholesky_step():
    # run to convergence, the Schur + PCG step (reduced solve, back-substitution)
    # is the exact damped step of the full system
    sc = synth.make_scene("small", seed=44, n_cams=5, n_pts=120)
    prob = ba.BAProblem(sc.n_cams, sc.n_pts, sc.cam_idx, sc.pt_idx, sc.obs)
    lin = prob.linearize((sc.cams0, sc.pts0))
    (dc, dp), steps = pcg.schur_pcg_step(prob, lin, 1e-3, 1e-6, 1e32, tol=1e-15, max_iters=200)
    dco, dpo = prob.solve(lin, 1e-3, 1e-6, 1e32)
    np.testing.assert_allclose(dc, dco, rtol=0, atol=1e-9 * np.abs(dco).max())
    np.testing.assert_allclose(dp, dpo, rtol=0, atol=1e-9 * np.abs(dpo).max())
    assert 0 < steps <= 200


def test_schur_pcg_one_step_is_the_steepest_descent_step_in_the_m_norm():
    # one PCG step from x = 0: x1 = alpha z0, z0 = M^-1 v, alpha = v^T z0 / z0^T S z0
    sc = synth.make_scene("small", seed=45, n_cams=4, n_pts=80)
    prob = ba.BAProblem(sc.n_cams, sc.n_pts, sc.cam_idx, sc.pt_idx, sc.obs)
    lin = prob.linearize((sc.cams0, sc.pts0))
    S, v, fc = pcg.reduced_system(prob, lin, 1e-2, 1e-6, 1e32)
    M = pcg.block_jacobi(S)
    z0 = M @ v
    x1 = (v @ z0) / (z0 @ S @ z0) * z0
    (dc, _), steps = pcg.schur_pcg_step(prob, lin, 1e-2, 1e-6, 1e32, tol=0.0, max_iters=1)
    assert steps == 1
    np.testing.assert_allclose(dc[fc].ravel(), x1, rtol=1e-12, atol=1e-16)
