"""Pins of the oracle's full-Hessian system (oracle/full.py): its Hessian and
gradient against a Hessian formed from finite-difference Jacobians, its
direct solve against the exact block-Cholesky step, its camera part against
the reduced camera system, the block-Jacobi preconditioner, and PCG on it
converging to the exact step.
"""
import numpy as np
import pytest

import test_oracle_pins as P
from oracle import ba, full, pcg, robust
from paper_2509_26581_amd import synth


def test_full_hessian_matches_finite_differences():
    # lambda = 0: H and -b equal J^T W J and -J^T W r with J by central
    # differences of the stacked residual (fixed vertices, inactive edges and
    # information matrices included)
    sc, prob = P._tiny(seed=7, loss=robust.HUBER)
    x = (sc.cams0, sc.pts0)
    lin = prob.linearize(x)
    H, v, fc, fp = full.full_system(prob, lin, 0.0, 1e-6, 1e32)
    Hd, bd, _, _ = P._dense_system(sc, prob, x, jac="fd")
    np.testing.assert_allclose(H, Hd, rtol=0, atol=1e-6 * np.abs(Hd).max())
    np.testing.assert_allclose(v, -bd, rtol=0, atol=1e-6 * np.abs(bd).max())
    assert H.shape == (9 * len(fc) + 3 * len(fp),) * 2


@pytest.mark.parametrize("lam", [1e-4, 1e-1])
def test_full_system_solve_is_the_exact_step(lam):
    sc, prob = P._tiny(seed=5)
    lin = prob.linearize((sc.cams0, sc.pts0))
    H, v, fc, fp = full.full_system(prob, lin, lam, 1e-6, 1e32)
    dc, dp = full.split(np.linalg.solve(H, v), prob, fc, fp)
    dco, dpo = prob.solve(lin, lam, 1e-6, 1e32)
    np.testing.assert_allclose(dc, dco, rtol=0, atol=1e-9 * np.abs(dco).max())
    np.testing.assert_allclose(dp, dpo, rtol=0, atol=1e-9 * np.abs(dpo).max())


def test_camera_part_equals_the_reduced_system_solve():
    sc = synth.make_scene("small", seed=34, n_cams=6, n_pts=200)
    prob = ba.BAProblem(sc.n_cams, sc.n_pts, sc.cam_idx, sc.pt_idx, sc.obs,
                        loss=robust.HUBER, delta=sc.delta)
    lin = prob.linearize((sc.cams0, sc.pts0))
    H, v, fc, fp = full.full_system(prob, lin, 1e-2, 1e-6, 1e32)
    S, vs, _ = pcg.reduced_system(prob, lin, 1e-2, 1e-6, 1e32)
    x = np.linalg.solve(H, v)
    np.testing.assert_allclose(x[:9 * len(fc)], np.linalg.solve(S, vs), rtol=0,
                               atol=1e-8 * np.abs(x).max())


def test_block_jacobi_full_inverts_the_diagonal_blocks():
    sc, prob = P._tiny(seed=5, fixed=False)
    lin = prob.linearize((sc.cams0, sc.pts0))
    H, _, fc, fp = full.full_system(prob, lin, 1e-3, 1e-6, 1e32)
    M = full.block_jacobi_full(H, len(fc))
    o = 9 * len(fc)
    for a in range(0, o, 9):
        np.testing.assert_allclose(M[a:a + 9, a:a + 9] @ H[a:a + 9, a:a + 9], np.eye(9), atol=1e-9)
    for a in range(o, H.shape[0], 3):
        np.testing.assert_allclose(M[a:a + 3, a:a + 3] @ H[a:a + 3, a:a + 3], np.eye(3), atol=1e-9)
    off = M.copy()
    for a in range(0, o, 9):
        off[a:a + 9, a:a + 9] = 0
    for a in range(o, H.shape[0], 3):
        off[a:a + 3, a:a + 3] = 0
    assert not off.any()


def test_full_pcg_converges_to_the_exact_step():
    sc = synth.make_scene("small", seed=34, n_cams=6, n_pts=200)
    prob = ba.BAProblem(sc.n_cams, sc.n_pts, sc.cam_idx, sc.pt_idx, sc.obs,
                        loss=robust.HUBER, delta=sc.delta)
    lin = prob.linearize((sc.cams0, sc.pts0))
    H, v, fc, fp = full.full_system(prob, lin, 1e-2, 1e-6, 1e32)
    x, steps, why = pcg.pcg(H, v, full.block_jacobi_full(H, len(fc)), tol=1e-13, max_iters=5000)
    assert why == pcg.DONE_CONVERGED
    dc, dp = full.split(x, prob, fc, fp)
    dco, dpo = prob.solve(lin, 1e-2, 1e-6, 1e32)
    np.testing.assert_allclose(dc, dco, rtol=0, atol=1e-7 * np.abs(dco).max())
    np.testing.assert_allclose(dp, dpo, rtol=0, atol=1e-7 * np.abs(dpo).max())
