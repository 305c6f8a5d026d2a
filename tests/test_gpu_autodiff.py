"""Forward-mode automatic differentiation of the edge residual on the GPU
(GBA_JACOBIAN_AUTODIFF): the residual written once over a generic scalar
type and evaluated on dual numbers, one seeded input per evaluation giving
one Jacobian column.  The edge evaluation entry point runs one lane per
(edge, column); the solver's linearisation evaluates an edge's columns in
its lane.  Checked against the oracle's dual-number Jacobians, against the
closed-form kernels, and through whole solves.
"""
import numpy as np
import pytest

from oracle import ba, camera, robust
from paper_2509_26581_amd import gba, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gba.load()


def _graph(sc, cams=None, precision=gba.GBA_FP64, info=None, loss=None, cam_fixed=None,
           pt_fixed=None, **opt):
    return gba.Graph.from_arrays(
        sc.cams0 if cams is None else cams, sc.pts0, sc.cam_idx, sc.pt_idx, sc.obs, info=info,
        loss=sc.loss if loss is None else loss, delta=sc.delta, precision=precision,
        options=gba.options(**opt), cam_fixed=cam_fixed, pt_fixed=pt_fixed)


def _info(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.5, 2.0, size=(n, 2))
    c = rng.uniform(-0.3, 0.3, size=n)
    return np.stack([a[:, 0], c, a[:, 1]], axis=1)


@pytest.mark.parametrize("loss", [robust.SQUARED, robust.HUBER])
def test_autodiff_edge_jacobians(loss):
    sc = synth.make_scene("small", seed=21, n_cams=8, n_pts=400, noise_px=2.0)
    cams = sc.cams0.copy()
    cams[0, 0:3] = 0.0                    # first-order rotation branch
    cams[1, 0:3] = [1e-10, -2e-10, 0.0]   # first-order rotation branch
    cams[2, 0:3] = [1e-5, 2e-5, -1e-5]    # series branch of the rotation
    cams[4, 0:3] = [2.0, -1.0, 0.5]       # a large rotation
    info = _info(sc.n_obs, 3)
    cf = np.zeros(8, bool)
    cf[3] = True
    pf = np.zeros(400, bool)
    pf[::7] = True
    kw = dict(cams=cams, info=info, loss=loss, cam_fixed=cf, pt_fixed=pf)
    ga = _graph(sc, jacobian=gba.GBA_JACOBIAN_AUTODIFF, **kw)
    gc = _graph(sc, **kw)
    r, jc, jp, w = gba.gba_eval_edges(ga.h, sc.n_obs)
    rc, jcc, jpc, wc = gba.gba_eval_edges(gc.h, sc.n_obs)
    # against the closed form (both FP64, different formulas): rounding level
    np.testing.assert_allclose(r, rc, rtol=0, atol=1e-9)
    sj = np.maximum(np.maximum(np.abs(jcc).max(axis=(1, 2)), np.abs(jpc).max(axis=(1, 2))), 1.0)
    assert (np.abs(jc - jcc).max(axis=(1, 2)) <= 1e-12 * sj).all()
    assert (np.abs(jp - jpc).max(axis=(1, 2)) <= 1e-12 * sj).all()
    np.testing.assert_allclose(w, wc, rtol=1e-12)
    # against the oracle's dual numbers (which differentiate through w / |w|:
    # its own rounding error grows like eps / |w| for small rotations)
    ro, jco, jpo = camera.residuals_and_jacobians(cams, sc.pts0, sc.cam_idx, sc.pt_idx, sc.obs)
    jco[cf[sc.cam_idx]] = 0.0
    jpo[pf[sc.pt_idx]] = 0.0
    theta = np.linalg.norm(cams[:, 0:3], axis=1)
    small = (theta > 1e-8) & (theta < 1e-3)
    tol = np.where(small, 1e-12 + 1e-16 / np.maximum(theta, 1e-300), 1e-12)[sc.cam_idx]
    so = np.maximum(np.maximum(np.abs(jco).max(axis=(1, 2)), np.abs(jpo).max(axis=(1, 2))), 1.0)
    assert (np.abs(jc - jco).max(axis=(1, 2)) <= tol * so).all()
    assert (np.abs(jp - jpo).max(axis=(1, 2)) <= tol * so).all()
    np.testing.assert_allclose(r, ro, rtol=0, atol=1e-9)


@pytest.mark.parametrize("precision,tol", [(gba.GBA_FP64, 1e-10), (gba.GBA_MIXED_FP32, 1e-6)])
def test_autodiff_solve_matches_analytic_and_oracle(precision, tol):
    # the solver with AD Jacobians takes the analytic solver's trajectory to
    # rounding and reaches the oracle's final cost
    sc = synth.make_scene("small", seed=0)
    kw = dict(precision=precision, pcg_max_iters=sc.pcg_max_iters, pcg_tol=1e-12)
    ga = _graph(sc, jacobian=gba.GBA_JACOBIAN_AUTODIFF, **kw)
    gc = _graph(sc, **kw)
    ra, rc = ga.solve(sc.trials), gc.solve(sc.trials)
    assert abs(ra.final_cost - rc.final_cost) <= tol * rc.final_cost
    for a, c in zip(ga.trials(), gc.trials()):
        # decisions agree while the decrease is above rounding; once
        # F - F' is within ~1e-9 F both take them from rounding noise
        if abs(c["cost"] - c["candidate_cost"]) > 1e-9 * c["cost"]:
            assert a["accepted"] == c["accepted"], (a, c)
    res = ba.solve(ba.BAProblem(sc.n_cams, sc.n_pts, sc.cam_idx, sc.pt_idx, sc.obs,
                                loss=sc.loss, delta=sc.delta), sc.cams0, sc.pts0, sc.trials)
    assert abs(ra.final_cost - res.cost) <= max(tol, 1e-10) * res.cost


def test_autodiff_normal_equations_equal_closed_form():
    sc = synth.make_scene("small", seed=31, n_cams=9, n_pts=500, noise_px=2.0)
    ga = _graph(sc, loss=robust.HUBER, jacobian=gba.GBA_JACOBIAN_AUTODIFF)
    gc = _graph(sc, loss=robust.HUBER)
    a = gba.gba_eval_normal_equations(ga.h, 9, 500)
    c = gba.gba_eval_normal_equations(gc.h, 9, 500)
    for x, y in zip(a, c):
        assert np.abs(x - y).max() <= 1e-12 * np.abs(y).max()
