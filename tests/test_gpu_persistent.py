"""The persistent PCG schedule on the GPU: every PCG iteration of a damped
step (product, partial reduction, update; the camera-major pass in the
fixed-order mode) run by one cooperative kernel whose phases are separated by
grid barriers, each problem of a batch stopping on its own device-side
decision.  It runs the same per-block arithmetic as the launched chunks, so
with fixed-order sums the two schedules agree bit for bit; with the default
LDS sums they agree to rounding and both match the oracle.
"""
import json
import os

import numpy as np
import pytest

from oracle import align, ba
from paper_2509_26581_amd import gba, synth

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gba.load()


def _graph(sc, precision=gba.GBA_FP64, **opt):
    return gba.Graph.from_arrays(sc.cams0, sc.pts0, sc.cam_idx, sc.pt_idx, sc.obs,
                                 loss=sc.loss, delta=sc.delta, precision=precision,
                                 options=gba.options(**opt))


def _trial_tuple(t):
    return (t["cost"], t["candidate_cost"], t["lam"], t["model_decrease"], t["step_norm"],
            t["accepted"], t["pcg_iters"])


@pytest.mark.parametrize("precision", [gba.GBA_FP64, gba.GBA_MIXED_FP32, gba.GBA_MIXED_BF16])
def test_persistent_equals_chunked_launches_bitwise(precision):
    # fixed-order sums: the persistent kernel runs the launched form's
    # per-block arithmetic in the same order (the camera-major pass included),
    # so trajectories and solutions agree bit for bit; a PCG tolerance of
    # 1e-10 makes the stopping iteration depend on the last bit
    sc = synth.make_scene("small", seed=5, n_cams=12, n_pts=800)
    kw = dict(precision=precision, pcg_max_iters=60, pcg_tol=1e-10, deterministic=1)
    a = _graph(sc, pcg_schedule=gba.GBA_PCG_CHUNKED, **kw)
    b = _graph(sc, pcg_schedule=gba.GBA_PCG_PERSISTENT, **kw)
    ra, rb = a.solve(8), b.solve(8)
    assert [_trial_tuple(t) for t in a.trials()] == [_trial_tuple(t) for t in b.trials()]
    assert ra.final_cost == rb.final_cost
    np.testing.assert_array_equal(a.cameras(), b.cameras())
    np.testing.assert_array_equal(a.points(), b.points())
    # repeated on one handle after a reset
    gba.gba_reset(b.h)
    rc = b.solve(8)
    assert rc.final_cost == ra.final_cost


@pytest.mark.parametrize("acc", [gba.GBA_ACC_AUTO, gba.GBA_ACC_CAMERA_BLOCKS])
def test_persistent_lm_trajectory_matches_the_oracle(acc):
    # default (LDS) sums, exact PCG: per-trial costs, damping and decisions
    # as the oracle's exact block-Cholesky LM; also on a graph built for the
    # camera-blocked pass, which the persistent kernel runs as the
    # camera-major pass
    sc = synth.make_scene("small", seed=0)
    g = _graph(sc, pcg_max_iters=sc.pcg_max_iters, pcg_tol=1e-14,
               pcg_schedule=gba.GBA_PCG_PERSISTENT, accumulation=acc)
    rep = g.solve(sc.trials)
    prob = ba.BAProblem(sc.n_cams, sc.n_pts, sc.cam_idx, sc.pt_idx, sc.obs,
                        loss=sc.loss, delta=sc.delta)
    res = ba.solve(prob, sc.cams0, sc.pts0, sc.trials)
    gt = g.trials()
    assert len(gt) == len(res.log)
    for a, b in zip(gt, res.log):
        assert abs(a["cost"] - b["cost"]) <= 1e-10 * b["cost"], (a, b)
        if abs(b["cost"] - b["candidate_cost"]) > 1e-9 * b["cost"]:
            assert a["accepted"] == b["accepted"], (a, b)
    assert abs(rep.final_cost - res.cost) <= 1e-10 * res.cost
    err = align.aligned_errors(g.cameras(), g.points(), res.x[0], res.x[1])
    assert err["rel"] <= 1e-6, err


def test_persistent_truncated_pcg_and_iteration_limit():
    # the iteration limit and the rejection-ratio stop act inside the
    # persistent loop as in the launched chunks (fixed-order sums: bitwise)
    sc = synth.make_scene("small", seed=34, n_cams=6, n_pts=200)
    for k, ratio in ((1, 0.0), (3, 0.0), (7, 0.0), (50, 1.5)):
        kw = dict(pcg_max_iters=k, pcg_tol=1e-30, deterministic=1, pcg_rejection_ratio=ratio)
        a = _graph(sc, pcg_schedule=gba.GBA_PCG_CHUNKED, **kw)
        b = _graph(sc, pcg_schedule=gba.GBA_PCG_PERSISTENT, **kw)
        da, pa, ia = gba.gba_eval_step(a.h, 1e-2, sc.n_cams, sc.n_pts)
        db, pb, ib = gba.gba_eval_step(b.h, 1e-2, sc.n_cams, sc.n_pts)
        assert ia == ib
        np.testing.assert_array_equal(da, db)
        np.testing.assert_array_equal(pa, pb)


def test_persistent_on_the_1m_observation_workload():
    # forced on a problem with 1,000 cameras (72 KB of LDS camera sums per
    # workgroup): the mixed-FP32 final cost against the oracle's stored solve
    gold = json.load(open(os.path.join(GOLD, "bal1m_seed0.json")))
    sc = synth.make_scene("bal1m", seed=0)
    g = _graph(sc, precision=gba.GBA_MIXED_FP32, pcg_max_iters=sc.pcg_max_iters,
               pcg_tol=sc.pcg_tol, pcg_schedule=gba.GBA_PCG_PERSISTENT)
    rep = g.solve(gold["trials"])
    rel = abs(rep.final_cost - gold["final_cost"]) / gold["final_cost"]
    assert rel <= 1e-4, rel
    print(f"bal1m persistent: final cost rel {rel:.3e}, {rep.pcg_iters_total} PCG iterations")


@pytest.mark.parametrize("precision", [gba.GBA_FP64, gba.GBA_MIXED_FP32])
def test_served_requests_persistent_equal_chunked_bitwise(precision):
    # a mix of requests on the server under both schedules, fixed-order sums:
    # every result bit for bit the same
    reqs = [synth.make_local_request(s, np_range=(300, 2500), k_range=(5, 24)) for s in range(6)]
    out = {}
    for sched in (gba.GBA_PCG_CHUNKED, gba.GBA_PCG_PERSISTENT):
        srv = gba.Server(precision=precision, budget_bytes=256 << 20, max_slots=64, pcg_tol=1e-8,
                         deterministic=1, pcg_schedule=sched)
        try:
            tickets = [srv.submit(r) for r in reqs]
            out[sched] = [srv.poll(t) for t in tickets]
        finally:
            srv.close()
    for a, b in zip(out[gba.GBA_PCG_CHUNKED], out[gba.GBA_PCG_PERSISTENT]):
        assert a["report"]["final_cost"] == b["report"]["final_cost"]
        np.testing.assert_array_equal(a["cams"], b["cams"])
        np.testing.assert_array_equal(a["pts"], b["pts"])


def test_schedule_option_is_validated():
    sc = synth.make_scene("small", seed=1, n_cams=4, n_pts=50)
    g = _graph(sc)
    with pytest.raises(gba.GbaError) as e:
        gba.gba_set_options(g.h, gba.options(pcg_schedule=3))
    assert e.value.status == -1
