"""Serving form on the GPU: local bundle-adjustment requests solved
concurrently by one server (batched LM trials over problem-aligned work
decompositions).  Checks that a served request gives the single-graph
solver's result and the oracle's within the precision policy's tolerances,
that each result is the same alone and in a mix (requests joining while
others run, admission under a small memory budget, a slot limit), and the
error paths.

By default camera partial sums inside a workgroup are combined with LDS
atomics, so results repeat to rounding only: those alone-versus-mix
comparisons use the mixed policy's tolerances (1e-4 cost, 1e-3 parameters).
With fixed-order sums (options.deterministic) a problem's arithmetic does not
depend on its batch mates or on timing, and the comparisons are bitwise.
"""
import time

import numpy as np
import pytest

from oracle import align, ba
from paper_2509_26581_amd import gba, synth

pytestmark = pytest.mark.gpu

SMALL = dict(np_range=(300, 2500), k_range=(5, 24))


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    gba.load()


def _req(seed, **kw):
    over = dict(SMALL)
    over.update(kw)
    return synth.make_local_request(seed, **over)


def _server(precision=gba.GBA_MIXED_FP32, budget=256 << 20, slots=64, **kw):
    kw.setdefault("pcg_tol", 1e-8)
    return gba.Server(precision=precision, budget_bytes=budget, max_slots=slots, **kw)


def _alone(r, precision, **kw):
    s = _server(precision, **kw)
    try:
        t = s.submit(r)
        return s.poll(t)
    finally:
        s.close()


def _rel(a, b):
    a, b = np.asarray(a, float), np.asarray(b, float)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _bitwise(x, y, what):
    assert x["report"]["final_cost"] == y["report"]["final_cost"], what
    assert x["report"]["trials"] == y["report"]["trials"], what
    assert x["report"]["accepted"] == y["report"]["accepted"], what
    assert x["report"]["pcg_iters_total"] == y["report"]["pcg_iters_total"], what
    assert x["report"]["termination_name"] == y["report"]["termination_name"], what
    np.testing.assert_array_equal(x["cams"], y["cams"], err_msg=what)
    np.testing.assert_array_equal(x["pts"], y["pts"], err_msg=what)


def _same(x, y, cost_tol, par_tol, what):
    rc = abs(x["report"]["final_cost"] - y["report"]["final_cost"]) / y["report"]["final_cost"]
    rp = max(_rel(x["cams"], y["cams"]), _rel(x["pts"], y["pts"]))
    assert rc <= cost_tol and rp <= par_tol, f"{what}: cost rel {rc:.3e}, params rel {rp:.3e}"


@pytest.mark.parametrize("precision", [gba.GBA_FP64, gba.GBA_MIXED_FP32])
@pytest.mark.parametrize("det", [0, 1])
def test_served_request_equals_graph_solve(precision, det):
    r = _req(11)
    # the single-graph path with the same options and decomposition sizes
    g = gba.Graph.from_arrays(r["cams"], r["pts"], r["cam_idx"], r["pt_idx"], r["uv"],
                              loss=gba.GBA_LOSS_HUBER, delta=1.0, precision=precision,
                              options=gba.options(pcg_tol=1e-8, deterministic=det),
                              cam_fixed=r["cam_fixed"])
    rep = g.solve(r["max_iters"])
    ref = {"cams": g.cameras(), "pts": g.points(), "report": rep.as_dict()}
    g.close()
    got = _alone(r, precision, tiles_per_block=16, edges_per_block=256, pts_per_block=256,
                 deterministic=det)
    if det:
        _bitwise(got, ref, "server vs graph (fixed-order sums)")
    else:
        assert got["report"]["trials"] == rep.trials
        _same(got, ref, 1e-4, 1e-3, "server vs graph")
        assert got["report"]["initial_cost"] == pytest.approx(rep.initial_cost, rel=1e-12)


def test_served_request_matches_oracle():
    r = _req(5, np_range=(400, 900), k_range=(6, 10))
    got = _alone(r, gba.GBA_MIXED_FP32)
    prob = ba.BAProblem(len(r["cams"]), len(r["pts"]), r["cam_idx"], r["pt_idx"], r["uv"],
                        cam_fixed=r["cam_fixed"], loss=1, delta=1.0)
    res = ba.solve(prob, r["cams"], r["pts"], r["max_iters"])
    rc = abs(got["report"]["final_cost"] - res.cost) / res.cost
    assert rc <= 1e-4, (got["report"]["final_cost"], res.cost)
    # two fixed keyframes fix the gauge: compare parameters directly
    rp = max(_rel(got["cams"], res.x[0]), _rel(got["pts"], res.x[1]))
    assert rp <= 1e-3, rp
    err = align.aligned_errors(got["cams"], got["pts"], res.x[0], res.x[1])
    assert err["rel"] <= 1e-3, err


@pytest.mark.parametrize("precision,det", [(gba.GBA_FP64, 1), (gba.GBA_MIXED_FP32, 1),
                                           (gba.GBA_MIXED_BF16, 1), (gba.GBA_MIXED_FP32, 0)])
def test_alone_and_in_a_mix_with_joins(precision, det):
    # each result is the same alone and in a mix that it joins while others
    # run: bitwise with fixed-order sums, within the mixed policy's
    # tolerances otherwise
    reqs = [_req(100 + k) for k in range(8)]
    alone = [_alone(r, precision, deterministic=det) for r in reqs]
    s = _server(precision, deterministic=det)
    try:
        first = [s.submit(r) for r in reqs[:4]]
        got = {first[0]: s.poll(first[0])}          # others still running
        late = [s.submit(r) for r in reqs[4:]]      # join a running batch
        tickets = first + late
        for t in tickets[1:]:
            got[t] = s.poll(t)
        st = s.stats()
    finally:
        s.close()
    for k, t in enumerate(tickets):
        if det:
            _bitwise(got[t], alone[k], f"request {k}")
        else:
            _same(got[t], alone[k], 1e-4, 1e-3, f"request {k}")
    assert st["completed"] == 8 and st["collected"] == 8 and st["rejected"] == 0
    assert st["mean_batch"] > 1.0 and st["repacks"] >= 2
    assert max(got[t]["batch_peak"] for t in tickets) >= 2


def test_admission_under_a_small_budget_and_slot_limit():
    reqs = [_req(200 + k) for k in range(10)]
    alone = [_alone(r, gba.GBA_FP64, deterministic=1) for r in reqs]
    budget = 48 << 20
    s = _server(gba.GBA_FP64, budget=budget, slots=3, deterministic=1)
    try:
        tickets = [s.submit(r) for r in reqs]
        got = [s.poll(t) for t in tickets]
        st = s.stats()
    finally:
        s.close()
    for k in range(10):
        _bitwise(got[k], alone[k], f"request {k}")
        assert got[k]["batch_peak"] <= 3
    assert st["bytes_peak"] <= budget
    assert st["completed"] == 10 and st["in_flight"] == 0 and st["queued"] == 0
    assert max(g["queue_ms"] for g in got) > 0.0


def test_rejections_and_errors():
    s = _server(budget=2 << 20)
    try:
        big = _req(7, np_range=(20000, 20000), k_range=(30, 30))
        with pytest.raises(gba.GbaError) as ei:
            s.submit(big)
        assert ei.value.status == -9                               # over budget
        r = _req(8)
        bad = dict(r, cam_idx=r["cam_idx"].copy())
        bad["cam_idx"][3] = len(r["cams"])
        with pytest.raises(gba.GbaError) as ei:
            s.submit(bad)
        assert ei.value.status == -2                               # unknown vertex
        nan = dict(r, uv=r["uv"].copy())
        nan["uv"][0, 0] = np.nan
        with pytest.raises(gba.GbaError) as ei:
            s.submit(nan)
        assert ei.value.status == -4
        with pytest.raises(gba.GbaError) as ei:
            gba.gba_server_poll(s.h, 12345, 1, 1)
        assert ei.value.status == -2                               # unknown ticket
        assert s.stats()["rejected"] == 3
    finally:
        s.close()


def test_requests_without_work_return_their_start():
    r = _req(9)
    fixed = dict(r, cam_fixed=np.ones(len(r["cams"]), bool),
                 pt_fixed=np.ones(len(r["pts"]), bool))
    empty = dict(r, cam_idx=r["cam_idx"][:0], pt_idx=r["pt_idx"][:0], uv=r["uv"][:0])
    s = _server()
    try:
        t1, t2, t3 = s.submit(fixed), s.submit(empty), s.submit(r)
        a, b, c = s.poll(t1), s.poll(t2), s.poll(t3)
    finally:
        s.close()
    for x in (a, b):
        assert x["report"]["termination_name"] == "NO_WORK" and x["report"]["trials"] == 0
        assert np.array_equal(x["cams"], r["cams"]) and np.array_equal(x["pts"], r["pts"])
    assert c["report"]["trials"] == r["max_iters"]
    assert c["report"]["final_cost"] < c["report"]["initial_cost"]


def test_poll_without_waiting():
    s = _server()
    try:
        t = s.submit(_req(10))
        deadline = time.time() + 60
        res = s.poll(t, wait=False)
        while res is None and time.time() < deadline:
            time.sleep(0.002)
            res = s.poll(t, wait=False)
        assert res is not None and res["report"]["trials"] > 0
    finally:
        s.close()
