"""Benchmark: LM iterations/s of bundle adjustment at 1M observations on one
MI355X, the PCG matvec roofline, the CPU oracle as a baseline, and p50/p99
latency of a local-BA request stream on the server.

Workload (synthetic, seeded): 1,000 cameras, 200,000 points, ~1.0M
observations (track length 2 + Geometric(1/4)), Huber delta = 1 px, 20 LM
trials per solve, PCG tolerance 1e-6 relative, at most 100 iterations.
One step = one 20-trial solve from the perturbed start (device-side reset of
the parameters, then gba_solve).  Inputs are resident on the device before the
timed region.

Visual-inertial (in the same JSON line, "vi"; alone with --vi): 2,000
keyframes with a 200 Hz IMU, 300k points, ~2.07M stereo observations, Huber,
LM with PCG on the keyframe Schur complement (W in FP32, FP64 arithmetic);
LM iter/s over the trials, the call's set-up reported apart.

At scale (in the same JSON line, "bal8m"): 10,000 cameras, 1M points, ~8M
observations, BF16 Jacobian copy, 15 LM trials per solve, run by this script
in a child process (--no-bal8m skips it).

Serving (in the same JSON line, "serving"): 512 local-BA requests (5-40
keyframes, 500-20k points, tracks 2-10 inside a local window, first two
keyframes fixed, 10 trials each, mixed FP32): one at a time, all at once
(saturated solves/s), and as a Poisson stream at 0.8x the saturated rate
(p50/p99 latency from submission to result).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp64|fp32|bf16]
                  [--workload bal1m|bal8m|small] [--no-cpu-baseline] [--no-serve] [--no-vi]
                  [--no-bal8m]
                  [--serve-only] [--accumulation 0|1|2] [--tiles-per-block N]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "LM iter/s + PCG HBM GB/s at 1M obs; p50/p99 latency for local-BA stream"
HBM_PEAK_GBS = 8000.0
PRECISIONS = {"fp64": (0, "f64", 8), "fp32": (1, "f32", 4), "bf16": (2, "f32+bf16", 2)}
# HBM bytes per matvec launch measured with rocprofv3 counters on the 1M-observation
# workload (FETCH_SIZE x 2 + WRITE_SIZE; the factor 2 from the streaming read of a
# 256 MiB buffer by gba_hbm_probe, whose FETCH_SIZE counts half of it); see
# profiles/.  None until measured for the current kernel.
MEASURED_TRAFFIC = {"fp32": 120250972, "fp64": 235340246, "bf16": 72177546}
MATVEC_WARMUP, MATVEC_LAUNCHES = 20, 200
SCHEDULES = {"auto": 0, "chunked": 1, "persistent": 2}
SOLVERS = {"schur": 0, "full": 1}
JACOBIANS = {"analytic": 0, "autodiff": 1, "dynamic": 2}


def matvec_algorithmic_bytes(n_obs, n_pts_active, jac_bytes, block_bytes):
    """Bytes the fused Schur product must move per launch: the two Jacobian
    blocks (24 entries per edge), the edge's camera index, and per point its
    CSR offset and the 6 unique entries of the inverse point block (stored in
    the block type: FP64, or FP32 in the mixed modes)."""
    return n_obs * (24 * jac_bytes + 4) + n_pts_active * (4 + 6 * block_bytes)


def full_product_algorithmic_bytes(n_obs, n_pts_active, n_cams, jac_bytes, vec_bytes, dynamic):
    """Bytes of one product of the full damped system's point pass
    (k_full_point_pass): per edge its two indices and either the stored
    Jacobian (24 entries) or, recomputed, its observation (FP64 u, v) and
    the parameters of its camera (9 FP64, once per camera) and point
    (3 FP64); per point its v_p, the p and q rows (read and written) and the
    diagonal of its block (3 + 6 + 6 + 3 vector entries); the camera partial
    flushes are left out."""
    per_edge = 8 + (16 if dynamic else 24 * jac_bytes)
    per_pt = 18 * vec_bytes + (24 if dynamic else 0)
    return n_obs * per_edge + n_pts_active * per_pt + (72 * n_cams if dynamic else 0)


def cpu_baseline(sc):
    """The oracle as it stands on a bounded sample: one LM trial (cost,
    linearisation, exact damped solve, candidate cost) of the same workload."""
    from oracle import ba
    threads = os.cpu_count()
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        blas = [i.get("num_threads") for i in info if i.get("user_api") == "blas"]
        if blas:
            threads = max(blas)
    except Exception:
        pass
    prob = ba.BAProblem(sc.n_cams, sc.n_pts, sc.cam_idx, sc.pt_idx, sc.obs,
                        loss=sc.loss, delta=sc.delta)
    t0 = time.perf_counter()
    res = ba.solve(prob, sc.cams0, sc.pts0, 1)
    dt = time.perf_counter() - t0
    return {"value": 1.0 / dt, "unit": "LM iter/s", "cores": int(threads), "kind": "oracle",
            "sample": "1 LM trial (initial cost, dual-number linearisation, exact block-"
                      "Cholesky damped solve, candidate cost) of the same 1M-observation "
                      "workload, seed 0; %.1f s" % dt,
            "trial_cost": res.log[0]["candidate_cost"]}


def serving_measurement(gba, synth, n_req, precision, budget, slots, tune_db, seed=0, schedule=0):
    """Local-BA stream on the server: (1) the same requests one at a time,
    (2) all submitted at once (saturated throughput), (3) a Poisson stream at
    0.8 x the saturated rate; latency = submission to result."""
    import numpy as np
    t0 = time.perf_counter()
    reqs = [synth.make_local_request(10_000 * seed + k) for k in range(n_req)]
    n_obs = [len(r["cam_idx"]) for r in reqs]
    print(f"[bench] serving: {n_req} local-BA requests generated in "
          f"{time.perf_counter() - t0:.1f} s (obs {min(n_obs)}..{max(n_obs)}, "
          f"mean {sum(n_obs) / n_req:.0f})", flush=True)

    def server():
        return gba.Server(precision=precision, budget_bytes=budget, max_slots=slots,
                          tune_db=tune_db, pcg_schedule=schedule)

    # (1) one at a time, on a prefix
    n_single = min(n_req, 64)
    s = server()
    lat = []
    t0 = time.perf_counter()
    for r in reqs[:n_single]:
        lat.append(s.poll(s.submit(r))["latency_ms"])
    single_s = time.perf_counter() - t0
    s.close()
    single = {"requests": n_single, "solves_per_s": round(n_single / single_s, 2),
              "p50_latency_ms": round(float(np.percentile(lat, 50)), 3),
              "p99_latency_ms": round(float(np.percentile(lat, 99)), 3)}
    print(f"[bench] serving one at a time: {single}", flush=True)
    # (2) saturated
    s = server()
    t0 = time.perf_counter()
    tickets = [s.submit(r) for r in reqs]
    for t in tickets:
        s.poll(t)
    sat_s = time.perf_counter() - t0
    sat_stats = s.stats()
    s.close()
    sat = n_req / sat_s
    print(f"[bench] serving saturated: {sat:.1f} solves/s, mean batch "
          f"{sat_stats['mean_batch']:.1f}", flush=True)
    # (3) Poisson stream at 0.8 x saturated
    rate = 0.8 * sat
    arrivals = synth.poisson_arrivals(n_req, rate, seed + 1)
    s = server()
    tickets = []
    t0 = time.perf_counter()
    for r, ta in zip(reqs, arrivals):
        dt = t0 + ta - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        tickets.append(s.submit(r))
    results = [s.poll(t) for t in tickets]
    st = s.stats()
    s.close()
    lat = [x["latency_ms"] for x in results]
    svc = [x["report"]["ms_total"] for x in results]
    out = {"requests": n_req, "precision": {0: "fp64", 1: "fp32", 2: "bf16"}[precision],
           "arrival_rate_per_s": round(rate, 2),
           "p50_latency_ms": round(float(np.percentile(lat, 50)), 3),
           "p99_latency_ms": round(float(np.percentile(lat, 99)), 3),
           "p50_service_ms": round(float(np.percentile(svc, 50)), 3),
           "p99_service_ms": round(float(np.percentile(svc, 99)), 3),
           "solves_per_s": round(st["solves_per_s"], 2),
           "saturated_solves_per_s": round(sat, 2),
           "one_at_a_time": single,
           "admitted": st["admitted"], "rejected": st["rejected"],
           "mean_batch": round(st["mean_batch"], 2), "repacks": st["repacks"],
           "budget_bytes": int(budget), "bytes_peak": int(st["bytes_peak"]), "max_slots": slots,
           "tiles_per_block": st["tiles_per_block"], "edges_per_block": st["edges_per_block"],
           "pts_per_block": st["pts_per_block"], "pcg_sync_every": st["pcg_sync_every"],
           "trials_per_request": reqs[0]["max_iters"]}
    print(f"[bench] serving stream: p50 {out['p50_latency_ms']} ms, p99 "
          f"{out['p99_latency_ms']} ms at {rate:.1f} req/s", flush=True)
    return out


def vi_measurement(gba, args):
    """The visual-inertial configuration: a smooth trajectory with a 200 Hz
    IMU, 2,000 keyframes 0.25 s apart, 300k points seen within three
    keyframes of their anchor in a rectified stereo pair (about 2M
    observations), Huber on the stereo terms (delta^2 = 7.815, the chi^2_3
    95% point); the IMU preintegrated on the GPU, then LM with PCG on the
    keyframe Schur complement or on the whole system (gba_vi_solve, FP64)."""
    import numpy as np
    from scipy.spatial.transform import Rotation

    from paper_2509_26581_amd import synth_vi
    t0 = time.perf_counter()
    sc = synth_vi.make_vi_scene(seed=0, n_kf=args.vi_kf, n_pts=args.vi_pts, window=3)
    K = sc.n_kf
    rng = np.random.default_rng(1)
    rot = Rotation.from_matrix(sc.R_true)
    dth = rng.normal(0, 0.01, (K, 3))
    dth[0] = 0.0
    R0 = (rot * Rotation.from_rotvec(dth)).as_rotvec()
    dp = rng.normal(0, 0.05, (K, 3))
    dv = rng.normal(0, 0.05, (K, 3))
    dp[0] = dv[0] = 0.0
    states = np.concatenate([R0, sc.p_true + dp, sc.v_true + dv, sc.bg_true, sc.ba_true], axis=1)
    pts0 = sc.pts + rng.normal(0, 0.05, sc.pts.shape)
    print(f"[bench] vi: {K} keyframes, {len(sc.pts)} points, {len(sc.st_kf)} stereo observations "
          f"(generated in {time.perf_counter() - t0:.1f} s)", flush=True)
    m = sc.gyro.shape[1]
    off = np.arange(K, dtype=np.int64) * m
    bias0 = np.concatenate([sc.bg_true[:-1], sc.ba_true[:-1]], axis=1)
    t0 = time.perf_counter()
    pre = gba.gba_vi_preintegrate(0, off, sc.gyro.reshape(-1, 3), sc.acc.reshape(-1, 3),
                                  sc.imu_dt, bias0, 1.7e-4, 2e-3)
    pre_s = time.perf_counter() - t0
    solver = gba.GBA_SOLVER_SCHUR if args.vi_solver == "schur" else gba.GBA_SOLVER_FULL
    prec = gba.GBA_MIXED_FP32 if args.vi_precision == "fp32" else gba.GBA_FP64
    opts = gba.vi_options(pcg_max_iters=100, pcg_tol=1e-6, solver=solver, precision=prec,
                          pcg_rejection_ratio=args.vi_ratio)
    kw = dict(sigma_px=1.0, huber_delta2=7.815, sigma_gw=2e-5, sigma_aw=3e-3, options=opts)
    trials = args.trials or 10
    gba.gba_vi_solve(0, states, pts0, sc.st_kf, sc.st_pt, sc.st_obs, sc.intr, pre, 1, **kw)  # warm-up
    t0 = time.perf_counter()
    _, _, rep, log = gba.gba_vi_solve(0, states, pts0, sc.st_kf, sc.st_pt, sc.st_obs, sc.intr,
                                      pre, trials, **kw)
    el = time.perf_counter() - t0
    return {"vi": {"workload": f"{K} keyframes (0.25 s apart, 200 Hz IMU), {len(sc.pts)} points, "
                               f"{len(sc.st_kf)} stereo observations, Huber delta^2 7.815, "
                               f"{trials} LM trials, PCG tol 1e-6 max 100"
                               + (f" rejection ratio {args.vi_ratio:g}" if args.vi_ratio > 0 else ""),
                   "solver": args.vi_solver,
                   "stream_storage": "f32" if prec == gba.GBA_MIXED_FP32 else "f64",
                   # the set-up of the call (orderings, allocation, uploads) is reported
                   # apart, as the graph build of the BA solve is
                   "lm_iter_per_s": round(rep["trials"] / ((rep["ms_total"] - rep["ms_other"]) * 1e-3), 3),
                   "ms_per_trial": round((rep["ms_total"] - rep["ms_other"]) / rep["trials"], 2),
                   "setup_ms": round(rep["ms_other"], 1), "call_s": round(el, 3),
                   "workspace_bytes": rep["workspace_bytes"],
                   "pcg_iters_per_trial": round(rep["pcg_iters_total"] / max(rep["trials"], 1), 2),
                   "initial_cost": rep["initial_cost"], "final_cost": rep["final_cost"],
                   "accepted": rep["accepted"], "trials": rep["trials"],
                   "preintegration_s": round(pre_s, 4), "dtype": "f64"}}


def bal8m_measurement():
    """The at-scale configuration (10,000 cameras, 1M points, ~8M
    observations, BF16 Jacobian copy, 15 LM trials per solve) run by this
    script in a child process; its LM iter/s, PCG iterations and product
    roofline, or the child's failure."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--workload", "bal8m", "--precision", "bf16",
           "--no-serve", "--no-vi", "--no-bal8m", "--no-cpu-baseline", "--no-compare",
           "--steps", "2", "--warmup", "1"]
    print("[bench] bal8m in a child process ...", flush=True)
    try:
        out = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
        rec = json.loads(out.stdout.strip().splitlines()[-1])
    except Exception as exc:   # reported in the line, not raised
        return {"error": repr(exc)[:200]}
    return {"workload": rec["config"]["workload"], "precision": "bf16",
            "lm_iter_per_s": rec["value"], "ms_per_step": rec["ms_per_step"],
            "pcg_iters_per_trial": rec["pcg_iters_per_trial"], "final_cost": rec["final_cost"],
            "roofline": rec["roofline"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp32", choices=list(PRECISIONS))
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the plain-FP64 comparison run")
    ap.add_argument("--workload", default="bal1m")
    ap.add_argument("--trials", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-timing", action="store_true")
    ap.add_argument("--accumulation", type=int, default=0,
                    help="camera sums of the Schur products: 0 auto, 1 LDS partials, 2 camera-major second pass")
    ap.add_argument("--tiles-per-block", type=int, default=0,
                    help="point tiles per point-pass workgroup (0: automatic)")
    ap.add_argument("--no-serve", action="store_true", help="skip the local-BA stream")
    ap.add_argument("--no-bal8m", action="store_true",
                    help="skip the 10k-camera configuration (reported as \"bal8m\")")
    ap.add_argument("--no-vi", action="store_true",
                    help="skip the visual-inertial configuration (reported as \"vi\")")
    ap.add_argument("--matvec-only", action="store_true",
                    help="only the back-to-back Schur-product timing (for kernel traces)")
    ap.add_argument("--serve-only", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=512)
    ap.add_argument("--serve-budget-mb", type=int, default=4096)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="before the run, one fill (write) and one streaming read "
                         "(gba_hbm_probe) of a buffer of this many MiB: calibrates HBM byte "
                         "counters")
    ap.add_argument("--deterministic", action="store_true",
                    help="fixed-order reductions (gba_options.deterministic)")
    ap.add_argument("--pcg-schedule", default="auto", choices=["auto", "chunked", "persistent"],
                    help="gba_options.pcg_schedule of the solve and the server")
    ap.add_argument("--solver", default="schur", choices=["schur", "full"],
                    help="gba_options.solver: Schur + PCG on the cameras, or PCG on the full system")
    ap.add_argument("--jacobian", default="analytic", choices=["analytic", "autodiff", "dynamic"],
                    help="gba_options.jacobian")
    ap.add_argument("--vi", action="store_true",
                    help="the visual-inertial configuration instead (2,000 keyframes, 300k points, "
                         "~2M stereo observations; gba_vi_solve, FP64)")
    ap.add_argument("--vi-kf", type=int, default=2000)
    ap.add_argument("--vi-pts", type=int, default=300_000)
    ap.add_argument("--vi-precision", default="fp32", choices=["fp32", "fp64"],
                    help="visual-inertial solve: the per-observation array its PCG products "
                         "stream in FP32 (FP64 arithmetic), or everything FP64")
    ap.add_argument("--vi-ratio", type=float, default=0.0,
                    help="visual-inertial PCG rejection ratio (0: none)")
    ap.add_argument("--vi-solver", default="schur", choices=["schur", "full"],
                    help="visual-inertial step: PCG on the keyframe Schur complement, or on the "
                         "whole system")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the solver has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2509_26581_amd import gba, synth

    if not os.path.exists(gba.LIB_PATH):
        from __graft_entry__ import build
        build()
    torch.cuda.set_device(0)
    if args.copy_probe_mb:
        nbytes = args.copy_probe_mb << 20
        buf = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
        buf.fill_(1.0)                                    # writes nbytes
        sink = torch.empty(2048, dtype=torch.float64, device="cuda")
        stream = torch.cuda.current_stream().cuda_stream
        us = gba.gba_hbm_probe(0, buf.data_ptr(), nbytes, sink.data_ptr(), 1, stream)
        torch.cuda.synchronize()
        print(f"[bench] byte-counter probe: fill of {args.copy_probe_mb} MiB, then one "
              f"streaming read of {args.copy_probe_mb} MiB by k_hbm_probe "
              f"({nbytes / us / 1e3:.0f} GB/s, {us:.1f} us)", flush=True)
        del buf, sink
    if args.vi:
        print(json.dumps(vi_measurement(gba, args)), flush=True)
        return
    prec_id, dtype_name, jac_bytes = PRECISIONS[args.precision]
    tune_db = os.path.join(ROOT, "paper_2509_26581_amd", "tune_db.txt")
    tune_db = tune_db if os.path.exists(tune_db) else None
    if args.serve_only:
        out = serving_measurement(gba, synth, args.serve_requests, prec_id,
                                  args.serve_budget_mb << 20, args.serve_slots, tune_db,
                                  schedule=SCHEDULES[args.pcg_schedule])
        print(json.dumps({"serving": out}), flush=True)
        return
    t0 = time.perf_counter()
    sc = synth.make_scene(args.workload, seed=0)
    trials = args.trials or sc.trials
    print(f"[bench] workload {args.workload}: {sc.n_cams} cams, {sc.n_pts} pts, {sc.n_obs} obs "
          f"(generated in {time.perf_counter() - t0:.1f} s)", flush=True)
    n_pts_active = int(np.unique(sc.pt_idx).size)
    vec_bytes = 8 if args.precision == "fp64" else 4
    if args.solver == "full":
        alg_bytes = full_product_algorithmic_bytes(sc.n_obs, n_pts_active, sc.n_cams, jac_bytes,
                                                   vec_bytes, args.jacobian == "dynamic")
        product_kernel = "k_full_point_pass<kMatvec> (full-system product, point pass)"
    else:
        alg_bytes = matvec_algorithmic_bytes(sc.n_obs, n_pts_active, jac_bytes, vec_bytes)
        # one problem's camera vector in LDS (FP64, 160 KB per CU) or two passes
        two_pass = 9 * 8 * sc.n_cams + 1024 > 160 * 1024 or args.accumulation in (2, 3) \
            or args.deterministic
        blocked = two_pass and not args.deterministic and args.accumulation != 2 and \
            (args.accumulation == 3 or sc.n_cams > 1024) and SCHEDULES[args.pcg_schedule] != 2
        product_kernel = ("k_point_pass<kMatvec> + k_cam_block_pass (two-pass Schur product)"
                          if blocked else
                          "k_point_pass<kMatvec> + k_cam_pass<kMatvec> (two-pass Schur product)"
                          if two_pass else "k_point_pass<kMatvec> (fused Schur product)")

    def run_options(timing):
        return gba.options(pcg_max_iters=sc.pcg_max_iters, pcg_tol=sc.pcg_tol,
                           timing=1 if timing else 0, accumulation=args.accumulation,
                           tiles_per_block=args.tiles_per_block,
                           deterministic=1 if args.deterministic else 0,
                           pcg_schedule=SCHEDULES[args.pcg_schedule],
                           solver=SOLVERS[args.solver], jacobian=JACOBIANS[args.jacobian])

    def make_graph(prec_id, timing):
        opts = run_options(timing)
        return gba.Graph.from_arrays(sc.cams0, sc.pts0, sc.cam_idx, sc.pt_idx, sc.obs,
                                     loss=sc.loss, delta=sc.delta, precision=prec_id,
                                     options=opts, use_torch=True)

    def matvec_roofline(g):
        """Schur products back to back (MATVEC_WARMUP, then MATVEC_LAUNCHES timed)
        at the starting parameters and lambda 1e-4: average duration per launch."""
        gba.gba_time_matvec(g.h, 1e-4, MATVEC_WARMUP)
        avg_us = gba.gba_time_matvec(g.h, 1e-4, MATVEC_LAUNCHES)
        achieved = alg_bytes / (avg_us * 1e-6) / 1e9
        traffic = (MEASURED_TRAFFIC.get(args.precision)
                   if args.workload == "bal1m" and args.solver == "schur" else None)
        return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": product_kernel,
                "avg_us": round(avg_us, 2), "launches": MATVEC_LAUNCHES,
                "algorithmic_bytes": int(alg_bytes)}

    if args.matvec_only:
        g = make_graph(prec_id, False)
        gba.gba_prepare(g.h)
        print(json.dumps({"matvec_only": matvec_roofline(g), "precision": args.precision,
                          "workload": args.workload}), flush=True)
        g.close()
        return

    def timed_run(prec_id):
        g = make_graph(prec_id, False)
        t0 = time.perf_counter()
        gba.gba_prepare(g.h)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t0
        for w in range(args.warmup):
            gba.gba_reset(g.h)
            rep = g.solve(trials)
            print(f"[bench] precision {prec_id} warmup {w}: {rep.trials} trials, "
                  f"{rep.ms_total:.1f} ms, cost {rep.initial_cost:.6e} -> {rep.final_cost:.6e}",
                  flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        reports = []
        for k in range(args.steps):
            gba.gba_reset(g.h)
            reports.append(g.solve(trials))
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        return g, reports, elapsed, build_s

    g, reports, elapsed, build_s = timed_run(prec_id)
    print(f"[bench] graph build + upload {build_s:.2f} s", flush=True)
    total_trials = sum(r.trials for r in reports)
    lm_iters_s = total_trials / elapsed
    last = reports[-1]
    # outside the timed region: the matvec roofline, then one solve with
    # per-phase HIP events for the breakdown
    gba.gba_reset(g.h)
    roofline = matvec_roofline(g)
    phases = None
    if not args.no_timing:
        gba.gba_reset(g.h)
        gba.gba_set_options(g.h, run_options(True))
        rt = g.solve(trials)
        phases = {k: round(getattr(rt, k), 3) for k in
                  ("ms_total", "ms_linearize", "ms_precond", "ms_pcg", "ms_other", "ms_matvec")}
        phases["matvec_launches_timed"] = rt.matvec_count
    g.close()
    compare = None
    if not args.no_compare and prec_id != 0:
        g64, r64, e64, _ = timed_run(0)
        g64.close()
        v64 = sum(r.trials for r in r64) / e64
        compare = {"fp64_lm_iter_per_s": round(v64, 3), "mixed_over_fp64": round(lm_iters_s / v64, 3),
                   "fp64_final_cost": r64[-1].final_cost,
                   "mixed_vs_fp64_final_cost_rel": abs(last.final_cost - r64[-1].final_cost) /
                   r64[-1].final_cost}
    line = {
        "metric": METRIC, "value": round(lm_iters_s, 3), "unit": "LM iter/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype_name, "data": "synthetic",
        "config": {"workload": f"{args.workload}: {sc.n_cams} cameras, {sc.n_pts} points, "
                               f"{sc.n_obs} observations, Huber 1px, {trials} LM trials/step, "
                               f"PCG tol {sc.pcg_tol} max {sc.pcg_max_iters}",
                   "precision": args.precision, "seed": 0,
                   "accumulation": {0: "auto", 1: "lds", 2: "camera_pass"}[args.accumulation],
                   "tiles_per_block": args.tiles_per_block or "auto",
                   "deterministic": bool(args.deterministic),
                   "pcg_schedule": args.pcg_schedule, "solver": args.solver,
                   "jacobian": args.jacobian},
        "obs_per_s": round(sc.n_obs * lm_iters_s, 1),
        "pcg_iters_per_trial": round(sum(r.pcg_iters_total for r in reports) / max(total_trials, 1), 2),
        "final_cost": last.final_cost, "initial_cost": last.initial_cost,
        "phase_ms_per_solve": phases,
        "graph_build_s": round(build_s, 3), "workspace_bytes": int(last.workspace_bytes),
        "roofline": roofline,
        "fp64_comparison": compare,
    }
    line["vi"] = None
    if not args.no_vi and args.workload == "bal1m":
        line["vi"] = vi_measurement(gba, args)["vi"]
    line["bal8m"] = None
    if not args.no_bal8m and args.workload == "bal1m":
        line["bal8m"] = bal8m_measurement()
    line["serving"] = None
    if not args.no_serve:
        line["serving"] = serving_measurement(gba, synth, args.serve_requests, prec_id,
                                              args.serve_budget_mb << 20, args.serve_slots,
                                              tune_db, schedule=SCHEDULES[args.pcg_schedule])
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a one-trial sample ...", flush=True)
        line["cpu_baseline"] = cpu_baseline(sc)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
