"""Autotuner of the serving decomposition sizes.

The batched kernels split every resident problem into workgroups of a fixed
number of point tiles (point passes), edges (cost), points (damping), and the
host checks the PCG state every `pcg_sync_every` iterations.  This tool runs a
saturated local-BA stream on the server for candidate sizes (coordinate
descent from the built-in sizes, one parameter at a time), keeps the fastest,
and writes the tuning database the server reads (`tune_db`):

    # comment lines
    fp32.tiles_per_block 16
    fp32.edges_per_block 1024
    ...

  python -m paper_2509_26581_amd.autotune [--precision fp32] [--requests 96]
                                          [--out paper_2509_26581_amd/tune_db.txt]
"""
import argparse
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2509_26581_amd import gba, synth  # noqa: E402

PRECISIONS = {"fp64": gba.GBA_FP64, "fp32": gba.GBA_MIXED_FP32, "bf16": gba.GBA_MIXED_BF16}
SPACE = {
    "tiles_per_block": [4, 8, 16, 32, 64],
    "edges_per_block": [256, 512, 1024, 2048],
    "pts_per_block": [256, 512, 1024],
    "pcg_sync_every": [4, 8, 16, 32],
}
START = {"tiles_per_block": 16, "edges_per_block": 1024, "pts_per_block": 512, "pcg_sync_every": 8}


def saturated_rate(reqs, precision, sizes, slots, budget, repeats=2):
    """Solves/s with every request submitted at once (best of `repeats`)."""
    best = 0.0
    for _ in range(repeats):
        s = gba.Server(precision=precision, budget_bytes=budget, max_slots=slots, **sizes)
        t0 = time.perf_counter()
        tickets = [s.submit(r) for r in reqs]
        for t in tickets:
            s.poll(t)
        dt = time.perf_counter() - t0
        s.close()
        best = max(best, len(reqs) / dt)
    return best


def tune(precision_name="fp32", n_req=96, slots=64, budget=4 << 30, seed=7, log=print):
    precision = PRECISIONS[precision_name]
    reqs = [synth.make_local_request(50_000 + seed * 1000 + k) for k in range(n_req)]
    cur = dict(START)
    cur_rate = saturated_rate(reqs, precision, cur, slots, budget)
    log(f"start {cur} -> {cur_rate:.1f} solves/s")
    trace = [(dict(cur), cur_rate)]
    for name, values in SPACE.items():
        for v in values:
            if v == cur[name]:
                continue
            cand = dict(cur, **{name: v})
            rate = saturated_rate(reqs, precision, cand, slots, budget)
            trace.append((cand, rate))
            log(f"  {name}={v}: {rate:.1f} solves/s")
            if rate > cur_rate * 1.02:       # keep only clear wins
                cur, cur_rate = cand, rate
        log(f"after {name}: {cur} -> {cur_rate:.1f} solves/s")
    return cur, cur_rate, trace


def write_db(path, precision_name, sizes, rate, n_req, slots):
    lines = []
    if os.path.exists(path):
        with open(path) as f:
            lines = [ln.rstrip("\n") for ln in f
                     if not ln.startswith(precision_name + ".")
                     and not ln.startswith(f"# {precision_name}:")]
    lines.append(f"# {precision_name}: {rate:.1f} solves/s saturated, {n_req} local-BA "
                 f"requests, {slots} slots")
    for k, v in sizes.items():
        lines.append(f"{precision_name}.{k} {v}")
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--precision", default="fp32", choices=list(PRECISIONS))
    ap.add_argument("--requests", type=int, default=96)
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--out", default=os.path.join(ROOT, "paper_2509_26581_amd", "tune_db.txt"))
    args = ap.parse_args()
    gba.load()
    sizes, rate, _ = tune(args.precision, args.requests, args.slots,
                          log=lambda m: print("[autotune]", m, flush=True))
    write_db(args.out, args.precision, sizes, rate, args.requests, args.slots)
    print(f"[autotune] wrote {args.out}: {sizes} ({rate:.1f} solves/s)", flush=True)


if __name__ == "__main__":
    main()
