"""Write the oracle's reference solve of the 1M-observation workload
(1,000 cameras, 200,000 points, seed 0, Huber delta = 1 px, 20 LM trials,
exact damped solves) to bal8m_proxy_seed0.json.  Calls only the input generator
and the CPU oracle.  Run: python tests/golden/make_golden_bal1m.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import ba  # noqa: E402
from paper_2509_26581_amd import synth  # noqa: E402


def main(seed=0, trials=15, out=os.path.join(HERE, "bal8m_proxy_seed0.json")):
    sc = synth.make_scene("bal8m_proxy", seed=seed)
    prob = ba.BAProblem(sc.n_cams, sc.n_pts, sc.cam_idx, sc.pt_idx, sc.obs,
                        loss=sc.loss, delta=sc.delta)
    t0 = time.time()
    res = ba.solve(prob, sc.cams0, sc.pts0, trials)
    dt = time.time() - t0
    cams, pts = res.x
    sample = np.arange(0, sc.n_pts, 100)
    doc = dict(
        source="oracle.ba.solve on synth.make_scene('bal8m_proxy', seed=%d), %d trials, "
               "initial lambda 1e-4, exact block-Cholesky steps" % (seed, trials),
        seed=seed, trials=trials, n_obs=int(sc.n_obs), seconds=dt,
        initial_cost=res.initial_cost, final_cost=res.cost,
        log=[{k: (float(v) if not isinstance(v, bool) else v) for k, v in e.items()}
             for e in res.log],
        cams=cams.tolist(), point_sample=sample.tolist(), points=pts[sample].tolist())
    with open(out, "w") as f:
        json.dump(doc, f)
    print("wrote", out, "final cost", res.cost, "in", dt, "s")


if __name__ == "__main__":
    main()
