"""Write the oracle's reference LM trajectories for the seeded workloads.

Calls only the FP64 oracle (and the seeded input generator).  Outputs
tests/golden/oracle_lm_config{0,1}.json with the initial and final cost and
the per-attempt history of the LM loop of Sec. 6.1 (10 iterations for the
tiny ring, 20 for the ladybug-like workload), and with --huber the same runs
under the Huber loss of Sec. 6.2 (delta 1 px) as oracle_lm_huber_config{c}.json.

    python tests/golden/make_golden.py [--huber] [config ...]
"""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from bal_synth import make_config, problem_stats  # noqa: E402

ITERS = {0: 10, 1: 20}


HUBER_DELTA = 1.0


def main(configs, huber=False):
    for c in configs:
        p = make_config(c)
        t0 = time.perf_counter()
        res = oracle.lm_solve(p.cameras, p.points, p.obs_cam, p.obs_pt, p.obs_uv,
                              oracle.LMOptions(max_iters=ITERS[c], huber_delta=HUBER_DELTA if huber else None))
        out = {
            "config": c,
            "huber_delta": HUBER_DELTA if huber else None,
            "stats": problem_stats(p),
            "lm_iters": ITERS[c],
            "initial_cost": res.cost0,
            "final_cost": res.final_cost,
            "status": res.status,
            "history": res.history,
            "oracle_seconds": time.perf_counter() - t0,
        }
        path = os.path.join(HERE, f"oracle_lm_huber_config{c}.json" if huber else f"oracle_lm_config{c}.json")
        with open(path, "w") as f:
            json.dump(out, f, indent=1)
        print(path, res.cost0, res.final_cost, res.status)


if __name__ == "__main__":
    args = [a for a in sys.argv[1:] if a != "--huber"]
    main([int(a) for a in args] or [0, 1], huber="--huber" in sys.argv[1:])
