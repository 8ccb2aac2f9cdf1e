"""Write the oracle's reference LM trajectories for the seeded workloads.

Calls only the FP64 oracle (and the seeded input generator).  Every run is the
LM loop of Sec. 6.1 with at most 10 attempts for the tiny ring, 20 for the
ladybug-like workload and 50 (the paper's limit) for the others:

  oracle_lm_config{0,1}.json       whole trajectory, assembled Schur complement
  oracle_lm_config3.json           venice-like: whole trajectory, the Schur
                                   complement applied to vectors
  oracle_lm_config2.json           batch of 256: every problem's own LM loop
                                   (final cost, decisions and PCG counts)
  oracle_first_attempt_config4.json  dense stress: the first attempt (lambda0)
  oracle_lm_config4.json           dense stress: whole trajectory (--full4)

With --huber the tiny and ladybug-like runs use the Huber loss of Sec. 6.2
(delta 1 px) and go to oracle_lm_huber_config{c}.json.

    python tests/golden/make_golden.py [--huber] [--full4] [--workers N] [config ...]
"""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from bal_synth import make_config, problem_stats, split_batch  # noqa: E402

ITERS = {0: 10, 1: 20, 2: 50, 3: 50, 4: 50}
# the assembled Schur complement for the small workloads, applied to vectors for the large ones
SOLVER = {0: "pcg", 1: "pcg", 2: "pcg", 3: "pcg_operator", 4: "pcg_operator"}
HUBER_DELTA = 1.0


def _write(name, out):
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(path, flush=True)


class _Progress:
    """Prints each LM attempt as the oracle finishes it (long runs)."""

    def __init__(self, tag):
        self.tag, self.t0 = tag, time.perf_counter()

    def __call__(self, h):
        print(f"{self.tag}: attempt {h['iter']} lambda {h['lambda']:.3g} cost {h['cost']:.10g} -> "
              f"{h['new_cost']:.10g} {'accepted' if h['accepted'] else 'rejected'}, {h['pcg_iters']} PCG, "
              f"{time.perf_counter() - self.t0:.0f} s", flush=True)


def trajectory(c, huber=False):
    p = make_config(c)
    t0 = time.perf_counter()
    opts = oracle.LMOptions(max_iters=ITERS[c], solver=SOLVER[c], huber_delta=HUBER_DELTA if huber else None)
    res = oracle.lm_solve(p.cameras, p.points, p.obs_cam, p.obs_pt, p.obs_uv, opts,
                          progress=_Progress(f"config {c}"))
    out = {
        "config": c,
        "huber_delta": HUBER_DELTA if huber else None,
        "solver": SOLVER[c],
        "stats": problem_stats(p),
        "lm_iters": ITERS[c],
        "initial_cost": res.cost0,
        "final_cost": res.final_cost,
        "status": res.status,
        "history": res.history,
        "oracle_seconds": time.perf_counter() - t0,
    }
    _write(f"oracle_lm_huber_config{c}.json" if huber else f"oracle_lm_config{c}.json", out)


def _batch_problem(args):
    i, q = args
    res = oracle.lm_solve(q.cameras, q.points, q.obs_cam, q.obs_pt, q.obs_uv,
                          oracle.LMOptions(max_iters=ITERS[2], solver=SOLVER[2]))
    return {"problem": i, "n_cams": q.n_cams, "n_points": q.n_points, "n_obs": q.n_obs,
            "initial_cost": res.cost0, "final_cost": res.final_cost, "status": res.status,
            "iterations": res.iterations,
            "decisions": "".join("A" if h["accepted"] else "R" for h in res.history),
            "pcg_iters": [h["pcg_iters"] for h in res.history],
            "new_costs": [h["new_cost"] for h in res.history]}


def batch(workers):
    from multiprocessing import Pool

    p = make_config(2)
    probs = split_batch(p)
    t0 = time.perf_counter()
    with Pool(workers) as pool:
        rows = []
        for r in pool.imap(_batch_problem, list(enumerate(probs))):
            rows.append(r)
            if len(rows) % 16 == 0:
                print(f"batch: {len(rows)} problems, {time.perf_counter() - t0:.0f} s", flush=True)
    _write("oracle_lm_config2.json", {
        "config": 2, "solver": SOLVER[2], "stats": problem_stats(p), "lm_iters": ITERS[2],
        "initial_cost": sum(r["initial_cost"] for r in rows), "final_cost": sum(r["final_cost"] for r in rows),
        "problems": rows, "oracle_seconds": time.perf_counter() - t0})


def first_attempt(c, lam=1e-4):
    """The first LM attempt at lambda0 (the linearization at the perturbed start)."""
    p = make_config(c)
    t0 = time.perf_counter()
    bk = oracle.build_bookkeeping(p.n_cams, p.n_points, p.obs_cam, p.obs_pt, p.obs_uv)
    st = oracle.state_from_bal(p.cameras, p.points)
    lin = oracle.linearize(st, bk, p.obs_uv)
    a = oracle.lm_attempt(st, bk, p.obs_uv, lin, lam, oracle.LMOptions(solver=SOLVER[c]))
    _write(f"oracle_first_attempt_config{c}.json", {
        "config": c, "solver": SOLVER[c], "stats": problem_stats(p), "lambda": lam,
        "initial_cost": lin.cost, "pred": a["pred"], "new_cost": a["new_cost"], "pcg_iters": a["pcg_iters"],
        "rel_res": a["rel_res"], "pcg_status": a["pcg_status"], "oracle_seconds": time.perf_counter() - t0})


if __name__ == "__main__":
    argv = sys.argv[1:]
    huber = "--huber" in argv
    full4 = "--full4" in argv
    workers = 4
    if "--workers" in argv:
        workers = int(argv[argv.index("--workers") + 1])
        del argv[argv.index("--workers"): argv.index("--workers") + 2]
    configs = [int(a) for a in argv if not a.startswith("--")] or [0, 1]
    for c in configs:
        if c == 2:
            batch(workers)
        elif c == 4:
            first_attempt(4)
            if full4:
                trajectory(4)
        else:
            trajectory(c, huber)
