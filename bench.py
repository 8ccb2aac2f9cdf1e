#!/usr/bin/env python
"""Benchmark of the square-root BA hot path on one MI355X.

Workload (default): the venice-like problem (1,778-camera ring, 1M landmarks
with k = min(400, 2 + floor(LogNormal(0.40, 1.30))) observations, ~5M
observations, 5.4 GB of landmark blocks resident in HBM), seeded synthetic
data, FP32.  One step is one full Levenberg-Marquardt solve (at most 50
attempts, the paper's limit) from the same perturbed start, with every input
resident in HBM: each attempt runs linearize, QR marginalization, Givens
damping, block-Jacobi + right-hand side, PCG, back-substitution, update and
cost.

Printed JSON line: time-to-1%-cost (the headline value, from the timed steps in
the production configuration: graph-captured PCG, no profiler), QR blocks/s
and the stage breakdown (one more profiled solve), PCG matvec GB/s with its
roofline (HIP events around back-to-back products on the resident blocks,
algorithmic bytes 4 (18 k^2 + 9 k) per landmark), the learned preconditioner
against block-Jacobi, the same solve in FP64 (libsqrtba64.so, "sqrt_ba_64"), and
the FP64 oracle's CPU baseline on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--config {1,2,3,4}]
    python bench.py --precision 64     # the FP64 library as the timed path
    python bench.py --calibrate-copy   # known-size copy, for counter scaling
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
FORCING_ETA = 0.1  # the paper's CG truncation (Sec. 6.1, as in Ceres)
HUBER_DELTA = 1.0  # the paper's robust loss parameter in pixels (Sec. 6.2)
WORKLOADS = {
    1: "ladybug-like: 500 cameras on a forward trajectory, 100k landmarks, k = 2 + Geom(1/3) clamped to 50, "
       "BAL camera model, 1 px noise",
    2: "batch of 256 ring problems: cameras U{5..60}, landmarks U{200..5000}, k ~ U{2..min(30, cameras)}",
    3: "venice-like: 1,778-camera ring, 1M landmarks, k = min(400, 2 + floor(LogNormal(0.40, 1.30)))",
    4: "dense stress: 2,000-camera ring, 50k landmarks, k = 50 + min(450, floor(Exp(160)))",
}
METRIC = "time-to-1%-cost (s), QR blocks/s, PCG matvec HBM GB/s; learned vs block-Jacobi"
GOLDEN = os.path.join(ROOT, "tests", "golden", "oracle_lm_config{}.json")
GOLDEN_HUBER = os.path.join(ROOT, "tests", "golden", "oracle_lm_huber_config{}.json")
# HBM counter readings of the product per workload (valid for the kernels and
# launch shapes they were taken with)
TRAFFIC_TAG = {1: "ladybug", 2: "batch256", 3: "venice", 4: "dense"}
# LM attempts per workload: 20 for the ladybug-like one (its stored oracle run),
# the paper's limit of 50 for the others (Sec. 6.1)
LM_ITERS = {1: 20, 2: 50, 3: 50, 4: 50}  # profiles/matvec_traffic_<tag>_<blocks>.json
KERNELS = os.path.join(ROOT, "paper_2103_01843_amd", "csrc", "kernels.hip")


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def kernels_hash() -> str:
    with open(KERNELS, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def time_to_tol(hist, t_tol_cost):
    for h in hist:
        if h["accepted"] and h["new_cost"] <= t_tol_cost:
            return h["t"]
    return float("inf")


def _host_cpu() -> dict:
    """Host facts recorded next to the CPU baseline: logical cores, model, sockets."""
    model, sockets = None, set()
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name") and model is None:
                    model = line.split(":", 1)[1].strip()
                elif line.startswith("physical id"):
                    sockets.add(line.split(":", 1)[1].strip())
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"nproc": usable, "cpu_count": os.cpu_count(), "cpu_model": model, "sockets": len(sockets) or None}


def _oracle_threads() -> str:
    try:
        from threadpoolctl import threadpool_info
        return ", ".join(f"{i.get('internal_api')} {i.get('num_threads')}" for i in threadpool_info())
    except Exception:
        return "unknown"


def _golden(cfg: int, lm_iters: int):
    """The stored oracle run of a workload if it used the same number of LM attempts."""
    if not os.path.exists(GOLDEN.format(cfg)):
        return None
    with open(GOLDEN.format(cfg)) as f:
        gold = json.load(f)
    return gold if gold.get("lm_iters") == lm_iters else None


def _cores_used(cpu0: float, wall0: float) -> dict:
    """Threads the oracle actually kept busy since (cpu0, wall0): its process CPU
    time over the wall time (numpy's element-wise and gather steps run on one
    thread, BLAS calls on the pool)."""
    cpu, wall = time.process_time() - cpu0, time.perf_counter() - wall0
    return {"cores": max(1, round(cpu / wall)) if wall > 0 else 1, "cpu_s": cpu, "wall_s": wall}


def cpu_baseline(problem, cfg: int, f_taus, lm_iters: int, budget_s: float = 30.0):
    """The FP64 oracle (numpy/scipy, as it is) timed on the host's cores.

    ladybug-like: the oracle's own LM loop on the whole workload, measured until
    its first accepted attempt at or below the 1% threshold (~20 s).
    batch of 256: the oracle's LM loop problem by problem, each until it reaches
    its own threshold, for as many problems as fit the budget; scaled to the
    whole batch by the observation count.
    venice-like and dense stress: one oracle attempt is minutes of CPU work, so
    the sample is the first attempt on a prefix of the landmarks (about 1M
    observations): linearization, the Schur complement applied to vectors with
    its preconditioner blocks, 10 PCG iterations, back-substitution and the new
    cost, each stage timed and scaled to the whole workload by the observation
    count; the stored oracle run of the workload gives the number of attempts,
    linearizations and PCG iterations until its cost first reaches the
    threshold, over which the scaled stage times are summed."""
    import numpy as np
    import oracle
    from bal_synth import split_batch
    from oracle.lm import cost_of
    from oracle.solvers import pcg

    host = _host_cpu()
    base = {"unit": "s", "kind": "oracle", "host": host, "threads": _oracle_threads()}
    p = problem
    if cfg == 1:
        f_tau = f_taus[0][2]
        t0, c0 = time.perf_counter(), time.process_time()
        bk = oracle.build_bookkeeping(p.n_cams, p.n_points, p.obs_cam, p.obs_pt, p.obs_uv)
        res = oracle.lm_solve(p.cameras, p.points, p.obs_cam, p.obs_pt, p.obs_uv, oracle.LMOptions(max_iters=lm_iters),
                              bk, progress=lambda h: h["accepted"] and h["new_cost"] <= f_tau)
        reached = res.status == "stopped"
        h = res.history[-1]
        return {**base, "value": h["t"] if reached else None, **_cores_used(c0, t0),
                "sample": (f"the oracle's LM loop (assembled Schur complement, block-Jacobi PCG) on the whole workload "
                           f"until its first accepted attempt at or below the 1% threshold: {res.iterations} attempts, "
                           f"{sum(x['pcg_iters'] for x in res.history)} PCG iterations, measured, "
                           f"{time.perf_counter() - t0:.1f} s including bookkeeping")}
    if cfg == 2:
        probs = split_batch(p)
        t0, c0 = time.perf_counter(), time.process_time()
        spent, obs_done, n_done = 0.0, 0, 0
        for i, q in enumerate(probs):
            f_tau = f_taus[i][2]
            res = oracle.lm_solve(q.cameras, q.points, q.obs_cam, q.obs_pt, q.obs_uv,
                                  oracle.LMOptions(max_iters=lm_iters),
                                  progress=lambda h, f=f_tau: h["accepted"] and h["new_cost"] <= f)
            if res.status != "stopped":
                return {**base, "value": None, **_cores_used(c0, t0), "sample": f"problem {i} did not reach its threshold"}
            spent += res.history[-1]["t"]
            obs_done += q.n_obs
            n_done += 1
            if time.perf_counter() - t0 > budget_s:
                break
        return {**base, "value": spent * p.n_obs / obs_done, **_cores_used(c0, t0),
                "sample": (f"the oracle's LM loop on the first {n_done} of {len(probs)} problems, each until it "
                           f"reaches its own 1% threshold (measured {spent:.1f} s over {obs_done} observations), "
                           f"scaled to all {p.n_obs} observations")}
    gold = _golden(cfg, lm_iters)
    if gold is None or "history" not in gold:
        return None
    f_tau = f_taus[0][2]
    n_lin, n_att, n_pcg, reached = 1, 0, 0, False
    for h in gold["history"]:
        n_att += 1
        n_pcg += h["pcg_iters"]
        if h["accepted"] and h["new_cost"] <= f_tau:
            reached = True
            break
        n_lin += 1 if h["accepted"] else 0
    if not reached:
        return {**base, "value": None, "cores": None, "sample": "the stored oracle run never reaches the threshold"}
    # prefix of the landmarks holding about 1M observations
    n_sub = int(np.searchsorted(np.cumsum(np.bincount(p.obs_pt, minlength=p.n_points)), 1_000_000)) + 1
    m = p.obs_pt < n_sub
    t = {}
    ta, ca = time.perf_counter(), time.process_time()
    bk = oracle.build_bookkeeping(p.n_cams, n_sub, p.obs_cam[m], p.obs_pt[m], p.obs_uv[m])
    st = oracle.state_from_bal(p.cameras, p.points[:n_sub])
    tb = time.perf_counter()
    lin = oracle.linearize(st, bk, p.obs_uv[m])
    t["linearize"] = time.perf_counter() - tb
    tb = time.perf_counter()
    op = oracle.reduced_system_operator(lin, 1e-4)
    t["reduced_system"] = time.perf_counter() - tb
    tb = time.perf_counter()
    res = pcg(op.matvec, op.b, op.blocks, 0.0, 10)
    t["pcg_iteration"] = (time.perf_counter() - tb) / max(1, res.iters)
    tb = time.perf_counter()
    dxl = oracle.back_substitute(op, res.x)
    oracle.model_decrease(lin, res.x, dxl)
    cost_of(oracle.apply_update(st, res.x.reshape(-1, 9) * lin.sp, dxl.reshape(-1, 3) * lin.sl), bk, p.obs_uv[m])
    t["back_substitution_and_cost"] = time.perf_counter() - tb
    used = _cores_used(ca, ta)
    sample_s = used["wall_s"]
    scale = p.n_obs / float(m.sum())
    est = scale * (n_lin * t["linearize"] + n_att * (t["reduced_system"] + t["back_substitution_and_cost"])
                   + n_pcg * t["pcg_iteration"])
    return {**base, "value": est, **used,
            "sample_stage_s": t, "sample_obs": int(m.sum()), "scale_by_obs": scale,
            "sample": (f"the oracle's first attempt on the first {n_sub} landmarks ({int(m.sum())} of {p.n_obs} "
                       f"observations, {sample_s:.1f} s: linearize, Schur complement applied to vectors with its "
                       f"block-Jacobi blocks, {res.iters} PCG iterations, back-substitution and cost), each stage "
                       f"scaled by the observation count, summed over the stored oracle run to the 1% threshold: "
                       f"{n_att} attempts, {n_lin} linearizations, {n_pcg} PCG iterations"),
            "oracle_run_in_build_container_s": gold["history"][n_att - 1]["t"]}


def learned_run(ctx, n_problems: int, lm_iters: int):
    """Train the learned preconditioner online on the solver's own PCG traces of
    a separate ladybug-like problem (its own seed), then solve the workload once
    more from the same start with it.  Training is outside the solve's clock."""
    import numpy as np
    import torch
    from bal_synth import BASE_SEED, make_forward_problem
    from paper_2103_01843_amd import Context

    t0 = time.perf_counter()
    tp = make_forward_problem(np.random.default_rng(BASE_SEED + 101))
    tc = Context(stream=torch.cuda.current_stream(), max_lm_iters=lm_iters)
    tc.load(tp.cameras, tp.points, tp.obs_cam, tp.obs_pt, tp.obs_uv, tp.cam_off, tp.pt_off)
    tc.bind_torch_workspace()
    tc.mlp_init(0)
    tc.pcg_trace(20, 64)
    tc.lm_solve()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    losses = []
    for chunk in range(8):
        losses.append(float(np.mean(tc.mlp_train(50, batch=4096, lr=1e-3, seed=chunk))))
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    theta = tc.mlp_get_params()
    n_samples = tc.trace_size()
    tc.close()
    log(f"learned: trace {t1 - t0:.2f} s, training {t2 - t1:.2f} s, loss {losses[0]:.4f} -> {losses[-1]:.4f}")
    ctx.mlp_set_params(theta)
    ctx.set_preconditioner("learned")
    ctx.restore_state()
    reps = ctx.lm_solve()
    hist = [ctx.history(i) for i in range(n_problems)]
    stats = ctx.learned_stats()
    ctx.set_preconditioner("block_jacobi")
    log(f"learned: {sum(r.total_pcg_iters for r in reps)} PCG iterations, final cost "
        f"{sum(r.final_cost for r in reps):.6g}, {stats}")
    return {"reports": reps, "history": hist, "trace_and_generate_s": t1 - t0, "train_s": t2 - t1,
            "train_steps": 400, "trace_solves_records": list(n_samples),
            "train_loss_first_last": [losses[0], losses[-1]], **stats}


def other_blocks_run(p, args, blocks: int, precision: int = 32):
    """Timed solves (same steps and warm-up) and the product timing with the given
    landmark-block form and precision; returns its reports, histories and figures."""
    import torch
    from paper_2103_01843_amd import Context

    ctx = Context(stream=torch.cuda.current_stream(), max_lm_iters=args.lm_iters, landmark_blocks=blocks,
                  precision=precision)
    ctx.load(p.cameras, p.points, p.obs_cam, p.obs_pt, p.obs_uv, p.cam_off, p.pt_off)
    ctx.bind_torch_workspace()
    ctx.save_state()
    ws = ctx.workspace_bytes()
    if blocks == 0 and not args.no_autotune:
        ctx.autotune(reps=10)
    for _ in range(args.warmup):
        ctx.restore_state()
        ctx.lm_solve()
    runs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.restore_state()
        reps = ctx.lm_solve()
        runs.append((reps, [ctx.history(i) for i in range(p.n_problems)]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    mv_ms, mv_bytes = ctx.time_product(reps=50)
    ctx.close()
    del ctx
    torch.cuda.empty_cache()
    log(f"{['explicit', 'implicit', 'explicit Schur complement'][blocks]} blocks, FP{precision}: "
        f"{1e3 * wall / args.steps:.1f} ms per solve, "
        f"product {1e3 * mv_ms:.1f} us, workspace {ws / 1e9:.2f} GB")
    return {"runs": runs, "wall": wall, "mv_ms": mv_ms, "mv_bytes": mv_bytes, "workspace_bytes": ws}


def calibrate_copy():
    import torch
    n = 1 << 28  # 1 GiB of float32
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 5}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--lm-iters", type=int, default=None, help="LM attempts (default: 20 ladybug-like, 50 else)")
    ap.add_argument("--config", type=int, default=3, choices=[1, 2, 3, 4],
                    help="workload: 1 ladybug-like, 2 batch of 256, 3 venice-like (default), 4 dense stress")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-preconditioner comparison")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default product launch shapes")
    ap.add_argument("--blocks", choices=["explicit", "implicit", "sc"], default="explicit",
                    help="landmark blocks of the timed solves: explicit (the paper's stored nullspace blocks "
                         "Q2^T J_p, O(k^2) per landmark; default), implicit (J_p and Q1 per observation, O(k)) "
                         "or sc (the explicit FP32 Schur-complement comparator, camera-pair blocks)")
    ap.add_argument("--no-other-blocks", action="store_true",
                    help="skip the extra measurement of the other landmark-block form")
    ap.add_argument("--no-forcing", action="store_true",
                    help="skip the solve with the forcing-sequence PCG truncation (eta = 0.1)")
    ap.add_argument("--no-huber", action="store_true",
                    help="skip the solve with the Huber loss (delta = 1 px, IRLS)")
    ap.add_argument("--precision", type=int, choices=[32, 64], default=32,
                    help="element type of the timed path: 32 (libsqrtba.so, the default) or 64 (libsqrtba64.so)")
    ap.add_argument("--no-fp64", action="store_true",
                    help="skip the FP64 solve of the same workload (reported as sqrt_ba_64)")
    ap.add_argument("--no-sc", action="store_true",
                    help="skip the explicit FP32 Schur-complement comparator (landmark_blocks = 2)")
    ap.add_argument("--tuning", default=None, metavar="EDGE,ROWS,SIDE,SEP,BATCH,PERSIST[,NT]",
                    help="fixed product bucket edge and launch shapes (rows_min_k, huge_rows, huge_side, "
                         "large_separate, small_rows, persist_wgs, and optionally stream_loads, else 0) instead "
                         "of autotuning, e.g. for counter runs under a profiler")
    ap.add_argument("--calibrate-copy", action="store_true")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for {max(args.gpus, world)}): the library has no multi-GPU "
              "path (landmark-sharded execution is not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.calibrate_copy:
        calibrate_copy()
        return

    import numpy as np
    import torch
    from bal_synth import make_config, problem_stats
    from paper_2103_01843_amd import Context

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    cfg = args.config
    if args.lm_iters is None:
        args.lm_iters = LM_ITERS[cfg]
    log(f"generating workload {cfg}: {WORKLOADS[cfg]}")
    p = make_config(cfg)
    stats = problem_stats(p)
    log(f"workload: {stats}")
    torch.cuda.synchronize()
    t_up = time.perf_counter()
    blocks = {"explicit": 0, "implicit": 1, "sc": 2}[args.blocks]
    ctx = Context(stream=torch.cuda.current_stream(), max_lm_iters=args.lm_iters, landmark_blocks=blocks,
                  precision=args.precision)
    ctx.load(p.cameras, p.points, p.obs_cam, p.obs_pt, p.obs_uv, p.cam_off, p.pt_off)
    ctx.bind_torch_workspace()
    ctx.save_state()  # first device use: host bookkeeping, then upload over PCIe
    torch.cuda.synchronize()
    upload_s = time.perf_counter() - t_up
    log(f"uploaded: workspace {ctx.workspace_bytes() / 1e9:.2f} GB in {upload_s:.2f} s (host bookkeeping + PCIe)")
    tuning = {"shape": ctx.get_tuning(), "autotuned": False}
    if args.tuning:
        keys = ["rows_min_k", "huge_rows", "huge_side", "large_separate", "small_rows", "persist_wgs",
                "stream_loads"]
        vals = [int(x) for x in args.tuning.split(",")]
        if len(vals) not in (6, 7):
            raise SystemExit("--tuning takes 6 or 7 comma-separated integers")
        ctx.set_tuning(**dict(zip(keys, vals + [0] * (7 - len(vals)))))
        tuning = {"shape": ctx.get_tuning(), "autotuned": False}
    elif blocks == 1:
        tuning["note"] = "the launch shapes belong to the explicit-block product; the implicit product has one"
    elif not args.no_autotune:
        t0 = time.perf_counter()
        best, trials = ctx.autotune(reps=10)
        tuning = {"shape": best, "autotuned": True, "seconds": time.perf_counter() - t0,
                  "trials": [dict(shape, ms=ms) for shape, ms in trials]}
        log(f"autotune: {best} from {len(trials)} candidates")
    for w in range(args.warmup):
        ctx.restore_state()
        rep = ctx.lm_solve()
        log(f"warmup {w}: {max(r.iterations for r in rep)} attempts, final cost {sum(r.final_cost for r in rep):.6g}, "
            f"{max(r.solve_seconds for r in rep):.3f} s")
    # timed steps: the production configuration (graph-captured PCG, no profiler)
    runs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        ctx.restore_state()
        reps = ctx.lm_solve()
        runs.append((reps, [ctx.history(i) for i in range(p.n_problems)]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for s, (reps, h) in enumerate(runs):
        log(f"step {s}: {max(r.iterations for r in reps)} attempts, {sum(r.total_pcg_iters for r in reps)} PCG "
            f"iterations, final cost {sum(r.final_cost for r in reps):.6g}, {max(r.solve_seconds for r in reps):.3f} s")
    # the product kernel's duration: HIP events around back-to-back launches on
    # the resident blocks of the workload (same shapes as the timed steps)
    mv_ms, mv_bytes = ctx.time_product(reps=50)
    # stage breakdown: one more solve from the same start with the profiler on
    # (HIP events around every stage; PCG iterations launched one by one)
    ctx.restore_state()
    ctx.profile_enable(True)
    ctx.lm_solve()
    prof = ctx.profile()
    ctx.profile_enable(False)
    # the paper's PCG truncation (forcing sequence, eta = 0.1) from the same start
    forcing = None
    if not args.no_forcing:
        ctx.set_options(pcg_forcing_eta=FORCING_ETA)
        ctx.restore_state()
        torch.cuda.synchronize()
        t0f = time.perf_counter()
        freps = ctx.lm_solve()
        torch.cuda.synchronize()
        forcing = {"reports": freps, "history": [ctx.history(i) for i in range(p.n_problems)],
                   "wall_s": time.perf_counter() - t0f}
        ctx.set_options(pcg_forcing_eta=0.0)
        log(f"forcing sequence: {max(r.iterations for r in freps)} attempts, "
            f"{sum(r.total_pcg_iters for r in freps)} PCG iterations, final cost {sum(r.final_cost for r in freps):.6g}")
    # the paper's experimental loss (Huber, 1 px, by IRLS) from the same start
    huber = None
    if not args.no_huber:
        ctx.set_options(huber_delta=HUBER_DELTA)
        ctx.restore_state()
        torch.cuda.synchronize()
        t0h = time.perf_counter()
        hreps = ctx.lm_solve()
        torch.cuda.synchronize()
        huber = {"reports": hreps, "history": [ctx.history(i) for i in range(p.n_problems)],
                 "wall_s": time.perf_counter() - t0h}
        ctx.set_options(huber_delta=0.0)
        log(f"huber loss: {max(r.iterations for r in hreps)} attempts, {sum(r.total_pcg_iters for r in hreps)} "
            f"PCG iterations, robust cost {sum(r.initial_cost for r in hreps):.6g} -> "
            f"{sum(r.final_cost for r in hreps):.6g}, {1e3 * huber['wall_s']:.1f} ms")
    learned = None
    if not args.no_learned and args.precision == 32:
        try:
            learned = learned_run(ctx, p.n_problems, args.lm_iters)
        except Exception as e:  # reported, never required
            log(f"learned comparison failed: {e!r}")
    ctx.close()
    del ctx
    torch.cuda.empty_cache()

    # the other landmark-block form on the same workload and start (implicit
    # blocks need no O(k^2) storage): timed solves and its product
    other = None
    if not args.no_other_blocks:
        try:
            other = other_blocks_run(p, args, 1 if blocks == 0 else 0, args.precision)
        except Exception as e:  # e.g. explicit FP64 blocks of the dense workload exceed the GPU's memory
            log(f"other landmark-block form skipped: {e}")
            other = {"skipped": str(e)}
    # the paper's explicit-solver comparator: FP32 Schur complement from the normal equations
    sc = None
    if not args.no_sc and blocks != 2 and args.precision == 32:
        try:
            sc = other_blocks_run(p, args, 2)
        except Exception as e:  # e.g. too many camera-pair contributions (dense workload)
            log(f"explicit Schur complement comparator skipped: {e}")
            sc = {"skipped": str(e)}

    # square-root BA in FP64 (the paper's double-precision variant), same form and start
    fp64 = None
    if not args.no_fp64 and args.precision == 32:
        try:
            fp64 = other_blocks_run(p, args, blocks, 64)
        except Exception as e:  # e.g. the FP64 workspace exceeds the GPU's memory (dense workload)
            log(f"FP64 solve skipped: {e}")
            fp64 = {"skipped": str(e)}

    # time to 1% cost per problem (appendix A.2), f* over the runs (and the oracle where stored)
    gold = _golden(cfg, args.lm_iters)
    oracle_finals = [None] * p.n_problems
    if gold and "problems" in gold and len(gold["problems"]) == p.n_problems:
        oracle_finals = [g["final_cost"] for g in gold["problems"]]
    elif gold and "final_cost" in gold and p.n_problems == 1:
        oracle_finals = [gold["final_cost"]]
    ttt_all, f_taus = [], []
    for i in range(p.n_problems):
        f0 = runs[0][0][i].initial_cost
        finals = [reps[i].final_cost for reps, _ in runs]
        if learned:
            finals.append(learned["reports"][i].final_cost)
        if forcing:
            finals.append(forcing["reports"][i].final_cost)
        if other and "runs" in other:
            finals += [reps[i].final_cost for reps, _ in other["runs"]]
        if sc and "runs" in sc:
            finals += [reps[i].final_cost for reps, _ in sc["runs"]]
        if fp64 and "runs" in fp64:
            finals += [reps[i].final_cost for reps, _ in fp64["runs"]]
        fstar = min(finals + ([oracle_finals[i]] if oracle_finals[i] is not None else []))
        f_tau = fstar + 0.01 * (f0 - fstar)
        f_taus.append((f0, fstar, f_tau))
        ttt_all.append([time_to_tol(h[i], f_tau) for _, h in runs])
    # a batch reaches the threshold when its last problem does
    ttt = [max(t[s] for t in ttt_all) for s in range(len(runs))]
    other_out = None
    if other and "skipped" in other:
        other_out = {"skipped": other["skipped"]}
    elif other:
        ttt_o = [max(time_to_tol(h[i], f_taus[i][2]) for i in range(p.n_problems)) for _, h in other["runs"]]
        ach = other["mv_bytes"] / (other["mv_ms"] * 1e-3) / 1e9 if other["mv_ms"] > 0 else None
        other_out = {
            "landmark_blocks": "explicit" if blocks else "implicit",
            "time_to_1pct_cost_s": statistics.median(ttt_o),
            "ms_per_step": 1e3 * other["wall"] / args.steps,
            "final_costs": [sum(r.final_cost for r in reps) for reps, _ in other["runs"]],
            "pcg_iters": sum(r.total_pcg_iters for r in other["runs"][-1][0]),
            "workspace_bytes": other["workspace_bytes"],
            "product": {"avg_launch_ms": other["mv_ms"], "algorithmic_bytes_per_launch": other["mv_bytes"],
                        "achieved_GBps": ach, "frac_of_hbm_peak": ach / HBM_PEAK_GBPS if ach else None},
        }
    forcing_out = None
    if forcing:
        forcing_out = {
            "eta": FORCING_ETA,
            "time_to_1pct_cost_s": max(time_to_tol(forcing["history"][i], f_taus[i][2]) for i in range(p.n_problems)),
            "ms_per_solve": 1e3 * forcing["wall_s"],
            "lm_attempts": max(r.iterations for r in forcing["reports"]),
            "pcg_iters": sum(r.total_pcg_iters for r in forcing["reports"]),
            "final_cost": sum(r.final_cost for r in forcing["reports"]),
        }
    sc_out = None
    if sc and "skipped" in sc:
        sc_out = {"skipped": sc["skipped"]}
    elif sc:
        def rejected(hist, resolvable=False):
            # resolvable: the model predicts a decrease of at least 1e-6 of the cost, which an FP32
            # evaluation of the cost can tell apart from rounding (past that both solvers decide on noise)
            return sum(sum(1 for h in hh if not h["accepted"] and (not resolvable or h["pred"] >= 1e-6 * h["cost"]))
                       for hh in hist)

        def breakdowns(hist, only_rejected=False):  # PCG stopped by p^T A p <= 0 (or r^T z <= 0, non-finite)
            return sum(sum(1 for h in hh if h["pcg_status"] == "breakdown" and not (only_rejected and h["accepted"]))
                       for hh in hist)
        ttt_sc = [max(time_to_tol(h[i], f_taus[i][2]) for i in range(p.n_problems)) for _, h in sc["runs"]]
        ach_sc = sc["mv_bytes"] / (sc["mv_ms"] * 1e-3) / 1e9 if sc["mv_ms"] > 0 else None
        sc_out = {
            "landmark_blocks": "explicit Schur complement (FP32, assembled camera-pair blocks)",
            "time_to_1pct_cost_s": statistics.median(ttt_sc),
            "ms_per_step": 1e3 * sc["wall"] / args.steps,
            "final_costs": [sum(r.final_cost for r in reps) for reps, _ in sc["runs"]],
            "rejected_attempts": rejected(sc["runs"][-1][1]),
            "sqrt_ba_rejected_attempts": rejected(runs[-1][1]),
            "rejected_resolvable": rejected(sc["runs"][-1][1], True),
            "sqrt_ba_rejected_resolvable": rejected(runs[-1][1], True),
            "pcg_breakdowns": breakdowns(sc["runs"][-1][1]),
            "rejected_with_pcg_breakdown": breakdowns(sc["runs"][-1][1], True),
            "sqrt_ba_pcg_breakdowns": breakdowns(runs[-1][1]),
            "pcg_iters": sum(r.total_pcg_iters for r in sc["runs"][-1][0]),
            "workspace_bytes": sc["workspace_bytes"],
            "product": {"avg_launch_ms": sc["mv_ms"], "algorithmic_bytes_per_launch": sc["mv_bytes"],
                        "achieved_GBps": ach_sc, "frac_of_hbm_peak": ach_sc / HBM_PEAK_GBPS if ach_sc else None},
        }
    fp64_out = None
    if fp64 and "skipped" in fp64:
        fp64_out = {"skipped": fp64["skipped"]}
    elif fp64:
        ttt_64 = [max(time_to_tol(h[i], f_taus[i][2]) for i in range(p.n_problems)) for _, h in fp64["runs"]]
        ach_64 = fp64["mv_bytes"] / (fp64["mv_ms"] * 1e-3) / 1e9 if fp64["mv_ms"] > 0 else None
        fp64_out = {
            "landmark_blocks": args.blocks,
            "time_to_1pct_cost_s": statistics.median(ttt_64),
            "ms_per_step": 1e3 * fp64["wall"] / args.steps,
            "fp64_over_fp32_ms_per_step": fp64["wall"] / wall,
            "final_costs": [sum(r.final_cost for r in reps) for reps, _ in fp64["runs"]],
            "pcg_iters": sum(r.total_pcg_iters for r in fp64["runs"][-1][0]),
            "rejected_attempts": sum(sum(1 for x in hh if not x["accepted"]) for hh in fp64["runs"][-1][1]),
            "workspace_bytes": fp64["workspace_bytes"],
            "product": {"avg_launch_ms": fp64["mv_ms"], "algorithmic_bytes_per_launch": fp64["mv_bytes"],
                        "achieved_GBps": ach_64, "frac_of_hbm_peak": ach_64 / HBM_PEAK_GBPS if ach_64 else None,
                        "fp64_over_fp32_ms": fp64["mv_ms"] / mv_ms if mv_ms > 0 else None},
        }
    huber_out = None
    if huber:
        hgold = None
        if os.path.exists(GOLDEN_HUBER.format(cfg)) and p.n_problems == 1:
            with open(GOLDEN_HUBER.format(cfg)) as f:
                hgold = json.load(f)
        h_ttt = []
        for i in range(p.n_problems):
            r = huber["reports"][i]
            fstar = min([r.final_cost] + ([hgold["final_cost"]] if hgold else []))
            h_ttt.append(time_to_tol(huber["history"][i], fstar + 0.01 * (r.initial_cost - fstar)))
        huber_out = {
            "delta_px": HUBER_DELTA,
            "time_to_1pct_cost_s": max(h_ttt),
            "ms_per_solve": 1e3 * huber["wall_s"],
            "lm_attempts": max(r.iterations for r in huber["reports"]),
            "pcg_iters": sum(r.total_pcg_iters for r in huber["reports"]),
            "initial_cost": sum(r.initial_cost for r in huber["reports"]),
            "final_cost": sum(r.final_cost for r in huber["reports"]),
            "oracle_final_cost": hgold["final_cost"] if hgold else None,
        }
    learned_out = None
    if learned:
        l_ttt = max(time_to_tol(learned["history"][i], f_taus[i][2]) for i in range(p.n_problems))
        learned_out = {k: v for k, v in learned.items() if k not in ("reports", "history")}
        learned_out.update({
            "time_to_1pct_cost_s": l_ttt,
            "plain_time_to_1pct_cost_s": statistics.median(ttt),
            "pcg_iters": sum(r.total_pcg_iters for r in learned["reports"]),
            "plain_pcg_iters": sum(r.total_pcg_iters for r in runs[-1][0]),
            "final_cost": sum(r.final_cost for r in learned["reports"]),
            "plain_final_cost": sum(r.final_cost for r in runs[-1][0]),
        })
    value = statistics.median(ttt)
    f0, fstar, f_tau = f_taus[0]
    finals = [sum(r.final_cost for r in reps) for reps, _ in runs]

    qr = prof["marginalize"]
    achieved = mv_bytes / (mv_ms * 1e-3) / 1e9 if mv_ms > 0 else None
    traffic, traffic_note = None, None
    ptag = "_fp64" if args.precision == 64 else ""
    tfile = (os.path.join(ROOT, "profiles", f"matvec_traffic_{TRAFFIC_TAG[cfg]}_{args.blocks}{ptag}.json")
             if cfg in TRAFFIC_TAG else None)
    if tfile and os.path.exists(tfile):
        with open(tfile) as f:
            tr = json.load(f)
        if tr.get("kernels_sha") == kernels_hash():  # counters of the current kernels only
            traffic = tr.get("bytes_per_launch")
            cur = ",".join(str(v) for v in tuning["shape"].values())
            traffic_note = (f"FETCH_SIZE x {tr['fetch_scale']:.3f} + WRITE_SIZE x {tr['write_scale']:.3f} per product, "
                            f"counters taken with launch shapes {tr['shape']}"
                            + ("" if tr["shape"] in (cur, "x", "default") else f" (this run's shapes: {cur})"))
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBPS if achieved else None, "traffic": traffic,
                "kernel": (("the PCG product over all landmark blocks (k_matvec, plus k_matvec_large / "
                           "k_matvec_rows + k_matvec_combine where those size classes exist)")
                          if args.blocks == "explicit" else
                          "the PCG product over implicit blocks (k_matvec_implicit)" if args.blocks == "implicit" else
                          "the product with the assembled FP32 Schur complement (k_sc_matvec)")
                + (", FP64 build (libsqrtba64.so)" if args.precision == 64 else ""),
                "avg_launch_ms": mv_ms, "algorithmic_bytes_per_launch": mv_bytes, "launches_timed": 50,
                "timing": ("HIP events around a captured graph of 50 back-to-back products on the resident blocks "
                           "(the PCG iterations run as graphs too), context stream"),
                "traffic_source": traffic_note,
                "profiled_pass_matvec_ms": prof["matvec"]["ms"] / max(1, prof["matvec"]["launches"])}
    qr_blocks_per_s = qr["units"] / (qr["ms"] * 1e-3) if qr["ms"] > 0 else None
    qr_gbps = qr["bytes"] / (qr["ms"] * 1e-3) / 1e9 if qr["ms"] > 0 else None

    batch = None
    if p.n_problems > 1:
        solve_s = sorted(r.solve_seconds for reps, _ in runs for r in reps)
        batch = {"problems": p.n_problems, "problems_per_s": p.n_problems * len(runs) / wall,
                 "p50_solve_s": solve_s[len(solve_s) // 2], "p99_solve_s": solve_s[min(len(solve_s) - 1,
                                                                                      int(0.99 * len(solve_s)))]}
    rel_oracle = None
    if all(f is not None for f in oracle_finals):
        tot = sum(r.final_cost for r in runs[0][0])
        rel_oracle = {"total": abs(tot - sum(oracle_finals)) / sum(oracle_finals),
                      "max_per_problem": max(abs(r.final_cost - o) / o for r, o in zip(runs[0][0], oracle_finals))}
    cpu = None
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a bounded sample")
        try:
            cpu = cpu_baseline(p, cfg, f_taus, args.lm_iters)
        except Exception as e:  # the baseline is reported, never required
            log(f"cpu baseline failed: {e!r}")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == 64 else "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[cfg], "landmark_blocks": args.blocks, "n_problems": p.n_problems,
                   "n_cams": stats["n_cams"], "n_points": stats["n_points"], "n_obs": stats["n_obs"],
                   "bhat_bytes": stats["bhat_bytes"], "lm_iters": args.lm_iters, "pcg_tol": 1e-6,
                   "pcg_max_iters": 500},
        "time_to_1pct_cost_s": ttt,
        "upload_s": upload_s,
        "time_to_1pct_cost_incl_upload_s": value + upload_s,
        "f0": f0, "f_star": fstar, "f_tau": f_tau, "final_costs": finals,
        "oracle_final_cost": (sum(oracle_finals) if all(f is not None for f in oracle_finals) else None),
        "final_cost_rel_to_oracle": rel_oracle,
        "batch": batch,
        "qr_blocks_per_s": qr_blocks_per_s,
        "qr_GBps": qr_gbps,
        "matvec_GBps": achieved,
        "stage_ms": {k: v["ms"] for k, v in prof.items()},
        "roofline": roofline,
        "tuning": tuning,
        "forcing_sequence": forcing_out,
        "huber_loss": huber_out,
        "explicit_sc_comparator": sc_out,
        ("explicit_blocks" if blocks else "implicit_blocks"): other_out,
        "learned_vs_block_jacobi": learned_out,
        "sqrt_ba_64": fp64_out,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
