#!/usr/bin/env python3
"""Benchmark of the batched bi-level planner on one MI355X.

Workload: one plan at paper-like scale (Alg. 1 with its lower level):
N = 1000 behavioural samples, T = 100 instants over 5 s, M = 10 neighbours,
L = 5 upper iterations, K = 20 projection iterations, FP32, on a seeded
synthetic highway scene. One step = one whole plan (sampling, Step-1 QP,
projection, residual/cost, elite selection, distribution update for all 5
upper iterations) with its inputs already resident in HBM.

Metric: lower-level QP solves per second = N * L / plan time.

Prints one JSON line (see the keys below), including the roofline of the
dominant kernel (lower_kernel, its launches timed with HIP events on the
library's stream over a second timed region of the same steps) and the FP64
oracle timed on host cores on a sample of the same scene. Beside the headline (FP32) the line carries
  mixed     the same plan with the lower level on the matrix cores
            (PLAN_PREC_FP16_SPLIT),
            and its position difference to the FP32 lower level on 256
            inputs (the error of both against the FP64 oracle is stated
            by the parity tests),
  served    the served stream of 256 requests in both precisions: each
            one's saturated rate, then the same Poisson arrivals at 0.5, 0.7
            and 0.9 of the FP32 saturated rate (p50/p99 latency),
  scale     1024 concurrent requests of N = 4096, T = 100, M = 20 in both
            precisions,
  mpc       the receding-horizon closed loop (MPC-Bi-Level): 1 and 256
            episodes replanning every 5 instants on synthetic traffic, loop
            rate, QP-solves/s, collisions and average speed,
  decoder   the same plan with iteration 0 drawn by the decoder sampler
            (App. A decoder MLP, random weights), both precisions,
  behaviours  the same plan with goal-position inputs (both precisions),
            one iteration from the fixed grid (MPC-Grid), and on a curved
            road with a lane closure (both precisions).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "lower-level QP solves/sec at ≤1e-4 m error; p99 plan latency (served)"
CFG_ID = 2
PEAK_ALU_TFLOPS = 78.6  # FP32 FMA without packed math: 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz


# Decoder sampler per sample: algorithmic flops of the App. A decoder (FMA =
# 2): 57 -> 1024, three 1024 -> 1024, 1024 -> 256, 256 -> 8; and the flops the
# matrix cores execute for blocks 2-5 in the FP16-split form (3 products).
DECODER_FLOPS = 2 * (57 * 1024 + 3 * 1024 * 1024 + 1024 * 256 + 256 * 8)
DECODER_MFMA_FLOPS = 3 * 2 * (3 * 1024 * 1024 + 1024 * 256)


def lower_flops_per_sample(T: int, M: int, K: int) -> float:
    """Algorithmic FP32 operations of one lower-level solve (FMA = 2,
    other arithmetic and transcendental = 1): Step 1 through its affine map,
    K target passes and xi-updates of Alg. 2 in the free coordinates, and the
    residual/cost pass. Per instant of a target pass: trajectory evaluation
    (45 FMA + 6 adds), 8 per neighbour (distance test), ~40 for the
    velocity/acceleration polar step and clips, 3 for the lane, 45 FMA for
    the accumulation of N^T g; per xi-update 271 (+30 for the multiplier);
    residual pass 126 + 9 M per instant."""
    step1 = 15 * 12 * 2
    per_pass_instant = 96 + 8 * M + 40 + 3 + 90
    per_update = 271 + 30
    residual = T * (126 + 9 * M)
    return step1 + K * per_update + K * T * per_pass_instant + residual


def profiled_traffic():
    """HBM bytes per lower_kernel launch of this workload from the committed
    rocprofv3 summary (FETCH_SIZE and WRITE_SIZE passes, calibrated by a copy
    of known size), or None if the kernels have changed since it was taken."""
    import hashlib
    import re
    try:
        text = open(os.path.join(ROOT, "profiles", "lower_kernel_plan-N1000-T100-M10.md")).read()
        src = open(os.path.join(ROOT, "paper_2212_02224_amd", "csrc", "kernels.hip"), "rb").read()
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_launch: (\d+)\s+kernels\.hip sha256: ([0-9a-f]+)", text)
    if not m or not hashlib.sha256(src).hexdigest().startswith(m.group(2)):
        return None
    return float(m.group(1))


def cpu_baseline(scene, c, threads: int):
    import oracle
    oracle.build(force=False)
    oracle.set_threads(threads)
    par = oracle.default_params(T=c["T"], M=c["M"], K=c["K"], L=c["L"])
    sc = oracle.Scene(scene.ego, scene.obstacles)
    N = c["N"] if threads >= 4 else 250
    t0 = time.perf_counter()
    oracle.plan(par, sc, scene.seed, N)
    dt = time.perf_counter() - t0
    return {"value": N * c["L"] / dt, "unit": "QP-solves/s", "cores": threads, "kind": "oracle",
            "sample": f"one full plan of the same scene: N={N} L={c['L']} K={c['K']} T={c['T']} M={c['M']}, "
                      f"FP64, OpenMP over samples ({dt:.2f} s)"}


def served_stream(pl, workload, n_req: int, seed: int = 4):
    """The served workload: n_req requests with N in {256, 512, 1000, 2048},
    M in {4, 10, 20}, T in {50, 100} (seeded), on synthetic scenes."""
    reqs = []
    for i, (N, M, T) in enumerate(workload.served_mix(n_req, seed)):
        s = workload.scene(4, i, M)
        reqs.append(pl.Request(N=N, T=T, ego=s.ego, obstacles=s.obstacles, seed=s.seed, request_id=i))
    return reqs


def run_served(pl, h, reqs, arrivals):
    """Submit each request at its arrival time (seconds after start), drive
    plan_progress until all finish; returns (latencies, makespan). Python's
    cyclic garbage collector is paused meanwhile (a collection of the
    interpreter's heap takes tens of ms and would land in the timings)."""
    import gc
    gc.collect()
    gc.disable()
    try:
        return _run_served(pl, h, reqs, arrivals)
    finally:
        gc.enable()


def _run_served(pl, h, reqs, arrivals):
    import numpy as np
    order = np.argsort(arrivals, kind="stable")
    pending = {}
    lat = np.zeros(len(reqs))
    t0 = time.perf_counter()
    k = 0
    while k < len(order) or pending:
        now = time.perf_counter() - t0
        while k < len(order) and arrivals[order[k]] <= now:
            i = int(order[k])
            pending[pl.plan_submit(h, reqs[i])] = i
            k += 1
        if not pending:
            continue
        pl.plan_progress(h)
        for t in list(pending):
            r = pl.plan_poll(h, t)
            if r is not None:
                if r.status != 0:
                    raise RuntimeError(f"served request failed: {pl.plan_last_error(h)}")
                lat[pending.pop(t)] = r.latency_s
    return lat, time.perf_counter() - t0


def served_bench(pl, workload, torch, n_req=256, slots=64, loads=(0.5, 0.7, 0.9)):
    """The served stream in both precisions, each with the host waiting for
    every iteration (served_run_ahead 0, the default) and with one iteration
    enqueued ahead: the saturated rate of each (all requests at t = 0), then
    the same Poisson arrival sequences for all at the given fractions of the
    FP32 saturated rate; p50/p99 latency."""
    import numpy as np
    L, K = 5, 20
    reqs = served_stream(pl, workload, n_req)
    solves = sum(r.N for r in reqs) * L
    handles, out = {}, {}
    for name, prec, ahead in (("f32", 0, 0), ("fp16_split", 1, 0), ("f32_run_ahead1", 0, 1),
                              ("fp16_split_run_ahead1", 1, 1)):
        cfg = pl.plan_config_init(T_set=[50, 100], M_set=[4, 10, 20], proj_iters=K, upper_iters=L, max_N=2048,
                                  max_requests=slots, precision=prec, served_run_ahead=ahead)
        ws = torch.empty(pl.plan_workspace_bytes(cfg), dtype=torch.uint8, device="cuda:0")
        h = pl.plan_create(cfg, workspace=ws, stream=torch.cuda.current_stream().cuda_stream)
        run_served(pl, h, reqs[:16], np.zeros(16))  # warm-up
        _, sat_span = run_served(pl, h, reqs, np.zeros(n_req))
        handles[name] = h
        out[name] = {"saturated_requests_per_s": n_req / sat_span, "saturated_solves_per_s": solves / sat_span,
                     "poisson": {}}
    lam_ref = out["f32"]["saturated_requests_per_s"]
    for frac in loads:
        arrivals = np.cumsum(np.random.default_rng(11).exponential(1.0 / (frac * lam_ref), n_req))
        for name, h in handles.items():
            lat, span = run_served(pl, h, reqs, arrivals)
            out[name]["poisson"][f"{frac:.1f}"] = {
                "arrival_rate_per_s": frac * lam_ref, "p50_latency_ms": 1e3 * float(np.percentile(lat, 50)),
                "p99_latency_ms": 1e3 * float(np.percentile(lat, 99)), "solves_per_s": solves / span}
    for name in out:
        ref = out[name]["poisson"]["0.7"] if "0.7" in out[name]["poisson"] else {}
        out[name].update({"p50_latency_ms": ref.get("p50_latency_ms"), "p99_latency_ms": ref.get("p99_latency_ms")})
    out["stream"] = {"requests": n_req, "slots": slots, "L": L, "K": K,
                     "mix": "N in {256,512,1000,2048}, M in {4,10,20}, T in {50,100}",
                     "loads": "Poisson arrivals at the given fractions of the FP32 saturated request rate; "
                              "p50/p99 above at 0.7"}
    return out


def scale_bench(pl, workload, torch, precision=0, n_req=1024, N=4096, T=100, M=20):
    """n_req concurrent requests of one size, all admitted at once (the
    sample budget holds them all); makespan, solves/s, p50/p99 latency."""
    import numpy as np
    L, K = 5, 20
    cfg = pl.plan_config_init(T_set=[T], M_set=[M], proj_iters=K, upper_iters=L, max_N=N, max_requests=n_req,
                              precision=precision)
    ws = torch.empty(pl.plan_workspace_bytes(cfg), dtype=torch.uint8, device="cuda:0")
    h = pl.plan_create(cfg, workspace=ws, stream=torch.cuda.current_stream().cuda_stream)
    reqs = []
    for i in range(n_req):
        s = workload.scene(5, i, M)
        reqs.append(pl.Request(N=N, T=T, ego=s.ego, obstacles=s.obstacles, seed=s.seed, request_id=i))
    run_served(pl, h, reqs[:4], np.zeros(4))  # warm-up
    pl.plan_profile(h, True)
    lat, span = run_served(pl, h, reqs, np.zeros(n_req))
    ms, cnt = pl.plan_profile_read(h)
    pl.plan_profile(h, False)
    # the batched solve's roofline: every upper iteration's lower launches
    # over all 4.19M resident samples, HIP-event timed
    flop = n_req * N * lower_flops_per_sample(T, M, K)
    lower_s = 1e-3 * ms["lower"] / L
    achieved = flop / lower_s / 1e12
    return {"requests": n_req, "N": N, "T": T, "M": M, "L": L, "K": K, "solves_per_s": n_req * N * L / span,
            "makespan_s": span, "p50_latency_ms": 1e3 * float(np.percentile(lat, 50)),
            "p99_latency_ms": 1e3 * float(np.percentile(lat, 99)),
            "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / PEAK_ALU_TFLOPS, "lower_ms_per_iteration": 1e3 * lower_s,
                         "flop_per_iteration": flop}}


def mpc_bench(pl, workload, torch, precision=0, episodes=256, cycles=20, n_exec=5, c=None, init=0):
    """Receding-horizon closed loop (MPC-Bi-Level): `episodes` synthetic
    highway scenes replan every cycle with the headline planner settings,
    execute n_exec instants and replan, all on the device. Loop rate per
    episode, plans and QP-solves per second, the paper's two metrics
    (episodes with a collision; average speed of the collision-free ones,
    the mean of |v| over the cycle states)."""
    import numpy as np
    N, T, M, L, K = c["N"], c["T"], c["M"], c["L"], c["K"]
    cfg = pl.plan_config_init(T_set=[T], M_set=[M], proj_iters=K, upper_iters=L, max_N=N,
                              max_requests=episodes, precision=precision)
    ws = torch.empty(pl.plan_workspace_bytes(cfg), dtype=torch.uint8, device="cuda:0")
    h = pl.plan_create(cfg, workspace=ws, stream=torch.cuda.current_stream().cuda_stream)
    reqs = []
    for i in range(episodes):
        s = workload.scene(7, i, M)
        reqs.append(pl.Request(N=N, T=T, ego=s.ego, obstacles=s.obstacles, seed=s.seed, request_id=i,
                               session_id=1 + i))
    warm_up = [pl.Request(N=r.N, T=r.T, ego=r.ego, obstacles=r.obstacles, seed=r.seed, session_id=10 ** 6 + i)
            for i, r in enumerate(reqs[:4])]
    pl.plan_mpc_run(h, warm_up, 1, n_exec, init=init, log=())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res, log = pl.plan_mpc_run(h, reqs, cycles, n_exec, init=init, log=("ego", "collided", "status", "cost"))
    dt = time.perf_counter() - t0
    hit = log["collided"].any(axis=1)
    speed = np.hypot(log["ego"][:, :, 2], log["ego"][:, :, 3]).mean(axis=1)
    return {"init": ("sampler", "warm")[init], "episodes": episodes, "cycles": cycles, "n_exec": n_exec,
            "N": N, "T": T, "M": M, "L": L, "K": K,
            "seconds": dt, "loop_rate_hz": cycles / dt, "plans_per_s": episodes * cycles / dt,
            "solves_per_s": episodes * cycles * N * L / dt,
            "failed_plans": int((log["status"] != 0).sum()),
            "infeasible_plans": int((log["cost"][:, :, 1] > 0).sum()),
            "episodes_with_collision": int(hit.sum()),
            "collided_cycles": int(log["collided"].sum()),
            "avg_speed_collision_free_mps": float(speed[~hit].mean()) if (~hit).any() else None,
            "driven_s": cycles * n_exec * cfg.t_f / (T - 1)}


def precision_gap(pl, workload, c, n_samples=256):
    """Lower level of both precisions on the same n_samples behavioural
    inputs of the headline scene (seeded: lane offsets +- N(0, 0.3^2), speeds
    U[5, 25]): largest position difference between the two trajectories. The
    Bernstein basis is nonnegative and sums to one, so each axis differs by at
    most the largest coefficient difference; the bound is reported."""
    import numpy as np
    rng = np.random.default_rng(2024)
    s = workload.scene(CFG_ID, 0, c["M"])
    lane = rng.choice([-3.5, 0.0, 3.5], size=(n_samples, 1))
    p = np.hstack([lane + 0.3 * rng.standard_normal((n_samples, 4)), rng.uniform(5.0, 25.0, (n_samples, 4))])
    xs = {}
    for prec in (0, 1):
        cfg = pl.plan_config_init(T_set=[c["T"]], M_set=[c["M"]], proj_iters=c["K"], max_N=n_samples,
                                  max_requests=1, precision=prec)
        h = pl.plan_create(cfg)
        req = pl.Request(N=n_samples, T=c["T"], ego=s.ego, obstacles=s.obstacles, seed=s.seed)
        xs[prec] = pl.plan_lower_solve(h, req, p)[1]
    d = np.abs(xs[1] - xs[0])
    bound = np.sqrt(d[:, :11].max(axis=1) ** 2 + d[:, 11:].max(axis=1) ** 2)
    return {"samples": n_samples, "unit": "m", "max": float(bound.max()), "p99": float(np.percentile(bound, 99)),
            "definition": "bound on max over t of |position(fp16_split) - position(f32)|"}


def time_plan(pl, torch, c, scene, precision, steps, warmup, road=None, decoder=None, **cfg_over):
    """One staged plan launched warmup + steps times in an uninstrumented
    timed region (the throughput), then steps times with HIP events recorded
    by every dispatch (kernel durations; the events cost host time per
    launch, so this region is not used for the throughput). Returns (elapsed
    s of the first region, kernel ms dict of the second, launch counts,
    result). road: (profile, x0, dx) of a curved road, else the straight road;
    decoder: weights of the decoder sampler, which then draws iteration 0
    from the scene's observation."""
    N, T, M, L, K = c["N"], c["T"], c["M"], c["L"], c["K"]
    L = cfg_over.pop("upper_iters", L)
    if decoder is not None:
        cfg_over["sampler"] = pl.PLAN_SAMPLER_DECODER
    cfg = pl.plan_config_init(T_set=[T], M_set=[M], proj_iters=K, upper_iters=L, max_N=N, max_requests=1,
                              precision=precision, **cfg_over)
    ws = torch.empty(pl.plan_workspace_bytes(cfg), dtype=torch.uint8, device="cuda:0")
    stream = torch.cuda.current_stream()
    h = pl.plan_create(cfg, workspace=ws, stream=stream.cuda_stream)
    rk = {} if road is None else dict(road=road[0], road_x0=road[1], road_dx=road[2])
    if decoder is not None:
        from paper_2212_02224_amd import workload
        pl.plan_set_decoder(h, decoder)
        rk["observation"] = workload.observation(scene, *(() if road is None else road))
    req = pl.Request(N=N, T=T, ego=scene.ego, obstacles=scene.obstacles, seed=scene.seed, **rk)
    pl.plan_stage(h, [req])  # inputs into HBM before the timed region
    for _ in range(warmup):
        pl.plan_launch(h)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        pl.plan_launch(h)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    pl.plan_profile(h, True)
    torch.cuda.synchronize()
    for _ in range(steps):
        pl.plan_launch(h)
    torch.cuda.synchronize()
    ms, cnt = pl.plan_profile_read(h)
    pl.plan_profile(h, False)
    res = pl.plan_collect(h)[0]
    if res.status != 0:
        raise RuntimeError(f"plan failed: {pl.plan_last_error(h)}")
    return t1 - t0, ms, cnt, res


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-served", action="store_true", help="skip the served (Poisson) measurement")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP16-split plan and the accuracy check")
    ap.add_argument("--no-scale", action="store_true", help="skip the 1024-request measurement")
    ap.add_argument("--no-mpc", action="store_true", help="skip the receding-horizon closed loop")
    ap.add_argument("--no-decoder", action="store_true", help="skip the plan drawn by the decoder sampler")
    ap.add_argument("--no-behaviours", action="store_true",
                    help="skip the goal-position, fixed-grid (MPC-Grid) and curved-road plans")
    ap.add_argument("--copy-probe", action="store_true",
                    help="after the timed region, copy 512 MiB device-to-device three times (a "
                         "kernel of known traffic that calibrates FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): requests are independent, "
              "so more GPUs would each run their own share; no multi-GPU figure is produced.",
              file=sys.stderr)
        return 2

    import torch
    import paper_2212_02224_amd as pl
    from paper_2212_02224_amd import workload

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    c = workload.CONFIGS[CFG_ID]
    N, T, M, L, K = c["N"], c["T"], c["M"], c["L"], c["K"]
    scene = workload.scene(CFG_ID, 0, M)
    print(f"[bench] plan {c['name']} fp32: {args.warmup} warm-up + {args.steps} timed steps", file=sys.stderr,
          flush=True)
    elapsed, ms, cnt, res = time_plan(pl, torch, c, scene, 0, args.steps, args.warmup)
    ms_per_step = 1e3 * elapsed / args.steps
    value = N * L * args.steps / elapsed
    lower_avg_ms = ms["lower"] / max(1, cnt["lower"])
    flop = N * lower_flops_per_sample(T, M, K)
    achieved = flop / (lower_avg_ms * 1e-3) / 1e12
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "QP-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": c["name"] + f"-L{L}-K{K}", "N": N, "T": T, "M": M, "L": L, "K": K,
                   "requests_per_step": 1},
        "roofline": {"bound": "alu", "kernel": "lower_kernel", "achieved": achieved,
                     "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_ALU_TFLOPS,
                     "traffic": profiled_traffic(), "traffic_unit": "bytes per launch",
                     "avg_ms": lower_avg_ms, "flop_per_launch": flop,
                     "launches": cnt["lower"]},
        "kernel_ms_per_step": {k: ms[k] / args.steps for k in ms},
        "plan": {"best_index": res.best_index, "cost_upper": res.cost_upper, "residual": res.residual},
    }
    if not args.no_mixed:
        print("[bench] plan fp16_split", file=sys.stderr, flush=True)
        el2, ms2, cnt2, res2 = time_plan(pl, torch, c, scene, 1, args.steps, args.warmup)
        avg2 = ms2["lower"] / max(1, cnt2["lower"])
        out["mixed"] = {"precision": "fp16_split", "value": N * L * args.steps / el2, "unit": "QP-solves/s",
                        "ms_per_step": 1e3 * el2 / args.steps, "kernel": "lower_mfma_kernel",
                        "lower_avg_ms": avg2, "achieved_alg_tflops": flop / (avg2 * 1e-3) / 1e12,
                        "kernel_ms_per_step": {k: ms2[k] / args.steps for k in ms2},
                        "plan": {"best_index": res2.best_index, "cost_upper": res2.cost_upper}}
        out["mixed"]["gap_to_f32"] = precision_gap(pl, workload, c)
    if not args.no_behaviours:
        # the other behavioural inputs of eq. behaviour_param on the same scene
        # and on a curved road (curvature and lane limits along x)
        out["behaviours"] = {}
        curve = workload.curved_road(CFG_ID, 0)
        for name, prec, over, Lb, rd in (("goals_f32", 0, dict(behaviour=pl.PLAN_BEHAV_GOALS), L, None),
                                         ("goals_fp16_split", 1, dict(behaviour=pl.PLAN_BEHAV_GOALS), L, None),
                                         ("grid_f32_L1", 0, dict(sampler=pl.PLAN_SAMPLER_GRID), 1, None),
                                         ("grid_goals_f32_L1", 0, dict(sampler=pl.PLAN_SAMPLER_GRID,
                                                                       behaviour=pl.PLAN_BEHAV_GOALS), 1, None),
                                         ("curved_road_f32", 0, {}, L, curve),
                                         ("curved_road_fp16_split", 1, {}, L, curve)):
            print(f"[bench] plan {name}", file=sys.stderr, flush=True)
            elb, msb, cntb, resb = time_plan(pl, torch, c, scene, prec, args.steps, args.warmup, road=rd,
                                             upper_iters=Lb, **over)
            out["behaviours"][name] = {"value": N * Lb * args.steps / elb, "unit": "QP-solves/s",
                                       "ms_per_plan": 1e3 * elb / args.steps, "L": Lb,
                                       "lower_avg_ms": msb["lower"] / max(1, cntb["lower"]),
                                       "plan": {"best_index": resb.best_index, "p_best": list(resb.p_best[:2]),
                                                "cost_upper": resb.cost_upper, "residual": resb.residual}}
    if args.copy_probe:
        src = torch.empty(512 << 20, dtype=torch.uint8, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
    if not args.no_served:
        print("[bench] served stream, both precisions", file=sys.stderr, flush=True)
        out["served"] = served_bench(pl, workload, torch)
    if not args.no_scale:
        out["scale"] = {}
        for name, prec in (("f32", 0), ("fp16_split", 1)):
            print(f"[bench] 1024 concurrent requests {name}", file=sys.stderr, flush=True)
            out["scale"][name] = scale_bench(pl, workload, torch, prec)
    if not args.no_mpc:
        out["mpc"] = {}
        for name, prec, eps, cyc, init in (("f32_1", 0, 1, 200, 0), ("f32_256", 0, 256, 20, 0),
                                           ("fp16_split_256", 1, 256, 20, 0), ("f32_256_warm", 0, 256, 20, 1)):
            print(f"[bench] closed loop {name}: {eps} episodes x {cyc} cycles", file=sys.stderr, flush=True)
            out["mpc"][name] = mpc_bench(pl, workload, torch, prec, eps, cyc, c=c, init=init)
    if not args.no_decoder:
        # the decoder sampler (App. A decoder MLP, random weights) drawing
        # iteration 0 of the headline plan
        out["decoder"] = {}
        dec = workload.decoder_weights(0)
        for name, prec in (("f32", 0), ("fp16_split", 1)):
            print(f"[bench] plan from the decoder sampler, {name}", file=sys.stderr, flush=True)
            eld, msd, cntd, resd = time_plan(pl, torch, c, scene, prec, args.steps, args.warmup, decoder=dec)
            dms = msd["decoder"] / max(1, cntd["decoder"])
            out["decoder"][name] = {
                "value": N * L * args.steps / eld, "unit": "QP-solves/s", "ms_per_plan": 1e3 * eld / args.steps,
                "decoder_ms_per_plan": dms, "lower_avg_ms": msd["lower"] / max(1, cntd["lower"]),
                "decoder_alg_tflops": N * DECODER_FLOPS / (dms * 1e-3) / 1e12,
                "decoder_mfma_frac": N * DECODER_MFMA_FLOPS / (dms * 1e-3) / 2.5e15,
                "plan": {"best_index": resd.best_index, "cost_upper": resd.cost_upper, "residual": resd.residual}}
    if not args.no_cpu_baseline:
        threads = min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(scene, c, threads)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
