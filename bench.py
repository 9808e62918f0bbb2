#!/usr/bin/env python3
"""Benchmark of the batched bi-level planner on one MI355X.

Headline workload: 1024 planning requests solved together, each N = 4096
behavioural samples, T = 100 instants over 5 s, M = 20 neighbours, L = 5
upper iterations, K = 20 projection iterations, FP32, on seeded synthetic
highway scenes (the largest configuration that fits one GPU). One step = the
whole hot path for all 1024 requests (sampling, Step-1 QP, projection,
residual/cost, elite selection, distribution update for all 5 upper
iterations) with the inputs already resident in HBM.

Metric: lower-level QP solves per second = requests * N * L / step time.

Prints one JSON line (see the keys below), including the roofline of the
dominant kernel (lower_kernel, its launches timed with HIP events on the
library's stream over a second timed region of the same steps) and the FP64
oracle timed on the host cores the process may use. Beside the headline the
line carries
  c2_plan   one plan of N = 1000, T = 100, M = 10 (the single-request
            latency case) in FP32, with its own roofline,
  mixed     that plan with the lower level on the matrix cores
            (PLAN_PREC_FP16_SPLIT), and the headline batch in that form,
  served    the served stream of 256 requests in both precisions: each
            one's saturated rate, then the same Poisson arrivals at 0.5, 0.7
            and 0.9 of the FP32 saturated rate (p50/p99 latency),
  scale     the headline's 1024 requests admitted through the served path,
            both precisions, with p50/p99 latency,
  mpc       the receding-horizon closed loop (MPC-Bi-Level): 1 and 256
            episodes replanning every 5 instants on synthetic traffic, loop
            rate, QP-solves/s, collisions and average speed,
  decoder   the C2 plan with iteration 0 drawn by the decoder sampler
            (App. A decoder MLP, random weights), both precisions,
  behaviours  the C2 plan with goal-position inputs (both precisions),
            one iteration from the fixed grid (MPC-Grid), and on a curved
            road with a lane closure (both precisions),
  accuracy_vs_oracle  (with the oracle leg) position error of the lower
            level of each precision against the FP64 oracle on the same
            samples of headline scenes.
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
CFG_ID = 5       # headline: 1024 concurrent requests of N = 4096, T = 100, M = 20
PLAN_CFG_ID = 2  # single plan: N = 1000, T = 100, M = 10
HEADLINE_REQUESTS = 1024
# FP32 form of the headline: 0 = PLAN_PREC_FP32 (every product on the vector
# ALUs), 2 = PLAN_PREC_FP32_MFMA (the dense products on the matrix cores in
# FP32); both FP32 throughout and held to the same parity bar
HEADLINE_PRECISION = 0
PRECISION_NAMES = {0: "fp32_valu", 1: "fp16_split", 2: "fp32_mfma"}
# the lower kernel of each form (as rocprofv3 names it at the headline's
# shape) and the key of its committed profile
KERNEL_NAMES = {0: "lower_kernel<2, false>", 1: "lower_mfma_kernel<4, false, false>",
                2: "lower_mfma_kernel<4, false, true>"}
PROFILE_KEYS = {0: "lower_kernel", 1: "lower_mfma_kernel-fp16_split", 2: "lower_mfma_kernel-fp32"}
PEAK_FP32_TFLOPS = 157.3  # MI355X published FP32 vector peak (needs packed FP32)
# FP32 FMA without packed math, the rate every kernel here is built for:
# 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
PEAK_ALU_TFLOPS = 78.6


# Decoder sampler per sample: algorithmic flops of the App. A decoder (FMA =
# 2): 57 -> 1024, three 1024 -> 1024, 1024 -> 256, 256 -> 8; and the flops the
# matrix cores execute for blocks 2-5 in the FP16-split form (3 products).
DECODER_FLOPS = 2 * (57 * 1024 + 3 * 1024 * 1024 + 1024 * 256 + 256 * 8)
DECODER_MFMA_FLOPS = 3 * 2 * (3 * 1024 * 1024 + 1024 * 256)


def alg_work_per_solve(T: int, M: int, K: int) -> dict:
    """Algorithmic work of one lower-level solve (Step 1 and K iterations of
    Alg. 2 with the residual/cost pass), counted from the method: FMA = 2
    flop, every other arithmetic operation and every transcendental 1.
      dense          the shared-matrix products per iteration: evaluation
                     [W; Wd; Wdd] xi and the transposed accumulation, 3T x 11
                     per axis each, and the 11 x 11 xi-update per axis,
                     2 (132 T + 484) flop;
      elementwise    per instant and iteration about 9 operations per
                     neighbour (distance and target) and 40 for the
                     velocity/acceleration polar step, clips and lane slack;
                     the residual/cost pass about 5 per neighbour + 15;
      transcendental per instant and iteration one per neighbour (the
                     rsqrt of the closed-form projection) and 6 for the
                     polar step."""
    dense = 2.0 * K * (132 * T + 484)
    elem = float(K * T * (9 * M + 40) + T * (5 * M + 15))
    transc = float(K * T * (M + 6))
    return {"dense": dense, "elementwise": elem, "transcendental": transc, "total": dense + elem + transc}


def profiled_traffic(kernel: str, workload_name: str):
    """HBM bytes per launch of `kernel` on this workload from the committed
    rocprofv3 summary (FETCH_SIZE and WRITE_SIZE passes, calibrated by a copy
    of known size), or None if the kernels have changed since it was taken."""
    import hashlib
    import re
    try:
        text = open(os.path.join(ROOT, "profiles", f"{kernel}_{workload_name}.md")).read()
        src = open(os.path.join(ROOT, "paper_2212_02224_amd", "csrc", "kernels.hip"), "rb").read()
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_launch: (\d+)\s+kernels\.hip sha256: ([0-9a-f]+)", text)
    if not m or not hashlib.sha256(src).hexdigest().startswith(m.group(2)):
        return None
    return float(m.group(1))


def host_cpus():
    """(threads granted to this process, nproc, CPU model), read at run time.
    The threads used are the process's CPU affinity, capped by
    OMP_NUM_THREADS when the machine sets it (its share of a shared host)."""
    affinity = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS", "")
    threads = min(affinity, int(omp)) if omp.isdigit() and int(omp) > 0 else affinity
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return threads, os.cpu_count(), model


def cpu_baseline_leg(pl, workload, n_sub=8, acc_scenes=2, acc_samples=512):
    """The FP64 oracle on the host cores (the CPU baseline), and the error of
    each GPU precision's lower level against it.

    Baseline (value): the headline workload's first upper iteration for the
    first n_sub of its 1024 requests (each N = 4096: sampling, Step 1, K = 20
    projection iterations, residual/cost, selection and update), OpenMP over
    samples on every granted thread; QP-solves/s, and the whole job's time
    extrapolated from it. Beside it: a single-thread figure (one C2 plan of
    250 samples, per-solve rate and the C2 plan time extrapolated to
    N = 1000), one whole C2 plan on every thread, one C1 plan single
    threaded, and the served stream (C4) from the first upper iteration of
    one request per (N, T) pair of its mix on every thread, extrapolated.

    Accuracy: the oracle's samples of acc_scenes headline scenes (its own
    draw, acc_samples each) through the oracle's lower level and through
    plan_lower_solve in each precision; per trajectory the largest position
    difference over the horizon (both evaluated in FP64 from the returned
    coefficients)."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    threads, nproc, model = host_cpus()
    out = {}
    c5 = workload.CONFIGS[CFG_ID]
    oracle.set_threads(threads)
    par5 = oracle.default_params(T=c5["T"], M=c5["M"], K=c5["K"], L=1)
    t0 = time.perf_counter()
    for i in range(n_sub):
        s = workload.scene(CFG_ID, i, c5["M"])
        oracle.plan(par5, oracle.Scene(s.ego, s.obstacles), s.seed, c5["N"])
    dt = time.perf_counter() - t0
    rate = n_sub * c5["N"] / dt
    job = HEADLINE_REQUESTS * c5["N"] * c5["L"]
    out["cpu_baseline"] = {
        "value": rate, "unit": "QP-solves/s", "cores": threads, "kind": "oracle",
        "sample": f"first upper iteration of {n_sub} of the headline's {HEADLINE_REQUESTS} requests "
                  f"(N={c5['N']} T={c5['T']} M={c5['M']} K={c5['K']}, FP64, OpenMP over samples, {dt:.1f} s); "
                  f"whole job extrapolated: {job / rate:.0f} s",
        "nproc": nproc, "cpu_model": model, "extrapolated_job_s": job / rate}
    c2, c1 = workload.CONFIGS[PLAN_CFG_ID], workload.CONFIGS[1]
    s2 = workload.scene(PLAN_CFG_ID, 0, c2["M"])
    par2 = oracle.default_params(T=c2["T"], M=c2["M"], K=c2["K"], L=c2["L"])
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.plan(par2, oracle.Scene(s2.ego, s2.obstacles), s2.seed, 250)
    dt1 = time.perf_counter() - t0
    s1 = workload.scene(1, 0, c1["M"])
    par1 = oracle.default_params(T=c1["T"], M=c1["M"], K=c1["K"], L=c1["L"])
    t0 = time.perf_counter()
    oracle.plan(par1, oracle.Scene(s1.ego, s1.obstacles), s1.seed, c1["N"])
    dtc1 = time.perf_counter() - t0
    oracle.set_threads(threads)
    t0 = time.perf_counter()
    oracle.plan(par2, oracle.Scene(s2.ego, s2.obstacles), s2.seed, c2["N"])
    dt2 = time.perf_counter() - t0
    out["cpu_baseline"]["single_thread"] = {
        "c2_solves_per_s": 250 * c2["L"] / dt1, "c2_plan_s_extrapolated": dt1 * c2["N"] / 250,
        "c1_plan_s": dtc1, "sample": "one C2 plan of 250 samples (L=5, K=20, T=100, M=10) and one C1 plan "
                                     "(N=64, L=3, K=10, T=50, M=4), one thread"}
    out["cpu_baseline"]["c2_plan_all_threads"] = {"solves_per_s": c2["N"] * c2["L"] / dt2, "plan_s": dt2}
    # C4, the served stream: the first upper iteration of one request for
    # each (N, T) of the stream's mix (its first request with that pair, so
    # its own M and scene), every thread; the stream's oracle time (L upper
    # iterations of every request) extrapolated by its solve count
    mix = workload.served_mix(SERVED_REQUESTS, SERVED_SEED)
    picked = {}
    for i, (N, M, T) in enumerate(mix):
        picked.setdefault((N, T), (i, N, M, T))
    t0 = time.perf_counter()
    sub = 0
    for i, N, M, T in sorted(picked.values()):
        s = workload.scene(4, i, M)
        oracle.plan(oracle.default_params(T=T, M=M, K=SERVED_K, L=1), oracle.Scene(s.ego, s.obstacles), s.seed, N)
        sub += N
    dt4 = time.perf_counter() - t0
    total4 = sum(N for N, _, _ in mix) * SERVED_L
    out["cpu_baseline"]["c4_stream_all_threads"] = {
        "solves_per_s": sub / dt4, "subset_s": dt4, "stream_s_extrapolated": total4 * dt4 / sub,
        "sample": f"first upper iteration of {len(picked)} of the served stream's {SERVED_REQUESTS} requests, "
                  f"one per (N, T) pair (K={SERVED_K}, M and scene their own, {sub} solves, {dt4:.1f} s); "
                  f"the stream's {total4} solves (L={SERVED_L}) extrapolated"}
    # accuracy of each GPU precision against the oracle, teacher-forced
    acc = {}
    for prec, name in ((pl.PLAN_PREC_FP32, "fp32_valu"), (pl.PLAN_PREC_FP32_MFMA, "fp32_mfma"),
                       (pl.PLAN_PREC_FP16_SPLIT, "fp16_split")):
        cfg = pl.plan_config_init(T_set=[c5["T"]], M_set=[c5["M"]], proj_iters=c5["K"], max_N=acc_samples,
                                  max_requests=1, precision=prec)
        h = pl.plan_create(cfg)
        errs = []
        for i in range(acc_scenes):
            s = workload.scene(CFG_ID, i, c5["M"])
            sc = oracle.Scene(s.ego, s.obstacles)
            p = oracle.sample(par5, s.seed, 0, acc_samples, True)
            xs_o = oracle.project(par5, sc, oracle.step1(par5, sc, p))
            req = pl.Request(N=acc_samples, T=c5["T"], ego=s.ego, obstacles=s.obstacles, seed=s.seed)
            xs_g = pl.plan_lower_solve(h, req, p)[1]
            W = oracle.basis(c5["T"], par5.t_f)[0]
            d = np.hypot((xs_g[:, :11] - xs_o[:, :11]) @ W.T, (xs_g[:, 11:] - xs_o[:, 11:]) @ W.T)
            errs.append(d.max(axis=1))
        pl.plan_destroy(h)
        e = np.concatenate(errs)
        acc[name] = {"max_m": float(e.max()), "p99_m": float(np.percentile(e, 99)),
                     "median_m": float(np.median(e)), "trajectories": int(e.size)}
    out["accuracy_vs_oracle"] = dict(acc, definition=(
        "per trajectory max over t_k of |(x, y)_gpu - (x, y)_oracle| (m), the oracle's own samples of "
        f"{acc_scenes} headline scenes (first iteration's draw) through both lower levels"))
    return out


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
        for t, r in pl.plan_poll_done(h, len(pending)):
            if r.status != 0:
                raise RuntimeError(f"served request failed: {pl.plan_last_error(h)}")
            lat[pending.pop(t)] = r.latency_s
    return lat, time.perf_counter() - t0


SERVED_REQUESTS, SERVED_SEED, SERVED_L, SERVED_K = 256, 4, 5, 20


def served_bench(pl, workload, torch, n_req=SERVED_REQUESTS, slots=64, loads=(0.5, 0.7, 0.9)):
    """The served stream in the FP32 and FP16-split forms, each with the host
    waiting for every iteration (served_run_ahead 0, the default) and with one
    iteration enqueued ahead, and in the FP32 matrix-core form: the saturated rate of each (all requests at t = 0), then
    the same Poisson arrival sequences for all at the given fractions of the
    FP32 saturated rate; p50/p99 latency."""
    import numpy as np
    L, K = SERVED_L, SERVED_K
    reqs = served_stream(pl, workload, n_req, SERVED_SEED)
    solves = sum(r.N for r in reqs) * L
    handles, out = {}, {}
    for name, prec, ahead in (("f32", 0, 0), ("fp16_split", 1, 0), ("fp32_mfma", 2, 0), ("f32_run_ahead1", 0, 1),
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
    # every upper iteration's lower launches over all 4.19M resident
    # samples, HIP-event timed
    flop = n_req * N * alg_work_per_solve(T, M, K)["total"]
    lower_s = 1e-3 * ms["lower"] / L
    achieved = flop / lower_s / 1e12
    return {"requests": n_req, "N": N, "T": T, "M": M, "L": L, "K": K, "solves_per_s": n_req * N * L / span,
            "makespan_s": span, "p50_latency_ms": 1e3 * float(np.percentile(lat, 50)),
            "p99_latency_ms": 1e3 * float(np.percentile(lat, 99)),
            "lower_ms_per_iteration": 1e3 * lower_s, "achieved_alg_tflops": achieved,
            "frac_of_157": achieved / PEAK_FP32_TFLOPS}


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


def time_batch(pl, torch, reqs, c, precision, steps, warmup):
    """The requests staged together (inputs in HBM), the whole hot path of
    all of them launched warmup + steps times in an uninstrumented timed
    region, then steps times with HIP events recorded by every dispatch
    (kernel durations). Returns (elapsed s of the first region, kernel ms,
    launch counts, results)."""
    T, M, L, K = c["T"], c["M"], c["L"], c["K"]
    cfg = pl.plan_config_init(T_set=[T], M_set=[M], proj_iters=K, upper_iters=L, max_N=max(r.N for r in reqs),
                              max_requests=len(reqs), precision=precision)
    ws = torch.empty(pl.plan_workspace_bytes(cfg), dtype=torch.uint8, device="cuda:0")
    h = pl.plan_create(cfg, workspace=ws, stream=torch.cuda.current_stream().cuda_stream)
    pl.plan_stage(h, reqs)
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
    res = pl.plan_collect(h)
    bad = [i for i, r in enumerate(res) if r.status != 0]
    if bad:
        raise RuntimeError(f"request {bad[0]} failed: {pl.plan_last_error(h)}")
    pl.plan_destroy(h)
    del ws
    return t1 - t0, ms, cnt, res


def roofline(prec, avg_ms, solves_per_launch, T, M, K, launches, workload_name, kernel=None):
    """Roofline entry of the lower-level kernel of precision form `prec`:
    algorithmic work per launch over its HIP-event duration, against the
    published FP32 vector peak and the FP32 rate without packed math."""
    w = alg_work_per_solve(T, M, K)
    flop = w["total"] * solves_per_launch
    achieved = flop / (avg_ms * 1e-3) / 1e12
    return {"bound": "alu", "kernel": kernel or KERNEL_NAMES[prec], "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
            "traffic": profiled_traffic(PROFILE_KEYS[prec], workload_name), "traffic_unit": "bytes per launch",
            "peak_non_packed": PEAK_ALU_TFLOPS, "frac_non_packed": achieved / PEAK_ALU_TFLOPS,
            "avg_ms": avg_ms, "launches": launches, "solves_per_launch": solves_per_launch,
            "work_per_solve": w, "work_per_launch": flop}


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


def copy_probe(torch):
    """Three device-to-device copies of 512 MiB: a kernel of known traffic
    that calibrates the FETCH_SIZE / WRITE_SIZE counters."""
    src = torch.empty(512 << 20, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()


def decoder_legs(pl, torch, workload, c, scene, steps, warmup):
    """The single plan with iteration 0 drawn by the decoder sampler (App. A
    decoder MLP, random weights of the paper's sizes), FP32 and FP16 split."""
    N, L = c["N"], c["L"]
    res = {}
    dec = workload.decoder_weights(0)
    for name, prec in (("f32", 0), ("fp16_split", 1)):
        print(f"[bench] plan from the decoder sampler, {name}", file=sys.stderr, flush=True)
        eld, msd, cntd, resd = time_plan(pl, torch, c, scene, prec, steps, warmup, decoder=dec)
        dms = msd["decoder"] / max(1, cntd["decoder"])
        res[name] = {
            "value": N * L * steps / eld, "unit": "QP-solves/s", "ms_per_plan": 1e3 * eld / steps,
            "decoder_ms_per_plan": dms, "lower_avg_ms": msd["lower"] / max(1, cntd["lower"]),
            "decoder_alg_tflops": N * DECODER_FLOPS / (dms * 1e-3) / 1e12,
            "decoder_mfma_frac": N * DECODER_MFMA_FLOPS / (dms * 1e-3) / 2.5e15,
            "plan": {"best_index": resd.best_index, "cost_upper": resd.cost_upper, "residual": resd.residual}}
    return res


def plan_legs(pl, torch, workload, c, args, out):
    """The single plan (the latency case) in FP32 and, unless --no-mixed, in
    the FP16 split, into out["c2_plan"] and out["mixed"]["c3_plan"]; returns
    the (steps, warm-up) it used."""
    N, T, M, L, K = c["N"], c["T"], c["M"], c["L"], c["K"]
    scene = workload.scene(PLAN_CFG_ID, 0, M)
    psteps, pwarm = max(args.steps, 50), max(args.warmup, 10)
    print(f"[bench] plan {c['name']} fp32: {pwarm} warm-up + {psteps} timed steps", file=sys.stderr, flush=True)
    el2, ms2, cnt2, res = time_plan(pl, torch, c, scene, 0, psteps, pwarm)
    out["c2_plan"] = {
        "workload": c["name"] + f"-L{L}-K{K}", "value": N * L * psteps / el2, "unit": "QP-solves/s",
        "ms_per_plan": 1e3 * el2 / psteps,
        "roofline": roofline(0, ms2["lower"] / max(1, cnt2["lower"]), N, T, M, K, cnt2["lower"], c["name"],
                             kernel="lower_kernel<1, false>"),
        "kernel_ms_per_step": {k: ms2[k] / psteps for k in ms2},
        "plan": {"best_index": res.best_index, "cost_upper": res.cost_upper, "residual": res.residual}}
    if not args.no_mixed:
        print("[bench] plan fp16_split", file=sys.stderr, flush=True)
        el3, ms3, cnt3, res3 = time_plan(pl, torch, c, scene, 1, psteps, pwarm)
        out["mixed"]["c3_plan"] = {
            "precision": "fp16_split", "value": N * L * psteps / el3, "unit": "QP-solves/s",
            "ms_per_plan": 1e3 * el3 / psteps,
            "roofline": roofline(1, ms3["lower"] / max(1, cnt3["lower"]), N, T, M, K, cnt3["lower"], c["name"],
                                 kernel="lower_mfma_kernel<1, false, false>"),
            "kernel_ms_per_step": {k: ms3[k] / psteps for k in ms3},
            "plan": {"best_index": res3.best_index, "cost_upper": res3.cost_upper, "residual": res3.residual}}
    return psteps, pwarm


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
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
    ap.add_argument("--precision", type=int, default=HEADLINE_PRECISION, choices=sorted(PRECISION_NAMES),
                    help="form of the headline batch (0 FP32 on the vector ALUs, 1 FP16 split, 2 FP32 on the "
                         "matrix cores); the default is the headline's")
    ap.add_argument("--plan-only", action="store_true",
                    help="only the single plan of N = 1000, T = 100, M = 10 in FP32 and, unless --no-mixed, in the "
                         "FP16 split (e.g. under a profiler); prints those entries alone")
    ap.add_argument("--decoder-only", action="store_true",
                    help="only the single plan drawn by the decoder sampler, FP32 then FP16 split (e.g. under a "
                         "profiler); prints that entry alone")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the headline batch (e.g. under a profiler: every lower_kernel launch is then "
                         "the headline's)")
    args = ap.parse_args()
    if args.headline_only:
        args.no_cpu_baseline = args.no_served = args.no_mixed = args.no_scale = True
        args.no_mpc = args.no_decoder = args.no_behaviours = True
    if args.plan_only:
        args.no_cpu_baseline = args.no_served = args.no_scale = True
        args.no_mpc = args.no_decoder = args.no_behaviours = True
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
    if args.decoder_only:
        c = workload.CONFIGS[PLAN_CFG_ID]
        out = {"decoder": decoder_legs(pl, torch, workload, c, workload.scene(PLAN_CFG_ID, 0, c["M"]),
                                       max(args.steps, 50), max(args.warmup, 10))}
        if args.copy_probe:
            copy_probe(torch)
        print(json.dumps(out), flush=True)
        return 0
    if args.plan_only:
        out = {"mixed": {}}
        c = workload.CONFIGS[PLAN_CFG_ID]
        plan_legs(pl, torch, workload, c, args, out)
        if args.copy_probe:
            copy_probe(torch)
        print(json.dumps(out), flush=True)
        return 0
    c5 = workload.CONFIGS[CFG_ID]
    N5, T5, M5, L5, K5 = c5["N"], c5["T"], c5["M"], c5["L"], c5["K"]
    wl5 = f"batch-{HEADLINE_REQUESTS}xN{N5}-T{T5}-M{M5}"
    reqs5 = []
    for i in range(HEADLINE_REQUESTS):
        s5 = workload.scene(CFG_ID, i, M5)
        reqs5.append(pl.Request(N=N5, T=T5, ego=s5.ego, obstacles=s5.obstacles, seed=s5.seed, request_id=i))
    hp = args.precision
    print(f"[bench] headline {wl5} {PRECISION_NAMES[hp]}: {args.warmup} warm-up + {args.steps} timed steps",
          file=sys.stderr, flush=True)
    elapsed, ms, cnt, res5 = time_batch(pl, torch, reqs5, c5, hp, args.steps, args.warmup)
    solves = HEADLINE_REQUESTS * N5 * L5
    out = {
        "metric": METRIC,
        "value": solves * args.steps / elapsed,
        "unit": "QP-solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{wl5}-L{L5}-K{K5}", "requests": HEADLINE_REQUESTS, "N": N5, "T": T5, "M": M5,
                   "L": L5, "K": K5, "precision": PRECISION_NAMES[hp]},
        "roofline": roofline(hp, ms["lower"] / max(1, cnt["lower"]), HEADLINE_REQUESTS * N5, T5, M5, K5,
                             cnt["lower"], wl5),
        "kernel_ms_per_step": {k: ms[k] / args.steps for k in ms},
        "infeasible_results": int(sum(1 for r in res5 if r.flags & pl.PLAN_F_INFEASIBLE)),
    }
    if not args.no_mixed:
        # the headline batch in the other forms: the other FP32 form and the
        # FP16 split (reduced precision)
        out["forms"] = {}
        for prec in (0, 2, 1):
            if prec == hp:
                continue
            name = PRECISION_NAMES[prec]
            print(f"[bench] headline {wl5} {name}", file=sys.stderr, flush=True)
            el5m, ms5m, cnt5m, _ = time_batch(pl, torch, reqs5, c5, prec, args.steps, args.warmup)
            out["forms"][name] = {
                "value": solves * args.steps / el5m, "unit": "QP-solves/s", "ms_per_step": 1e3 * el5m / args.steps,
                "roofline": roofline(prec, ms5m["lower"] / max(1, cnt5m["lower"]), HEADLINE_REQUESTS * N5, T5, M5,
                                     K5, cnt5m["lower"], wl5),
                "kernel_ms_per_step": {k: ms5m[k] / args.steps for k in ms5m}}
        out["mixed"] = {}
    del reqs5, res5
    if args.copy_probe:
        copy_probe(torch)
    if args.headline_only:
        print(json.dumps(out), flush=True)
        return 0

    # the single plan (latency case)
    c = workload.CONFIGS[PLAN_CFG_ID]
    N, T, M, L, K = c["N"], c["T"], c["M"], c["L"], c["K"]
    scene = workload.scene(PLAN_CFG_ID, 0, M)
    psteps, pwarm = plan_legs(pl, torch, workload, c, args, out)
    args.steps, args.warmup = psteps, pwarm  # the C2-based legs below
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
    if not args.no_served:
        print("[bench] served stream, both precisions", file=sys.stderr, flush=True)
        out["served"] = served_bench(pl, workload, torch)
    if not args.no_scale:
        out["scale"] = {}
        for name, prec in (("f32", 0), ("fp32_mfma", 2), ("fp16_split", 1)):
            print(f"[bench] 1024 concurrent requests {name}", file=sys.stderr, flush=True)
            out["scale"][name] = scale_bench(pl, workload, torch, prec)
    if not args.no_mpc:
        out["mpc"] = {}
        for name, prec, eps, cyc, init in (("f32_1", 0, 1, 200, 0), ("f32_256", 0, 256, 20, 0),
                                           ("fp16_split_256", 1, 256, 20, 0), ("f32_256_warm", 0, 256, 20, 1)):
            print(f"[bench] closed loop {name}: {eps} episodes x {cyc} cycles", file=sys.stderr, flush=True)
            out["mpc"][name] = mpc_bench(pl, workload, torch, prec, eps, cyc, c=c, init=init)
    if not args.no_decoder:
        out["decoder"] = decoder_legs(pl, torch, workload, c, scene, args.steps, args.warmup)
    if not args.no_cpu_baseline:
        print("[bench] FP64 oracle on the host cores, and its accuracy check", file=sys.stderr, flush=True)
        out.update(cpu_baseline_leg(pl, workload))
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
