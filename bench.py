"""Benchmark: Potts spin-flip attempts/ns of population annealing on one MI355X.

Workload (one "step" of this benchmark = one complete PA run, i.e. one pass of
the whole hot path -- initial population, 400 x (resample + 10 sweeps +
population statistics) -- over the synthetic input):
  plain PA, 2D q=10 Potts, L=32 periodic, R=20000, beta 0 -> 1.6 in 400 equal
  steps, theta=10 checkerboard Metropolis sweeps, Poisson resampling, energy
  histograms and the FP64 free-energy estimator reported per step, seed 2.

attempts = sum_{i=1}^{K-1} theta * R_i * N.  The timed region is a sequence of
whole runs (plan on the host, device work, results copied back), bracketed by
torch.cuda.synchronize().  Per-kernel durations are measured with HIP events
on the run's stream inside the library.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Potts spin-flip attempts/ns on 1 MI355X (batched vs plain), p99 run latency"

# VALU issue peak of MI355X, one wave64 instruction per CU per clock:
# 256 CUs x 64 lanes x 2.4 GHz = 39.3e12 lane-instructions/s.  Measured with
# streams of independent instructions: an uninterrupted stream of simple ops
# (v_and/v_xor/v_add/v_sub/v_bitop3) issues at 1.5-1.67x that, every other
# kind the sweep uses at 0.90-0.96x (v_perm, v_bcnt, v_lshl_add, v_xad,
# v_and_or; a simple op with a scalar operand too), and mixed streams at
# 0.95-1.055x (perm + bitop3 + xor: 1.055x).  The sweep is such a mix, so this
# peak is its bound up to about 5 %; MIX_PEAK_LANE_OPS is the best measured
# mixed-stream rate.  (The fp32 vector figure, 157.3 TFLOP/s, is the
# dual-issue FMA rate, which integer mixes cannot use.)
VALU_PEAK_LANE_OPS = 256 * 64 * 2.4e9
MIX_PEAK_LANE_OPS = 1.055 * VALU_PEAK_LANE_OPS

# VALU lane-instructions per spin-flip attempt of k_sweep on this workload,
# from rocprofv3 SQ_INSTS_VALU x 64 / attempts (gather, sweeps and energy
# epilogue; profiles/k_sweep_32x32_q10_R20000.md; 256 lanes per replica).
INSTR_PER_ATTEMPT = 33.30

# HBM bytes per k_sweep launch on this workload, from rocprofv3 FETCH_SIZE and
# WRITE_SIZE (scaled by 2.00 and 1.00, the factors the plain 256 MiB copy of
# --copy-calibration gives): (10652.0 * 2 + 20624.8) KiB;
# profiles/k_sweep_32x32_q10_R20000.md.  The algorithmic bytes are 2 * R * N =
# 41 MB (gather + store); repeated ancestors are served from cache.
SWEEP_TRAFFIC_BYTES = (10652.0 * 2.0 + 20624.8) * 1024

WORKLOAD = dict(L=32, q=10, R=20000, K=401, beta_max=1.6, theta=10, seed=2)


def workload_desc(pa):
    w = WORKLOAD
    n = w["K"] - 1
    beta = np.array([w["beta_max"] * i / n for i in range(n + 1)])
    return pa.Desc(w["L"], w["q"], w["R"], beta, w["theta"], w["seed"],
                   resample=pa.RESAMPLE_POISSON, outputs=pa.OUT_HIST)


def attempts_of(R_i, theta, N):
    return float(theta) * float(N) * float(np.asarray(R_i[1:], dtype=np.float64).sum())


def batched_vs_plain(pa, torch, ctx, runs, reps=1):
    """The same runs as separate pa_run calls and as one pa_run_batch."""
    descs = [pa.Desc(**r) for r in runs]
    att = sum(float(r["theta"]) * r["L"] ** 2 * float(np.sum(pa.pa_plan_tables(d)[1][1:]))
              for r, d in zip(runs, descs))
    ws_b = torch.empty(pa.pa_plan_batch(descs), dtype=torch.uint8, device="cuda:0")
    ws_p = torch.empty(max(pa.pa_plan(d).workspace_bytes for d in descs), dtype=torch.uint8,
                       device="cuda:0")
    for d in descs[:2]:
        pa.pa_run(ctx, d, workspace=ws_p)
    pa.pa_run_batch(ctx, descs, workspace=ws_b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for d in descs:
            pa.pa_run(ctx, d, workspace=ws_p)
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        pa.pa_run_batch(ctx, descs, workspace=ws_b)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    # the same batch replayed as a captured HIP graph (captured in the warm-up)
    ctx.set_graphs(True)
    pa.pa_run_batch(ctx, descs, workspace=ws_b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        pa.pa_run_batch(ctx, descs, workspace=ws_b)
    torch.cuda.synchronize()
    t_graph = (time.perf_counter() - t0) / reps
    ctx.set_graphs(False)
    del ws_b, ws_p
    return {"runs": len(runs), "attempts": att,
            "plain_attempts_per_ns": att / t_plain / 1e9, "plain_ms": t_plain * 1e3,
            "batched_attempts_per_ns": att / t_batch / 1e9, "batched_ms": t_batch * 1e3,
            "graph_attempts_per_ns": att / t_graph / 1e9, "graph_ms": t_graph * 1e3,
            "speedup": t_plain / min(t_batch, t_graph)}


def serving(pa, torch, ctx, n_requests, capacity_attempts_per_ns, rho=0.8,
            arena_bytes=24 << 30, max_slots=16):
    """The first n_requests of the 500-request stream, arriving as a Poisson
    process at rho x capacity / mean request attempts; p50/p99 latency."""
    import threading
    from paper_1704_01888_amd import workloads
    reqs = workloads.serving_requests(500)[:n_requests]
    descs = [pa.Desc(**r) for r in reqs]
    atts = [float(r["theta"]) * r["L"] ** 2 * float(np.sum(pa.pa_plan_tables(d)[1][1:]))
            for r, d in zip(reqs, descs)]
    mean_att = float(np.mean(atts))
    rate = rho * capacity_attempts_per_ns * 1e9 / mean_att          # requests per second
    arrivals = workloads.poisson_arrivals(n_requests, rate)
    sv = pa.Server(ctx, arena_bytes=arena_bytes, max_slots=max_slots)
    tickets = [None] * n_requests
    lat = [None] * n_requests
    t0 = time.perf_counter()

    def submitter():
        for i, d in enumerate(descs):
            delay = arrivals[i] - (time.perf_counter() - t0)
            if delay > 0:
                time.sleep(delay)
            tickets[i] = sv.submit(d)

    th = threading.Thread(target=submitter)
    th.start()
    for i in range(n_requests):
        while tickets[i] is None:
            time.sleep(0.0005)
        _, tm = sv.wait(tickets[i])
        lat[i] = (tm["done_us"] - tm["arrival_us"]) * 1e-3
    th.join()
    makespan = time.perf_counter() - t0
    sv.stop()
    lat = np.array(lat)
    return {"requests": n_requests, "offered_load": rho, "arrival_rate_per_s": rate,
            "attempts": float(sum(atts)), "attempts_per_ns": sum(atts) / makespan / 1e9,
            "latency_ms_p50": float(np.percentile(lat, 50)),
            "latency_ms_p99": float(np.percentile(lat, 99)),
            "latency_ms_max": float(lat.max()), "makespan_s": makespan,
            "arena_GB": arena_bytes / 2**30, "max_slots": max_slots}


def cpu_baseline(n_steps: int):
    """The oracle on the host cores: the same workload cut to its first
    n_steps temperature steps."""
    import oracle
    w = WORKLOAD
    n = w["K"] - 1
    beta = np.array([w["beta_max"] * i / n for i in range(n + 1)])[: n_steps + 1]
    od = oracle.Desc(w["L"], w["q"], w["R"], beta, w["theta"], w["seed"],
                     resample=oracle.RESAMPLE_POISSON)
    t0 = time.perf_counter()
    out = oracle.run(od, hist=True)
    dt = time.perf_counter() - t0
    att = attempts_of(out["R_i"], w["theta"], w["L"] ** 2)
    return {"value": att / dt / 1e9, "unit": "attempts/ns", "cores": int(out["n_threads"]),
            "kind": "oracle",
            "sample": f"same workload, initial population + first {n_steps} of {n} temperature "
                      f"steps ({att:.3g} attempts, {dt:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain lines")
    ap.add_argument("--serve-requests", type=int, default=32,
                    help="requests of the serving line (0 = skip)")
    ap.add_argument("--cpu-steps", type=int, default=50,
                    help="temperature steps of the oracle's CPU-baseline sample (0 = skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 256 MiB device-to-device three times (reference kernel of "
                         "known size for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--profile-run", metavar="L,q,R,K,theta",
                    help="only one plain run of this shape (beta 0 -> 1.0 in K-1 equal steps, "
                         "multinomial, seed 7), for profiling; prints its kernel times")
    args = ap.parse_args()
    if args.profile_run:
        import torch
        import paper_1704_01888_amd as pa
        L, q, R, K, theta = (int(x) for x in args.profile_run.split(","))
        ctx = pa.Context(0)
        d = pa.Desc(L, q, R, np.array([1.0 * i / (K - 1) for i in range(K)]), theta, 7,
                    resample=pa.RESAMPLE_MULTINOMIAL)
        ctx.set_profiling(True)
        out = pa.pa_run(ctx, d)
        att = attempts_of(out["R_i"], theta, L * L)
        ms = dict(zip(pa.KERNEL_NAMES, (float(x) for x in out["kernel_ms"])))
        print(json.dumps({"L": L, "q": q, "R": R, "K": K, "theta": theta, "kernel_ms": ms,
                          "sweep_attempts_per_ns": att / (ms["sweep"] * 1e6)}))
        return
    if args.copy_calibration:
        import torch
        a = torch.ones(256 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copied_bytes": 256 << 20, "times": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU design is described but not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1704_01888_amd as pa

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    pa.lib()
    ctx = pa.Context(0)
    desc = workload_desc(pa)
    info = pa.pa_plan(desc)
    ws = torch.empty(int(info.workspace_bytes), dtype=torch.uint8, device="cuda:0")
    N = desc.N

    for _ in range(args.warmup):
        pa.pa_run(ctx, desc, workspace=ws)
    torch.cuda.synchronize()

    total_att = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = pa.pa_run(ctx, desc, workspace=ws)
        total_att += attempts_of(out["R_i"], desc.theta, N)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = total_att / dt / 1e9

    # One more run, outside the timed region, with every kernel bracketed by
    # HIP events on the run's stream: per-kernel durations.
    ctx.set_profiling(True)
    prof = pa.pa_run(ctx, desc, workspace=ws)
    ctx.set_profiling(False)
    kernel_ms = prof["kernel_ms"]
    kernel_n = prof["kernel_launches"]
    prof_att = attempts_of(prof["R_i"], desc.theta, N)
    sweep = pa.KERNEL_NAMES.index("sweep")
    sweep_s = kernel_ms[sweep] / 1e3
    sweep_avg_ms = kernel_ms[sweep] / max(kernel_n[sweep], 1)
    sweep_rate = prof_att / sweep_s if sweep_s > 0 else 0.0   # attempts/s inside the sweep kernel
    achieved = sweep_rate * INSTR_PER_ATTEMPT / 1e12
    peak = VALU_PEAK_LANE_OPS / 1e12
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "attempts/ns",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {
            "workload": "plain PA, 2D q=10 Potts, L=32 periodic, R=20000, beta 0->1.6 in 400 "
                        "equal steps, theta=10, Poisson resampling, per-step energy histograms "
                        "and FP64 free energy, Philox4x32-10 seed=2",
            "L": 32, "q": 10, "R": 20000, "K": 401, "theta": 10, "form": "plain",
            "parallelism": "1 GPU",
        },
        "roofline": {
            "bound": "alu",
            "kernel": "k_sweep",
            "achieved": achieved,
            "peak": peak,
            "unit": "T lane-instructions/s",
            "frac": achieved / peak,
            "traffic": SWEEP_TRAFFIC_BYTES,
            "instr_per_attempt": INSTR_PER_ATTEMPT,
            "frac_of_measured_mix_peak": achieved / (MIX_PEAK_LANE_OPS / 1e12),
            "sweep_attempts_per_ns": sweep_rate / 1e9,
            "sweep_avg_launch_ms": sweep_avg_ms,
        },
        "kernel_ms_per_run": {k: float(v) for k, v in zip(pa.KERNEL_NAMES, kernel_ms)},
    }
    if not args.no_batched:
        from paper_1704_01888_amd import workloads
        result["batched"] = {
            "20 runs of 8x8 q=8 R=1000, 200 steps, theta=10, multinomial":
                batched_vs_plain(pa, torch, ctx, workloads.small_runs(20), reps=3),
            "20 runs L in {16..64}, q in {5..20}, R in [1e4,1e5], 300 steps, theta=10, Poisson":
                batched_vs_plain(pa, torch, ctx, workloads.mixed_runs(20), reps=1),
        }
    if args.serve_requests > 0:
        mixed = result.get("batched", {}).get(
            "20 runs L in {16..64}, q in {5..20}, R in [1e4,1e5], 300 steps, theta=10, Poisson")
        capacity = mixed["batched_attempts_per_ns"] if mixed else value
        result["serving"] = serving(pa, torch, ctx, args.serve_requests, capacity)
    if args.cpu_steps > 0:
        result["cpu_baseline"] = cpu_baseline(args.cpu_steps)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
