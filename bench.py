"""Benchmark: Potts spin-flip attempts/ns of population annealing on one MI355X.

Headline workload (the largest single-GPU configuration):
  plain PA, 2D q=10 Potts, L=128 periodic, R=200000, beta 0 -> 1.6 in 500
  equal steps, theta=20 checkerboard Metropolis sweeps per step, Poisson
  resampling, uint8 spins double-buffered in HBM, Philox4x32-10 seed=4.

One benchmark "step" is one temperature step of that run: the resampling from
beta_{i-1} to beta_i (weights, draws, copy numbers, ancestors), the gather of
every new replica from its ancestor fused with theta = 20 sweeps at beta_i, the
energies, and the population statistics with the FP64 free-energy term
(Sec. 2 of the paper, steps 2-4).  The run is created (initial population,
3.3 GB) before the timed region; `--warmup` steps run untimed, then exactly
`--steps` steps are timed between two device synchronisations.

attempts = sum over the timed steps of theta * R_i * N.  The sweep kernel's
launches during the timed steps are bracketed by HIP events on the run's
stream (inside the library); their average gives the roofline entry.

Further entries on the same JSON line: the 32x32 workload as whole runs, the
batched forms against one-run-per-launch, the serving loop over the
500-request stream (p50/p99 latency), the issue-rate ceiling of the sweep
kernel, and the oracle timed on the host cores (cpu_baseline).
"""
from __future__ import annotations

import argparse
import collections
import json
import os
import re
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Potts spin-flip attempts/ns on 1 MI355X (batched vs plain), p99 run latency"

# Integer vector peak of MI355X: the fp32 vector rate, 157.3 TFLOP/s, is 128
# FMA lanes per compute unit and clock (256 CUs x 128 x 2 flop x 2.4 GHz); as
# 32-bit operations per second that is 256 x 128 x 2.4e9 = 78.6e12.
INT_OPS_PEAK = 256 * 128 * 2.4e9
# Algorithmic 32-bit operations per spin-flip attempt of the sweep: half a
# Philox4x32-10 block (10 wide multiplies, 20 xors), the proposal, the eight
# neighbour comparisons and the energy difference, the acceptance test and
# select -- 35-45 by the plain count, 40 taken as the figure.
ALG_OPS_PER_ATTEMPT = 40

# HBM bytes per sweep launch at 128x128, R = 2e5: rocprofv3 FETCH_SIZE x 2.00
# + WRITE_SIZE x 1.00 (the factors a plain 256 MiB copy gives), average of the
# step launches 1-3: (2 x 1603274 + 3200009) KiB; 2 R_i N = 6.55e9 bytes are
# algorithmic (gather + store).
SWEEP_TRAFFIC_BYTES = (2.0 * 1603274 + 3200009) * 1024

RUN_128 = dict(L=128, q=10, R=200000, K=501, beta_max=1.6, theta=20, seed=4)
RUN_32 = dict(L=32, q=10, R=20000, K=401, beta_max=1.6, theta=10, seed=2)

SWEEP_SYMBOL = "_ZN2pa12_GLOBAL__N_17k_sweepILj128ELj512ELb1ELb0EEEvNS_9SweepArgsE"


def linear_desc(pa, w, outputs=0):
    n = w["K"] - 1
    beta = np.array([w["beta_max"] * i / n for i in range(n + 1)])
    return pa.Desc(w["L"], w["q"], w["R"], beta, w["theta"], w["seed"],
                   resample=pa.RESAMPLE_POISSON, outputs=outputs)


def attempts_of(R_i, theta, N):
    return float(theta) * float(N) * float(np.asarray(R_i, dtype=np.float64).sum())


# ---------------------------------------------------------------------------
# Issue-rate ceiling of the sweep kernel
# ---------------------------------------------------------------------------
def probe_class(op: str) -> str:
    """Probe kind whose issue rate prices a vector instruction of the sweep."""
    if op.startswith("v_mad_u64_u32"):
        return "mad64"
    if op.startswith("v_bitop3"):
        return "bitop3"
    if op.startswith("v_perm"):
        return "perm"
    if op.startswith("v_sad"):
        return "sad"
    if op.startswith("v_xad"):
        return "xad"
    if op.startswith("v_mul_hi"):
        return "mulhi"
    if op.startswith(("v_cmp", "v_cndmask", "v_addc", "v_subb")):
        return "cmpsel"
    return "xor"


def sweep_mix(lib_path: str, symbol: str = SWEEP_SYMBOL, attempts_per_iter: int = 32):
    """Vector instructions per attempt of the sweep's theta loop, by probe
    kind, read from the AMD assembly of the built library's gfx950 code object.  At
    L = 128 with 512 lanes a lane updates 8 pairs per half-sweep, so one
    iteration of the theta loop (both colours, fully unrolled) is 32 attempts
    per lane."""
    llvm = "/opt/rocm/llvm/bin"
    tmp = os.path.join(os.environ.get("TMPDIR", "/tmp"), f"pa_sweep_{os.getpid()}")
    try:
        # the library's device code is an offload bundle in its .hip_fatbin section
        subprocess.run([f"{llvm}/llvm-objcopy", f"--dump-section=.hip_fatbin={tmp}.bundle", lib_path,
                        f"{tmp}.host"], check=True, capture_output=True)
        subprocess.run([f"{llvm}/clang-offload-bundler", "--unbundle", "--type=o",
                        f"--input={tmp}.bundle", "--targets=hipv4-amdgcn-amd-amdhsa--gfx950",
                        f"--output={tmp}.elf"], check=True, capture_output=True)
        dis = subprocess.run([f"{llvm}/llvm-objdump", "-d", "--no-show-raw-insn",
                              f"--disassemble-symbols={symbol}", f"{tmp}.elf"],
                             check=True, capture_output=True, text=True).stdout
    finally:
        for ext in (".bundle", ".host", ".elf"):
            if os.path.exists(tmp + ext):
                os.remove(tmp + ext)
    insts = []
    for ln in dis.splitlines():
        m = re.match(r"\s+(\S+)\s*(.*?)\s*//\s*([0-9A-F]+):", ln)
        if m:
            insts.append((int(m.group(3), 16), m.group(1), ln))
    if not insts:
        raise RuntimeError("sweep kernel not found in the code object")
    a0 = insts[0][0]
    loops = []
    for a, op, ln in insts:
        t = re.search(r"\+0x([0-9a-f]+)>", ln)
        if "branch" in op and t and a0 + int(t.group(1), 16) < a:
            loops.append((a0 + int(t.group(1), 16), a))
    # the theta loop: the longest backward branch that holds no other loop
    loops.sort(key=lambda x: x[1] - x[0], reverse=True)
    lo, hi = next(l for l in loops if not any(o != l and l[0] < o[0] and o[1] < l[1]
                                              and o[1] - o[0] > 64 for o in loops))
    ops = [op for a, op, _ in insts if lo <= a <= hi and op.startswith("v_")]
    if sum(op.startswith("v_mad_u64_u32") for op in ops) < attempts_per_iter:
        raise RuntimeError("unexpected shape of the theta loop")
    by_kind = collections.Counter(probe_class(op) for op in ops)
    return {k: v / attempts_per_iter for k, v in sorted(by_kind.items())}, len(ops) / attempts_per_iter


def issue_ceiling(ctx, lib_path):
    """Attempts/ns the sweep loop cannot exceed: its instructions per attempt
    of each kind, each at that kind's measured issue rate, one after another;
    and the same from the measured rate of a stream mixed like the loop."""
    import paper_1704_01888_amd as pa
    rates = {k: ctx.issue_probe(k) for k in pa.PROBE_KINDS}
    try:
        mix, per_attempt = sweep_mix(lib_path)
    except (OSError, subprocess.CalledProcessError, RuntimeError, StopIteration) as e:
        return {"probe_lane_instr_per_s": rates, "error": f"instruction mix unavailable: {e}"}
    s_per_attempt = sum(n / rates[k] for k, n in mix.items())
    return {
        "probe_lane_instr_per_s": rates,
        "loop_instr_per_attempt": per_attempt,
        "loop_mix_per_attempt": mix,
        "ceiling_attempts_per_ns": 1.0 / s_per_attempt / 1e9,
        "mixed_stream_ceiling_attempts_per_ns": rates["mix"] / per_attempt / 1e9,
    }


# ---------------------------------------------------------------------------
# Further entries
# ---------------------------------------------------------------------------
def whole_runs(pa, torch, ctx, w, reps=3):
    """The workload as complete runs (initial population, every step, results
    copied back), one after another."""
    desc = linear_desc(pa, w, outputs=pa.OUT_HIST)
    ws = torch.empty(int(pa.pa_plan(desc).workspace_bytes), dtype=torch.uint8, device="cuda:0")
    pa.pa_run(ctx, desc, workspace=ws)
    torch.cuda.synchronize()
    att = 0.0
    t0 = time.perf_counter()
    for _ in range(reps):
        out = pa.pa_run(ctx, desc, workspace=ws)
        att += attempts_of(out["R_i"][1:], desc.theta, desc.N)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    del ws
    return {"runs": reps, "attempts_per_ns": att / dt / 1e9, "ms_per_run": dt / reps * 1e3}


def batched_vs_plain(pa, torch, ctx, runs, reps=1):
    """The same runs as separate pa_run calls and as one pa_run_batch: the
    segmented launches (the default), team launches for every run that
    qualifies, and the segmented step sequence replayed as a HIP graph."""
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

    def timed(fn):
        # the median of reps timed calls (a rare host-side stall of tens of
        # milliseconds would otherwise dominate a mean of a few short calls)
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    t_plain = timed(lambda: [pa.pa_run(ctx, d, workspace=ws_p) for d in descs])
    t_batch = timed(lambda: pa.pa_run_batch(ctx, descs, workspace=ws_b))     # segmented launches

    def in_mode(mode):
        ctx.set_batch_mode(mode)
        pa.pa_run_batch(ctx, descs, workspace=ws_b)
        torch.cuda.synchronize()
        t = timed(lambda: pa.pa_run_batch(ctx, descs, workspace=ws_b))
        return t, ctx.batch_info()

    t_team, (team_runs, team_launches) = in_mode(pa.BATCH_TEAM)
    ctx.set_batch_mode(pa.BATCH_SEGMENTED)
    ctx.set_graphs(True)
    pa.pa_run_batch(ctx, descs, workspace=ws_b)        # capture
    torch.cuda.synchronize()
    t_graph = timed(lambda: pa.pa_run_batch(ctx, descs, workspace=ws_b))
    ctx.set_graphs(False)
    del ws_b, ws_p
    return {"runs": len(runs), "attempts": att,
            "plain_attempts_per_ns": att / t_plain / 1e9, "plain_ms": t_plain * 1e3,
            "batched_attempts_per_ns": att / t_batch / 1e9, "batched_ms": t_batch * 1e3,
            "team_attempts_per_ns": att / t_team / 1e9, "team_ms": t_team * 1e3,
            "team_runs": team_runs, "team_launches": team_launches,
            "graph_attempts_per_ns": att / t_graph / 1e9, "graph_ms": t_graph * 1e3,
            "speedup": t_plain / min(t_batch, t_team, t_graph)}


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
        if (i + 1) % 100 == 0:
            print(f"serving: {i + 1} of {n_requests} requests done", file=sys.stderr, flush=True)
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


def cpu_baseline(replicas: int):
    """The oracle on the host cores: the headline workload with its population
    cut to `replicas`, initial population and first temperature step."""
    import oracle
    w = RUN_128
    n = w["K"] - 1
    beta = np.array([w["beta_max"] * i / n for i in range(n + 1)])[:2]
    od = oracle.Desc(w["L"], w["q"], replicas, beta, w["theta"], w["seed"],
                     resample=oracle.RESAMPLE_POISSON)
    t0 = time.perf_counter()
    out = oracle.run(od)
    dt = time.perf_counter() - t0
    att = attempts_of(out["R_i"][1:], w["theta"], w["L"] ** 2)
    return {"value": att / dt / 1e9, "unit": "attempts/ns", "cores": int(out["n_threads"]),
            "kind": "oracle",
            "sample": f"the 128x128, q=10, theta=20 workload with R cut to {replicas}: initial "
                      f"population + first temperature step ({att:.3g} attempts, {dt:.1f} s, "
                      f"initial population included)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-vs-plain lines")
    ap.add_argument("--serve-requests", type=int, default=500,
                    help="requests of the serving line (0 = skip)")
    ap.add_argument("--cpu-replicas", type=int, default=30000,
                    help="population of the oracle's CPU-baseline sample (0 = skip)")
    ap.add_argument("--no-probe", action="store_true", help="skip the issue-rate ceiling")
    ap.add_argument("--issue-probe", action="store_true",
                    help="only the issue-rate probes and the sweep's instruction mix")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 256 MiB device-to-device three times (reference kernel of "
                         "known size for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    ap.add_argument("--profile-steps", type=int, default=0, metavar="S",
                    help="only the headline run's initial population and S steps, for profiling")
    ap.add_argument("--profile-run", default="", metavar="L:R:K:THETA",
                    help="only whole runs of an LxL, q=10 lattice with R replicas, K temperatures "
                         "to beta = 1.6 and THETA sweeps per step (Poisson, seed 2, per-step "
                         "histograms), for profiling")
    ap.add_argument("--profile-reps", type=int, default=1, help="repetitions of --profile-run")
    ap.add_argument("--profile-batch", action="store_true",
                    help="only the batch of 20 runs of 8x8, q=8, R=1000, 200 steps: segmented, "
                         "then in team launches, twice each, for profiling")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU design is described but not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1704_01888_amd as pa

    if args.copy_calibration:
        a = torch.ones(256 << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copied_bytes": 256 << 20, "times": 3}))
        return
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    pa.lib()
    # the profiling modes sweep with the default shapes, the others with the
    # package's tuned shapes (as any Context does)
    ctx = pa.Context(0, tune_cache=not (args.profile_run or args.profile_steps or args.profile_batch))
    if args.issue_probe:
        print(json.dumps(issue_ceiling(ctx, pa.LIB_PATH)), flush=True)
        return

    if args.profile_batch:
        from paper_1704_01888_amd import workloads
        descs = [pa.Desc(**r) for r in workloads.small_runs(20)]
        ws = torch.empty(pa.pa_plan_batch(descs), dtype=torch.uint8, device="cuda:0")
        for mode in (pa.BATCH_SEGMENTED, pa.BATCH_TEAM):
            ctx.set_batch_mode(mode)
            for _ in range(2):
                pa.pa_run_batch(ctx, descs, workspace=ws)
        torch.cuda.synchronize()
        print(json.dumps({"profiled_batch": "20 runs of 8x8, q=8, R=1000, 200 steps", "team": ctx.batch_info()}))
        return
    if args.profile_run:
        L, R, K, theta = (int(x) for x in args.profile_run.split(":"))
        w = dict(L=L, q=10, R=R, K=K, beta_max=1.6, theta=theta, seed=2)
        d = linear_desc(pa, w, outputs=pa.OUT_HIST)
        ws = torch.empty(int(pa.pa_plan(d).workspace_bytes), dtype=torch.uint8, device="cuda:0")
        t0 = time.perf_counter()
        att = 0.0
        for _ in range(args.profile_reps):
            out = pa.pa_run(ctx, d, workspace=ws)
            att += attempts_of(out["R_i"][1:], theta, L * L)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        print(json.dumps({"profiled_run": w, "reps": args.profile_reps, "attempts_per_ns": att / dt / 1e9}))
        return

    desc = linear_desc(pa, RUN_128)
    N = desc.N
    R_sched = pa.pa_plan_tables(desc)[1]
    if args.profile_steps:
        run = pa.Run(ctx, desc)
        run.advance(args.profile_steps)
        run.sync()
        run.finish()
        print(json.dumps({"profiled_steps": args.profile_steps}))
        return
    if args.warmup + args.steps > desc.K - 1:
        print(f"warmup + steps must be at most {desc.K - 1}", file=sys.stderr)
        sys.exit(2)

    print("headline: initial population", file=sys.stderr, flush=True)
    run = pa.Run(ctx, desc)                       # 3.3 GB initial population, untimed
    for _ in range(args.warmup):
        run.advance(1)
    run.sync()
    ctx.set_profiling(True)                       # events around the timed steps' launches
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        run.advance(1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.set_profiling(False)
    prof = run.finish()
    first = args.warmup + 1
    att = attempts_of(R_sched[first:first + args.steps], desc.theta, N)
    value = att / dt / 1e9
    print(f"headline: {value:.1f} attempts/ns", file=sys.stderr, flush=True)

    sweep = pa.KERNEL_NAMES.index("sweep")
    n_launch = int(prof["kernel_launches"][sweep])
    sweep_avg_s = prof["kernel_ms"][sweep] / 1e3 / max(n_launch, 1)
    att_per_launch = att / max(n_launch, 1)
    sweep_rate = att_per_launch / sweep_avg_s                    # attempts/s inside the kernel
    achieved = ALG_OPS_PER_ATTEMPT * sweep_rate
    roofline = {
        "bound": "alu",
        "kernel": "k_sweep",
        "achieved": achieved / 1e12,
        "peak": INT_OPS_PEAK / 1e12,
        "unit": "T int32 lane-ops/s",
        "frac": achieved / INT_OPS_PEAK,
        "traffic": SWEEP_TRAFFIC_BYTES,
        "alg_ops_per_attempt": ALG_OPS_PER_ATTEMPT,
        "attempts_per_launch": att_per_launch,
        "sweep_avg_launch_ms": sweep_avg_s * 1e3,
        "sweep_attempts_per_ns": sweep_rate / 1e9,
        "kernel_ms_per_step": {k: float(v) / args.steps for k, v in zip(pa.KERNEL_NAMES, prof["kernel_ms"])},
    }
    if not args.no_probe:
        ceil = issue_ceiling(ctx, pa.LIB_PATH)
        roofline["issue_ceiling"] = ceil
        if "ceiling_attempts_per_ns" in ceil:
            roofline["frac_of_issue_ceiling"] = sweep_rate / 1e9 / ceil["ceiling_attempts_per_ns"]
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
            "workload": "plain PA, 2D q=10 Potts, L=128 periodic, R=200000, beta 0->1.6 in 500 "
                        "equal steps, theta=20, Poisson resampling, uint8 spins double-buffered, "
                        "Philox4x32-10 seed=4; one step = resampling + 20 sweeps + statistics",
            "L": 128, "q": 10, "R": 200000, "K": 501, "theta": 20, "form": "plain",
            "timed_steps": [first, first + args.steps - 1], "parallelism": "1 GPU",
        },
        "roofline": roofline,
    }
    print("32x32 whole runs", file=sys.stderr, flush=True)
    result["whole_runs_32x32_q10_R20000"] = whole_runs(pa, torch, ctx, RUN_32)
    if not args.no_batched:
        from paper_1704_01888_amd import workloads
        print("batched lines", file=sys.stderr, flush=True)
        result["batched"] = {
            "20 runs of 8x8 q=8 R=1000, 200 steps, theta=10, multinomial":
                batched_vs_plain(pa, torch, ctx, workloads.small_runs(20), reps=5),
            "20 runs L in {16..64}, q in {5..20}, R in [1e4,1e5], 300 steps, theta=10, Poisson":
                batched_vs_plain(pa, torch, ctx, workloads.mixed_runs(20), reps=1),
        }
    if args.serve_requests > 0:
        mixed = result.get("batched", {}).get(
            "20 runs L in {16..64}, q in {5..20}, R in [1e4,1e5], 300 steps, theta=10, Poisson")
        capacity = mixed["batched_attempts_per_ns"] if mixed else value
        print(f"serving {args.serve_requests} requests", file=sys.stderr, flush=True)
        result["serving"] = serving(pa, torch, ctx, args.serve_requests, capacity)
    if args.cpu_replicas > 0:
        print("cpu baseline", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(args.cpu_replicas)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
