"""The benchmark script's contract: the workload it times, the attempt count
behind its throughput, its one-GPU limit, the CPU-baseline object, and (on a
GPU) the keys and units of the JSON line it prints."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import bench
import paper_1704_01888_amd as pa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True,
                       timeout=60, cwd=ROOT)
    assert p.returncode == 2
    assert p.stdout == ""
    assert "one GPU" in p.stderr and "--gpus 2" in p.stderr


def test_workload_is_the_32x32_q10_poisson_run():
    d = bench.workload_desc(pa)
    assert (d.L, d.q, d.R, d.theta, d.seed) == (32, 10, 20000, 10, 2)
    assert d.resample == pa.RESAMPLE_POISSON and d.outputs & pa.OUT_HIST
    # 400 equal steps from beta = 0 to 1.6
    assert d.K == 401 and d.beta[0] == 0.0 and d.beta[-1] == 1.6
    np.testing.assert_allclose(np.diff(d.beta), 1.6 / 400, rtol=0, atol=1e-15)
    # the plan accepts it (validation and sizing run on the host)
    assert pa.pa_plan(d).workspace_bytes > 2 * d.R * d.N


def test_attempts_count_the_sweeps_of_every_step_after_the_first():
    # R_0 is the initial population, which is not swept before resampling
    assert bench.attempts_of(np.array([7, 5, 3, 4]), 10, 4) == 10 * 4 * (5 + 3 + 4)
    assert bench.attempts_of(np.array([9]), 10, 4) == 0.0


def test_roofline_constants_are_consistent():
    assert bench.VALU_PEAK_LANE_OPS == pytest.approx(256 * 64 * 2.4e9)
    assert bench.MIX_PEAK_LANE_OPS > bench.VALU_PEAK_LANE_OPS
    # per launch: at least the algorithmic gather + store of the population
    w = bench.WORKLOAD
    assert bench.SWEEP_TRAFFIC_BYTES >= 2 * w["R"] * w["L"] ** 2 * 0.9
    assert 20.0 < bench.INSTR_PER_ATTEMPT < 60.0


def test_cpu_baseline_object():
    cb = bench.cpu_baseline(1)
    assert set(cb) == {"value", "unit", "cores", "kind", "sample"}
    assert cb["kind"] == "oracle" and cb["unit"] == "attempts/ns"
    assert cb["cores"] >= 1 and cb["value"] > 0
    assert "first 1 of 400 temperature steps" in cb["sample"]


@pytest.mark.gpu
def test_json_line_keys_and_units():
    cmd = [sys.executable, BENCH, "--steps", "1", "--warmup", "0", "--no-batched",
           "--serve-requests", "0", "--cpu-steps", "1"]
    p = subprocess.run(cmd, capture_output=True, text=True, timeout=110, cwd=ROOT)
    assert p.returncode == 0, p.stderr[-2000:]
    lines = [ln for ln in p.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    r = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline"):
        assert k in r, k
    assert r["n_gpus"] == 1 and r["steps"] == 1 and r["warmup"] == 0
    assert r["unit"] == "attempts/ns" and r["higher_is_better"] is True
    assert r["dtype"] == "u8" and r["data"] == "synthetic" and r["vs_baseline"] is None
    assert r["config"]["workload"] and r["config"]["L"] == 32 and r["config"]["R"] == 20000
    assert r["value"] > 0 and r["ms_per_step"] > 0
    rf = r["roofline"]
    assert rf["bound"] in ("hbm", "mfma", "alu")
    assert rf["frac"] == pytest.approx(rf["achieved"] / rf["peak"])
    assert 0.0 < rf["frac"] < 1.2
    # the kernel is at least as fast as the whole run around it
    assert rf["sweep_attempts_per_ns"] >= r["value"]
    assert r["cpu_baseline"]["kind"] == "oracle"
