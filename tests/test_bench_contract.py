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


def test_headline_workload_is_the_128x128_q10_poisson_run():
    d = bench.linear_desc(pa, bench.RUN_128)
    assert (d.L, d.q, d.R, d.theta, d.seed) == (128, 10, 200000, 20, 4)
    assert d.resample == pa.RESAMPLE_POISSON
    # 500 equal steps from beta = 0 to 1.6
    assert d.K == 501 and d.beta[0] == 0.0 and d.beta[-1] == 1.6
    np.testing.assert_allclose(np.diff(d.beta), 1.6 / 500, rtol=0, atol=1e-15)
    # double-buffered population: at least two copies of R_cap replicas
    assert pa.pa_plan(d).workspace_bytes > 2 * d.R * d.N


def test_attempts_count_theta_sweeps_of_every_replica_of_the_given_steps():
    assert bench.attempts_of(np.array([5, 3, 4]), 10, 4) == 10 * 4 * (5 + 3 + 4)
    assert bench.attempts_of(np.array([], dtype=np.uint64), 10, 4) == 0.0


def test_roofline_constants_are_consistent():
    # 157.3 TFLOP/s of fp32 FMA = 128 lanes per CU and clock at 2.4 GHz
    assert bench.INT_OPS_PEAK == pytest.approx(157.3e12 / 2, rel=2e-3)
    assert 35 <= bench.ALG_OPS_PER_ATTEMPT <= 45


def test_probe_classes_cover_the_sweep_instruction_kinds():
    assert bench.probe_class("v_mad_u64_u32") == "mad64"
    assert bench.probe_class("v_bitop3_b32") == "bitop3"
    assert bench.probe_class("v_cmp_le_u32_sdwa") == "cmpsel"
    assert bench.probe_class("v_cndmask_b32_e32") == "cmpsel"
    assert bench.probe_class("v_addc_co_u32_e32") == "cmpsel"
    assert bench.probe_class("v_xor_b32_e32") == "xor"
    assert set(bench.probe_class(k) for k in ("v_perm_b32", "v_sad_u8", "v_xad_u32",
                                               "v_mul_hi_u32")) == {"perm", "sad", "xad", "mulhi"}
    assert {bench.probe_class(op) for op in ("v_mad_u64_u32", "v_and_b32")} <= set(pa.PROBE_KINDS)


def test_sweep_mix_reads_the_built_kernel():
    """The theta loop of the 128x128 sweep kernel, read from the built library's code
    object: about 31 vector instructions per attempt, 9 of them multiply-adds
    (Philox and the proposal)."""
    if not os.path.exists("/opt/rocm/llvm/bin/llvm-objdump"):
        pytest.skip("no llvm-objdump")
    mix, per_attempt = bench.sweep_mix(pa.LIB_PATH)
    assert 25 < per_attempt < 40
    assert 8.0 <= mix["mad64"] <= 10.0
    assert sum(mix.values()) == pytest.approx(per_attempt)


def test_cpu_baseline_object():
    cb = bench.cpu_baseline(50)
    assert set(cb) == {"value", "unit", "cores", "kind", "sample"}
    assert cb["kind"] == "oracle" and cb["unit"] == "attempts/ns"
    assert cb["cores"] >= 1 and cb["value"] > 0
    assert "R cut to 50" in cb["sample"] and "first temperature step" in cb["sample"]


@pytest.mark.gpu
def test_json_line_keys_and_units():
    cmd = [sys.executable, BENCH, "--steps", "2", "--warmup", "1", "--no-batched",
           "--serve-requests", "0", "--cpu-replicas", "50"]
    p = subprocess.run(cmd, capture_output=True, text=True, timeout=110, cwd=ROOT)
    assert p.returncode == 0, p.stderr[-2000:]
    lines = [ln for ln in p.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1
    r = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
              "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
              "roofline", "cpu_baseline"):
        assert k in r, k
    assert r["n_gpus"] == 1 and r["steps"] == 2 and r["warmup"] == 1
    assert r["unit"] == "attempts/ns" and r["higher_is_better"] is True
    assert r["dtype"] == "u8" and r["data"] == "synthetic" and r["vs_baseline"] is None
    assert r["config"]["workload"] and r["config"]["L"] == 128 and r["config"]["R"] == 200000
    assert r["value"] > 0 and r["ms_per_step"] > 0
    rf = r["roofline"]
    assert rf["bound"] in ("hbm", "mfma", "alu")
    assert rf["frac"] == pytest.approx(rf["achieved"] / rf["peak"])
    assert 0.0 < rf["frac"] < 1.0
    # the kernel cannot issue faster than its instruction kinds allow
    assert 0.0 < rf["frac_of_issue_ceiling"] < 1.0
    # the kernel is at least as fast as the whole run around it
    assert rf["sweep_attempts_per_ns"] >= r["value"]
    assert r["cpu_baseline"]["kind"] == "oracle"
