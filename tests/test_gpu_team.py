"""Team launches of pa_run_batch (one cooperative launch per sweep class for
the runs with small populations, one device-wide barrier per step) against
separate pa_run calls, the segmented batch form and the oracle: every output
bit-identical (FP64 estimators within 1e-12), for all four team classes, the
three resampling modes, heating and ground-state starts, q above 128,
populations of 1, 2 and 8192, one-step runs, and batches that mix team and
segmented runs.  Segmented launches are the default mode.  A batch stopped
from another thread returns PA_ERR_CANCELLED and leaves the context usable."""
import threading
import time

import numpy as np
import pytest

import oracle
import paper_1704_01888_amd as pa
from paper_1704_01888_amd.workloads import linear_betas, small_runs

pytestmark = pytest.mark.gpu

ALL = pa.OUT_HIST | pa.OUT_MAG | pa.OUT_FINAL | pa.OUT_DIGEST | pa.OUT_WIDTHS
KEYS_EXACT = ("R_i", "E_sum", "E_mean", "hist", "Mt_sum", "M_mean", "mhist", "width_e", "width_m",
              "final_spins", "final_E", "last_anc", "digest")


@pytest.fixture(scope="module")
def ctx():
    c = pa.Context(0)
    c.set_batch_mode(pa.BATCH_TEAM)
    yield c
    c.close()


def _same(a, b):
    for k in KEYS_EXACT:
        if k in a and k in b:
            assert (a[k] == b[k]).all(), k
    np.testing.assert_allclose(a["minus_beta_F"], b["minus_beta_F"], rtol=1e-12, atol=0)
    np.testing.assert_allclose(a["lnQ"], b["lnQ"], rtol=1e-12, atol=1e-13)


TEAM = [
    dict(L=8, q=8, R=1000, beta=linear_betas(1.6, 200), theta=10, seed=1, resample=1),
    dict(L=8, q=200, R=500, beta=linear_betas(2.0, 30), theta=3, seed=11, resample=0),
    dict(L=16, q=10, R=3000, beta=linear_betas(1.6, 60), theta=3, seed=12, resample=0),
    dict(L=16, q=6, R=8192, beta=linear_betas(1.4, 9), theta=2, seed=13, resample=1),
    dict(L=16, q=8, R=1, beta=linear_betas(1.5, 30), theta=2, seed=14, resample=1),
    dict(L=8, q=5, R=2, beta=linear_betas(1.5, 25), theta=2, seed=15, resample=1),
    dict(L=32, q=5, R=800, beta=linear_betas(1.2, 20), theta=2, seed=16, resample=2),
    dict(L=32, q=10, R=1537, beta=linear_betas(1.6, 12), theta=2, seed=17, resample=0),
    dict(L=64, q=8, R=300, beta=linear_betas(3.0, 15)[::-1].copy(), theta=2, seed=18, resample=1, init=1),
    dict(L=64, q=20, R=130, beta=linear_betas(1.4, 10), theta=3, seed=19, resample=0),
    dict(L=8, q=8, R=700, beta=linear_betas(1.0, 1), theta=4, seed=20, resample=0),
]
SEGMENTED = [   # not team runs: a population above 8192, a lattice side without a team kernel
    dict(L=16, q=8, R=10000, beta=linear_betas(1.3, 6), theta=2, seed=30, resample=1),
    dict(L=12, q=5, R=250, beta=linear_betas(1.2, 25), theta=2, seed=31, resample=0),
]


def test_team_batch_equals_separate_runs_segmented_batch_and_oracle(ctx):
    cases = TEAM + SEGMENTED
    descs = [pa.Desc(outputs=ALL, **c) for c in cases]
    print(f"\nteam batch of {len(descs)} runs", flush=True)
    ctx.set_batch_mode(pa.BATCH_TEAM)
    got = pa.pa_run_batch(ctx, descs)
    team_runs, launches = ctx.batch_info()
    # classes (L, lanes per replica, q <= 128): (8,16,y) (8,16,n) (16,64,y) (32,256,y) (64,512,y)
    assert team_runs == len(TEAM) and launches == 5
    ctx.set_batch_mode(pa.BATCH_SEGMENTED)
    try:
        seg = pa.pa_run_batch(ctx, descs)
        assert ctx.batch_info() == (0, 0)
    finally:
        ctx.set_batch_mode(pa.BATCH_TEAM)
    for c, d, g, s in zip(cases, descs, got, seg):
        _same(g, s)
        _same(g, pa.pa_run(ctx, d))
    for c, g in zip(cases[1:7], got[1:7]):      # the oracle on the smaller team runs
        want = oracle.run(oracle.Desc(**c), hist=True, final=True, digest=True)
        _same(g, want)


@pytest.mark.parametrize("lanes", [16, 8])
def test_team_batch_of_the_small_run_workload(ctx, lanes):
    """20 runs of 8x8, q = 8, R = 1000, 200 steps (the benchmark's small-run
    batch) swept with 16 and with 8 lanes per replica: one team launch, each
    run equal to its pa_run and the first to the oracle."""
    runs = small_runs(20)
    descs = [pa.Desc(outputs=pa.OUT_HIST | pa.OUT_FINAL | pa.OUT_DIGEST, **r) for r in runs]
    before = ctx.tune_get(8, 8, 1000)
    ctx.tune_set(8, 0, 0, lanes, 4)
    try:
        got = pa.pa_run_batch(ctx, descs)
        assert ctx.batch_info() == (20, 1)
    finally:
        ctx.tune_set(8, 0, 0, before["lanes"], before["waves_per_block"])
    for d, g in zip(descs, got):
        _same(g, pa.pa_run(ctx, d))
    _same(got[0], oracle.run(oracle.Desc(**runs[0]), hist=True, final=True, digest=True))


def test_team_batch_repeats_and_reuses_a_workspace(ctx):
    import torch
    descs = [pa.Desc(outputs=pa.OUT_FINAL | pa.OUT_DIGEST, **c) for c in TEAM[:4]]
    ws = torch.empty(pa.pa_plan_batch(descs), dtype=torch.uint8, device="cuda:0")
    first = pa.pa_run_batch(ctx, descs, workspace=ws)
    for _ in range(2):
        pa.pa_run(ctx, descs[2])
        again = pa.pa_run_batch(ctx, descs, workspace=ws)
        for a, b in zip(first, again):
            _same(a, b)


def test_a_new_context_batches_in_segmented_launches():
    descs = [pa.Desc(outputs=pa.OUT_FINAL | pa.OUT_DIGEST, **c) for c in (TEAM[0], TEAM[2], SEGMENTED[1])]
    c = pa.Context(0)
    try:
        got = pa.pa_run_batch(c, descs)
        assert c.batch_info() == (0, 0)
        for d, g in zip(descs, got):
            _same(g, pa.pa_run(c, d))
    finally:
        c.close()


def test_more_runs_than_one_launch_holds_are_split_into_launches(ctx):
    """300 runs of 8x8 need 600 resident workgroups as teams of two: the
    group is split in halves until each launch fits."""
    cases = [dict(L=8, q=8, R=100, beta=linear_betas(1.5, 5), theta=2, seed=500 + r, resample=r % 2)
             for r in range(300)]
    descs = [pa.Desc(outputs=pa.OUT_FINAL | pa.OUT_DIGEST, **c) for c in cases]
    got = pa.pa_run_batch(ctx, descs)
    runs_in_teams, launches = ctx.batch_info()
    assert runs_in_teams == 300 and launches >= 3
    for k in range(0, 300, 37):
        _same(got[k], pa.pa_run(ctx, descs[k]))


def test_abort_from_another_thread_cancels_and_the_context_stays_usable(ctx):
    long = [pa.Desc(L=16, q=8, R=1000, beta=linear_betas(1.5, 100000), theta=1, seed=40 + r,
                    resample=1) for r in range(2)]
    box = {}

    def work():
        t0 = time.perf_counter()
        try:
            pa.pa_run_batch(ctx, long)
            box["status"] = 0
        except pa.PAError as e:
            box["status"] = e.status
        box["seconds"] = time.perf_counter() - t0

    print("\nlong team batch, aborted after 0.5 s", flush=True)
    th = threading.Thread(target=work)
    th.start()
    time.sleep(0.5)
    ctx.abort_batch()
    th.join(timeout=60)
    assert not th.is_alive()
    print(f"returned {box} ", flush=True)
    assert box["status"] == pa.PA_ERR_CANCELLED
    # the context runs the next batch normally
    descs = [pa.Desc(outputs=pa.OUT_FINAL | pa.OUT_DIGEST, **c) for c in TEAM[:3]]
    got = pa.pa_run_batch(ctx, descs)
    assert ctx.batch_info()[0] == 3
    for d, g in zip(descs, got):
        _same(g, pa.pa_run(ctx, d))
