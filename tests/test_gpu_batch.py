"""Batched runs (pa_run_batch) against separate runs and the oracle: every
output of every run bit-identical (FP64 estimators within 1e-12)."""
import numpy as np
import pytest

import oracle
import paper_1704_01888_amd as pa
from paper_1704_01888_amd.workloads import linear_betas

pytestmark = pytest.mark.gpu

KEYS_EXACT = ("R_i", "E_sum", "E_mean", "hist", "final_spins", "final_E", "last_anc", "digest")


@pytest.fixture(scope="module")
def ctx():
    c = pa.Context(0)
    yield c
    c.close()


def _same(a, b):
    for k in KEYS_EXACT:
        if k in a and k in b:
            assert (a[k] == b[k]).all(), k
    np.testing.assert_allclose(a["minus_beta_F"], b["minus_beta_F"], rtol=1e-12, atol=0)
    np.testing.assert_allclose(a["lnQ"], b["lnQ"], rtol=1e-12, atol=1e-13)


MIXED = [
    dict(L=8, q=8, R=300, beta=linear_betas(1.6, 20), theta=3, seed=1, resample=1),
    dict(L=16, q=10, R=700, beta=linear_betas(1.4, 12), theta=2, seed=2, resample=0),
    dict(L=12, q=5, R=250, beta=linear_betas(1.2, 25), theta=2, seed=3, resample=0),
    dict(L=4, q=3, R=333, beta=linear_betas(1.5, 7), theta=4, seed=4, resample=2),
    dict(L=24, q=20, R=129, beta=linear_betas(1.9, 9), theta=1, seed=5, resample=0),
    dict(L=32, q=6, R=200, beta=linear_betas(3.0, 10)[::-1].copy(), theta=2, seed=6, resample=0, init=1),
    dict(L=8, q=200, R=100, beta=linear_betas(2.0, 15), theta=2, seed=7, resample=1),
    dict(L=64, q=8, R=40, beta=np.array([0.0]), theta=2, seed=8, resample=0),
]


def test_batch_equals_separate_runs_and_oracle(ctx):
    descs = [pa.Desc(outputs=pa.OUT_HIST | pa.OUT_FINAL | pa.OUT_DIGEST, **c) for c in MIXED]
    print(f"\nbatch of {len(descs)} runs", flush=True)
    got = pa.pa_run_batch(ctx, descs)
    for c, d, g in zip(MIXED, descs, got):
        single = pa.pa_run(ctx, d)
        _same(g, single)
        want = oracle.run(oracle.Desc(**c), hist=True, final=True, digest=True)
        _same(g, want)


def test_batch_of_identical_shapes_differs_only_by_seed(ctx):
    cfg = [dict(L=16, q=8, R=500, beta=linear_betas(1.3, 15), theta=3, seed=100 + r, resample=1)
           for r in range(6)]
    descs = [pa.Desc(outputs=pa.OUT_FINAL, **c) for c in cfg]
    got = pa.pa_run_batch(ctx, descs)
    for d, g in zip(descs, got):
        _same(g, pa.pa_run(ctx, d))
    assert not (got[0]["final_spins"] == got[1]["final_spins"]).all()


def test_graph_replays_equal_eager(ctx):
    """The captured graph replayed several times (with eager runs and
    synchronisations in between) gives the eager results every time."""
    import torch
    cfg = MIXED[:6]
    descs = [pa.Desc(outputs=pa.OUT_HIST | pa.OUT_FINAL, **c) for c in cfg]
    eager = pa.pa_run_batch(ctx, descs)
    ws = torch.empty(pa.pa_plan_batch(descs), dtype=torch.uint8, device="cuda:0")
    ctx.set_graphs(True)
    try:
        for rep in range(3):
            got = pa.pa_run_batch(ctx, descs, workspace=ws)
            for a, b in zip(got, eager):
                _same(a, b)
            pa.pa_run(ctx, descs[0])          # eager work between replays
            torch.cuda.synchronize()
    finally:
        ctx.set_graphs(False)


def test_runs_sharing_a_schedule_with_different_weight_scales(ctx):
    """Runs of one (L, beta schedule) share the plan's tables in a batch; the
    weights depend on the population cap too (K_b), so runs of different R
    must still match their separate runs, and the first the oracle."""
    beta = linear_betas(1.5, 12)
    cfg = [dict(L=16, q=8, R=R, beta=beta, theta=2, seed=200 + k, resample=m)
           for k, (R, m) in enumerate([(1000, 1), (3000, 1), (1000, 0), (5000, 2), (9000, 0), (1000, 1)])]
    descs = [pa.Desc(outputs=pa.OUT_HIST | pa.OUT_FINAL | pa.OUT_DIGEST, **c) for c in cfg]
    got = pa.pa_run_batch(ctx, descs)
    for d, g in zip(descs, got):
        _same(g, pa.pa_run(ctx, d))
    _same(got[1], oracle.run(oracle.Desc(**cfg[1]), hist=True, final=True, digest=True))


def test_populations_just_above_the_small_population_limit(ctx):
    """Populations of 4097 to 8192 replicas (above the one-workgroup
    resampling of the post launch, so through the sampling and count-scan
    launches) in pa_run and pa_run_batch equal the oracle."""
    cfg = [dict(L=16, q=8, R=4500, beta=linear_betas(1.5, 10), theta=2, seed=210, resample=1),
           dict(L=16, q=10, R=7000, beta=linear_betas(1.6, 10), theta=2, seed=211, resample=0),
           dict(L=8, q=8, R=8192, beta=linear_betas(1.5, 12), theta=3, seed=212, resample=1)]
    descs = [pa.Desc(outputs=pa.OUT_HIST | pa.OUT_FINAL | pa.OUT_DIGEST, **c) for c in cfg]
    for d in descs:
        assert 4096 < pa.pa_plan(d).R_cap <= 8192
    got = pa.pa_run_batch(ctx, descs)
    for c, d, g in zip(cfg, descs, got):
        want = oracle.run(oracle.Desc(**c), hist=True, final=True, digest=True)
        _same(pa.pa_run(ctx, d), want)
        _same(g, want)
