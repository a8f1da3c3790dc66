"""Lattices beyond one workgroup's LDS (L > 256, tiled half-sweeps in HBM)
against the CPU oracle through the C ABI: spins, energies, histograms,
ancestors, magnetisation and widths bit-exact; FP64 estimators within 1e-12.
Sizes span several row tiles with a ragged last tile, up to L = 4096; theta
from 0 to 3 gives one to three tiled launches per step (each launch fuses two
half-sweeps and alternates between two buffers)."""
import numpy as np
import pytest

import oracle
import paper_1704_01888_amd as pa
from paper_1704_01888_amd.workloads import linear_betas

pytestmark = pytest.mark.gpu

ALL = pa.OUT_HIST | pa.OUT_FINAL | pa.OUT_MAG | pa.OUT_WIDTHS | pa.OUT_DIGEST


@pytest.fixture(scope="module")
def ctx():
    c = pa.Context(0)
    yield c
    c.close()


def _compare(got, want):
    for k in ("R_i", "E_sum", "E_mean", "hist", "last_anc", "final_E", "final_spins",
              "Mt_sum", "M_mean", "mhist", "width_e", "width_m", "digest"):
        if k in want and k in got:
            assert (got[k] == want[k]).all(), k
    np.testing.assert_allclose(got["lnQ"], want["lnQ"], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(got["minus_beta_F"], want["minus_beta_F"], rtol=1e-12, atol=0)


def _both(ctx, outputs=ALL, **kw):
    print(f"\ncase: L={kw['L']} q={kw['q']} R={kw['R']} K={len(kw['beta'])} theta={kw['theta']} "
          f"resample={kw.get('resample', 0)} init={kw.get('init', 0)}", flush=True)
    got = pa.pa_run(ctx, pa.Desc(outputs=outputs, **kw))
    want = oracle.run(oracle.Desc(**kw), hist=bool(outputs & pa.OUT_HIST),
                      final=bool(outputs & pa.OUT_FINAL), magnetisation=bool(outputs & pa.OUT_MAG),
                      widths=bool(outputs & pa.OUT_WIDTHS), digest=bool(outputs & pa.OUT_DIGEST))
    return got, want


CASES = [
    # 63-row tiles, the last one 8 rows
    dict(L=260, q=10, R=6, beta=linear_betas(1.5, 3), theta=2, seed=41, resample=0, bin_e=3),
    # q beyond the 7-bit fast path
    dict(L=320, q=200, R=5, beta=linear_betas(2.0, 2), theta=3, seed=42, resample=1, bin_m=2),
    # heating from ground states
    dict(L=512, q=8, R=4, beta=linear_betas(3.0, 2)[::-1].copy(), theta=1, seed=43, resample=0, init=1),
    # resampling off
    dict(L=1024, q=3, R=3, beta=linear_betas(1.0, 1), theta=2, seed=44, resample=2),
    # no sweeps: the step only copies the ancestors
    dict(L=272, q=6, R=7, beta=linear_betas(1.2, 3), theta=0, seed=45, resample=1),
    # beta up to 6: the dE = 4 threshold is zero (exact 64-bit threshold form);
    # a power-of-two side (fixed layout) and another one
    dict(L=512, q=5, R=3, beta=linear_betas(6.0, 2), theta=1, seed=51, resample=0),
    dict(L=264, q=5, R=3, beta=linear_betas(6.0, 2), theta=1, seed=52, resample=1),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"L{c['L']}q{c['q']}")
def test_large_lattice_parity(ctx, case):
    got, want = _both(ctx, **case)
    _compare(got, want)


def test_largest_lattice_4096(ctx):
    case = dict(L=4096, q=10, R=2, beta=linear_betas(1.4, 1), theta=1, seed=46, resample=1)
    got, want = _both(ctx, outputs=pa.OUT_FINAL | pa.OUT_MAG | pa.OUT_DIGEST, **case)
    _compare(got, want)


def test_large_lattice_stepwise_and_resume(ctx):
    """Step by step against orc_step from the device's own previous state, then
    a reload of step 2 continues bit-identically."""
    kw = dict(L=384, q=10, R=12, beta=linear_betas(1.6, 4), theta=2, seed=47, resample=0)
    d = pa.Desc(outputs=pa.OUT_FINAL, **kw)
    od = oracle.Desc(**kw)
    _, _, Kb = oracle.plan(od)
    run = pa.Run(ctx, d)
    prev = run.read()
    saved = None
    for i in range(1, d.K):
        run.advance(1)
        cur = run.read()
        spins, E, anc = oracle.step(od, i, Kb, prev["spins"], prev["E"], cur["R_cur"])
        assert (cur["anc"] == anc).all()
        assert (cur["E"] == E).all()
        assert (cur["spins"] == spins).all()
        if i == 2:
            saved = cur
        prev = cur
    full = run.finish()
    run2 = pa.Run(ctx, d)
    run2.load(2, saved["spins"], full["minus_beta_F"][2])
    run2.advance(d.K - 1 - 2)
    res = run2.finish()
    assert (res["final_spins"] == full["final_spins"]).all()
    np.testing.assert_allclose(res["minus_beta_F"][2:], full["minus_beta_F"][2:], rtol=1e-12)


def test_batch_mixing_tiled_and_lds_runs(ctx):
    cases = [CASES[0], dict(L=16, q=8, R=300, beta=linear_betas(1.3, 3), theta=2, seed=48, resample=0),
             CASES[4]]
    descs = [pa.Desc(outputs=ALL, **c) for c in cases]
    got = pa.pa_run_batch(ctx, descs)
    for c, d, g in zip(cases, descs, got):
        _compare(g, pa.pa_run(ctx, d))


def test_tiled_runs_in_graphs_and_serving(ctx):
    """A tiled run inside a replayed HIP graph and inside the serving loop
    gives the results of pa_run."""
    import torch
    cases = [CASES[0], dict(L=16, q=8, R=300, beta=linear_betas(1.3, 3), theta=2, seed=49, resample=0)]
    descs = [pa.Desc(outputs=pa.OUT_FINAL | pa.OUT_MAG, **c) for c in cases]
    single = [pa.pa_run(ctx, d) for d in descs]
    ws = torch.empty(pa.pa_plan_batch(descs), dtype=torch.uint8, device="cuda:0")
    ctx.set_graphs(True)
    try:
        for rep in range(2):
            for g, s in zip(pa.pa_run_batch(ctx, descs, workspace=ws), single):
                _compare(g, s)
            torch.cuda.synchronize()
    finally:
        ctx.set_graphs(False)
    server = pa.Server(ctx, arena_bytes=256 << 20, max_slots=4)
    try:
        tickets = [server.submit(d) for d in descs]
        for t, s in zip(tickets, single):
            got, _ = server.wait(t)
            _compare(got, s)
    finally:
        server.stop()


def test_tiled_previous_population_is_kept(ctx):
    """After a step the previous population (read_slots previous=True) is the
    population before the step: the tiled launches never write it."""
    kw = dict(L=320, q=6, R=6, beta=linear_betas(1.2, 2), theta=3, seed=50, resample=0)
    run = pa.Run(ctx, pa.Desc(**kw))
    before = run.read()["spins"]
    run.advance(1)
    slots = np.arange(before.shape[0], dtype=np.uint32)
    assert (run.read_slots(slots, previous=True) == before).all()
    run.finish()
    cur, cand = ctx.get_lanes(512)
    assert cur == 0 and cand == []
