"""Magnetisation (eq. (4)-(5)) and histogram widths (Sec. 4) of the HIP path
against the CPU oracle, through the C ABI.

Bar: the sums of M~, the M~ histograms and M-bar bit-exact (M-bar is the same
IEEE expression of the same integers on both sides); the widths bit-exact (the
same bin counts enter the same sequence of IEEE operations)."""
import numpy as np
import pytest

import oracle
import paper_1704_01888_amd as pa
from paper_1704_01888_amd.workloads import linear_betas

pytestmark = pytest.mark.gpu

ALL = pa.OUT_HIST | pa.OUT_MAG | pa.OUT_WIDTHS


@pytest.fixture(scope="module")
def ctx():
    c = pa.Context(0)
    yield c
    c.close()


def _check_same(got, want):
    for k in ("R_i", "E_sum", "hist", "Mt_sum", "mhist"):
        assert (got[k] == want[k]).all(), k
    for k in ("E_mean", "M_mean", "width_e", "width_m"):
        assert (got[k] == want[k]).all(), (k, np.nonzero(got[k] != want[k]))


def _oracle(case):
    return oracle.run(oracle.Desc(**case), hist=True, magnetisation=True, widths=True)


CASES = [
    # one replica per 8 lanes, unit bins
    dict(L=8, q=8, R=500, beta=linear_betas(1.6, 30), theta=5, seed=31, resample=0),
    # several bins per level group, multinomial
    dict(L=16, q=6, R=700, beta=linear_betas(1.5, 20), theta=4, seed=32, resample=1, bin_e=3, bin_m=2),
    # generic lattice kernel
    dict(L=12, q=3, R=300, beta=linear_betas(1.2, 15), theta=3, seed=33, resample=0, bin_e=2),
    dict(L=32, q=10, R=300, beta=linear_betas(1.6, 12), theta=3, seed=34, resample=0, bin_e=4, bin_m=4),
    # one wave per replica, q beyond the 7-bit fast path
    dict(L=64, q=200, R=40, beta=linear_betas(2.0, 5), theta=2, seed=35, resample=0, bin_e=5, bin_m=7),
    # several waves per replica (per-state counters in LDS)
    dict(L=128, q=255, R=12, beta=linear_betas(1.5, 3), theta=1, seed=36, resample=0, bin_e=9, bin_m=3),
    dict(L=96, q=10, R=10, beta=linear_betas(1.5, 3), theta=1, seed=37, resample=0),
    # heating from ground states (eq. (6)): M~ = N at the start
    dict(L=16, q=10, R=400, beta=linear_betas(3.0, 20)[::-1].copy(), theta=3, seed=38, resample=0,
         init=1, bin_e=2, bin_m=2),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"L{c['L']}q{c['q']}R{c['R']}")
def test_magnetisation_and_widths_parity(ctx, case):
    print(f"\ncase: L={case['L']} q={case['q']} R={case['R']} K={len(case['beta'])}", flush=True)
    got = pa.pa_run(ctx, pa.Desc(outputs=ALL, **case))
    _check_same(got, _oracle(case))


def test_multiwave_replicas_of_64x64(ctx):
    """64 x 64 with each candidate of several waves per replica (per-state
    counts, bond and digest sums across waves)."""
    _, cand = ctx.get_lanes(64)
    multi = [g for g in cand if g > 64]
    assert multi
    case = dict(L=64, q=8, R=50, beta=linear_betas(1.5, 4), theta=2, seed=39, resample=0, bin_e=2)
    want = _oracle(case)
    try:
        for g in multi:
            ctx.set_lanes(64, g)
            _check_same(pa.pa_run(ctx, pa.Desc(outputs=ALL, **case)), want)
    finally:
        ctx.set_lanes(64, 0)


def test_magnetisation_without_stored_histograms(ctx):
    """PA_OUT_MAG | PA_OUT_WIDTHS without PA_OUT_HIST: two histogram buffers
    are reused across the steps; the statistics still match."""
    case = dict(L=16, q=8, R=600, beta=linear_betas(1.6, 25), theta=3, seed=40, resample=0, bin_m=2)
    got = pa.pa_run(ctx, pa.Desc(outputs=pa.OUT_MAG | pa.OUT_WIDTHS, **case))
    want = _oracle(case)
    for k in ("Mt_sum", "M_mean", "width_e", "width_m", "E_sum"):
        assert (got[k] == want[k]).all(), k
    assert "mhist" not in got and "hist" not in got


def test_batched_runs_carry_the_observables(ctx):
    cases = [CASES[0], CASES[1], CASES[3], CASES[7]]
    descs = [pa.Desc(outputs=ALL, **c) for c in cases]
    got = pa.pa_run_batch(ctx, descs)
    for c, g in zip(cases, got):
        _check_same(g, _oracle(c))
