"""Sweep-kernel shapes: every lane-count candidate gives the oracle's results
bit for bit (spins, histograms, magnetisation and digests), and the autotuner
picks one of the candidates. L = 12, 20 and 24 have replicas that span wave
boundaries (barriers between half-sweeps, per-replica sums in LDS); their
populations leave the last workgroup partly idle."""
import numpy as np
import pytest

import oracle
import paper_1704_01888_amd as pa
from paper_1704_01888_amd.workloads import linear_betas

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = pa.Context(0)
    yield c
    c.close()


CASES = {
    4: dict(R=300, q=3), 8: dict(R=500, q=8), 12: dict(R=77, q=4), 16: dict(R=300, q=10),
    20: dict(R=45, q=7), 24: dict(R=37, q=10), 32: dict(R=120, q=6),
    48: dict(R=60, q=5), 64: dict(R=40, q=20), 96: dict(R=20, q=8), 128: dict(R=9, q=10), 192: dict(R=5, q=6),
    256: dict(R=3, q=200),
}


@pytest.mark.parametrize("L", sorted(CASES))
def test_every_lane_choice_matches_oracle(ctx, L):
    kw = dict(L=L, beta=linear_betas(1.5, 4), theta=2, seed=L, resample=0, **CASES[L])
    want = oracle.run(oracle.Desc(**kw), final=True, hist=True, magnetisation=True, digest=True)
    _, cands = ctx.get_lanes(L)
    assert len(cands) >= 1
    try:
        for g in cands:
            ctx.set_lanes(L, g)
            assert ctx.get_lanes(L)[0] == g
            print(f"\nL={L} lanes={g}", flush=True)
            got = pa.pa_run(ctx, pa.Desc(outputs=pa.OUT_FINAL | pa.OUT_HIST | pa.OUT_MAG | pa.OUT_DIGEST, **kw))
            for key in ("final_spins", "final_E", "hist", "Mt_sum", "mhist", "digest"):
                assert (got[key] == want[key]).all(), key
            np.testing.assert_allclose(got["minus_beta_F"], want["minus_beta_F"], rtol=1e-12)
    finally:
        ctx.set_lanes(L, 0)


def test_autotune_picks_a_candidate(ctx):
    for L in (16, 24, 128):
        best, rate = ctx.autotune(L, 10)
        assert best in ctx.get_lanes(L)[1]
        assert ctx.get_lanes(L)[0] == best
        assert rate > 0
        ctx.set_lanes(L, 0)
    with pytest.raises(pa.PAError):
        ctx.set_lanes(16, 7)
