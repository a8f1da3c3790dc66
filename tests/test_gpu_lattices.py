"""Lattice sides that are even but not multiples of 4 (L = 2, 6, 10, 18, ...)
on the device: the byte kernel, against the oracle.

The model (Sec. 3, eq. (3)) is any periodic L x L lattice; the checkerboard
update needs L even.  For L = 2 (mod 4) a row holds an odd number of sites of
each colour, so the pairs of sites that share a Philox block straddle rows.
Bar: spins, energies, histograms, copy numbers, ancestors, digests and M~
bit-exact; ln Q and -beta F within 1e-12 relative.
"""
import numpy as np
import pytest

import exact
import oracle
import paper_1704_01888_amd as pa
from paper_1704_01888_amd.workloads import linear_betas
from test_oracle_pins import one_sweep_transition_counts, transitions_match

pytestmark = pytest.mark.gpu

RTOL = 1e-12


@pytest.fixture(scope="module")
def ctx():
    c = pa.Context(0)
    yield c
    c.close()


def _compare(got, want, mag=False):
    for k in ("R_i", "E_sum", "E_mean", "digest", "hist", "final_spins", "final_E", "last_anc"):
        assert (got[k] == want[k]).all(), k
    if mag:
        for k in ("Mt_sum", "M_mean", "mhist", "width_e", "width_m"):
            assert (got[k] == want[k]).all(), k
    np.testing.assert_allclose(got["lnQ"], want["lnQ"], rtol=RTOL, atol=1e-13)
    np.testing.assert_allclose(got["minus_beta_F"], want["minus_beta_F"], rtol=RTOL, atol=0)


CASES = [
    dict(L=2, q=2, R=500, beta=linear_betas(2.0, 20), theta=3, seed=1, resample=0),
    dict(L=2, q=3, R=777, beta=linear_betas(1.5, 12), theta=2, seed=2, resample=1),
    dict(L=2, q=20, R=300, beta=linear_betas(3.0, 8), theta=4, seed=3, resample=0),
    dict(L=6, q=3, R=1000, beta=linear_betas(1.6, 30), theta=5, seed=4, resample=0),
    dict(L=6, q=255, R=100, beta=linear_betas(2.0, 6), theta=2, seed=5, resample=1),
    dict(L=10, q=5, R=1500, beta=linear_betas(1.4, 25), theta=4, seed=6, resample=0),
    dict(L=10, q=10, R=400, beta=linear_betas(6.0, 5), theta=2, seed=7, resample=1),
    dict(L=18, q=8, R=600, beta=linear_betas(1.5, 15), theta=3, seed=8, resample=0),
    dict(L=30, q=6, R=200, beta=linear_betas(1.3, 6), theta=2, seed=9, resample=2),
    dict(L=66, q=10, R=65, beta=linear_betas(1.5, 4), theta=2, seed=10, resample=0),
    dict(L=254, q=8, R=5, beta=linear_betas(1.3, 2), theta=1, seed=11, resample=0),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"L{c['L']}q{c['q']}R{c['R']}")
def test_full_run_parity_L_2_mod_4(ctx, case):
    print(f"\ncase: {case['L']}x{case['L']} q={case['q']} R={case['R']} K={len(case['beta'])}",
          flush=True)
    mag = case["L"] <= 18
    outs = pa.OUT_HIST | pa.OUT_FINAL | pa.OUT_DIGEST | (pa.OUT_MAG | pa.OUT_WIDTHS if mag else 0)
    got = pa.pa_run(ctx, pa.Desc(outputs=outs, **case))
    want = oracle.run(oracle.Desc(**case), hist=True, final=True, digest=True,
                      magnetisation=mag, widths=mag)
    _compare(got, want, mag)


def test_heating_from_ground_states_L6(ctx):
    case = dict(L=6, q=6, R=400, beta=linear_betas(3.0, 20)[::-1].copy(), theta=3, seed=12,
                resample=0, init=1)
    got = pa.pa_run(ctx, pa.Desc(outputs=pa.OUT_HIST | pa.OUT_FINAL | pa.OUT_DIGEST, **case))
    want = oracle.run(oracle.Desc(**case), hist=True, final=True, digest=True)
    _compare(got, want)


def test_batch_with_L_2_mod_4_equals_separate_runs(ctx):
    """Byte-kernel runs share batched launches with dword-kernel runs."""
    cases = [CASES[3], CASES[5], dict(L=8, q=8, R=300, beta=linear_betas(1.6, 20), theta=3,
                                      seed=13, resample=1), CASES[0]]
    descs = [pa.Desc(outputs=pa.OUT_HIST | pa.OUT_FINAL | pa.OUT_DIGEST, **c) for c in cases]
    for d, g in zip(descs, pa.pa_run_batch(ctx, descs)):
        s = pa.pa_run(ctx, d)
        for k in ("R_i", "E_sum", "digest", "hist", "final_spins", "last_anc"):
            assert (g[k] == s[k]).all(), k


def test_one_sweep_transitions_L2_on_the_device(ctx):
    """The 2 x 2, q = 3 lattice: every one of the 81 configurations loaded 2000
    times (pa_run_load), one sweep at beta = 0.7 with resampling off.  Every
    replica equals the oracle's sweep of the same slot, and the configurations
    reached follow the exact one-sweep transition matrix, whose stationary
    vector is the Boltzmann distribution (the oracle pins hold the matrix
    itself to it)."""
    q, beta, reps = 3, 0.7, 2000
    betas = np.array([0.0, beta, beta])
    confs = np.array([[a // 27, (a // 9) % 3, (a // 3) % 3, a % 3] for a in range(81)], np.uint8)
    start = np.repeat(confs, reps, axis=0)
    d = pa.Desc(2, q, len(start), betas, 1, seed=31, resample=pa.RESAMPLE_NONE)
    run = pa.Run(ctx, d)
    run.load(1, start, 0.0)
    run.advance(1)
    end = run.read(E=False, anc=False, counts=False)["spins"]
    run.finish()
    od = oracle.Desc(2, q, len(start), betas, 1, seed=31, resample=oracle.RESAMPLE_NONE)
    T = oracle.thresholds(beta)
    for k in range(0, len(start), 97):
        assert (end[k] == oracle.one_sweep(od, 2, 0, k, T, start[k])).all(), k
    counts = one_sweep_transition_counts(lambda k, c: end[k], q, reps)
    P, _ = exact.one_sweep_matrix_L2(q, beta)
    assert transitions_match(counts, P) > 1e-4
