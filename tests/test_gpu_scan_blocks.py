"""The multi-workgroup weight and count scans against the CPU oracle.

The weight scan C and the count scan of the slot map run one workgroup per
block of replicas; each workgroup sums the elements before its block itself.
Blocks hold one row of 4096 replicas up to 64 blocks and more rows beyond
(R > 262144). The copy counts alternate between two buffers by step parity;
each count-scan launch clears the other buffer over the extent the step before
used, in strides of the launch's blocks. The cases: a population of several
rows per block; a Poisson population fluctuating around one block (4096), so
that the clearing runs past one stride; strongly skewed weights (long runs of
copies in the slot map); a population of three rows per block; populations at
the edges of one 32768-value read (the register-held weights and the bounded
last tile). Bar as for
every parity test:
population sizes, histograms, copy numbers, ancestors, spins and digests
bit-exact, ln Q and -beta F within 1e-12.
"""
import numpy as np
import pytest

import oracle
import paper_1704_01888_amd as pa
from paper_1704_01888_amd.workloads import linear_betas

pytestmark = pytest.mark.gpu

OUT = pa.OUT_HIST | pa.OUT_FINAL | pa.OUT_DIGEST

CASES = [
    # 300000 replicas: 37 blocks of two 4096-rows each
    dict(L=4, q=3, R=300000, beta=linear_betas(1.2, 3), theta=1, seed=61, resample=1),
    dict(L=4, q=5, R=300000, beta=linear_betas(1.4, 3), theta=2, seed=62, resample=0),
    # Poisson around one block: R_i crosses 4096 from step to step
    dict(L=8, q=4, R=4096, beta=linear_betas(1.2, 40), theta=1, seed=63, resample=0),
    # strongly skewed weights (steps of up to 1.5 in beta): one ancestor takes
    # about 14700 of 20000 copies, about 20 take more than 8 (written by the wave)
    dict(L=8, q=3, R=20000, beta=np.array([0.0, 0.5, 1.5, 3.0]), theta=1, seed=64, resample=1),
    dict(L=8, q=3, R=20000, beta=np.array([0.0, 0.5, 1.5, 3.0]), theta=1, seed=64, resample=0),
    # 600000 replicas: 49 blocks of three 4096-rows each
    dict(L=4, q=3, R=600000, beta=linear_betas(1.2, 2), theta=1, seed=65, resample=1),
    # the edges of a one-round read (32 values per thread of 1024): 32768 replicas
    # fill it exactly, with the weights taken from registers; 32769 is one whole
    # read plus one value, the most the general path leaves to its bounded tail;
    # 32766 and 32767 leave two and three values after the last 16-byte load
    dict(L=4, q=3, R=32768, beta=linear_betas(1.2, 3), theta=1, seed=66, resample=1),
    dict(L=4, q=3, R=32769, beta=linear_betas(1.2, 3), theta=1, seed=67, resample=1),
    dict(L=4, q=4, R=32766, beta=linear_betas(1.2, 3), theta=1, seed=68, resample=1),
    dict(L=4, q=4, R=32767, beta=linear_betas(1.2, 3), theta=1, seed=69, resample=1),
]


@pytest.fixture(scope="module")
def ctx():
    c = pa.Context(0)
    yield c
    c.close()


def _compare(got, want):
    for k in ("R_i", "E_sum", "E_mean", "hist", "digest", "last_anc", "final_E", "final_spins"):
        assert (got[k] == want[k]).all(), k
    np.testing.assert_allclose(got["lnQ"], want["lnQ"], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(got["minus_beta_F"], want["minus_beta_F"], rtol=1e-12, atol=0)


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"L{c['L']}R{c['R']}r{c['resample']}b{c['beta'][-1]:g}")
def test_scan_blocks_parity(ctx, case):
    print(f"\ncase: L={case['L']} q={case['q']} R={case['R']} K={len(case['beta'])} "
          f"resample={case['resample']}", flush=True)
    got = pa.pa_run(ctx, pa.Desc(outputs=OUT, **case))
    want = oracle.run(oracle.Desc(**case), hist=True, final=True, digest=True)
    _compare(got, want)
    if case["R"] == 4096:
        # the population did cross the block size in both directions
        assert (want["R_i"] > 4096).any() and (want["R_i"] <= 4096).any()
    if case["beta"][-1] == 3.0:
        assert np.bincount(want["last_anc"]).max() > 1000


def test_scan_blocks_batched(ctx):
    """The same runs in one batched launch sequence give the single-run results."""
    descs = [pa.Desc(outputs=OUT, **c) for c in CASES]
    single = [pa.pa_run(ctx, d) for d in descs]
    for g, s in zip(pa.pa_run_batch(ctx, descs), single):
        _compare(g, s)
