"""Parity with the oracle at the full sizes of the five benchmark workloads.

  8x8, q=8, R=1000, multinomial: the whole run, in test_gpu_parity.FULL_CASES;
  32x32, q=10, R=2e4, 400 steps: the whole run, every step;
  128x128, q=10, R=2e5, 500 steps, theta=20: steps 0 and 1 whole (every spin
      of every replica, through the population digest), the last step sampled;
  the mixed batch of 20 runs (L 16..64, R 1e4..1e5, 300 steps): batched =
      separate runs at every step, the smallest run whole against the oracle,
      the first and last steps of the largest-L and largest-R runs sampled;
  the serving stream: 24 requests at their own sizes through the server =
      alone at every step, the three smallest whole against the oracle, the
      first and last steps of the largest sampled.

"Whole" compares per step: population size, the exact energy sum and mean,
the energy histogram, the population digest (every spin of every replica in
every slot), ln Q and -beta F (1e-12 relative), and at the end the final
population, energies and ancestors.  "Sampled" compares all ancestors and copy
numbers of the step with the oracle's resampling of the device's previous
energies, and re-sweeps a random sample of new replicas from their ancestors
in the oracle (spins and energies bit-exact).  The method is Sec. 2 of the
paper (steps 2-4, eq. (1)-(2)).
"""
import numpy as np
import pytest

import oracle
import paper_1704_01888_amd as pa
from paper_1704_01888_amd import workloads

pytestmark = pytest.mark.gpu

RTOL = 1e-12


@pytest.fixture(scope="module")
def ctx():
    c = pa.Context(0)
    yield c
    c.close()


def _note(msg):
    print(f"\n{msg}", flush=True)


def _compare_whole(got, want, steps=None, final=True):
    sl = slice(None) if steps is None else slice(0, steps)
    for k in ("R_i", "E_sum", "E_mean", "digest", "hist"):
        assert (got[k][sl] == want[k][sl]).all(), k
    np.testing.assert_allclose(got["lnQ"][sl], want["lnQ"][sl], rtol=RTOL, atol=1e-13)
    np.testing.assert_allclose(got["minus_beta_F"][sl], want["minus_beta_F"][sl], rtol=RTOL, atol=0)
    if final:
        for k in ("final_spins", "final_E", "last_anc"):
            assert (got[k] == want[k]).all(), k


def _same_runs(a, b):
    for k in ("R_i", "E_sum", "E_mean", "digest", "hist"):
        assert (a[k] == b[k]).all(), k
    np.testing.assert_allclose(a["lnQ"], b["lnQ"], rtol=RTOL, atol=1e-13)
    np.testing.assert_allclose(a["minus_beta_F"], b["minus_beta_F"], rtol=RTOL, atol=0)


def _check_step(run, od, Kb, i, prev_E, rng, n_samples):
    """Step i of `run` (just advanced) against the oracle: every ancestor and
    copy number from the device's energies of step i-1, and n_samples new
    replicas re-swept from their ancestors."""
    cur = run.read(spins=False)
    assert cur["step"] == i
    r, anc, _ = oracle.resample(od, i, Kb, prev_E, cur["R_cur"])
    assert (cur["anc"] == anc).all(), f"step {i}: ancestors"
    assert (cur["counts"] == r).all(), f"step {i}: copy numbers"
    slots = np.sort(rng.choice(cur["R_cur"], size=min(n_samples, cur["R_cur"]),
                               replace=False)).astype(np.uint32)
    new = run.read_slots(slots)
    old = run.read_slots(anc[slots], previous=True)
    for j, k in enumerate(slots):
        want = oracle.sweep_replica(od, i, int(k), old[j])
        assert (new[j] == want).all(), f"step {i} slot {k}"
        assert cur["E"][k] == oracle.energy(od.L, want), f"step {i} slot {k}: energy"
    return cur["E"]


def _sampled_first_and_last(ctx, kw, rng, n_samples):
    """Steps 1 and K-1 of a run sampled against the oracle (the device advances
    through the steps between)."""
    d = pa.Desc(**kw)
    od = oracle.Desc(**kw)
    _, _, Kb = oracle.plan(od)
    run = pa.Run(ctx, d)
    E = run.read(spins=False, anc=False, counts=False)["E"]
    run.advance(1)
    _check_step(run, od, Kb, 1, E, rng, n_samples)
    K = d.K
    if K > 3:
        run.advance(K - 3)
        E = run.read(spins=False, anc=False, counts=False)["E"]
        run.advance(1)
        _check_step(run, od, Kb, K - 1, E, rng, n_samples)
    run.finish()


@pytest.mark.timeout(600)
def test_32x32_q10_R20000_every_step(ctx):
    """32x32, q=10, R=2e4, 400 equal steps to beta = 1.6, theta=10, Poisson,
    seed 2: the whole run, all 401 populations."""
    kw = dict(L=32, q=10, R=20000, beta=workloads.linear_betas(1.6, 400), theta=10, seed=2,
              resample=0)
    _note("32x32 q=10 R=20000 K=401 theta=10 seed=2: whole run")
    got = pa.pa_run(ctx, pa.Desc(outputs=pa.OUT_HIST | pa.OUT_DIGEST | pa.OUT_FINAL, **kw))
    want = oracle.run(oracle.Desc(**kw), hist=True, final=True, digest=True)
    _compare_whole(got, want)


RUN_128 = dict(L=128, q=10, R=200000, beta=workloads.linear_betas(1.6, 500), theta=20, seed=4,
               resample=0)


@pytest.mark.timeout(600)
def test_128x128_q10_R200000_first_steps_whole(ctx):
    """128x128, q=10, R=2e5, theta=20, Poisson, seed 4: the initial population
    and the population after the first step (resampling + 20 sweeps, 6.6e10
    attempts), every spin, against the oracle stepping from its own initial
    population."""
    _note("128x128 q=10 R=200000 theta=20 seed=4: steps 0 and 1 whole")
    d = pa.Desc(outputs=pa.OUT_HIST | pa.OUT_DIGEST, **RUN_128)
    run = pa.Run(ctx, d)
    run.advance(1)
    got = run.finish()
    kw2 = dict(RUN_128, beta=RUN_128["beta"][:2])
    # the truncated schedule has the same weight precision (R_cap rounds to 2^18)
    assert oracle.plan(oracle.Desc(**kw2))[2] == oracle.plan(oracle.Desc(**RUN_128))[2]
    want = oracle.run(oracle.Desc(**kw2), hist=True, digest=True)
    _compare_whole(got, want, steps=2, final=False)


@pytest.mark.timeout(600)
def test_128x128_q10_R200000_last_step_sampled(ctx):
    """The same run's last step (499 -> 500, beta 1.5968 -> 1.6), reached on the
    device: all 2e5 ancestors and copy numbers, and 256 re-swept replicas."""
    _note("128x128 q=10 R=200000 theta=20 seed=4: step 500 sampled")
    d = pa.Desc(**RUN_128)
    od = oracle.Desc(**RUN_128)
    _, _, Kb = oracle.plan(od)
    run = pa.Run(ctx, d)
    run.advance(d.K - 2)
    E = run.read(spins=False, anc=False, counts=False)["E"]
    run.advance(1)
    _check_step(run, od, Kb, d.K - 1, E, np.random.default_rng(499), 256)
    run.finish()


MIXED = workloads.mixed_runs(20)


@pytest.mark.timeout(600)
def test_mixed_batch_of_20_equals_separate_runs(ctx):
    """The 20 runs (L in {16,24,32,48,64}, q in {5,6,8,10,20}, R in [1e4, 1e5],
    300 steps, seeds 3000-3019) as one batch and one by one: every output of
    every step identical."""
    _note("mixed batch: 20 runs batched vs separate, every step")
    outs = pa.OUT_HIST | pa.OUT_DIGEST | pa.OUT_FINAL
    descs = [pa.Desc(outputs=outs, **kw) for kw in MIXED]
    batched = pa.pa_run_batch(ctx, descs)
    for r, d in enumerate(descs):
        single = pa.pa_run(ctx, d)
        _same_runs(batched[r], single)
        for k in ("final_spins", "final_E", "last_anc"):
            assert (batched[r][k] == single[k]).all(), (r, k)
    # the run with the least work, whole against the oracle
    work = [kw["theta"] * kw["L"] ** 2 * kw["R"] for kw in MIXED]
    r = int(np.argmin(work))
    _note(f"mixed batch: run {r} (L={MIXED[r]['L']} q={MIXED[r]['q']} R={MIXED[r]['R']}) "
          "whole against the oracle")
    want = oracle.run(oracle.Desc(**MIXED[r]), hist=True, final=True, digest=True)
    _compare_whole(batched[r], want)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("which", ["largest_L", "largest_R"])
def test_mixed_batch_sampled_first_and_last_steps(ctx, which):
    if which == "largest_L":
        r = max(range(len(MIXED)), key=lambda i: (MIXED[i]["L"], MIXED[i]["R"]))
    else:
        r = max(range(len(MIXED)), key=lambda i: MIXED[i]["R"])
    kw = MIXED[r]
    _note(f"mixed batch run {r}: L={kw['L']} q={kw['q']} R={kw['R']}: steps 1 and 300 sampled")
    _sampled_first_and_last(ctx, kw, np.random.default_rng(r), 96)


SERVED = workloads.serving_requests(500)[:24]


@pytest.mark.timeout(600)
def test_serving_stream_requests_equal_alone_and_oracle(ctx):
    """The first 24 requests of the 500-request stream (L in {16..128}, R up to
    1e5, 200-500 steps) through the server with up to 8 in flight: each result
    equals the same run alone at every step; the three with the least work
    equal the oracle's whole run."""
    _note("serving: 24 requests of the stream at their own sizes")
    outs = pa.OUT_HIST | pa.OUT_DIGEST | pa.OUT_FINAL
    descs = [pa.Desc(outputs=outs, **kw) for kw in SERVED]
    sv = pa.Server(ctx, arena_bytes=24 << 30, max_slots=8)
    try:
        tickets = [sv.submit(d) for d in descs]
        served = [sv.wait(t)[0] for t in tickets]
    finally:
        sv.stop()
    for k, d in enumerate(descs):
        alone = pa.pa_run(ctx, d)
        _same_runs(served[k], alone)
        for key in ("final_spins", "final_E", "last_anc"):
            assert (served[k][key] == alone[key]).all(), (k, key)
    work = [kw["theta"] * kw["L"] ** 2 * kw["R"] * (len(kw["beta"]) - 1) for kw in SERVED]
    for k in np.argsort(work)[:3]:
        _note(f"serving request {k} whole against the oracle")
        want = oracle.run(oracle.Desc(**SERVED[k]), hist=True, final=True, digest=True)
        _compare_whole(served[k], want)


@pytest.mark.timeout(600)
def test_serving_stream_largest_request_sampled(ctx):
    work = [kw["theta"] * kw["L"] ** 2 * kw["R"] * (len(kw["beta"]) - 1) for kw in SERVED]
    k = int(np.argmax(work))
    kw = SERVED[k]
    _note(f"serving request {k}: L={kw['L']} q={kw['q']} R={kw['R']} K={len(kw['beta'])}: "
          "first and last steps sampled")
    _sampled_first_and_last(ctx, kw, np.random.default_rng(k), 96)
