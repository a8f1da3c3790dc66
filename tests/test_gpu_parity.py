"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bar: spins, energies, histograms, copy numbers, ancestors and population sizes
bit-exact; the FP64 estimators ln Q and -beta F within 1e-12 relative (the
device sums the histogram terms in a different order than the oracle; every
term and the logarithms are the same IEEE operations, so the difference is a
few ulps of the sum); E-bar exact (one correctly rounded division of the same
integers).
"""
import numpy as np
import pytest

import oracle
import paper_1704_01888_amd as pa

pytestmark = pytest.mark.gpu

RTOL = 1e-12


def lin_beta(bmax, n):
    return np.array([bmax * i / n for i in range(n + 1)])


@pytest.fixture(scope="module")
def ctx():
    c = pa.Context(0)
    yield c
    c.close()


def _both(ctx, hist=True, final=True, **kw):
    outputs = (pa.OUT_HIST if hist else 0) | (pa.OUT_FINAL if final else 0) | pa.OUT_DIGEST
    print(f"\ncase: {kw.get('L')}x{kw.get('L')} q={kw.get('q')} R={kw.get('R')} "
          f"K={len(kw['beta'])} theta={kw.get('theta')} resample={kw.get('resample', 0)} "
          f"init={kw.get('init', 0)}", flush=True)
    got = pa.pa_run(ctx, pa.Desc(outputs=outputs, **kw))
    want = oracle.run(oracle.Desc(**kw), hist=hist, final=final, digest=True)
    return got, want


def _compare(got, want, hist=True, final=True):
    assert (got["R_i"] == want["R_i"]).all()
    assert (got["E_sum"] == want["E_sum"]).all()
    assert (got["E_mean"] == want["E_mean"]).all()
    assert (got["digest"] == want["digest"]).all()
    if hist:
        assert (got["hist"] == want["hist"]).all()
    if final:
        assert (got["last_anc"] == want["last_anc"]).all()
        assert (got["final_E"] == want["final_E"]).all()
        assert (got["final_spins"] == want["final_spins"]).all()
    np.testing.assert_allclose(got["lnQ"], want["lnQ"], rtol=RTOL, atol=1e-13)
    np.testing.assert_allclose(got["minus_beta_F"], want["minus_beta_F"], rtol=RTOL, atol=0)


FULL_CASES = [
    # 8x8, q=8, R=1000, 200 equal steps to beta = 1.6, theta = 10, multinomial, seed 1
    dict(L=8, q=8, R=1000, beta=lin_beta(1.6, 200), theta=10, seed=1, resample=1),
    dict(L=16, q=10, R=1500, beta=lin_beta(1.6, 60), theta=5, seed=2, resample=0),
    dict(L=4, q=3, R=777, beta=lin_beta(1.6, 30), theta=3, seed=3, resample=0),
    dict(L=12, q=5, R=501, beta=lin_beta(1.2, 20), theta=4, seed=4, resample=1),
    dict(L=20, q=6, R=300, beta=lin_beta(1.3, 12), theta=3, seed=5, resample=0),
    dict(L=24, q=20, R=257, beta=lin_beta(1.9, 10), theta=2, seed=6, resample=0),
    dict(L=48, q=8, R=130, beta=lin_beta(1.4, 6), theta=2, seed=7, resample=0),
    dict(L=64, q=10, R=70, beta=lin_beta(1.5, 5), theta=2, seed=8, resample=1),
    dict(L=128, q=10, R=21, beta=lin_beta(1.6, 3), theta=2, seed=9, resample=0),
    dict(L=32, q=2, R=400, beta=lin_beta(1.0, 10), theta=3, seed=2**33 + 7, resample=0),
    dict(L=8, q=255, R=100, beta=lin_beta(2.0, 8), theta=3, seed=11, resample=0),
    dict(L=8, q=4, R=1, beta=lin_beta(1.0, 5), theta=3, seed=12, resample=1),
    # beta up to 6: the dE = 4 threshold is zero (exact 64-bit threshold form)
    dict(L=16, q=4, R=300, beta=lin_beta(6.0, 6), theta=2, seed=14, resample=1),
    dict(L=12, q=3, R=200, beta=lin_beta(6.0, 4), theta=2, seed=15, resample=0),
    # the draws' search: weights exp(-dbeta dE) with dbeta = 1 over an energy spread of
    # about a hundred put the cumulative weights far from linear, so the window around
    # x R / 2^64 fails its check and all replicas are searched; many small steps keep
    # the weights even and the window holds
    dict(L=8, q=10, R=4000, beta=lin_beta(4.0, 4), theta=2, seed=16, resample=1),
    dict(L=8, q=10, R=5000, beta=lin_beta(1.6, 40), theta=2, seed=17, resample=0),
]


@pytest.mark.parametrize("case", FULL_CASES, ids=lambda c: f"L{c['L']}q{c['q']}R{c['R']}")
def test_full_run_parity(ctx, case):
    got, want = _both(ctx, **case)
    _compare(got, want)


def test_lattice_256(ctx):
    """Largest lattice of the paper (Table I): one 64 KB replica per workgroup."""
    case = dict(L=256, q=8, R=5, beta=lin_beta(1.3, 2), theta=1, seed=13, resample=0)
    got, want = _both(ctx, **case)
    _compare(got, want)


def test_heating_from_ground_states(ctx):
    """Sec. 5 eq. (6) start and a negative dbeta schedule (E_ref = max E)."""
    case = dict(L=16, q=6, R=400, beta=lin_beta(3.0, 30)[::-1].copy(), theta=3, seed=14,
                resample=0, init=1)
    got, want = _both(ctx, **case)
    _compare(got, want)


def test_resampling_off(ctx):
    case = dict(L=16, q=10, R=300, beta=lin_beta(1.6, 10), theta=3, seed=15, resample=2)
    got, want = _both(ctx, **case)
    _compare(got, want)


def test_theta_zero_and_single_temperature(ctx):
    got, want = _both(ctx, L=8, q=8, R=333, beta=lin_beta(1.0, 6), theta=0, seed=16, resample=0)
    _compare(got, want)
    got, want = _both(ctx, L=8, q=8, R=333, beta=np.array([0.0]), theta=5, seed=16, resample=0)
    _compare(got, want)


def test_zero_beta_steps(ctx):
    """dbeta = 0 gives ln Q = 0 exactly on the device too."""
    got, want = _both(ctx, L=8, q=3, R=200, beta=np.zeros(4), theta=2, seed=17, resample=0)
    _compare(got, want)
    assert (got["lnQ"] == 0.0).all()


def test_stepwise_state_parity(ctx):
    """Each step of a run against orc_step from the device's own previous state:
    ancestors, copy numbers, spins and energies bit-exact."""
    kw = dict(L=32, q=10, R=3000, beta=lin_beta(1.6, 40), theta=4, seed=18, resample=0)
    d = pa.Desc(**kw)
    od = oracle.Desc(**kw)
    _, _, Kb = oracle.plan(od)
    run = pa.Run(ctx, d)
    prev = run.read()
    for i in range(1, 6):
        run.advance(1)
        cur = run.read()
        assert cur["step"] == i
        spins, E, anc = oracle.step(od, i, Kb, prev["spins"], prev["E"], cur["R_cur"])
        assert (cur["anc"] == anc).all()
        assert (cur["counts"] == np.bincount(anc, minlength=prev["R_cur"])).all()
        assert (cur["E"] == E).all()
        assert (cur["spins"] == spins).all()
        prev = cur
    run.finish()


def test_load_resume_is_bit_identical(ctx):
    """Checkpoint/resume: a run reloaded from its step-5 population continues
    exactly like the uninterrupted run (every random number is a function of
    logical indices only)."""
    kw = dict(L=16, q=8, R=800, beta=lin_beta(1.4, 12), theta=3, seed=19, resample=0,
              outputs=pa.OUT_FINAL)
    d = pa.Desc(**kw)
    full = pa.pa_run(ctx, d)
    run = pa.Run(ctx, d)
    run.advance(5)
    st = run.read()
    partial = run.finish()
    run2 = pa.Run(ctx, d)
    run2.load(5, st["spins"], partial["minus_beta_F"][5])
    run2.advance(d.K - 1 - 5)
    res = run2.finish()
    assert (res["final_spins"] == full["final_spins"]).all()
    assert (res["E_sum"][5:] == full["E_sum"][5:]).all()
    np.testing.assert_allclose(res["minus_beta_F"][5:], full["minus_beta_F"][5:], rtol=RTOL)


def test_checkpoint_file_mid_run(ctx, tmp_path):
    """A checkpoint file written mid-run (population, step, -beta F of that
    step, run description) resumes in a new run that finishes bit-identically
    to the original, which continues after writing it."""
    kw = dict(L=32, q=10, R=900, beta=lin_beta(1.5, 10), theta=2, seed=23, resample=0,
              outputs=pa.OUT_FINAL | pa.OUT_HIST | pa.OUT_DIGEST)
    d = pa.Desc(**kw)
    run = pa.Run(ctx, d)
    run.advance(4)
    step, mbf = run.free_energy()
    assert step == 4
    path = tmp_path / "ckpt.npz"
    run.checkpoint(path)
    run.advance(d.K - 1 - 4)
    full = run.finish()
    assert full["minus_beta_F"][4] == mbf
    res_run = pa.Run.resume(ctx, path)
    res_run.advance(d.K - 1 - 4)
    res = res_run.finish()
    assert (res["final_spins"] == full["final_spins"]).all()
    for k in ("R_i", "E_sum", "hist", "digest"):
        assert (res[k][4:] == full[k][4:]).all(), k
    np.testing.assert_allclose(res["minus_beta_F"][4:], full["minus_beta_F"][4:], rtol=RTOL)


def _sampled_full_size_step(ctx, kw, n_steps, n_samples, seed):
    """Full-size run: every step's ancestors bit-exact against the oracle's
    resampling of the device energies; a random sample of replicas re-swept by
    the oracle from the device's previous population, bit-exact."""
    d = pa.Desc(**kw)
    od = oracle.Desc(**kw)
    _, _, Kb = oracle.plan(od)
    rng = np.random.default_rng(seed)
    run = pa.Run(ctx, d)
    prev = run.read(spins=False, anc=False, counts=False)
    for i in range(1, n_steps + 1):
        run.advance(1)
        cur = run.read(spins=False)
        r, anc, _ = oracle.resample(od, i, Kb, prev["E"], cur["R_cur"])
        assert (cur["anc"] == anc).all()
        assert (cur["counts"] == r).all()
        slots = np.sort(rng.choice(cur["R_cur"], size=n_samples, replace=False)).astype(np.uint32)
        new = run.read_slots(slots)
        old = run.read_slots(anc[slots], previous=True)
        for j, k in enumerate(slots):
            want = oracle.sweep_replica(od, i, int(k), old[j])
            assert (new[j] == want).all(), f"step {i} slot {k}"
            assert cur["E"][k] == oracle.energy(d.L, want)
        prev = cur
    run.finish()


def test_full_size_32x32_q10(ctx):
    """32x32, q=10, R=2*10^4, 400 steps to beta = 1.6, theta = 10, Poisson, seed 2:
    the first steps at full size, sampled."""
    kw = dict(L=32, q=10, R=20000, beta=lin_beta(1.6, 400), theta=10, seed=2, resample=0)
    _sampled_full_size_step(ctx, kw, n_steps=3, n_samples=64, seed=1)
