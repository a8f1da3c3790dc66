"""Pins of the CPU oracle against results that do not come from the oracle.

Each test names the passage of the paper (arXiv:1704.01888) it checks, or the
independent result it uses: published known-answer vectors, rocRAND's own
Philox engine, closed forms, exact enumeration / transfer matrix / Kaufman's
finite-torus Ising partition function (tests/exact.py), and statistics with
stated bounds.  CPU only.
"""
import math
import os
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats

import oracle
import exact

HERE = os.path.dirname(os.path.abspath(__file__))


def lin_beta(beta_max, n):
    """beta_i = beta_max * i / n, i = 0..n, computed once in double."""
    return np.array([beta_max * i / n for i in range(n + 1)], dtype=np.float64)


# --------------------------------------------------------------------------
# Philox4x32-10
# --------------------------------------------------------------------------
def test_philox_known_answers():
    """Known-answer vectors published with Random123 (Salmon et al., SC'11)."""
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) >= 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = oracle.philox(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_philox_matches_rocrand_engine():
    """The oracle's Philox against rocRAND's independent header-only engine
    (run on the CPU), on random keys and counters."""
    rng = np.random.default_rng(12345)
    n = 400
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64)
    ctr[:, 1] &= (1 << 30) - 1   # rocRAND addresses counter words 0,1 as a 64-bit offset / 4
    key = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64)
    with tempfile.TemporaryDirectory() as td:
        exe = os.path.join(td, "rr")
        subprocess.run(["hipcc", "-O1", "-x", "hip", "--offload-arch=gfx950", "-o", exe,
                        os.path.join(HERE, "rocrand_philox_ref.cpp")], check=True,
                       capture_output=True)
        inp = "\n".join(" ".join(f"{int(x):x}" for x in list(c) + list(k))
                        for c, k in zip(ctr, key)) + "\n"
        res = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True)
    lines = res.stdout.strip().split("\n")
    assert len(lines) == n
    for c, k, line in zip(ctr, key, lines):
        want = [int(x, 16) for x in line.split()]
        got = [int(x) for x in oracle.philox(c, k)]
        assert got == want


# --------------------------------------------------------------------------
# Energy, eq. (3)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("L", [2, 4, 8, 32])
def test_energy_closed_forms(L):
    """All spins equal: E_0 = -2N (Sec. 6).  A two-colouring of the
    periodic lattice (L even) satisfies no bond: E = 0."""
    N = L * L
    for a in (0, 3, 7):
        assert oracle.energy(L, np.full(N, a, np.uint8)) == -2 * N
    cb = np.array([(x + y) % 2 for y in range(L) for x in range(L)], np.uint8)
    assert oracle.energy(L, cb) == 0
    assert oracle.energy(L, cb * 5 + 2) == 0


@pytest.mark.parametrize("L,q", [(2, 3), (2, 4), (4, 2)])
def test_energy_density_of_states(L, q):
    """Histogram of orc_energy over every configuration equals the density of
    states of the transfer matrix (and sums to q^N, Z at beta = 0)."""
    g_oracle = exact.dos_brute(L, q, energy=lambda s: oracle.energy(L, s))
    g_tm = exact.dos_transfer(L, q)
    assert (g_oracle == g_tm).all()
    assert g_tm.sum() == q ** (L * L)


# --------------------------------------------------------------------------
# Step 1: the initial population
# --------------------------------------------------------------------------
def test_random_init_statistics():
    """At beta_0 = 0 spins are i.i.d. uniform; the 2N bond indicators are
    pairwise independent with mean 1/q, so E[E] = -2N/q and
    Var E = 2N (1/q)(1 - 1/q) exactly."""
    L, q, R = 8, 8, 4000
    d = oracle.Desc(L, q, R, [0.0], 0, seed=77)
    o = oracle.run(d, final=True)
    N = L * L
    E = o["final_E"].astype(np.float64)
    mu, var = -2 * N / q, 2 * N * (1 / q) * (1 - 1 / q)
    assert abs(E.mean() - mu) < 5 * math.sqrt(var / R)
    # variance of the sample variance ~ 2 var^2 / R for near-normal E
    assert abs(E.var() - var) < 5 * var * math.sqrt(2 / R) + 0.5
    counts = np.bincount(o["final_spins"].ravel(), minlength=q)
    assert len(counts) == q
    assert stats.chisquare(counts).pvalue > 1e-4


def test_ground_init():
    """eq. (6): each replica has all spins equal to alpha, alpha uniform over
    the q states."""
    L, q, R = 4, 5, 5000
    d = oracle.Desc(L, q, R, [3.0], 0, seed=5, init=oracle.INIT_GROUND)
    o = oracle.run(d, final=True)
    s = o["final_spins"]
    assert (s == s[:, :1]).all()
    assert (o["final_E"] == -2 * L * L).all()
    assert stats.chisquare(np.bincount(s[:, 0], minlength=q)).pvalue > 1e-4
    # eq. (7)-(8): -beta F = ln q - beta E_0 with E_0 = -2N
    assert o["minus_beta_F"][0] == pytest.approx(math.log(q) + 2 * L * L * 3.0, rel=1e-15)


# --------------------------------------------------------------------------
# Step 3: Metropolis sweeps
# --------------------------------------------------------------------------
def test_sweep_visits_every_site_once():
    """At beta = 0 every move is accepted; with q = 2 the proposal is always
    the other state, so one sweep flips every site iff each site is attempted
    an odd number of times (once)."""
    for L in (2, 4, 6, 8):
        d = oracle.Desc(L, 2, 1, [0.0, 0.0], 1, seed=3, resample=oracle.RESAMPLE_NONE)
        s0 = oracle.init_replica(d, 0)
        T = oracle.thresholds(0.0)
        s1 = oracle.one_sweep(d, 1, 0, 0, T, s0)
        assert (s1 == 1 - s0).all()


def test_proposal_never_current_state_and_uniform():
    """The proposal is uniform over the q - 1 states other than the current
    one: at beta = 0 (all accepted) one sweep from the all-zero state sends
    each site to 1..q-1 uniformly, never 0."""
    L, q = 32, 6
    d = oracle.Desc(L, q, 1, [0.0, 0.0], 1, seed=11, resample=oracle.RESAMPLE_NONE)
    T = oracle.thresholds(0.0)
    counts = np.zeros(q, np.int64)
    for k in range(40):
        s1 = oracle.one_sweep(d, 1, 0, k, T, np.zeros(L * L, np.uint8))
        counts += np.bincount(s1, minlength=q)
    assert counts[0] == 0
    assert stats.chisquare(counts[1:]).pvalue > 1e-4


def test_stationary_distribution_L2():
    """Detailed balance of the sweep: after many sweeps at fixed beta with
    resampling off, independent replicas of the 2 x 2, q = 3 lattice are
    distributed over all 81 configurations as exp(-beta E) / Z."""
    L, q, R, beta = 2, 3, 30000, 0.7
    betas = np.array([0.0] + [beta] * 4)
    d = oracle.Desc(L, q, R, betas, 5, seed=21, resample=oracle.RESAMPLE_NONE)
    o = oracle.run(d, final=True)
    s = o["final_spins"].astype(np.int64)
    idx = s[:, 0] * 27 + s[:, 1] * 9 + s[:, 2] * 3 + s[:, 3]
    counts = np.bincount(idx, minlength=81)
    confs = np.array([[a // 27, (a // 9) % 3, (a // 3) % 3, a % 3] for a in range(81)], np.uint8)
    E = np.array([oracle.energy(2, c) for c in confs], np.float64)
    p = np.exp(-beta * E)
    p /= p.sum()
    assert stats.chisquare(counts, p * R).pvalue > 1e-4


@pytest.mark.parametrize("q", [2, 3])
@pytest.mark.parametrize("beta", [0.3, 0.7, 1.5])
def test_one_sweep_matrix_leaves_boltzmann_stationary(q, beta):
    """The exact one-sweep transition matrix of the 2 x 2 lattice built from the
    proposal and acceptance rule (independently of the oracle) is stochastic
    and leaves exp(-beta E) / Z stationary to 1e-9: the only departure from
    detailed balance is the flooring of the thresholds to multiples of 2^-32."""
    P, E = exact.one_sweep_matrix_L2(q, beta)
    assert np.abs(P.sum(axis=1) - 1.0).max() < 1e-12
    pi = np.exp(-beta * E)
    pi /= pi.sum()
    assert np.abs(pi @ P - pi).max() < 1e-9


def one_sweep_transition_counts(sweep, q, n_slots):
    """Counts [q^4, q^4] of (start, end) configurations of one sweep of the
    2 x 2 lattice, every start configuration taken n_slots times; sweep(k,
    spins) returns the swept spins of slot k."""
    confs = np.array([[a // q ** 3, (a // q ** 2) % q, (a // q) % q, a % q] for a in range(q ** 4)],
                     np.uint8)
    counts = np.zeros((q ** 4, q ** 4), np.int64)
    k = 0
    for a, c in enumerate(confs):
        for _ in range(n_slots):
            s = sweep(k, c)
            counts[a, int(s[0]) * q ** 3 + int(s[1]) * q ** 2 + int(s[2]) * q + int(s[3])] += 1
            k += 1
    return counts


def transitions_match(counts, P):
    """Chi-square of all rows against the exact matrix (cells with an expected
    count of at least 5; the rest of each row pooled into one cell)."""
    chi2, dof = 0.0, 0
    for a in range(P.shape[0]):
        n = counts[a].sum()
        e = P[a] * n
        big = e >= 5
        obs = list(counts[a][big]) + [counts[a][~big].sum()]
        exp_ = list(e[big]) + [e[~big].sum()]
        if exp_[-1] < 1e-12:
            obs, exp_ = obs[:-1], exp_[:-1]
            assert counts[a][~big].sum() == 0
        chi2 += sum((o - x) ** 2 / x for o, x in zip(obs, exp_))
        dof += len(obs) - 1
    return stats.chi2.sf(chi2, dof)


def test_oracle_one_sweep_follows_the_exact_matrix_L2():
    """The oracle's sweep of the 2 x 2, q = 3 lattice, started 300 times from
    each of the 81 configurations (different slots, so different random
    words), lands on the configurations with the exact matrix's
    probabilities."""
    q, beta = 3, 0.7
    d = oracle.Desc(2, q, 1, np.array([0.0, beta]), 1, seed=77, resample=oracle.RESAMPLE_NONE)
    T = oracle.thresholds(beta)
    counts = one_sweep_transition_counts(lambda k, c: oracle.one_sweep(d, 1, 0, k, T, c), q, 300)
    P, _ = exact.one_sweep_matrix_L2(q, beta)
    assert transitions_match(counts, P) > 1e-4


def test_mcmc_mean_energy_L4_q3():
    """Metropolis alone (no resampling) at fixed beta on 4 x 4, q = 3 reaches
    the exact <E> of the transfer-matrix density of states."""
    L, q, R, beta = 4, 3, 4000, 0.9
    betas = np.array([0.0] + [beta] * 6)
    d = oracle.Desc(L, q, R, betas, 10, seed=8, resample=oracle.RESAMPLE_NONE)
    o = oracle.run(d)
    g = exact.dos_transfer(L, q)
    mu, var = exact.mean_E_from_dos(g, beta), exact.var_E_from_dos(g, beta)
    assert abs(o["E_mean"][-1] - mu) < 5 * math.sqrt(var / R)


# --------------------------------------------------------------------------
# Step 2 and eq. (1): resampling
# --------------------------------------------------------------------------
def _injected_energies(R, N, seed):
    rng = np.random.default_rng(seed)
    return rng.integers(-2 * N, min(-2 * N + 40, 1), size=R).astype(np.int32)


def test_multinomial_counts_sum_and_means():
    """Sum of copy numbers equals the number of draws; E[r_j] = n W_j / S with
    W_j = round(2^Kb exp(-|dbeta| d_j)) (chi-square over many seeds)."""
    L, R, n_seeds = 8, 50, 400
    N = L * L
    E = _injected_energies(R, N, 1)
    betas = np.array([0.0, 0.08])
    tot = np.zeros(R, np.int64)
    Kb = 57
    for seed in range(n_seeds):
        d = oracle.Desc(L, 3, R, betas, 0, seed=seed, resample=oracle.RESAMPLE_MULTINOMIAL)
        r, anc, eref = oracle.resample(d, 1, Kb, E, R)
        assert r.sum() == R
        assert (np.diff(anc.astype(np.int64)) >= 0).all()
        assert (np.bincount(anc, minlength=R) == r).all()
        tot += r
    assert eref == E.min()
    W, D = oracle.weights(0.08, Kb, N)
    w = W[E - E.min()].astype(np.float64)
    expect = n_seeds * R * w / w.sum()
    assert stats.chisquare(tot, expect).pvalue > 1e-4


def test_ancestor_intervals_are_half_open():
    """Draw u in {0..S-1} selects the replica j with C_{j-1} <= u < C_j, so
    replica j is drawn with probability exactly W_j / S and a zero-weight
    replica never.  With only Kb = 2 bits of weight precision S is small and
    u lands on the interval ends often enough to see an off-by-one."""
    L, R, n_seeds = 8, 30, 600
    N = L * L
    E = _injected_energies(R, N, 3)
    E[0] = E.max() + 10        # replica 0 gets weight 0
    betas = np.array([0.0, 0.2])
    Kb = 2
    W, D = oracle.weights(0.2, Kb, N)
    w = np.array([W[e - E.min()] if e - E.min() < D else 0 for e in E], np.float64)
    assert w[0] == 0 and w.sum() < 4 * R
    tot = np.zeros(R, np.int64)
    for seed in range(n_seeds):
        d = oracle.Desc(L, 3, R, betas, 0, seed=seed, resample=oracle.RESAMPLE_MULTINOMIAL)
        r, anc, eref = oracle.resample(d, 1, Kb, E, R)
        tot += r
    assert tot[0] == 0
    keep = w > 0
    assert (tot[~keep] == 0).all()
    expect = n_seeds * R * w[keep] / w.sum()
    assert stats.chisquare(tot[keep], expect).pvalue > 1e-4


def test_weights_fixed_point():
    """W(0) = 2^Kb exactly (the reference replica); W vanishes from D on;
    W(d) / 2^Kb approximates exp(-|dbeta| d) to half a unit in the last place."""
    W, D = oracle.weights(0.01, 45, 64)
    assert int(W[0]) == 2 ** 45
    assert (W[D:] == 0).all() and (W[:D] > 0).all()
    d = np.arange(len(W))
    assert np.all(np.abs(W.astype(np.float64) - np.ldexp(np.exp(-0.01 * d), 45)) <= 0.5)


def test_poisson_sampler_is_poisson():
    """orc_poisson maps a uniform grid of u onto the Poisson pmf: every k
    receives the mass p(k) up to one grid cell."""
    for lam in (3.0, 37.5, 1000.0, 20000.0):
        n = 200000
        u = (np.arange(n) + 0.5) / n
        ks = np.array([oracle.poisson(lam, x) for x in u])
        kmax = ks.max()
        counts = np.bincount(ks, minlength=kmax + 1)
        pmf = stats.poisson.pmf(np.arange(kmax + 1), lam) * n
        assert np.all(np.abs(counts - pmf) <= 2.0 + 1e-6 * n)


def test_poisson_schedule_conserves_population_in_expectation():
    """eq. (1): R_i = sum_j r_j with sum_j mean = R, so R_i ~ Pois(R): mean R and
    variance R over many steps."""
    R, K = 2000, 4001
    d = oracle.Desc(8, 4, R, np.zeros(K), 0, seed=99)
    R_sched, R_cap, Kb = oracle.plan(d)
    x = R_sched[1:].astype(np.float64)
    assert R_sched[0] == R
    assert abs(x.mean() - R) < 5 * math.sqrt(R / len(x))
    assert abs(x.var() / R - 1) < 5 * math.sqrt(2 / len(x))
    assert R_cap == int(R_sched.max())
    assert Kb == 63 - math.ceil(math.log2(R_cap))


def test_poisson_marginal_copy_numbers():
    """eq. (1): the copy number of replica j is Pois(mu_j) with
    mu_j = (R / R_prev) tau_j.  Compared with a direct per-replica sampler
    (numpy) by mean, variance and a two-sample chi-square."""
    L, R = 8, 40
    N = L * L
    E = _injected_energies(R, N, 2)
    betas = np.array([0.0, 0.05])
    tau = np.exp(-0.05 * (E - E.min()).astype(np.float64))
    mu = R * tau / tau.sum()
    j = int(np.argmax(mu))
    samples = []
    for seed in range(3000):
        d = oracle.Desc(L, 3, R, betas, 0, seed=seed)
        R_sched, cap, Kb = oracle.plan(d)
        r, anc, _ = oracle.resample(d, 1, Kb, E, int(R_sched[1]))
        samples.append(int(r[j]))
    s = np.array(samples, np.float64)
    assert abs(s.mean() - mu[j]) < 5 * math.sqrt(mu[j] / len(s))
    assert abs(s.var() / mu[j] - 1) < 5 * math.sqrt(2 / len(s)) + 0.02
    direct = np.random.default_rng(0).poisson(mu[j], size=len(s))
    kmax = int(max(s.max(), direct.max())) + 1
    a = np.bincount(s.astype(int), minlength=kmax)
    b = np.bincount(direct, minlength=kmax)
    keep = (a + b) >= 10
    table = np.vstack([a[keep], b[keep]])
    assert stats.chi2_contingency(table).pvalue > 1e-4


def test_theta_zero_copies_ancestors():
    """With theta = 0 each new replica is a byte copy of its ancestor, its
    energy is carried along, and the histogram counts R_i replicas."""
    L, q, R = 8, 8, 300
    betas = lin_beta(1.0, 5)
    d0 = oracle.Desc(L, q, R, betas[:1], 0, seed=4, resample=oracle.RESAMPLE_MULTINOMIAL)
    start = oracle.run(d0, final=True)
    d = oracle.Desc(L, q, R, betas[:2], 0, seed=4, resample=oracle.RESAMPLE_MULTINOMIAL)
    o = oracle.run(d, final=True, hist=True)
    anc = o["last_anc"]
    assert (o["final_spins"] == start["final_spins"][anc]).all()
    assert (o["final_E"] == start["final_E"][anc]).all()
    assert o["hist"][1].sum() == o["R_i"][1]


# --------------------------------------------------------------------------
# eq. (2): the free-energy estimator
# --------------------------------------------------------------------------
def test_lnQ_zero_step_is_zero_and_mean_exact():
    """A step with dbeta = 0 gives Q = 1, ln Q = 0 exactly; E-bar is the exact
    integer sum over R_i rounded once."""
    L, q, R = 4, 3, 500
    betas = np.array([0.0, 0.0, 0.0])
    d = oracle.Desc(L, q, R, betas, 2, seed=6)
    o = oracle.run(d, final=True)
    assert o["lnQ"][1] == 0.0 and o["lnQ"][2] == 0.0
    assert o["minus_beta_F"][2] == (L * L) * math.log(q)
    assert o["E_sum"][-1] == int(o["final_E"].astype(np.int64).sum())
    assert o["E_mean"][-1] == o["E_sum"][-1] / float(o["R_i"][-1])


def test_first_step_Q_is_unbiased():
    """From beta_0 = 0 the replicas are uniform configurations, so
    E[Q_1] = sum_E g(E) e^{-dbeta E} / q^N = Z(dbeta) / q^N exactly."""
    L, q, R, db = 4, 3, 200, 0.6
    g = exact.dos_transfer(L, q)
    exact_Q = math.exp(exact.lnZ_from_dos(g, db) - L * L * math.log(q))
    Qs = []
    for seed in range(300):
        d = oracle.Desc(L, q, R, np.array([0.0, db]), 0, seed=seed)
        Qs.append(math.exp(oracle.run(d)["lnQ"][1]))
    Qs = np.array(Qs)
    assert abs(Qs.mean() - exact_Q) < 5 * Qs.std() / math.sqrt(len(Qs))


def _pa_free_energy_check(L, q, R, betas, theta, n_seeds, exact_lnZ, resample, idx):
    diffs = []
    for seed in range(n_seeds):
        d = oracle.Desc(L, q, R, betas, theta, seed=1000 + seed, resample=resample)
        o = oracle.run(d)
        diffs.append([o["minus_beta_F"][i] - exact_lnZ(betas[i]) for i in idx])
    diffs = np.array(diffs)
    mean, se = diffs.mean(axis=0), diffs.std(axis=0, ddof=1) / math.sqrt(n_seeds)
    return mean, se


def test_pa_free_energy_exact_L4_q3():
    """eq. (2) with ln Z_{beta0} = N ln q against the exact ln Z of the 4 x 4,
    q = 3 lattice along a cooling protocol through beta_t = ln(1 + sqrt 3)."""
    L, q = 4, 3
    g = exact.dos_transfer(L, q)
    betas = lin_beta(1.6, 40)
    idx = [10, 20, 30, 40]
    mean, se = _pa_free_energy_check(L, q, 1000, betas, 5, 20,
                                     lambda b: exact.lnZ_from_dos(g, b),
                                     oracle.RESAMPLE_POISSON, idx)
    assert np.all(np.abs(mean) < 5 * se + 2e-3), (mean, se)


def test_pa_free_energy_kaufman_L8_ising():
    """q = 2 Potts (the Ising model) on 8 x 8: eq. (2) against Kaufman's exact
    finite-torus partition function, Z_Potts(beta) = e^{beta N} Z_Ising(beta/2)."""
    L, q = 8, 2
    betas = lin_beta(1.4, 35)
    idx = [10, 20, 35]
    mean, se = _pa_free_energy_check(L, q, 1000, betas, 5, 20,
                                     lambda b: exact.potts_q2_lnZ(L, b),
                                     oracle.RESAMPLE_MULTINOMIAL, idx)
    assert np.all(np.abs(mean) < 5 * se + 5e-3), (mean, se)


def test_heating_run_from_ground_states():
    """Sec. 5-6: a heating run (dbeta < 0) from ground states at beta = 3 with
    ln Z_inf = ln q + 2N beta (eq. (7)-(8)) reproduces the exact ln Z."""
    L, q = 4, 3
    g = exact.dos_transfer(L, q)
    betas = lin_beta(3.0, 60)[::-1].copy()
    idx = [20, 40, 60]
    diffs = []
    for seed in range(12):
        d = oracle.Desc(L, q, 1000, betas, 5, seed=seed, init=oracle.INIT_GROUND)
        o = oracle.run(d)
        diffs.append([o["minus_beta_F"][i] - exact.lnZ_from_dos(g, betas[i]) for i in idx])
    diffs = np.array(diffs)
    mean, se = diffs.mean(axis=0), diffs.std(axis=0, ddof=1) / math.sqrt(len(diffs))
    assert np.all(np.abs(mean) < 5 * se + 3e-3), (mean, se)


def test_energy_means_follow_exact_curve():
    """eq. (4): the population mean energy of a cooling PA run on 4 x 4, q = 3
    follows the exact <E>(beta)."""
    L, q, R = 4, 3, 3000
    g = exact.dos_transfer(L, q)
    betas = lin_beta(1.6, 40)
    d = oracle.Desc(L, q, R, betas, 5, seed=31)
    o = oracle.run(d)
    for i in (8, 16, 25, 32, 40):
        mu, var = exact.mean_E_from_dos(g, betas[i]), exact.var_E_from_dos(g, betas[i])
        assert abs(o["E_mean"][i] - mu) < 6 * math.sqrt(var / o["R_i"][i]) + 0.02


# --------------------------------------------------------------------------
# Validation
# --------------------------------------------------------------------------
def test_validation_rejects_bad_descriptions():
    ok = oracle.Desc(8, 8, 10, [0.0, 0.5], 1, 1)
    assert oracle.validate(ok) == 0
    bad = [
        oracle.Desc(7, 8, 10, [0.0, 0.5], 1, 1),            # odd L
        oracle.Desc(8, 1, 10, [0.0, 0.5], 1, 1),            # q < 2
        oracle.Desc(8, 256, 10, [0.0, 0.5], 1, 1),          # q > 255
        oracle.Desc(8, 8, 0, [0.0, 0.5], 1, 1),             # R = 0
        oracle.Desc(8, 8, 10, [0.1, 0.5], 1, 1),            # random init needs beta_0 = 0
        oracle.Desc(8, 8, 10, [0.0, float("nan")], 1, 1),   # non-finite beta
        oracle.Desc(8, 8, 10, [0.0, -0.5], 1, 1),           # negative beta
    ]
    for b in bad:
        assert oracle.validate(b) != 0


# --------------------------------------------------------------------------
# eq. (4)-(5): magnetisation
# --------------------------------------------------------------------------
def test_mtilde_closed_forms():
    """M~ = N for a ground state (M = N); a two-colouring with two states has
    M~ = N/2; eq. (5) gives M = 0 for an exactly equal split over q states."""
    for L, q in ((4, 3), (8, 8), (6, 2)):
        N = L * L
        assert oracle.mtilde(L, q, np.full(N, q - 1, np.uint8)) == N
        cb = np.array([(x + y) % 2 for y in range(L) for x in range(L)], np.uint8)
        assert oracle.mtilde(L, q, cb) == N // 2
    s = np.arange(16, dtype=np.uint8) % 4           # 4 states, 4 sites each
    assert oracle.mtilde(4, 4, s) == 4


def test_magnetisation_stationary_mean_L2():
    """Metropolis alone at fixed beta on 2 x 2, q = 3: the population mean of
    M (eq. (4)-(5)) equals the exact Boltzmann average over all 81
    configurations, and the M~ histogram adds up to R."""
    L, q, R, beta = 2, 3, 30000, 0.7
    betas = np.array([0.0] + [beta] * 4)
    d = oracle.Desc(L, q, R, betas, 5, seed=21, resample=oracle.RESAMPLE_NONE)
    o = oracle.run(d, magnetisation=True)
    confs = np.array([[a // 27, (a // 9) % 3, (a // 3) % 3, a % 3] for a in range(81)], np.uint8)
    E = np.array([oracle.energy(2, c) for c in confs], np.float64)
    mt = np.array([np.bincount(c, minlength=q).max() for c in confs], np.float64)
    M = (q * mt - 4) / (q - 1)
    p = np.exp(-beta * E)
    p /= p.sum()
    mean, var = (p * M).sum(), (p * M * M).sum() - (p * M).sum() ** 2
    assert abs(o["M_mean"][-1] - mean) < 5 * np.sqrt(var / R)
    assert o["mhist"][-1].sum() == R
    assert o["Mt_sum"][-1] == int((np.arange(5) * o["mhist"][-1]).sum())


# --------------------------------------------------------------------------
# Sec. 4: full width at half maximum of the population histograms
# --------------------------------------------------------------------------
def _fwhm_fine_grid(h, B, pts_per_bin=2000):
    """Independent reading of the width: sample the piecewise-linear curve
    through the bin counts (zero beyond the ends) on a fine grid and measure
    the span of the points at or above half the maximum."""
    c = np.add.reduceat(np.asarray(h, np.float64), np.arange(0, len(h), B))
    xs = np.arange(-1, len(c) + 1)
    ys = np.concatenate([[0.0], c, [0.0]])
    grid = np.linspace(-1, len(c), (len(c) + 1) * pts_per_bin + 1)
    above = grid[np.interp(grid, xs, ys) >= 0.5 * c.max()]
    return (above[-1] - above[0]) * B, B / pts_per_bin


def test_fwhm_closed_forms():
    """A single filled level has width one level; n equal levels have width n;
    a tent of height H and slope s has width H/s; bins of B levels over an
    n-level plateau (n divisible by B) give n."""
    assert oracle.fwhm(np.array([0, 0, 7, 0])) == 1.0
    assert oracle.fwhm(np.array([5])) == 1.0
    assert oracle.fwhm(np.array([0, 3, 3, 3, 3, 3, 0])) == 5.0
    tent = np.array([max(0, 12 - 3 * abs(j - 10)) for j in range(21)])
    assert oracle.fwhm(tent) == 4.0
    assert oracle.fwhm(np.array([2, 2, 2, 2, 2, 2, 0, 0]), 2) == 6.0
    assert oracle.fwhm(np.zeros(9, np.uint32)) == 0.0


def test_fwhm_gaussian():
    """Bin counts of a Gaussian of standard deviation sigma (in levels): the
    width is 2 sqrt(2 ln 2) sigma up to the linear-interpolation error."""
    sigma, c = 25.0, 200.0
    j = np.arange(401)
    h = np.rint(1e6 * np.exp(-0.5 * ((j - c) / sigma) ** 2)).astype(np.uint32)
    want = 2 * np.sqrt(2 * np.log(2)) * sigma
    assert abs(oracle.fwhm(h) - want) < 0.01


def test_fwhm_against_fine_grid_reading():
    """Random histograms with one or several peaks, bins of 1..5 levels: the
    width agrees with a fine-grid measurement of the same curve to the grid
    spacing, and with explicit re-binning."""
    rng = np.random.default_rng(11)
    for t in range(60):
        n = int(rng.integers(1, 80))
        h = rng.integers(0, 50, size=n).astype(np.uint32)
        if t % 3 == 0:
            h[: n // 2] = 0
        B = int(rng.integers(1, 6))
        got = oracle.fwhm(h, B)
        if h.sum() == 0:
            assert got == 0.0
            continue
        want, tol = _fwhm_fine_grid(h, B)
        assert abs(got - want) <= 2 * tol, (t, got, want)
        rebinned = np.add.reduceat(h, np.arange(0, n, B)).astype(np.uint32)
        assert oracle.fwhm(rebinned) * B == got


def test_widths_and_magnetisation_of_ground_states():
    """A population entirely in ground states (eq. (6), no sweeps): M~ = N and
    M-bar = N (eq. (5)); both histograms are single levels, so the widths are
    one level: 1/N in e and q/((q-1) N) in m."""
    L, q = 8, 5
    N = L * L
    d = oracle.Desc(L, q, 300, np.array([3.0]), 0, seed=3, resample=oracle.RESAMPLE_NONE,
                    init=oracle.INIT_GROUND)
    o = oracle.run(d, magnetisation=True, widths=True)
    assert o["Mt_sum"][0] == 300 * N and o["M_mean"][0] == N
    assert o["width_e"][0] == 1.0 / N
    assert o["width_m"][0] == (1.0 * q) / ((q - 1) * N)


# --------------------------------------------------------------------------
# Sec. 6 (Fig. 3) free-energy crossing; Tables I-III width maxima
# --------------------------------------------------------------------------
def test_crossing_of_two_straight_lines():
    """Lines -beta F = a - b beta and c - d beta cross at (a - c) / (b - d);
    linear interpolation between grid points is exact for lines."""
    beta = np.linspace(0.5, 2.0, 151)
    for a, b, c, d in ((10.0, 3.0, 8.0, 1.5), (0.0, -1.0, -2.2, -2.9)):
        x = (a - c) / (b - d)
        fc, fh = a - b * beta, c - d * beta
        assert abs(oracle.crossing(beta, fc, fh) - x) < 1e-12


def test_crossing_takes_the_sharpest_sign_change():
    """Noise-level sign changes of the difference elsewhere do not move the
    crossing; a grid without a down-crossing is an error."""
    beta = np.linspace(0.0, 3.0, 301)
    x = 1.426
    fc = 100.0 - 50.0 * (beta - x) * (beta > x)
    fh = 100.0 + 80.0 * (x - beta) * (beta < x) * -1.0
    # equal slopes far from x; tiny alternating noise near beta = 0.2 and 2.8
    fh = fh + 1e-9 * np.where(np.abs(beta - 0.2) < 0.05, np.sin(200 * beta), 0.0)
    fc = fc + 1e-9 * np.where(np.abs(beta - 2.8) < 0.05, np.cos(200 * beta), 0.0)
    got = oracle.crossing(beta, fc, fh)
    assert abs(got - x) < 0.01
    with pytest.raises(ValueError):
        oracle.crossing(beta, fh - 1.0, fh)


def test_width_maxima_first_argmax():
    beta = np.array([0.5, 1.0, 1.25, 2.0])
    i, w, T = oracle.width_maxima(beta, np.array([0.1, 0.4, 0.4, 0.2]))
    assert (i, w, T) == (1, 0.4, 1.0)


@pytest.mark.parametrize("q", [6, 10])
def test_oracle_free_energy_crossing_at_beta_t(q):
    """Sec. 6 / Fig. 3 with the oracle alone: cooling from beta = 0 (ln Z = N ln q)
    and heating from ground states at beta = 3 (eq. (6)-(8)) give -beta F curves
    that cross within one grid step of the transition point ln(1 + sqrt q) of the
    2D Potts model (16 x 16, R = 2000, dbeta = 0.02, theta = 5; the finite-size
    shift at this size is below one step).  A wrong normalisation or sign in
    eq. (2) or eq. (8) moves the crossing far away."""
    n = 150
    beta = np.array([3.0 * i / n for i in range(n + 1)])
    c = oracle.run(oracle.Desc(16, q, 2000, beta, 5, 10 + q))
    h = oracle.run(oracle.Desc(16, q, 2000, beta[::-1].copy(), 5, 20 + q, init=oracle.INIT_GROUND))
    x = oracle.crossing(beta, c["minus_beta_F"], h["minus_beta_F"][::-1])
    assert abs(x - math.log(1 + math.sqrt(q))) < 0.02
