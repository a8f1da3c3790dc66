"""Seeded synthetic run descriptions (input generation only).

The paper's workloads are random initial populations annealed along a
temperature protocol (Sec. 2); there is no dataset.  These helpers produce the
run descriptions used by the benchmark and the tests: lattice side, q,
population size, the inverse-temperature array beta_i = beta_max * i / n
(computed once in double precision, never by repeated addition), sweeps per
step and seed.
"""
from __future__ import annotations

import math

import numpy as np


def linear_betas(beta_max: float, n_steps: int) -> np.ndarray:
    return np.array([beta_max * i / n_steps for i in range(n_steps + 1)], dtype=np.float64)


def beta_t(q: int) -> float:
    """Transition point of the 2D q-state Potts model, ln(1 + sqrt q) (Sec. 3)."""
    return math.log(1.0 + math.sqrt(q))


# Table I protocol: the step is 1/N_beta on [f_lo, f_hi], 0.01 on [c_lo, f_lo)
# and (f_hi, c_hi], and 0.05 below c_lo and above c_hi; (c_lo, f_lo, f_hi, c_hi).
TABLE_REGIONS = {
    6: (0.995, 1.135, 1.305, 1.545),
    8: (1.11, 1.25, 1.42, 1.66),
    10: (1.165, 1.305, 1.475, 1.715),
    20: (1.595, 1.735, 1.905, 2.145),
}


def _segment(start: float, end: float, n: int):
    """n equal steps from start to end, the last point exactly end."""
    return [start + (end - start) * j / n for j in range(1, n)] + [end]


def table_betas(q: int, n_beta: int = 1000, coarse_tail: int = 5) -> np.ndarray:
    """Piecewise cooling protocol of Tables I-III for q in {6, 8, 10, 20}:
    steps of 0.05 from 0 up to c_lo (anchored at c_lo; the first step is the
    remainder), 0.01 up to f_lo, 1/n_beta up to f_hi, 0.01 up to c_hi, then
    coarse_tail steps of 0.05 beyond c_hi (the paper does not state where the
    runs end)."""
    c_lo, f_lo, f_hi, c_hi = TABLE_REGIONS[q]
    low = [c_lo - 0.05 * j for j in range(int(c_lo / 0.05) + 1)][::-1]
    pts = [0.0] + [b for b in low if b > 0.0]
    pts += _segment(c_lo, f_lo, int(round((f_lo - c_lo) / 0.01)))
    n_fine = (f_hi - f_lo) * n_beta
    if abs(n_fine - round(n_fine)) > 1e-9:
        raise ValueError("n_beta must divide the fine region into whole steps")
    pts += _segment(f_lo, f_hi, int(round(n_fine)))
    pts += _segment(f_hi, c_hi, int(round((c_hi - f_hi) / 0.01)))
    pts += [c_hi + 0.05 * j for j in range(1, coarse_tail + 1)]
    return np.array(pts, dtype=np.float64)


def small_runs(n_runs: int = 20, seed0: int = 1):
    """n_runs runs of 8x8, q=8, R=1000, 200 equal steps to beta = 1.6, theta = 10,
    multinomial resampling, seeds seed0, seed0+1, ... (dicts of desc fields)."""
    return [dict(L=8, q=8, R=1000, beta=linear_betas(1.6, 200), theta=10, seed=seed0 + r,
                 resample=1) for r in range(n_runs)]


def mixed_runs(n_runs: int = 20, rng_seed: int = 3, n_steps: int = 300, theta: int = 10):
    """n_runs independent runs with L in {16,24,32,48,64}, q in {5,6,8,10,20},
    R uniform in [1e4, 1e5], each annealed to 1.1 ln(1 + sqrt q) in n_steps
    equal steps, theta sweeps, Poisson resampling, seed 3000 + r."""
    rng = np.random.default_rng(rng_seed)
    runs = []
    for r in range(n_runs):
        L = int(rng.choice([16, 24, 32, 48, 64]))
        q = int(rng.choice([5, 6, 8, 10, 20]))
        R = int(rng.integers(10_000, 100_001))
        runs.append(dict(L=L, q=q, R=R, beta=linear_betas(1.1 * beta_t(q), n_steps), theta=theta,
                         seed=3000 + r, resample=0))
    return runs


def serving_requests(n_requests: int = 500, rng_seed: int = 5, theta: int = 10):
    """Request stream: L in {16,32,64,128}, q in {5,6,8,10,20}, R = round(10^U(3,5)),
    200..500 equal steps to 1.1 ln(1 + sqrt q), theta sweeps, Poisson resampling,
    seed 5000 + k (dicts of desc fields, in arrival order)."""
    rng = np.random.default_rng(rng_seed)
    reqs = []
    for k in range(n_requests):
        L = int(rng.choice([16, 32, 64, 128]))
        q = int(rng.choice([5, 6, 8, 10, 20]))
        R = int(round(10 ** rng.uniform(3.0, 5.0)))
        n_steps = int(rng.integers(200, 501))
        reqs.append(dict(L=L, q=q, R=R, beta=linear_betas(1.1 * beta_t(q), n_steps), theta=theta,
                         seed=5000 + k, resample=0))
    return reqs


def poisson_arrivals(n: int, rate_per_s: float, rng_seed: int = 55) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of the given rate."""
    rng = np.random.default_rng(rng_seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))
