"""Host-only analysis calls of the library (no device work) against the
oracle's independent versions, and the Table I-III schedules."""
import numpy as np
import pytest

import oracle
import paper_1704_01888_amd as pa
from paper_1704_01888_amd.workloads import TABLE_REGIONS, table_betas


def test_width_maxima_matches_oracle():
    rng = np.random.default_rng(4)
    for _ in range(50):
        K = int(rng.integers(1, 300))
        beta = np.sort(rng.uniform(0.1, 3.0, K))
        w = rng.uniform(0, 1, K)
        if K > 3:
            w[rng.integers(0, K)] = w.max()           # ties: first index wins
        assert pa.width_maxima(beta, w) == oracle.width_maxima(beta, w)
    assert pa.width_maxima(np.array([0.0, 1.0]), np.array([2.0, 1.0]))[2] == np.inf
    with pytest.raises(pa.PAError):
        pa.width_maxima(np.array([1.0]), np.array([np.nan]))


def test_crossing_matches_oracle():
    rng = np.random.default_rng(5)
    beta = np.linspace(0.0, 3.0, 301)
    for _ in range(50):
        x = rng.uniform(0.5, 2.5)
        fc = -rng.uniform(1, 5) * (beta - x) + rng.normal(0, 0.05, beta.size)
        fh = rng.normal(0, 0.05, beta.size)
        try:
            want = oracle.crossing(beta, fc, fh)
        except ValueError:
            with pytest.raises(pa.PAError):
                pa.free_energy_crossing(beta, fc, fh)
            continue
        assert pa.free_energy_crossing(beta, fc, fh) == want


def test_crossing_rejects_bad_grids():
    with pytest.raises(pa.PAError):
        pa.free_energy_crossing(np.array([0.0, 0.0]), np.array([1.0, -1.0]), np.zeros(2))
    with pytest.raises(pa.PAError):
        pa.free_energy_crossing(np.array([0.0]), np.array([1.0]), np.zeros(1))


@pytest.mark.parametrize("q", sorted(TABLE_REGIONS))
def test_table_schedules(q):
    """Tables I-III protocol: steps of 1/N_beta exactly across [f_lo, f_hi],
    0.01 next to it, 0.05 outside, region boundaries on the grid."""
    c_lo, f_lo, f_hi, c_hi = TABLE_REGIONS[q]
    for n_beta in (100, 200, 500, 1000, 2000):
        b = table_betas(q, n_beta)
        d = np.diff(b)
        assert b[0] == 0.0 and (d > 0).all()
        for edge in (c_lo, f_lo, f_hi, c_hi):
            assert edge in b
        fine = (b[:-1] >= f_lo) & (b[1:] <= f_hi)
        assert fine.sum() == round((f_hi - f_lo) * n_beta)
        np.testing.assert_allclose(d[fine], 1.0 / n_beta, rtol=1e-9)
        mid = ((b[:-1] >= c_lo) & (b[1:] <= f_lo)) | ((b[:-1] >= f_hi) & (b[1:] <= c_hi))
        np.testing.assert_allclose(d[mid], 0.01, rtol=1e-9)
        outer = (b[1:] <= c_lo) | (b[:-1] >= c_hi)
        assert (d[outer] <= 0.05 + 1e-12).all() and (d[outer][1:] > 0.05 - 1e-12).all()
