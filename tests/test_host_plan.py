"""Host logic of the GPU library, checked on the CPU (no device calls):
the library loads and exports every symbol of include/pa.h, validates run
descriptions, and builds the same integer plan tables (Metropolis
thresholds, population schedule, resampling weights) as the independent
oracle."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle
import paper_1704_01888_amd as pa

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "pa.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(pa_[a-z_]+)\s*\(", src)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    lib = pa.lib()
    declared = _header_functions()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(pa.EXPORTS) == declared


def lin_beta(bmax, n):
    return np.array([bmax * i / n for i in range(n + 1)])


CASES = [
    dict(L=8, q=8, R=1000, beta=lin_beta(1.6, 200), theta=10, seed=1, resample=1),
    dict(L=32, q=10, R=20000, beta=lin_beta(1.6, 400), theta=10, seed=2, resample=0),
    dict(L=128, q=10, R=200000, beta=lin_beta(1.6, 500), theta=20, seed=4, resample=0),
    dict(L=16, q=6, R=777, beta=lin_beta(3.0, 30)[::-1].copy(), theta=3, seed=2**40 + 5,
         resample=0, init=1),
]


@pytest.mark.parametrize("case", CASES)
def test_plan_tables_match_oracle(case):
    d = pa.Desc(**case)
    od = oracle.Desc(**case)
    T, R_sched = pa.pa_plan_tables(d)
    o_sched, o_cap, o_kb = oracle.plan(od)
    assert (R_sched == o_sched).all()
    for i in range(d.K):
        assert (T[i] == oracle.thresholds(d.beta[i])[1:]).all()
    info = pa.pa_plan(d)
    assert info.R_cap == o_cap and info.Kb == o_kb and info.R_final == o_sched[-1]
    popb = 2 * o_cap * d.N
    assert info.workspace_bytes >= popb


@pytest.mark.parametrize("adb,Kb,N", [(0.004, 48, 1024), (0.0032, 45, 16384), (0.008, 53, 64),
                                      (0.0, 45, 64), (0.2, 2, 64), (1.7, 60, 256)])
def test_weight_tables_match_oracle(adb, Kb, N):
    W, D = pa.pa_weight_table(adb, Kb, N)
    Wo, Do = oracle.weights(adb, Kb, N)
    assert D == Do and (W == Wo).all()


def test_validation():
    good = dict(L=8, q=8, R=10, beta=[0.0, 0.5], theta=1, seed=1)
    pa.pa_plan(pa.Desc(**good))
    for bad, status in [
        (dict(good, L=7), pa.PA_ERR_INVALID),
        (dict(good, q=1), pa.PA_ERR_INVALID),
        (dict(good, q=256), pa.PA_ERR_INVALID),
        (dict(good, R=0), pa.PA_ERR_INVALID),
        (dict(good, beta=[0.1, 0.5]), pa.PA_ERR_INVALID),
        (dict(good, beta=[0.0, float("inf")]), pa.PA_ERR_INVALID),
        (dict(good, beta=[0.0, -1.0]), pa.PA_ERR_INVALID),
        (dict(good, theta=2**27), pa.PA_ERR_INVALID),
        (dict(good, L=1), pa.PA_ERR_INVALID),
        (dict(good, L=4100), pa.PA_ERR_UNSUPPORTED),
        (dict(good, L=258), pa.PA_ERR_UNSUPPORTED),
        (dict(good, outputs=32), pa.PA_ERR_INVALID),
        (dict(good, outputs=pa.OUT_WIDTHS, bin_e=2 * 64 + 2), pa.PA_ERR_INVALID),
    ]:
        with pytest.raises(pa.PAError) as e:
            pa.pa_plan(pa.Desc(**bad))
        assert e.value.status == status, bad


def test_poisson_schedule_statistics_from_library():
    """eq. (1): the library's population sizes are Pois(R) (mean and variance)."""
    R, K = 5000, 3001
    T, R_sched = pa.pa_plan_tables(pa.Desc(8, 4, R, np.zeros(K), 0, 123))
    x = R_sched[1:].astype(float)
    assert abs(x.mean() - R) < 5 * math.sqrt(R / len(x))
    assert abs(x.var() / R - 1) < 5 * math.sqrt(2 / len(x))


def test_poisson_capacity_error_matches_oracle():
    """With R = 1 the Poisson schedule draws R_i = 0 with probability 1/e; both
    the library and the oracle report it (PA_ERR_CAPACITY) for the same seeds."""
    beta = np.linspace(0.0, 1.0, 6)
    seen_err = seen_ok = 0
    for seed in range(40):
        try:
            pa.pa_plan(pa.Desc(8, 4, 1, beta, 1, seed))
            lib_ok = True
        except pa.PAError as e:
            assert e.status == pa.PA_ERR_CAPACITY
            lib_ok = False
        try:
            oracle.plan(oracle.Desc(8, 4, 1, beta, 1, seed))
            orc_ok = True
        except ValueError:
            orc_ok = False
        assert lib_ok == orc_ok
        seen_ok += lib_ok
        seen_err += not lib_ok
    assert seen_ok > 0 and seen_err > 0


def test_large_lattices_plan_compact_tables():
    """Lattices beyond LDS are planned (tiled device path); the weight tables
    keep only their nonzero prefix, so the workspace is dominated by the two
    population buffers even for 4096 x 4096 and many distinct dbeta."""
    beta = np.array([1.6 * i / 400 for i in range(401)])
    info = pa.pa_plan(pa.Desc(L=4096, q=10, R=4, beta=beta, theta=1, seed=1, resample=1))
    pop = 2 * 4 * 4096 * 4096
    assert pop <= info.workspace_bytes < pop + 200 * 2**20
    info = pa.pa_plan(pa.Desc(L=260, q=10, R=100, beta=beta, theta=1, seed=1))
    assert info.workspace_bytes < 2 * info.R_cap * 260 * 260 + 20 * 2**20


def test_lattice_sides_accepted_and_rejected():
    """Even L from 2 up: multiples of 4 up to 4096 and L = 2 (mod 4) up to 254
    run on the device; odd L is invalid for the checkerboard update (Sec. 3
    lattice, the update needs two colours)."""
    base = dict(q=4, R=10, beta=np.array([0.0, 0.5, 1.0]), theta=1, seed=1)
    for L in (2, 4, 6, 10, 18, 254, 256, 4096):
        assert pa.pa_plan(pa.Desc(L=L, **base)).workspace_bytes > 0
    for L, status in ((3, pa.PA_ERR_INVALID), (7, pa.PA_ERR_INVALID), (258, pa.PA_ERR_UNSUPPORTED),
                      (4098, pa.PA_ERR_UNSUPPORTED)):
        with pytest.raises(pa.PAError) as e:
            pa.pa_plan(pa.Desc(L=L, **base))
        assert e.value.status == status, L
