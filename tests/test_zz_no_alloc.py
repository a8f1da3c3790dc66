"""pa_run_static (the run in the library's fixed device workspace, for callers
that cannot allocate) against pa_run with a caller workspace: two calls in a
row, the second on a smaller run, each bit-identical to pa_run (FP64
estimators included: the same kernels on the same inputs); a run whose
workspace exceeds the fixed array is refused."""
import numpy as np
import pytest

import paper_1704_01888_amd as pa
from paper_1704_01888_amd.workloads import linear_betas

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = pa.Context(0)
    yield c
    c.close()


def _same(a, b):
    for k in ("R_i", "E_sum", "E_mean", "lnQ", "minus_beta_F", "hist", "digest", "final_spins",
              "final_E", "last_anc"):
        assert (a[k] == b[k]).all(), k


def test_static_workspace_runs_equal_pa_run(ctx):
    outs = pa.OUT_HIST | pa.OUT_FINAL | pa.OUT_DIGEST
    big = pa.Desc(32, 10, 20000, linear_betas(1.6, 40), 10, 2, resample=pa.RESAMPLE_POISSON,
                  outputs=outs)
    small = pa.Desc(8, 8, 1000, linear_betas(1.6, 200), 10, 1, resample=pa.RESAMPLE_MULTINOMIAL,
                    outputs=outs)
    assert pa.pa_plan(big).workspace_bytes <= pa.STATIC_SCRATCH_BYTES
    print("\npa_run_static: 32x32 R=2e4 K=41, then 8x8 R=1000 K=201", flush=True)
    got_big = pa.pa_run_static(ctx, big)
    got_small = pa.pa_run_static(ctx, small)      # the array keeps the first call's contents
    _same(got_big, pa.pa_run(ctx, big))
    _same(got_small, pa.pa_run(ctx, small))


def test_static_workspace_refuses_larger_runs(ctx):
    d = pa.Desc(128, 10, 20000, linear_betas(1.0, 3), 1, 3)
    assert pa.pa_plan(d).workspace_bytes > pa.STATIC_SCRATCH_BYTES
    with pytest.raises(pa.PAError) as e:
        pa.pa_run_static(ctx, d)
    assert e.value.status == pa.PA_ERR_NOMEM
