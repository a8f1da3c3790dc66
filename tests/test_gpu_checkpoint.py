"""Checkpoints through the C ABI (pa_checkpoint, pa_resume, pa_serve_checkpoint,
pa_serve_resume) against the oracle.

A checkpoint taken on the device at step k is (a) byte for byte the file the
format statement of include/pa.h gives for that state, (b) continued by the
oracle to the oracle's own uninterrupted result, and (c) continued by the
device to the device's uninterrupted result, bit-exactly from step k on
(ln Q and -beta F within 1e-12 between device and oracle).
"""
import time

import numpy as np
import pytest

import oracle
import paper_1704_01888_amd as pa
from paper_1704_01888_amd.workloads import linear_betas
from test_checkpoint_format import write_checkpoint

pytestmark = pytest.mark.gpu

RTOL = 1e-12


@pytest.fixture(scope="module")
def ctx():
    c = pa.Context(0)
    yield c
    c.close()


def _same_from(a, b, k, exact_fp=True):
    for key in ("R_i", "E_sum", "E_mean", "digest", "hist"):
        assert (a[key][k:] == b[key][k:]).all(), key
    for key in ("final_spins", "final_E", "last_anc"):
        assert (a[key] == b[key]).all(), key
    if exact_fp:
        assert (a["minus_beta_F"][k:] == b["minus_beta_F"][k:]).all()
    else:
        np.testing.assert_allclose(a["minus_beta_F"][k:], b["minus_beta_F"][k:], rtol=RTOL, atol=0)
        np.testing.assert_allclose(a["lnQ"][k + 1:], b["lnQ"][k + 1:], rtol=RTOL, atol=1e-13)


CASES = [
    dict(L=16, q=8, R=900, beta=linear_betas(1.5, 24), theta=3, seed=41, resample=0),
    dict(L=6, q=5, R=700, beta=linear_betas(1.4, 15), theta=2, seed=42, resample=1),
    dict(L=512, q=10, R=6, beta=linear_betas(1.5, 6), theta=1, seed=43, resample=0),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"L{c['L']}")
def test_device_checkpoint_format_oracle_and_device_resume(ctx, case, tmp_path):
    outs = pa.OUT_HIST | pa.OUT_FINAL | pa.OUT_DIGEST
    d = pa.Desc(outputs=outs, **case)
    k = d.K // 2
    print(f"\ncase: {d.L}x{d.L} q={d.q} R={d.R} K={d.K}, checkpoint at step {k}", flush=True)
    full = pa.pa_run(ctx, d)
    run = pa.Run(ctx, d)
    run.advance(k)
    path = tmp_path / "dev.pack"
    run.checkpoint(path)
    st = run.read(anc=False, counts=False)
    step, mbf = run.free_energy()
    run.finish()
    assert step == k
    # (a) the documented bytes for this state
    ref = tmp_path / "ref.pack"
    write_checkpoint(ref, d, k, st["spins"], mbf, int(st["E"].astype(np.int64).sum()), outputs=outs)
    assert path.read_bytes() == ref.read_bytes()
    # (b) the oracle continues it to its own uninterrupted run
    od = oracle.Desc(**case)
    ck = oracle.read_checkpoint(path)
    cont = oracle.run_from(ck["desc"], ck["step"], ck["spins"], ck["minus_beta_F"], hist=True,
                           final=True, digest=True)
    whole = oracle.run(od, hist=True, final=True, digest=True)
    _same_from(cont, whole, k)
    _same_from(full, whole, 0, exact_fp=False)
    # (c) the device continues it to its own uninterrupted run
    res = pa.Run.resume(ctx, path)
    res.advance(d.K - 1 - k)
    got = res.finish()
    _same_from(got, full, k)


def test_resume_refuses_a_file_whose_energies_do_not_match(ctx, tmp_path):
    d = pa.Desc(outputs=pa.OUT_FINAL, **CASES[0])
    run = pa.Run(ctx, d)
    run.advance(3)
    st = run.read(anc=False, counts=False)
    step, mbf = run.free_energy()
    run.finish()
    bad = tmp_path / "bad.pack"
    write_checkpoint(bad, d, step, st["spins"], mbf, int(st["E"].astype(np.int64).sum()) + 1,
                     outputs=pa.OUT_FINAL)
    with pytest.raises(pa.PAError) as e:
        pa.Run.resume(ctx, bad)
    assert e.value.status == pa.PA_ERR_INVALID


def test_serving_ticket_checkpoint_and_resume(ctx, tmp_path):
    """A running ticket is checkpointed at a step boundary of the serving loop
    while it goes on; the file resumed as a new request (and by the oracle)
    reproduces the uninterrupted run from its step on."""
    kw = dict(L=32, q=10, R=6000, beta=linear_betas(1.6, 120), theta=10, seed=44, resample=0)
    d = pa.Desc(outputs=pa.OUT_HIST | pa.OUT_FINAL | pa.OUT_DIGEST, **kw)
    full = pa.pa_run(ctx, d)
    sv = pa.Server(ctx, arena_bytes=1 << 30, max_slots=2)
    try:
        t = sv.submit(d)
        path = tmp_path / "ticket.pack"
        deadline = time.time() + 60
        while True:                         # queued until admitted
            try:
                sv.checkpoint(t, path)
                break
            except pa.PAError as e:
                assert e.status == pa.PA_ERR_BUSY and time.time() < deadline
                time.sleep(0.001)
        served, _ = sv.wait(t)
        _same_from(served, full, 0)
        _, k, _ = pa.checkpoint_info(path)
        assert 0 <= k < d.K - 1
        t2 = sv.resume(path)
        resumed, _ = sv.wait(t2)
    finally:
        sv.stop()
    _same_from(resumed, full, k)
    ck = oracle.read_checkpoint(path)
    cont = oracle.run_from(ck["desc"], ck["step"], ck["spins"], ck["minus_beta_F"], hist=True,
                           final=True, digest=True)
    _same_from(resumed, cont, k, exact_fp=False)
    with pytest.raises(pa.PAError):
        sv.checkpoint(t, path)              # server stopped
