"""Serving loop (pa_serve_*): continuous batching inside a device arena.
Every result in the mix equals the same run alone (bit-exact; FP64 within
1e-12); admission by workspace footprint; cancel, timeout and stop."""
import time

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
    for k in ("R_i", "E_sum", "E_mean", "final_spins", "final_E", "last_anc", "hist"):
        if k in a:
            assert (a[k] == b[k]).all(), k
    np.testing.assert_allclose(a["minus_beta_F"], b["minus_beta_F"], rtol=1e-12, atol=0)


REQS = [
    dict(L=16, q=8, R=900, beta=linear_betas(1.5, 40), theta=3, seed=1, resample=0),
    dict(L=8, q=5, R=2000, beta=linear_betas(1.3, 25), theta=4, seed=2, resample=1),
    dict(L=32, q=10, R=400, beta=linear_betas(1.6, 30), theta=2, seed=3, resample=0),
    dict(L=24, q=20, R=300, beta=linear_betas(1.9, 12), theta=2, seed=4, resample=0),
    dict(L=12, q=6, R=700, beta=linear_betas(1.2, 50), theta=1, seed=5, resample=2),
    dict(L=16, q=6, R=500, beta=linear_betas(3.0, 20)[::-1].copy(), theta=2, seed=6, resample=0, init=1),
    dict(L=64, q=8, R=100, beta=linear_betas(1.4, 8), theta=2, seed=7, resample=1),
    dict(L=4, q=3, R=999, beta=linear_betas(1.0, 60), theta=2, seed=8, resample=0),
]


def _descs():
    return [pa.Desc(outputs=pa.OUT_FINAL | pa.OUT_HIST, **c) for c in REQS]


def test_serving_results_equal_alone(ctx):
    descs = _descs()
    alone = [pa.pa_run(ctx, d) for d in descs]
    sv = pa.Server(ctx, arena_bytes=1 << 30, max_slots=5)
    tickets = []
    for i, d in enumerate(descs):
        tickets.append(sv.submit(d))
        if i % 3 == 2:
            time.sleep(0.01)          # later requests arrive while others run
    for t, want in zip(tickets, alone):
        got, tm = sv.wait(t)
        _same(got, want)
        assert tm["arrival_us"] <= tm["admit_us"] <= tm["done_us"]
    sv.stop()


def test_admission_by_footprint_queues(ctx):
    descs = [pa.Desc(L=32, q=8, R=4000, beta=linear_betas(1.4, 30), theta=2, seed=40 + r,
                     outputs=pa.OUT_FINAL) for r in range(4)]
    size = pa.pa_plan(descs[0]).workspace_bytes
    assert size > (4 << 20)
    # room for two runs (plus the descriptor region), not three
    arena = int(2.5 * size) + (1 << 20)
    sv = pa.Server(ctx, arena_bytes=arena, max_slots=8)
    tickets = [sv.submit(d) for d in descs]
    results = [sv.wait(t) for t in tickets]
    sv.stop()
    for d, (got, tm) in zip(descs, results):
        _same(got, pa.pa_run(ctx, d))
    admits = sorted(tm["admit_us"] for _, tm in results)
    dones = sorted(tm["done_us"] for _, tm in results)
    assert admits[2] >= dones[0]        # the third run waited for memory
    assert admits[1] < dones[0]         # the first two ran together


def test_oversized_request_rejected(ctx):
    sv = pa.Server(ctx, arena_bytes=8 << 20, max_slots=2)
    big = pa.Desc(L=64, q=8, R=5000, beta=linear_betas(1.0, 3), theta=1, seed=1)
    with pytest.raises(pa.PAError) as e:
        sv.submit(big)
    assert e.value.status == pa.PA_ERR_NOMEM
    sv.stop()


def test_cancel_timeout_and_stop(ctx):
    sv = pa.Server(ctx, arena_bytes=1 << 28, max_slots=1)
    long_run = pa.Desc(L=32, q=10, R=4000, beta=linear_betas(1.6, 400), theta=10, seed=11)
    queued = pa.Desc(L=8, q=8, R=100, beta=linear_betas(1.0, 5), theta=1, seed=12)
    t1 = sv.submit(long_run)
    t2 = sv.submit(queued)               # waits: one slot only
    with pytest.raises(pa.PAError) as e:
        sv.wait(t1, timeout_us=0)
    assert e.value.status == pa.PA_ERR_TIMEOUT
    sv.cancel(t2)
    sv.cancel(t1)
    for t in (t1, t2):
        with pytest.raises(pa.PAError) as e:
            sv.wait(t)
        assert e.value.status == pa.PA_ERR_CANCELLED
    # after cancellation the slot is free again
    t3 = sv.submit(queued)
    got, _ = sv.wait(t3)
    _same(got, pa.pa_run(ctx, queued))
    sv.submit(long_run)
    sv.submit(queued)
    sv.stop()                            # the admitted run finishes, the queued one is dropped
    sv2 = pa.Server(ctx, arena_bytes=1 << 28, max_slots=1)
    got, _ = sv2.wait(sv2.submit(queued))
    _same(got, pa.pa_run(ctx, queued))
    sv2.stop()


def test_stop_while_waits_are_blocked(ctx):
    """pa_serve_stop while other threads are blocked in pa_serve_wait on queued
    tickets (one slot, a longer request running): stop returns, the running
    request finishes, every queued wait returns PA_ERR_CANCELLED afterwards;
    two waits on one ticket: one consumes it, the other gets PA_ERR_INVALID
    (or the same cancellation when it consumed it first)."""
    import ctypes
    import threading
    long_run = pa.Desc(64, 10, 50000, linear_betas(1.4, 200), 10, 31, resample=0)   # ~0.4 s
    short = [pa.Desc(8, 5, 300, linear_betas(1.0, 10), 2, 40 + k, resample=1) for k in range(4)]
    sv = pa.Server(ctx, arena_bytes=1 << 30, max_slots=1)
    t_long = sv.submit(long_run)
    t_q = [sv.submit(d) for d in short]
    statuses = {}

    def waiter(name, ticket):
        tm = pa.Timing()
        statuses[name] = pa.lib().pa_serve_wait(ctx.handle, ctypes.c_uint64(ticket), ctypes.c_int64(-1),
                                                 ctypes.byref(tm))

    threads = [threading.Thread(target=waiter, args=(f"q{k}", t)) for k, t in enumerate(t_q)]
    threads.append(threading.Thread(target=waiter, args=("dup", t_q[0])))
    for th in threads:
        th.start()
    time.sleep(0.05)
    sv.stop()
    for th in threads:
        th.join(timeout=60)
        assert not th.is_alive()
    assert statuses["q1"] == statuses["q2"] == statuses["q3"] == pa.PA_ERR_CANCELLED
    assert sorted([statuses["q0"], statuses["dup"]]) in (
        sorted([pa.PA_ERR_CANCELLED, pa.PA_ERR_INVALID]), [pa.PA_ERR_CANCELLED] * 2)
    # a new server can start on the same context after stop
    sv2 = pa.Server(ctx, arena_bytes=1 << 28, max_slots=2)
    got, _ = sv2.wait(sv2.submit(short[0]))
    sv2.stop()
    assert (got["R_i"] == pa.pa_run(ctx, short[0])["R_i"]).all()
    del t_long
