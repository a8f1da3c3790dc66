"""Tuned sweep shapes (pa_tune, pa_tune_set / get, pa_tune_save / load).

Every shape a lattice side has (each lane count with a kernel, each number of
waves per workgroup that fits) gives the oracle's result bit for bit; the
tuner keeps a measured shape per (L, q class, population class); the cache
file round-trips and refuses shapes a side does not have; runs of one kernel
class with different tuned workgroup sizes share a batch correctly."""
import json

import numpy as np
import pytest

import oracle
import paper_1704_01888_amd as pa
from paper_1704_01888_amd.workloads import linear_betas

pytestmark = pytest.mark.gpu

KEYS = ("R_i", "E_sum", "hist", "final_spins", "final_E", "last_anc", "digest")


@pytest.fixture(scope="module")
def ctx():
    c = pa.Context(0)
    yield c
    c.close()


def _same(a, b):
    for k in KEYS:
        assert (a[k] == b[k]).all(), k
    np.testing.assert_allclose(a["minus_beta_F"], b["minus_beta_F"], rtol=1e-12, atol=0)


def _shapes(ctx, L):
    """Every (lanes, waves per workgroup) the library accepts for L."""
    lanes = {ctx.tune_get(L, 8, 300)["lanes"]}
    _, cands = ctx.get_lanes(L)
    lanes.update(c for c in cands if c)
    out = []
    for G in sorted(lanes):
        for w in range(1, 17):
            try:
                ctx.tune_set(L, 0, 0, G, w)
            except pa.PAError:
                continue
            out.append((G, w))
    return out


@pytest.mark.parametrize("L", [4, 6, 8, 12, 16, 20, 24, 32, 64])
def test_every_shape_matches_the_oracle(ctx, L):
    c = dict(L=L, q=8, R=300, beta=linear_betas(1.4, 5), theta=2, seed=60 + L, resample=0)
    want = oracle.run(oracle.Desc(**c), hist=True, final=True, digest=True)
    d = pa.Desc(outputs=pa.OUT_HIST | pa.OUT_FINAL | pa.OUT_DIGEST, **c)
    shapes = _shapes(ctx, L)
    assert len(shapes) >= 1
    print(f"\nL={L}: shapes {shapes}", flush=True)
    for G, w in shapes:
        ctx.tune_set(L, 0, 0, G, w)
        got_shape = ctx.tune_get(L, 8, 300)
        assert (got_shape["lanes"], got_shape["waves_per_block"]) == (G, w)
        _same(pa.pa_run(ctx, d), want)


def test_tune_keeps_the_fastest_shape_and_the_file_round_trips(ctx, tmp_path):
    a = ctx.tune(8, 8, 1000)
    b = ctx.tune(24, 10, 20000)
    print(f"\ntuned {a} {b}", flush=True)
    assert a["attempts_per_ns"] > 0 and b["attempts_per_ns"] > 0
    assert (a["r_class"], b["r_class"]) == (0, 2)
    for e, (L, q, R) in ((a, (8, 8, 1000)), (b, (24, 10, 20000))):
        g = ctx.tune_get(L, q, R)
        assert (g["lanes"], g["waves_per_block"]) == (e["lanes"], e["waves_per_block"])
    path = tmp_path / "tune.jsonl"
    ctx.tune_save(path)
    lines = [json.loads(ln) for ln in path.read_text().splitlines()]
    assert all(ln["arch"].startswith("gfx") for ln in lines)
    other = pa.Context(0)
    try:
        assert other.tune_load(path) == len(lines)
        for e, (L, q, R) in ((a, (8, 8, 1000)), (b, (24, 10, 20000))):
            g = other.tune_get(L, q, R)
            assert (g["lanes"], g["waves_per_block"]) == (e["lanes"], e["waves_per_block"])
        # another architecture's lines are skipped; a shape L does not have is refused
        foreign = dict(lines[0], arch="gfx000", L=16, lanes=64, waves_per_block=2)
        path2 = tmp_path / "foreign.jsonl"
        path2.write_text(json.dumps(foreign) + "\n")
        assert other.tune_load(path2) == 0
        bad = dict(lines[0], lanes=3)
        path3 = tmp_path / "bad.jsonl"
        path3.write_text(json.dumps(bad) + "\n")
        with pytest.raises(pa.PAError) as e:
            other.tune_load(path3)
        assert e.value.status == pa.PA_ERR_INVALID
        path4 = tmp_path / "garbled.jsonl"
        path4.write_text('{"arch": "gfx950", "L": 8\n')
        with pytest.raises(pa.PAError):
            other.tune_load(path4)
    finally:
        other.close()


@pytest.mark.parametrize("mode", ["segmented", "team"])
def test_one_class_with_two_tuned_workgroup_sizes_in_a_batch(ctx, mode):
    # 8x8 runs of population classes 0 and 1 with different waves per workgroup
    ctx.tune_set(8, 0, 0, 16, 1)
    ctx.tune_set(8, 0, 1, 16, 8)
    cases = [dict(L=8, q=8, R=500, beta=linear_betas(1.5, 20), theta=3, seed=70, resample=1),
             dict(L=8, q=8, R=3000, beta=linear_betas(1.5, 25), theta=3, seed=71, resample=0),
             dict(L=8, q=6, R=700, beta=linear_betas(1.2, 12), theta=2, seed=72, resample=0)]
    descs = [pa.Desc(outputs=pa.OUT_HIST | pa.OUT_FINAL | pa.OUT_DIGEST, **c) for c in cases]
    ctx.set_batch_mode(pa.BATCH_TEAM if mode == "team" else pa.BATCH_SEGMENTED)
    try:
        got = pa.pa_run_batch(ctx, descs)
        if mode == "team":
            assert ctx.batch_info() == (3, 2)        # one launch per workgroup size
    finally:
        ctx.set_batch_mode(pa.BATCH_SEGMENTED)
    for d, g in zip(descs, got):
        _same(g, pa.pa_run(ctx, d))
