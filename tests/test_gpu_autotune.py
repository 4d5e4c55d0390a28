"""The autotuner (labs_autotune, labs_autotune_batch) on the GPU, through the C ABI: it tunes into
a private cache file, plans created afterwards with automatic options take the tuned launch form
(single-length batches by their length, mixed-length batches by their own key), and those plans
give the oracle's walks bit for bit."""
import numpy as np
import pytest

from oracle import oracle as o

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SEED = 2011000068
TUNED = ("variant", "waves_per_block", "probe_width", "persistent")


@pytest.fixture(scope="module")
def labs():
    import paper_2011_00068_amd as labs

    labs.lib()
    return labs


def _check_against_oracle(labs, cfgs, picks):
    plan = labs.WalkPlan(cfgs)
    opts = plan.opts()
    plan.run()
    res = plan.results()
    plan.close()
    for i in picks:
        c = cfgs[i]
        ref = o.walk(c.L, SEED, c.walk_id, steps=c.steps, table_log2=c.table_log2, trace=bool(c.flags & 1))
        for k in ("best_isl", "best_step", "final_isl", "best_bits", "final_bits", "flip_evals", "restarts", "traps"):
            assert res[i][k] == ref[k], (c.L, c.walk_id, k)
        if c.flags & 1:
            assert np.array_equal(res[i]["trace"], ref["trace"])
    return opts


def test_autotune_single_length(labs, tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("LABS_AUTOTUNE_CACHE", str(cache))
    best = labs.autotune(255, 256)
    lines = cache.read_text().split()
    assert lines[1] == "255" and [int(v) for v in lines[2:6]] == [best[k] for k in TUNED]
    # a plan of the same length with automatic options runs the tuned form
    cfgs = [labs.make_cfg(255, SEED, w, steps=700, table_log2=16, trace=(w % 16 == 0)) for w in range(128)]
    opts = _check_against_oracle(labs, cfgs, range(0, 128, 16))
    assert {k: opts[k] for k in TUNED} == {k: best[k] for k in TUNED}
    # a length of another kernel shape does not take the L = 255 entry: with a later L = 255 entry
    # of non-default options, L = 255 takes it and L = 101 keeps the untuned defaults
    with open(cache, "a") as f:
        f.write(f"{lines[0]} 255 2 8 1 2\n")  # a later entry wins
    plan = labs.WalkPlan([labs.make_cfg(255, SEED, 0, steps=10)])
    assert {k: plan.opts()[k] for k in TUNED} == {"variant": 2, "waves_per_block": 8, "probe_width": 1,
                                                   "persistent": 2}
    plan.close()
    plan = labs.WalkPlan([labs.make_cfg(101, SEED, 0, steps=10)])
    assert plan.opts()["variant"] == labs.VARIANT_MFMA and plan.opts()["waves_per_block"] == 1
    plan.close()


def test_autotune_mixed_batch(labs, tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("LABS_AUTOTUNE_CACHE", str(cache))
    lengths = list(range(201, 304, 2))
    cfgs = [labs.make_cfg(L, SEED, w, steps=500, table_log2=16, trace=(w == 0)) for L in lengths for w in range(3)]
    best = labs.autotune_batch(cfgs)
    assert cache.read_text().split()[1] == "M201-303"
    opts = _check_against_oracle(labs, cfgs, range(0, len(cfgs), 13))
    assert {k: opts[k] for k in TUNED} == {k: best[k] for k in TUNED}
    # the mixed entry is not taken by a single-length batch, nor by a mix of another range
    with open(cache, "a") as f:
        f.write(f"{cache.read_text().split()[0]} M201-303 2 8 1 2\n")  # a later entry wins
    plan = labs.WalkPlan(cfgs[:6])  # L = 201, 203 only: another key
    assert plan.opts()["variant"] == labs.VARIANT_MFMA and plan.opts()["waves_per_block"] == 1
    plan.close()
    plan = labs.WalkPlan(cfgs)
    assert {k: plan.opts()[k] for k in TUNED} == {"variant": 2, "waves_per_block": 8, "probe_width": 1,
                                                   "persistent": 2}
    plan.close()
    with pytest.raises(labs.LabsError) as e:
        labs.autotune_batch([labs.make_cfg(200, SEED, 0)])
    assert e.value.code == labs.LABS_EINVAL
