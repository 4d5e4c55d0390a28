"""The other full-size workloads on the GPU, through the C ABI: the L = 101 batch (1,024 walks x
10^5 steps) on the automatic (matrix-core) and the bit-sliced walker with sampled walks against the
oracle, and the uneven batch of every odd L in
[201, 303] x 64 walks x 10^6 steps in one launch, checked by properties that hold at any size
(each walk's best / final ISL is the ISL of its best / final bits, evaluation counts) and by
invariance under splitting the walks over several launches, with sampled long walks against the
oracle; and full-GPU batches of 16,384 walks of the one-tile (L = 255) and two-tile (L = 303)
matrix-core walker with sampled walks against the oracle."""
import numpy as np
import pytest

from oracle import oracle as o

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SEED = 2011000068


@pytest.fixture(scope="module")
def labs():
    import paper_2011_00068_amd as labs

    labs.lib()
    return labs


@pytest.mark.parametrize("variant", [0, 1])  # automatic (the matrix cores), bit-sliced
def test_l101_batch_full_size(labs, variant):
    # (two runs of the plan, as bench.py times it: the second reuses the tables under new epochs)
    cfgs = [labs.make_cfg(101, SEED, w, steps=100000, table_log2=16) for w in range(1024)]
    plan = labs.WalkPlan(cfgs, variant=variant)
    plan.run()
    first = plan.results()
    plan.run()
    res = plan.results()
    plan.close()
    assert res == first
    for w in (0, 513):
        r = o.walk(101, SEED, w, steps=100000, table_log2=16)
        for k in ("best_isl", "best_step", "final_isl", "best_bits", "final_bits", "restarts", "traps", "flip_evals"):
            assert res[w][k] == r[k], (w, k)
    for w in range(0, 1024, 37):
        r = res[w]
        assert r["steps_done"] == 100000 and r["flip_evals"] == 100000 * 51
        assert o.isl(o.skew_expand(101, r["best_bits"])) == r["best_isl"]
        assert o.isl(o.skew_expand(101, r["final_bits"])) == r["final_isl"]


def test_uneven_batch_full_size(labs):
    lengths = list(range(201, 304, 2))
    cfgs = [labs.make_cfg(L, SEED, w, steps=10 ** 6, table_log2=16) for L in lengths for w in range(64)]
    one = labs.WalkPlan(cfgs)  # one launch, all 3,328 walks, mixed shapes
    one.run()
    res = one.results()
    ms, launches = one.last_timing()
    one.close()
    assert launches == 1
    split = labs.WalkPlan(cfgs, steps_per_launch=333333, persistent=2)  # 4 launches, pulled walks
    split.run()
    res2 = split.results()
    split.close()
    for a, b in zip(res, res2):
        assert a == b
    for i in range(0, len(cfgs), 53):
        L = cfgs[i].L
        r = res[i]
        assert r["steps_done"] == 10 ** 6 and r["flip_evals"] == 10 ** 6 * ((L + 1) // 2)
        assert o.isl(o.skew_expand(L, r["best_bits"])) == r["best_isl"]
        assert o.isl(o.skew_expand(L, r["final_bits"])) == r["final_isl"]
    # the uneven batch shares its first steps with a short run of the same walks
    short = [labs.make_cfg(L, SEED, 0, steps=300, table_log2=16, trace=True) for L in lengths[::9]]
    p = labs.WalkPlan(short)
    p.run()
    rs = p.results()
    p.close()
    for c, r in zip(short, rs):
        ref = o.walk(c.L, SEED, 0, steps=300, table_log2=16, trace=True)
        assert np.array_equal(r["trace"], ref["trace"])


def test_uneven_batch_long_walks_match_oracle(labs):
    # The uneven batch's launch (all 52 lengths x 64 walks in one grid of the mixed-length
    # matrix-core kernel, replayed from a hipGraph) run for 2 x 10^5 steps, past the point where
    # the 2^16-word visited tables start to evict; three of its walks (shortest, headline and
    # longest length) compared with the oracle in every result field, from the graph's second
    # replay (tables reused under new epochs), which equals the first.
    from concurrent.futures import ThreadPoolExecutor

    steps = 200000
    lengths = list(range(201, 304, 2))
    cfgs = [labs.make_cfg(L, SEED, w, steps=steps, table_log2=16) for L in lengths for w in range(64)]
    plan = labs.WalkPlan(cfgs, use_graph=True)
    assert plan.opts()["variant"] == labs.VARIANT_MFMA
    plan.run()
    first = plan.results()
    plan.run()
    res = plan.results()
    _, launches = plan.last_timing()
    plan.close()
    assert res == first
    assert launches == 1
    picks = [(201, 0), (255, 17), (303, 63)]
    with ThreadPoolExecutor(max_workers=len(picks)) as ex:
        refs = list(ex.map(lambda p: o.walk(p[0], SEED, p[1], steps=steps, table_log2=16), picks))
    for (L, w), ref in zip(picks, refs):
        got = res[lengths.index(L) * 64 + w]
        for k in ("best_isl", "best_step", "steps_done", "flip_evals", "hit_step", "watch_step", "final_isl",
                  "restarts", "traps", "best_bits", "final_bits"):
            assert got[k] == ref[k], (L, w, k, got[k], ref[k])


@pytest.mark.parametrize("L", [255, 303])  # the one-tile and the two-tile matrix-core walker
def test_full_gpu_batches_of_each_walker_shape(labs, L):
    # The batches that compare the two walker shapes (16,384 walks x 2,000 steps, two rounds of
    # resident waves): 12 walks spread over the grid (first, last and the round boundaries) against
    # the oracle in every result field, and every walk's best / final ISL against the ISL of its
    # best / final bits.
    from concurrent.futures import ThreadPoolExecutor

    walks, steps = 16384, 2000
    cfgs = [labs.make_cfg(L, SEED, w, steps=steps, table_log2=16) for w in range(walks)]
    plan = labs.WalkPlan(cfgs)
    assert plan.opts()["variant"] == labs.VARIANT_MFMA
    plan.run()
    plan.run()  # the second run, as timed: tables reused under new epochs
    res = plan.results()
    plan.close()
    picks = [0, 1, 4095, 4096, 5119, 5120, 8191, 8192, 10239, 12288, 16382, 16383]
    with ThreadPoolExecutor(max_workers=8) as ex:
        refs = list(ex.map(lambda w: o.walk(L, SEED, w, steps=steps, table_log2=16), picks))
    for w, ref in zip(picks, refs):
        for k in ("best_isl", "best_step", "steps_done", "flip_evals", "hit_step", "watch_step", "final_isl",
                  "restarts", "traps", "best_bits", "final_bits"):
            assert res[w][k] == ref[k], (L, w, k, res[w][k], ref[k])
    rng = np.random.default_rng(L)
    for w in rng.choice(walks, 64, replace=False):
        r = res[int(w)]
        assert r["steps_done"] == steps and r["flip_evals"] == steps * ((L + 1) // 2)
        assert o.isl(o.skew_expand(L, r["best_bits"])) == r["best_isl"]
        assert o.isl(o.skew_expand(L, r["final_bits"])) == r["final_isl"]
