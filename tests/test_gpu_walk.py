"""GPU parity of the walk (Section 3, Algorithm 1 in its self-avoiding-walk reading) against the
oracle, through the C ABI: full trajectories (chosen flip and ISL per step), every flip score of
every step, and the per-walk results, bit for bit."""
import numpy as np
import pytest

from oracle import oracle as o

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SEED = 2011000068
RESULT_KEYS = ("best_isl", "best_step", "steps_done", "flip_evals", "hit_step", "watch_step",
               "final_isl", "restarts", "traps", "best_bits", "final_bits")


@pytest.fixture(scope="module")
def labs():
    import paper_2011_00068_amd as labs

    labs.lib()
    return labs


def oracle_walk(c, trace=False, score_trace=False):
    return o.walk(c.L, c.seed, c.walk_id, steps=c.steps, table_log2=c.table_log2,
                  restart_period=c.restart_period, target_isl=c.target_isl, watch_isl=c.watch_isl,
                  trace=trace, score_trace=score_trace)


def assert_same(g, r, what=""):
    for k in RESULT_KEYS:
        assert g[k] == r[k], (what, k, g[k], r[k])
    if "trace" in r and "trace" in g:
        T = r["steps_done"]
        assert np.array_equal(g["trace"][:T], r["trace"][:T]), what
    if "scores" in r and "scores" in g:
        T = r["steps_done"]
        assert np.array_equal(g["scores"][:T], r["scores"][:T]), what


@pytest.mark.parametrize("variant", [1, 2, 3], ids=["bitslice", "direct", "mfma"])
def test_l31_single_walk_full_trajectory(labs, variant):
    # L = 31, one walk of 20,000 steps, exact table (2^16 >= 2^n): every step's chosen flip, ISL
    # and all 16 flip scores equal the oracle's.
    c = labs.make_cfg(31, SEED, 0, steps=20000, table_log2=16, trace=True, score_trace=True)
    plan = labs.WalkPlan([c], variant=variant)
    plan.run()
    g = plan.results()[0]
    plan.close()
    r = oracle_walk(c, trace=True, score_trace=True)
    assert_same(g, r, "L31")
    assert g["best_isl"] == 79  # the enumerated skew optimum


@pytest.mark.parametrize("variant", [1, 2, 3], ids=["bitslice", "direct", "mfma"])
def test_plan_reruns_reuse_tables(labs, variant):
    # A plan's runs reuse its visited tables without clearing them: every start and restart takes
    # the table's next epoch, and a table is cleared only on its first use or when its epochs run
    # out (3 for a 2^2-word table, 7 for 2^3).  Six runs in a row, with restarts and traps, in
    # hashed tables and in tables addressed by the free bits (L = 3, 31, 41): each equals the
    # oracle, whose table is cleared at every start.
    cfgs = [labs.make_cfg(255, SEED, 0, steps=400, table_log2=2, restart_period=37, trace=True),
            labs.make_cfg(3, SEED, 1, steps=60, table_log2=2, restart_period=7, trace=True),
            labs.make_cfg(5, SEED, 2, steps=80, table_log2=2, trace=True),
            labs.make_cfg(13, SEED, 3, steps=300, table_log2=3, trace=True),
            labs.make_cfg(101, SEED, 4, steps=300, table_log2=3, restart_period=50, trace=True),
            labs.make_cfg(31, SEED, 5, steps=2000, table_log2=16, restart_period=300, trace=True),
            labs.make_cfg(41, SEED, 6, steps=1500, table_log2=21, restart_period=200, trace=True),
            labs.make_cfg(7, SEED, 7, steps=200, table_log2=4, trace=True),
            labs.make_cfg(13, SEED, 8, steps=600, table_log2=7, trace=True),
            labs.make_cfg(21, SEED, 9, steps=3000, table_log2=11, trace=True)]
    refs = [oracle_walk(c, trace=True) for c in cfgs]
    assert sum(r["traps"] for r in refs) >= 30
    plan = labs.WalkPlan(cfgs, variant=variant)
    for run in range(6):
        plan.run()
        for i, (g, r) in enumerate(zip(plan.results(), refs)):
            assert_same(g, r, f"run {run}, L = {cfgs[i].L}")
    plan.close()


def test_chunked_plan_reruns_reuse_tables(labs):
    # The same with the walks cut into launches of 37 steps (each launch resumes a walk from its
    # state record, epoch included) and the pulling persistent grid: three runs, each equal to
    # the oracle.
    cfgs = [labs.make_cfg(255, SEED, 0, steps=300, table_log2=2, restart_period=29, trace=True),
            labs.make_cfg(7, SEED, 7, steps=200, table_log2=4, trace=True),
            labs.make_cfg(101, SEED, 4, steps=300, table_log2=3, restart_period=50, trace=True),
            labs.make_cfg(303, SEED, 2, steps=250, table_log2=3, restart_period=41, trace=True)]
    refs = [oracle_walk(c, trace=True) for c in cfgs]
    plan = labs.WalkPlan(cfgs, steps_per_launch=37, persistent=2)
    for run in range(3):
        plan.run()
        for i, (g, r) in enumerate(zip(plan.results(), refs)):
            assert_same(g, r, f"run {run}, L = {cfgs[i].L}")
    plan.close()


@pytest.mark.parametrize("L", [3, 5, 7, 9, 13, 33, 63, 65, 95, 97, 101, 127, 129, 131, 191, 193, 201,
                               255, 257, 259, 303, 321, 383])
def test_short_walks_every_shape(labs, L):
    # every kernel shape (flip groups x window words), edge lengths included
    cfgs = [labs.make_cfg(L, SEED + L, w, steps=300, table_log2=12, trace=True, score_trace=True)
            for w in range(3)]
    for variant in (1, 2, 3):
        got = labs.WalkPlan(cfgs, variant=variant)
        got.run()
        res = got.results()
        got.close()
        for w, c in enumerate(cfgs):
            assert_same(res[w], oracle_walk(c, trace=True, score_trace=True), (L, w, variant))


def test_l101_batch_sample(labs):
    # L = 101 batch (1,024 walks in the full workload): 128 walks x 3,000 steps, per-walk
    # results for all, full traces for the first 8.
    cfgs = [labs.make_cfg(101, SEED, w, steps=3000, table_log2=16, trace=(w < 8)) for w in range(128)]
    plan = labs.WalkPlan(cfgs)
    plan.run()
    res = plan.results()
    plan.close()
    for w in range(0, 128, 9):
        assert_same(res[w], oracle_walk(cfgs[w], trace=(w < 8)), w)
    for w in range(8):
        assert_same(res[w], oracle_walk(cfgs[w], trace=True), w)


def test_mixed_lengths_one_launch(labs):
    # the uneven batch: every odd L in [201, 303] in one launch, 2 walks each
    cfgs = []
    for L in range(201, 304, 2):
        for w in range(2):
            cfgs.append(labs.make_cfg(L, SEED, w, steps=150, table_log2=16, trace=True))
    plan = labs.WalkPlan(cfgs)
    plan.run()
    res = plan.results()
    plan.close()
    for i, c in enumerate(cfgs):
        assert_same(res[i], oracle_walk(c, trace=True), (c.L, c.walk_id))


def test_restarts_traps_targets(labs):
    cfgs = [
        labs.make_cfg(5, SEED, 0, steps=60, table_log2=8, trace=True, score_trace=True),   # traps
        labs.make_cfg(7, SEED, 1, steps=200, table_log2=3, trace=True),                    # tiny table
        labs.make_cfg(51, SEED, 7, steps=205, restart_period=40, trace=True, score_trace=True),
        labs.make_cfg(101, SEED, 9, steps=500, target_isl=1500, trace=True),
        labs.make_cfg(101, SEED, 9, steps=500, watch_isl=1500, trace=True),
        labs.make_cfg(101, SEED, 9, steps=0),
        labs.make_cfg(255, SEED, 3, steps=300, restart_period=64, table_log2=10, trace=True),
    ]
    for variant in (1, 2, 3):
        plan = labs.WalkPlan(cfgs, variant=variant)
        plan.run()
        res = plan.results()
        plan.close()
        for i, c in enumerate(cfgs):
            r = oracle_walk(c, trace=bool(c.flags & 1), score_trace=bool(c.flags & 2))
            assert_same(res[i], r, (i, variant))
    assert res[0]["traps"] >= 1


def test_restarts_traps_targets_untraced(labs):
    # the same cases without traces or scores run the step loop built without trace tests; a
    # batch mixing traced and untraced walks runs both forms side by side
    cfgs = [
        labs.make_cfg(5, SEED, 0, steps=60, table_log2=8),
        labs.make_cfg(7, SEED, 1, steps=200, table_log2=3),
        labs.make_cfg(51, SEED, 7, steps=205, restart_period=40),
        labs.make_cfg(101, SEED, 9, steps=500, target_isl=1500),
        labs.make_cfg(101, SEED, 9, steps=500, watch_isl=1500),
        labs.make_cfg(101, SEED, 9, steps=500, target_isl=1500, watch_isl=1700, restart_period=97),
        labs.make_cfg(255, SEED, 3, steps=300, restart_period=64, table_log2=10),
        labs.make_cfg(255, SEED, 3, steps=300, restart_period=64, table_log2=10, trace=True),
        labs.make_cfg(201, SEED, 5, steps=400, restart_period=150, watch_isl=3000),
        # tables addressed by the free bits (n <= table_log2), untraced
        labs.make_cfg(31, SEED, 0, steps=3000, table_log2=16),
        labs.make_cfg(41, SEED, 2, steps=2000, table_log2=21, restart_period=700),
    ]
    for variant in (1, 2, 3):
        for opt in (dict(), dict(steps_per_launch=61)):
            plan = labs.WalkPlan(cfgs, variant=variant, **opt)
            plan.run()
            res = plan.results()
            plan.close()
            for i, c in enumerate(cfgs):
                r = oracle_walk(c, trace=bool(c.flags & 1), score_trace=bool(c.flags & 2))
                assert_same(res[i], r, (i, variant, opt))
    assert res[0]["traps"] >= 1


def test_target_met_by_start_state(labs):
    start_isl = o.isl(o.skew_expand(101, o.start_bits(101, SEED, 4, 0)))
    c = labs.make_cfg(101, SEED, 4, steps=100, target_isl=start_isl)
    plan = labs.WalkPlan([c])
    plan.run()
    g = plan.results()[0]
    plan.close()
    assert g["hit_step"] == 0 and g["steps_done"] == 0
    assert_same(g, oracle_walk(c))


def test_launch_options_do_not_change_results(labs):
    cfgs = [labs.make_cfg(L, SEED, w, steps=700, table_log2=14, restart_period=256, trace=True)
            for L in (61, 201, 255, 303) for w in range(4)]
    ref = None
    options = [
        dict(variant=1, waves_per_block=1, probe_width=1),
        dict(variant=1, waves_per_block=2, probe_width=2),
        dict(variant=1, waves_per_block=4, probe_width=4, persistent=2),
        dict(variant=1, waves_per_block=8, probe_width=2, steps_per_launch=97),
        dict(variant=2, waves_per_block=1, probe_width=1, steps_per_launch=250),
        dict(variant=1, probe_width=2, steps_per_launch=128, use_graph=True),
        dict(variant=1, plain=True),
    ]
    for opt in options:
        plan = labs.WalkPlan(cfgs, **opt)
        for rep in range(2):
            plan.run()
            res = plan.results()
            if ref is None:
                ref = res
            for a, b in zip(ref, res):
                assert_same(a, b, opt)
        plan.close()
    for i in (0, 5, 10, 15):
        assert_same(ref[i], oracle_walk(cfgs[i], trace=True), i)


def test_mfma_launch_options_and_mixed_lengths(labs):
    # the matrix-core form under every launch option, on a batch mixing its shapes (one and two
    # tiles)
    cfgs = [labs.make_cfg(L, SEED, w, steps=600, table_log2=14, restart_period=200, trace=True)
            for L in (5, 33, 61, 129, 131, 191, 253, 255, 257, 259, 303, 321, 383) for w in range(3)]
    ref = None
    for opt in (dict(variant=1), dict(variant=3), dict(variant=3, waves_per_block=4, persistent=2),
                dict(variant=3, steps_per_launch=77), dict(variant=3, use_graph=True, steps_per_launch=150)):
        plan = labs.WalkPlan(cfgs, **opt)
        plan.run()
        res = plan.results()
        plan.close()
        if ref is None:
            ref = res
        for a, b in zip(ref, res):
            assert_same(a, b, opt)
    for i in (0, 4, 9, 13, 20, 23, 24, 28, 31, 35, 38):
        assert_same(ref[i], oracle_walk(cfgs[i], trace=True), i)


def test_l255_headline_full_size(labs):
    # the L = 255 headline workload exactly as bench.py runs it (16,384 walks x 4,768 steps, restart
    # period 2^20, stop at F >= 8.5, watch F >= 5): sampled walks against the oracle, properties on
    # a stride of the rest.  bench.py times the plan's later runs, which reuse the tables under a
    # new epoch instead of clearing them: the third run equals the first, walk for walk.
    import bench

    cfgs = bench.cfgs(labs, bench.WALKS, bench.STEPS)
    plan = labs.WalkPlan(cfgs)
    plan.run()
    first = plan.results()
    plan.run()
    plan.run()
    res = plan.results()
    plan.close()
    assert res == first
    for w in (0, 1, 8191, 16383):
        assert_same(res[w], oracle_walk(cfgs[w]), w)
    for w in range(0, bench.WALKS, 61):
        r = res[w]
        assert r["steps_done"] == bench.STEPS or r["hit_step"] >= 0
        assert r["flip_evals"] == r["steps_done"] * 128
        assert o.isl(o.skew_expand(255, r["best_bits"])) == r["best_isl"]
        assert o.isl(o.skew_expand(255, r["final_bits"])) == r["final_isl"]
        assert r["best_isl"] <= r["final_isl"]


def test_walk_batch_entry_point(labs):
    cfgs = [labs.make_cfg(41, SEED, w, steps=400, trace=True) for w in range(5)]
    res = labs.walk_batch(cfgs)
    for w, c in enumerate(cfgs):
        assert_same(res[w], oracle_walk(c, trace=True), w)


def test_walk_rejects_oversized_buffers(labs):
    # two traced walks of 2^40 steps ask for 2^41 trace records: refused before any allocation
    cfgs = [labs.make_cfg(31, SEED, w, steps=1 << 40, trace=True) for w in range(2)]
    with pytest.raises(labs.LabsError) as e:
        labs.WalkPlan(cfgs)
    assert e.value.code == labs.LABS_ENOMEM


def test_walk_rejects_bad_config(labs):
    for bad in (dict(L=4), dict(L=1), dict(L=385), dict(table_log2=0), dict(table_log2=31), dict(steps=-1)):
        kw = dict(L=31, seed=1, walk_id=0, steps=10, table_log2=16)
        kw.update(bad)
        c = labs.make_cfg(**kw)
        with pytest.raises(labs.LabsError) as e:
            labs.WalkPlan([c])
        assert e.value.code == labs.LABS_EINVAL


def _restart_state_cases(labs, traced):
    # walks restarting after every step at L = 21 (exact table) whose best is a restart state, and
    # watch / target levels first met by a restart state (found with the oracle)
    L, S, n = 21, 40, 11
    cfgs = []
    for w in range(300):
        r = o.walk(L, SEED, w, steps=S, restart_period=1, table_log2=n + 1, trace=True)
        starts = {o.start_bits(L, SEED, w, k): k for k in range(1, S)}
        if r["best_bits"] in starts and r["best_step"] == starts[r["best_bits"]]:
            cfgs.append(labs.make_cfg(L, SEED, w, steps=S, restart_period=1, table_log2=n + 1, trace=traced))
            lvl = r["best_isl"]
            cfgs.append(labs.make_cfg(L, SEED, w, steps=S, restart_period=1, table_log2=n + 1, watch_isl=lvl,
                                      trace=traced))
            cfgs.append(labs.make_cfg(L, SEED, w, steps=S, restart_period=1, table_log2=n + 1, target_isl=lvl,
                                      trace=traced))
        if len(cfgs) >= 12:
            break
    assert len(cfgs) >= 6
    # traps (L = 5, exact table) and periodic restarts at the matrix-core lengths
    cfgs.append(labs.make_cfg(5, SEED, 3, steps=50, table_log2=8, trace=traced))
    cfgs.append(labs.make_cfg(255, SEED, 6, steps=30, restart_period=1, table_log2=10, trace=traced))
    return cfgs


@pytest.mark.parametrize("traced", [True, False], ids=["traced", "untraced"])
def test_restart_states_count_for_best_hit_watch(labs, traced):
    cfgs = _restart_state_cases(labs, traced)
    for variant in (1, 2, 3):
        for opt in (dict(), dict(steps_per_launch=7)):
            plan = labs.WalkPlan(cfgs, variant=variant, **opt)
            plan.run()
            res = plan.results()
            plan.close()
            for i, c in enumerate(cfgs):
                assert_same(res[i], oracle_walk(c, trace=traced), (i, variant, opt))
    # some of them stop at a target met by a restart state
    assert any(c.target_isl >= 0 for c in cfgs)
