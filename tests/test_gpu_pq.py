"""GPU parity of the best-first search with a bounded queue (labs_pq_walk_batch; Algorithm 1
taken literally, Section 3, with the optional second table of xLastovka) against the oracle,
through the C ABI: full traces (move and ISL per iteration), every iteration's flip scores and
the per-walk results, bit for bit."""
import numpy as np
import pytest

from oracle import oracle as o

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SEED = 2011000068
KEYS = ("best_isl", "best_step", "steps_done", "flip_evals", "hit_step", "watch_step", "final_isl",
        "restarts", "traps", "best_bits", "final_bits")


@pytest.fixture(scope="module")
def labs():
    import paper_2011_00068_amd as labs

    labs.lib()
    return labs


def oracle_pq(c, Q, nlog2):
    return o.walk(c.L, c.seed, c.walk_id, steps=c.steps, table_log2=c.table_log2,
                  restart_period=c.restart_period, target_isl=c.target_isl, watch_isl=c.watch_isl,
                  trace=bool(c.flags & 1), score_trace=bool(c.flags & 2), pq_capacity=Q, nbr_table_log2=nlog2)


def assert_same(g, r, what=""):
    for k in KEYS:
        assert g[k] == r[k], (what, k, g[k], r[k])
    for k in ("trace", "scores"):
        if k in r and k in g:
            T = r["steps_done"]
            assert np.array_equal(g[k][:T], r[k][:T]), (what, k)


@pytest.mark.parametrize("L", [5, 7, 31, 63, 65, 127, 129, 191, 255, 257, 303, 383])
def test_capacity_one_equals_the_walk(labs, L):
    cfgs = [labs.make_cfg(L, SEED + L, w, steps=300, table_log2=10, restart_period=97, trace=True,
                          score_trace=True) for w in range(3)]
    got, _ = labs.pq_walk_batch(cfgs, 1)
    walk = labs.walk_batch(cfgs)
    for w, c in enumerate(cfgs):
        assert_same(got[w], walk[w], (L, w, "walk"))
        assert_same(got[w], oracle_pq(c, 1, 0), (L, w, "oracle"))


@pytest.mark.parametrize("L", [3, 9, 31, 61, 101, 127, 201, 255, 301, 383])
@pytest.mark.parametrize("Q,nlog2", [(2, 0), (8, 0), (64, 0), (16, 12), (64, 5)])
def test_queue_matches_oracle(labs, L, Q, nlog2):
    cfgs = [labs.make_cfg(L, SEED, w, steps=250, table_log2=12, trace=True, score_trace=(w == 0))
            for w in range(2)]
    got, _ = labs.pq_walk_batch(cfgs, Q, nlog2)
    for w, c in enumerate(cfgs):
        assert_same(got[w], oracle_pq(c, Q, nlog2), (L, Q, nlog2, w))


def test_restarts_traps_targets(labs):
    cfgs = [
        labs.make_cfg(5, SEED, 0, steps=80, table_log2=8, trace=True, score_trace=True),
        labs.make_cfg(7, SEED, 1, steps=200, table_log2=3, trace=True),
        labs.make_cfg(51, SEED, 7, steps=205, restart_period=40, trace=True, score_trace=True),
        labs.make_cfg(101, SEED, 9, steps=500, target_isl=1500, trace=True),
        labs.make_cfg(101, SEED, 9, steps=500, watch_isl=1500, trace=True),
        labs.make_cfg(101, SEED, 9, steps=0),
        labs.make_cfg(255, SEED, 3, steps=300, restart_period=64, table_log2=10, trace=True),
    ]
    for Q, nlog2 in ((1, 0), (4, 0), (32, 9), (3, 2)):
        got, _ = labs.pq_walk_batch(cfgs, Q, nlog2)
        for i, c in enumerate(cfgs):
            assert_same(got[i], oracle_pq(c, Q, nlog2), (i, Q, nlog2))


def test_mixed_lengths_one_call(labs):
    cfgs = [labs.make_cfg(L, SEED, w, steps=120, table_log2=14, trace=True) for L in range(201, 304, 6)
            for w in range(2)]
    got, ms = labs.pq_walk_batch(cfgs, 24, 10)
    assert ms > 0
    for i, c in enumerate(cfgs):
        assert_same(got[i], oracle_pq(c, 24, 10), (c.L, c.walk_id))


def test_l255_batch_sample(labs):
    # the best-first benchmark shape: L = 255, queue of 64, 2,048 searches x 1,000 iterations;
    # sampled searches against the oracle, properties on the rest
    cfgs = [labs.make_cfg(255, SEED, w, steps=1000, table_log2=16) for w in range(2048)]
    for nlog2 in (0, 16):
        got, _ = labs.pq_walk_batch(cfgs, 64, nlog2)
        for w in (0, 1023, 2047):
            assert_same(got[w], oracle_pq(cfgs[w], 64, nlog2), (w, nlog2))
        for w in range(0, 2048, 97):
            r = got[w]
            assert r["steps_done"] == 1000
            assert r["flip_evals"] <= 1000 * 128
            assert o.isl(o.skew_expand(255, r["best_bits"])) == r["best_isl"]
            assert o.isl(o.skew_expand(255, r["final_bits"])) == r["final_isl"]


def test_rejects_bad_options(labs):
    c = [labs.make_cfg(31, 1, 0, steps=10, table_log2=16)]
    for Q, nlog2 in ((0, 0), (65, 0), (4, -1), (4, 31)):
        with pytest.raises(labs.LabsError) as e:
            labs.pq_walk_batch(c, Q, nlog2)
        assert e.value.code == labs.LABS_EINVAL
    with pytest.raises(labs.LabsError) as e:
        labs.pq_walk_batch([labs.make_cfg(31, 1, 0, steps=1 << 31, table_log2=16)], 4)
    assert e.value.code == labs.LABS_EINVAL


def test_restart_states_count(labs):
    # a restart every iteration (and every trap) at short lengths: restart states count for the
    # best, hit and watch like the initial state, at the iteration after which they are occupied
    cfgs = []
    for w in range(6):
        cfgs.append(labs.make_cfg(21, SEED, w, steps=40, restart_period=1, table_log2=12, trace=True))
        ref = o.walk(21, SEED, w, steps=40, restart_period=1, table_log2=12, pq_capacity=3)
        cfgs.append(labs.make_cfg(21, SEED, w, steps=40, restart_period=2, table_log2=12,
                                  watch_isl=ref["best_isl"], target_isl=ref["best_isl"] + 8, trace=True))
    cfgs.append(labs.make_cfg(5, SEED, 4, steps=60, table_log2=8, trace=True))
    for Q, nlog2 in ((1, 0), (3, 0), (8, 5)):
        got, _ = labs.pq_walk_batch(cfgs, Q, nlog2)
        for i, c in enumerate(cfgs):
            assert_same(got[i], oracle_pq(c, Q, nlog2), (i, Q, nlog2))
