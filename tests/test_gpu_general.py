"""GPU parity of the walk over general (not skew-symmetric) sequences (labs_general_walk_batch;
the unrestricted problem of Section 1, Eq. (1)-(3) over every shift) against the oracle, through
the C ABI: full traces, every step's flip scores and the per-walk results, bit for bit."""
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


def oracle_general(c):
    return o.walk(c.L, c.seed, c.walk_id, steps=c.steps, table_log2=c.table_log2,
                  restart_period=c.restart_period, target_isl=c.target_isl, watch_isl=c.watch_isl,
                  trace=bool(c.flags & 1), score_trace=bool(c.flags & 2), general=True)


def assert_same(g, r, what=""):
    for k in KEYS:
        assert g[k] == r[k], (what, k, g[k], r[k])
    for k in ("trace", "scores"):
        if k in r and k in g:
            T = r["steps_done"]
            assert np.array_equal(g[k][:T], r[k][:T]), (what, k)


@pytest.mark.parametrize("L", [3, 4, 5, 8, 13, 32, 33, 34, 63, 64, 65, 66, 96, 97, 98, 127, 128, 129, 130,
                               160, 161, 162, 191, 192])
def test_every_shape_matches_oracle(labs, L):
    cfgs = [labs.make_cfg(L, SEED + L, w, steps=250, table_log2=12, restart_period=90, trace=True,
                          score_trace=True) for w in range(3)]
    got, ms = labs.general_walk_batch(cfgs)
    assert ms >= 0
    for w, c in enumerate(cfgs):
        assert_same(got[w], oracle_general(c), (L, w))


def test_targets_traps_exact_table(labs):
    cfgs = [
        labs.make_cfg(4, SEED, 0, steps=60, table_log2=8, trace=True, score_trace=True),  # traps
        labs.make_cfg(13, SEED, 1, steps=3000, table_log2=14, target_isl=6, trace=True),   # Barker 13
        labs.make_cfg(20, SEED, 2, steps=500, table_log2=22, trace=True),                  # exact table
        labs.make_cfg(100, SEED, 3, steps=400, watch_isl=1600, trace=True),
        labs.make_cfg(150, SEED, 4, steps=0),
    ]
    got, _ = labs.general_walk_batch(cfgs)
    for i, c in enumerate(cfgs):
        assert_same(got[i], oracle_general(c), i)
    assert got[0]["traps"] >= 1
    assert got[1]["best_isl"] == 6 and got[1]["hit_step"] > 0


def _seq(L, x):
    return np.array([-1 if (x >> j) & 1 else 1 for j in range(L)], dtype=np.int8)


def test_flip_scores_every_length(labs):
    # every L in [3, 192]: random states, all +1, all -1 and the alternating sequence (whose
    # correlations |C_k| = L - k leave the int8 range from L = 129 on: the two-pass product)
    for L in range(3, 193):
        rng = np.random.default_rng(L)
        alt = sum(1 << j for j in range(1, L, 2))
        xs = [int(rng.integers(0, 1 << 62)) | (int(rng.integers(0, 1 << 62)) << 62) |
              (int(rng.integers(0, 1 << 62)) << 124) for _ in range(2)]
        xs = [x & ((1 << L) - 1) for x in xs] + [0, (1 << L) - 1, alt]
        got = labs.general_flip_scores(L, xs).cpu().numpy()
        for i, x in enumerate(xs):
            s = _seq(L, x)
            C = np.array([0] + [int(np.dot(s[: L - k].astype(np.int64), s[k:])) for k in range(1, L)])
            want = [o.flip_isl_general(s, j, C) for j in range(L)]
            assert np.array_equal(got[i], want), (L, i)
    # the plain definition on a few states
    for L in (3, 64, 65, 128, 129, 192):
        x = (1 << L) - 1
        got = labs.general_flip_scores(L, [x]).cpu().numpy()[0]
        assert all(got[j] == o.flip_isl_general(_seq(L, x), j) for j in range(L)), L


def test_flip_scores_rejects_bad_lengths(labs):
    for L in (2, 193):
        with pytest.raises(labs.LabsError) as e:
            labs.general_flip_scores(L, [1])
        assert e.value.code == labs.LABS_EINVAL


def test_targets_traps_exact_table_untraced(labs):
    # the same kinds of walks without traces (the step loop built without trace tests, for tables
    # addressed by the free bits and by the hash)
    cfgs = [
        labs.make_cfg(4, SEED, 0, steps=60, table_log2=8),
        labs.make_cfg(13, SEED, 1, steps=3000, table_log2=14, target_isl=6),
        labs.make_cfg(20, SEED, 2, steps=1500, table_log2=22, restart_period=500),
        labs.make_cfg(100, SEED, 3, steps=400, watch_isl=1600),
    ]
    got, _ = labs.general_walk_batch(cfgs)
    for i, c in enumerate(cfgs):
        assert_same(got[i], oracle_general(c), i)


def test_mixed_lengths_and_batch_sample(labs):
    cfgs = [labs.make_cfg(L, SEED, w, steps=2000, table_log2=16) for L in (64, 101, 128, 192) for w in range(256)]
    got, _ = labs.general_walk_batch(cfgs)
    for i in (0, 255, 256, 511, 700, 1023):
        assert_same(got[i], oracle_general(cfgs[i]), i)
    for i in range(0, len(cfgs), 37):
        r, L = got[i], cfgs[i].L
        assert r["flip_evals"] == r["steps_done"] * L
        s = np.array([-1 if (r["best_bits"] >> j) & 1 else 1 for j in range(L)], dtype=np.int8)
        assert o.isl(s) == r["best_isl"]


def test_rejects_bad_config(labs):
    for bad in (dict(L=2), dict(L=193), dict(table_log2=0), dict(steps=-1), dict(steps=(1 << 30) + 1)):
        kw = dict(L=31, seed=1, walk_id=0, steps=10, table_log2=16)
        kw.update(bad)
        with pytest.raises(labs.LabsError) as e:
            labs.general_walk_batch([labs.make_cfg(**kw)])
        assert e.value.code == labs.LABS_EINVAL


def test_restart_states_count(labs):
    # general walks restarting after every step (and trapping at L = 4): restart states count for
    # the best, hit and watch like the initial state
    cfgs = []
    for w in range(6):
        ref = o.walk(12, SEED, w, steps=40, restart_period=1, table_log2=13, general=True)
        cfgs.append(labs.make_cfg(12, SEED, w, steps=40, restart_period=1, table_log2=13, trace=True))
        cfgs.append(labs.make_cfg(12, SEED, w, steps=40, restart_period=1, table_log2=13,
                                  watch_isl=ref["best_isl"], target_isl=ref["best_isl"], trace=True))
    cfgs.append(labs.make_cfg(4, SEED, 5, steps=50, table_log2=8, trace=True))
    got, _ = labs.general_walk_batch(cfgs)
    for i, c in enumerate(cfgs):
        assert_same(got[i], oracle_general(c), i)
