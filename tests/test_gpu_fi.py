"""GPU parity of the first-improvement search with perturbations (labs_fi_walk_batch; the method
of Dimitrov et al. described in Section 2) against the oracle, through the C ABI: full traces
(move or perturbation, ISL per step), every step's flip scores and the per-walk results, bit for
bit, at every kernel shape (matrix-core scoring at every length), with
restarts, targets, watch levels and perturbation sizes from 1 to 32 symbols."""
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


def oracle_fi(c, P):
    return o.walk(c.L, c.seed, c.walk_id, steps=c.steps, restart_period=c.restart_period, target_isl=c.target_isl,
                  watch_isl=c.watch_isl, trace=bool(c.flags & 1), score_trace=bool(c.flags & 2), fi_perturb=P)


def assert_same(g, r, what=""):
    for k in KEYS:
        assert g[k] == r[k], (what, k, g[k], r[k])
    for k in ("trace", "scores"):
        if k in r and k in g:
            T = r["steps_done"]
            assert np.array_equal(g[k][:T], r[k][:T]), (what, k)


@pytest.mark.parametrize("L", [3, 5, 7, 31, 63, 65, 101, 127, 129, 131, 191, 193, 195, 201, 255, 257, 259, 303,
                               321, 383])
def test_every_shape_matches_oracle(labs, L):
    n = (L + 1) // 2
    P = min(3, n)
    cfgs = [labs.make_cfg(L, SEED + L, w, steps=300, restart_period=110, trace=True, score_trace=(w == 0))
            for w in range(3)]
    got, ms = labs.fi_walk_batch(cfgs, P)
    assert ms >= 0
    for w, c in enumerate(cfgs):
        r = oracle_fi(c, P)
        assert_same(got[w], r, (L, w))
    assert any(g["traps"] > 0 for g in got)  # perturbations happened


@pytest.mark.parametrize("P", [1, 2, 5, 16, 32])
def test_perturbation_sizes(labs, P):
    cfgs = [labs.make_cfg(L, SEED, w, steps=250, trace=True) for L in (63, 101, 255) for w in range(2)]
    got, _ = labs.fi_walk_batch(cfgs, P)
    for i, c in enumerate(cfgs):
        assert_same(got[i], oracle_fi(c, P), (c.L, P, i))


def test_targets_watch_restarts_and_mixed_lengths(labs):
    free = o.walk(101, SEED, 9, steps=400, fi_perturb=3, trace=True)
    level = int(free["trace"][150, 1])
    cfgs = [
        labs.make_cfg(101, SEED, 9, steps=400, target_isl=level, trace=True),
        labs.make_cfg(101, SEED, 9, steps=400, watch_isl=level, trace=True),
        labs.make_cfg(21, SEED, 2, steps=60, restart_period=1, trace=True),
        labs.make_cfg(255, SEED, 4, steps=500, restart_period=70, watch_isl=7000),
        labs.make_cfg(255, SEED, 4, steps=0),
        labs.make_cfg(31, SEED, 0, steps=3000),  # reaches the skew optimum ISL 79
    ] + [labs.make_cfg(L, SEED, 1, steps=200) for L in range(201, 304, 10)]
    got, _ = labs.fi_walk_batch(cfgs, 3)
    for i, c in enumerate(cfgs):
        assert_same(got[i], oracle_fi(c, 3), i)
    assert got[0]["hit_step"] >= 0 and got[0]["steps_done"] == got[0]["hit_step"]
    assert got[5]["best_isl"] == 79


def test_l255_batch_sample(labs):
    # a full-width batch at the headline length: sampled searches against the oracle
    cfgs = [labs.make_cfg(255, SEED, w, steps=2000) for w in range(4096)]
    got, _ = labs.fi_walk_batch(cfgs, 3)
    for w in (0, 1, 2047, 4095):
        assert_same(got[w], oracle_fi(cfgs[w], 3), w)
    for w in range(0, 4096, 97):
        r = got[w]
        assert o.isl(o.skew_expand(255, r["best_bits"])) == r["best_isl"]
        assert o.isl(o.skew_expand(255, r["final_bits"])) == r["final_isl"]


def test_rejects_bad_options(labs):
    for P in (0, 33):
        with pytest.raises(labs.LabsError) as e:
            labs.fi_walk_batch([labs.make_cfg(101, SEED, 0, steps=10)], P)
        assert e.value.code == labs.LABS_EINVAL
    with pytest.raises(labs.LabsError) as e:
        labs.fi_walk_batch([labs.make_cfg(7, SEED, 0, steps=10)], 5)  # more than n = 4 symbols
    assert e.value.code == labs.LABS_EINVAL
