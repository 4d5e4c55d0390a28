"""Internal-consistency pins of the oracle's walk (the paper leaves the tie-break, the visited
table, the random start and the restart rule open; the oracle fixes them as its module header
states): the fast walk equals the walk
that recomputes every score from scratch, the bounded table equals an exact visited set while
nothing is evicted, the walk is self-avoiding, and restarts / targets behave as specified."""
import numpy as np
import pytest

from oracle import oracle as o

SEED = 2011000068


@pytest.mark.parametrize("L,steps", [(31, 3000), (101, 300), (201, 40), (303, 15)])
def test_fast_walk_equals_brute_force_walk(L, steps):
    a = o.walk(L, SEED, 3, steps=steps, trace=True, score_trace=True)
    b = o.walk(L, SEED, 3, steps=steps, trace=True, score_trace=True, brute=True)
    assert np.array_equal(a["trace"], b["trace"])
    assert np.array_equal(a["scores"], b["scores"])
    for key in ("best_isl", "best_step", "final_isl", "best_bits", "final_bits"):
        assert a[key] == b[key]


def _states(L, start, trace):
    x = start
    out = [x]
    for j, _ in trace:
        assert j >= 0
        x ^= 1 << int(j)
        out.append(x)
    return out


@pytest.mark.parametrize("L,steps,log2", [(31, 20000, 16), (101, 3000, 24)])
def test_bounded_table_equals_ideal_set_and_walk_self_avoids(L, steps, log2):
    a = o.walk(L, SEED, 0, steps=steps, table_log2=log2, trace=True)
    b = o.walk(L, SEED, 0, steps=steps, table_log2=log2, trace=True, ideal=True)
    assert np.array_equal(a["trace"], b["trace"])
    if b["traps"] == 0:
        xs = _states(L, o.start_bits(L, SEED, 0, 0), b["trace"])
        assert len(set(xs)) == len(xs)  # no state visited twice
        # ISL in the trace is the ISL of the state reached
        for x, (_, isl) in list(zip(xs[1:], b["trace"]))[:: max(1, steps // 50)]:
            assert o.isl(o.skew_expand(L, x)) == isl


def test_trace_scores_are_flip_scores_of_current_state():
    L = 61
    r = o.walk(L, SEED, 1, steps=50, trace=True, score_trace=True)
    xs = _states(L, o.start_bits(L, SEED, 1, 0), r["trace"])
    for t in range(50):
        assert np.array_equal(r["scores"][t], o.flip_scores(L, xs[t], brute=True))
        j, isl = r["trace"][t]
        assert isl == r["scores"][t][j]


def test_moves_take_best_unvisited_flip_lowest_index():
    L = 41
    r = o.walk(L, SEED, 2, steps=400, trace=True, score_trace=True, ideal=True)
    xs = _states(L, o.start_bits(L, SEED, 2, 0), r["trace"])
    seen = {xs[0]}
    for t in range(400):
        cand = [(int(r["scores"][t][j]), j) for j in range((L + 1) // 2)
                if (xs[t] ^ (1 << j)) not in seen]
        assert r["trace"][t][0] == min(cand)[1]
        seen.add(xs[t + 1])


def test_best_is_first_minimum_of_trace():
    L = 101
    r = o.walk(L, SEED, 4, steps=2000, trace=True)
    start_isl = o.isl(o.skew_expand(L, o.start_bits(L, SEED, 4, 0)))
    isl = np.concatenate([[start_isl], r["trace"][:, 1]])
    assert r["best_isl"] == isl.min()
    assert r["best_step"] == int(np.argmin(isl))  # strict improvement keeps the first
    xs = _states(L, o.start_bits(L, SEED, 4, 0), r["trace"])
    assert r["best_bits"] == xs[r["best_step"]]
    assert r["final_bits"] == xs[-1]
    assert r["flip_evals"] == 2000 * 51 and r["steps_done"] == 2000


def test_l31_walk_reaches_enumerated_optimum():
    opt = int(o.enum_skew(31).min())
    assert opt == 79
    r = o.walk(31, SEED, 0, steps=20000, table_log2=16)
    assert r["best_isl"] == opt


def test_restart_period_starts_from_next_random_state():
    L, R = 51, 40
    r = o.walk(L, SEED, 7, steps=R + 5, restart_period=R, trace=True, score_trace=True)
    assert r["restarts"] == 1
    x1 = o.start_bits(L, SEED, 7, 1)
    assert np.array_equal(r["scores"][R], o.flip_scores(L, x1, brute=True))
    # budget exactly R: no restart at the end
    r2 = o.walk(L, SEED, 7, steps=R, restart_period=R)
    assert r2["restarts"] == 0


def test_target_stops_and_watch_records():
    L = 101
    free = o.walk(L, SEED, 9, steps=500, trace=True)
    target = int(free["trace"][120, 1])
    first = int(np.argmax(free["trace"][:, 1] <= target)) + 1
    hit = o.walk(L, SEED, 9, steps=500, target_isl=target)
    assert hit["hit_step"] == first and hit["steps_done"] == first
    watch = o.walk(L, SEED, 9, steps=500, watch_isl=target)
    assert watch["watch_step"] == first and watch["steps_done"] == 500
    # a target met by the start state stops at step 0
    start_isl = o.isl(o.skew_expand(L, o.start_bits(L, SEED, 9, 0)))
    z = o.walk(L, SEED, 9, steps=500, target_isl=start_isl)
    assert z["hit_step"] == 0 and z["steps_done"] == 0


def test_trapped_walk_restarts():
    # L = 5 has 8 skew states; with an exact table the walk exhausts them, traps and restarts.
    r = o.walk(5, SEED, 0, steps=40, trace=True, table_log2=8)
    assert r["traps"] >= 1 and r["restarts"] == r["traps"]
    assert -1 in r["trace"][:, 0]


def _restart_every_step_statement(L, walk_id, steps):
    """The walk with a restart after every step and an exact table, stated independently from the
    start draws and the plain flip definition: from each start state x_r (occupied at step r) the
    one move goes to its best flip (lowest index on ties; nothing but x_r is visited yet), occupied
    at step r + 1, and the next start state follows at that same step."""
    occupied = []
    for r in range(steps):
        x = o.start_bits(L, SEED, walk_id, r)
        occupied.append((x, r))
        j = int(np.argmin(o.flip_scores(L, x, brute=True)))
        occupied.append((x ^ (1 << j), r + 1))
    return occupied, [o.isl(o.skew_expand(L, x)) for x, _ in occupied]


def test_restart_states_count_like_the_start_state():
    # Every occupied state counts for best, hit and watch: the start state (step 0), each
    # committed state, and each restart state (at the step after which it is occupied).  Found
    # among 300 walks: some whose best is a restart state, and levels first met by a restart state.
    L, S = 21, 40
    n = (L + 1) // 2
    best_from_restart = level_from_restart = 0
    for w in range(300):
        occ, isls = _restart_every_step_statement(L, w, S)
        r = o.walk(L, SEED, w, steps=S, restart_period=1, table_log2=n + 1)
        i = int(np.argmin(isls))  # first strict minimum
        assert (r["best_isl"], r["best_step"], r["best_bits"]) == (isls[i], occ[i][1], occ[i][0]), w
        assert r["restarts"] == S - 1 and r["steps_done"] == S
        best_from_restart += i % 2 == 0 and i > 0
        # a level met first by a restart state r >= 1: watch records its step, a target stops there
        for k in range(2, len(occ), 2):
            if min(isls[:k]) > isls[k]:
                level = isls[k]
                wr = o.walk(L, SEED, w, steps=S, restart_period=1, table_log2=n + 1, watch_isl=level)
                assert wr["watch_step"] == occ[k][1] and wr["steps_done"] == S
                tr = o.walk(L, SEED, w, steps=S, restart_period=1, table_log2=n + 1, target_isl=level)
                assert tr["hit_step"] == occ[k][1] and tr["steps_done"] == occ[k][1]
                assert tr["final_bits"] == occ[k][0] and tr["restarts"] == occ[k][1]
                level_from_restart += 1
                break
    assert best_from_restart > 0 and level_from_restart > 0


def test_trap_restart_state_counts():
    # L = 5 (8 skew states) with an exact table traps every few steps; each trap's restart state
    # is occupied at the trap step and counts for the best like any other state
    r = o.walk(5, SEED, 0, steps=40, trace=True, table_log2=8)
    start_isl = o.isl(o.skew_expand(5, o.start_bits(5, SEED, 0, 0)))
    isl = np.concatenate([[start_isl], r["trace"][:, 1]])
    assert r["traps"] >= 1
    assert r["best_isl"] == isl.min() and r["best_step"] == int(np.argmin(isl))
