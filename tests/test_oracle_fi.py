"""Pins of the oracle's first-improvement search with perturbations (ref_fi_walk; the method of
Dimitrov et al. as Section 2 describes it): the incremental scores equal the plain definition,
an independent numpy statement of the same reading gives the same trajectory, every move is the
first improving flip in index order, perturbations happen exactly at one-flip local minima and
flip P distinct symbols, a perturbation of all n free symbols is the negation symmetry (ISL
unchanged), the perturbation draw is uniform, and at L = 31 the search reaches the enumerated
skew optimum.  The scan order, the perturbation draw and its size are readings of what the paper
leaves open (parity unpinned beyond these checks)."""
import numpy as np
import pytest

from oracle import oracle as o

SEED = 2011000068


def _isl_np(L, x):
    n = (L + 1) // 2
    c = n - 1
    s = np.array([-1 if (x >> j) & 1 else 1 for j in range(n)], dtype=np.int64)
    full = np.concatenate([s, [s[c - i] * (-1 if i % 2 else 1) for i in range(1, c + 1)]])
    corr = np.correlate(full, full, mode="full")[L:]  # C_1 .. C_{L-1} (Eq. (1))
    return int(np.sum(corr * corr))


def _draw(n, seed, walk_id, k, P):
    # the perturbation draw restated from SplitMix64 outputs
    kw = o.sm64_at(seed, walk_id)
    kp = o.sm64_at(kw, (1 << 32) + k)
    out, i = [], 0
    while len(out) < P:
        j = ((o.sm64_at(kp, i) >> 32) * n) >> 32
        if j not in out:
            out.append(j)
        i += 1
    return out


def _python_fi(L, walk_id, steps, P, restart_period=0):
    n = (L + 1) // 2
    restart = 0
    x = o.start_bits(L, SEED, walk_id, restart)
    isl = _isl_np(L, x)
    best, best_step, best_x = isl, 0, x
    trace, flips, k = [], 0, 0
    for t in range(steps):
        scores = [_isl_np(L, x ^ (1 << j)) for j in range(n)]
        improving = [j for j in range(n) if scores[j] < isl]
        if improving:
            j = improving[0]
            x ^= 1 << j
            flips += j + 1
            move = j
        else:
            for j in _draw(n, SEED, walk_id, k, P):
                x ^= 1 << j
            k += 1
            flips += n + P
            move = -1
        isl = _isl_np(L, x)
        trace.append((move, isl))
        if isl < best:
            best, best_step, best_x = isl, t + 1, x
        if restart_period and (t + 1) % restart_period == 0 and t + 1 < steps:
            restart += 1
            x = o.start_bits(L, SEED, walk_id, restart)
            isl = _isl_np(L, x)
            if isl < best:
                best, best_step, best_x = isl, t + 1, x
    return {"best_isl": best, "best_step": best_step, "best_bits": best_x, "final_bits": x, "final_isl": isl,
            "flip_evals": flips, "traps": k, "restarts": restart,
            "trace": np.array(trace, dtype=np.int32).reshape(-1, 2)}


@pytest.mark.parametrize("L,P,R", [(7, 1, 0), (15, 2, 0), (21, 3, 0), (31, 3, 50), (41, 5, 0), (25, 13, 0)])
def test_matches_independent_statement(L, P, R):
    steps = 150
    want = _python_fi(L, 4, steps, P, R)
    got = o.walk(L, SEED, 4, steps=steps, fi_perturb=P, restart_period=R, trace=True)
    for k in ("best_isl", "best_step", "best_bits", "final_bits", "final_isl", "flip_evals", "traps", "restarts"):
        assert got[k] == want[k], (k, got[k], want[k])
    assert np.array_equal(got["trace"], want["trace"])
    assert got["traps"] > 0  # perturbations did happen


@pytest.mark.parametrize("L,P", [(31, 3), (101, 4), (255, 3)])
def test_incremental_equals_plain_definition(L, P):
    steps = {31: 400, 101: 120, 255: 40}[L]
    a = o.walk(L, SEED, 1, steps=steps, fi_perturb=P, trace=True, score_trace=True)
    b = o.walk(L, SEED, 1, steps=steps, fi_perturb=P, trace=True, score_trace=True, brute=True)
    assert np.array_equal(a["trace"], b["trace"]) and np.array_equal(a["scores"], b["scores"])


def test_moves_are_first_improvements_and_perturbations_local_minima():
    L, P, steps = 45, 3, 300
    n = (L + 1) // 2
    r = o.walk(L, SEED, 2, steps=steps, fi_perturb=P, trace=True, score_trace=True)
    x = o.start_bits(L, SEED, 2, 0)
    isl = o.isl(o.skew_expand(L, x))
    evals, k = 0, 0
    for t in range(steps):
        sc = o.flip_scores(L, x, brute=True)
        assert np.array_equal(r["scores"][t], sc)
        j, new_isl = (int(v) for v in r["trace"][t])
        if j >= 0:
            assert sc[j] < isl and all(sc[:j] >= isl)  # the first strict improvement
            x ^= 1 << j
            evals += j + 1
        else:
            assert all(sc >= isl)  # a one-flip local minimum
            picks = o.perturb_indices(n, SEED, 2, k, P)
            assert len(set(picks)) == P and all(0 <= v < n for v in picks)
            for v in picks:
                x ^= 1 << v
            k += 1
            evals += n + P
        assert o.isl(o.skew_expand(L, x)) == new_isl
        isl = new_isl
    assert r["final_bits"] == x and r["flip_evals"] == evals and r["traps"] == k > 0


def test_perturbing_every_symbol_is_the_negation_symmetry():
    # P = n flips every free symbol: the whole sequence is negated, which keeps every C_k (Eq. (1)),
    # so the ISL after a perturbation equals the local minimum's
    L = 27
    n = (L + 1) // 2
    r = o.walk(L, SEED, 6, steps=200, fi_perturb=n, trace=True)
    isl_before = o.isl(o.skew_expand(L, o.start_bits(L, SEED, 6, 0)))
    seen = 0
    for j, isl in r["trace"]:
        if j < 0:
            assert isl == isl_before
            seen += 1
        isl_before = isl
    assert seen > 0


def test_perturbation_draw_is_uniform_and_distinct():
    # 4,000 draws of 3 symbols out of n = 51: every symbol about equally often (chi-square, 50
    # degrees of freedom, far below the 0.1 % point 86.7)
    n, P, draws = 51, 3, 4000
    counts = np.zeros(n)
    for k in range(draws):
        picks = o.perturb_indices(n, SEED, 11, k, P)
        assert len(set(picks)) == P
        counts[picks] += 1
    expect = draws * P / n
    chi2 = float(np.sum((counts - expect) ** 2 / expect))
    assert chi2 < 86.7
    assert o.perturb_indices(5, SEED, 0, 0, 5) != o.perturb_indices(5, SEED, 0, 1, 5)
    assert sorted(o.perturb_indices(5, SEED, 0, 3, 5)) == [0, 1, 2, 3, 4]


def test_l31_reaches_enumerated_optimum():
    r = o.walk(31, SEED, 0, steps=3000, fi_perturb=3)
    assert r["best_isl"] == int(o.enum_skew(31).min()) == 79


def test_target_watch_and_restarts():
    L = 101
    free = o.walk(L, SEED, 9, steps=400, fi_perturb=3, trace=True)
    level = int(free["trace"][150, 1])
    first = int(np.argmax(free["trace"][:, 1] <= level)) + 1
    hit = o.walk(L, SEED, 9, steps=400, fi_perturb=3, target_isl=level)
    assert hit["hit_step"] == first and hit["steps_done"] == first
    watch = o.walk(L, SEED, 9, steps=400, fi_perturb=3, watch_isl=level)
    assert watch["watch_step"] == first and watch["steps_done"] == 400
    rr = o.walk(L, SEED, 9, steps=400, fi_perturb=3, restart_period=100)
    assert rr["restarts"] == 3


def test_bad_arguments():
    for L, P in ((31, 17), (101, 33)):  # more than n, or more than 32 symbols
        with pytest.raises(RuntimeError):
            o.walk(L, SEED, 0, steps=10, fi_perturb=P)
