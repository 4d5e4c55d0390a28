"""Pins of the oracle's general (not skew-symmetric) walk: the one-flip evaluation against the
plain definition and numpy, the walk against its brute-force form, an exact visited set and an
independent Python statement, and the Barker-13 optimum found by brute force over all 2^13."""
import random

import numpy as np
import pytest

from oracle import oracle as o


def _np_isl(s):
    L = len(s)
    return int(sum(int(np.dot(s[: L - k].astype(np.int64), s[k:].astype(np.int64))) ** 2 for k in range(1, L)))


@pytest.mark.parametrize("L", [3, 4, 5, 8, 13, 32, 33, 64, 65, 100, 127, 128, 129, 192])
def test_flip_scores_match_definition(L):
    rng = np.random.default_rng(L)
    for _ in range(3):
        s = rng.choice(np.array([-1, 1], dtype=np.int8), size=L)
        C = o.corr(s)
        for j in range(L):
            t = s.copy()
            t[j] = -t[j]
            want = _np_isl(t)
            assert o.flip_isl_general(s, j) == want
            assert o.flip_isl_general(s, j, C) == want


@pytest.mark.parametrize("L", [3, 6, 13, 31, 64, 101, 150, 192])
def test_incremental_walk_equals_brute_walk(L):
    kw = dict(steps=120, table_log2=12, restart_period=50, general=True, trace=True, score_trace=True)
    a = o.walk(L, 4, 1, **kw)
    b = o.walk(L, 4, 1, brute=True, **kw)
    for k in a:
        if k in ("trace", "scores"):
            assert np.array_equal(a[k], b[k])
        else:
            assert a[k] == b[k], k


def test_bounded_table_equals_exact_set_and_never_revisits():
    for L in (9, 12, 16, 20):
        kw = dict(steps=400, table_log2=L + 1, general=True, trace=True)
        a = o.walk(L, 6, 0, **kw)
        b = o.walk(L, 6, 0, ideal=True, **kw)
        assert np.array_equal(a["trace"], b["trace"])
        assert a["best_isl"] == b["best_isl"]
        if a["restarts"] == 0:
            x = o.start_bits_general(L, 6, 0, 0)
            seen = {x}
            for j, _ in a["trace"]:
                x ^= 1 << int(j)
                assert x not in seen
                seen.add(x)


def _python_walk(L, seed, walk_id, steps):
    """The self-avoiding walk over general sequences, stated independently (exact visited set,
    numpy ISL, lowest flip index on ties, restart when every neighbour is visited)."""
    def seq(x):
        return np.array([-1 if (x >> i) & 1 else 1 for i in range(L)], dtype=np.int8)

    restart = 0
    x = o.start_bits_general(L, seed, walk_id, 0)
    seen = {x}
    best = _np_isl(seq(x))
    trace = []
    for _ in range(steps):
        opts = [(_np_isl(seq(x ^ (1 << j))), j) for j in range(L) if (x ^ (1 << j)) not in seen]
        if not opts:
            restart += 1
            x = o.start_bits_general(L, seed, walk_id, restart)
            seen = {x}
            trace.append((-1, _np_isl(seq(x))))
            continue
        v, j = min(opts)
        x ^= 1 << j
        seen.add(x)
        best = min(best, v)
        trace.append((j, v))
    return best, np.array(trace, dtype=np.int32)


@pytest.mark.parametrize("L", [4, 7, 10, 13])
def test_walk_matches_independent_statement(L):
    best, trace = _python_walk(L, 8, 3, 150)
    r = o.walk(L, 8, 3, steps=150, table_log2=L + 2, general=True, trace=True)
    assert r["best_isl"] == best
    assert np.array_equal(r["trace"], trace)


def test_barker13_is_reached_and_optimal():
    # brute force over all 2^13 sequences: the minimum ISL is 6 (Barker 13)
    idx = np.arange(1 << 13)
    S = 1 - 2 * ((idx[:, None] >> np.arange(13)[None, :]) & 1)
    isl = sum(np.sum(S[:, : 13 - k] * S[:, k:], axis=1) ** 2 for k in range(1, 13))
    assert int(isl.min()) == 6
    assert o.walk(13, 1, 0, steps=2000, table_log2=14, general=True)["best_isl"] == 6


def test_start_bits_cover_all_symbols():
    for L in (3, 64, 65, 192):
        xs = {o.start_bits_general(L, 1, w, 0) for w in range(32)}
        assert all(x >> L == 0 for x in xs)
        assert len(xs) == min(32, 1 << L)
    # the skew start draws the same stream over the n free symbols
    assert o.start_bits_general(101, 5, 2, 1) & ((1 << 51) - 1) == o.start_bits(101, 5, 2, 1)
