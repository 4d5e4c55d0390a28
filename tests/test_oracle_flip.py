"""Pins of the oracle's incremental one-flip evaluation against the plain definition."""
import random

import numpy as np
import pytest

from oracle import oracle as o
from tests import table1


@pytest.mark.parametrize("L", list(range(3, 304, 2)))
def test_incremental_equals_brute_force_every_flip(L):
    # Every flip of random skew sequences, every odd L in [3, 303]: the incremental score
    # equals the ISL recomputed from Eq. (1)-(2) after negating s_j and its mirror.
    rng = random.Random(1000 + L)
    n = (L + 1) // 2
    reps = 3 if L <= 101 else 1
    for _ in range(reps):
        x = rng.getrandbits(n)
        assert np.array_equal(o.flip_scores(L, x, brute=True), o.flip_scores(L, x, brute=False))


@pytest.mark.parametrize("row", table1.rows()[::7], ids=lambda r: f"L{r['L']}")
def test_incremental_on_table1_sequences(row):
    s = o.hex_decode(row["hex"], row["L"])
    x = o.skew_bits(s)
    assert np.array_equal(o.flip_scores(row["L"], x, True), o.flip_scores(row["L"], x, False))


def test_flip_keeps_skew_and_is_an_involution():
    rng = random.Random(5)
    L = 101
    n = 51
    x = rng.getrandbits(n)
    s = o.skew_expand(L, x)
    base = o.isl(s)
    for j in range(n):
        t = s.copy()
        t[j] = -t[j]
        if L - 1 - j != j:
            t[L - 1 - j] = -t[L - 1 - j]
        assert o.is_skew(t)
        assert o.skew_bits(t) == x ^ (1 << j)
        assert o.flip_isl_brute(t, j) == base


def test_centre_flip_is_not_the_general_formula():
    # The centre symbol has no separate mirror: its correlation change is half of what the
    # two-symbol formula would give.  The brute-force comparison above would catch either
    # mistake; this checks the centre explicitly on all skew sequences of L = 9.
    L, n = 9, 5
    for x in range(1 << n):
        s = o.skew_expand(L, x)
        assert o.flip_isl_incr(s, o.corr(s), n - 1) == o.flip_isl_brute(s, n - 1)
