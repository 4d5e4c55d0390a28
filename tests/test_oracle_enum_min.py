"""Pins of the oracle's grouped skew-space minimum (Section 1's search-space reduction, Eq. (2),
(4)) against brute force over all 2^L sequences and an independent numpy evaluation."""
import numpy as np
import pytest

from oracle import oracle as o


def _np_skew(L, xs):
    """Expand free-bit vectors (numpy uint64) to +-1 sequences with the literal Eq. (4):
    s_j from bit j for j <= c, s_{c+i} = (-1)^i s_{c-i}."""
    n = (L + 1) // 2
    c = n - 1
    bits = (xs[:, None] >> np.arange(n, dtype=np.uint64)[None, :]) & np.uint64(1)
    S = np.empty((len(xs), L), dtype=np.int64)
    S[:, :n] = 1 - 2 * bits.astype(np.int64)
    for i in range(1, c + 1):
        S[:, c + i] = (-1) ** i * S[:, c - i]
    return S


def _np_isl(S):
    L = S.shape[1]
    isl = np.zeros(S.shape[0], dtype=np.int64)
    for k in range(1, L):
        Ck = np.sum(S[:, : L - k] * S[:, k:], axis=1)
        isl += Ck * Ck
    return isl


def _np_min(isl, xs):
    m = isl.min()
    hit = isl == m
    return int(m), int(hit.sum()), int(xs[hit].min())


@pytest.mark.parametrize("L", [3, 5, 7, 9, 11, 13, 15])
def test_full_space_matches_all_sequences_brute_force(L):
    # all 2^L sequences, filtered by the literal Eq. (4): minimum ISL, how many skew sequences
    # reach it, and the lowest free-bit vector among them
    idx = np.arange(1 << L, dtype=np.int64)
    S = 1 - 2 * ((idx[:, None] >> np.arange(L)[None, :]) & 1)
    n = (L + 1) // 2
    c = n - 1
    keep = np.ones(1 << L, dtype=bool)
    for i in range(1, c + 1):
        keep &= S[:, c + i] == ((-1) ** i) * S[:, c - i]
    S = S[keep]
    x = idx[keep] & ((1 << n) - 1)
    want = _np_min(_np_isl(S), x)
    got = o.enum_skew_min(L)
    assert (got["min_isl"], got["count"], got["first_x"]) == want
    assert got["states"] == 1 << n == len(x)


def test_barker_optima():
    # Barker 11 and 13 are skew-symmetric with ISL 5 and 6 (Section 1's definitions)
    assert o.enum_skew_min(11)["min_isl"] == 5
    assert o.enum_skew_min(13)["min_isl"] == 6


@pytest.mark.parametrize("L,r0,cnt", [(25, 0, 1 << 10), (41, 12345, 3000), (61, 1 << 27, 1500),
                                      (101, 987654321, 400), (125, (1 << 61) - 300, 300)])
def test_block_matches_numpy(L, r0, cnt):
    # a block of groups: the four members x, x^A, x^O, x^A^O of each x = r << 2 evaluated by
    # numpy with the literal Eq. (4) and Eq. (2)
    n = (L + 1) // 2
    A = (1 << n) - 1
    O = sum(1 << j for j in range(1, n, 2))
    r = np.arange(r0, r0 + cnt, dtype=np.uint64)
    base = r << np.uint64(2)
    xs = np.concatenate([base, base ^ np.uint64(A), base ^ np.uint64(O), base ^ np.uint64(A ^ O)])
    want = _np_min(_np_isl(_np_skew(L, xs)), xs)
    got = o.enum_skew_min(L, r0, r0 + cnt)
    assert (got["min_isl"], got["count"], got["first_x"]) == want
    assert got["states"] == 4 * cnt


def test_groups_cover_the_space_once():
    # every x of the n-bit space lies in exactly one group {r<<2, ^A, ^O, ^A^O}
    for L in (5, 9, 13):
        n = (L + 1) // 2
        A = (1 << n) - 1
        O = sum(1 << j for j in range(1, n, 2))
        seen = []
        for r in range(1 << (n - 2)):
            b = r << 2
            seen += [b, b ^ A, b ^ O, b ^ A ^ O]
        assert sorted(seen) == list(range(1 << n))


def test_empty_and_bad_blocks():
    assert o.enum_skew_min(31, 5, 5) == {"min_isl": -1, "count": 0, "first_x": 0, "states": 0}
    for args in ((31, 0, (1 << 14) + 1), (31, 6, 5), (32, 0, 1), (127, 0, 1)):
        with pytest.raises(ValueError):
            o.enum_skew_min(*args)
