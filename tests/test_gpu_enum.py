"""GPU parity of the grouped skew-space minimum (labs_enum_skew_min; Eq. (2), (4), Section 1's
search-space reduction) against the oracle, through the C ABI: whole spaces up to L = 41, blocks
at the start, middle and end of the space for every word count up to L = 125, and whole spaces
at L = 61 .. 69 (one to two launches) checked by properties and by the oracle around the result."""
import pytest

from oracle import oracle as o

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

KEYS = ("min_isl", "count", "first_x", "states")


@pytest.fixture(scope="module")
def labs():
    import paper_2011_00068_amd as labs

    labs.lib()
    return labs


def same(g, r):
    return tuple(g[k] for k in KEYS) == tuple(r[k] for k in KEYS)


@pytest.mark.parametrize("L", list(range(3, 42, 2)))
def test_whole_space_matches_oracle(labs, L):
    g = labs.enum_skew_min(L)
    r = o.enum_skew_min(L)
    assert same(g, r), (g, r)


def test_whole_space_agrees_with_stored_enumeration(labs):
    # the per-sequence enumeration of the same space (labs_enum_skew_dev) gives the same minimum,
    # count and lowest argument
    for L in (23, 31, 37):
        isl = labs.enum_skew(L).cpu().numpy()
        m = int(isl.min())
        hits = (isl == m).nonzero()[0]
        g = labs.enum_skew_min(L)
        assert (g["min_isl"], g["count"], g["first_x"]) == (m, len(hits), int(hits[0]))
    assert labs.enum_skew_min(31)["min_isl"] == 79


@pytest.mark.parametrize("L", [43, 61, 63, 65, 67, 95, 97, 99, 125])
def test_blocks_match_oracle(labs, L):
    n = (L + 1) // 2
    groups = 1 << (n - 2)
    width = 1 << 13 if L <= 67 else 1 << 11
    for r0 in (0, groups // 2 - width // 3, groups - width):
        for w in (width, 1, 7, 1001):  # ragged tails of the per-lane passes
            g = labs.enum_skew_min(L, r0, r0 + w)
            r = o.enum_skew_min(L, r0, r0 + w)
            assert same(g, r), (L, r0, w, g, r)


def _group_of(L, x):
    n = (L + 1) // 2
    A = (1 << n) - 1
    O = sum(1 << j for j in range(1, n, 2))
    for m in (x, x ^ A, x ^ O, x ^ A ^ O):
        if m & 3 == 0:
            return m >> 2
    raise AssertionError


@pytest.mark.parametrize("L", [61, 63, 69])
def test_whole_space_large(labs, L):
    # L = 69 covers 2^33 groups: more than one launch.  Checks: first_x reaches min_isl; halves
    # of the space combine to the whole; the oracle agrees on a block around first_x's group.
    n = (L + 1) // 2
    groups = 1 << (n - 2)
    g = labs.enum_skew_min(L)
    assert g["states"] == 1 << n
    assert g["min_isl"] > 0 and g["count"] >= 4 and g["count"] % 4 == 0
    assert o.isl(o.skew_expand(L, g["first_x"])) == g["min_isl"]
    a = labs.enum_skew_min(L, 0, groups // 2)
    b = labs.enum_skew_min(L, groups // 2, groups)
    assert min(a["min_isl"], b["min_isl"]) == g["min_isl"]
    parts = [p for p in (a, b) if p["min_isl"] == g["min_isl"]]
    assert sum(p["count"] for p in parts) == g["count"]
    assert min(p["first_x"] for p in parts) == g["first_x"]
    r = _group_of(L, g["first_x"])
    lo, hi = max(0, r - 700), min(groups, r + 700)
    near_g = labs.enum_skew_min(L, lo, hi)
    near_r = o.enum_skew_min(L, lo, hi)
    assert same(near_g, near_r)
    assert near_r["min_isl"] == g["min_isl"]


def test_empty_and_bad_blocks(labs):
    g = labs.enum_skew_min(61, 17, 17)
    assert (g["min_isl"], g["count"], g["first_x"], g["states"]) == (-1, 0, 0, 0)
    for args in ((61, 0, (1 << 29) + 1), (61, 9, 8), (127, 0, 1), (62, 0, 1), (1, 0, 1)):
        with pytest.raises(labs.LabsError) as e:
            labs.enum_skew_min(*args)
        assert e.value.code == labs.LABS_EINVAL


def _exhaustive_word_ops(L, sequences):
    # 3 word operations per 32-bit word of the L - k overlapping positions and 2 for C_k^2, per
    # even lag k, for every sequence scored (one per group of four)
    return sequences * sum(3 * ((L - k + 31) // 32) + 2 for k in range(2, L, 2))


@pytest.mark.parametrize("L", [13, 31, 61])
def test_word_ops_count(labs, L):
    # the branch and bound evaluates at most the exhaustive count of (sequence, lag) pairs and at
    # least every lag of one sequence per wave pass of 8 groups per lane; a block of one group
    # scores exactly one sequence at every lag (nothing to compare it with, so no cut)
    n = (L + 1) // 2
    groups = 1 << (n - 2)
    g = labs.enum_skew_min(L)
    assert 0 < g["word_ops"] <= _exhaustive_word_ops(L, groups)
    one = labs.enum_skew_min(L, groups // 3, groups // 3 + 1)
    assert one["word_ops"] == _exhaustive_word_ops(L, 1)
    assert labs.enum_skew_min(L, 5, 5)["word_ops"] == 0
