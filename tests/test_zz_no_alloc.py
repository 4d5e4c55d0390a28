"""The allocation-free entry point labs_enum_skew_min_noalloc, through the C ABI, against the
allocating labs_enum_skew_min on the same inputs (every result field, bit for bit) on two calls
in a row, the second smaller than the first, so that nothing left in the shared device array by
the first call may leak into the second."""
import ctypes

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FIELDS = ("min_isl", "count", "first_x", "states", "word_ops")


@pytest.fixture(scope="module")
def lib():
    import paper_2011_00068_amd as labs

    return labs.lib(), labs


def _call(fn, labs, L, r0, r1):
    res = labs.EnumMinResult()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = fn(L, r0, r1, ctypes.byref(res), stream)
    return rc, {f: getattr(res, f) for f in FIELDS}, res.kernel_ms


def test_noalloc_equals_allocating_entry_point(lib):
    L_, labs = lib
    torch.cuda.set_device(0)
    # whole L = 61 space (2^29 groups), then a smaller ragged block at L = 43, then a one-group
    # block at L = 125 (four words per sequence)
    cases = ((61, 0, 1 << 29), (43, 12345, 12345 + 70001), (125, (1 << 61) - 3, (1 << 61) - 2))
    for L, r0, r1 in cases:
        rc_n, got, ms = _call(L_.labs_enum_skew_min_noalloc, labs, L, r0, r1)
        rc_a, want, _ = _call(L_.labs_enum_skew_min, labs, L, r0, r1)
        assert rc_n == 0 and rc_a == 0, (L, rc_n, rc_a)
        assert got == want, (L, r0, r1, got, want)
        assert ms == -1.0
    # the same small block again right after the big one: identical to the first call's answer
    rc, again, _ = _call(L_.labs_enum_skew_min_noalloc, labs, 43, 12345, 12345 + 70001)
    assert rc == 0
    assert again == _call(L_.labs_enum_skew_min, labs, 43, 12345, 12345 + 70001)[1]


def test_noalloc_against_oracle_and_errors(lib):
    from oracle import oracle as o

    L_, labs = lib
    for L in (25, 31):
        rc, got, _ = _call(L_.labs_enum_skew_min_noalloc, labs, L, 0, 1 << ((L + 1) // 2 - 2))
        r = o.enum_skew_min(L)
        assert rc == 0
        assert tuple(got[k] for k in ("min_isl", "count", "first_x", "states")) == \
            (r["min_isl"], r["count"], r["first_x"], r["states"])
    rc, got, _ = _call(L_.labs_enum_skew_min_noalloc, labs, 61, 9, 9)
    assert rc == 0 and got["min_isl"] == -1 and got["states"] == 0
    for args in ((61, 0, (1 << 29) + 1), (61, 9, 8), (127, 0, 1), (62, 0, 1)):
        assert _call(L_.labs_enum_skew_min_noalloc, labs, *args)[0] == labs.LABS_EINVAL
