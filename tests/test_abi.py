"""The C ABI: liblabs.so loads on a CPU-only host and exports every entry point include/labs.h
declares (no compute call is made here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "labs.h")
LIB = os.path.join(ROOT, "paper_2011_00068_amd", "liblabs.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(labs_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ("labs_isl", "labs_merit", "labs_walk_batch", "labs_search_submit", "labs_search_poll"):
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblabs.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert missing == []


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblabs.so not built")
def test_binding_lists_every_declared_symbol():
    import paper_2011_00068_amd as labs

    assert sorted(labs.EXPORTS) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblabs.so not built")
def test_strerror_without_device():
    lib = ctypes.CDLL(LIB)
    lib.labs_strerror.restype = ctypes.c_char_p
    assert lib.labs_strerror(0) == b"ok"
    assert lib.labs_strerror(-2) == b"sequence is not skew-symmetric"


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblabs.so not built")
def test_isl_threshold_through_the_abi():
    """labs_isl_threshold (Eq. (3)): F >= num/den <=> ISL <= floor(L^2 den / (2 num)).  Host
    arithmetic, so it runs without a GPU.  Checked on the F >= 8 and F >= 8.5 bounds at the ends and
    middle of Table 1's range and, for random arguments, by the defining inequalities of the floor
    (never by re-evaluating the same formula)."""
    import random

    lib = ctypes.CDLL(LIB)
    f = lib.labs_isl_threshold
    f.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
    out = ctypes.c_int64()

    def thr(L, num, den):
        rc = f(L, num, den, ctypes.byref(out))
        return rc, out.value

    # F = L^2 / (2 ISL): the largest ISL with F >= 8 is floor(L^2 / 16), with F >= 8.5 floor(L^2 / 17)
    for L, f8, f85 in ((201, 2525, 2376), (255, 4064, 3825), (303, 5738, 5400)):
        assert thr(L, 8, 1) == (0, f8)
        assert thr(L, 17, 2) == (0, f85)
        assert L * L / (2 * f8) >= 8.0 > L * L / (2 * (f8 + 1))
    rng = random.Random(2011000068)
    for _ in range(2000):
        L = rng.randint(1, 65535)
        num = rng.randint(1, 10 ** 6)
        den = rng.randint(1, 10 ** 6)
        rc, t = thr(L, num, den)
        assert rc == 0
        # t is the largest integer with 2 num t <= L^2 den
        assert 2 * num * t <= L * L * den < 2 * num * (t + 1)
    assert thr(255, 1, 1 << 62) == (0, (1 << 63) - 1)  # clamped
    for bad in ((0, 8, 1), (65536, 8, 1), (255, 0, 1), (255, 8, 0), (255, -1, 1)):
        assert thr(*bad)[0] == -1, bad
    assert f(255, 8, 1, None) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblabs.so not built")
def test_hex_codec_through_the_abi():
    """labs_from_hex / labs_to_hex (Table 1's notation, Section 4) against the oracle's codec: all 52
    printed rows, random sequences of every length 1..70 and of Table 1's lengths, and the error
    cases.  Host code, so it runs without a GPU."""
    import random

    import numpy as np

    from oracle import oracle as o
    from tests import table1

    lib = ctypes.CDLL(LIB)
    lib.labs_from_hex.argtypes = [ctypes.c_char_p, ctypes.c_int32, ctypes.c_void_p]
    lib.labs_to_hex.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_char_p, ctypes.c_int32]

    def from_hex(h, L):
        out = np.zeros(L, dtype=np.int8)
        return lib.labs_from_hex(h.encode(), L, out.ctypes.data), out

    def to_hex(s, cap=None):
        a = np.ascontiguousarray(s, dtype=np.int8)
        buf = ctypes.create_string_buffer((len(a) + 3) // 4 + 1 if cap is None else max(cap, 1))
        rc = lib.labs_to_hex(len(a), a.ctypes.data, buf, (len(a) + 3) // 4 + 1 if cap is None else cap)
        return rc, buf.value.decode()

    for row in table1.rows():
        rc, s = from_hex(row["hex"], row["L"])
        assert rc == 0
        assert np.array_equal(s, o.hex_decode(row["hex"], row["L"]))
        assert from_hex(row["hex"].lower(), row["L"])[1].tolist() == s.tolist()
        rc, h = to_hex(s)
        assert rc == 0 and h == o.hex_encode(s)
        assert h.lstrip("0") == row["hex"].lstrip("0")
    rng = random.Random(2011000068)
    for L in list(range(1, 71)) + list(range(201, 304, 2)):
        s = np.array([rng.choice((1, -1)) for _ in range(L)], dtype=np.int8)
        rc, h = to_hex(s)
        assert rc == 0 and h == o.hex_encode(s) and len(h) == (L + 3) // 4
        assert np.array_equal(from_hex(h, L)[1], s)
        assert np.array_equal(from_hex("00" + h, L)[1], s)  # extra leading zero digits drop too
    # symbol 0 is +1, 1 is -1, most significant bit first: "B" = 1011 -> - + - -
    assert from_hex("B", 4)[1].tolist() == [-1, 1, -1, -1]
    assert from_hex("3", 2)[1].tolist() == [-1, -1]
    assert to_hex([1, -1, 1, 1, -1])[1] == "09"
    EINVAL = -1
    assert from_hex("F", 3)[0] == EINVAL  # a dropped leading bit is 1
    untouched = np.full(5, 7, dtype=np.int8)  # a failed decode leaves s_out as it was
    assert lib.labs_from_hex(b"1G", 5, untouched.ctypes.data) == EINVAL and (untouched == 7).all()
    assert lib.labs_from_hex(b"21", 5, untouched.ctypes.data) == EINVAL and (untouched == 7).all()
    assert from_hex("0", 5)[0] == EINVAL  # fewer bits than symbols
    assert from_hex("0G", 5)[0] == EINVAL
    assert from_hex("1", 0)[0] == EINVAL
    assert to_hex([1, 0, -1])[0] == EINVAL
    assert to_hex([1] * 8, cap=2)[0] == EINVAL  # 2 digits need 3 bytes
    import paper_2011_00068_amd as labs

    row = table1.rows()[27]
    assert labs.to_hex(labs.from_hex(row["hex"], row["L"])) == o.hex_encode(o.hex_decode(row["hex"], row["L"]))
    with pytest.raises(labs.LabsError):
        labs.from_hex("F", 3)


@pytest.mark.skipif(not os.path.exists(LIB), reason="liblabs.so not built")
def test_empty_walk_batches_are_refused_without_device_work():
    """Every entry point that runs walks or searches refuses n_walks = 0 with LABS_EINVAL before it
    touches a device, so the check holds on a CPU-only host too."""
    lib = ctypes.CDLL(LIB)
    vp = ctypes.c_void_p
    EINVAL = -1
    h = vp()
    assert lib.labs_walk_plan_create(0, None, None, ctypes.byref(h)) == EINVAL
    assert lib.labs_walk_batch(0, None, None, None, None, None) == EINVAL
    opts = (ctypes.c_int32 * 16)()  # non-NULL options; only n_walks is at fault
    assert lib.labs_pq_walk_batch(0, None, opts, None, None, None, None, None) == EINVAL
    assert lib.labs_fi_walk_batch(0, None, opts, None, None, None, None, None) == EINVAL
    assert lib.labs_general_walk_batch(0, None, None, None, None, None, None) == EINVAL
    assert lib.labs_walk_plan_create(-3, None, None, ctypes.byref(h)) == EINVAL
