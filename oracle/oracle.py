"""ctypes front-end of the oracle (labs_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the package smoke check and by the
CPU-baseline leg of the benchmark.  The GPU library never imports it, and nothing here is shared
with it.  Free-bit vectors are Python ints (bit j = free symbol s_j is -1); sequences are numpy
int8 arrays of +1/-1.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblabs_oracle.so")

MAX_WORDS = 8  # 64-bit free-bit words, n <= 512
BRUTE = 1
IDEAL = 2
GENERAL = 4

_lib = None


def lib():
    """Loads (building on first use) the oracle's shared library."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(
        os.path.join(HERE, "labs_oracle.c")
    ):
        from . import build as _b  # noqa: WPS433

        _b.build()
    L = ctypes.CDLL(LIB_PATH)
    i8p = ctypes.POINTER(ctypes.c_int8)
    i64p = ctypes.POINTER(ctypes.c_int64)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    i32p = ctypes.POINTER(ctypes.c_int32)
    L.ref_corr.argtypes = [ctypes.c_int32, i8p, i64p]
    L.ref_isl.argtypes = [ctypes.c_int32, i8p]
    L.ref_isl.restype = ctypes.c_int64
    L.ref_merit.argtypes = [ctypes.c_int32, i8p]
    L.ref_merit.restype = ctypes.c_double
    L.ref_psl.argtypes = [ctypes.c_int32, i8p]
    L.ref_psl.restype = ctypes.c_int64
    L.ref_is_skew.argtypes = [ctypes.c_int32, i8p]
    L.ref_is_skew.restype = ctypes.c_int
    L.ref_skew_expand.argtypes = [ctypes.c_int32, u64p, i8p]
    L.ref_skew_bits.argtypes = [ctypes.c_int32, i8p, u64p, ctypes.c_int32]
    L.ref_hex_decode.argtypes = [ctypes.c_char_p, ctypes.c_int32, i8p]
    L.ref_hex_decode.restype = ctypes.c_int
    L.ref_hex_encode.argtypes = [ctypes.c_int32, i8p, ctypes.c_char_p, ctypes.c_int32]
    L.ref_hex_encode.restype = ctypes.c_int
    L.ref_flip_isl_brute.argtypes = [ctypes.c_int32, i8p, ctypes.c_int32]
    L.ref_flip_isl_brute.restype = ctypes.c_int64
    L.ref_flip_isl_incr.argtypes = [ctypes.c_int32, i8p, i64p, ctypes.c_int32]
    L.ref_flip_isl_incr.restype = ctypes.c_int64
    L.ref_flip_scores.argtypes = [ctypes.c_int32, u64p, i64p, ctypes.c_int]
    L.ref_sm64_at.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    L.ref_sm64_at.restype = ctypes.c_uint64
    L.ref_start_bits.argtypes = [
        ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, u64p, ctypes.c_int32
    ]
    L.ref_zobrist.argtypes = [ctypes.c_int32]
    L.ref_zobrist.restype = ctypes.c_uint64
    L.ref_walk.argtypes = [ctypes.POINTER(WalkCfg), ctypes.POINTER(WalkResult), i32p, i32p]
    L.ref_walk.restype = ctypes.c_int
    L.ref_pq_walk.argtypes = [ctypes.POINTER(WalkCfg), ctypes.c_int32, ctypes.c_int32,
                              ctypes.POINTER(WalkResult), i32p, i32p]
    L.ref_pq_walk.restype = ctypes.c_int
    L.ref_flip_isl_general_brute.argtypes = [ctypes.c_int32, i8p, ctypes.c_int32]
    L.ref_flip_isl_general_brute.restype = ctypes.c_int64
    L.ref_flip_isl_general_incr.argtypes = [ctypes.c_int32, i8p, i64p, ctypes.c_int32]
    L.ref_flip_isl_general_incr.restype = ctypes.c_int64
    L.ref_start_bits_general.argtypes = [
        ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, u64p, ctypes.c_int32
    ]
    L.ref_fi_walk.argtypes = [ctypes.POINTER(WalkCfg), ctypes.c_int32, ctypes.POINTER(WalkResult), i32p, i32p]
    L.ref_fi_walk.restype = ctypes.c_int
    L.ref_perturb_indices.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64,
                                      ctypes.c_int32, i32p]
    L.ref_perturb_indices.restype = ctypes.c_int32
    L.ref_enum_skew.argtypes = [ctypes.c_int32, i64p]
    L.ref_enum_skew.restype = ctypes.c_int
    L.ref_enum_skew_min.argtypes = [ctypes.c_int32, ctypes.c_uint64, ctypes.c_uint64, i64p, u64p, u64p]
    L.ref_enum_skew_min.restype = ctypes.c_int
    _lib = L
    return L


class WalkCfg(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32),
        ("table_log2", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("walk_id", ctypes.c_uint32),
        ("flags", ctypes.c_uint32),
        ("steps", ctypes.c_int64),
        ("restart_period", ctypes.c_int64),
        ("target_isl", ctypes.c_int64),
        ("watch_isl", ctypes.c_int64),
    ]


class WalkResult(ctypes.Structure):
    _fields_ = [
        ("best_isl", ctypes.c_int64),
        ("best_step", ctypes.c_int64),
        ("steps_done", ctypes.c_int64),
        ("flip_evals", ctypes.c_int64),
        ("hit_step", ctypes.c_int64),
        ("watch_step", ctypes.c_int64),
        ("final_isl", ctypes.c_int64),
        ("restarts", ctypes.c_int32),
        ("traps", ctypes.c_int32),
        ("best_bits", ctypes.c_uint32 * (2 * MAX_WORDS)),
        ("final_bits", ctypes.c_uint32 * (2 * MAX_WORDS)),
    ]


def _i8(s):
    a = np.ascontiguousarray(np.asarray(s, dtype=np.int8))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))


def _words(x: int):
    arr = (ctypes.c_uint64 * MAX_WORDS)()
    for w in range(MAX_WORDS):
        arr[w] = (x >> (64 * w)) & 0xFFFFFFFFFFFFFFFF
    return arr


def _int_from_u32(words, n):
    v = 0
    for w in range((n + 31) // 32):
        v |= int(words[w]) << (32 * w)
    return v & ((1 << n) - 1)


# --- definitions ---------------------------------------------------------------------------

def corr(s):
    a, p = _i8(s)
    out = np.zeros(len(a), dtype=np.int64)
    lib().ref_corr(len(a), p, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return out


def isl(s) -> int:
    a, p = _i8(s)
    return int(lib().ref_isl(len(a), p))


def merit(s) -> float:
    a, p = _i8(s)
    return float(lib().ref_merit(len(a), p))


def psl(s) -> int:
    a, p = _i8(s)
    return int(lib().ref_psl(len(a), p))


def is_skew(s) -> bool:
    a, p = _i8(s)
    return bool(lib().ref_is_skew(len(a), p))


def skew_expand(L: int, x: int):
    out = np.zeros(L, dtype=np.int8)
    lib().ref_skew_expand(L, _words(x), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)))
    return out


def skew_bits(s) -> int:
    a, p = _i8(s)
    arr = (ctypes.c_uint64 * MAX_WORDS)()
    lib().ref_skew_bits(len(a), p, arr, MAX_WORDS)
    return sum(int(arr[w]) << (64 * w) for w in range(MAX_WORDS))


def hex_decode(hexstr: str, L: int):
    out = np.zeros(L, dtype=np.int8)
    rc = lib().ref_hex_decode(hexstr.encode(), L, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)))
    if rc != 0:
        raise ValueError(f"hex_decode failed ({rc})")
    return out


def hex_encode(s) -> str:
    a, p = _i8(s)
    buf = ctypes.create_string_buffer(len(a) // 4 + 8)
    rc = lib().ref_hex_encode(len(a), p, buf, len(buf))
    if rc < 0:
        raise ValueError("hex_encode failed")
    return buf.value.decode()


# --- one-flip evaluation -------------------------------------------------------------------

def flip_isl_brute(s, j: int) -> int:
    a, p = _i8(s)
    return int(lib().ref_flip_isl_brute(len(a), p, j))


def flip_isl_incr(s, C, j: int) -> int:
    a, p = _i8(s)
    Cc = np.ascontiguousarray(np.asarray(C, dtype=np.int64))
    return int(lib().ref_flip_isl_incr(len(a), p, Cc.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), j))


def flip_scores(L: int, x: int, brute: bool = False):
    n = (L + 1) // 2
    out = np.zeros(n, dtype=np.int64)
    lib().ref_flip_scores(L, _words(x), out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), int(brute))
    return out


# --- random numbers --------------------------------------------------------------------------

def sm64_at(seed: int, i: int) -> int:
    return int(lib().ref_sm64_at(seed & 0xFFFFFFFFFFFFFFFF, i & 0xFFFFFFFFFFFFFFFF))


def start_bits(L: int, seed: int, walk_id: int, restart: int) -> int:
    arr = (ctypes.c_uint64 * MAX_WORDS)()
    lib().ref_start_bits(L, seed & 0xFFFFFFFFFFFFFFFF, walk_id, restart, arr, MAX_WORDS)
    return sum(int(arr[w]) << (64 * w) for w in range(MAX_WORDS))


def start_bits_general(L: int, seed: int, walk_id: int, restart: int) -> int:
    arr = (ctypes.c_uint64 * MAX_WORDS)()
    lib().ref_start_bits_general(L, seed & 0xFFFFFFFFFFFFFFFF, walk_id, restart, arr, MAX_WORDS)
    return sum(int(arr[w]) << (64 * w) for w in range(MAX_WORDS))


def flip_isl_general(s, j, C=None):
    """ISL of the general sequence s with s_j negated: by the plain definition, or incrementally
    from the correlation table C when it is given."""
    s = np.ascontiguousarray(s, dtype=np.int8)
    i8p = ctypes.POINTER(ctypes.c_int8)
    if C is None:
        return int(lib().ref_flip_isl_general_brute(len(s), s.ctypes.data_as(i8p), j))
    C = np.ascontiguousarray(C, dtype=np.int64)
    return int(lib().ref_flip_isl_general_incr(len(s), s.ctypes.data_as(i8p),
                                               C.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), j))


def zobrist(j: int) -> int:
    return int(lib().ref_zobrist(j))


# --- the walk --------------------------------------------------------------------------------

def walk(L, seed, walk_id=0, steps=1000, table_log2=16, restart_period=0, target_isl=-1,
         watch_isl=-1, brute=False, ideal=False, trace=False, score_trace=False, pq_capacity=0,
         nbr_table_log2=0, general=False, fi_perturb=0):
    """Runs one walk; returns a dict of results (+ 'trace' (steps,2) / 'scores' (steps,n)).
    pq_capacity > 0 runs the best-first search with a queue of that capacity instead (and
    nbr_table_log2 > 0 adds the second table of evaluated neighbours).  general=True walks over
    general sequences (all L symbols free).  fi_perturb > 0 runs the first-improvement search
    with perturbations of that many symbols instead (traps = perturbations)."""
    n = L if general else (L + 1) // 2
    cfg = WalkCfg(L, table_log2, seed & 0xFFFFFFFFFFFFFFFF, walk_id,
                  (BRUTE if brute else 0) | (IDEAL if ideal else 0) | (GENERAL if general else 0),
                  steps, restart_period, target_isl, watch_isl)
    res = WalkResult()
    tr = np.zeros((max(steps, 1), 2), dtype=np.int32) if trace else None
    sc = np.zeros((max(steps, 1), n), dtype=np.int32) if score_trace else None
    i32p = ctypes.POINTER(ctypes.c_int32)
    trp = tr.ctypes.data_as(i32p) if tr is not None else None
    scp = sc.ctypes.data_as(i32p) if sc is not None else None
    if fi_perturb > 0:
        rc = lib().ref_fi_walk(ctypes.byref(cfg), fi_perturb, ctypes.byref(res), trp, scp)
    elif pq_capacity > 0:
        rc = lib().ref_pq_walk(ctypes.byref(cfg), pq_capacity, nbr_table_log2, ctypes.byref(res), trp, scp)
    else:
        rc = lib().ref_walk(ctypes.byref(cfg), ctypes.byref(res), trp, scp)
    if rc != 0:
        raise RuntimeError(f"ref_walk failed ({rc})")
    out = {
        "best_isl": res.best_isl, "best_step": res.best_step, "steps_done": res.steps_done,
        "flip_evals": res.flip_evals, "hit_step": res.hit_step, "watch_step": res.watch_step,
        "final_isl": res.final_isl, "restarts": res.restarts, "traps": res.traps,
        "best_bits": _int_from_u32(res.best_bits, n), "final_bits": _int_from_u32(res.final_bits, n),
    }
    if tr is not None:
        out["trace"] = tr[: res.steps_done]
    if sc is not None:
        out["scores"] = sc[: res.steps_done]
    return out


def perturb_indices(n: int, seed: int, walk_id: int, k: int, P: int):
    """The free symbols that perturbation k of a first-improvement walk flips (in draw order)."""
    out = np.zeros(P, dtype=np.int32)
    got = lib().ref_perturb_indices(n, seed & 0xFFFFFFFFFFFFFFFF, walk_id, k, P,
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return [int(v) for v in out[:got]]


def enum_skew(L: int):
    n = (L + 1) // 2
    out = np.zeros(1 << n, dtype=np.int64)
    rc = lib().ref_enum_skew(L, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    if rc != 0:
        raise ValueError("enum_skew failed")
    return out


def enum_skew_min(L: int, r_begin: int = 0, r_end=None):
    """Lowest ISL over the symmetry groups r_begin .. r_end - 1 of the skew space (all of it by
    default): {"min_isl", "count", "first_x", "states"}."""
    n = (L + 1) // 2
    if r_end is None:
        r_end = 1 << (n - 2)
    mn = ctypes.c_int64()
    cnt = ctypes.c_uint64()
    first = ctypes.c_uint64()
    rc = lib().ref_enum_skew_min(L, r_begin, r_end, ctypes.byref(mn), ctypes.byref(cnt), ctypes.byref(first))
    if rc != 0:
        raise ValueError("enum_skew_min: bad arguments")
    return {"min_isl": mn.value, "count": cnt.value, "first_x": first.value, "states": 4 * (r_end - r_begin)}
