"""Python binding of liblabs (include/labs.h): argument marshalling only.

Every function here forwards to the C ABI of the in-tree liblabs.so, whose gfx950 kernels do all
the work; nothing is computed in Python.  torch is used for device memory and streams: device
buffers are torch CUDA tensors and the stream is torch's current stream.  torch is imported
before liblabs.so is loaded so that both share the one HIP runtime of the process.

If liblabs.so has not been built (``python -m paper_2011_00068_amd.build`` or
``__graft_entry__.build()``), ``lib()`` raises: there is no fallback.
"""
import ctypes
import os
import time

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblabs.so")

LABS_OK = 0
LABS_EINVAL = -1
LABS_ENOTSKEW = -2
LABS_ENOMEM = -3
LABS_EPENDING = -4
LABS_ENOTFOUND = -5
LABS_EDEVICE = -6
LABS_EDOM = -7
LABS_ECANCELLED = -8

WALK_L_MAX = 383
X_WORDS = 6
TRACE = 1
TRACE_SCORES = 2

VARIANT_AUTO = 0
VARIANT_BITSLICE = 1
VARIANT_DIRECT = 2
VARIANT_MFMA = 3

JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_CANCELLED = 0, 1, 2, 3

# Every symbol include/labs.h declares (checked by the tests).
EXPORTS = [
    "labs_strerror", "labs_last_error", "labs_device_info", "labs_probe_lds_read",
    "labs_isl", "labs_merit", "labs_isl_threshold", "labs_from_hex", "labs_to_hex", "labs_isl_batch_dev", "labs_enum_skew_dev", "labs_enum_skew_min",
    "labs_enum_skew_min_noalloc",
    "labs_flip_scores_dev",
    "labs_walk_batch", "labs_walk_plan_create", "labs_walk_plan_run", "labs_walk_plan_results",
    "labs_walk_plan_get_opts", "labs_walk_plan_last_timing", "labs_walk_plan_destroy",
    "labs_autotune", "labs_autotune_batch", "labs_pq_walk_batch", "labs_fi_walk_batch", "labs_general_walk_batch", "labs_general_flip_scores_dev",
    "labs_server_create", "labs_search_submit", "labs_search_poll", "labs_search_wait",
    "labs_search_cancel", "labs_search_release", "labs_server_stats", "labs_server_destroy",
]


class LabsError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        msg = ""
        if _lib is not None:
            msg = _lib.labs_last_error().decode(errors="replace")
            name = _lib.labs_strerror(code).decode()
        else:
            name = str(code)
        super().__init__(f"{where}: {name} ({code}){': ' + msg if msg else ''}")


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
        ("best_bits", ctypes.c_uint32 * X_WORDS),
        ("final_bits", ctypes.c_uint32 * X_WORDS),
    ]


class PlanOpts(ctypes.Structure):
    _fields_ = [
        ("variant", ctypes.c_int32),
        ("waves_per_block", ctypes.c_int32),
        ("probe_width", ctypes.c_int32),
        ("plain", ctypes.c_int32),
        ("steps_per_launch", ctypes.c_int64),
        ("use_graph", ctypes.c_int32),
        ("persistent", ctypes.c_int32),
    ]


class EnumMinResult(ctypes.Structure):
    _fields_ = [
        ("min_isl", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("count", ctypes.c_uint64),
        ("first_x", ctypes.c_uint64),
        ("states", ctypes.c_uint64),
        ("kernel_ms", ctypes.c_double),
        ("word_ops", ctypes.c_uint64),
    ]


class PqOpts(ctypes.Structure):
    _fields_ = [("capacity", ctypes.c_int32), ("nbr_table_log2", ctypes.c_int32)]


class FiOpts(ctypes.Structure):
    _fields_ = [("perturb_bits", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class ServerOpts(ctypes.Structure):
    _fields_ = [
        ("device_mem_bytes", ctypes.c_int64),
        ("table_log2", ctypes.c_int32),
        ("steps_per_tick", ctypes.c_int32),
        ("max_walks", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
    ]


class SearchReq(ctypes.Structure):
    _fields_ = [
        ("L", ctypes.c_int32),
        ("n_walks", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("flip_budget", ctypes.c_int64),
        ("target_F_num", ctypes.c_int64),
        ("target_F_den", ctypes.c_int64),
    ]


class SearchStatus(ctypes.Structure):
    _fields_ = [
        ("state", ctypes.c_int32),
        ("best_walk", ctypes.c_int32),
        ("best_isl", ctypes.c_int64),
        ("best_F", ctypes.c_double),
        ("hit_step", ctypes.c_int64),
        ("hit_walk", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("steps_done", ctypes.c_int64),
        ("flip_evals", ctypes.c_int64),
        ("t_submit", ctypes.c_double),
        ("t_admit", ctypes.c_double),
        ("t_done", ctypes.c_double),
        ("best_bits", ctypes.c_uint32 * X_WORDS),
    ]


_lib = None


def lib():
    """The loaded liblabs.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"liblabs.so not found at {LIB_PATH}: build it with __graft_entry__.build() "
            "(there is no CPU fallback)"
        )
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    P = ctypes.POINTER
    L.labs_strerror.restype = ctypes.c_char_p
    L.labs_strerror.argtypes = [ctypes.c_int]
    L.labs_last_error.restype = ctypes.c_char_p
    L.labs_last_error.argtypes = []
    L.labs_device_info.argtypes = [ctypes.c_char_p, i32, P(i32), P(i32)]
    L.labs_probe_lds_read.argtypes = [i32, P(ctypes.c_double), P(ctypes.c_double)]
    L.labs_isl.argtypes = [i32, vp, P(i64)]
    L.labs_merit.argtypes = [i32, vp, P(ctypes.c_double)]
    L.labs_isl_threshold.argtypes = [i32, i64, i64, P(i64)]
    L.labs_from_hex.argtypes = [ctypes.c_char_p, i32, vp]
    L.labs_to_hex.argtypes = [i32, vp, ctypes.c_char_p, i32]
    L.labs_isl_batch_dev.argtypes = [i32, i32, vp, vp, vp, vp, vp, vp]
    L.labs_enum_skew_dev.argtypes = [i32, vp, vp]
    L.labs_enum_skew_min.argtypes = [i32, u64, u64, P(EnumMinResult), vp]
    L.labs_enum_skew_min_noalloc.argtypes = [i32, u64, u64, P(EnumMinResult), vp]
    L.labs_flip_scores_dev.argtypes = [i32, i32, vp, vp, i32, vp]
    L.labs_walk_batch.argtypes = [i32, P(WalkCfg), P(WalkResult), vp, vp, vp]
    L.labs_walk_plan_create.argtypes = [i32, P(WalkCfg), P(PlanOpts), P(vp)]
    L.labs_walk_plan_run.argtypes = [vp, vp]
    L.labs_walk_plan_results.argtypes = [vp, P(WalkResult), vp, vp]
    L.labs_walk_plan_get_opts.argtypes = [vp, P(PlanOpts)]
    L.labs_walk_plan_last_timing.argtypes = [vp, P(ctypes.c_double), P(i32)]
    L.labs_walk_plan_destroy.argtypes = [vp]
    L.labs_walk_plan_destroy.restype = None
    L.labs_autotune.argtypes = [i32, i32, P(PlanOpts)]
    L.labs_autotune_batch.argtypes = [i32, P(WalkCfg), P(PlanOpts)]
    L.labs_pq_walk_batch.argtypes = [i32, P(WalkCfg), P(PqOpts), P(WalkResult), vp, vp,
                                     P(ctypes.c_double), vp]
    L.labs_fi_walk_batch.argtypes = [i32, P(WalkCfg), P(FiOpts), P(WalkResult), vp, vp, P(ctypes.c_double), vp]
    L.labs_general_walk_batch.argtypes = [i32, P(WalkCfg), P(WalkResult), vp, vp, P(ctypes.c_double), vp]
    L.labs_general_flip_scores_dev.argtypes = [i32, i32, vp, vp, vp]
    L.labs_server_create.argtypes = [P(ServerOpts), P(vp)]
    L.labs_search_submit.argtypes = [vp, P(SearchReq), P(u64)]
    L.labs_search_poll.argtypes = [vp, u64, P(SearchStatus)]
    L.labs_search_wait.argtypes = [vp, u64, i64, P(SearchStatus)]
    L.labs_search_cancel.argtypes = [vp, u64]
    L.labs_search_release.argtypes = [vp, u64]
    L.labs_server_stats.argtypes = [vp, P(i64), P(i32), P(i32), P(i64)]
    L.labs_server_destroy.argtypes = [vp]
    L.labs_server_destroy.restype = None
    _lib = L
    return L


def _check(rc, where):
    if rc != LABS_OK:
        raise LabsError(rc, where)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def device_info():
    name = ctypes.create_string_buffer(64)
    cu, clk = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().labs_device_info(name, 64, ctypes.byref(cu), ctypes.byref(clk)), "labs_device_info")
    return {"name": name.value.decode(), "compute_units": cu.value, "clock_khz": clk.value}


def probe_lds_read(bytes_per_lane=8):
    """LDS read bandwidth of the device in bytes/s for 4-, 8- or 16-byte reads per lane (a
    measurement aid for the walk kernels' LDS roof; see labs_probe_lds_read)."""
    bps = ctypes.c_double()
    ms = ctypes.c_double()
    _check(lib().labs_probe_lds_read(int(bytes_per_lane), ctypes.byref(bps), ctypes.byref(ms)),
           "labs_probe_lds_read")
    return {"bytes_per_s": bps.value, "ms": ms.value}


# --- definitions -------------------------------------------------------------------------------

def _host_i8(s):
    import numpy as np

    a = np.ascontiguousarray(np.asarray(s, dtype=np.int8))
    return a, ctypes.c_void_p(a.ctypes.data)


def isl(s) -> int:
    a, p = _host_i8(s)
    out = ctypes.c_int64()
    _check(lib().labs_isl(len(a), p, ctypes.byref(out)), "labs_isl")
    return out.value


def merit(s) -> float:
    a, p = _host_i8(s)
    out = ctypes.c_double()
    _check(lib().labs_merit(len(a), p, ctypes.byref(out)), "labs_merit")
    return out.value


def from_hex(hexstr, L):
    """labs_from_hex: Table 1's hex notation (Section 4) to L symbols +1 / -1 (numpy int8)."""
    import numpy as np

    out = np.empty(int(L), dtype=np.int8)
    _check(lib().labs_from_hex(hexstr.encode(), int(L), out.ctypes.data), "labs_from_hex")
    return out


def to_hex(s) -> str:
    """labs_to_hex: symbols +1 / -1 to Table 1's hex notation, ceil(L/4) upper-case digits."""
    a, p = _host_i8(s)
    buf = ctypes.create_string_buffer((len(a) + 3) // 4 + 1)
    _check(lib().labs_to_hex(len(a), p, buf, len(buf)), "labs_to_hex")
    return buf.value.decode()


def isl_batch(s_dev, with_F=True, with_psl=True, with_corr=False):
    """s_dev: int8 CUDA tensor [count, L].  Returns (isl int64, F float64 | None, psl int32 |
    None, corr int32 [count, L] | None), all CUDA tensors on the current stream."""
    assert s_dev.is_cuda and s_dev.dtype == torch.int8 and s_dev.dim() == 2
    s_dev = s_dev.contiguous()
    count, L = s_dev.shape
    dev = s_dev.device
    isl_t = torch.empty(count, dtype=torch.int64, device=dev)
    F_t = torch.empty(count, dtype=torch.float64, device=dev) if with_F else None
    psl_t = torch.empty(count, dtype=torch.int32, device=dev) if with_psl else None
    corr_t = torch.empty(count, L, dtype=torch.int32, device=dev) if with_corr else None
    _check(lib().labs_isl_batch_dev(L, count, _ptr(s_dev), _ptr(isl_t), _ptr(F_t), _ptr(psl_t),
                                    _ptr(corr_t), _stream()), "labs_isl_batch_dev")
    return isl_t, F_t, psl_t, corr_t


def enum_skew(L, device="cuda"):
    n = (L + 1) // 2
    out = torch.empty(1 << n, dtype=torch.int32, device=device)
    _check(lib().labs_enum_skew_dev(L, _ptr(out), _stream()), "labs_enum_skew_dev")
    return out


def enum_skew_min(L, r_begin=0, r_end=None):
    """Lowest ISL over the symmetry groups r_begin .. r_end - 1 of the odd-length-L skew space
    (the whole space by default): {"min_isl", "count", "first_x", "states", "kernel_ms",
    "word_ops"}."""
    n = (L + 1) // 2
    if r_end is None:
        r_end = 1 << max(0, n - 2)
    res = EnumMinResult()
    _check(lib().labs_enum_skew_min(L, r_begin, r_end, ctypes.byref(res), _stream()), "labs_enum_skew_min")
    return {"min_isl": res.min_isl, "count": res.count, "first_x": res.first_x, "states": res.states,
            "kernel_ms": res.kernel_ms, "word_ops": res.word_ops}


def enum_skew_min_noalloc(L, r_begin=0, r_end=None):
    """enum_skew_min through labs_enum_skew_min_noalloc (no device allocation; kernel_ms = -1)."""
    n = (L + 1) // 2
    if r_end is None:
        r_end = 1 << max(0, n - 2)
    res = EnumMinResult()
    _check(lib().labs_enum_skew_min_noalloc(L, r_begin, r_end, ctypes.byref(res), _stream()),
           "labs_enum_skew_min_noalloc")
    return {"min_isl": res.min_isl, "count": res.count, "first_x": res.first_x, "states": res.states,
            "kernel_ms": res.kernel_ms, "word_ops": res.word_ops}


def x_words(x: int):
    """Free-bit vector (Python int) -> list of LABS_X_WORDS uint32 words."""
    return [(x >> (32 * w)) & 0xFFFFFFFF for w in range(X_WORDS)]


def words_to_int(words, n):
    v = 0
    for w in range((n + 31) // 32):
        v |= int(words[w]) << (32 * w)
    return v & ((1 << n) - 1)


def flip_scores(L, xs, variant=VARIANT_BITSLICE, device="cuda"):
    """Scores of every flip of each skew state in xs (Python ints).  Returns int32 [count, n]."""
    n = (L + 1) // 2
    words = torch.tensor([x_words(x) for x in xs], dtype=torch.int64).to(torch.int32)
    x_dev = words.to(device).contiguous()
    out = torch.empty(len(xs), n, dtype=torch.int32, device=device)
    _check(lib().labs_flip_scores_dev(L, len(xs), _ptr(x_dev), _ptr(out), variant, _stream()),
           "labs_flip_scores_dev")
    return out


def general_flip_scores(L, xs, device="cuda"):
    """Scores of every one-symbol flip of each general sequence in xs (Python ints, bit j = b_j).
    Returns int32 [count, L]."""
    words = torch.tensor([x_words(x) for x in xs], dtype=torch.int64).to(torch.int32)
    x_dev = words.to(device).contiguous()
    out = torch.empty(len(xs), L, dtype=torch.int32, device=device)
    _check(lib().labs_general_flip_scores_dev(L, len(xs), _ptr(x_dev), _ptr(out), _stream()),
           "labs_general_flip_scores_dev")
    return out


# --- walks -------------------------------------------------------------------------------------

def make_cfg(L, seed, walk_id=0, steps=1000, table_log2=16, restart_period=0, target_isl=-1,
             watch_isl=-1, trace=False, score_trace=False):
    flags = (TRACE if trace else 0) | (TRACE_SCORES if score_trace else 0)
    return WalkCfg(L, table_log2, seed & 0xFFFFFFFFFFFFFFFF, walk_id, flags, steps, restart_period,
                   target_isl, watch_isl)


def _result_dict(r, n):
    return {
        "best_isl": r.best_isl, "best_step": r.best_step, "steps_done": r.steps_done,
        "flip_evals": r.flip_evals, "hit_step": r.hit_step, "watch_step": r.watch_step,
        "final_isl": r.final_isl, "restarts": r.restarts, "traps": r.traps,
        "best_bits": words_to_int(r.best_bits, n), "final_bits": words_to_int(r.final_bits, n),
    }


def _split_traces(cfgs, trace_buf, score_buf, general=False):
    import numpy as np

    traces, scores = [], []
    to = so = 0
    for c in cfgs:
        n = c.L if general else (c.L + 1) // 2
        if c.flags & TRACE:
            traces.append(np.frombuffer(trace_buf, dtype=np.int32)[2 * to: 2 * (to + c.steps)].reshape(c.steps, 2).copy())
            to += c.steps
        else:
            traces.append(None)
        if c.flags & TRACE_SCORES:
            scores.append(np.frombuffer(score_buf, dtype=np.int32)[so: so + c.steps * n].reshape(c.steps, n).copy())
            so += c.steps * n
        else:
            scores.append(None)
    return traces, scores


class WalkPlan:
    """A batch of walks with resident device state (labs_walk_plan_*)."""

    def __init__(self, cfgs, variant=VARIANT_AUTO, waves_per_block=0, probe_width=0, plain=False,
                 steps_per_launch=0, use_graph=False, persistent=0):
        self.cfgs = list(cfgs)
        arr = (WalkCfg * len(self.cfgs))(*self.cfgs)
        self._arr = arr
        opts = PlanOpts(variant, waves_per_block, probe_width, int(plain), steps_per_launch,
                        int(use_graph), persistent)
        h = ctypes.c_void_p()
        _check(lib().labs_walk_plan_create(len(self.cfgs), arr, ctypes.byref(opts), ctypes.byref(h)),
               "labs_walk_plan_create")
        self._h = h
        self.trace_records = sum(c.steps for c in self.cfgs if c.flags & TRACE)
        self.score_entries = sum(c.steps * ((c.L + 1) // 2) for c in self.cfgs if c.flags & TRACE_SCORES)

    def opts(self):
        o = PlanOpts()
        _check(lib().labs_walk_plan_get_opts(self._h, ctypes.byref(o)), "labs_walk_plan_get_opts")
        return {f: getattr(o, f) for f, _ in PlanOpts._fields_}

    def run(self, stream=None):
        s = _stream() if stream is None else ctypes.c_void_p(stream)
        _check(lib().labs_walk_plan_run(self._h, s), "labs_walk_plan_run")

    def results(self):
        n_w = len(self.cfgs)
        res = (WalkResult * n_w)()
        tbuf = ctypes.create_string_buffer(8 * self.trace_records) if self.trace_records else None
        sbuf = ctypes.create_string_buffer(4 * self.score_entries) if self.score_entries else None
        _check(lib().labs_walk_plan_results(self._h, res, tbuf, sbuf), "labs_walk_plan_results")
        out = [_result_dict(res[i], (self.cfgs[i].L + 1) // 2) for i in range(n_w)]
        traces, scores = _split_traces(self.cfgs, tbuf.raw if tbuf else b"", sbuf.raw if sbuf else b"")
        for i in range(n_w):
            if traces[i] is not None:
                out[i]["trace"] = traces[i]
            if scores[i] is not None:
                out[i]["scores"] = scores[i]
        return out

    def last_timing(self):
        ms = ctypes.c_double()
        nl = ctypes.c_int32()
        _check(lib().labs_walk_plan_last_timing(self._h, ctypes.byref(ms), ctypes.byref(nl)),
               "labs_walk_plan_last_timing")
        return ms.value, nl.value

    def close(self):
        if self._h:
            lib().labs_walk_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def walk_batch(cfgs, stream=None):
    """labs_walk_batch: run walks to completion; returns result dicts (with traces if asked)."""
    cfgs = list(cfgs)
    arr = (WalkCfg * len(cfgs))(*cfgs)
    res = (WalkResult * len(cfgs))()
    tr = sum(c.steps for c in cfgs if c.flags & TRACE)
    sc = sum(c.steps * ((c.L + 1) // 2) for c in cfgs if c.flags & TRACE_SCORES)
    tbuf = ctypes.create_string_buffer(8 * tr) if tr else None
    sbuf = ctypes.create_string_buffer(4 * sc) if sc else None
    s = _stream() if stream is None else ctypes.c_void_p(stream)
    _check(lib().labs_walk_batch(len(cfgs), arr, res, tbuf, sbuf, s), "labs_walk_batch")
    out = [_result_dict(res[i], (cfgs[i].L + 1) // 2) for i in range(len(cfgs))]
    traces, scores = _split_traces(cfgs, tbuf.raw if tbuf else b"", sbuf.raw if sbuf else b"")
    for i in range(len(cfgs)):
        if traces[i] is not None:
            out[i]["trace"] = traces[i]
        if scores[i] is not None:
            out[i]["scores"] = scores[i]
    return out


def pq_walk_batch(cfgs, capacity, nbr_table_log2=0, stream=None):
    """labs_pq_walk_batch: best-first searches with a bounded queue (and optionally the second
    table); returns (result dicts with traces if asked, device milliseconds)."""
    cfgs = list(cfgs)
    arr = (WalkCfg * len(cfgs))(*cfgs)
    res = (WalkResult * len(cfgs))()
    tr = sum(c.steps for c in cfgs if c.flags & TRACE)
    sc = sum(c.steps * ((c.L + 1) // 2) for c in cfgs if c.flags & TRACE_SCORES)
    tbuf = ctypes.create_string_buffer(8 * tr) if tr else None
    sbuf = ctypes.create_string_buffer(4 * sc) if sc else None
    ms = ctypes.c_double()
    s = _stream() if stream is None else ctypes.c_void_p(stream)
    opts = PqOpts(capacity, nbr_table_log2)
    _check(lib().labs_pq_walk_batch(len(cfgs), arr, ctypes.byref(opts), res, tbuf, sbuf, ctypes.byref(ms), s),
           "labs_pq_walk_batch")
    out = [_result_dict(res[i], (cfgs[i].L + 1) // 2) for i in range(len(cfgs))]
    traces, scores = _split_traces(cfgs, tbuf.raw if tbuf else b"", sbuf.raw if sbuf else b"")
    for i in range(len(cfgs)):
        if traces[i] is not None:
            out[i]["trace"] = traces[i]
        if scores[i] is not None:
            out[i]["scores"] = scores[i]
    return out, ms.value


def fi_walk_batch(cfgs, perturb_bits=3, stream=None):
    """labs_fi_walk_batch: first-improvement searches with perturbations of perturb_bits symbols;
    returns (result dicts with traces if asked, device milliseconds).  traps = perturbations."""
    cfgs = list(cfgs)
    arr = (WalkCfg * len(cfgs))(*cfgs)
    res = (WalkResult * len(cfgs))()
    tr = sum(c.steps for c in cfgs if c.flags & TRACE)
    sc = sum(c.steps * ((c.L + 1) // 2) for c in cfgs if c.flags & TRACE_SCORES)
    tbuf = ctypes.create_string_buffer(8 * tr) if tr else None
    sbuf = ctypes.create_string_buffer(4 * sc) if sc else None
    ms = ctypes.c_double()
    s = _stream() if stream is None else ctypes.c_void_p(stream)
    opts = FiOpts(perturb_bits, 0)
    _check(lib().labs_fi_walk_batch(len(cfgs), arr, ctypes.byref(opts), res, tbuf, sbuf, ctypes.byref(ms), s),
           "labs_fi_walk_batch")
    out = [_result_dict(res[i], (cfgs[i].L + 1) // 2) for i in range(len(cfgs))]
    traces, scores = _split_traces(cfgs, tbuf.raw if tbuf else b"", sbuf.raw if sbuf else b"")
    for i in range(len(cfgs)):
        if traces[i] is not None:
            out[i]["trace"] = traces[i]
        if scores[i] is not None:
            out[i]["scores"] = scores[i]
    return out, ms.value


def general_walk_batch(cfgs, stream=None):
    """labs_general_walk_batch: walks over general (not skew-symmetric) sequences; returns
    (result dicts with traces if asked, device milliseconds).  Bits cover all L symbols."""
    cfgs = list(cfgs)
    arr = (WalkCfg * len(cfgs))(*cfgs)
    res = (WalkResult * len(cfgs))()
    tr = sum(c.steps for c in cfgs if c.flags & TRACE)
    sc = sum(c.steps * c.L for c in cfgs if c.flags & TRACE_SCORES)
    tbuf = ctypes.create_string_buffer(8 * tr) if tr else None
    sbuf = ctypes.create_string_buffer(4 * sc) if sc else None
    ms = ctypes.c_double()
    s = _stream() if stream is None else ctypes.c_void_p(stream)
    _check(lib().labs_general_walk_batch(len(cfgs), arr, res, tbuf, sbuf, ctypes.byref(ms), s),
           "labs_general_walk_batch")
    out = [_result_dict(res[i], cfgs[i].L) for i in range(len(cfgs))]
    traces, scores = _split_traces(cfgs, tbuf.raw if tbuf else b"", sbuf.raw if sbuf else b"", general=True)
    for i in range(len(cfgs)):
        if traces[i] is not None:
            out[i]["trace"] = traces[i]
        if scores[i] is not None:
            out[i]["scores"] = scores[i]
    return out, ms.value


def autotune(L, n_walks):
    """labs_autotune: the fastest launch form for n_walks walks of length L (stored in the cache)."""
    o = PlanOpts()
    _check(lib().labs_autotune(L, n_walks, ctypes.byref(o)), "labs_autotune")
    return {f: getattr(o, f) for f, _ in PlanOpts._fields_}


def autotune_batch(cfgs):
    """labs_autotune_batch: the fastest launch form for this batch of walk configurations."""
    cfgs = list(cfgs)
    arr = (WalkCfg * len(cfgs))(*cfgs)
    o = PlanOpts()
    _check(lib().labs_autotune_batch(len(cfgs), arr, ctypes.byref(o)), "labs_autotune_batch")
    return {f: getattr(o, f) for f, _ in PlanOpts._fields_}


# --- serving -----------------------------------------------------------------------------------

def isl_threshold(L, num, den):
    """labs_isl_threshold: the integer form of F >= num/den at length L (Eq. (3))."""
    out = ctypes.c_int64()
    _check(lib().labs_isl_threshold(int(L), int(num), int(den), ctypes.byref(out)), "labs_isl_threshold")
    return out.value


class Server:
    """labs_server_*: continuous-batching search service."""

    def __init__(self, device_mem_bytes=8 << 30, table_log2=16, steps_per_tick=256, max_walks=0):
        opts = ServerOpts(device_mem_bytes, table_log2, steps_per_tick, max_walks, 0)
        h = ctypes.c_void_p()
        _check(lib().labs_server_create(ctypes.byref(opts), ctypes.byref(h)), "labs_server_create")
        self._h = h

    def submit(self, L, n_walks, seed, flip_budget, target_F=None):
        num, den = (0, 1) if target_F is None else target_F
        req = SearchReq(L, n_walks, seed & 0xFFFFFFFFFFFFFFFF, flip_budget, num, den)
        jid = ctypes.c_uint64()
        _check(lib().labs_search_submit(self._h, ctypes.byref(req), ctypes.byref(jid)), "labs_search_submit")
        return jid.value

    @staticmethod
    def _status_dict(st, L=None):
        d = {f: getattr(st, f) for f, _ in SearchStatus._fields_ if f not in ("best_bits", "reserved")}
        d["best_bits_words"] = list(st.best_bits)
        return d

    def poll(self, job_id):
        st = SearchStatus()
        rc = lib().labs_search_poll(self._h, job_id, ctypes.byref(st))
        if rc not in (LABS_OK, LABS_EPENDING):
            _check(rc, "labs_search_poll")
        return rc == LABS_OK, self._status_dict(st)

    def wait(self, job_id, timeout_ms=-1):
        st = SearchStatus()
        rc = lib().labs_search_wait(self._h, job_id, timeout_ms, ctypes.byref(st))
        if rc not in (LABS_OK, LABS_EPENDING):
            _check(rc, "labs_search_wait")
        return rc == LABS_OK, self._status_dict(st)

    def cancel(self, job_id):
        _check(lib().labs_search_cancel(self._h, job_id), "labs_search_cancel")

    def release(self, job_id):
        """Drops a finished job's record (labs_search_release)."""
        _check(lib().labs_search_release(self._h, job_id), "labs_search_release")

    def stats(self):
        ticks, res, peak, flips = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(lib().labs_server_stats(self._h, ctypes.byref(ticks), ctypes.byref(res), ctypes.byref(peak),
                                       ctypes.byref(flips)), "labs_server_stats")
        return {"ticks": ticks.value, "resident_walks": res.value, "peak_walks": peak.value,
                "flip_evals": flips.value}

    def close(self):
        if self._h:
            lib().labs_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def wall():
    return time.perf_counter()
