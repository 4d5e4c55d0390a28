"""Pins of the oracle's best-first search with a bounded queue (Algorithm 1 taken literally,
Section 3; the xLastovka second table as an option): with capacity 1 it is the self-avoiding walk
(itself pinned), and for small L it equals an independent Python statement of the same reading
(heap-free list queue, exact visited sets, ISL by numpy from Eq. (1)-(2) and (4))."""
import numpy as np
import pytest

from oracle import oracle as o

KEYS = ("best_isl", "best_step", "steps_done", "flip_evals", "hit_step", "watch_step", "final_isl",
        "restarts", "traps", "best_bits", "final_bits")


def same(a, b):
    for k in KEYS:
        assert a[k] == b[k], (k, a[k], b[k])
    if "trace" in a and "trace" in b:
        assert np.array_equal(a["trace"], b["trace"])
    if "scores" in a and "scores" in b:
        assert np.array_equal(a["scores"], b["scores"])


@pytest.mark.parametrize("L", [3, 5, 7, 9, 13, 31, 61, 101, 201, 255])
def test_capacity_one_is_the_walk(L):
    for rp, tl, tgt in ((0, 10, -1), (37, 8, -1), (0, 16, L * L // 11), (50, 3, -1)):
        kw = dict(steps=250, table_log2=tl, restart_period=rp, target_isl=tgt, watch_isl=L * L // 9,
                  trace=True, score_trace=True)
        same(o.walk(L, 11, 2, **kw), o.walk(L, 11, 2, pq_capacity=1, **kw))


def _isl_np(L, x):
    n = (L + 1) // 2
    c = n - 1
    s = np.empty(L, dtype=np.int64)
    for j in range(n):
        s[j] = -1 if (x >> j) & 1 else 1
    for i in range(1, c + 1):
        s[c + i] = (-1) ** i * s[c - i]
    return int(sum(int(np.dot(s[: L - k], s[k:])) ** 2 for k in range(1, L)))


class _Bounded:
    """The second table as a bounded direct-mapped table: slot = top `log2` bits of the Zobrist
    hash, stored word = hash | 1, a record overwrites."""

    def __init__(self, n, log2):
        self.z = [o.zobrist(j) for j in range(n)]
        self.log2 = log2
        self.T = {}

    def h(self, x):
        v = 0
        for j, zj in enumerate(self.z):
            if (x >> j) & 1:
                v ^= zj
        return v

    def __contains__(self, x):
        hx = self.h(x)
        return self.T.get(hx >> (64 - self.log2)) == (hx | 1)

    def add(self, x):
        hx = self.h(x)
        self.T[hx >> (64 - self.log2)] = hx | 1


def _python_best_first(L, seed, walk_id, steps, Q, nbr, nbr_log2=None):
    """The reading of Algorithm 1 stated independently: exact visited set, list queue, and the
    second table exact (nbr_log2 None) or bounded."""
    n = (L + 1) // 2
    restart = 0

    def new_n2():
        return set() if nbr_log2 is None else _Bounded(n, nbr_log2)


    def start():
        return o.start_bits(L, seed, walk_id, restart)

    x = start()
    isl = _isl_np(L, x)
    HT, N2, queue = {x}, new_n2(), []
    best, best_step, best_x = isl, 0, x
    flips = traps = 0
    trace = []
    for t in range(steps):
        seen = [nbr and (x ^ (1 << j)) in N2 for j in range(n)]
        for j in range(n):
            xn = x ^ (1 << j)
            if seen[j]:
                continue
            flips += 1
            if xn in HT:
                continue
            if nbr:
                N2.add(xn)
            v = _isl_np(L, xn)
            e = (v, t, j, xn)
            if len(queue) < Q:
                queue.append(e)
            else:
                w = max(queue)
                if e < w:
                    queue[queue.index(w)] = e
            if v < best:
                best, best_step, best_x = v, t + 1, xn
        f = None
        while queue:
            m = min(queue)
            queue.remove(m)
            if m[3] not in HT:
                f = m
                break
        if f is None:
            traps += 1
            restart += 1
            x = start()
            isl = _isl_np(L, x)
            HT, N2, queue = {x}, new_n2(), []
            trace.append((-1, isl))
            if isl < best:  # a restart state counts like the initial state
                best, best_step, best_x = isl, t + 1, x
            continue
        x, isl = f[3], f[0]
        HT.add(x)
        trace.append((f[2] if f[1] == t else -2, isl))
    return {"best_isl": best, "best_step": best_step, "best_bits": best_x, "final_bits": x, "final_isl": isl,
            "flip_evals": flips, "traps": traps, "trace": np.array(trace, dtype=np.int32).reshape(-1, 2)}


@pytest.mark.parametrize("L,Q,nbr", [(15, 2, False), (15, 5, True), (21, 3, False), (21, 64, False),
                                     (21, 8, True), (27, 16, True), (7, 4, False), (9, 2, True)])
def test_matches_independent_statement(L, Q, nbr):
    n = (L + 1) // 2
    steps = 120
    want = _python_best_first(L, 5, 1, steps, Q, nbr)
    got = o.walk(L, 5, 1, steps=steps, table_log2=n + 1, pq_capacity=Q, nbr_table_log2=(n + 1) if nbr else 0,
                 trace=True)
    for k in ("best_isl", "best_step", "best_bits", "final_bits", "final_isl", "flip_evals", "traps"):
        assert got[k] == want[k], (k, got[k], want[k])
    assert np.array_equal(got["trace"], want["trace"])


@pytest.mark.parametrize("L,Q,nlog2", [(21, 8, 3), (25, 4, 5), (31, 16, 6)])
def test_bounded_second_table_matches_independent_statement(L, Q, nlog2):
    # a second table far smaller than the neighbourhood: slot collisions between neighbours of
    # one state are frequent, so the look-up-before-recording and last-index-wins rules matter
    steps = 150
    want = _python_best_first(L, 9, 2, steps, Q, True, nbr_log2=nlog2)
    got = o.walk(L, 9, 2, steps=steps, table_log2=(L + 3) // 2, pq_capacity=Q, nbr_table_log2=nlog2, trace=True)
    for k in ("best_isl", "best_step", "best_bits", "final_bits", "final_isl", "flip_evals", "traps"):
        assert got[k] == want[k], (k, got[k], want[k])
    assert np.array_equal(got["trace"], want["trace"])


def test_properties_long_lengths():
    for L, Q, nbr in ((201, 64, 0), (255, 16, 14), (303, 4, 0)):
        n = (L + 1) // 2
        r = o.walk(L, 3, 0, steps=400, table_log2=14, pq_capacity=Q, nbr_table_log2=nbr, trace=True)
        assert r["steps_done"] == 400
        assert r["flip_evals"] <= 400 * n
        assert o.isl(o.skew_expand(L, r["best_bits"])) == r["best_isl"]
        assert o.isl(o.skew_expand(L, r["final_bits"])) == r["final_isl"]
        assert r["best_isl"] <= int(r["trace"][:, 1].min())
        if Q > 1:
            assert (r["trace"][:, 0] == -2).any()  # the queue serves older entries too


def test_bad_arguments():
    for kw in (dict(pq_capacity=1, nbr_table_log2=31), dict(pq_capacity=1, nbr_table_log2=-1)):
        with pytest.raises(RuntimeError):
            o.walk(31, 1, 0, steps=10, **kw)
