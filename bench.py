"""Benchmark of the skew-symmetric LABS walk on one MI355X.

A step is one whole job of the L = 255 headline workload: 16,384 independent walks from seeded
uniform +-1 starts, random restarts every 2^20 steps, a visited table of 2^16 entries per walk,
run until a walk reaches F >= 8.5 or the job has made 10^10 flip evaluations (4,768 steps per
walk).  The walk state is resident in HBM before the timed region (a plan); each timed step resets
every walk to its start state and runs the job to completion on the GPU.

Printed: one JSON line with the throughput in flip evaluations per second (the paper's speed
unit, Section 3: one evaluated flip = one function evaluation), the roofline of the walk kernel,
the oracle timed on the host cores on a bounded sample of the same workload, the plain
one-walk-per-launch form on a sample, and time-to-target statistics (F >= 8, and the lower,
labelled F >= 5 that most walks reach within the budget); then (unless --no-extras) the L = 101
batch at low occupancy, an uneven batch of all 52 lengths, the serving workload and the saturated
server, the exhaustive skew minimum at L = 61 and 69, the best-first search with a bounded queue
(with and without the second table), the first-improvement search with perturbations, and the
walk over general sequences at L = 192.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

L = 255
N = (L + 1) // 2
WALKS = 16384
FLIP_BUDGET = 10 ** 10
STEPS = FLIP_BUDGET // (WALKS * N)  # 4768 steps per walk
SEED = 2011000068
TABLE_LOG2 = 16
RESTART = 1 << 20
# stop at F >= 8.5; record the first step at F >= 5 (the lower, labelled target most walks reach
# within the budget).  Their integer ISL bounds (Eq. (3)) come from labs_isl_threshold in main().
TARGET_F = (17, 2)
WATCH_F = (5, 1)
TARGET_ISL = WATCH_ISL = None
F8_ISL = None  # F >= 8: reached by a walk exactly when its best ISL is at most this bound
# algorithmic int32 operations per flip evaluation: for each of the (L-1)/2 even shifts,
# u = s_{j+k} + s_{j-k}, t = C_k + sigma_j u, acc += t^2  (one add, two multiply-adds)
ALG_OPS_PER_FLIP = 3 * (L - 1) // 2
# MI355X: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz int32 VALU lane-operations per second
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# MI355X published dense int8 matrix-core peak (no sparsity), operations per second
INT8_MFMA_PEAK_TOPS = 5000.0
KERNEL_SOURCES = ["paper_2011_00068_amd/csrc/walk_impl.hpp", "paper_2011_00068_amd/csrc/device_common.hpp",
                  "paper_2011_00068_amd/csrc/mfma_walker.hpp", "paper_2011_00068_amd/csrc/walk_inst_mfma.hip"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "walk_L255_16384_traffic.json")


def source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def set_thresholds(labs):
    """The integer ISL bounds of the stop, watch and F >= 8 levels (labs_isl_threshold, Eq. (3))."""
    global TARGET_ISL, WATCH_ISL, F8_ISL
    TARGET_ISL = labs.isl_threshold(L, *TARGET_F)  # 3825
    WATCH_ISL = labs.isl_threshold(L, *WATCH_F)  # 6502
    F8_ISL = labs.isl_threshold(L, 8, 1)  # 4064


def cfgs(labs, walks, steps):
    if TARGET_ISL is None:
        set_thresholds(labs)
    return [labs.make_cfg(L, SEED, w, steps=steps, table_log2=TABLE_LOG2, restart_period=RESTART,
                          target_isl=TARGET_ISL, watch_isl=WATCH_ISL) for w in range(walks)]


def time_to_target(results, ms_per_job, steps):
    """Time to the first state at the watched F >= 5 per walk: its step times the job's time per
    step (all walks advance together).  Censored walks (no hit within the budget) count as never,
    so a percentile is reported only when at least that share of the walks hit."""
    import numpy as np

    hit = np.array([r["watch_step"] for r in results], dtype=np.int64)
    ok = hit >= 0
    frac = float(ok.mean())
    per_step_ms = ms_per_job / steps
    out = {"threshold_F": WATCH_F[0] / WATCH_F[1], "isl_threshold": WATCH_ISL, "hit_fraction": frac,
           "censored": frac < 0.5, "p50_s": None, "p99_s": None}
    if ok.any():
        times = np.sort(np.where(ok, hit * per_step_ms / 1000.0, np.inf))
        p50 = times[int(0.50 * (len(times) - 1))]
        p99 = times[int(0.99 * (len(times) - 1))]
        out["p50_s"] = None if not np.isfinite(p50) else float(p50)
        out["p99_s"] = None if not np.isfinite(p99) else float(p99)
    return out


def time_to_f8(results):
    """F >= 8 (ISL <= floor(L^2 / 16) = 4064): a walk reached it exactly when its best ISL is at
    most that bound, so the hit fraction is exact without a watch level; its time is not recorded
    (the watch level is F >= 5), so the percentiles are reported only as censored."""
    import numpy as np

    best = np.array([r["best_isl"] for r in results], dtype=np.int64)
    frac = float((best <= F8_ISL).mean())
    return {"threshold_F": 8.0, "isl_threshold": F8_ISL, "hit_fraction": frac, "censored": True,
            "p50_s": None, "p99_s": None, "best_isl": int(best.min()), "best_F": L * L / (2.0 * best.min())}


def cpu_baseline(budget_s=10.0):
    """The oracle as it stands, on a bounded sample of the workload: whole walks (all 4,768 steps
    each) over a thread pool (ctypes releases the GIL), one round of one walk per thread after
    another until about budget_s seconds have passed."""
    from concurrent.futures import ThreadPoolExecutor

    from oracle import oracle as o

    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    o.lib()

    def one(w):
        return o.walk(L, SEED, w, steps=STEPS, table_log2=TABLE_LOG2, restart_period=RESTART,
                      target_isl=TARGET_ISL, watch_isl=WATCH_ISL)

    res = []
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        while time.perf_counter() - t0 < budget_s and len(res) < WALKS:
            res += list(ex.map(one, range(len(res), min(WALKS, len(res) + threads))))
    dt = time.perf_counter() - t0
    flips = sum(r["flip_evals"] for r in res)
    # the same on one thread, on the walks that follow (about a quarter of the budget)
    one_flips, one_walks = 0, 0
    t1 = time.perf_counter()
    while time.perf_counter() - t1 < budget_s / 4 and len(res) + one_walks < WALKS:
        one_flips += one(len(res) + one_walks)["flip_evals"]
        one_walks += 1
    dt1 = time.perf_counter() - t1
    return {"value": flips / dt, "unit": "flip-evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{len(res)} of the {WALKS} walks, all {STEPS} steps each, L={L}, "
                      f"{threads} threads; {dt:.1f} s wall",
            "one_thread": {"value": one_flips / dt1 if dt1 > 0 else None, "walks": one_walks},
            "host": host_cpu()}, res


def host_cpu():
    """The host CPU the oracle ran on: model name and the logical CPUs this process may use."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "logical_cpus_available": len(os.sched_getaffinity(0))}


def plain_form(labs, walks=32):
    """The plain one-walk-per-launch form: the same walks, one kernel launch per walk, serialised
    on one stream (a sample of the job's walks)."""
    import torch

    plan = labs.WalkPlan(cfgs(labs, walks, STEPS), plain=True)
    plan.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res = plan.results()
    plan.close()
    flips = sum(r["flip_evals"] for r in res)
    per_walk_ms = dt * 1000.0 / walks
    return {"value": flips / dt, "unit": "flip-evals/s", "walks": walks,
            "ms_per_walk": per_walk_ms,
            "time_to_F5": time_to_target(res, per_walk_ms, STEPS), "time_to_F8": time_to_f8(res)}, res


def serving(labs, rate=20.0, n_requests=100, seed=SEED, target_F=(8, 1), steps_per_tick=256):
    """The serving workload: Poisson arrivals (seeded), each request one odd L uniform in
    [201, 303] with 256 walks, 10^8 flip evaluations and stop threshold target_F (F >= 8), admitted
    by device memory for walk state.  Returns latency percentiles (submission to completion: the
    budget spent, or the tick in which a walk reached the threshold) and aggregate throughput;
    with a reachable threshold the latency of the requests that reached it is time to target."""
    import numpy as np

    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    lengths = rng.choice(np.arange(201, 304, 2), size=n_requests)
    srv = labs.Server(device_mem_bytes=8 << 30, table_log2=TABLE_LOG2, steps_per_tick=steps_per_tick)
    t0 = time.perf_counter()
    jobs = []
    next_t = 0.0
    for i in range(n_requests):
        next_t += gaps[i]
        delay = next_t - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        jobs.append((int(lengths[i]), srv.submit(int(lengths[i]), 256, seed + i, 10 ** 8, target_F=target_F)))
    lat, hit_lat, flips, hits = [], [], 0, 0
    for L, j in jobs:
        done, st = srv.wait(j, timeout_ms=600000)
        lat.append(st["t_done"] - st["t_submit"])
        flips += st["flip_evals"]
        hits += st["hit_step"] >= 0
        if st["hit_step"] >= 0:
            hit_lat.append(st["t_done"] - st["t_submit"])
    wall = time.perf_counter() - t0
    stats = srv.stats()
    srv.close()
    lat = np.sort(np.array(lat))
    out = {"requests": n_requests, "rate_per_s": rate, "walks_per_request": 256,
           "flip_budget_per_request": 10 ** 8, "target_F": target_F[0] / target_F[1],
           "p50_latency_s": float(lat[int(0.50 * (len(lat) - 1))]),
           "p99_latency_s": float(lat[int(0.99 * (len(lat) - 1))]),
           "aggregate_flip_evals_per_s": flips / wall, "hit_fraction": hits / n_requests,
           "wall_s": wall, "ticks": stats["ticks"], "peak_resident_walks": stats["peak_walks"]}
    if hit_lat:
        # time to target (submission to the tick that saw the first walk reach it), p99 only when
        # at least 99 % of the requests reached it
        h = np.sort(np.array(hit_lat))
        out["time_to_target_p50_s"] = float(h[int(0.50 * (len(h) - 1))]) if hits * 2 >= n_requests else None
        out["time_to_target_p99_s"] = float(h[int(0.99 * (len(h) - 1))]) if hits * 100 >= 99 * n_requests else None
    return out


def serving_f5(labs):
    """The serving workload with the labelled lower threshold F >= 5, which requests reach: time
    to target per request."""
    return serving(labs, target_F=(5, 1))


def serving_capacity(labs, n_requests=96, seed=SEED + 1):
    """The server saturated: every request (one odd L uniform in [201, 303], 256 walks, 10^8 flip
    evaluations, no target) submitted at once, more than the 8 GiB slot pool holds; the aggregate
    flip-evaluation rate from the first submission to the last completion."""
    import numpy as np

    rng = np.random.default_rng(seed)
    lengths = rng.choice(np.arange(201, 304, 2), size=n_requests)
    srv = labs.Server(device_mem_bytes=8 << 30, table_log2=TABLE_LOG2, steps_per_tick=256)
    t0 = time.perf_counter()
    jobs = [srv.submit(int(Lr), 256, seed + i, 10 ** 8) for i, Lr in enumerate(lengths)]
    flips = 0
    for j in jobs:
        done, st = srv.wait(j, timeout_ms=600000)
        flips += st["flip_evals"]
        srv.release(j)
    wall = time.perf_counter() - t0
    stats = srv.stats()
    srv.close()
    return {"requests": n_requests, "walks_per_request": 256, "flip_budget_per_request": 10 ** 8,
            "wall_s": wall, "aggregate_flip_evals_per_s": flips / wall, "ticks": stats["ticks"],
            "peak_resident_walks": stats["peak_walks"]}


def latency(labs, steps=200000):
    """Where a walk step's time goes when the GPU is not full (run with --only latency): the uneven
    batch (52 lengths x 64 walks, one launch) with visited tables of 2^16 and of 2^8 words (the latter
    always in cache), one walk per length alone (52 waves), and L = 255 batches of 1, 1,024, 3,328
    and 8,192 walks (1 .. 8 waves per SIMD); microseconds per step of the launch."""
    import torch

    def timed(cfg):
        plan = labs.WalkPlan(cfg)
        plan.run()
        torch.cuda.synchronize()
        plan.run()
        ms, _ = plan.last_timing()
        plan.close()
        return ms

    out = {"steps": steps, "uneven_us_per_step": {}, "one_walk_per_length_us_per_step": {}, "l255_us_per_step": {}}
    lengths = range(201, 304, 2)
    for tl in (16, 8):
        cfg = [labs.make_cfg(Lx, SEED, w, steps=steps, table_log2=tl) for Lx in lengths for w in range(64)]
        out["uneven_us_per_step"][f"table_2^{tl}"] = timed(cfg) * 1000.0 / steps
        cfg = [labs.make_cfg(Lx, SEED, 0, steps=steps, table_log2=tl) for Lx in lengths]
        out["one_walk_per_length_us_per_step"][f"table_2^{tl}"] = timed(cfg) * 1000.0 / steps
    for nw in (1, 1024, 3328, 8192):
        cfg = [labs.make_cfg(L, SEED, w, steps=steps // 4, table_log2=TABLE_LOG2) for w in range(nw)]
        out["l255_us_per_step"][f"{nw}_walks"] = timed(cfg) * 1000.0 / (steps // 4)
    return out


def shapes(labs, walks=16384, steps=2000):
    """The one-tile and the two-tile matrix-core walker side by side (run with --only shapes, or
    under rocprofv3 --pmc for their instructions per step): full-GPU batches of 16,384 walks x
    2,000 steps at L = 255 (c = 127, one tile) and L = 303 (c = 151, two tiles); microseconds per
    step of the launch (second run of each plan)."""
    import torch

    out = {"walks": walks, "steps": steps}
    for Lx in (255, 303):
        plan = labs.WalkPlan([labs.make_cfg(Lx, SEED, w, steps=steps, table_log2=TABLE_LOG2) for w in range(walks)])
        plan.run()
        torch.cuda.synchronize()
        plan.run()
        ms, _ = plan.last_timing()
        plan.close()
        out[f"L{Lx}_us_per_step"] = ms * 1000.0 / steps
    return out


def uneven_batch(labs):
    """Every odd L in [201, 303] x 64 walks x 10^6 steps in one launch of mixed shapes,
    replayed from a captured hipGraph."""
    import torch

    cfg = [labs.make_cfg(L, SEED, w, steps=10 ** 6, table_log2=TABLE_LOG2) for L in range(201, 304, 2)
           for w in range(64)]
    plan = labs.WalkPlan(cfg, use_graph=True)
    variant = plan.opts()["variant"]
    plan.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.run()
    ms, launches = plan.last_timing()
    wall = time.perf_counter() - t0
    res = plan.results()
    plan.close()
    flips = sum(r["flip_evals"] for r in res)
    alg = sum(r["flip_evals"] * 3 * (c.L - 1) // 2 for r, c in zip(res, cfg)) / (ms / 1000.0) / 1e12
    return {"walks": len(cfg), "steps_per_walk": 10 ** 6, "launches": launches, "hipgraph": True, "kernel_ms": ms,
            "flip_evals_per_s": flips / wall,
            # the launch lasts as long as its slowest walk's 10^6 dependent steps
            "us_per_step": ms * 1000.0 / 10 ** 6,
            "roofline": matrix_or_alu_roofline(variant, alg)}


def matrix_or_alu_roofline(variant, alg_tops):
    """The walk kernel's roofline for alg_tops algorithmic TOP/s: the dense int8 matrix-core peak
    when the flip scoring runs on the matrix cores (variant 3), else the int32 VALU peak."""
    if variant == 3:
        return {"bound": "mfma", "achieved": alg_tops, "peak": INT8_MFMA_PEAK_TOPS, "unit": "TOP/s",
                "frac": alg_tops / INT8_MFMA_PEAK_TOPS}
    return {"bound": "alu", "achieved": alg_tops, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
            "frac": alg_tops / VALU_PEAK_TOPS}


def low_occupancy(labs, Lx=101, walks=1024, steps=10 ** 5):
    """The L = 101 batch: 1,024 walks (one wavefront per SIMD) x 10^5 steps, visited tables of
    2^16 words, one launch; throughput at low occupancy, where a step's dependent latency and not
    the issue rate bounds the kernel."""
    import torch

    cfg = [labs.make_cfg(Lx, SEED, w, steps=steps, table_log2=TABLE_LOG2) for w in range(walks)]
    plan = labs.WalkPlan(cfg)
    opts = plan.opts()
    plan.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.run()
    ms, launches = plan.last_timing()
    wall = time.perf_counter() - t0
    res = plan.results()
    plan.close()
    flips = sum(r["flip_evals"] for r in res)
    alg = flips * 3 * (Lx - 1) // 2 / (ms / 1000.0) / 1e12
    best = min(r["best_isl"] for r in res)
    return {"L": Lx, "walks": walks, "steps_per_walk": steps, "launches": launches, "kernel_ms": ms,
            "flip_evals": flips, "flip_evals_per_s": flips / wall, "us_per_step": ms * 1000.0 / steps,
            "kernel": "k_walk_mfma" if opts["variant"] == 3 else "k_walk", "plan_opts": opts,
            "roofline": dict(matrix_or_alu_roofline(opts["variant"], alg), alg_ops_per_flip=3 * (Lx - 1) // 2),
            "best_isl": best, "best_F": Lx * Lx / (2.0 * best)}


def best_first(labs, walks=WALKS, steps=1000):
    """Algorithm 1 taken literally: best-first search with a queue of 64 entries per search
    (impxLast), and with the second table of evaluated neighbours as well (xLastovka), at the
    headline length; flip evaluations per second, and the merit factors reached."""
    import numpy as np

    cfg = [labs.make_cfg(L, SEED, w, steps=steps, table_log2=TABLE_LOG2) for w in range(walks)]
    labs.pq_walk_batch(cfg[:256], 64)  # warm the launch path
    out = {"L": L, "searches": walks, "iterations": steps, "capacity": 64}
    for name, nlog2 in (("impxLast", 0), ("xLastovka", TABLE_LOG2)):
        res, ms = labs.pq_walk_batch(cfg, 64, nlog2)
        evals = sum(r["flip_evals"] for r in res)
        best = np.array([r["best_isl"] for r in res], dtype=np.float64)
        # the scoring of every iteration runs on the matrix-core walker
        alg = steps * walks * N * ALG_OPS_PER_FLIP / (ms / 1000.0) / 1e12
        out[name] = {"nbr_table_log2": nlog2, "kernel_ms": ms, "flip_evals": evals,
                     "flip_evals_per_s": evals / (ms / 1000.0),
                     "roofline": dict(matrix_or_alu_roofline(3, alg), alg_ops_per_flip=ALG_OPS_PER_FLIP,
                                      note="algorithmic operations of the n flips scored per iteration"),
                     "mean_best_F": float(np.mean(L * L / (2.0 * best))), "max_best_F": float(L * L / (2.0 * best.min()))}
    return out


def first_improvement(labs, walks=WALKS, steps=4768, P=3):
    """The first-improvement search with perturbations of 3 symbols (Section 2's description of
    Dimitrov et al.'s method) at the headline length: the evaluations the sequential method counts
    (j + 1 per move, n + P per perturbation), the flips the kernel scores (n per step, all of them in
    parallel), and the merit factors reached within the headline's steps per walk."""
    import numpy as np

    cfg = [labs.make_cfg(L, SEED, w, steps=steps) for w in range(walks)]
    labs.fi_walk_batch(cfg[:256], P)  # warm the launch path
    res, ms = labs.fi_walk_batch(cfg, P)
    evals = sum(r["flip_evals"] for r in res)
    scored = sum(r["steps_done"] for r in res) * N
    best = np.array([r["best_isl"] for r in res], dtype=np.float64)
    alg = scored * ALG_OPS_PER_FLIP / (ms / 1000.0) / 1e12
    return {"L": L, "searches": walks, "steps": steps, "perturb_bits": P, "kernel_ms": ms,
            "flip_evals": evals, "flip_evals_per_s": evals / (ms / 1000.0),
            "scored_flips_per_s": scored / (ms / 1000.0),
            "perturbations_per_step": sum(r["traps"] for r in res) / sum(r["steps_done"] for r in res),
            "roofline": dict(matrix_or_alu_roofline(3, alg), alg_ops_per_flip=ALG_OPS_PER_FLIP,
                             note="algorithmic operations of the scored flips"),
            "mean_best_F": float(np.mean(L * L / (2.0 * best))), "max_best_F": float(L * L / (2.0 * best.min()))}


def general_walk(labs, Lg=192, walks=WALKS, steps=2000):
    """The walk over general sequences (all L symbols free, every shift counts) at the longest
    supported length: flip evaluations per second and the roofline with 3 (L-1) algorithmic
    operations per evaluation (one add and two multiply-adds per shift) against the int8
    matrix-core peak (its correlation sums run as int8 tiles)."""
    cfg = [labs.make_cfg(Lg, SEED, w, steps=steps, table_log2=TABLE_LOG2) for w in range(walks)]
    labs.general_walk_batch(cfg[:256])  # warm the launch path
    res, ms = labs.general_walk_batch(cfg)
    evals = sum(r["flip_evals"] for r in res)
    alg = evals * 3 * (Lg - 1) / (ms / 1000.0) / 1e12
    best = min(r["best_isl"] for r in res)
    return {"L": Lg, "walks": walks, "steps_per_walk": steps, "kernel_ms": ms, "flip_evals": evals,
            "flip_evals_per_s": evals / (ms / 1000.0),
            "roofline": dict(matrix_or_alu_roofline(3, alg), alg_ops_per_flip=3 * (Lg - 1)),
            "best_isl": best, "best_F": Lg * Lg / (2.0 * best)}


def enum_alg_ops_per_group(Lx):
    """Word operations to score one sequence with the bit-packed form of Eq. (1)-(2): for each even
    lag k, per 32-bit word of the L - k overlapping positions a funnel shift, a masked xor and a
    popcount-accumulate, then one shift-or and one multiply-add for C_k^2."""
    return sum(3 * ((Lx - k + 31) // 32) + 2 for k in range(2, Lx, 2))


def enumeration(labs, lengths=(61, 69)):
    """The whole skew space of each length, minimum ISL by exhaustive search on the GPU (one
    sequence scored per symmetry group of four).  The roofline counts the word operations of the
    (sequence, lag) pairs the branch and bound actually evaluated (the kernel reports them); the
    exhaustive count is given beside it."""
    out = []
    for Lx in lengths:
        labs.enum_skew_min(Lx, 0, 1 << 12)  # warm the launch path
        t0 = time.perf_counter()
        r = labs.enum_skew_min(Lx)
        wall = time.perf_counter() - t0
        groups = r["states"] // 4
        alg = r["word_ops"] / (r["kernel_ms"] / 1000.0) / 1e12
        exhaustive = groups * enum_alg_ops_per_group(Lx)
        out.append({"L": Lx, "sequences": r["states"], "min_isl": r["min_isl"],
                    "F": Lx * Lx / (2.0 * r["min_isl"]), "optimal_sequences": r["count"],
                    "first_x": hex(r["first_x"]), "kernel_ms": r["kernel_ms"], "wall_s": wall,
                    "sequences_per_s": r["states"] / wall,
                    "roofline": {"bound": "alu", "achieved": alg, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                                 "frac": alg / VALU_PEAK_TOPS, "word_ops_evaluated": r["word_ops"],
                                 "word_ops_exhaustive": exhaustive,
                                 "evaluated_share": r["word_ops"] / exhaustive,
                                 "alg_ops_per_group": enum_alg_ops_per_group(Lx)}})
    return out


def counter_summary():
    """The committed rocprofv3 counter summary of the walk kernel (HBM bytes per launch scaled by
    the copy calibration, VALU issue occupancy), if it was taken on the current kernel source;
    else None."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != source_hash():
        return None
    return t


def device_summary(labs, cnt):
    """The device and its clocks: the maximum shader clock the runtime reports, and the effective
    one of the walk kernel from the committed counter summary (GPU busy cycles per XCD,
    rocprofv3 GRBM_GUI_ACTIVE / 8, over the launch's rocprofv3 duration), which the peaks are
    quoted against at the nominal 2.4 GHz."""
    out = {"name": None, "compute_units": None, "max_sclk_mhz": None, "sclk_measured_mhz": None}
    try:
        d = labs.device_info()
        out.update(name=d["name"], compute_units=d["compute_units"], max_sclk_mhz=d["clock_khz"] / 1000.0)
    except labs.LabsError as e:
        print(f"device info failed: {e}", file=sys.stderr)
    if cnt and cnt.get("gpu_cycles_per_xcd") and cnt.get("avg_launch_ns_rocprof"):
        out["sclk_measured_mhz"] = cnt["gpu_cycles_per_xcd"] / cnt["avg_launch_ns_rocprof"] * 1000.0
    return out


def lds_summary(labs, cnt):
    """The walk kernel against the LDS roof: the share of cycles in which the LDS pipe of a compute
    unit is busy (rocprofv3 SQ_LDS_IDX_ACTIVE over GRBM_GUI_ACTIVE cycles, of which bank-conflict
    cycles), from the committed counter summary, next to the device's LDS read bandwidth measured
    now (8- and 16-byte reads per lane; the walk kernels issue 1- to 8-byte accesses, which move at
    most 128 bytes per cycle per compute unit)."""
    out = {"active_frac": None, "bank_conflict_frac": None, "active_cycles_per_step": None,
           "peak_read_8B_TBps": None, "peak_read_16B_TBps": None}
    if cnt and "lds_active_frac" in cnt:
        out["active_frac"] = cnt["lds_active_frac"]
        out["bank_conflict_frac"] = cnt["lds_bank_conflict_frac"]
        out["active_cycles_per_step"] = cnt["lds_active_cycles_per_step"]
    try:
        out["peak_read_8B_TBps"] = labs.probe_lds_read(8)["bytes_per_s"] / 1e12
        out["peak_read_16B_TBps"] = labs.probe_lds_read(16)["bytes_per_s"] / 1e12
    except labs.LabsError as e:
        print(f"LDS probe failed: {e}", file=sys.stderr)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--variant", type=int, default=0,
                    help="walk kernel variant: 0 auto, 1 bit-sliced, 2 direct, 3 matrix cores")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain-form comparison")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the serving, uneven-batch, enumeration, best-first and general-walk measurements")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes (the reference "
                         "kernel that scales the FETCH_SIZE / WRITE_SIZE counters) and exit")
    ap.add_argument("--only", choices=["low_occupancy", "uneven_batch", "serving", "serving_F5", "serving_capacity",
                                       "enumeration",
                                       "best_first", "general_walk", "first_improvement", "latency", "shapes"],
                    help="run only this measurement and print its JSON (for profiling)")
    ap.add_argument("--probe-lds", action="store_true",
                    help="only measure the LDS read bandwidth (4-, 8- and 16-byte reads per lane) and exit")
    args = ap.parse_args()
    if args.probe_lds:
        import paper_2011_00068_amd as labs

        for w in (4, 8, 16):
            r = labs.probe_lds_read(w)
            print(json.dumps({"lds_read_bytes_per_lane": w, "bytes_per_s": r["bytes_per_s"], "ms": r["ms"]}),
                  flush=True)
        return
    if args.calibrate_copy:
        import torch

        src = torch.ones(args.calibrate_copy, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": args.calibrate_copy, "copies": 3}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (the library has no multi-GPU path); got --gpus {args.gpus}",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2011_00068_amd as labs

    torch.cuda.set_device(0)
    set_thresholds(labs)
    if args.only:
        legs = {"low_occupancy": low_occupancy, "uneven_batch": uneven_batch, "serving": serving,
                "serving_F5": serving_f5,
                "serving_capacity": serving_capacity, "first_improvement": first_improvement,
                "latency": latency, "shapes": shapes,
                "enumeration": enumeration, "best_first": best_first, "general_walk": general_walk}
        print(json.dumps({args.only: legs[args.only](labs)}), flush=True)
        return
    plan = labs.WalkPlan(cfgs(labs, WALKS, STEPS), variant=args.variant)
    opts = plan.opts()
    for _ in range(args.warmup):
        plan.run()
    torch.cuda.synchronize()
    kernel_ms = []
    launches = 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.run()
        ms, launches = plan.last_timing()  # waits for this run; device time of its walk launches
        kernel_ms.append(ms)
    torch.cuda.synchronize()
    wall_s = time.perf_counter() - t0
    res = plan.results()
    plan.close()

    flips_per_job = sum(r["flip_evals"] for r in res)
    ms_per_step = wall_s * 1000.0 / args.steps
    value = flips_per_job / (ms_per_step / 1000.0)

    avg_kernel_ms = sum(kernel_ms) / len(kernel_ms)
    per_launch_ms = avg_kernel_ms / max(1, launches)
    alg_ops_per_launch = flips_per_job * ALG_OPS_PER_FLIP / max(1, launches)
    achieved = alg_ops_per_launch / (per_launch_ms / 1000.0) / 1e12
    cnt = counter_summary()
    # The flip scoring's correlation sums run as int8 x int8 -> int32 matrix-core tiles, so the
    # roof of the algorithmic operations (381 per evaluation) is the dense int8 peak.  The kernel
    # is far below it: each walk's product is two small matrix-core operations on a serial chain,
    # and the roof that binds is instruction issue (the VALU, SALU and LDS-pipe shares from the
    # counters).
    roofline = dict(matrix_or_alu_roofline(opts["variant"], achieved),
                    traffic=cnt["hbm_bytes_per_launch"] if cnt else None,
                    kernel="k_walk_mfma" if opts["variant"] == 3 else "k_walk",
                    kernel_ms_per_launch=per_launch_ms,
                    alg_ops_per_flip=ALG_OPS_PER_FLIP,
                    binding={"roof": "VALU issue",
                             # rocprofv3 counters of the same launch: share of the SIMDs' VALU
                             # issue cycles in use (VALU instructions x 4 cycles per wave64
                             # instruction / SIMD cycles), and the same for SALU and the LDS pipe
                             "valu_issue_frac": cnt["valu_issue_busy_frac"] if cnt else None,
                             "salu_issue_frac": cnt.get("salu_issue_busy_frac") if cnt else None,
                             "lds_pipe_frac": cnt.get("lds_active_frac") if cnt else None,
                             "valu_insts_per_step": cnt["valu_insts_per_step"] if cnt else None,
                             "mfma_insts_per_step": cnt.get("mfma_insts_per_step") if cnt else None},
                    lds=lds_summary(labs, cnt))
    if opts["variant"] != 3:
        # the bit-sliced and direct layouts execute another number of operations per evaluation
        # than the algorithmic count, so no fraction of a peak is claimed for them
        roofline["frac"] = None

    line = {
        "metric": "flip-evals/s at L=255 (batched walks, % INT32 VALU peak); p50 time-to-F>=8",
        "value": value,
        "unit": "flip-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int8xint8->int32 MFMA + int32 VALU",
        "data": "synthetic",
        "config": {"workload": "L255_16384walks_1e10flips", "L": L, "walks": WALKS,
                   "steps_per_walk": STEPS, "table_log2": TABLE_LOG2, "restart_period": RESTART,
                   "target_F": 8.5, "watch_F": WATCH_F[0] / WATCH_F[1], "parallelism": "none (1 GPU)",
                   # persistent = 1: one wave per walk, hardware-dispatched (not the pulling grid)
                   "plan_opts": opts},
        "roofline": roofline,
        "device": device_summary(labs, cnt),
        "time_to_F5": time_to_target(res, ms_per_step, STEPS),
        "time_to_F8": time_to_f8(res),
    }
    if not args.no_plain:
        line["plain_form"], _ = plain_form(labs)
    if not args.no_extras:
        line["low_occupancy"] = low_occupancy(labs)
        line["uneven_batch"] = uneven_batch(labs)
        line["serving"] = serving(labs)
        line["serving_F5"] = serving_f5(labs)
        line["serving_capacity"] = serving_capacity(labs)
        line["enumeration"] = enumeration(labs)
        line["best_first"] = best_first(labs)
        line["first_improvement"] = first_improvement(labs)
        line["general_walk"] = general_walk(labs)
    if not args.no_cpu:
        line["cpu_baseline"], _ = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
