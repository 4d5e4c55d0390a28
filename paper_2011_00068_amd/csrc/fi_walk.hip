// fi_walk.hip -- first-improvement search with perturbations: the method of Dimitrov et al. as
// Brest & Boskovic describe it (arXiv:2011.00068, Section 2).  From the current skew-symmetric
// sequence the search moves at once to the first flip, in index order, whose ISL is strictly
// lower, and scans again from that sequence; when no flip improves (a local minimum of the
// one-flip neighbourhood) it flips P randomly chosen free symbols and goes on from there.  There
// is no visited table.
//
// One search per 64-lane wavefront with the walkers' scoring of all n flips of the current state
// from the lane-held correlation table: the matrix-core walker at every length (measured 12-17 %
// faster than the bit-sliced one at L = 31..127).  The first improving flip is one wave-wide minimum over keys (j << 24 |
// ISL_j) of the improving flips (ISL < 2^24 up to L = 383).  A perturbation draws its symbols on
// the scalar unit from the counter generator: perturbation k of walk w reads the words
// sm(sm(sm(seed, w), 2^32 + k), i), i = 0, 1, ..., and takes floor((word >> 32) n / 2^32) unless
// already drawn, until P symbols (at most 65536 words); each is applied by the walker's
// incremental commit, and the ISL is then summed from the updated table.
//
// Function evaluations (Section 3's unit) follow the sequential method: j + 1 for a move at flip
// j (flips 0 .. j were evaluated), n + P for a perturbation.  Every occupied state counts for best,
// target and watch (start states included); trace records (j, or -1 for a perturbation; ISL
// after the step); `traps` of the result counts the perturbations.
#include <hip/hip_runtime.h>

#include "mfma_walker.hpp"

namespace liblabs {

namespace {

template <class W>
__device__ __forceinline__ void run_fi(WalkState *__restrict__ wsp, int P, int32_t *__restrict__ trace,
                                       int32_t *__restrict__ scores, typename W::Lds *lds, const uint64_t *zk)
{
    constexpr int G = W::kG;
    int lane = lane_id();
    asm volatile("" : "+v"(lane));
    WalkState &ws = *wsp;

    W w;
    w.lane = lane;
    w.set_length(su(ws.L));
    w.lds = lds;
    w.zk = zk;
    w.init_lanes(lane);
    const int n = w.n;
    const uint64_t seed = su(ws.seed);
    const uint32_t walk_id = su(ws.walk_id);
    const int32_t steps = (int32_t)su(ws.steps);
    const int64_t R = su(ws.restart_period);
    const int64_t target = su(ws.target_isl);
    const int64_t watch = su(ws.watch_isl);
    const int64_t trace_off = su(ws.trace_offset);
    const int64_t score_off = su(ws.score_offset);
    int32_t *trp = trace_off >= 0 ? trace + 2 * trace_off : nullptr;
    int32_t *scp = score_off >= 0 ? scores + score_off : nullptr;
    const int32_t tgt = target < 0 ? -1 : (int32_t)min<int64_t>(target, INT32_MAX);
    const int32_t wch = watch < 0 ? -1 : (int32_t)min<int64_t>(watch, INT32_MAX);
    const int32_t R32 = (int32_t)min<int64_t>(R, INT32_MAX);
    const uint64_t key_w = sm_at(seed, walk_id); // root of the perturbation draws

    int32_t restart_idx = 0, restarts = 0, perturbs = 0;
    int32_t t = 0;
    int64_t flips = 0;
    int32_t best32 = INT32_MAX, best_step = 0, hit = -1, wstep = -1;
    uint32_t best_x[kXWords];
#pragma unroll
    for (int i = 0; i < kXWords; i++)
        best_x[i] = 0u;

    auto start = [&]() {
        start_bits(seed, walk_id, (uint32_t)restart_idx, n, w.x);
        w.rebuild();
    };
    // an occupied state (after step ts): best, hit and watch
    auto note = [&](int32_t ts) {
        if (w.isl < best32) {
            best32 = w.isl;
            best_step = ts;
#pragma unroll
            for (int i = 0; i < kXWords; i++)
                best_x[i] = w.x[i];
        }
        if (tgt >= 0 && hit < 0 && w.isl <= tgt)
            hit = ts;
        if (wch >= 0 && wstep < 0 && w.isl <= wch)
            wstep = ts;
    };
    start();
    note(0);

    while (t < steps && !(tgt >= 0 && hit >= 0)) {
        asm volatile("" : "+v"(w.lane));
        w.prepare();
        int32_t isl_j[G];
        w.score(isl_j);
        uint32_t key = 0xFFFFFFFFu;
#pragma unroll
        for (int g = 0; g < G; g++) {
            const int j = w.flip(g);
            if (j < n && isl_j[g] < w.isl)
                key = min(key, ((uint32_t)j << 24) | (uint32_t)isl_j[g]);
            if (scp && j < n)
                scp[j] = isl_j[g];
        }
        if (scp)
            scp += n;
        key = uniform(wave_min_u32(key));
        int32_t move;
        if (key != 0xFFFFFFFFu) {
            const int js = (int)(key >> 24);
            w.commit(js, (int32_t)(key & 0xFFFFFFu));
            flips += js + 1;
            move = js;
        } else {
            // a local minimum: flip P distinct symbols drawn for perturbation `perturbs`
            const uint64_t key_p = sm_at(key_w, (1ull << 32) + (uint64_t)(uint32_t)perturbs);
            uint32_t drawn[kXWords];
#pragma unroll
            for (int i = 0; i < kXWords; i++)
                drawn[i] = 0u;
            int got = 0;
            for (uint32_t i = 0; got < P && i < 65536u; i++) {
                const uint64_t u = sm_at(key_p, (uint64_t)i);
                const int j = (int)uniform((uint32_t)(((u >> 32) * (uint64_t)n) >> 32));
                if (xbit_uniform(drawn, j))
                    continue;
                xflip_uniform(drawn, j);
                w.commit(j, 0);
                got++;
            }
            int32_t sq = 0;
#pragma unroll
            for (int q = 0; q < W::QR; q++)
                sq += w.Cv[q] * w.Cv[q];
            w.isl = wave_sum_i32(sq);
            perturbs++;
            flips += n + got;
            move = -1;
        }
        t++;
        if (trp) {
            if (w.lane == 0) {
                trp[0] = move;
                trp[1] = w.isl;
            }
            trp += 2;
        }
        note(t);
        if (R32 > 0 && (t % R32) == 0 && t < steps && !(tgt >= 0 && hit >= 0)) {
            restarts++;
            restart_idx++;
            start();
            note(t);
        }
    }

    lds_fence();
    if (lane == 0) {
        ws.t = t;
        ws.flips = flips;
        ws.hit_step = hit;
        ws.watch_step = wstep;
        ws.best_isl = best32;
        ws.best_step = best_step;
        ws.h = w.h;
        ws.isl = w.isl;
        ws.restart_idx = restart_idx;
        ws.restarts = restarts;
        ws.traps = perturbs;
#pragma unroll
        for (int i = 0; i < kXWords; i++) {
            ws.x[i] = w.x[i];
            ws.best_x[i] = best_x[i];
        }
        ws.status = kDone;
    }
}

// walker per shape: the matrix cores (the bit-sliced walker remains as the MFMA = false form)
template <int SHAPE, bool MFMA = true> struct FiWalkerOf;
template <int SHAPE> struct FiWalkerOf<SHAPE, false> {
    using W = Walker<ShapeGK<SHAPE>::G, ShapeGK<SHAPE>::KW, false>;
    static constexpr int waves = 8;
};
template <int SHAPE> struct FiWalkerOf<SHAPE, true> {
    static constexpr bool big = SHAPE >= 5;
    using Lds = typename std::conditional<big, WaveLdsMfmaBig, WaveLdsMfma>::type;
    using W = MfmaWalker<SHAPE == 0 ? 2 : MfmaKW<SHAPE>::value, big, Lds>;
    static constexpr int waves = big ? 5 : 8;
};

template <int SHAPE>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(FiWalkerOf<SHAPE>::waves)))
    k_fi_walk(WalkState *__restrict__ states, int32_t count, const int32_t *__restrict__ order, int P,
              int32_t *__restrict__ trace, int32_t *__restrict__ scores)
{
    using W = typename FiWalkerOf<SHAPE>::W;
    __shared__ uint64_t zk[kNMax];
    __shared__ typename W::Lds lds;
    fill_zobrist(zk);
    const int idx = (int)blockIdx.x;
    if (idx >= count)
        return;
    run_fi<W>(&states[order[idx]], P, trace, scores, &lds, zk);
}

} // namespace

hipError_t launch_fi_walk(int shape, WalkState *states, int32_t count, const int32_t *order, int P, int32_t *trace,
                          int32_t *scores, hipStream_t stream)
{
    if (count <= 0)
        return hipSuccess;
    const dim3 grid((unsigned)count), block(64);
    switch (shape) {
    case 0: hipLaunchKernelGGL(k_fi_walk<0>, grid, block, 0, stream, states, count, order, P, trace, scores); break;
    case 1: hipLaunchKernelGGL(k_fi_walk<1>, grid, block, 0, stream, states, count, order, P, trace, scores); break;
    case 2: hipLaunchKernelGGL(k_fi_walk<2>, grid, block, 0, stream, states, count, order, P, trace, scores); break;
    case 3: hipLaunchKernelGGL(k_fi_walk<3>, grid, block, 0, stream, states, count, order, P, trace, scores); break;
    case 4: hipLaunchKernelGGL(k_fi_walk<4>, grid, block, 0, stream, states, count, order, P, trace, scores); break;
    case 5: hipLaunchKernelGGL(k_fi_walk<5>, grid, block, 0, stream, states, count, order, P, trace, scores); break;
    case 6: hipLaunchKernelGGL(k_fi_walk<6>, grid, block, 0, stream, states, count, order, P, trace, scores); break;
    case 7: hipLaunchKernelGGL(k_fi_walk<7>, grid, block, 0, stream, states, count, order, P, trace, scores); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

} // namespace liblabs
