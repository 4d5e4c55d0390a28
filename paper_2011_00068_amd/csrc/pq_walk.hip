// pq_walk.hip -- best-first search with a bounded priority queue: Algorithm 1 of Brest &
// Boskovic (arXiv:2011.00068, Section 3) taken literally, optionally with the second table of
// evaluated neighbours that the xLastovka algorithm keeps and impxLast drops (Section 3).
//
// One walk per 64-lane wavefront, as the self-avoiding walk: the scoring of the n flips of the
// current state is the walker's (matrix-core or bit-sliced by shape, below; the flips a lane owns
// follow the walker's mapping: flip(g), owner_lane, owner_slot).  The queue lives in registers,
// one entry per lane, sorted by (ISL, iteration that generated the entry, flip index): lane 0 is
// the front, lane q-1 the last of q entries.  Because every entry offered in an iteration was
// generated after all entries already queued, and the iteration offers its entries in ascending
// (ISL, flip) order, a new entry's place is the number of queued entries with ISL <= its ISL;
// inserting shifts the lanes above by one (DPP wave_shr), removing the front shifts them down
// (wave_shl).  An entry holds the state's free bits and hash so that a queued state that is not
// a neighbour of the current one can be rebuilt from scratch when it reaches the front.
//
// Per iteration: score every flip; look the neighbours up in the second table (all of them,
// against the table as it was before the iteration); record the evaluated, unvisited neighbours
// in the second table (when several map to one slot, the highest flip index is stored, as
// sequential recording in index order leaves it); offer the candidates (ISL below the last entry
// of a full queue) to the queue in ascending (ISL, flip) order, probing the visited table for a
// few of the smallest unprobed candidates at a time, only when the smallest one left is unprobed
// (with the second table every unskipped neighbour is probed, since its recording depends on
// it); take the front entry whose state is not visited; move there (incremental update for a
// neighbour, rebuild from its free bits otherwise).
#include <hip/hip_runtime.h>

#include "mfma_walker.hpp"

namespace liblabs {

namespace {

constexpr int kPqProbe = 4;     // visited-table probes issued together
constexpr int kPqNearFlips = 24; // an older queue entry this close is reached by single flips (cheaper than a rebuild)

__device__ __forceinline__ bool readlane_b(bool v, int l)
{
    return __builtin_amdgcn_readlane((int)v, l) != 0;
}

// the walker's LDS block and the second-table partner list
template <class Base> struct WaveLdsPqT : Base {
    int16_t nxt[kNMax]; // next higher flip whose neighbours share this flip's second-table slot
};

// walker per shape: the one-tile matrix-core walker for shapes 2..4 (L = 129..255), the bit-sliced
// one elsewhere.  The queue's registers next to the walker's set the occupancy: measured on 16,384
// searches x 1,000 iterations (queue of 64), the matrix cores gain 4 % at L = 201 and 255 and lose
// 25-27 % at L = 61 and 101 and 6-25 % at L = 303 and 383 (two tiles).
template <int SHAPE> struct PqWalkerOf {
    static constexpr bool mfma = SHAPE >= 2 && SHAPE <= 4;
    using Lds = WaveLdsPqT<typename std::conditional<mfma, WaveLdsMfma, WaveLdsBits>::type>;
    using type = typename std::conditional<mfma, MfmaWalker<MfmaKW<SHAPE>::value, false, Lds>,
                                           Walker<ShapeGK<SHAPE>::G, ShapeGK<SHAPE>::KW, false>>::type;
};

__device__ __forceinline__ int32_t wave_shr1(int32_t v)
{
    return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false); // lane i <- lane i-1
}

__device__ __forceinline__ int32_t wave_shl1(int32_t v)
{
    return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, false); // lane i <- lane i+1
}

// The queue: one entry per lane.
struct Queue {
    int32_t isl;       // INT32_MAX past the last entry
    int32_t gen;       // iteration that generated the entry
    int32_t j;         // flip of the generating state
    uint32_t hlo, hhi; // hash of the entry's state
    uint32_t x[kXWords];

    __device__ __forceinline__ void clear()
    {
        isl = INT32_MAX;
        gen = -1;
        j = 0;
        hlo = hhi = 0;
#pragma unroll
        for (int i = 0; i < kXWords; i++)
            x[i] = 0;
    }

    // lanes above pos take the entry below them; lane pos takes the new entry
    __device__ __forceinline__ void insert(int lane, int pos, int32_t nisl, int32_t ngen, int32_t nj, uint64_t nh,
                                           const uint32_t (&nx)[kXWords])
    {
        const bool up = lane > pos, at = lane == pos;
        int32_t v;
        v = wave_shr1(isl);
        isl = at ? nisl : (up ? v : isl);
        v = wave_shr1(gen);
        gen = at ? ngen : (up ? v : gen);
        v = wave_shr1(j);
        j = at ? nj : (up ? v : j);
        v = wave_shr1((int32_t)hlo);
        hlo = at ? (uint32_t)nh : (up ? (uint32_t)v : hlo);
        v = wave_shr1((int32_t)hhi);
        hhi = at ? (uint32_t)(nh >> 32) : (up ? (uint32_t)v : hhi);
#pragma unroll
        for (int i = 0; i < kXWords; i++) {
            v = wave_shr1((int32_t)x[i]);
            x[i] = at ? nx[i] : (up ? (uint32_t)v : x[i]);
        }
    }

    // every lane takes the entry above it (the front entry leaves); lane 63 becomes empty
    __device__ __forceinline__ void pop_front(int lane)
    {
        const bool last = lane == kWave - 1;
        int32_t v;
        v = wave_shl1(isl);
        isl = last ? INT32_MAX : v;
        v = wave_shl1(gen);
        gen = last ? -1 : v;
        v = wave_shl1(j);
        j = last ? 0 : v;
        v = wave_shl1((int32_t)hlo);
        hlo = last ? 0u : (uint32_t)v;
        v = wave_shl1((int32_t)hhi);
        hhi = last ? 0u : (uint32_t)v;
#pragma unroll
        for (int i = 0; i < kXWords; i++) {
            v = wave_shl1((int32_t)x[i]);
            x[i] = last ? 0u : (uint32_t)v;
        }
    }
};

template <class W, class PqLds>
__device__ __forceinline__ void run_pq(WalkState *__restrict__ wsp, uint64_t *__restrict__ tables,
                                       uint64_t *__restrict__ N, int nlog2, int cap, int32_t *__restrict__ trace,
                                       int32_t *__restrict__ scores, PqLds *lds, const uint64_t *zk)
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
    const int tlog2 = su(ws.table_log2);
    const bool exact = n <= tlog2;
    const bool nbr = nlog2 > 0;
    const bool nexact = nbr && n <= nlog2;
    const uint64_t seed = su(ws.seed);
    const uint32_t walk_id = su(ws.walk_id);
    const int32_t steps = (int32_t)su(ws.steps);
    const int64_t R = su(ws.restart_period);
    const int64_t target = su(ws.target_isl);
    const int64_t watch = su(ws.watch_isl);
    uint64_t *T = tables + su(ws.table_offset);
    const int64_t trace_off = su(ws.trace_offset);
    const int64_t score_off = su(ws.score_offset);
    int32_t *trp = trace_off >= 0 ? trace + 2 * trace_off : nullptr;
    int32_t *scp = score_off >= 0 ? scores + score_off : nullptr;

    // second-table slot partners: neighbours j and j' of one state share a slot exactly when the
    // top nlog2 bits of their Zobrist keys agree (the state's hash is XORed into both)
    int32_t nxt0[G];
#pragma unroll
    for (int g = 0; g < G; g++) {
        const int j = w.flip(g);
        int p = -1;
        if (nbr && !nexact && j < n) {
            const uint64_t sj = zk[j] >> (64 - nlog2);
            for (int q2 = j + 1; q2 < n; q2++) {
                if ((zk[q2] >> (64 - nlog2)) == sj) {
                    p = q2;
                    break;
                }
            }
        }
        nxt0[g] = p;
        if (j < kNMax)
            lds->nxt[j] = (int16_t)p;
    }
    lds_fence();

    Queue pq;
    pq.clear();
    int q = 0;

    int32_t restart_idx = 0, restarts = 0, traps = 0;
    int32_t t = 0;
    int64_t flips = 0;
    const int32_t tgt = target < 0 ? -1 : (int32_t)min<int64_t>(target, INT32_MAX);
    const int32_t wch = watch < 0 ? -1 : (int32_t)min<int64_t>(watch, INT32_MAX);
    const int32_t R32 = (int32_t)min<int64_t>(R, INT32_MAX);

    auto start = [&]() {
        start_bits(seed, walk_id, (uint32_t)restart_idx, n, w.x);
        clear_table(T, tlog2);
        if (nbr)
            clear_table(N, nlog2);
        w.rebuild();
        if (lane == 0)
            T[slot_of(w.h, w.x[0], exact, tlog2)] = w.h | 1ull;
        pq.clear();
        q = 0;
    };
    start();
    int32_t best32 = w.isl;
    int32_t best_step = 0;
    uint32_t best_x[kXWords];
#pragma unroll
    for (int i = 0; i < kXWords; i++)
        best_x[i] = w.x[i];
    int32_t hit = (tgt >= 0 && w.isl <= tgt) ? 0 : -1;
    int32_t wstep = (wch >= 0 && w.isl <= wch) ? 0 : -1;
    // a restart state counts for the best like the initial state, occupied after iteration ts
    auto note_start = [&](int32_t ts) {
        if (w.isl < best32) {
            best32 = w.isl;
            best_step = ts;
#pragma unroll
            for (int i = 0; i < kXWords; i++)
                best_x[i] = w.x[i];
        }
    };

    while (t < steps && !(tgt >= 0 && hit >= 0)) {
        asm volatile("" : "+v"(w.lane));
        w.prepare();
        int32_t isl_j[G];
        w.score(isl_j);
        if (scp) {
#pragma unroll
            for (int g = 0; g < G; g++) {
                const int j = w.flip(g);
                if (j < n)
                    scp[j] = isl_j[g];
            }
            scp += n;
        }

        // look-ups against the tables as they were before this iteration
        const int32_t thr = (q == cap) ? readlane_i(pq.isl, cap - 1) : INT32_MAX;
        // Without the second table the visited table is probed lazily, a batch of the smallest
        // unprobed candidates at a time (a candidate can only matter once it is the smallest
        // left); with it, every unskipped neighbour is probed, since its recording depends on it.
        uint32_t cand[G];
        bool ins[G], known[G], visited[G];
        uint64_t hn[G];
        uint32_t x0n[G];
        int skipped = 0;
#pragma unroll
        for (int g = 0; g < G; g++) {
            const int j = w.flip(g);
            const bool valid = j < n;
            const int jj = valid ? j : 0;
            hn[g] = w.h ^ zk[jj];
            x0n[g] = w.x[0];
            if (jj < 32)
                x0n[g] ^= 1u << jj;
            bool nh = false;
            if (nbr && valid)
                nh = N[slot_of(hn[g], x0n[g], nexact, nlog2)] == (hn[g] | 1ull);
            visited[g] = false;
            if (nbr && valid && !nh)
                visited[g] = T[slot_of(hn[g], x0n[g], exact, tlog2)] == (hn[g] | 1ull);
            known[g] = nbr;
            ins[g] = valid && !nh && !visited[g];
            cand[g] = (ins[g] && isl_j[g] < thr) ? (((uint32_t)isl_j[g] << 8) | (uint32_t)j) : 0xFFFFFFFFu;
            skipped += __builtin_popcountll(ballot(nh));
        }
        flips += n - skipped;

        // record the evaluated, unvisited neighbours in the second table
        if (nbr) {
            uint64_t M[G];
#pragma unroll
            for (int g = 0; g < G; g++)
                M[g] = ballot(ins[g]);
#pragma unroll
            for (int g = 0; g < G; g++) {
                if (ins[g]) {
                    bool later = false;
                    int p = nxt0[g];
                    while (p >= 0 && !later) {
                        uint64_t m = M[0];
#pragma unroll
                        for (int g2 = 1; g2 < G; g2++)
                            m = (W::owner_slot(p) == g2) ? M[g2] : m;
                        later = ((m >> W::owner_lane(p)) & 1ull) != 0ull;
                        p = lds->nxt[p];
                    }
                    if (!later) {
                        const int j = w.flip(g);
                        uint32_t x0 = w.x[0];
                        if (j < 32)
                            x0 ^= 1u << j;
                        N[slot_of(hn[g], x0, nexact, nlog2)] = hn[g] | 1ull;
                    }
                }
            }
        }

        // offer the candidates in ascending (ISL, flip) order
        while (true) {
            uint32_t km = cand[0];
#pragma unroll
            for (int g = 1; g < G; g++)
                km = min(km, cand[g]);
            const uint32_t k = wave_min_u32(km);
            if (k == 0xFFFFFFFFu)
                break;
            const int32_t nisl = (int32_t)(k >> 8);
            const int jn = (int)(k & 255u);
            if (q == cap && nisl >= readlane_i(pq.isl, cap - 1))
                break;
            bool kn = false, vis = false;
#pragma unroll
            for (int g = 0; g < G; g++) {
                kn = (w.flip(g) == jn) ? known[g] : kn;
                vis = (w.flip(g) == jn) ? visited[g] : vis;
            }
            const int owner = W::owner_lane(jn);
            if (!readlane_b(kn, owner)) {
                // probe the kPqProbe smallest unprobed candidates together
                uint32_t uk[G];
#pragma unroll
                for (int g = 0; g < G; g++)
                    uk[g] = known[g] ? 0xFFFFFFFFu : cand[g];
                bool sel[G];
#pragma unroll
                for (int g = 0; g < G; g++)
                    sel[g] = false;
#pragma unroll
                for (int b = 0; b < kPqProbe; b++) {
                    uint32_t um = uk[0];
#pragma unroll
                    for (int g = 1; g < G; g++)
                        um = min(um, uk[g]);
                    const uint32_t u = wave_min_u32(um);
                    if (u == 0xFFFFFFFFu)
                        break;
#pragma unroll
                    for (int g = 0; g < G; g++) {
                        const bool me = w.flip(g) == (int)(u & 255u);
                        sel[g] = sel[g] || me;
                        uk[g] = me ? 0xFFFFFFFFu : uk[g];
                    }
                }
#pragma unroll
                for (int g = 0; g < G; g++) {
                    if (sel[g]) {
                        visited[g] = T[slot_of(hn[g], x0n[g], exact, tlog2)] == (hn[g] | 1ull);
                        known[g] = true;
                    }
                }
#pragma unroll
                for (int g = 0; g < G; g++)
                    vis = (w.flip(g) == jn) ? visited[g] : vis;
            }
            if (readlane_b(vis, owner)) {
#pragma unroll
                for (int g = 0; g < G; g++)
                    cand[g] = (w.flip(g) == jn) ? 0xFFFFFFFFu : cand[g];
                continue;
            }
            uint32_t nx[kXWords];
#pragma unroll
            for (int i = 0; i < kXWords; i++)
                nx[i] = w.x[i];
            xflip_uniform(nx, jn);
            if (nisl < best32) {
                best32 = nisl;
                best_step = t + 1;
#pragma unroll
                for (int i = 0; i < kXWords; i++)
                    best_x[i] = nx[i];
            }
            const uint64_t zn = zk[jn];
            const uint64_t nh = w.h ^ (((uint64_t)uniform((uint32_t)(zn >> 32)) << 32) | uniform((uint32_t)zn));
            const int pos = __builtin_popcountll(ballot(w.lane < q && pq.isl <= nisl));
            pq.insert(w.lane, pos, nisl, t, jn, nh, nx);
            q = min(q + 1, cap);
#pragma unroll
            for (int g = 0; g < G; g++)
                cand[g] = (w.flip(g) == jn) ? 0xFFFFFFFFu : cand[g];
        }
        // entries past the capacity are not part of the queue
        if (w.lane >= cap)
            pq.clear();

        // take the front entry whose state has not been visited
        bool found = false;
        int32_t e_isl = 0, e_gen = 0, e_j = 0;
        uint64_t e_h = 0;
        uint32_t e_x[kXWords];
#pragma unroll
        for (int i = 0; i < kXWords; i++)
            e_x[i] = 0;
        while (q > 0) {
            e_isl = readlane_i(pq.isl, 0);
            e_gen = readlane_i(pq.gen, 0);
            e_j = readlane_i(pq.j, 0);
            e_h = ((uint64_t)readlane(pq.hhi, 0) << 32) | readlane(pq.hlo, 0);
#pragma unroll
            for (int i = 0; i < kXWords; i++)
                e_x[i] = readlane(pq.x[i], 0);
            pq.pop_front(w.lane);
            q--;
            // an entry offered in this iteration was probed then, and the table has not changed
            // since: it is unvisited without a second look
            if (e_gen == t) {
                found = true;
                break;
            }
            uint64_t got = 0;
            if (w.lane == 0)
                got = T[slot_of(e_h, e_x[0], exact, tlog2)];
            const uint64_t g0 = ((uint64_t)readlane((uint32_t)(got >> 32), 0) << 32) | readlane((uint32_t)got, 0);
            if (g0 != (e_h | 1ull)) {
                found = true;
                break;
            }
        }

        int32_t move;
        if (!found) {
            traps++;
            restarts++;
            restart_idx++;
            start();
            note_start(t + 1);
            move = -1;
        } else {
            if (e_gen == t) {
                w.commit(e_j, e_isl);
                move = e_j;
            } else {
                // an older entry: reach it by single flips when it is near (each flip updates the
                // table incrementally), else rebuild from its free bits
                int dist = 0;
#pragma unroll
                for (int i = 0; i < kXWords; i++)
                    dist += __builtin_popcount(w.x[i] ^ e_x[i]);
                if (dist <= kPqNearFlips) {
#pragma unroll
                    for (int i = 0; i < kXWords; i++) {
                        uint32_t d = w.x[i] ^ e_x[i];
                        while (d != 0u) {
                            const int b = __builtin_ctz(d);
                            d &= d - 1u;
                            w.commit(32 * i + b, 0);
                        }
                    }
                    int32_t sq = 0;
#pragma unroll
                    for (int q = 0; q < W::QR; q++)
                        sq += w.Cv[q] * w.Cv[q];
                    w.isl = wave_sum_i32(sq);
                } else {
#pragma unroll
                    for (int i = 0; i < kXWords; i++)
                        w.x[i] = e_x[i];
                    w.rebuild();
                }
                move = -2;
            }
            if (w.lane == 0)
                T[slot_of(w.h, w.x[0], exact, tlog2)] = w.h | 1ull;
        }
        t++;
        if (trp) {
            if (w.lane == 0) {
                trp[0] = move;
                trp[1] = w.isl;
            }
            trp += 2;
        }
        if (tgt >= 0 && hit < 0 && best32 <= tgt)
            hit = t;
        if (wch >= 0 && wstep < 0 && best32 <= wch)
            wstep = t;
        if (found && R32 > 0 && (t % R32) == 0 && t < steps && !(tgt >= 0 && hit >= 0)) {
            restarts++;
            restart_idx++;
            start();
            note_start(t);
            if (tgt >= 0 && hit < 0 && best32 <= tgt)
                hit = t;
            if (wch >= 0 && wstep < 0 && best32 <= wch)
                wstep = t;
        }
    }

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
        ws.traps = traps;
#pragma unroll
        for (int i = 0; i < kXWords; i++) {
            ws.x[i] = w.x[i];
            ws.best_x[i] = best_x[i];
        }
        ws.status = kDone;
    }
}

template <int SHAPE>
__global__ void __launch_bounds__(64) k_pq_walk(WalkState *__restrict__ states, int32_t count,
                                                const int32_t *__restrict__ order, uint64_t *__restrict__ tables,
                                                uint64_t *__restrict__ nbr_tables, int nlog2, int cap,
                                                int32_t *__restrict__ trace, int32_t *__restrict__ scores)
{
    using W = typename PqWalkerOf<SHAPE>::type;
    __shared__ uint64_t zk[kNMax];
    __shared__ typename PqWalkerOf<SHAPE>::Lds lds;
    fill_zobrist(zk);
    const int idx = (int)blockIdx.x;
    if (idx >= count)
        return;
    const int wi = order[idx];
    uint64_t *N = nlog2 > 0 ? nbr_tables + ((int64_t)wi << nlog2) : nullptr;
    run_pq<W>(&states[wi], tables, N, nlog2, cap, trace, scores, &lds, zk);
}

} // namespace

hipError_t launch_pq_walk(int shape, WalkState *states, int32_t count, const int32_t *order, uint64_t *tables,
                          uint64_t *nbr_tables, int nlog2, int cap, int32_t *trace, int32_t *scores,
                          hipStream_t stream)
{
    if (count <= 0)
        return hipSuccess;
    const dim3 grid((unsigned)count), block(64);
    switch (shape) {
    case 0: hipLaunchKernelGGL(k_pq_walk<0>, grid, block, 0, stream, states, count, order, tables, nbr_tables, nlog2, cap, trace, scores); break;
    case 1: hipLaunchKernelGGL(k_pq_walk<1>, grid, block, 0, stream, states, count, order, tables, nbr_tables, nlog2, cap, trace, scores); break;
    case 2: hipLaunchKernelGGL(k_pq_walk<2>, grid, block, 0, stream, states, count, order, tables, nbr_tables, nlog2, cap, trace, scores); break;
    case 3: hipLaunchKernelGGL(k_pq_walk<3>, grid, block, 0, stream, states, count, order, tables, nbr_tables, nlog2, cap, trace, scores); break;
    case 4: hipLaunchKernelGGL(k_pq_walk<4>, grid, block, 0, stream, states, count, order, tables, nbr_tables, nlog2, cap, trace, scores); break;
    case 5: hipLaunchKernelGGL(k_pq_walk<5>, grid, block, 0, stream, states, count, order, tables, nbr_tables, nlog2, cap, trace, scores); break;
    case 6: hipLaunchKernelGGL(k_pq_walk<6>, grid, block, 0, stream, states, count, order, tables, nbr_tables, nlog2, cap, trace, scores); break;
    case 7: hipLaunchKernelGGL(k_pq_walk<7>, grid, block, 0, stream, states, count, order, tables, nbr_tables, nlog2, cap, trace, scores); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

} // namespace liblabs
