// walk_inst_mfma.hip -- instantiates the walk kernel and the batched one-flip evaluation with
// the matrix-core scoring (mfma_walker.hpp) for every shape (L <= 383): one tile for c <= 127,
// two for 128 <= c <= 191.

#include "mfma_walker.hpp"

namespace liblabs {

namespace {

// walker and LDS layout per shape: the small layout for c <= 127, the big one beyond and for
// the mixed-length kernel (SHAPE < 0), whose walkers all use it
template <int SHAPE> struct MfmaShape {
    static constexpr bool big = SHAPE >= 5;
    using Lds = typename std::conditional<SHAPE >= 0 && SHAPE <= 4, WaveLdsMfma, WaveLdsMfmaBig>::type;
    // occupancy target: eight waves per SIMD fit the one-tile walker's registers (64 VGPRs)
    static constexpr int waves = (SHAPE >= 0 && SHAPE <= 4) ? 8 : 5;
};

template <int SHAPE, int PW>
__device__ __forceinline__ void run_any_mfma(WalkState *ws, uint64_t *tables, int32_t *trace, int32_t *scores,
                                             int64_t chunk, typename MfmaShape<SHAPE>::Lds *lds,
                                             const uint64_t *zk)
{
    using Lds = typename MfmaShape<SHAPE>::Lds;
    if constexpr (SHAPE >= 0) {
        run_walk<MfmaWalker<MfmaKW<SHAPE>::value, MfmaShape<SHAPE>::big, Lds>, PW>(ws, tables, trace, scores, chunk,
                                                                                  lds, zk);
    } else {
        switch (shape_for_length_dev(ws->L)) {
        case 0: run_walk<MfmaWalker<1, false, Lds>, PW>(ws, tables, trace, scores, chunk, lds, zk); break;
        case 1: run_walk<MfmaWalker<2, false, Lds>, PW>(ws, tables, trace, scores, chunk, lds, zk); break;
        case 2: run_walk<MfmaWalker<3, false, Lds>, PW>(ws, tables, trace, scores, chunk, lds, zk); break;
        case 3: run_walk<MfmaWalker<3, false, Lds>, PW>(ws, tables, trace, scores, chunk, lds, zk); break;
        case 4: run_walk<MfmaWalker<4, false, Lds>, PW>(ws, tables, trace, scores, chunk, lds, zk); break;
        case 5: run_walk<MfmaWalker<4, true, Lds>, PW>(ws, tables, trace, scores, chunk, lds, zk); break;
        case 6: run_walk<MfmaWalker<5, true, Lds>, PW>(ws, tables, trace, scores, chunk, lds, zk); break;
        default: run_walk<MfmaWalker<6, true, Lds>, PW>(ws, tables, trace, scores, chunk, lds, zk); break;
        }
    }
}

template <int SHAPE, int PW>
__global__ void __launch_bounds__(64 * kMaxWavesPerBlock)
    __attribute__((amdgpu_waves_per_eu(MfmaShape<SHAPE>::waves))) k_walk_mfma(
        WalkState *__restrict__ states, int32_t n_walks, const int32_t *__restrict__ order,
        uint64_t *__restrict__ tables, int32_t *__restrict__ trace, int32_t *__restrict__ scores, int64_t chunk,
        int32_t *__restrict__ counter)
{
    using Lds = typename MfmaShape<SHAPE>::Lds;
    __shared__ uint64_t zk[kNMax];
    extern __shared__ __align__(16) unsigned char dyn_smem[];
    fill_zobrist(zk);
    const int wave = (int)uniform(threadIdx.x >> 6);
    const int wpb = (int)(blockDim.x >> 6);
    Lds *lds = reinterpret_cast<Lds *>(dyn_smem) + wave;
    int idx = (int)blockIdx.x * wpb + wave;
    bool first = true;
    while (true) {
        if (counter != nullptr) {
            int got = 0;
            if (lane_id() == 0)
                got = atomicAdd(counter, 1);
            idx = __builtin_amdgcn_readlane(got, 0);
        } else if (!first) {
            break;
        }
        first = false;
        if (idx >= n_walks)
            break;
        const int wi = order ? order[idx] : idx;
        run_any_mfma<SHAPE, PW>(&states[wi], tables, trace, scores, chunk, lds, zk);
    }
}

template <int KW, bool BIG>
__global__ void __launch_bounds__(64) k_flip_scores_mfma(int L, int count, const uint32_t *__restrict__ xs,
                                                         int32_t *__restrict__ out)
{
    using Lds = typename std::conditional<BIG, WaveLdsMfmaBig, WaveLdsMfma>::type;
    __shared__ uint64_t zk[kNMax];
    __shared__ Lds lds;
    fill_zobrist(zk);
    const int r = (int)blockIdx.x;
    if (r >= count)
        return;
    MfmaWalker<KW, BIG, Lds> w;
    w.lane = lane_id();
    w.set_length(L);
    w.lds = &lds;
    w.zk = zk;
    w.init_lanes(w.lane);
#pragma unroll
    for (int i = 0; i < kXWords; i++)
        w.x[i] = xs[(int64_t)r * kXWords + i];
    w.rebuild();
    w.prepare();
    constexpr int G = MfmaWalker<KW, BIG, Lds>::G;
    int32_t isl_j[G];
    w.score(isl_j);
#pragma unroll
    for (int g = 0; g < G; g++) {
        const int j = w.flip(g);
        if (j < w.n)
            out[(int64_t)r * w.n + j] = isl_j[g];
    }
}

} // namespace

WalkKernel pick_walk_kernel_mfma(int shape)
{
    switch (shape) {
    case 0: return k_walk_mfma<0, 2>;
    case 1: return k_walk_mfma<1, 2>;
    case 2: return k_walk_mfma<2, 2>;
    case 3: return k_walk_mfma<3, 2>;
    case 4: return k_walk_mfma<4, 2>;
    case 5: return k_walk_mfma<5, 2>;
    case 6: return k_walk_mfma<6, 2>;
    case 7: return k_walk_mfma<7, 2>;
    case -1: return k_walk_mfma<-1, 2>;
    default: return nullptr;
    }
}

size_t mfma_wave_lds_bytes(int shape)
{
    return (shape >= 0 && shape <= 4) ? sizeof(WaveLdsMfma) : sizeof(WaveLdsMfmaBig);
}

hipError_t launch_flip_scores_mfma(int L, int count, const uint32_t *x, int32_t *scores, hipStream_t stream)
{
    void (*k)(int, int, const uint32_t *, int32_t *) = nullptr;
    switch (shape_for_length(L)) {
    case 0: k = k_flip_scores_mfma<1, false>; break;
    case 1: k = k_flip_scores_mfma<2, false>; break;
    case 2: k = k_flip_scores_mfma<3, false>; break;
    case 3: k = k_flip_scores_mfma<3, false>; break;
    case 4: k = k_flip_scores_mfma<4, false>; break;
    case 5: k = k_flip_scores_mfma<4, true>; break;
    case 6: k = k_flip_scores_mfma<5, true>; break;
    case 7: k = k_flip_scores_mfma<6, true>; break;
    default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k, dim3(count), dim3(64), 0, stream, L, count, x, scores);
    return hipGetLastError();
}

} // namespace liblabs
