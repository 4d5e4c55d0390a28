// walk_kernels.hip -- launch wrappers of the walk kernels, the batched one-flip evaluation
// kernel and the small state kernels.  The walk itself is in walk_impl.hpp; its kernels are
// instantiated in walk_inst_*.hip (one translation unit per variant and probe width).

#include "walk_impl.hpp"

namespace liblabs {

int shape_for_length(int L) { return shape_for_length_dev(L); }


int shape_groups(int shape)
{
    static const int g[8] = {1, 1, 2, 2, 2, 3, 3, 3};
    return g[shape & 7];
}

__global__ void k_reset(WalkState *__restrict__ states, const WalkState *__restrict__ pristine,
                        int32_t n_walks, int32_t *__restrict__ counter)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < n_walks) {
        // a run starts its walks afresh on the tables of the previous run: the table epochs
        // carry over, so that a start takes the next epoch instead of clearing the table
        const int32_t ep = states[i].table_epoch;
        states[i] = pristine[i];
        states[i].table_epoch = ep;
    }
    if (i == 0 && counter)
        *counter = 0;
}

// ---------------------------------------------------------------------------------------------
// Launch wrappers.
// ---------------------------------------------------------------------------------------------

static WalkKernel pick_kernel(const WalkLaunch &lp)
{
    if (lp.variant == LABS_VARIANT_MFMA)
        return pick_walk_kernel_mfma(lp.shape);
    const bool direct = lp.variant == LABS_VARIANT_DIRECT;
    return direct ? (lp.probe_width >= 2 ? pick_walk_kernel_direct_pw2(lp.shape)
                                         : pick_walk_kernel_direct_pw1(lp.shape))
                  : (lp.probe_width >= 2 ? pick_walk_kernel_bits_pw2(lp.shape)
                                         : pick_walk_kernel_bits_pw1(lp.shape));
}

static size_t wave_lds_bytes(int variant, int shape)
{
    if (variant == LABS_VARIANT_MFMA)
        return mfma_wave_lds_bytes(shape);
    return variant == LABS_VARIANT_DIRECT ? sizeof(WaveLdsDirect) : sizeof(WaveLdsBits);
}

int resident_walk_waves(const WalkLaunch &lp)
{
    const int wpb = lp.waves_per_block;
    const size_t lds = (size_t)wpb * wave_lds_bytes(lp.variant, lp.shape);
    int blocks = 0, dev = 0, cus = 0;
    if (!pick_kernel(lp))
        return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, reinterpret_cast<const void *>(pick_kernel(lp)),
                                                     64 * wpb, lds) != hipSuccess)
        return 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return blocks * wpb * cus;
}

hipError_t launch_walk(const WalkLaunch &lp, WalkState *states, int32_t n_walks, const int32_t *order,
                       uint64_t *tables, int32_t *trace, int32_t *scores, int32_t *counter,
                       hipStream_t stream)
{
    WalkKernel k = pick_kernel(lp);
    const int wpb = lp.waves_per_block;
    if (!k)
        return hipErrorInvalidValue;
    if (wpb < 1 || wpb > kMaxWavesPerBlock)
        return hipErrorInvalidConfiguration; // the kernel is compiled for at most 8 waves per block
    const size_t lds = (size_t)wpb * wave_lds_bytes(lp.variant, lp.shape);
    int blocks;
    int32_t *ctr = nullptr;
    if (lp.persistent) {
        blocks = (lp.grid_waves + wpb - 1) / wpb;
        ctr = counter;
    } else {
        blocks = (n_walks + wpb - 1) / wpb;
    }
    if (blocks <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k, dim3(blocks), dim3(64 * wpb), lds, stream, states, n_walks, order, tables, trace,
                       scores, lp.chunk, ctr);
    return hipGetLastError();
}

hipError_t launch_reset(WalkState *states, const WalkState *pristine, int32_t n_walks, int32_t *counter,
                        hipStream_t stream)
{
    const int blocks = (n_walks + 255) / 256;
    hipLaunchKernelGGL(k_reset, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, stream, states, pristine, n_walks,
                       counter);
    return hipGetLastError();
}

__global__ void k_zero_counter(int32_t *counter)
{
    if (threadIdx.x == 0)
        *counter = 0;
}

hipError_t launch_zero_counter(int32_t *counter, hipStream_t stream)
{
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, stream, counter);
    return hipGetLastError();
}

hipError_t launch_flip_scores(int32_t variant, int L, int count, const uint32_t *x, int32_t *scores,
                              hipStream_t stream)
{
    if (count <= 0)
        return hipSuccess;
    if (variant == LABS_VARIANT_MFMA)
        return launch_flip_scores_mfma(L, count, x, scores, stream);
    const bool direct = variant == LABS_VARIANT_DIRECT;
    void (*k)(int, int, const uint32_t *, int32_t *) = nullptr;
#define LABS_PICK(S)                                                                                  \
    case S: k = direct ? k_flip_scores<S, true> : k_flip_scores<S, false>; break;
    switch (shape_for_length(L)) {
        LABS_PICK(0) LABS_PICK(1) LABS_PICK(2) LABS_PICK(3) LABS_PICK(4) LABS_PICK(5) LABS_PICK(6)
        LABS_PICK(7)
    default: return hipErrorInvalidValue;
    }
#undef LABS_PICK
    hipLaunchKernelGGL(k, dim3(count), dim3(64), 0, stream, L, count, x, scores);
    return hipGetLastError();
}

} // namespace liblabs
