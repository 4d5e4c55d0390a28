// enum_kernels.hip -- the exhaustive minimum over the skew-symmetric space of one odd length
// (Eq. (2), (4); Section 1's search-space reduction), grouped by the two ISL-preserving
// symmetries of skew sequences: negation (x -> x ^ A, A = the n free bits) and alternation
// s_i -> (-1)^i s_i (x -> x ^ O, O = the free bits at odd positions).  Every free-bit vector lies in exactly one group
// {x, x^A, x^O, x^A^O} with x = r << 2, so the kernel scores one member per group (a quarter of
// the 2^n sequences) and counts four.
//
// Work per sequence is plain ALU: the L-bit sequence sits in NW = ceil(L / 32) registers, and for
// every even lag k (odd lags vanish on skew sequences) C_k = (L - k) - 2 popcount((s ^ (s >> k))
// masked to the L - k overlapping positions).  One lane scores B sequences per pass so that the
// per-lag masks, computed on the scalar unit, are shared.  No memory traffic in the loop.
#include <hip/hip_runtime.h>

#include "device_common.hpp"
#include "internal.hpp"

namespace liblabs {

namespace {

constexpr int kEnumBlock = 256;
constexpr int kEnumB = 8;

// x -> the L-bit sequence (bit 1 = symbol -1) in w[0..NW-1], w[NW] = 0: bits 0..c are x, bit
// c + i is bit c - i of x flipped for odd i (Eq. (4)).  hi_mask / alt: bits c+1..2c, and the odd
// ones among them, as 128-bit values; sh = 127 - 2c.
template <int NW>
__device__ __forceinline__ void expand(uint64_t x, int sh, unsigned __int128 hi_mask, unsigned __int128 alt,
                                       uint32_t (&w)[NW + 1])
{
    const uint64_t rev = __builtin_bitreverse64(x);
    unsigned __int128 v;
    if (NW <= 2) // L <= 63: 2c <= 62, sh >= 65
        v = (unsigned __int128)(rev >> (sh - 64));
    else // L >= 65: sh <= 63
        v = ((unsigned __int128)rev << (64 - sh)) | ((unsigned __int128)(rev >> sh) << 64);
    v = ((v & hi_mask) ^ alt) | (unsigned __int128)x;
#pragma unroll
    for (int i = 0; i < NW; i++)
        w[i] = (uint32_t)(v >> (32 * i));
    w[NW] = 0u;
}

// popcount(x) + acc with a wave-uniform acc taken straight from a scalar register.
__device__ __forceinline__ uint32_t bcnt_acc_s(uint32_t x, uint32_t acc)
{
    uint32_t r;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "s"(acc));
    return r;
}

// acc + (2e + 1)^2 for |2e + 1| < 2^23: one shift-or and one 24-bit multiply-add.
__device__ __forceinline__ uint32_t sq_acc(uint32_t e, uint32_t acc)
{
    const uint32_t C = (e << 1) | 1u;
    uint32_t r;
    asm("v_mad_i32_i24 %0, %1, %1, %2" : "=v"(r) : "v"(C), "v"(acc));
    return r;
}

__device__ __forceinline__ uint64_t group_min(uint64_t x, uint64_t A, uint64_t O)
{
    uint64_t m = x;
    m = (x ^ A) < m ? (x ^ A) : m;
    m = (x ^ O) < m ? (x ^ O) : m;
    m = (x ^ A ^ O) < m ? (x ^ A ^ O) : m;
    return m;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v)
{
    const uint32_t hi = wave_min_u32((uint32_t)(v >> 32));
    const uint32_t lo = wave_min_u32((uint32_t)(v >> 32) == hi ? (uint32_t)v : 0xFFFFFFFFu);
    return ((uint64_t)hi << 32) | lo;
}

// (the word operations of both sides add up whatever their minima)
__device__ __forceinline__ void fold(EnumPartial &a, const EnumPartial &b)
{
    const uint64_t ops = a.word_ops + b.word_ops;
    if (b.min_isl != 0xFFFFFFFFu) {
        if (b.min_isl < a.min_isl) {
            a = b;
        } else if (b.min_isl == a.min_isl) {
            a.count += b.count;
            a.first_x = b.first_x < a.first_x ? b.first_x : a.first_x;
        }
    }
    a.word_ops = ops;
}

// Fold (best, cnt, first) of every thread of the block, and the word operations of its waves
// (wave-uniform), into part (read-modify-write: one slot per block, the same block index on every
// launch of one enumeration).
__device__ void block_merge(uint32_t best, uint32_t cnt, uint64_t first, uint64_t ops, EnumPartial *part)
{
    __shared__ uint32_t s_best[kEnumBlock / kWave];
    __shared__ uint32_t s_cnt[kEnumBlock / kWave];
    __shared__ uint64_t s_first[kEnumBlock / kWave];
    __shared__ uint64_t s_ops[kEnumBlock / kWave];
    const uint32_t wb = wave_min_u32(best);
    const uint32_t wc = (uint32_t)wave_sum_i32(best == wb ? (int32_t)cnt : 0);
    const uint64_t wf = wave_min_u64(best == wb ? first : ~0ull);
    const int wave = (int)(threadIdx.x / kWave);
    if (lane_id() == 0) {
        s_best[wave] = wb;
        s_cnt[wave] = wc;
        s_first[wave] = wf;
        s_ops[wave] = ops;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        EnumPartial p = part[blockIdx.x];
        for (int i = 0; i < (int)(blockDim.x / kWave); i++) {
            EnumPartial w;
            w.min_isl = s_best[i];
            w.reserved = 0;
            w.count = s_cnt[i];
            w.first_x = s_first[i];
            w.word_ops = s_ops[i];
            fold(p, w);
        }
        part[blockIdx.x] = p;
    }
}

// Groups r_begin .. r_begin + r_count - 1 (r_count <= 2^32), B consecutive groups per lane pass.
template <int NW>
__global__ void __launch_bounds__(kEnumBlock) k_enum_min(int L, uint64_t r_begin, uint64_t r_count,
                                                         EnumPartial *__restrict__ part)
{
    const int n = (L + 1) / 2, c = n - 1;
    const uint64_t A = (n == 64) ? ~0ull : ((1ull << n) - 1ull);
    uint64_t O = 0;
    for (int j = 1; j < n; j += 2)
        O |= 1ull << j;
    unsigned __int128 hi_mask = 0, alt = 0;
    for (int i = 1; i <= c; i++) {
        hi_mask |= (unsigned __int128)1 << (c + i);
        if (i & 1)
            alt |= (unsigned __int128)1 << (c + i);
    }
    const int sh = 127 - 2 * c;

    uint32_t best = 0xFFFFFFFFu, cnt = 0;
    uint64_t first = ~0ull;
    // algorithmic word operations of the (sequence, lag) pairs this wave evaluates: 3 per word of
    // the L - k overlapping positions (funnel shift, masked xor, popcount) and 2 for C_k^2, summed
    // over the lags each pass actually runs (wave-uniform)
    uint64_t ops = 0;
    // Pruning bound (wave-uniform): the lowest ISL any lane of the wave has found, and what this
    // block slot holds from earlier launches of the same enumeration.  Every C_k^2 >= 0, so a
    // partial sum above the bound is above the minimum: once every sequence of the wave's pass is
    // above it, the pass stops (a sequence at the minimum is never cut, so the minimum, its
    // multiplicity and its lowest argument are unchanged).
    const uint32_t bound0 = part[blockIdx.x].min_isl;
    const uint64_t n_pass = (r_count + kEnumB - 1) / kEnumB;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    // the loop runs per wave (every lane stays active for the wave-wide reductions); lanes past
    // the last pass compute a sequence that is never recorded or counted as live
    const uint64_t wave_base = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(uint32_t)(kWave - 1));
    for (uint64_t g0 = wave_base; g0 < n_pass; g0 += stride) {
        const uint64_t g = g0 + lane_id();
        const bool valid = g < n_pass;
        const uint32_t bound = min(bound0, wave_min_u32(best));
        // sequences of this wave pass inside the block (all of them but in the last passes)
        uint32_t seqs = (uint32_t)(kWave * kEnumB);
        if ((g0 + kWave) * kEnumB > r_count)
            seqs = (uint32_t)wave_sum_i32(valid ? (int32_t)min<uint64_t>(kEnumB, r_count - g * kEnumB) : 0);
        uint32_t w[kEnumB][NW + 1];
        uint32_t isl[kEnumB];
#pragma unroll
        for (int u = 0; u < kEnumB; u++) {
            const uint64_t r = r_begin + g * kEnumB + u;
            expand<NW>(r << 2, sh, hi_mask, alt, w[u]);
            isl[u] = 0;
        }
        bool cut = false;
#pragma unroll
        for (int q = 0; q < NW && !cut; q++) {
#pragma unroll 1
            for (int b = (q == 0 ? 2 : 0); b < 32; b += 2) {
                const int k = 32 * q + b;
                if (k >= L)
                    break;
                const int len = L - k;
                ops += (uint64_t)seqs * (uint64_t)(3 * ((len + 31) / 32) + 2);
                uint32_t m[NW];
#pragma unroll
                for (int i = 0; i < NW; i++) {
                    const int rem = len - 32 * i;
                    m[i] = rem >= 32 ? 0xFFFFFFFFu : (rem <= 0 ? 0u : ((1u << rem) - 1u));
                }
#pragma unroll
                for (int u = 0; u < kEnumB; u++) {
                    // e = disagreements - (len + 1) / 2, so that C_k = 2 d - len = 2 e + 1
                    uint32_t e = bcnt_acc_s((w[u][0] ^ funnel(w[u][q + 1], w[u][q], b)) & m[0],
                                            (uint32_t)(-(len + 1) / 2));
#pragma unroll
                    for (int i = 1; i < NW - q; i++)
                        e = bcnt_acc((w[u][i] ^ funnel(w[u][i + q + 1], w[u][i + q], b)) & m[i], e);
                    isl[u] = sq_acc(e, isl[u]);
                }
                bool live = false;
#pragma unroll
                for (int u = 0; u < kEnumB; u++)
                    live = live || isl[u] <= bound;
                live = live && valid;
                if (ballot(live) == 0ull) {
                    cut = true;
                    break;
                }
            }
        }
        if (cut)
            continue;
        uint32_t lo = isl[0];
#pragma unroll
        for (int u = 1; u < kEnumB; u++)
            lo = isl[u] < lo ? isl[u] : lo;
        if (lo > best)
            continue;
#pragma unroll
        for (int u = 0; u < kEnumB; u++) {
            const uint64_t r = r_begin + g * kEnumB + u;
            if (g * kEnumB + u < r_count && isl[u] <= best) {
                const uint64_t f = group_min(r << 2, A, O);
                if (isl[u] < best) {
                    best = isl[u];
                    cnt = 4;
                    first = f;
                } else {
                    cnt += 4;
                    first = f < first ? f : first;
                }
            }
        }
    }
    block_merge(best, cnt, first, ops, part);
}

__global__ void k_enum_part_init(EnumPartial *part, int count)
{
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i < count) {
        EnumPartial p;
        p.min_isl = 0xFFFFFFFFu;
        p.reserved = 0;
        p.count = 0;
        p.first_x = ~0ull;
        p.word_ops = 0;
        part[i] = p;
    }
}

// One block folds count partials into out.
__global__ void __launch_bounds__(kEnumBlock) k_enum_final(const EnumPartial *__restrict__ part, int count,
                                                           EnumPartial *__restrict__ out)
{
    __shared__ EnumPartial s_p[kEnumBlock];
    EnumPartial acc;
    acc.min_isl = 0xFFFFFFFFu;
    acc.reserved = 0;
    acc.count = 0;
    acc.first_x = ~0ull;
    acc.word_ops = 0;
    for (int i = (int)threadIdx.x; i < count; i += (int)blockDim.x)
        fold(acc, part[i]);
    s_p[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < (int)blockDim.x; i++)
            fold(acc, s_p[i]);
        *out = acc;
    }
}

template <int NW>
int resident_blocks()
{
    static int cached = 0;
    if (cached)
        return cached;
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_enum_min<NW>, kEnumBlock, 0) != hipSuccess)
        return 0;
    cached = std::max(1, cus * std::max(1, per_cu));
    return cached;
}

} // namespace

int enum_min_blocks(int L)
{
    switch ((L + 31) / 32) {
    case 1: return resident_blocks<1>();
    case 2: return resident_blocks<2>();
    case 3: return resident_blocks<3>();
    case 4: return resident_blocks<4>();
    }
    return 0;
}

hipError_t launch_enum_part_init(EnumPartial *part, int count, hipStream_t stream)
{
    hipLaunchKernelGGL(k_enum_part_init, dim3((count + 255) / 256), dim3(256), 0, stream, part, count);
    return hipGetLastError();
}

hipError_t launch_enum_min(int L, uint64_t r_begin, uint64_t r_count, EnumPartial *part, int blocks,
                           hipStream_t stream)
{
    const uint64_t lanes_needed = (r_count + kEnumB - 1) / kEnumB;
    const uint64_t blocks_needed = (lanes_needed + kEnumBlock - 1) / kEnumBlock;
    const int grid = (int)std::min<uint64_t>((uint64_t)blocks, std::max<uint64_t>(1, blocks_needed));
    switch ((L + 31) / 32) {
    case 1: hipLaunchKernelGGL(k_enum_min<1>, dim3(grid), dim3(kEnumBlock), 0, stream, L, r_begin, r_count, part); break;
    case 2: hipLaunchKernelGGL(k_enum_min<2>, dim3(grid), dim3(kEnumBlock), 0, stream, L, r_begin, r_count, part); break;
    case 3: hipLaunchKernelGGL(k_enum_min<3>, dim3(grid), dim3(kEnumBlock), 0, stream, L, r_begin, r_count, part); break;
    case 4: hipLaunchKernelGGL(k_enum_min<4>, dim3(grid), dim3(kEnumBlock), 0, stream, L, r_begin, r_count, part); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_enum_final(const EnumPartial *part, int count, EnumPartial *out, hipStream_t stream)
{
    hipLaunchKernelGGL(k_enum_final, dim3(1), dim3(kEnumBlock), 0, stream, part, count, out);
    return hipGetLastError();
}

} // namespace liblabs
