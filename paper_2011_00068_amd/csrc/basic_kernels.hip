// basic_kernels.hip -- batched definitions of Section 1 (Eq. (1)-(3), PSL) for arbitrary
// sequences, and exhaustive evaluation of every skew-symmetric sequence (Eq. (4)).
//
// Both work on bit-packed sequences (bit i = 1 <=> s_i = -1), using
//   C_k = (L - k) - 2 popcount(B xor (B >> k))   over the L - k valid positions,
// which is Eq. (1) with s_i s_{i+k} = 1 - 2 (b_i xor b_{i+k}).

#include "internal.hpp"

namespace liblabs {

// One workgroup per sequence; the sequence is packed into LDS and each thread owns a stride of
// shifts k.  L <= 65535 (2048 words + padding).
constexpr int kIslBlock = 256;

__global__ void __launch_bounds__(kIslBlock) k_isl_batch(int L, int count, const int8_t *__restrict__ s,
                                                         int64_t *__restrict__ isl, double *__restrict__ F,
                                                         int32_t *__restrict__ psl, int32_t *__restrict__ corr)
{
    extern __shared__ uint32_t bits[]; // nw + 2 words, zero padded
    __shared__ int64_t red_isl[kIslBlock / 64];
    __shared__ int32_t red_psl[kIslBlock / 64];
    const int r = (int)blockIdx.x;
    if (r >= count)
        return;
    const int nw = (L + 31) / 32;
    const int8_t *seq = s + (int64_t)r * L;
    // pack: thread w builds word w from 32 symbols
    for (int w = (int)threadIdx.x; w < nw + 2; w += kIslBlock) {
        uint32_t v = 0;
        if (w < nw) {
            for (int b = 0; b < 32; b++) {
                const int i = 32 * w + b;
                if (i < L && seq[i] < 0)
                    v |= 1u << b;
            }
        }
        bits[w] = v;
    }
    __syncthreads();
    int64_t my_isl = 0;
    int32_t my_psl = 0;
    for (int k = (int)threadIdx.x; k < L; k += kIslBlock) {
        const int valid = L - k;
        const int base = k >> 5, off = k & 31;
        int diff = 0;
        for (int w = 0; 32 * w < valid; w++) {
            const uint32_t sh = funnel(bits[base + w + 1], bits[base + w], off);
            diff += popc((bits[w] ^ sh) & low_mask(valid - 32 * w));
        }
        const int32_t Ck = valid - 2 * diff;
        if (corr)
            corr[(int64_t)r * L + k] = Ck;
        if (k >= 1) {
            my_isl += (int64_t)Ck * Ck;
            my_psl = max(my_psl, Ck < 0 ? -Ck : Ck);
        }
    }
    // block reduction: waves first (lanes via readlane sums of 32-bit halves would overflow,
    // so reduce int64 through LDS)
    for (int off = 32; off >= 1; off >>= 1) {
        my_isl += __shfl_down(my_isl, off, 64);
        my_psl = max(my_psl, __shfl_down(my_psl, off, 64));
    }
    const int wave = (int)(threadIdx.x >> 6);
    if (lane_id() == 0) {
        red_isl[wave] = my_isl;
        red_psl[wave] = my_psl;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t tot = 0;
        int32_t pk = 0;
        for (int i = 0; i < kIslBlock / 64; i++) {
            tot += red_isl[i];
            pk = max(pk, red_psl[i]);
        }
        isl[r] = tot;
        if (F)
            F[r] = tot == 0 ? -1.0 : ((double)L * (double)L) / (2.0 * (double)tot);
        if (psl)
            psl[r] = pk;
    }
}

// One thread per skew sequence: free bits x (bit j <=> s_j = -1), mirrored by Eq. (4).
__global__ void __launch_bounds__(256) k_enum_skew(int L, int32_t *__restrict__ out)
{
    const int n = (L + 1) / 2, c = n - 1;
    const uint64_t x = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= (1ull << n))
        return;
    uint64_t B = x;
    for (int i = 1; i <= c; i++) {
        const uint64_t b = ((x >> (c - i)) & 1ull) ^ (uint64_t)(i & 1);
        B |= b << (c + i);
    }
    int32_t acc = 0;
    for (int k = 1; k < L; k++) {
        const uint64_t m = (1ull << (L - k)) - 1ull;
        const int32_t Ck = (L - k) - 2 * __popcll((B ^ (B >> k)) & m);
        acc += Ck * Ck;
    }
    out[x] = acc;
}

hipError_t launch_isl_batch(int L, int count, const int8_t *s, int64_t *isl, double *F, int32_t *psl,
                            int32_t *corr, hipStream_t stream)
{
    if (count <= 0)
        return hipSuccess;
    const size_t lds = sizeof(uint32_t) * (size_t)((L + 31) / 32 + 2);
    hipLaunchKernelGGL(k_isl_batch, dim3(count), dim3(kIslBlock), lds, stream, L, count, s, isl, F, psl, corr);
    return hipGetLastError();
}

hipError_t launch_enum_skew(int L, int32_t *isl, hipStream_t stream)
{
    const int n = (L + 1) / 2;
    const uint64_t total = 1ull << n;
    const int blocks = (int)((total + 255) / 256);
    hipLaunchKernelGGL(k_enum_skew, dim3(blocks), dim3(256), 0, stream, L, isl);
    return hipGetLastError();
}

} // namespace liblabs
