// probe_kernels.hip -- a measurement aid, not part of the method: a kernel that streams reads
// out of LDS, used to measure the LDS read bandwidth that bounds the walk kernels' LDS traffic.

#include "internal.hpp"

namespace liblabs {
namespace {

constexpr int kProbeThreads = 256;
constexpr int kProbeLdsWords = 16384; // 64 KB
constexpr int kProbeRows = 16;        // reads per round, one per row of kProbeThreads * W words

// Every lane reads W dwords from each of 16 rows (consecutive lanes, consecutive addresses: no
// bank conflicts) per round; the empty asm statement keeps the reads inside the round loop.  The
// sum is stored so that nothing is optimised away.
template <int W>
__global__ void __launch_bounds__(kProbeThreads) k_lds_read_probe(uint32_t *out, int rounds)
{
    static_assert(kProbeRows * kProbeThreads * W <= kProbeLdsWords, "rows exceed the LDS block");
    __shared__ uint32_t buf[kProbeLdsWords];
    const int tid = threadIdx.x;
    for (int i = tid; i < kProbeLdsWords; i += kProbeThreads)
        buf[i] = (uint32_t)i * 2654435761u;
    __syncthreads();
    const uint32_t *p = &buf[tid * W];
    uint32_t acc = 0;
    for (int r = 0; r < rounds; r++) {
        asm volatile("" ::: "memory");
#pragma unroll
        for (int k = 0; k < kProbeRows; k++) {
            const uint32_t *q = p + k * kProbeThreads * W;
            if constexpr (W == 4) {
                const uint4 v = *reinterpret_cast<const uint4 *>(q);
                acc += v.x + v.y + v.z + v.w;
            } else if constexpr (W == 2) {
                const uint2 v = *reinterpret_cast<const uint2 *>(q);
                acc += v.x + v.y;
            } else {
                acc += *q;
            }
        }
    }
    out[(size_t)blockIdx.x * kProbeThreads + tid] = acc;
}

} // namespace

int lds_probe_threads() { return kProbeThreads; }

double lds_probe_bytes(int bytes_per_lane, int blocks, int rounds)
{
    return (double)blocks * kProbeThreads * (double)rounds * kProbeRows * bytes_per_lane;
}

hipError_t launch_lds_read_probe(int bytes_per_lane, int blocks, int rounds, uint32_t *out, hipStream_t stream)
{
    switch (bytes_per_lane) {
    case 4: k_lds_read_probe<1><<<blocks, kProbeThreads, 0, stream>>>(out, rounds); break;
    case 8: k_lds_read_probe<2><<<blocks, kProbeThreads, 0, stream>>>(out, rounds); break;
    case 16: k_lds_read_probe<4><<<blocks, kProbeThreads, 0, stream>>>(out, rounds); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

} // namespace liblabs
