// gen_walk.hip -- the self-avoiding walk over general (not skew-symmetric) sequences: the
// unrestricted problem that the skew-symmetric restriction of Section 1 reduces.  All L symbols
// are free, a flip negates one symbol, and every shift k = 1 .. L-1 counts (odd ones included).
// The walk itself (table, probes, restarts, stop rules) is the skew walk's (run_walk); only the
// walker differs.  L <= 192 (the free bits of a state fill the same six 32-bit words).
//
// Scoring (from Eq. (1)): with s_i = 1 - 2 b_i and flip j,
//   dC_k = -2 s_j u_k,  u_k = p_k + q_k,  p_k = s_{j+k} [j+k <= L-1],  q_k = s_{j-k} [j-k >= 0],
//   ISL_j = sum_k (C_k + dC_k)^2 = ISL - 4 s_j G_j + 4 H_j,  G_j = sum_k C_k u_k,  H_j = sum_k u_k^2.
// With prefix sums PSX[a] = sum_{k=1..a} C_k, windows Wp[k-1] = b_{j+k}, Wq[k-1] = b_{j-k} and
// np = L-1-j, nq = j, m = min(np, nq):
//   G_j = PSX[np] + PSX[nq] - 2 sum_k C_k (Wp + Wq),
//   H_j = np + nq + 2 R_j,  R_j = sum_{k<=m} s_{j+k} s_{j-k} = m - 2 popcount((Wp ^ Wq) & low m),
// and sum_k C_k W_k is bit-sliced exactly as in the skew walker: one ballot per bit plane of C
// and 64 shifts, an AND + popcount per 32 shifts, Horner over the planes.
//
// Lane l owns flips j = l + 64 g (g < G = ceil(L/64)) and shifts k = l + 64 q + 1 (q < QR =
// ceil((L-1)/64)); KW = ceil((L-1)/32) window words.  The sequence lives in LDS as a forward bit
// string (bit a = b_a) and a reversed one (bit a = b_{191-a}) so that both windows are funnel
// shifts of 32-bit words.
#include <hip/hip_runtime.h>

#include "walk_impl.hpp"

namespace liblabs {

namespace {

constexpr int kGenLMax = kXWords * 32; // 192
constexpr int kGenWords = 16;          // bit-string words, zero padded past the sequence
constexpr int kGenRV = kGenLMax - 1;   // reversed string: bit a = b_{kGenRV - a}
constexpr int kGenSeqOff = kGenLMax;   // s_i at s8[kGenSeqOff + i]; zero padding covers every j +- k
constexpr int kGenSeqBytes = 3 * kGenLMax;

struct WaveLdsGen {
    uint32_t fw[kGenWords]; // bit a = b_a: the free bits (words 0 .. kXWords-1), zero padded
    uint32_t rv[kGenWords];
    uint32_t bestx[kXWords]; // free bits of the best state of the walk so far
    int32_t book[8];         // the walk loop's rarely updated bookkeeping
    int32_t C[kGenLMax + 1];   // C_k at index k, 0 past L-1
    int32_t psx[kGenLMax + 1]; // psx[a] = sum_{k=1..a} C_k
    int8_t s8[kGenSeqBytes];   // s_i at kGenSeqOff + i, 0 elsewhere
};

template <int G, int KW>
struct GenWalker {
    static constexpr int kG = G;
    static constexpr int QR = (KW + 1) / 2;
    using Lds = WaveLdsGen;

    int L, c, n;
    int lane;
    int32_t isl;
    uint64_t h;
    uint32_t x[kXWords]; // free bits; current only where commit<true> is used (else in lds->fw)
    uint32_t x0;         // free bits 0..31, always current
    int32_t Cv[QR];
    int32_t mult[G]; // -4 s_j (0 past the last flip)
    int planes;
    Lds *lds;
    const uint64_t *zk;

    __device__ __forceinline__ uint32_t *x_lds() const { return lds->fw; }
    __device__ __forceinline__ uint32_t *best_lds() const { return lds->bestx; }
    __device__ __forceinline__ int32_t *book_lds() const { return lds->book; }

    // b_js (uniform) from the lane that scores flip js: mult > 0 iff s_js = -1
    __device__ __forceinline__ uint32_t sbit_of(int js) const
    {
        int32_t v = 0;
#pragma unroll
        for (int g = 0; g < G; g++)
            v = (g == (js >> 6)) ? __builtin_amdgcn_readlane(mult[g], js & 63) : v;
        return v > 0 ? 1u : 0u;
    }

    __device__ __forceinline__ void set_length(int len)
    {
        L = len;
        n = len;
        c = -1; // no centre: every flip negates one symbol
    }

    __device__ __forceinline__ int flip(int g) const { return lane + 64 * g; }

    __device__ __forceinline__ void init_lanes(int) {}

    __device__ inline uint32_t bit(int i) const
    {
        if (i < 0 || i >= L)
            return 0u;
        return (lds->fw[i >> 5] >> (i & 31)) & 1u;
    }

    // Bit strings from x, C_k from scratch (Eq. (1)), ISL (Eq. (2)), Zobrist hash.
    __device__ __forceinline__ void rebuild()
    {
        const int lane = this->lane;
        x0 = x[0];
        if (lane < kGenWords) {
            uint32_t f = 0, r = 0;
#pragma unroll
            for (int i = 0; i < kXWords; i++) {
                f = (lane == i) ? x[i] : f;
                r = (lane == kXWords - 1 - i) ? __builtin_bitreverse32(x[i]) : r;
            }
            lds->fw[lane] = f;
            lds->rv[lane] = r;
        }
        lds_fence();
        for (int i = lane; i < kGenSeqBytes; i += kWave) {
            const int pos = i - kGenSeqOff;
            lds->s8[i] = (pos >= 0 && pos < L) ? (int8_t)(1 - 2 * (int)bit(pos)) : (int8_t)0;
        }
        int32_t sbit[G];
#pragma unroll
        for (int g = 0; g < G; g++) {
            const int j = lane + 64 * g;
            sbit[g] = (j < n) ? (int32_t)bit(j) : 0;
            mult[g] = j < n ? 8 * sbit[g] - 4 : 0;
        }
        int32_t sq = 0;
#pragma unroll
        for (int q = 0; q < QR; q++) {
            const int k = lane + 64 * q + 1;
            int32_t Ck = 0;
            if (k < L) {
                const int cnt = L - k;
                int diff = 0;
                for (int w = 0; 32 * w < cnt; w++) {
                    const uint32_t base = lds->fw[w];
                    const uint32_t shifted = funnel(lds->fw[(k >> 5) + w + 1], lds->fw[(k >> 5) + w], k & 31);
                    diff += popc((base ^ shifted) & low_mask(cnt - 32 * w));
                }
                Ck = cnt - 2 * diff;
            }
            Cv[q] = Ck;
            sq += Ck * Ck;
        }
        isl = wave_sum_i32(sq);
        uint64_t hz = 0;
#pragma unroll
        for (int g = 0; g < G; g++) {
            const int j = lane + 64 * g;
            if (j < n && sbit[g])
                hz ^= zk[j];
        }
        h = wave_xor_u64(hz);
    }

    // C to LDS, prefix sums, number of bit planes.
    __device__ __forceinline__ void prepare()
    {
        const int lane = this->lane;
        int32_t running = 0;
        uint32_t mag = 0;
#pragma unroll
        for (int q = 0; q < QR; q++) {
            const int k = lane + 64 * q + 1;
            lds->C[k] = Cv[q];
            const int32_t inc = wave_inclusive_scan(Cv[q]) + running;
            lds->psx[k] = inc;
            running = readlane_i(inc, 63);
            mag |= (uint32_t)(Cv[q] ^ (Cv[q] >> 31));
        }
        if (lane == 0)
            lds->psx[0] = 0;
        mag = wave_or_u32(mag);
        planes = (mag == 0) ? 1 : 33 - __builtin_clz(mag);
        lds_fence();
    }

    __device__ __forceinline__ void score(int32_t (&isl_j)[G])
    {
        const int lane = this->lane;
        // static window word counts of flip group g: p covers k <= L-1-j, q covers k <= j
        constexpr int PWg[3] = {KW, KW - 2 > 0 ? KW - 2 : 0, KW - 4 > 0 ? KW - 4 : 0};
        constexpr int QWg[3] = {KW < 2 ? KW : 2, KW < 4 ? KW : 4, KW < 6 ? KW : 6};
        uint32_t wp[G][KW], wq[G][KW];
#pragma unroll
        for (int g = 0; g < G; g++) {
            const int j = min(lane + 64 * g, n - 1);
            const int a0 = j + 1;
            const int b0 = kGenRV - j + 1;
            uint32_t lo = lds->fw[a0 >> 5];
#pragma unroll
            for (int w = 0; w < PWg[g]; w++) {
                const uint32_t hi = lds->fw[(a0 >> 5) + w + 1];
                wp[g][w] = funnel(hi, lo, a0 & 31);
                lo = hi;
            }
            lo = lds->rv[b0 >> 5];
#pragma unroll
            for (int w = 0; w < QWg[g]; w++) {
                const uint32_t hi = lds->rv[(b0 >> 5) + w + 1];
                wq[g][w] = funnel(hi, lo, b0 & 31);
                lo = hi;
            }
        }
        int32_t acc[G];
        {
            uint32_t pl[KW];
#pragma unroll
            for (int q = 0; q < QR; q++) {
                const uint64_t m = ballot(Cv[q] < 0);
                pl[2 * q] = (uint32_t)m;
                if (2 * q + 1 < KW)
                    pl[2 * q + 1] = (uint32_t)(m >> 32);
            }
#pragma unroll
            for (int g = 0; g < G; g++) {
                uint32_t s = 0;
#pragma unroll
                for (int w = 0; w < PWg[g]; w++)
                    s = bcnt_acc(pl[w] & wp[g][w], s);
#pragma unroll
                for (int w = 0; w < QWg[g]; w++)
                    s = bcnt_acc(pl[w] & wq[g][w], s);
                acc[g] = -(int32_t)s;
            }
        }
        for (int t = planes - 2; t >= 0; t--) {
            uint32_t pl[KW];
#pragma unroll
            for (int q = 0; q < QR; q++) {
                const uint64_t m = ballot(((Cv[q] >> t) & 1) != 0);
                pl[2 * q] = (uint32_t)m;
                if (2 * q + 1 < KW)
                    pl[2 * q + 1] = (uint32_t)(m >> 32);
            }
#pragma unroll
            for (int g = 0; g < G; g++) {
                uint32_t s = (uint32_t)acc[g] << 1;
#pragma unroll
                for (int w = 0; w < PWg[g]; w++)
                    s = bcnt_acc(pl[w] & wp[g][w], s);
#pragma unroll
                for (int w = 0; w < QWg[g]; w++)
                    s = bcnt_acc(pl[w] & wq[g][w], s);
                acc[g] = (int32_t)s;
            }
        }
#pragma unroll
        for (int g = 0; g < G; g++) {
            const int j = min(lane + 64 * g, n - 1);
            const int np = L - 1 - j, nq = j, m = min(np, nq);
            const int RW = PWg[g] < QWg[g] ? PWg[g] : QWg[g];
            uint32_t rc = 0;
#pragma unroll
            for (int w = 0; w < RW; w++)
                rc = bcnt_acc((wp[g][w] ^ wq[g][w]) & low_mask(m - 32 * w), rc);
            // ISL - 4 s_j G_j + 4 H_j with H_j = (L-1) + 2 (m - 2 rc); |G_j| <= L^2: 24-bit products
            const int32_t Gj = lds->psx[np] + lds->psx[nq] - 2 * acc[g];
            isl_j[g] = mad24(mult[g], Gj, mad24((int32_t)rc, -16, isl + 4 * (L - 1) + 8 * m));
        }
    }

    // Commit flip js (uniform): C_k += dC_k, bit strings, x, hash.
    template <bool REG_X = true>
    __device__ __forceinline__ void commit(int js, int32_t isl_new)
    {
        const int lane = this->lane;
        const uint32_t bjs = REG_X ? xbit_uniform(x, js) : sbit_of(js);
        // dC_k = -2 s_js (s_{js+k} + s_{js-k}), read from the zero-padded sequence bytes (so
        // shifts past either end add nothing)
        const int32_t fct = bjs ? 2 : -2;
        const int8_t *pb = lds->s8 + kGenSeqOff + js + 1 + lane;
        const int8_t *qb = lds->s8 + kGenSeqOff + js - 1 - lane;
#pragma unroll
        for (int q = 0; q < QR; q++)
            Cv[q] = mad24_u((int32_t)pb[64 * q] + (int32_t)qb[-64 * q], fct, Cv[q]);
        lds_fence();
        if (lane == 0) {
            lds->fw[js >> 5] ^= 1u << (js & 31);
            lds->s8[kGenSeqOff + js] = (int8_t)(-lds->s8[kGenSeqOff + js]);
        }
        if (lane == 1) {
            const int a = kGenRV - js;
            lds->rv[a >> 5] ^= 1u << (a & 31);
        }
        lds_fence();
#pragma unroll
        for (int g = 0; g < G; g++)
            mult[g] = (lane + 64 * g == js) ? -mult[g] : mult[g];
        if (REG_X)
            xflip_uniform(x, js);
        x0 ^= js < 32 ? 1u << js : 0u;
        if (REG_X) { // else the caller sets h (it has the neighbour's hash from its probe)
            const uint64_t z = zk[js];
            h ^= ((uint64_t)uniform((uint32_t)(z >> 32)) << 32) | uniform((uint32_t)z);
        }
        isl = isl_new;
    }
};

template <int SHAPE> struct GenShape;
template <> struct GenShape<0> { static constexpr int G = 1, KW = 1; }; //        L <= 33
template <> struct GenShape<1> { static constexpr int G = 1, KW = 2; }; //  34 <= L <= 64
template <> struct GenShape<2> { static constexpr int G = 2, KW = 2; }; //        L == 65
template <> struct GenShape<3> { static constexpr int G = 2, KW = 3; }; //  66 <= L <= 97
template <> struct GenShape<4> { static constexpr int G = 2, KW = 4; }; //  98 <= L <= 128
template <> struct GenShape<5> { static constexpr int G = 3, KW = 4; }; //        L == 129
template <> struct GenShape<6> { static constexpr int G = 3, KW = 5; }; // 130 <= L <= 161
template <> struct GenShape<7> { static constexpr int G = 3, KW = 6; }; // 162 <= L <= 192

template <int SHAPE>
__global__ void __launch_bounds__(64) k_walk_general(WalkState *__restrict__ states, int32_t count,
                                                     const int32_t *__restrict__ order, uint64_t *__restrict__ tables,
                                                     int32_t *__restrict__ trace, int32_t *__restrict__ scores)
{
    __shared__ uint64_t zk[kNMax];
    __shared__ WaveLdsGen lds;
    fill_zobrist(zk);
    const int idx = (int)blockIdx.x;
    if (idx >= count)
        return;
    using W = GenWalker<GenShape<SHAPE>::G, GenShape<SHAPE>::KW>;
    run_walk<W, 2>(&states[order[idx]], tables, trace, scores, 0, &lds, zk);
}

} // namespace

int general_shape_for_length(int L)
{
    if (L <= 33) return 0;
    if (L <= 64) return 1;
    if (L == 65) return 2;
    if (L <= 97) return 3;
    if (L <= 128) return 4;
    if (L == 129) return 5;
    if (L <= 161) return 6;
    return 7;
}

hipError_t launch_walk_general(int shape, WalkState *states, int32_t count, const int32_t *order, uint64_t *tables,
                               int32_t *trace, int32_t *scores, hipStream_t stream)
{
    if (count <= 0)
        return hipSuccess;
    const dim3 grid((unsigned)count), block(64);
    switch (shape) {
    case 0: hipLaunchKernelGGL(k_walk_general<0>, grid, block, 0, stream, states, count, order, tables, trace, scores); break;
    case 1: hipLaunchKernelGGL(k_walk_general<1>, grid, block, 0, stream, states, count, order, tables, trace, scores); break;
    case 2: hipLaunchKernelGGL(k_walk_general<2>, grid, block, 0, stream, states, count, order, tables, trace, scores); break;
    case 3: hipLaunchKernelGGL(k_walk_general<3>, grid, block, 0, stream, states, count, order, tables, trace, scores); break;
    case 4: hipLaunchKernelGGL(k_walk_general<4>, grid, block, 0, stream, states, count, order, tables, trace, scores); break;
    case 5: hipLaunchKernelGGL(k_walk_general<5>, grid, block, 0, stream, states, count, order, tables, trace, scores); break;
    case 6: hipLaunchKernelGGL(k_walk_general<6>, grid, block, 0, stream, states, count, order, tables, trace, scores); break;
    case 7: hipLaunchKernelGGL(k_walk_general<7>, grid, block, 0, stream, states, count, order, tables, trace, scores); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

} // namespace liblabs
