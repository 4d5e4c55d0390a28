// gen_walk.hip -- the self-avoiding walk over general (not skew-symmetric) sequences: the
// unrestricted problem that the skew-symmetric restriction of Section 1 reduces.  All L symbols
// are free, a flip negates one symbol, and every shift k = 1 .. L-1 counts (odd ones included).
// The walk itself (table, probes, restarts, stop rules) is the skew walk's (run_walk); only the
// walker differs.  L <= 192 (the free bits of a state fill the same six 32-bit words).
//
// Scoring (from Eq. (1)): with s_i = 1 - 2 b_i and flip j,
//   dC_k = -2 s_j u_k,  u_k = p_k + q_k,  p_k = s_{j+k} [j+k <= L-1],  q_k = s_{j-k} [j-k >= 0],
//   ISL_j = sum_k (C_k + dC_k)^2 = ISL - 4 s_j G_j + 4 H_j,  G_j = sum_k C_k u_k,  H_j = sum_k u_k^2,
// with H_j = (L-1) + 2 R_j, R_j = sum_{k <= min(j, L-1-j)} s_{j+k} s_{j-k}.  G_j, a product of
// Hankel windows of the sequence with the correlation table, runs on the matrix cores (see
// GenMfmaWalker); R_j is kept per flip across commits.
//
// Lane l owns flips j = l + 64 g (g < G = ceil(L/64)) and shifts k = l + 64 q + 1 (q < 3).
#include <hip/hip_runtime.h>

#include <cstddef>

#include "mfma_walker.hpp"
#include "walk_impl.hpp"

namespace liblabs {

namespace {

constexpr int kGenLMax = kXWords * 32; // 192
constexpr int kGenWords = 16;          // bit-string words, zero padded past the sequence
constexpr int kGenRV = kGenLMax - 1;   // reversed string: s_{kGenRV - u} at byte u

// ---------------------------------------------------------------------------------------------
// Matrix-core walker for general sequences.  T_j = G_j = Y_j + Z_j with Y_j = sum_k C_k s_{j+k}
// and Z_j = sum_k C_k s_{j-k} (k = 1 .. L-1, s = 0 outside the sequence) is a product of Hankel
// windows of the sequence with a Toeplitz arrangement of C, as in the skew matrix-core walker:
// with B[t][nn] = C_{t-nn} (0 unless 1 <= t-nn <= L-1) and A[row][t] = S[t + 16 i + off],
// D[row][nn] = sum_k C_k S[k + nn + 16 i + off], i.e. Y at j = h + off (h = 16 i + nn) for the
// forward string SF[u] = s_u, and Z at j = 191 - off - h for the reversed string RV[u] = s_{191-u}.
// Lane l receives row 4 i + r, column nn with h = l, so the four kinds of the first tile give
//   Y_l, Y_{64+l}, Z_{63-l}, Z_{127-l}   (SF + 0, SF + 64, RV + 128, RV + 64)
// and the second tile (L > 128)  Y_{128+l}, Z_{191-l}   (SF + 128, RV + 0; two kinds unused):
// lane l owns flips l, 64 + l, 128 + l and takes their Z from lane 63 - l (one ds_bpermute each).
//   ISL_j = ISL - 4 s_j G_j + 4 H_j,  H_j = (L-1) + 2 R_j,  R_j = sum_{k <= min(j, L-1-j)} s_{j+k} s_{j-k},
// and R_j is kept per lane across commits: flipping s_js changes the one term of R_j (j != js)
// that holds s_js, by -2 s_js s_{2j-js} when 0 <= 2j-js <= L-1.  C beyond the int8 range is
// split as 64 hi + lo with a second pass, as in the skew walker.
constexpr int kGmSfPad = 192;  // zero bytes before s_0 in sf, so that s_{2j-js} needs no range test
constexpr int kGmStrBytes = 432; // string bytes the tiles read (offsets up to 128, 4 K blocks)
constexpr int kGmCopyBytes = 288; // one copy of C: byte 20 + k - r in copy r
struct alignas(16) WaveLdsGenMfma {
    uint32_t xw[kGenWords];   // bit a = b_a: the free bits (words 0 .. kXWords-1), zero padded
    uint32_t bestx[kXWords];  // free bits of the best state of the walk so far
    int32_t book[8];          // the walk loop's rarely updated bookkeeping
    uint8_t pad0[200];
    int8_t sf[kGmSfPad + kGmStrBytes]; // s_u at sf[kGmSfPad + u], 0 elsewhere
    uint8_t pad1[144];
    int8_t rv[kGmStrBytes];   // s_{191-u} at rv[u], 0 elsewhere
    uint32_t cb[4][kGmCopyBytes / 4];
};
// the A operands of a row group fall 64 bytes apart modulo 256 (distinct banks): SF at 0, RV at 64
static_assert((offsetof(WaveLdsGenMfma, sf) + kGmSfPad) % 256 == 0, "SF bank offset");
static_assert(offsetof(WaveLdsGenMfma, rv) % 256 == 64, "RV bank offset");
static_assert(offsetof(WaveLdsGenMfma, cb) % 16 == 0, "C copies aligned");

template <int G, int KB>
struct GenMfmaWalker {
    static constexpr int kG = G;
    static constexpr int QR = 3; // shifts k = lane + 64 q + 1
    using Lds = WaveLdsGenMfma;
    // K blocks of the first tile.  Its Y kinds (SF + off) read s at j + k <= L - 1, i.e. t <= L - 1,
    // and its Z kinds (RV + 128, RV + 64) read s at j - k >= 0 with j <= 127 - 16 i, i.e. t <= 127:
    // two blocks with one tile (L <= 128), three with two (L <= 192).  The second tile's Z kind
    // (RV + 0, j <= 191) reaches t <= L + 14 and keeps KB.
    static constexpr int KB1 = G <= 2 ? (KB < 2 ? KB : 2) : (KB < 3 ? KB : 3);

    int L, c, n;
    int lane;
    int32_t isl;
    uint64_t h;
    uint32_t x[kXWords]; // free bits; current only where commit<true> is used (else in lds->xw)
    uint32_t x0;         // free bits 0..31, always current
    int32_t Cv[QR];
    int32_t mult[G];     // -4 s_j (0 past the last flip)
    int32_t Rv[G];       // R_j of the owned flips
    int planes;          // 9 when some |C_k| > 127 (two passes), else 8
    Lds *lds;
    const uint64_t *zk;
    uint32_t ta, ta2, tb; // LDS addresses of this lane's A (tiles 1, 2) and B words of K block 0
    int32_t bsrc;         // ds_bpermute source of Z: lane 63 - lane

    __device__ __forceinline__ uint32_t *x_lds() const { return lds->xw; }
    __device__ __forceinline__ void sync_x_lds() {} // every commit keeps lds->xw current
    __device__ __forceinline__ uint32_t *best_lds() const { return lds->bestx; }
    __device__ __forceinline__ int32_t *book_lds() const { return lds->book; }

    __device__ __forceinline__ void set_length(int len)
    {
        L = len;
        n = len;
        c = -1;
    }

    __device__ __forceinline__ int flip(int g) const { return lane + 64 * g; }

    __device__ __forceinline__ void init_lanes(int ln)
    {
        const int nn = ln & 15, slice = ln >> 4;
        const int kind = ln & 3, ib = (ln & 15) >> 2;
        const uint32_t sf0 = (uint32_t)(uintptr_t)(lds->sf + kGmSfPad);
        const uint32_t rv0 = (uint32_t)(uintptr_t)lds->rv;
        const uint32_t w = 16u * (uint32_t)(slice + ib);
        ta = (kind == 0 ? sf0 : kind == 1 ? sf0 + 64u : kind == 2 ? rv0 + 128u : rv0 + 64u) + w;
        ta2 = (kind == 0 ? sf0 + 128u : kind == 1 ? rv0 : kind == 2 ? sf0 : rv0 + 128u) + w;
        const int r = (4 - (nn & 3)) & 3; // the copy whose window of C_{t0-nn ..} starts on a dword
        tb = (uint32_t)(uintptr_t)(reinterpret_cast<const int8_t *>(lds->cb[r]) + 20 + 16 * slice - nn - r);
        bsrc = (63 - ln) << 2;
        asm volatile("" : "+v"(ta), "+v"(ta2), "+v"(tb), "+v"(bsrc));
    }

    __device__ inline uint32_t bit(int i) const
    {
        if (i < 0 || i >= L)
            return 0u;
        return (lds->xw[i >> 5] >> (i & 31)) & 1u;
    }

    // Strings and C copies from x, C_k from scratch (Eq. (1)), ISL (Eq. (2)), R_j, Zobrist hash.
    __device__ __forceinline__ void rebuild()
    {
        const int lane = this->lane;
        x0 = x[0];
        if (lane < kGenWords) {
            uint32_t f = 0;
#pragma unroll
            for (int i = 0; i < kXWords; i++)
                f = (lane == i) ? x[i] : f;
            lds->xw[lane] = f;
        }
        for (int i = lane; i < 4 * (kGmCopyBytes / 4); i += kWave)
            lds->cb[i / (kGmCopyBytes / 4)][i % (kGmCopyBytes / 4)] = 0u;
        lds_fence();
        for (int i = lane; i < kGmSfPad + kGmStrBytes; i += kWave) {
            const int pos = i - kGmSfPad;
            lds->sf[i] = (pos >= 0 && pos < L) ? (int8_t)(1 - 2 * (int)bit(pos)) : (int8_t)0;
        }
        for (int i = lane; i < kGmStrBytes; i += kWave) {
            const int pos = kGenRV - i;
            lds->rv[i] = (pos >= 0 && pos < L) ? (int8_t)(1 - 2 * (int)bit(pos)) : (int8_t)0;
        }
        lds_fence();
        int32_t sbit[G];
#pragma unroll
        for (int g = 0; g < G; g++) {
            const int j = lane + 64 * g;
            sbit[g] = (j < n) ? (int32_t)bit(j) : 0;
            mult[g] = j < n ? 8 * sbit[g] - 4 : 0;
            int32_t r = 0;
            const int m = j < n ? min(L - 1 - j, j) : 0;
            const int8_t *sp = lds->sf + kGmSfPad + j;
            for (int k = 1; k <= m; k++)
                r += (int32_t)sp[k] * (int32_t)sp[-k];
            Rv[g] = r;
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
                    const uint32_t base = lds->xw[w];
                    const uint32_t shifted = funnel(lds->xw[(k >> 5) + w + 1], lds->xw[(k >> 5) + w], k & 31);
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

    // C bytes into the four shifted copies: part 0 C itself, part 1 its low six bits (0..63),
    // part 2 C >> 6 (-3..2 for |C| <= 191).
    __device__ __forceinline__ void put_c(int part)
    {
        int8_t *cp = reinterpret_cast<int8_t *>(lds->cb[0]) + 20 + 1 + lane;
#pragma unroll
        for (int q = 0; q < QR; q++) {
            const int32_t v = part == 0 ? Cv[q] : (part == 1 ? (Cv[q] & 63) : (Cv[q] >> 6));
#pragma unroll
            for (int r = 0; r < 4; r++)
                cp[64 * q + r * (kGmCopyBytes - 1)] = (int8_t)v;
        }
    }

    __device__ __forceinline__ void prepare()
    {
        bool wide = false;
#pragma unroll
        for (int q = 0; q < QR; q++)
            wide = wide || (uint32_t)(Cv[q] + 128) > 255u;
        planes = ballot(wide) != 0ull ? 9 : 8;
        put_c(0);
        if (planes > 8)
            put_c(1);
        lds_fence();
    }

    template <int NKB>
    __device__ __forceinline__ mfma_v4i tile(uint32_t a_addr) const
    {
        const lds_cv4 *ap4 = (const lds_cv4 *)(uintptr_t)a_addr;
        const lds_cu32 *bp = (const lds_cu32 *)(uintptr_t)tb;
        mfma_v4i a[NKB], b[NKB];
#pragma unroll
        for (int kb = 0; kb < NKB; kb++) {
            a[kb] = ap4[4 * kb];
            b[kb] = mfma_v4i{(int)bp[16 * kb], (int)bp[16 * kb + 1], (int)bp[16 * kb + 2], (int)bp[16 * kb + 3]};
        }
        mfma_v4i acc = {0, 0, 0, 0};
#pragma unroll
        for (int kb = 0; kb < NKB; kb++)
            acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[kb], b[kb], acc, 0, 0, 0);
        return acc;
    }

    template <int NKB>
    __device__ __forceinline__ mfma_v4i tile_all(uint32_t a_addr)
    {
        mfma_v4i d = tile<NKB>(a_addr);
        if (planes > 8) {
            put_c(2);
            lds_fence();
            const mfma_v4i hi = tile<NKB>(a_addr);
            d = d + hi * 64;
        }
        return d;
    }

    __device__ __forceinline__ void score(int32_t (&isl_j)[G])
    {
        int32_t base[G];
        const int32_t isl4 = isl + 4 * (L - 1);
#pragma unroll
        for (int g = 0; g < G; g++)
            base[g] = mad24(Rv[g], 8, isl4);
        const mfma_v4i d = tile_all<KB1>(ta);
        // |G_j| <= 2 L^2: 24-bit products
        isl_j[0] = mad24(mult[0], d[0] + __builtin_amdgcn_ds_bpermute(bsrc, d[2]), base[0]);
        if constexpr (G >= 2)
            isl_j[1] = mad24(mult[1], d[1] + __builtin_amdgcn_ds_bpermute(bsrc, d[3]), base[1]);
        if constexpr (G >= 3) {
            if (planes > 8) // the copies hold hi now: lo again for the second tile
                put_c(1);
            const mfma_v4i d2 = tile_all<KB>(ta2);
            isl_j[2] = mad24(mult[2], d2[0] + __builtin_amdgcn_ds_bpermute(bsrc, d2[1]), base[2]);
        }
    }

    // Commit flip js (uniform): C_k += dC_k, R_j, strings, x, hash.
    template <bool REG_X = true>
    __device__ __forceinline__ void commit(int js, int32_t isl_new)
    {
        const int lane = this->lane;
        const int ol = js & 63, slot = js >> 6;
        int32_t mj = __builtin_amdgcn_readlane(mult[0], ol);
#pragma unroll
        for (int g = 1; g < G; g++)
            mj = slot == g ? __builtin_amdgcn_readlane(mult[g], ol) : mj;
        const uint32_t bjs = mj > 0 ? 1u : 0u; // s_js = -1
        // dC_k = -2 s_js (s_{js+k} + s_{js-k}) and dR_j = -2 s_js s_{2j-js}, read from the
        // zero-padded strings (no range tests)
        const int32_t fct = bjs ? 2 : -2;
        const int8_t *pb = lds->sf + kGmSfPad + js + 1 + lane;
        const int8_t *qb = lds->rv + kGenRV - js + 1 + lane;
#pragma unroll
        for (int q = 0; q < QR; q++)
            Cv[q] = mad24_u((int32_t)pb[64 * q] + (int32_t)qb[64 * q], fct, Cv[q]);
#pragma unroll
        for (int g = 0; g < G; g++) {
            const int j = lane + 64 * g;
            const int32_t v = (int32_t)lds->sf[kGmSfPad + 2 * j - js];
            Rv[g] = j != js ? mad24_u(v, fct, Rv[g]) : Rv[g];
        }
        lds_fence();
        // lane 0: the byte of s_js in sf and the free bit; lane 1: the byte in rv (0x01 and 0xFF
        // swap under xor 0xFE); the free-bit toggle uses a lane-varying word address
        if (lane < 2) {
            const int b = lane == 0 ? (int)offsetof(WaveLdsGenMfma, sf) + kGmSfPad + js
                                    : (int)offsetof(WaveLdsGenMfma, rv) + kGenRV - js;
            atomicXor(reinterpret_cast<uint32_t *>(lds) + (b >> 2), 0xFEu << (8 * (b & 3)));
            atomicXor(&lds->xw[(js >> 5) ^ lane], lane == 0 ? 1u << (js & 31) : 0u);
        }
        lds_fence();
        const bool own = lane == ol;
#pragma unroll
        for (int g = 0; g < G; g++)
            mult[g] = (own && slot == g) ? -mult[g] : mult[g];
        if (REG_X)
            xflip_uniform(x, js);
        x0 ^= js < 32 ? 1u << js : 0u;
        if (REG_X) {
            const uint64_t z = zk[js];
            h ^= ((uint64_t)uniform((uint32_t)(z >> 32)) << 32) | uniform((uint32_t)z);
        }
        isl = isl_new;
    }
};

// shapes: G flip groups of 64, KB K blocks of 64 shifts (t = k + nn <= L + 14 < 64 KB)
template <int SHAPE> struct GenShape;
template <> struct GenShape<0> { static constexpr int G = 1, KB = 1; }; //        L <= 33
template <> struct GenShape<1> { static constexpr int G = 1, KB = 2; }; //  34 <= L <= 64
template <> struct GenShape<2> { static constexpr int G = 2, KB = 2; }; //        L == 65
template <> struct GenShape<3> { static constexpr int G = 2, KB = 2; }; //  66 <= L <= 97
template <> struct GenShape<4> { static constexpr int G = 2, KB = 3; }; //  98 <= L <= 128
template <> struct GenShape<5> { static constexpr int G = 3, KB = 3; }; //        L == 129
template <> struct GenShape<6> { static constexpr int G = 3, KB = 3; }; // 130 <= L <= 161
template <> struct GenShape<7> { static constexpr int G = 3, KB = 4; }; // 162 <= L <= 192

template <int SHAPE>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(8)))
    k_walk_general(WalkState *__restrict__ states, int32_t count, const int32_t *__restrict__ order,
                   uint64_t *__restrict__ tables, int32_t *__restrict__ trace, int32_t *__restrict__ scores)
{
    __shared__ uint64_t zk[kNMax];
    __shared__ WaveLdsGenMfma lds;
    fill_zobrist(zk);
    const int idx = (int)blockIdx.x;
    if (idx >= count)
        return;
    using W = GenMfmaWalker<GenShape<SHAPE>::G, GenShape<SHAPE>::KB>;
    run_walk<W, 2>(&states[order[idx]], tables, trace, scores, 0, &lds, zk);
}

// ISL_j of every flip of a batch of states (free bits, kXWords words per state), out[r * L + j]
template <int SHAPE>
__global__ void __launch_bounds__(64) k_general_flip_scores(int L, int count, const uint32_t *__restrict__ xs,
                                                            int32_t *__restrict__ out)
{
    __shared__ uint64_t zk[kNMax];
    __shared__ WaveLdsGenMfma lds;
    fill_zobrist(zk);
    const int r = (int)blockIdx.x;
    if (r >= count)
        return;
    using W = GenMfmaWalker<GenShape<SHAPE>::G, GenShape<SHAPE>::KB>;
    W w;
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
    int32_t isl_j[W::kG];
    w.score(isl_j);
#pragma unroll
    for (int g = 0; g < W::kG; g++) {
        const int j = w.flip(g);
        if (j < w.n)
            out[(int64_t)r * w.n + j] = isl_j[g];
    }
}

} // namespace

hipError_t launch_general_flip_scores(int L, int count, const uint32_t *x, int32_t *scores, hipStream_t stream)
{
    if (count <= 0)
        return hipSuccess;
    void (*k)(int, int, const uint32_t *, int32_t *) = nullptr;
    switch (general_shape_for_length(L)) {
    case 0: k = k_general_flip_scores<0>; break;
    case 1: k = k_general_flip_scores<1>; break;
    case 2: k = k_general_flip_scores<2>; break;
    case 3: k = k_general_flip_scores<3>; break;
    case 4: k = k_general_flip_scores<4>; break;
    case 5: k = k_general_flip_scores<5>; break;
    case 6: k = k_general_flip_scores<6>; break;
    case 7: k = k_general_flip_scores<7>; break;
    default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k, dim3(count), dim3(64), 0, stream, L, count, x, scores);
    return hipGetLastError();
}

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
