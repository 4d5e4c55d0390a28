// walk_impl.hpp -- the gfx950 kernels of the skew-symmetric self-avoiding walk
// (Section 3, Algorithm 1 of Brest & Boskovic, arXiv:2011.00068, in its self-avoiding-walk
// reading) and of the batched one-flip evaluation.
//
// Mapping: one walk per 64-lane wavefront.  Lane l owns the flips j = l + 64 g (g < G flip
// groups) and the even shifts k = 2 kappa + 2 with kappa = l + 64 q.  All walk state lives in
// registers and a per-wave LDS block; HBM holds only the walk's visited table and its resume
// record.  Everything is int32 / uint32 / uint64 integer arithmetic, bit-exact.
//
// Scoring (the one-flip evaluation, derived from Eq. (1) and (4)).  With s_i = 1 - 2 b_i, L =
// 2c + 1, flip j < c negating s_j and s_m (m = L-1-j), and d = m - j:
//   dC_k = -4 s_j u_jk,  u_jk = p_k + q_k - [k = d] p_k,
//   p_k = s_{j+k} [j+k <= L-1],  q_k = s_{j-k} [j-k >= 0],
// and for the centre j = c: u_ck = q_k.  The flipped ISL is
//   ISL_j = sum_k (C_k + dC_k)^2 = ISL - 8 s_j G_j + 16 H_j,
//   G_j = sum_k C_k u_jk,  H_j = sum_k u_jk^2.
// Two variants compute it:
//  * BITSLICE: C is held as P two's-complement bit planes (P = bits of max |C_k|, one ballot
//    per plane; the two lowest planes are constant, since every even-shift correlation of a
//    skew sequence is congruent to L mod 4) and the sequence as bit strings split by index
//    parity; the windows
//    Wp[kappa] = b_{j+k}, Wq[kappa] = b_{j-k} are funnel shifts of those strings, so
//      sum_kappa C_kappa (Wp + Wq) = sum_t w_t [popc(plane_t & Wp) + popc(plane_t & Wq)],
//    and with prefix sums of C (PSX) over the valid shifts
//      G_j = PSX[np] + PSX[nq] - 2 sum C (Wp + Wq) - C_d s_m,
//      H_j = np + nq + 2 R_j - 1 - 2 s_m q_d,  R_j = sum_{k <= j} s_{j+k} s_{j-k},
//    where np / nq count the valid p / q shifts.  The centre uses G = PSX[nq] - 2 sum C Wq and
//    H = nq.
//  * DIRECT: the sequence as int8 in LDS (zero padded), C as int32 in LDS, and the sum of
//    (C_k - 4 s_j u_jk)^2 accumulated term by term, with the k = d term fixed up afterwards.
// Both keep that zero-padded int8 copy of the sequence: the commit reads p_k and q_k from it
// (so shifts past either end need no test), and the bit-sliced assembly reads q_d from it.

#pragma once

#include <type_traits>

#include "internal.hpp"

namespace liblabs {

// ---------------------------------------------------------------------------------------------
// Per-wave LDS block.
// ---------------------------------------------------------------------------------------------
constexpr int kSeqOff = 384;   // s_i stored at s8[kSeqOff + i]
constexpr int kSeqBytes = 1280; // zero padding on both sides covers every j +- k

struct WaveLdsBits {
    uint32_t par[2][kParWords]; // bit a of par[p] = b_{2a+p} (0 past the sequence end)
    uint32_t rev[2][kRevWords]; // bit a of rev[p] = bit (kNA-1-a) of par[p], 0 past kNA-1
    uint32_t xw[kXWords];       // free bits (kept current by every commit)
    uint32_t bestx[kXWords];    // free bits of the best state of the walk so far
    int32_t book[8];            // the walk loop's rarely updated bookkeeping
    int32_t C[kCMax + 1];       // C_{2 kappa + 2} at index kappa (0 for kappa >= c)
    int32_t psx[kCMax + 2];     // psx[a] = sum_{kappa < a} C
    int8_t s8[kSeqBytes];       // s_i at kSeqOff + i, 0 elsewhere
};

// both variants keep the same block (the direct one scores from s8, the bit-sliced one commits
// from it)
using WaveLdsDirect = WaveLdsBits;
template <bool DIRECT> struct LdsOf { using type = WaveLdsBits; };

// A walker's commit split into a read part and an apply part (CommitRead, see the matrix-core
// walker), or none.
struct NoCommitRead {};
template <class W, class = void> struct CommitReadOf {
    using type = NoCommitRead;
    static constexpr bool value = false;
};
template <class W> struct CommitReadOf<W, std::void_t<typename W::CommitRead>> {
    using type = typename W::CommitRead;
    static constexpr bool value = W::kSpecRead;
};

// Whether a walker's step loop gives its commit phase issue priority over its scoring phase
// (W::kIssuePrio, default no).  With many waves per SIMD, a wave whose probe is out then finishes
// its commit ahead of waves that are still scoring; measured faster for the full-GPU L = 255
// batch (2.6 %), slower with few waves per SIMD or mixed shapes in one launch (1.3 %).
template <class W, class = void> struct IssuePrioOf {
    static constexpr bool value = false;
};
template <class W> struct IssuePrioOf<W, std::void_t<decltype(W::kIssuePrio)>> {
    static constexpr bool value = W::kIssuePrio;
};

__device__ inline void lds_fence() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront"); __builtin_amdgcn_wave_barrier(); }

// ---------------------------------------------------------------------------------------------
// Uniform helpers on free-bit vectors held as kXWords uniform words.
// ---------------------------------------------------------------------------------------------
__device__ inline uint32_t xbit_uniform(const uint32_t (&x)[kXWords], int j)
{
    uint32_t w = 0;
#pragma unroll
    for (int i = 0; i < kXWords; i++)
        w = (i == (j >> 5)) ? x[i] : w;
    return (w >> (j & 31)) & 1u;
}

__device__ inline void xflip_uniform(uint32_t (&x)[kXWords], int j)
{
#pragma unroll
    for (int i = 0; i < kXWords; i++)
        x[i] ^= (i == (j >> 5)) ? (1u << (j & 31)) : 0u;
}

// Start state of restart r (SplitMix64 words, bit j of x = bit j%64 of word j/64, j < n).
__device__ inline void start_bits(uint64_t seed, uint32_t walk_id, uint32_t restart, int n,
                                  uint32_t (&x)[kXWords])
{
    const uint64_t kw = sm_at(seed, walk_id);
    const uint64_t kr = sm_at(kw, restart);
#pragma unroll
    for (int w = 0; w < kXWords / 2; w++) {
        uint64_t v = sm_at(kr, (uint64_t)w);
        const int lo = 64 * w;
        if (lo >= n)
            v = 0;
        else if (n - lo < 64)
            v &= (1ull << (n - lo)) - 1ull;
        // the words are wave-uniform; keep them in scalar registers
        x[2 * w] = uniform((uint32_t)v);
        x[2 * w + 1] = uniform((uint32_t)(v >> 32));
    }
}

// ---------------------------------------------------------------------------------------------
// Per-lane constants of the bit-sliced scoring of one flip j (they depend only on L and j, so a
// walk computes them once and keeps them in registers; the per-step work then reads them).
// ---------------------------------------------------------------------------------------------
struct FlipConst {
    const uint32_t *wp; // par[j&1] word holding bit hj+1 (start of the p window)
    const uint32_t *wq; // rev[j&1] word holding bit kNA-hj (start of the q window)
    uint32_t sp;        // p-window shift hj+1; the q-window shift kNA-hj = 1 - sp (mod 32)
    const int32_t *psx_np, *psx_nq; // PSX at the counts of valid p / q shifts
    const int32_t *c_kd;            // C at the excluded shift d = L-1-2j (a zero word for the centre)
    const int8_t *qd;               // s_{j-d} (a zero byte where j - d < 0 and for the centre)
    int32_t hc;                     // np + 3 nq - 1 (H_j without the data-dependent terms); nq
                                    // for the centre
    int32_t nq;                     // valid q shifts: floor(j/2)
};

// ---------------------------------------------------------------------------------------------
// The walker: one wave's view of one walk.
//   G  = flip groups (n <= 64 G), KW = 32-bit words of a shift window (c <= 32 KW).
// ---------------------------------------------------------------------------------------------
template <int G, int KW, bool DIRECT>
struct Walker {
    static constexpr int kG = G;
    static constexpr int QR = (KW + 1) / 2; // lane-held C registers: kappa = lane + 64 q
    using Lds = typename LdsOf<DIRECT>::type;

    int L, c, n;
    int lane; // lane id, laundered every step so that lane-derived values are recomputed
    int32_t isl;
    uint64_t h;
    uint32_t x[kXWords]; // free bits; current only where commit<true> is used (else in lds->xw)
    uint32_t x0;         // free bits 0..31, always current (they address the exact table)
    int32_t Cv[QR];
    int32_t mult[G];  // factor of T_j (see score()): -8 s_j, -4 s_c for the centre, 0 past it
    int32_t eps8;     // 8 (-1)^(c-j) for this lane's flips (the parity of j - lane is even)
    int planes;
    Lds *lds;
    const uint64_t *zk;
    FlipConst fc[G];

    __device__ __forceinline__ void set_length(int len)
    {
        L = len;
        c = (L - 1) / 2;
        n = c + 1;
    }

    // flip scored in slot g of this lane
    __device__ __forceinline__ int flip(int g) const { return lane + 64 * g; }
    // the lane and the slot g that own flip j
    __device__ __forceinline__ static int owner_lane(int j) { return j & 63; }
    __device__ __forceinline__ static int owner_slot(int j) { return j >> 6; }

    // LDS copies of the current and of the best free bits
    __device__ __forceinline__ uint32_t *x_lds() const { return lds->xw; }
    __device__ __forceinline__ uint32_t *best_lds() const { return lds->bestx; }
    __device__ __forceinline__ int32_t *book_lds() const { return lds->book; }
    __device__ __forceinline__ void sync_x_lds() {} // every commit keeps lds->xw current

    // b_js (uniform) from the lane that scores flip js: mult > 0 iff s_js = -1
    __device__ __forceinline__ uint32_t sbit_of(int js) const
    {
        int32_t v = 0;
#pragma unroll
        for (int g = 0; g < G; g++)
            v = (g == (js >> 6)) ? __builtin_amdgcn_readlane(mult[g], js & 63) : v;
        return v > 0 ? 1u : 0u;
    }

    __device__ __forceinline__ void init_lanes(int ln)
    {
        eps8 = ((c - ln) & 1) ? -8 : 8;
        if constexpr (!DIRECT)
            setup_lanes(ln);
    }

    // Per-lane constants of the owned flips (bit-sliced variant).
    __device__ __forceinline__ void setup_lanes(int ln)
    {
#pragma unroll
        for (int g = 0; g < G; g++) {
            const int j = min(ln + 64 * g, c);
            const int p = j & 1, hj = j >> 1;
            const int nq = hj;
            const int np = c - ((j + 1) >> 1);
            FlipConst &f = fc[g];
            f.sp = (uint32_t)(hj + 1);
            f.wp = &lds->par[p][(hj + 1) >> 5];
            f.wq = &lds->rev[p][(kNA - hj) >> 5];
            f.psx_np = &lds->psx[np];
            f.psx_nq = &lds->psx[nq];
            f.nq = nq;
            if (j < c) {
                f.c_kd = &lds->C[c - 1 - j];
                f.qd = &lds->s8[kSeqOff + 3 * j - 2 * c]; // s_{j-d}, j - d = 3j - 2c >= -2c
                f.hc = np + 3 * nq - 1;
            } else { // the centre (and the unused slots past it)
                f.c_kd = &lds->C[c];
                f.qd = &lds->s8[0];
                f.hc = nq;
            }
        }
    }

    // b_i of the full sequence (Eq. (4) mirror for i > c), read from the LDS copy of x.
    __device__ inline uint32_t seq_bit(int i) const
    {
        if (i < 0 || i >= L)
            return 0u;
        const int f = (i <= c) ? i : 2 * c - i;
        const uint32_t b = (lds->xw[f >> 5] >> (f & 31)) & 1u;
        return (i <= c) ? b : (b ^ (uint32_t)((i - c) & 1));
    }

    // Rebuild everything derived from x: bit strings, C_k from scratch (Eq. (1)), ISL (Eq. (2)),
    // Zobrist hash.
    __device__ __forceinline__ void rebuild()
    {
        const int lane = this->lane;
        x0 = x[0];
        if (lane == 0) {
#pragma unroll
            for (int w = 0; w < kXWords; w++)
                lds->xw[w] = x[w];
        }
        lds_fence();
        // parity strings and their reversals, 64 bit positions per ballot
#pragma unroll
        for (int r = 0; r < 3; r++) {
            const int a = lane + 64 * r;
            const int ar = kNA - 1 - a;
#pragma unroll
            for (int p = 0; p < 2; p++) {
                const uint64_t m = ballot(seq_bit(2 * a + p) != 0u);
                const uint64_t mr = ballot(seq_bit(2 * ar + p) != 0u);
                if (lane == 0) {
                    lds->par[p][2 * r] = (uint32_t)m;
                    lds->par[p][2 * r + 1] = (uint32_t)(m >> 32);
                    lds->rev[p][2 * r] = (uint32_t)mr;
                    lds->rev[p][2 * r + 1] = (uint32_t)(mr >> 32);
                }
            }
        }
        if (lane < 2 * (kParWords - 6)) {
            lds->par[lane & 1][6 + (lane >> 1)] = 0u;
        }
        if (lane < 2 * (kRevWords - 6)) {
            lds->rev[lane & 1][6 + (lane >> 1)] = 0u;
        }
        for (int i = lane; i < kSeqBytes; i += kWave) {
            const int pos = i - kSeqOff;
            lds->s8[i] = (pos >= 0 && pos < L) ? (int8_t)(1 - 2 * (int)seq_bit(pos)) : (int8_t)0;
        }
        // prepare() writes C_kappa for kappa < 64 QR; the zero word C_c may lie past that
        for (int i = lane; i < kCMax + 1; i += kWave)
            lds->C[i] = 0;
        lds_fence();
        // per-lane free bits of the owned flips
        int32_t sbit[G];
#pragma unroll
        for (int g = 0; g < G; g++) {
            const int j = lane + 64 * g;
            sbit[g] = (j <= c) ? (int32_t)seq_bit(j) : 0;
            const int32_t sj = 1 - 2 * sbit[g];
            mult[g] = j < c ? -8 * sj : (j == c ? -4 * sj : 0);
        }
        // C_k for even k from the parity strings: pairs (i, i+k) share the parity of i, and
        // s_i s_{i+k} = 1 - 2 (b_i xor b_{i+k}).
        int32_t sq = 0;
#pragma unroll
        for (int q = 0; q < QR; q++) {
            const int kappa = lane + 64 * q;
            int32_t Ck = 0;
            if (kappa < c) {
                const int k = 2 * kappa + 2;
                const int sh = kappa + 1;
#pragma unroll
                for (int p = 0; p < 2; p++) {
                    const int last = L - 1 - k - p; // largest 2a with 2a + p + k <= L-1
                    const int cnt = last >= 0 ? last / 2 + 1 : 0;
                    int diff = 0;
                    for (int w = 0; 32 * w < cnt; w++) {
                        const uint32_t base = lds->par[p][w];
                        const uint32_t shifted =
                            funnel(lds->par[p][(sh >> 5) + w + 1], lds->par[p][(sh >> 5) + w], sh & 31);
                        diff += popc((base ^ shifted) & low_mask(cnt - 32 * w));
                    }
                    Ck += cnt - 2 * diff;
                }
            }
            Cv[q] = Ck;
            sq += Ck * Ck;
        }
        isl = wave_sum_i32(sq);
        uint64_t hz = 0;
#pragma unroll
        for (int g = 0; g < G; g++) {
            const int j = lane + 64 * g;
            if (j <= c && sbit[g])
                hz ^= zk[j];
        }
        h = wave_xor_u64(hz);
    }

    // Per-step preparation: C to LDS, prefix sums, number of bit planes.
    __device__ __forceinline__ void prepare()
    {
        const int lane = this->lane;
        int32_t running = 0;
        uint32_t mag = 0; // OR of |C| - [C < 0]: its bit length is the magnitude bits needed
#pragma unroll
        for (int q = 0; q < QR; q++) {
            const int kappa = lane + 64 * q;
            lds->C[kappa] = Cv[q];
            const int32_t inc = wave_inclusive_scan(Cv[q]) + running;
            lds->psx[kappa + 1] = inc;
            running = readlane_i(inc, 63);
            mag |= (uint32_t)(Cv[q] ^ (Cv[q] >> 31));
        }
        if (lane == 0)
            lds->psx[0] = 0;
        mag = wave_or_u32(mag);
        planes = (mag == 0) ? 1 : 33 - __builtin_clz(mag);
        lds_fence();
    }

    // Score every owned flip: isl_j[g] = ISL after flip j = lane + 64 g (garbage for j > c).
    __device__ __forceinline__ void score(int32_t (&isl_j)[G])
    {
        const int lane = this->lane;
        if constexpr (!DIRECT) {
            uint32_t wp[G][KW];
            uint32_t wq[G][G];
#pragma unroll
            for (int g = 0; g < G; g++) {
                const FlipConst &f = fc[g];
                uint32_t lo = f.wp[0];
#pragma unroll
                for (int w = 0; w < KW - g; w++) {
                    const uint32_t hi = f.wp[w + 1];
                    wp[g][w] = funnel(hi, lo, (int)f.sp);
                    lo = hi;
                }
                lo = f.wq[0];
#pragma unroll
                for (int w = 0; w <= g; w++) {
                    const uint32_t hi = f.wq[w + 1];
                    wq[g][w] = funnel(hi, lo, (int)(1u - f.sp));
                    lo = hi;
                }
            }
            // bit-plane sums, most significant (sign) plane first (Horner: acc = 2 acc + plane sum)
            int32_t acc[G];
            {
                uint32_t pl[KW];
#pragma unroll
                for (int q = 0; q < QR; q++) {
                    const uint64_t m = ballot(Cv[q] < 0); // sign plane = bit planes-1
                    pl[2 * q] = (uint32_t)m;
                    if (2 * q + 1 < KW)
                        pl[2 * q + 1] = (uint32_t)(m >> 32);
                }
#pragma unroll
                for (int g = 0; g < G; g++) {
                    uint32_t s = 0;
#pragma unroll
                    for (int w = 0; w < KW - g; w++)
                        s = bcnt_acc(pl[w] & wp[g][w], s);
#pragma unroll
                    for (int w = 0; w <= g; w++)
                        s = bcnt_acc(pl[w] & wq[g][w], s);
                    acc[g] = -(int32_t)s;
                }
            }
            // planes 2 .. P-2 from ballots; at least three planes, so that the sign plane is never
            // one of the two lowest
            for (int t = max(planes, 3) - 2; t >= 2; t--) {
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
                    for (int w = 0; w < KW - g; w++)
                        s = bcnt_acc(pl[w] & wp[g][w], s);
#pragma unroll
                    for (int w = 0; w <= g; w++)
                        s = bcnt_acc(pl[w] & wq[g][w], s);
                    acc[g] = (int32_t)s;
                }
            }
            // the two lowest planes are the same for every shift: a flip moves C_k by a multiple of
            // 4 and the flips connect every skew sequence of length L, so all even-shift
            // correlations are congruent mod 4 (to L), odd: bit 0 is set, bit 1 is set iff
            // L = 3 mod 4.  Their contribution is r * popcount(W) with r = L mod 4.
            {
                const int32_t r = L & 3;
#pragma unroll
                for (int g = 0; g < G; g++) {
                    uint32_t sw = 0;
#pragma unroll
                    for (int w = 0; w < KW - g; w++)
                        sw = bcnt_acc(wp[g][w], sw);
#pragma unroll
                    for (int w = 0; w <= g; w++)
                        sw = bcnt_acc(wq[g][w], sw);
                    acc[g] = (acc[g] << 2) + r * (int32_t)sw;
                }
            }
            // assemble ISL_j.  With T_j = PSX[np] + PSX[nq] - 2 acc = sum_k C_k (p_k + q_k) and
            // s_m = (-1)^(c-j) s_j:
            //   ISL_j = ISL - 8 s_j (T_j - s_m C_d) + 16 (hc - 4 rc - 2 s_m q_d)
            //         = ISL + 16 hc - 64 rc + 8 (-1)^(c-j) C_d - 8 s_j (T_j + 4 (-1)^(c-j) q_d).
            // For the centre, Wp equals Wq (Eq. (4) mirrors every even offset onto itself), so rc = 0,
            // T_c = 2 G_c, and with hc = nq, C_d = q_d = 0 and the factor -4 s_c the same
            // expression gives ISL - 8 s_c G_c + 16 nq: every flip is assembled without branches.
#pragma unroll
            for (int g = 0; g < G; g++) {
                const FlipConst &f = fc[g];
                // R_j = nq - 2 rc, rc = differing bits of Wp and Wq over the both-sided shifts
                uint32_t rc = 0;
#pragma unroll
                for (int w = 0; w < g; w++)
                    rc = bcnt_acc((w < KW - g ? wp[g][w] : 0u) ^ wq[g][w], rc);
                // nq lies in [32 g, 32 g + 31]: the low (nq - 32 g) bits of word g are both-sided
                const uint32_t rmask = (1u << (f.nq & 31)) - 1u;
                rc = bcnt_acc(((g < KW - g ? wp[g][g] : 0u) ^ wq[g][g]) & rmask, rc);
                const int32_t T = *f.psx_np + *f.psx_nq - 2 * acc[g];
                // |C_d| <= L, |T| <= L^2 / 2, factors within 8: 24-bit products
                const int32_t base = isl + 16 * f.hc - 64 * (int32_t)rc + __mul24(eps8, *f.c_kd);
                isl_j[g] = mad24(mult[g], mad24((int32_t)*f.qd, eps8 >> 1, T), base);
            }
        } else {
            // direct sum of squares over the even shifts
            const int8_t *s8 = lds->s8;
#pragma unroll
            for (int g = 0; g < G; g++) {
                const int j = lane + 64 * g;
                const int jc = min(j, c);
                const int32_t sj4 = 4 * (int32_t)s8[kSeqOff + jc];
                const int pbase = (jc == c) ? kSeqOff + L : kSeqOff + jc; // centre: p_k = 0
                const int qbase = kSeqOff + jc;
                int32_t acc = 0;
                for (int kappa = 0; kappa < c; kappa++) {
                    const int k = 2 * kappa + 2;
                    const int32_t u = (int32_t)s8[pbase + k] + (int32_t)s8[qbase - k];
                    const int32_t tt = lds->C[kappa] - sj4 * u;
                    acc += tt * tt;
                }
                if (jc < c) {
                    const int kd = c - 1 - jc;
                    const int d = 2 * kd + 2;
                    const int32_t qd = s8[qbase - d];
                    const int32_t wrong = lds->C[kd] - sj4 * ((int32_t)s8[pbase + d] + qd);
                    const int32_t right = lds->C[kd] - sj4 * qd;
                    acc += right * right - wrong * wrong;
                }
                isl_j[g] = acc;
            }
        }
    }

    // Commit flip js (uniform): update C_k by dC_k, the bit strings / sequence, the free bits
    // (lds->xw and x0; the register copy x and the hash as well when REG_X).
    template <bool REG_X = true>
    __device__ __forceinline__ void commit(int js, int32_t isl_new)
    {
        const int lane = this->lane;
        const uint32_t bjs = REG_X ? xbit_uniform(x, js) : sbit_of(js);
        const int hjs = js >> 1;
        const int pis = js & 1;
        const int nps = (js == c) ? 0 : c - ((js + 1) >> 1);
        const int kds = (js == c) ? -1 : c - 1 - js;
        // dC_k = -4 s_js (p_k + q_k) with p_k = s_{js+k}, q_k = s_{js-k} read from the zero-padded
        // sequence bytes (so lanes with kappa >= c add nothing), p without the excluded shift d;
        // at the centre p = q and u = q, so the factor is halved instead
        const int32_t fct = (js == c) ? (bjs ? 2 : -2) : (bjs ? 4 : -4);
        const int8_t *pb = lds->s8 + kSeqOff + js + 2 + 2 * lane;
        const int8_t *qb = lds->s8 + kSeqOff + js - 2 - 2 * lane;
#pragma unroll
        for (int q = 0; q < QR; q++) {
            const int32_t pv = (lane + 64 * q == kds) ? 0 : (int32_t)pb[128 * q];
            Cv[q] = mad24_u(pv + (int32_t)qb[-128 * q], fct, Cv[q]);
        }
        lds_fence();
        // lane 0: js, lane 1: the mirror m = 2c - js (half index nps); the free bit itself from
        // lane 0 (lane 1 xors 0 into a neighbouring word: a lane-varying address keeps the compiler from
        // turning the toggle into a cross-lane reduction)
        if (lane < (js != c ? 2 : 1)) {
            const int pos = lane ? 2 * c - js : js;
            lds->s8[kSeqOff + pos] = (int8_t)(-lds->s8[kSeqOff + pos]);
            if constexpr (!DIRECT) {
                const int a = lane ? nps : hjs;
                atomicXor(&lds->par[pis][a >> 5], 1u << (a & 31));
                const int ar = kNA - 1 - a;
                atomicXor(&lds->rev[pis][ar >> 5], 1u << (ar & 31));
            }
            atomicXor(&lds->xw[(js >> 5) ^ lane], lane == 0 ? 1u << (js & 31) : 0u);
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

// ---------------------------------------------------------------------------------------------
// Visited table access.  Probes are issued by a subset of lanes (divergent), so they are
// vector loads; stores are plain vector stores.
// ---------------------------------------------------------------------------------------------
// A launch advances a walk by at most this many steps (the per-launch counters are 32-bit).
constexpr int32_t kMaxStepsPerLaunch = (1 << 30);

__device__ inline void clear_table(uint64_t *T, int log2)
{
    const int lane = lane_id();
    uint4 *T4 = reinterpret_cast<uint4 *>(T);
    const int64_t n4 = (int64_t)1 << (log2 - 1);
    const uint4 z = make_uint4(0u, 0u, 0u, 0u);
    for (int64_t i = lane; i < n4; i += kWave)
        T4[i] = z;
}

__device__ inline uint64_t slot_of(uint64_t hh, uint32_t x0, bool exact, int log2)
{
    return exact ? (uint64_t)x0 : (hh >> (64 - log2));
}

// Table epochs.  A walk's table holds the entries of its current start (or restart) and stale
// ones of earlier starts; an entry written during epoch e is the word (h | 1) ^ (e << (64 - log2)),
// i.e. the state's entry with the epoch XORed into its top log2 bits.  A probe during epoch e
// compares with the same form, so a stale entry (epoch e' != e) can never match: in a hashed
// table the top log2 bits of h are the slot, equal for every state stored there, so the two words
// differ in e ^ e' there; in a table addressed by the free bits, a slot holds a single state and
// the words again differ in e ^ e'.  Nor does a cleared word (0) match: bit 0 of every expected
// word is set.  So a
// probe answers as it would in a table cleared at the start, and a start only takes the next
// epoch; the 2^log2 words are cleared when the epochs 1 .. 2^log2 - 1 have all been used, and
// when the table's contents are unknown (epoch 0: a walk state that has never run on it).  The
// slot comes from the hash alone; a probe XORs the tag into the word it expects while its load is
// in flight.
// The high word of the tag e << (64 - log2) (its low word is 0: log2 <= 30).
__device__ inline uint32_t epoch_tag_hi(uint32_t ep, int log2)
{
    return ep << (32 - log2);
}

// The epoch of a new start after epoch ep (clearing the table when none is left).
__device__ inline uint32_t next_epoch(uint64_t *T, int log2, uint32_t ep)
{
    if (ep == 0u || ep >= (1u << log2) - 1u) {
        clear_table(T, log2);
        return 1u;
    }
    return ep + 1u;
}

// ---------------------------------------------------------------------------------------------
// One walk, advanced until its budget, its target, or the launch's step limit.
// ---------------------------------------------------------------------------------------------
// TRACE = false: the walk records no trace and no scores, and the step loop carries no test for
// them.  EXACT: 1 / 0 when the table is known to be addressed by the free bits (n <= table_log2)
// / by the hash, -1 when the walk decides at run time (run_walk below picks the instantiation).
template <class W, int PW, bool TRACE, int EXACT = -1>
__device__ __forceinline__ void run_walk_impl(WalkState *__restrict__ wsp, uint64_t *__restrict__ tables,
                         int32_t *__restrict__ trace, int32_t *__restrict__ scores, int64_t chunk,
                         typename W::Lds *lds, const uint64_t *zk)
{
    constexpr int G = W::kG;
    int lane = lane_id();
    asm volatile("" : "+v"(lane)); // nothing lane-derived is hoisted out of the walk
    WalkState &ws = *wsp;

    const int32_t status0 = su(ws.status);
    if (status0 == kDone)
        return;

    W w;
    w.lane = lane;
    w.set_length(su(ws.L));
    w.lds = lds;
    w.zk = zk;
    w.init_lanes(lane);
    const int L = w.L, n = w.n;
    const int tlog2 = su(ws.table_log2);
    const bool exact = EXACT >= 0 ? EXACT != 0 : n <= tlog2;
    const uint64_t seed = su(ws.seed);
    const uint32_t walk_id = su(ws.walk_id);
    const int64_t steps = su(ws.steps);
    const int64_t R = su(ws.restart_period);
    const int64_t target = su(ws.target_isl);
    const int64_t watch = su(ws.watch_isl);
    uint64_t *T = tables + su(ws.table_offset);
    uint32_t ep = (uint32_t)su(ws.table_epoch); // the table's epoch (see epoch_tag_hi)
    uint32_t tag_hi = 0;
    const int64_t trace_off = su(ws.trace_offset);
    const int64_t score_off = su(ws.score_offset);

    int64_t t, flips, hit, wstep, best_isl, best_step;
    int32_t restart_idx, restarts, traps;
    // The free bits live in LDS during the walk (the walker's x_lds(), and best_lds() for the
    // best state), so that the hot loop keeps none of them in scalar registers.
    uint32_t *const xl = w.x_lds();
    uint32_t *const bl = w.best_lds();

    if (status0 == kFresh) {
        restart_idx = 0;
        start_bits(seed, walk_id, 0u, n, w.x);
        ep = next_epoch(T, tlog2, ep);
        tag_hi = epoch_tag_hi(ep, tlog2);
        w.rebuild();
        if (lane == 0)
            T[slot_of(w.h, w.x0, exact, tlog2)] = (w.h | 1ull) ^ ((uint64_t)tag_hi << 32);
        t = 0;
        flips = 0;
        restarts = 0;
        traps = 0;
        best_isl = w.isl;
        best_step = 0;
        if (lane < kXWords)
            bl[lane] = xl[lane];
        hit = (target >= 0 && w.isl <= target) ? 0 : -1;
        wstep = (watch >= 0 && w.isl <= watch) ? 0 : -1;
    } else {
#pragma unroll
        for (int i = 0; i < kXWords; i++)
            w.x[i] = su(ws.x[i]);
        if (lane < kXWords)
            bl[lane] = ws.best_x[lane];
        restart_idx = su(ws.restart_idx);
        restarts = su(ws.restarts);
        traps = su(ws.traps);
        t = su(ws.t);
        flips = su(ws.flips);
        hit = su(ws.hit_step);
        wstep = su(ws.watch_step);
        best_isl = su(ws.best_isl);
        best_step = su(ws.best_step);
        tag_hi = epoch_tag_hi(ep, tlog2);
        w.rebuild();
    }

    // Per-launch bookkeeping in 32-bit uniform registers (scalar compares): ts counts the steps
    // of this launch, rem the steps to the next multiple of R (a periodic restart).
    const int64_t t0 = t;
    const int64_t flips0 = flips;
    int64_t t_end = steps;
    if (chunk > 0 && t + chunk < t_end)
        t_end = t + chunk;
    const int64_t cap = su(ws.step_cap);
    if (cap < t_end)
        t_end = cap;
    const int32_t nsteps = (int32_t)max<int64_t>(0, min<int64_t>(t_end - t0, (int64_t)kMaxStepsPerLaunch));
    const int32_t tgt = target < 0 ? -1 : (int32_t)min<int64_t>(target, INT32_MAX);
    const int32_t wch = watch < 0 ? -1 : (int32_t)min<int64_t>(watch, INT32_MAX);
    const int32_t R32 = (int32_t)min<int64_t>(R, INT32_MAX);
    int32_t rem = (R > 0) ? (int32_t)min<int64_t>((t0 / R + 1) * R - t0, INT32_MAX) : INT32_MAX;
    const bool hit_found0 = hit >= 0;
    const bool watch_found0 = wstep >= 0;
    // The step loop runs while ts < lim; reaching the target sets lim = -1 (stopped).  The inner
    // loop below runs to lim_in, the earlier of lim and the next periodic restart.
    int32_t lim = (tgt >= 0 && hit_found0) ? -1 : nsteps;
    int32_t lim_in = lim;
    // A committed state needs bookkeeping only if its ISL is at most thr: a new best, or the target
    // or watch level not reached before.  That bookkeeping (rarely updated) lives in LDS, so the
    // step loop carries only thr and lim: book[0] best ISL, [1] its step in this launch, [2] / [3]
    // the steps that reached the target / watch level (-1: not in this launch), [4] / [5] whether
    // they have been reached.
    auto threshold = [&](int32_t best, bool hf, bool wf) -> int32_t {
        int32_t v = best - 1;
        if (tgt >= 0 && !hf)
            v = max(v, tgt);
        if (wch >= 0 && !wf)
            v = max(v, wch);
        return v;
    };
    int32_t thr = threshold((int32_t)best_isl, hit_found0, watch_found0);
    int32_t *const bk = w.book_lds();
    if (lane == 0) {
        bk[0] = (int32_t)best_isl;
        bk[1] = -1;
        bk[2] = -1;
        bk[3] = -1;
        bk[4] = hit_found0;
        bk[5] = watch_found0;
    }
    // A state occupied after step ts of this launch with ISL <= thr: update best / hit / watch
    // (uniform updates first, then one lane-0 store block, so that thr and lim stay scalar).
    // Committed states and restart states alike (a restart is the walk's initialisation again).
    auto note_state = [&](int32_t ts_at) {
        int32_t best = su(bk[0]);
        int32_t hf = su(bk[4]), wf = su(bk[5]);
        const bool nb = w.isl < best;
        const bool nh = tgt >= 0 && !hf && w.isl <= tgt;
        const bool nw = wch >= 0 && !wf && w.isl <= wch;
        best = nb ? w.isl : best;
        hf |= nh ? 1 : 0;
        wf |= nw ? 1 : 0;
        lim = nh ? -1 : lim;
        lim_in = nh ? -1 : lim_in;
        thr = su(threshold(best, hf != 0, wf != 0));
        if (nb) {
            w.sync_x_lds();
            if (w.lane < kXWords)
                bl[w.lane] = xl[w.lane];
        }
        if (w.lane == 0) {
            bk[0] = best;
            if (nb)
                bk[1] = ts_at;
            if (nh)
                bk[2] = ts_at;
            if (nw)
                bk[3] = ts_at;
            bk[4] = hf;
            bk[5] = wf;
        }
    };
    // steps left before the budget, as seen from this launch (periodic restarts stop there)
    const int32_t left32 = (int32_t)min<int64_t>(steps - t0, INT32_MAX);
    int32_t *trp = (TRACE && trace_off >= 0) ? trace + 2 * (trace_off + t0) : nullptr;
    int32_t *scp = (TRACE && score_off >= 0) ? scores + score_off + t0 * n : nullptr;
    int32_t ts = 0;

    // The hot loop below only ever commits moves; restarts (a trap, or a periodic one) leave it
    // and are done by the outer loop, so the loop-carried walk state stays in scalar registers.
    bool need_restart = false;
    int32_t *trap_trp = nullptr; // trace record of a trap step, written once the restart is done
    // The flip back to the state left by the last step leads to a visited state unless the insert
    // of the current state overwrote that state's slot (slots are below 2^30): such a flip needs
    // no probe.  jskip = that flip, or -1.
    uint32_t slot_cur = (uint32_t)slot_of(w.h, w.x0, exact, tlog2);
    int32_t jskip = -1;
    while (true) {
        if (need_restart) {
            need_restart = false;
            restarts++;
            restart_idx++;
            start_bits(seed, walk_id, (uint32_t)restart_idx, n, w.x);
            // The last step's store: after a trap, the word for hash 0 at the slot of the state
            // the trap moved to, which is not that state's entry; cleared (by the lanes that
            // stored it) so that no later epoch can meet it.  Otherwise an entry of the ending
            // epoch, which no probe can match any more anyway.
            T[slot_cur] = 0ull;
            ep = next_epoch(T, tlog2, ep);
            tag_hi = epoch_tag_hi(ep, tlog2);
            w.rebuild();
            slot_cur = (uint32_t)slot_of(w.h, w.x0, exact, tlog2);
            jskip = -1;
            if (lane == 0)
                T[slot_cur] = (w.h | 1ull) ^ ((uint64_t)tag_hi << 32);
            if (TRACE && trap_trp && lane == 0) {
                trap_trp[0] = -1;
                trap_trp[1] = w.isl;
            }
            trap_trp = nullptr;
            lds_fence(); // the new free bits in LDS before note_state copies them
            if (w.isl <= thr)
                note_state(ts);
        }
        // One exit, at the bottom: with a second exit (a break) the compiler copies every
        // loop-carried register once per step on the way back to the top.  The loop ends at a
        // trap, at lim or at the next periodic restart (rem steps away), so that the restart
        // countdown and the trap count are settled once per inner loop, not per step.
        lim_in = rem < lim - ts ? ts + rem : lim;
        const int32_t ts_in = ts;
        int32_t trapped = 0; // 1 after a trap (which ends the inner loop)
        if (ts < lim_in) do {
            // Keep per-lane index arithmetic inside the loop instead of pinning ~100 VGPRs of
            // loop invariants for the whole walk: the values are cheap to recompute and the
            // registers are worth more as occupancy.
            asm volatile("" : "+v"(w.lane));
            if constexpr (IssuePrioOf<W>::value)
                __builtin_amdgcn_s_setprio(0); // scoring: below the waves that are committing
            w.prepare();
            int32_t isl_j[G];
            w.score(isl_j);
            uint32_t keys[G];
#pragma unroll
            for (int g = 0; g < G; g++) {
                const int j = w.flip(g);
                keys[g] = (j < n && j != jskip) ? (((uint32_t)isl_j[g] << 8) | (uint32_t)j) : 0xFFFFFFFFu;
                if (TRACE && scp && j < n)
                    scp[j] = isl_j[g];
            }

            // best non-visited flip: take the PW smallest keys, probe them together
            int js = -1;
            int32_t isl_new = INT32_MAX; // (a trap's: above every threshold)
            uint64_t h_new = 0; // hash of the chosen neighbour (from its probe)
            static_assert(PW >= 1 && PW <= 2, "one or two candidates per probe round");
            uint32_t cand[PW];
            // the commit's reads for the best candidate, taken while its probe is in flight
            [[maybe_unused]] typename CommitReadOf<W>::type pre;
            int js_pre = -1;
            // One round: the PW best keys, probed together; true when it settles the step (a move
            // found, or no candidate left).
            auto probe_round = [&]() -> bool {
                // candidate i: the smallest key above candidate i - 1, i.e. the smallest of the
                // keys minus (candidate i - 1) + 1 in unsigned arithmetic, which sends the keys
                // at or below candidate i - 1 past every other one (keys are distinct but for the
                // empty key ~0, and a wave holds more keys than candidates)
                uint32_t base = 0;
#pragma unroll
                for (int i = 0; i < PW; i++) {
                    uint32_t km = keys[0] - base;
#pragma unroll
                    for (int g = 1; g < G; g++)
                        km = min(km, keys[g] - base);
                    cand[i] = wave_min_u32(km) + base;
                    // (on the scalar unit: left to itself the compiler adds on the vector unit to
                    // reuse the carry as the test for an empty candidate)
                    asm("s_add_u32 %0, %1, 1" : "=s"(base) : "s"(cand[i]) : "scc");
                }
                if (cand[0] == 0xFFFFFFFFu)
                    return true; // every flip leads to a visited state
                // lane i probes candidate i
                uint32_t my = cand[0];
                if constexpr (PW > 1)
                    my = (uint32_t)write_lane<1>((int32_t)my, (int32_t)cand[1]);
                const int jm = min((int)(my & 255u), n - 1);
                const uint64_t hc = w.h ^ zk[jm];
                const uint32_t x0 = w.x0 ^ (jm < 32 ? 1u << (jm & 31) : 0u);
                // every lane loads (lanes from PW on repeat lane 0's probe, an empty candidate reads
                // the slot of flip n - 1: all addresses are valid); only the candidates' lanes count
                const uint64_t got = T[slot_of(hc, x0, exact, tlog2)];
                if constexpr (IssuePrioOf<W>::value)
                    __builtin_amdgcn_s_setprio(1); // the probe is out: commit ahead of scoring waves
                if constexpr (CommitReadOf<W>::value) {
                    js_pre = (int)(cand[0] & 255u);
                    pre = w.commit_read(js_pre);
                }
                uint64_t pmask = 0;
#pragma unroll
                for (int i = 0; i < PW; i++)
                    pmask |= cand[i] != 0xFFFFFFFFu ? 1ull << i : 0ull;
                const uint64_t okmask = ballot(got != ((hc | 1ull) ^ ((uint64_t)tag_hi << 32))) & pmask;
                if (okmask != 0ull) {
                    const int first = __builtin_ctzll(okmask);
                    uint32_t pick = cand[0];
#pragma unroll
                    for (int i = 1; i < PW; i++)
                        pick = (first == i) ? cand[i] : pick;
                    js = (int)(pick & 255u);
                    isl_new = (int32_t)(pick >> 8);
                    h_new = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(hc >> 32), first) << 32) |
                            (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)hc, first);
                    return true;
                }
                return cand[PW - 1] == 0xFFFFFFFFu; // no candidate left for another round
            };
            // the first round settles almost every step; the loop after it is the rare case of PW
            // visited candidates in a row
            if (!probe_round()) {
                do {
#pragma unroll
                    for (int i = 0; i < PW; i++) {
#pragma unroll
                        for (int g = 0; g < G; g++)
                            keys[g] = keys[g] == cand[i] ? 0xFFFFFFFFu : keys[g];
                    }
                } while (!probe_round());
            }

            ts++;
            // Trapped (every flip leads to a visited state): the walk restarts, which rebuilds all
            // of the walker's state and empties its table (the next epoch), so committing any flip
            // first (flip 0) is harmless; the step then takes one path whether or not it trapped.
            // The trap's table store (hash 0) is cleared by the restart, and its ISL (INT32_MAX)
            // passes no threshold.  A trap also ends the inner loop (lim_in = ts).
            trapped = (int32_t)((uint32_t)js >> 31);
            lim_in = js < 0 ? ts : lim_in;
            js = max(js, 0);
            if constexpr (CommitReadOf<W>::value) {
                if (js == js_pre)
                    w.template commit_apply<false>(js, isl_new, pre);
                else
                    w.template commit<false>(js, isl_new);
            } else {
                w.template commit<false>(js, isl_new);
            }
            w.h = h_new;
            {
                const uint32_t s_new = (uint32_t)slot_of(w.h, w.x0, exact, tlog2);
                // every lane stores the same word to the same address (one memory request, and
                // no exec mask to save and restore around a one-lane store); the address is
                // formed on the vector unit (one 64-bit shift-add instead of four scalar ops)
                uint32_t sv = s_new;
                asm volatile("" : "+v"(sv));
                T[sv] = (w.h | 1ull) ^ ((uint64_t)tag_hi << 32);
                jskip = s_new != slot_cur ? js : -1;
                slot_cur = s_new;
            }
            if (TRACE && trp) {
                if (trapped)
                    trap_trp = trp; // written once the restart is done
                else if (w.lane == 0) {
                    trp[0] = js;
                    trp[1] = w.isl;
                }
                trp += 2;
            }
            if (TRACE && scp)
                scp += n;
            if (w.isl <= thr)
                note_state(ts);
        } while (ts < lim_in);
        traps += trapped;
        rem -= ts - ts_in;
        // a restart after a trap, or the periodic one (not after the last step, not once
        // stopped); a trap replaces a periodic restart due at the same step
        need_restart = trapped || (rem == 0 && ts < left32 && lim >= 0);
        rem = rem == 0 ? R32 : rem;
        if (!need_restart)
            break;
    }
    t = t0 + ts;
    flips = flips0 + (int64_t)ts * n;
    lds_fence();
    const int32_t best_ts = su(bk[1]), hit_ts = su(bk[2]), watch_ts = su(bk[3]);
    best_isl = su(bk[0]);
    if (best_ts >= 0)
        best_step = t0 + best_ts;
    if (hit_ts >= 0)
        hit = t0 + hit_ts;
    if (watch_ts >= 0)
        wstep = t0 + watch_ts;

    w.sync_x_lds();
    lds_fence();
    if (lane < kXWords) {
        ws.x[lane] = xl[lane];
        ws.best_x[lane] = bl[lane];
    }
    if (lane == 0) {
        ws.t = t;
        ws.flips = flips;
        ws.hit_step = hit;
        ws.watch_step = wstep;
        ws.best_isl = best_isl;
        ws.best_step = best_step;
        ws.h = w.h;
        ws.table_epoch = (int32_t)ep;
        ws.isl = w.isl;
        ws.restart_idx = restart_idx;
        ws.restarts = restarts;
        ws.traps = traps;
        ws.status = (t >= steps || (target >= 0 && hit >= 0)) ? kDone : kRunning;
    }
    (void)L;
}

// free symbols n of a walk of length L for walker W (the flips it scores)
template <class W>
__device__ __forceinline__ int free_symbols(int L)
{
    W w;
    w.set_length(L);
    return w.n;
}

template <class W, int PW>
__device__ __forceinline__ void run_walk(WalkState *__restrict__ wsp, uint64_t *__restrict__ tables,
                         int32_t *__restrict__ trace, int32_t *__restrict__ scores, int64_t chunk,
                         typename W::Lds *lds, const uint64_t *zk)
{
    if (su(wsp->trace_offset) >= 0 || su(wsp->score_offset) >= 0)
        run_walk_impl<W, PW, true>(wsp, tables, trace, scores, chunk, lds, zk);
    else if (free_symbols<W>(su(wsp->L)) <= su(wsp->table_log2))
        run_walk_impl<W, PW, false, 1>(wsp, tables, trace, scores, chunk, lds, zk);
    else
        run_walk_impl<W, PW, false, 0>(wsp, tables, trace, scores, chunk, lds, zk);
}

// ---------------------------------------------------------------------------------------------
// Shapes.
// ---------------------------------------------------------------------------------------------
//  shape : (G, KW)   lengths
//    0   : (1, 1)    c <= 32
//    1   : (1, 2)    33 <= c <= 63
//    2   : (2, 2)    c == 64
//    3   : (2, 3)    65 <= c <= 96
//    4   : (2, 4)    97 <= c <= 127
//    5   : (3, 4)    c == 128
//    6   : (3, 5)    129 <= c <= 160
//    7   : (3, 6)    161 <= c <= 191
__host__ __device__ inline int shape_for_length_dev(int L)
{
    const int c = (L - 1) / 2;
    if (c <= 32) return 0;
    if (c <= 63) return 1;
    if (c == 64) return 2;
    if (c <= 96) return 3;
    if (c <= 127) return 4;
    if (c == 128) return 5;
    if (c <= 160) return 6;
    return 7;
}


template <int SHAPE> struct ShapeGK;
template <> struct ShapeGK<0> { static constexpr int G = 1, KW = 1; };
template <> struct ShapeGK<1> { static constexpr int G = 1, KW = 2; };
template <> struct ShapeGK<2> { static constexpr int G = 2, KW = 2; };
template <> struct ShapeGK<3> { static constexpr int G = 2, KW = 3; };
template <> struct ShapeGK<4> { static constexpr int G = 2, KW = 4; };
template <> struct ShapeGK<5> { static constexpr int G = 3, KW = 4; };
template <> struct ShapeGK<6> { static constexpr int G = 3, KW = 5; };
template <> struct ShapeGK<7> { static constexpr int G = 3, KW = 6; };

// ---------------------------------------------------------------------------------------------
// Kernels.
// ---------------------------------------------------------------------------------------------
__device__ inline void fill_zobrist(uint64_t *zk)
{
    for (int j = threadIdx.x; j < kNMax; j += blockDim.x)
        zk[j] = zobrist_key(j);
    __syncthreads();
}

// SHAPE >= 0: every walk has that shape.  SHAPE < 0: any shape, dispatched per walk.
template <int SHAPE, bool DIRECT, int PW>
__device__ __forceinline__ void run_any(WalkState *ws, uint64_t *tables, int32_t *trace, int32_t *scores,
                               int64_t chunk, typename LdsOf<DIRECT>::type *lds, const uint64_t *zk)
{
    if constexpr (SHAPE >= 0) {
        run_walk<Walker<ShapeGK<SHAPE>::G, ShapeGK<SHAPE>::KW, DIRECT>, PW>(ws, tables, trace, scores, chunk, lds, zk);
    } else {
        switch (shape_for_length_dev(ws->L)) {
        case 0: run_walk<Walker<1, 1, DIRECT>, PW>(ws, tables, trace, scores, chunk, lds, zk); break;
        case 1: run_walk<Walker<1, 2, DIRECT>, PW>(ws, tables, trace, scores, chunk, lds, zk); break;
        case 2: run_walk<Walker<2, 2, DIRECT>, PW>(ws, tables, trace, scores, chunk, lds, zk); break;
        case 3: run_walk<Walker<2, 3, DIRECT>, PW>(ws, tables, trace, scores, chunk, lds, zk); break;
        case 4: run_walk<Walker<2, 4, DIRECT>, PW>(ws, tables, trace, scores, chunk, lds, zk); break;
        case 5: run_walk<Walker<3, 4, DIRECT>, PW>(ws, tables, trace, scores, chunk, lds, zk); break;
        case 6: run_walk<Walker<3, 5, DIRECT>, PW>(ws, tables, trace, scores, chunk, lds, zk); break;
        default: run_walk<Walker<3, 6, DIRECT>, PW>(ws, tables, trace, scores, chunk, lds, zk); break;
        }
    }
}

constexpr int kMaxWavesPerBlock = 8;


// Occupancy target of the walk kernel per shape: the smaller shapes fit 8 waves per SIMD (64
// VGPRs), the 3-group shapes keep more windows in registers.
template <int SHAPE> struct WavesPerEu { static constexpr int value = (SHAPE >= 0 && SHAPE <= 4) ? 8 : 6; };

template <int SHAPE, bool DIRECT, int PW>
__global__ void __launch_bounds__(64 * kMaxWavesPerBlock)
    __attribute__((amdgpu_waves_per_eu(WavesPerEu<SHAPE>::value))) k_walk(WalkState *__restrict__ states, int32_t n_walks,
                                              const int32_t *__restrict__ order,
                                              uint64_t *__restrict__ tables, int32_t *__restrict__ trace,
                                              int32_t *__restrict__ scores, int64_t chunk,
                                              int32_t *__restrict__ counter)
{
    using Lds = typename LdsOf<DIRECT>::type;
    __shared__ uint64_t zk[kNMax];
    extern __shared__ __align__(16) unsigned char dyn_smem[];
    fill_zobrist(zk);
    // wave index within the block: uniform across the wave, said so explicitly so that every
    // value derived from it (walk index, state pointer, LDS block) stays in scalar registers
    const int wave = (int)uniform(threadIdx.x >> 6);
    const int wpb = (int)(blockDim.x >> 6);
    Lds *lds = reinterpret_cast<Lds *>(dyn_smem) + wave;
    // one walk per wave (counter == nullptr), or the persistent form: every wave pulls walks
    // from the counter until the list is exhausted
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
        run_any<SHAPE, DIRECT, PW>(&states[wi], tables, trace, scores, chunk, lds, zk);
    }
}

template <int SHAPE, bool DIRECT>
__global__ void __launch_bounds__(64) k_flip_scores(int L, int count, const uint32_t *__restrict__ xs,
                                                    int32_t *__restrict__ out)
{
    using Lds = typename LdsOf<DIRECT>::type;
    constexpr int G = ShapeGK<SHAPE>::G, KW = ShapeGK<SHAPE>::KW;
    __shared__ uint64_t zk[kNMax];
    __shared__ Lds lds;
    fill_zobrist(zk);
    const int r = (int)blockIdx.x;
    if (r >= count)
        return;
    Walker<G, KW, DIRECT> w;
    w.lane = lane_id();
    w.L = L;
    w.c = (L - 1) / 2;
    w.n = w.c + 1;
    w.lds = &lds;
    w.zk = zk;
    w.init_lanes(w.lane);
#pragma unroll
    for (int i = 0; i < kXWords; i++)
        w.x[i] = xs[(int64_t)r * kXWords + i];
    w.rebuild();
    w.prepare();
    int32_t isl_j[G];
    w.score(isl_j);
    const int lane = lane_id();
#pragma unroll
    for (int g = 0; g < G; g++) {
        const int j = lane + 64 * g;
        if (j < w.n)
            out[(int64_t)r * w.n + j] = isl_j[g];
    }
}

using WalkKernel = void (*)(WalkState *, int32_t, const int32_t *, uint64_t *, int32_t *, int32_t *,
                            int64_t, int32_t *);

// One translation unit per (variant, probe width) instantiates the kernels of every shape.
WalkKernel pick_walk_kernel_bits_pw1(int shape);
WalkKernel pick_walk_kernel_bits_pw2(int shape);
WalkKernel pick_walk_kernel_direct_pw1(int shape);
WalkKernel pick_walk_kernel_direct_pw2(int shape);
WalkKernel pick_walk_kernel_mfma(int shape);

} // namespace liblabs
