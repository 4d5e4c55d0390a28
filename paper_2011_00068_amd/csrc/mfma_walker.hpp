// mfma_walker.hpp -- the skew walker with its flip scoring on the matrix cores (gfx950
// v_mfma_i32_16x16x64_i8): one tile for L <= 255 (c <= 127), two up to L = 383 (c <= 191).
//
// Scoring (derived from Eq. (1) and (4), as in the bit-sliced walker): for flip j = 2h + p
// (parity p = j & 1, h = j >> 1, mirror m = L-1-j, d = m - j = 2 (c - j), kappa_d = c-1-j)
//   ISL_j = ISL - 8 s_j G_j + 16 H_j,
//   G_j = sum_kappa C'_kappa (p_kappa + q_kappa) - C'_{kappa_d} s_m,   C'_kappa = C_{2 kappa + 2},
//   H_j = np + 3 nq - 1 - 2 [q_d valid] - 4 rc'_j,
// with p_kappa = s^p_{h+1+kappa}, q_kappa = s^p_{h-1-kappa} (s^p_u = s_{2u+p}, 0 outside the
// sequence), np / nq the counts of valid p / q shifts and rc'_j the number of both-sided shifts
// kappa < nq, kappa != kappa_d, where p and q differ.  Since s_m = (-1)^(c-j) s_j, the excluded
// term contributes 8 (-1)^(c-j) C'_{kappa_d} whatever the sign of s_j, and
//   ISL_j = ISL + 16 hc_j - 64 rc'_j + 8 (-1)^(c-j) C'_{kappa_d} - 8 s_j T_j,
//   T_j = Y_j + Z_j,  Y_j = sum_kappa C'_kappa s^p_{h+1+kappa},  Z_j = sum_kappa C'_kappa s^p_{h-1-kappa}.
// For the centre j = c (p = q, Eq. (4)): G_c = T_c / 2 and H_c = nq, which the same expression
// gives with hc = nq, no rc' bits, a zero word for C'_{kappa_d} and the factor -4 s_c for T_c.
//
// Y and Z are correlations of the small integer vector C' with +-1 strings, i.e. products of a
// Hankel matrix of the sequence with a Toeplitz arrangement of C'.  One 16x16 tile holds all of
// them: row r = 4 i + kind, column nn, h = 16 i + nn, K index t = kappa + 1 + nn:
//   A[r][t] = S_kind[t + 16 i]   (kind 0/1: s^0, s^1;  kind 2/3: s^p_{63-u}, so that row kind 2+p
//                                 column nn yields Z at h' = 63 - h; 0 outside the sequence),
//   B[t][nn] = C'_{t-1-nn}        (0 outside 0 <= t-1-nn < c),
// so D[r][nn] = sum_t A B is Y (kind p) at h and Z (kind 2+p) at 63 - h.  Every A row is an
// aligned 16-byte window of a byte copy of one string; every B column is a 16-byte window of C'
// starting at byte t0 - 1 - nn, read from whichever of four copies of C' shifted by 0..3 bytes
// puts it on a dword boundary (each step writes C' into all four).  K = 64 KB covers every t of a
// nonzero term, t <= c (see KB below).
// C' fits int8 unless |C_k| > 127; then C' = 64 hi + lo (lo in 0..63, hi in -4..3) and a second
// pass adds 64 x the hi tile.  Lane layout of the instruction (checked on gfx950): lane l holds
// row / column l % 16 of A / B and K slice 16 (l / 16) .. +15 in its four registers' bytes, and D
// register r of lane l is D[4 (l / 16) + r][l % 16]; so lane l receives Y_j, Y_{j+1} for h = l
// and Z for h = 63 - l, which one ds_bpermute brings to lane h.
//
// Lane l owns flips j = 2 l and 2 l + 1 (the same h, both parities).  The correlation table is
// lane-held as in the bit-sliced walker.
//
// rc'_j is kept per owned flip across commits instead of being recounted every step.  Committing
// js (negating s_js and its mirror m' = 2c - js, where s_m' = (-1)^(c-js) s_js) toggles whether
// p and q differ in at most two terms s_{j+k} s_{j-k} of flip j, and only for j of the parity of
// js: the term with end js (partner 2 j - js; not counted when that partner is the mirror of j,
// the excluded shift) and the term with end m' (partner 2 j - m'; the same term when js = c).
// A term whose ends were equal now differs and the reverse, so for j < c, j != js
//   d rc'_j = s_js (s_{2j-js} + (-1)^(c-js) [js != c] s_{2j-m'}),
// with s taken before the commit and 0 outside the sequence (the partners are never js or m').
// The parity bit strings are then read only when a walk (re)starts, so commits no longer update
// them.
#pragma once

#include "walk_impl.hpp"

namespace liblabs {

typedef int mfma_v4i __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) const uint32_t lds_cu32; // LDS words, read
typedef __attribute__((address_space(3))) const mfma_v4i lds_cv4;  // 16-byte aligned LDS quads, read

// Per-wave LDS block.  The small layout serves c <= 127 (one tile, four strings); the big one
// serves up to c = 191 (a second tile for half indices 64..127 with two more strings, longer
// strings and C' copies) and every walker of a mixed-length launch.
//
// The A operand of a tile is one 16-byte read per lane.  The 16 lanes of a row group read kinds
// 0..3 x 4 windows of 16 bytes at the same K offset, so the strings that one tile reads must sit
// at distinct multiples of 16 dwords modulo 64 for the group to cover 64 distinct banks.  Small
// layout: strings 80 dwords apart from dword 16 (16, 32, 48, 0 mod 64).  Big layout: strings 0..3
// 144 apart from dword 32 (32, 48, 0, 16), then strings 4 and 5 (the second tile's kinds 2/3,
// read beside kinds 0/1 at +16 dwords, i.e. 48 and 0 mod 64) at 32 and 16 mod 64.
//
// The rc' update of a commit reads s^p at half indices down to -63 (small) / -95 (big) from the
// kind-p strings: zero words before string 0 (the first 16 / 32 dwords of sbuf) and the gap
// between strings 0 and 1 (16 / 52 dwords) are kept zero for it.
template <int NSTR, int SEQ_DWORDS, int C_DWORDS, int C_WORDS>
struct alignas(16) WaveLdsMfmaT {
    static constexpr int kStrings = NSTR;
    static constexpr int kSeqDwords = SEQ_DWORDS; // string bytes used: 4 kSeqDwords
    static constexpr int kCDwords = C_DWORDS;     // one copy of C': byte 20 + kappa - r in copy r
    static constexpr int kCWords = C_WORDS;       // C' at kappa (0 for kappa >= c; C'_c is the zero word)
    // dword offset of string k in sbuf
    __host__ __device__ static constexpr int str_off(int k)
    {
        return NSTR == 4 ? 16 + 80 * k : 32 + (k < 4 ? 144 * k : 576 + 112 * (k - 4));
    }
    static constexpr int kSbufDwords = str_off(NSTR - 1) + SEQ_DWORDS;
    static_assert(NSTR == 4 || NSTR == 6, "four or six strings");
    static_assert(NSTR == 4 ? (80 >= SEQ_DWORDS) : (144 >= SEQ_DWORDS && 112 >= SEQ_DWORDS &&
                                                    576 >= 3 * 144 + SEQ_DWORDS),
                  "strings overlap");
    // A commit writes the mirror's byte of a kind-2+p string (one-tile walker, in either layout)
    // or kind-4+p string (two tiles) at 63 - a / 127 - a for its half index a <= c (127 / 191):
    // half indices the string does not hold land up to 64 bytes before it, in the gap after the
    // previous string, which nothing reads (the two-tile walker's kind-2+p write goes to a dummy
    // word instead)
    static_assert(4 * (str_off(2) - str_off(1) - SEQ_DWORDS) >= 64 &&
                      4 * (str_off(3) - str_off(2) - SEQ_DWORDS) >= 64 &&
                      (NSTR == 4 || (4 * (str_off(4) - str_off(3) - SEQ_DWORDS) >= 64 &&
                                     4 * (str_off(5) - str_off(4) - SEQ_DWORDS) >= 64)),
                  "64 free bytes before each string a mirror byte can miss");
    // zero bytes before the kind-p strings (string 0: the leading pad; string 1: the gap)
    static_assert(4 * str_off(0) >= (NSTR == 4 ? 63 : 95) &&
                      4 * (str_off(1) - str_off(0) - SEQ_DWORDS) >= (NSTR == 4 ? 63 : 95),
                  "zero pads of the rc' reads");
    uint32_t par[2][kParWords];       // bit a of par[p] = b_{2a+p} (0 past the sequence end)
    uint32_t rev[2][kRevWords];       // bit a of rev[p] = bit (kNA-1-a) of par[p], 0 past kNA-1
    uint32_t xw[kXWords];             // free bits (kept current by every commit)
    uint32_t bestx[kXWords];          // free bits of the best state of the walk so far
    int32_t book[8];                  // the walk loop's rarely updated bookkeeping
    int32_t C[C_WORDS];               // C'_kappa at index kappa
    uint32_t sbuf[kSbufDwords];       // +-1 byte strings of the A operands, string k at str_off(k)
    uint32_t cb[4][C_DWORDS];         // C' as int8, four copies shifted by 0..3 bytes

    __device__ __forceinline__ uint32_t *str(int k) { return sbuf + str_off(k); }
    __device__ __forceinline__ const uint32_t *str(int k) const { return sbuf + str_off(k); }
};
// strings: kind p (s^p), kind 2+p (s^p_{63-u}) and, big only, kind 4+p (s^p_{127-u})
static_assert(sizeof(uint32_t) * (2 * kParWords + 2 * kRevWords + 2 * kXWords + 8) % 16 == 0,
              "the C' table and the strings start 16-byte aligned");
using WaveLdsMfma = WaveLdsMfmaT<4, 64, 56, 128>;
using WaveLdsMfmaBig = WaveLdsMfmaT<6, 92, 74, 192>;
static_assert(offsetof(WaveLdsMfma, sbuf) % 16 == 0 && offsetof(WaveLdsMfmaBig, sbuf) % 16 == 0,
              "strings 16-byte aligned");

// v where cond is false, 0 where it is true: one v_cndmask on the lane mask of cond (a select,
// never a branch around the computation of v)
__device__ __forceinline__ int32_t drop_where(bool cond, int32_t v)
{
    const uint64_t m = __builtin_amdgcn_ballot_w64(cond);
    int32_t r;
    asm("v_cndmask_b32_e64 %0, %1, 0, %2" : "=v"(r) : "v"(v), "s"(m));
    return r;
}

// v where cond is false, -v where it is true
__device__ __forceinline__ int32_t negate_where(bool cond, int32_t v)
{
    const uint64_t m = __builtin_amdgcn_ballot_w64(cond);
    int32_t r;
    asm("v_cndmask_b32_e64 %0, %1, %2, %3" : "=v"(r) : "v"(v), "v"(-v), "s"(m));
    return r;
}

__device__ __forceinline__ uint32_t nibble_bytes(uint32_t nib)
{
    // 4 bits -> 4 bytes of 0/1 (the shifted copies never overlap, so the product has no carries)
    return (nib * 0x00204081u) & 0x01010101u;
}

// Per-lane constants of one owned flip (they depend only on L and j).
struct MfmaFlip {
    const int32_t *c_kd; // C'_{kappa_d}; the zero word C'_c for the centre (and past it)
    int32_t hc;          // np + 3 nq - 1 - 2 [q_d valid]; nq for the centre
    int32_t rcf;         // factor of rc'_j: -64 for j < c, 0 for the centre and past it (whose rc
                         // the commits do not keep)
};

// Window words of the matrix-core walker per shape: those of the bit-sliced walker, except that
// shape 2 (c = 64, one length) takes the three-word walker, so that the two-word one serves
// c <= 63 with a single K block.
template <int SHAPE> struct MfmaKW {
    static constexpr int value = SHAPE == 2 ? 3 : ShapeGK<SHAPE>::KW;
};

// KW: shift window words (c <= 32 KW; c <= 63 for KW = 2, see MfmaKW); BIG: flips up to
// c = 191 (two tiles, four flips per lane: j = 2 l + g for g < 2 and j = 128 + 2 l + (g - 2)
// for g >= 2, i.e. half index l and 64 + l); LdsT: the LDS layout (big whenever BIG, or in a
// mixed-length launch).
template <int KW, bool BIG = false, class LdsT = WaveLdsMfma>
struct MfmaWalker {
    static constexpr int G = BIG ? 4 : 2;
    static constexpr int kG = G;
    static constexpr int QR = (KW + 1) / 2;
    // K blocks of 64: a tile's Y term at half index h reads s^p at h + 1 + kappa = h + t - nn <= c
    // (the string is 0 past the sequence; h >= nn), so t <= c; its Z term at 63 - h reads s^p at
    // 63 - 16 i - t >= 0, so t <= 63.  Every nonzero term has t <= the largest c of the walker
    // (127 with one tile, 191 with two).
    static constexpr int kCMaxW = BIG ? (32 * KW < 191 ? 32 * KW : 191) : (KW == 1 ? 32 : KW == 2 ? 63 : KW == 3 ? 96 : 127);
    static constexpr int KB = (kCMaxW + 64) / 64;
    // K blocks of the second tile (BIG): its Y terms at half index 64 + h need t = kappa + 1 + nn
    // <= c - 64 <= 127 (the string is 0 past the sequence), its Z terms at half index h' <= c / 2
    // need t <= h' + 15 <= 111, so two blocks hold every term of an existing flip
    static constexpr int KB2 = KB < 2 ? KB : 2;
    static constexpr int kCBytes = 4 * LdsT::kCDwords;  // distance of the C' copies
    using Lds = LdsT;
    static_assert(!BIG || LdsT::kStrings == 6, "the second tile needs the big layout");
    static_assert(64 * KB + (BIG ? 112 : 48) <= 4 * LdsT::kSeqDwords, "A windows past the strings");

    int L, c, n;
    int lane;
    int32_t isl;
    uint64_t h;
    uint32_t x[kXWords]; // free bits; current only where commit<true> is used (else in lds->xw)
    uint32_t x0;         // free bits 0..31, always current
    int32_t Cv[QR];
    int32_t rc[G];       // rc'_j of the owned flips (0 for j >= c), kept across commits
    int32_t mult[G];     // factor of T_j: -8 s_j (-4 s_c for the centre, 0 past it)
    int planes;
    int32_t eps8[2];     // 8 (-1)^(c-j) for j of parity 0 / 1 (uniform)
    Lds *lds;
    const uint64_t *zk;
    MfmaFlip fc[G];
    uint32_t ta, tb;   // LDS addresses of this lane's A and B words of K block 0 (see init_lanes())
    uint32_t ta2;      // the same for the second tile's A operand (BIG)
    int32_t bsrc;      // ds_bpermute source of Z: lane 63 - lane

    __device__ __forceinline__ int flip(int g) const { return (g < 2 ? 0 : 128) + 2 * lane + (g & 1); }
    // the lane and the slot g that own flip j
    __device__ __forceinline__ static int owner_lane(int j) { return (j & 127) >> 1; }
    __device__ __forceinline__ static int owner_slot(int j) { return (j >> 7) * 2 + (j & 1); }

    __device__ __forceinline__ uint32_t *x_lds() const { return lds->xw; }
    __device__ __forceinline__ uint32_t *best_lds() const { return lds->bestx; }
    __device__ __forceinline__ int32_t *book_lds() const { return lds->book; }

    __device__ __forceinline__ void set_length(int len)
    {
        L = len;
        c = (L - 1) / 2;
        n = c + 1;
        eps8[0] = (c & 1) ? -8 : 8;
        eps8[1] = -eps8[0];
    }

    __device__ __forceinline__ void init_lanes(int ln)
    {
        {
            // Lane (slice, nn) of a tile needs A bytes S_kind[t0 + 16 ib ..] and the 16 bytes
            // C'_{i0 .. i0+15}, i0 = t0 - 1 - nn, t0 = 16 slice + 64 kb; copy r = (i0 + 20) mod 4 of
            // C' holds them from a dword boundary.  K block kb is 16 dwords further in both.  The
            // second tile (half indices 64 + h) reads kinds 0/1 64 bytes further and, for kinds
            // 2/3, the strings s^p_{127-u}.
            const int nn = ln & 15, slice = ln >> 4;
            const int kind = ln & 3, ib = (ln & 15) >> 2;
            const int r = (3 - nn) & 3;
            ta = (uint32_t)(uintptr_t)(lds->str(kind) + 4 * (slice + ib));
            ta2 = BIG ? (uint32_t)(uintptr_t)(lds->str(kind < 2 ? kind : kind + 2) + 4 * (slice + ib) + (kind < 2 ? 16 : 0)) : 0u;
            tb = (uint32_t)(uintptr_t)&lds->cb[r][(16 * slice - 1 - nn + 20 - r) >> 2];
            bsrc = (63 - ln) << 2;
            // whole addresses, so that every load is one base register plus an offset
            asm volatile("" : "+v"(ta), "+v"(tb), "+v"(bsrc));
            if constexpr (BIG)
                asm volatile("" : "+v"(ta2));
        }
#pragma unroll
        for (int g = 0; g < G; g++) {
            const int j = (g < 2 ? 0 : 128) + 2 * ln + (g & 1);
            const int nq = j >> 1;
            const int np = c - ((j + 1) >> 1);
            MfmaFlip &f = fc[g];
            if (j < c) {
                const int kd = c - 1 - j; // <= 62 for the second tile's flips
                const bool qdv = kd < nq;
                f.c_kd = &lds->C[kd];
                f.hc = np + 3 * nq - 1 - (qdv ? 2 : 0);
                f.rcf = -64;
            } else {
                f.c_kd = &lds->C[c];
                f.hc = nq;
                f.rcf = 0;
            }
        }
    }

    // The free bits into lds->xw from the kind-p strings (bit j set where s_j = -1): commit<false>
    // keeps only the strings current, and the walk reads the free bits rarely (a new best state,
    // the end of a launch).
    __device__ __forceinline__ void sync_x_lds()
    {
        const int lane = this->lane;
        typedef __attribute__((address_space(3))) const int8_t lds_ci8;
        const uint32_t s0 = (uint32_t)(uintptr_t)lds->str(0);
        const uint32_t d1 = 4u * (uint32_t)(Lds::str_off(1) - Lds::str_off(0));
#pragma unroll
        for (int r = 0; r < kXWords / 2; r++) {
            const int j = 64 * r + lane; // half index j / 2 < 96: inside the strings
            const int32_t v = *(lds_ci8 *)(uintptr_t)(s0 + (uint32_t)(j & 1) * d1 + (uint32_t)(j >> 1));
            const uint64_t m = ballot(j < n && v < 0);
            if (lane == 0) {
                lds->xw[2 * r] = (uint32_t)m;
                lds->xw[2 * r + 1] = (uint32_t)(m >> 32);
            }
        }
        lds_fence();
    }

    __device__ inline uint32_t seq_bit(int i) const
    {
        if (i < 0 || i >= L)
            return 0u;
        const int f = (i <= c) ? i : 2 * c - i;
        const uint32_t b = (lds->xw[f >> 5] >> (f & 31)) & 1u;
        return (i <= c) ? b : (b ^ (uint32_t)((i - c) & 1));
    }

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
        if (lane < 2 * (kParWords - 6))
            lds->par[lane & 1][6 + (lane >> 1)] = 0u;
        if (lane < 2 * (kRevWords - 6))
            lds->rev[lane & 1][6 + (lane >> 1)] = 0u;
        for (int i = lane; i < 4 * LdsT::kCDwords; i += kWave)
            lds->cb[i / LdsT::kCDwords][i % LdsT::kCDwords] = 0u;
        // the zero pads before the kind-p strings
        for (int i = lane; i < LdsT::str_off(0); i += kWave)
            lds->sbuf[i] = 0u;
        for (int i = LdsT::str_off(0) + LdsT::kSeqDwords + lane; i < LdsT::str_off(1); i += kWave)
            lds->sbuf[i] = 0u;
        // prepare() writes C'_kappa for kappa < 64 QR; the zero word C'_c may lie past that (c = 64)
        for (int i = lane; i < LdsT::kCWords; i += kWave)
            lds->C[i] = 0;
        lds_fence();
        // +-1 byte strings: kind p from par[p] at half index u = 4 i + b, kind 2+p from rev[p] at
        // bit 128 + u (= s^p_{63-u}), kind 4+p from rev[p] at bit 64 + u (= s^p_{127-u}); 0 where
        // the half index is outside the sequence
        for (int i = lane; i < LdsT::kSeqDwords; i += kWave) {
#pragma unroll
            for (int k4 = 0; k4 < LdsT::kStrings; k4++) {
                const int p = k4 & 1, kind = k4 >> 1;
                const int bitpos = (kind == 0 ? 0 : (kind == 1 ? 128 : 64)) + 4 * i;
                uint32_t valid = 0;
#pragma unroll
                for (int b = 0; b < 4; b++) {
                    const int u = kind == 0 ? 4 * i + b : (kind == 1 ? 63 : 127) - (4 * i + b);
                    valid |= (u >= 0 && 2 * u + p <= L - 1) ? 1u << b : 0u;
                }
                uint32_t word = 0;
                if (valid) // (the word index stays inside the strings where any byte is valid)
                    word = kind == 0 ? lds->par[p][bitpos >> 5] : lds->rev[p][bitpos >> 5];
                const uint32_t bits = (word >> (bitpos & 31)) & valid;
                lds->str(k4)[i] = nibble_bytes(valid) | (nibble_bytes(bits) * 0xFEu);
            }
        }
        uint32_t sb2[G];
#pragma unroll
        for (int g = 0; g < G; g++) {
            const int j = flip(g);
            sb2[g] = (j <= c) ? seq_bit(j) : 0u;
            const int32_t s = 1 - 2 * (int32_t)sb2[g];
            mult[g] = j < c ? -8 * s : (j == c ? -4 * s : 0);
        }
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
                    const int last = L - 1 - k - p;
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
            const int j = flip(g);
            if (j <= c && sb2[g])
                hz ^= zk[j];
        }
        h = wave_xor_u64(hz);
        init_rc();
        lds_fence();
    }

    // rc'_j of the owned flips from the parity bit strings (a walk's start and every launch's
    // resume): the number of both-sided shifts kappa < nq, kappa != kappa_d, at which the p window
    // (bits h+1 .. of par[p]) and the q window (bits kNA-h .. of rev[p]) differ.
    __device__ __forceinline__ void init_rc()
    {
        const int lane = this->lane;
        const uint32_t sp = (uint32_t)(lane + 1); // window shifts: h+1 and kNA-h = 1 - sp (mod 32)
        const uint32_t *wp = &lds->par[0][(lane + 1) >> 5];
        const uint32_t *wq = &lds->rev[0][(kNA - lane) >> 5];
#pragma unroll
        for (int g = 0; g < G; g++) {
            const int j = flip(g);
            const int nq = j >> 1;
            uint32_t m0 = 0u, m1 = 0u, m2 = 0u;
            if (j < c) {
                const int kd = c - 1 - j;
                // bits kappa < nq (nq <= 63, or 64 <= nq <= 95 in the second tile)
                uint64_t m = g < 2 ? (1ull << nq) - 1ull : ~0ull;
                if (kd < nq)
                    m &= ~(1ull << kd);
                m0 = (uint32_t)m;
                m1 = (uint32_t)(m >> 32);
                m2 = g < 2 ? 0u : (1u << (nq - 64)) - 1u;
            }
            // the second tile's windows start 64 bits further in par, 64 bits earlier in rev
            const uint32_t *wpg = wp + (g & 1) * kParWords + (g < 2 ? 0 : 2);
            const uint32_t *wqg = wq + (g & 1) * kRevWords - (g < 2 ? 0 : 2);
            const uint32_t wp0 = funnel(wpg[1], wpg[0], (int)sp);
            const uint32_t wp1 = funnel(wpg[2], wpg[1], (int)sp);
            const uint32_t wq0 = funnel(wqg[1], wqg[0], (int)(1u - sp));
            const uint32_t wq1 = funnel(wqg[2], wqg[1], (int)(1u - sp));
            uint32_t r = popc((wp0 ^ wq0) & m0) + popc((wp1 ^ wq1) & m1);
            if (g >= 2) {
                const uint32_t wp2 = funnel(wpg[3], wpg[2], (int)sp);
                const uint32_t wq2 = funnel(wqg[3], wqg[2], (int)(1u - sp));
                r += popc((wp2 ^ wq2) & m2);
            }
            rc[g] = (int32_t)r;
        }
    }

    // C' to LDS (for the excluded-shift term), whether C' fits int8, and C' bytes for the B
    // operand.
    __device__ __forceinline__ void prepare()
    {
        const int lane = this->lane;
#pragma unroll
        for (int q = 0; q < QR; q++)
            lds->C[lane + 64 * q] = Cv[q];
        // some |C'_kappa| above the int8 range?  |C'_kappa| <= L - 2 - 2 kappa <= 127 from
        // kappa = (L - 129) / 2 on: the first 64 shifts for L <= 255, the first 128 beyond
        bool wide = (uint32_t)(Cv[0] + 128) > 255u;
        if constexpr (BIG)
            wide = wide || (uint32_t)(Cv[1] + 128) > 255u;
        planes = ballot(wide) != 0ull ? 9 : 8; // only "fits int8 or not" is used
        put_c(0);
        if (planes > 8)
            put_c(1); // C' does not fit: its low six bits first (the high part follows in score())
        lds_fence();
    }

    // C' bytes into the four shifted copies: part 0 C' itself, part 1 its low six bits (0..63),
    // part 2 C' >> 6 (-6..5 for |C'| <= 381).
    __device__ __forceinline__ void put_c(int part)
    {
        int8_t *cp = reinterpret_cast<int8_t *>(lds->cb[0]) + 20 + lane;
#pragma unroll
        for (int q = 0; q < QR; q++) {
            const int32_t v = part == 0 ? Cv[q] : (part == 1 ? (Cv[q] & 63) : (Cv[q] >> 6));
#pragma unroll
            for (int r = 0; r < 4; r++)
                cp[64 * q + r * (kCBytes - 1)] = (int8_t)v;
        }
    }

    // One K-sweep of a tile (A operand at LDS address a_addr, NKB blocks) with the C' bytes now
    // in the copies.
    template <int NKB>
    __device__ __forceinline__ mfma_v4i tile(uint32_t a_addr) const
    {
        // A windows start on 16-byte boundaries (one 16-byte read), B windows on dword boundaries
        const lds_cv4 *ap4 = (const lds_cv4 *)(uintptr_t)a_addr;
        const lds_cu32 *bp = (const lds_cu32 *)(uintptr_t)tb;
        // every operand load first, so that one LDS latency covers the whole K sweep
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

    // the product of a tile, with the second sweep of a wide C' (C' = 64 hi + lo)
    template <int NKB = KB>
    __device__ __forceinline__ mfma_v4i tile_all(uint32_t a_addr)
    {
        mfma_v4i d = tile<NKB>(a_addr);
        if (planes > 8) {
            // the copies held lo (the caller rewrites them with lo again afterwards when several
            // tiles use them); the wave's LDS operations run in order, so the reads above complete
            // before the hi bytes overwrite them
            put_c(2);
            lds_fence();
            const mfma_v4i hi = tile<NKB>(a_addr);
            d = d + hi * 64;
        }
        return d;
    }

    __device__ __forceinline__ void score(int32_t (&isl_j)[G])
    {
        const int lane = this->lane;
        // the part without T first (table reads that do not wait for the tile):
        // base_j = ISL + 16 hc - 64 rc' + 8 (-1)^(c-j) C'_{kappa_d}
        int32_t base[G];
#pragma unroll
        for (int g = 0; g < G; g++) {
            const MfmaFlip &f = fc[g];
            // |C'| <= 381: a 24-bit product
            base[g] = mad24(rc[g], f.rcf, isl + 16 * f.hc) + __mul24(eps8[g & 1], *f.c_kd);
        }
        (void)lane;
        const mfma_v4i d = tile_all(ta);
        // Z for h = lane sits in lane 63 - lane; |T| <= 191 * 381: 24-bit products
        isl_j[0] = mad24(mult[0], d[0] + __builtin_amdgcn_ds_bpermute(bsrc, d[2]), base[0]);
        isl_j[1] = mad24(mult[1], d[1] + __builtin_amdgcn_ds_bpermute(bsrc, d[3]), base[1]);
        if constexpr (BIG) {
            if (planes > 8) // the copies hold hi now: lo again for the second tile
                put_c(1);
            const mfma_v4i d2 = tile_all<KB2>(ta2);
            // second tile: Y for half index 64 + lane, Z for 127 - lane (brought from lane 63 - lane)
            isl_j[2] = mad24(mult[2], d2[0] + __builtin_amdgcn_ds_bpermute(bsrc, d2[2]), base[2]);
            isl_j[3] = mad24(mult[3], d2[1] + __builtin_amdgcn_ds_bpermute(bsrc, d2[3]), base[3]);
        }
    }

    // What a commit of flip js reads, and the per-lane changes it derives from it.  The walker's
    // state is not touched, so a walk can take this for its best candidate while that candidate's
    // table probe is in flight, and apply it once the probe has confirmed the candidate.
    struct CommitRead {
        int32_t dq[QR];           // C'_kappa += f dq[q] (kappa = lane + 64 q)
        int32_t d[BIG ? 2 : 1];   // rc' of half index 64 t + lane: += f0 d[t] (p = 0), f1 d[t] (p = 1)
        int32_t f, f0, f1;        // uniform factors
        int32_t sjs, emir, hjs, nps;
        uint32_t sp_a, sq_a, sr_a;
    };
    // whether a walk takes commit_read for its best candidate during the probe: measured faster for
    // c <= 63 (L = 101: 4.6 % per step), slower for the longer shapes, whose registers it crowds
    static constexpr bool kSpecRead = KW <= 2 && !BIG;
    // issue priority for the commit phase (see IssuePrioOf): the one-tile shape of the widest
    // window (c <= 127, the L = 193 .. 255 walks) in a launch of that shape alone
    static constexpr bool kIssuePrio = KW == 4 && !BIG && std::is_same<LdsT, WaveLdsMfma>::value;

    __device__ __forceinline__ CommitRead commit_read(int js) const
    {
        // The index arithmetic of a commit is wave-uniform and runs on the scalar unit; the vector
        // instructions are the per-lane reads, selects and updates.
        const int lane = this->lane;
        CommitRead r;
        // the lane that scores js and its slot (one tile: js < 128, slot = js & 1)
        const int ol = BIG ? (js & 127) >> 1 : js >> 1;
        const int slot = BIG ? (js >> 7) * 2 + (js & 1) : js & 1;
        // mult of js at its owner lane: -8 s_js, or -4 s_c at the centre
        int32_t mj = __builtin_amdgcn_readlane(mult[0], ol);
        if constexpr (G == 2) {
            // both slots' values, then one scalar select (left to itself the compiler branches)
            const int32_t m1 = __builtin_amdgcn_readlane(mult[1], ol);
            asm("s_cmp_eq_u32 %1, 0\n\ts_cselect_b32 %0, %2, %3" : "=s"(mj) : "s"(slot), "s"(mj), "s"(m1) : "scc");
        } else {
#pragma unroll
            for (int g = 1; g < G; g++)
                mj = slot == g ? __builtin_amdgcn_readlane(mult[g], ol) : mj;
        }
        r.f = mj >> 1;                               // -4 s_js (-2 s_c at the centre)
        const int32_t sjs = ~((mj >> 31) << 1);      // s_js before the commit: -1 if mj > 0, else 1
        const int hjs = js >> 1;
        const int pis = js & 1;
        // (at the centre js = c these give kds = -1, no excluded shift, and nps = hjs)
        const int kds = c - 1 - js;                  // the excluded shift kappa_d of js
        typedef __attribute__((address_space(3))) const int8_t lds_ci8;
        // byte addresses of the strings of kind p, 2+p and (big) 4+p
        const uint32_t s0 = (uint32_t)(uintptr_t)lds->str(0);
        const uint32_t sp_a = s0 + (uint32_t)pis * 4u * (uint32_t)(Lds::str_off(1) - Lds::str_off(0));
        const uint32_t sq_a = sp_a + 4u * (uint32_t)(Lds::str_off(2) - Lds::str_off(0));
        const uint32_t sr_a = BIG ? (uint32_t)(uintptr_t)lds->str(4) +
                                        (uint32_t)pis * 4u * (uint32_t)(Lds::str_off(5) - Lds::str_off(4))
                                  : 0u;
        r.sjs = sjs;
        r.hjs = hjs;
        r.nps = c - hjs - pis;                       // half index of the mirror m' = 2c - js
        r.sp_a = sp_a;
        r.sq_a = sq_a;
        r.sr_a = sr_a;
        // dC'_kappa = -4 s_js (p_kappa + q_kappa), p without the excluded shift kappa_d, read from
        // the +-1 byte strings (0 past either end, so lanes with kappa >= c add nothing): p from
        // s^p at hjs + 1 + kappa, q = s^p_{hjs-1-kappa} from the reversed string (s^p_{63-u}, or
        // s^p_{127-u} when half indices reach past 64); at the centre p = q and u = q, so the
        // factor is halved instead
        // (the uniform bases go through readfirstlane, a no-op on a scalar, so that the per-lane
        // offsets stay one add and the constant ones fold into the reads' offset fields)
        lds_ci8 *const pl = (lds_ci8 *)(uintptr_t)su(sp_a + (uint32_t)(hjs + 1)) + lane;
        lds_ci8 *const ql = (lds_ci8 *)(uintptr_t)su((BIG ? sr_a + 128u : sq_a + 64u) - (uint32_t)hjs) + lane;
        int32_t pv[QR], qv[QR];
#pragma unroll
        for (int q = 0; q < QR; q++) {
            pv[q] = pl[64 * q];
            qv[q] = ql[64 * q];
        }
#pragma unroll
        for (int q = 0; q < QR; q++)
            r.dq[q] = drop_where(lane + 64 * q == kds, pv[q]) + qv[q];
        // rc'_j of the owned flips of js's parity (see the file header).  Partner 2 j - js is s^p at
        // half index u1 = 2h - hjs >= -63 (-95 big), read from the kind-p string, whose zero pad
        // covers the negative ones; partner 2 j - m' is s^p at u2 = 2h + hjs + p - c, read as byte
        // 63 - u2 of the kind-2+p string (127 - u2 of the kind-4+p string when BIG), which holds 0
        // past the sequence's start; u2 < 64 (< 128) for every flip j < c.  Flips j >= c read
        // anything and keep it (their rc' is not used).  The term of partner 2 j - js is dropped
        // where it is the excluded shift of j (js = 3 j - 2c, i.e. 3 h = hjs + c - p), and flip js
        // itself does not change.  s_m' = (-1)^(c - js) s_js (also at the centre, where m' = js).
        const int32_t emir = pis ? -(eps8[0] >> 3) : (eps8[0] >> 3); // (-1)^(c - js)
        r.emir = emir;
        const int32_t eps = js == c ? 0 : emir;
        r.f1 = pis ? sjs : 0;
        r.f0 = sjs - r.f1;
        const int tri = hjs + c - pis;
        lds_ci8 *const a1 = (lds_ci8 *)(uintptr_t)su(sp_a - (uint32_t)hjs) + 2 * lane;
        lds_ci8 *const a2 =
            (lds_ci8 *)(uintptr_t)su((BIG ? sr_a : sq_a) + (uint32_t)((BIG ? 127 : 63) - hjs - pis + c)) - 2 * lane;
#pragma unroll
        for (int t = 0; t < (BIG ? 2 : 1); t++) {
            const int32_t h = 64 * t + lane;
            const int32_t v1 = a1[128 * t];
            const int32_t v2 = a2[-128 * t];
            r.d[t] = drop_where(h == hjs, mad24_u(v2, eps, drop_where(3 * h == tri, v1)));
        }
        return r;
    }

    // Commit flip js with what commit_read(js) returned (nothing written since).
    template <bool REG_X = true>
    __device__ __forceinline__ void commit_apply(int js, int32_t isl_new, const CommitRead &r)
    {
        typedef __attribute__((address_space(3))) int8_t lds_i8;
#pragma unroll
        for (int q = 0; q < QR; q++)
            Cv[q] = mad24_u(r.dq[q], r.f, Cv[q]);
#pragma unroll
        for (int t = 0; t < (BIG ? 2 : 1); t++) {
            rc[2 * t] = mad24_u(r.d[t], r.f0, rc[2 * t]);
            rc[2 * t + 1] = mad24_u(r.d[t], r.f1, rc[2 * t + 1]);
        }
        // the flipped symbol (lane 0) and its mirror m' = 2c - js (lane 1; the centre again when js
        // = c) in the +-1 byte strings: kind p at byte a, kind 2+p at byte 63 - a (when a <= 63; a
        // dummy word otherwise), kind 4+p at byte 127 - a, each written with its new value; the
        // parity bit strings are rebuilt at the next (re)start.  No byte read above is written here
        // (the one at the mirror is the excluded shift, whose value is not used).  Every lane
        // writes: lanes 2..63 repeat lane 1's byte (the same address and value), which costs no
        // exec mask around the writes.
        {
            const uint32_t sp_a = r.sp_a, sq_a = r.sq_a, sr_a = r.sr_a;
            (void)sq_a;
            (void)sr_a;
            // (per-lane values by v_writelane: lane 0's replaces the others', no compare and select)
            const int a = write_lane<0>(r.nps, r.hjs);
            const int32_t v = write_lane<0>(-r.emir * r.sjs, -r.sjs);
            *(lds_i8 *)(uintptr_t)(sp_a + (uint32_t)a) = (int8_t)v;
            if constexpr (BIG) {
                *(lds_i8 *)(uintptr_t)(sr_a + 127u - (uint32_t)a) = (int8_t)v; // (a <= c: beyond 127 into the gap)
                const uint32_t qa = a <= 63 ? sq_a + 63u - (uint32_t)a
                                            : (uint32_t)(uintptr_t)reinterpret_cast<int8_t *>(&lds->book[7]);
                *(lds_i8 *)(uintptr_t)qa = (int8_t)v;
            } else {
                *(lds_i8 *)(uintptr_t)(sq_a + 63u - (uint32_t)a) = (int8_t)v; // (a <= c: beyond 63 into the gap)
            }
            // (the free bits in lds->xw are not kept: sync_x_lds() reads them off the strings)
        }
        lds_fence();
#pragma unroll
        for (int g = 0; g < G; g++)
            mult[g] = negate_where(flip(g) == js, mult[g]);
        if (REG_X)
            xflip_uniform(x, js);
        x0 ^= js < 32 ? 1u << js : 0u;
        if (REG_X) { // else the caller sets h (it has the neighbour's hash from its probe)
            const uint64_t z = zk[js];
            h ^= ((uint64_t)uniform((uint32_t)(z >> 32)) << 32) | uniform((uint32_t)z);
        }
        isl = isl_new;
    }

    template <bool REG_X = true>
    __device__ __forceinline__ void commit(int js, int32_t isl_new)
    {
        if constexpr (kSpecRead) {
            commit_apply<REG_X>(js, isl_new, commit_read(js));
        } else {
            // the same steps in one piece (the split form measured slower for these shapes)
            // The index arithmetic of a commit is wave-uniform and runs on the scalar unit; the vector
            // instructions are the per-lane reads, selects and updates.
            const int lane = this->lane;
            // the lane that scores js and its slot (one tile: js < 128, slot = js & 1)
            const int ol = BIG ? (js & 127) >> 1 : js >> 1;
            const int slot = BIG ? (js >> 7) * 2 + (js & 1) : js & 1;
            // mult of js at its owner lane: -8 s_js, or -4 s_c at the centre
            int32_t mj = __builtin_amdgcn_readlane(mult[0], ol);
            if constexpr (G == 2) {
                // both slots' values, then one scalar select (left to itself the compiler branches)
                const int32_t m1 = __builtin_amdgcn_readlane(mult[1], ol);
                asm("s_cmp_eq_u32 %1, 0\n\ts_cselect_b32 %0, %2, %3" : "=s"(mj) : "s"(slot), "s"(mj), "s"(m1) : "scc");
            } else {
#pragma unroll
                for (int g = 1; g < G; g++)
                    mj = slot == g ? __builtin_amdgcn_readlane(mult[g], ol) : mj;
            }
            const int32_t f = mj >> 1;                   // -4 s_js (-2 s_c at the centre)
            const int32_t sjs = ~((mj >> 31) << 1);      // s_js before the commit: -1 if mj > 0, else 1
            const int hjs = js >> 1;
            const int pis = js & 1;
            // (at the centre js = c these give kds = -1, no excluded shift, and nps = hjs)
            const int kds = c - 1 - js;                  // the excluded shift kappa_d of js
            const int nps = c - hjs - pis;               // half index of the mirror m' = 2c - js
            // byte addresses of the strings of kind p, 2+p and (big) 4+p
            typedef __attribute__((address_space(3))) const int8_t lds_ci8;
            typedef __attribute__((address_space(3))) int8_t lds_i8;
            const uint32_t s0 = (uint32_t)(uintptr_t)lds->str(0);
            const uint32_t sp_a = s0 + (uint32_t)pis * 4u * (uint32_t)(Lds::str_off(1) - Lds::str_off(0));
            const uint32_t sq_a = sp_a + 4u * (uint32_t)(Lds::str_off(2) - Lds::str_off(0));
            const uint32_t sr_a = BIG ? (uint32_t)(uintptr_t)lds->str(4) +
                                            (uint32_t)pis * 4u * (uint32_t)(Lds::str_off(5) - Lds::str_off(4))
                                      : 0u;
            // dC'_kappa = -4 s_js (p_kappa + q_kappa), p without the excluded shift kappa_d, read from
            // the +-1 byte strings (0 past either end, so lanes with kappa >= c add nothing): p from
            // s^p at hjs + 1 + kappa, q = s^p_{hjs-1-kappa} from the reversed string (s^p_{63-u}, or
            // s^p_{127-u} when half indices reach past 64); at the centre p = q and u = q, so the
            // factor is halved instead
            // (the uniform bases go through readfirstlane, a no-op on a scalar, so that the per-lane
            // offsets stay one add and the constant ones fold into the reads' offset fields)
            lds_ci8 *const pl = (lds_ci8 *)(uintptr_t)su(sp_a + (uint32_t)(hjs + 1)) + lane;
            lds_ci8 *const ql = (lds_ci8 *)(uintptr_t)su((BIG ? sr_a + 128u : sq_a + 64u) - (uint32_t)hjs) + lane;
            int32_t pv[QR], qv[QR];
#pragma unroll
            for (int q = 0; q < QR; q++) {
                pv[q] = pl[64 * q];
                qv[q] = ql[64 * q];
            }
#pragma unroll
            for (int q = 0; q < QR; q++)
                Cv[q] = mad24_u(drop_where(lane + 64 * q == kds, pv[q]) + qv[q], f, Cv[q]);
            // rc'_j of the owned flips of js's parity (see the file header).  Partner 2 j - js is s^p at
            // half index u1 = 2h - hjs >= -63 (-95 big), read from the kind-p string, whose zero pad
            // covers the negative ones; partner 2 j - m' is s^p at u2 = 2h + hjs + p - c, read as byte
            // 63 - u2 of the kind-2+p string (127 - u2 of the kind-4+p string when BIG), which holds 0
            // past the sequence's start; u2 < 64 (< 128) for every flip j < c.  Flips j >= c read
            // anything and keep it (their rc' is not used).  The term of partner 2 j - js is dropped
            // where it is the excluded shift of j (js = 3 j - 2c, i.e. 3 h = hjs + c - p), and flip js
            // itself does not change.  s_m' = (-1)^(c - js) s_js (also at the centre, where m' = js).
            const int32_t emir = pis ? -(eps8[0] >> 3) : (eps8[0] >> 3); // (-1)^(c - js)
            {
                const int32_t eps = js == c ? 0 : emir;
                const int32_t f1 = pis ? sjs : 0, f0 = sjs - f1;
                const int tri = hjs + c - pis;
                lds_ci8 *const a1 = (lds_ci8 *)(uintptr_t)su(sp_a - (uint32_t)hjs) + 2 * lane;
                lds_ci8 *const a2 =
                    (lds_ci8 *)(uintptr_t)su((BIG ? sr_a : sq_a) + (uint32_t)((BIG ? 127 : 63) - hjs - pis + c)) - 2 * lane;
#pragma unroll
                for (int t = 0; t < (BIG ? 2 : 1); t++) {
                    const int32_t h = 64 * t + lane;
                    const int32_t v1 = a1[128 * t];
                    const int32_t v2 = a2[-128 * t];
                    const int32_t d = drop_where(h == hjs, mad24_u(v2, eps, drop_where(3 * h == tri, v1)));
                    rc[2 * t] = mad24_u(d, f0, rc[2 * t]);
                    rc[2 * t + 1] = mad24_u(d, f1, rc[2 * t + 1]);
                }
            }
            // the flipped symbol (lane 0) and its mirror m' = 2c - js (lane 1; the centre again when js
            // = c) in the +-1 byte strings: kind p at byte a, kind 2+p at byte 63 - a (when a <= 63; a
            // dummy word otherwise), kind 4+p at byte 127 - a, each written with its new value; the
            // parity bit strings are rebuilt at the next (re)start.  No byte read above is written here
            // (the one at the mirror is the excluded shift, whose value is not used).  Every lane
            // writes: lanes 2..63 repeat lane 1's byte (the same address and value), which costs no
            // exec mask around the writes.
            {
                // (per-lane values by v_writelane: lane 0's replaces the others', no compare and select)
                const int a = write_lane<0>(nps, hjs);
                const int32_t v = write_lane<0>(-emir * sjs, -sjs);
                *(lds_i8 *)(uintptr_t)(sp_a + (uint32_t)a) = (int8_t)v;
                if constexpr (BIG) {
                    *(lds_i8 *)(uintptr_t)(sr_a + 127u - (uint32_t)a) = (int8_t)v; // (a <= c: beyond 127 into the gap)
                    const uint32_t qa = a <= 63 ? sq_a + 63u - (uint32_t)a
                                                : (uint32_t)(uintptr_t)reinterpret_cast<int8_t *>(&lds->book[7]);
                    *(lds_i8 *)(uintptr_t)qa = (int8_t)v;
                } else {
                    *(lds_i8 *)(uintptr_t)(sq_a + 63u - (uint32_t)a) = (int8_t)v; // (a <= c: beyond 63 into the gap)
                }
                // (the free bits in lds->xw are not kept: sync_x_lds() reads them off the strings)
            }
            lds_fence();
#pragma unroll
            for (int g = 0; g < G; g++)
                mult[g] = negate_where(flip(g) == js, mult[g]);
            if (REG_X)
                xflip_uniform(x, js);
            x0 ^= js < 32 ? 1u << js : 0u;
            if (REG_X) { // else the caller sets h (it has the neighbour's hash from its probe)
                const uint64_t z = zk[js];
                h ^= ((uint64_t)uniform((uint32_t)(z >> 32)) << 32) | uniform((uint32_t)z);
            }
            isl = isl_new;
        }
    }
};

} // namespace liblabs
