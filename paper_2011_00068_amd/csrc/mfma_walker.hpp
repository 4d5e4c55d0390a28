// mfma_walker.hpp -- the skew walker with its flip scoring on the matrix cores (gfx950
// v_mfma_i32_16x16x64_i8), for L <= 255 (c <= 127).
//
// The expensive part of scoring is, for every flip j = 2h + p (parity p = j & 1, h = j >> 1),
//   Y_j = sum_kappa C'_kappa b^p_{h+1+kappa}   and   Z_j = sum_kappa C'_kappa b^p_{h-1-kappa},
// with C'_kappa = C_{2 kappa + 2} and b^p_u = b_{2u+p} the bits of the parity-p half of the
// sequence (Y + Z is sum_k C_k (Wp + Wq) of the bit-sliced walker; the assembly of ISL_j from it
// is the same).  Both are correlations of the small integer vector C' with 0/1 strings, i.e.
// products of a 0/1 Hankel matrix with a Toeplitz arrangement of C'.  One 16x16 tile holds all
// of them: row m = 4 i + kind, column nn, h = 16 i + nn, K index t = kappa + 1 + nn:
//   A[m][t] = S_kind[t + 16 i]   (kind 0/1: b^0, b^1;  kind 2/3: b^p_{63-u}, so that row kind 2+p
//                                 column nn yields Z at h' = 63 - h),
//   B[t][nn] = C'_{t-1-nn}        (0 outside 0 <= t-1-nn < c),
// so D[m][nn] = sum_t A B is Y (kind p) at h and Z (kind 2+p) at 63 - h.  Every A row is an
// aligned 16-byte window of a byte copy of one string (no shifted copies needed); every B column
// is a 16-byte window of C' starting at byte t0 - 1 - nn, read from whichever of four copies of C'
// shifted by 0..3 bytes puts it on a dword boundary (each step writes C' into all four).  K = 64 KB covers
// t <= c + 15.  C' fits int8 unless |C_k| > 127; then C' = 64 hi + lo (lo in 0..63, hi in
// -4..3) and a second pass adds 64 x the hi tile.  Lane layout of the instruction (checked on
// gfx950): lane l holds row / column l % 16 of A / B and K slice 16 (l / 16) .. +15 in its four
// registers' bytes, and D register r of lane l is D[4 (l / 16) + r][l % 16]; so lane l receives
// Y_j, Y_{j+1} for h = l and Z for h = 63 - l, which one ds_bpermute brings to lane h.
//
// Lane l owns flips j = 2 l and 2 l + 1; the correlation table (lane-held C), its prefix sums,
// the parity bit strings, the commit and the rest of the assembly are the bit-sliced walker's.
#pragma once

#include "walk_impl.hpp"

namespace liblabs {

typedef int mfma_v4i __attribute__((ext_vector_type(4)));

constexpr int kMfmaSeqDwords = 64; // 256 bytes per string copy
constexpr int kMfmaSeqStride = 66; // copies 2 dwords apart in bank order: the four copies read by one
                                   // A load fall on two bank sets instead of one
constexpr int kMfmaCDwords = 56;   // one copy of C': byte 20 + kappa - r in copy r, zero elsewhere
constexpr int kMfmaCBytes = 4 * kMfmaCDwords;

struct WaveLdsMfma : WaveLdsBits {
    uint32_t sb[4][kMfmaSeqStride]; // byte copies of the A strings (first kMfmaSeqDwords used)
    uint32_t cb[4][kMfmaCDwords];   // C' as int8, four copies shifted by 0..3 bytes
};

__device__ __forceinline__ uint32_t nibble_bytes(uint32_t nib)
{
    // 4 bits -> 4 bytes of 0/1 (the shifted copies never overlap, so the product has no carries)
    return (nib * 0x00204081u) & 0x01010101u;
}

__device__ __forceinline__ uint32_t alignbyte(uint32_t hi, uint32_t lo, uint32_t sh)
{
    return __builtin_amdgcn_alignbyte(hi, lo, sh);
}

template <int KW>
struct MfmaWalker {
    static constexpr int kG = 2;
    static constexpr int G = 2;
    static constexpr int QR = (KW + 1) / 2;
    static constexpr int KB = (32 * KW + 16 + 63) / 64; // K blocks of 64
    using Lds = WaveLdsMfma;

    int L, c, n;
    int lane;
    int32_t isl;
    uint64_t h;
    uint32_t x[kXWords];
    int32_t Cv[QR];
    int32_t sbit[G];
    int planes;
    Lds *lds;
    const uint64_t *zk;
    FlipConst fc[G];

    __device__ __forceinline__ int flip(int g) const { return 2 * lane + g; }

    __device__ __forceinline__ void set_length(int len)
    {
        L = len;
        c = (L - 1) / 2;
        n = c + 1;
    }

    __device__ __forceinline__ void init_lanes(int ln)
    {
#pragma unroll
        for (int g = 0; g < G; g++) {
            const int j = min(2 * ln + g, c);
            const int p = j & 1, hj = j >> 1;
            const int nq = hj;
            const int np = c - ((j + 1) >> 1);
            FlipConst &f = fc[g];
            f.sp = (uint32_t)(hj + 1);
            f.wp = &lds->par[p][(hj + 1) >> 5];
            f.wq = &lds->rev[p][(kNA - hj) >> 5];
            f.psx_np = &lds->psx[np];
            f.psx_nq = &lds->psx[nq];
            f.c_kd = &lds->C[max(c - 1 - j, 0)];
            const int iq = 3 * j - 2 * c;
            const int a = max(iq, 0) >> 1;
            f.qd_word = &lds->par[p][a >> 5];
            f.qd_shift = (uint32_t)(a & 31);
            f.m_par = (uint32_t)((c - j) & 1);
            f.hconst = np + 3 * nq - 1;
            f.nq = nq;
        }
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
        for (int i = lane; i < 4 * kMfmaCDwords; i += kWave)
            lds->cb[i / kMfmaCDwords][i % kMfmaCDwords] = 0u;
        lds_fence();
        // byte copies of the strings: kind p from par[p] at bit u, kind 2+p from rev[p] at bit
        // 128 + u (= b^p_{63-u}, zero past u = 63)
#pragma unroll
        for (int k4 = 0; k4 < 4; k4++) {
            const int p = k4 & 1;
            const int bitpos = (k4 < 2 ? 0 : 128) + 4 * lane;
            const uint32_t word = (k4 < 2) ? lds->par[p][bitpos >> 5] : lds->rev[p][bitpos >> 5];
            lds->sb[k4][lane] = nibble_bytes((word >> (bitpos & 31)) & 0xFu);
        }
#pragma unroll
        for (int g = 0; g < G; g++) {
            const int j = 2 * lane + g;
            sbit[g] = (j <= c) ? (int32_t)seq_bit(j) : 0;
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
            const int j = 2 * lane + g;
            if (j <= c && sbit[g])
                hz ^= zk[j];
        }
        h = wave_xor_u64(hz);
        lds_fence();
    }

    // C to LDS, prefix sums, whether C' fits int8; C' bytes for the B operand.
    __device__ __forceinline__ void prepare()
    {
        const int lane = this->lane;
        int32_t running = 0;
        bool wide = false; // some |C_k| above the int8 range
#pragma unroll
        for (int q = 0; q < QR; q++) {
            const int kappa = lane + 64 * q;
            lds->C[kappa] = Cv[q];
            const int32_t inc = wave_inclusive_scan(Cv[q]) + running;
            lds->psx[kappa + 1] = inc;
            running = readlane_i(inc, 63);
            wide = wide || (uint32_t)(Cv[q] + 128) > 255u;
        }
        if (lane == 0)
            lds->psx[0] = 0;
        planes = ballot(wide) != 0ull ? 9 : 8; // only "fits int8 or not" is used
        put_c(planes <= 8 ? 0 : 1); // C' itself, or its low six bits (the high part follows later)
        lds_fence();
    }

    // C' bytes into the four shifted copies: part 0 C' itself, part 1 its low six bits (0..63),
    // part 2 C' >> 6 (-4..3 for |C'| <= 253).
    __device__ __forceinline__ void put_c(int part)
    {
        int8_t *cp = reinterpret_cast<int8_t *>(lds->cb[0]) + 20 + lane;
#pragma unroll
        for (int q = 0; q < QR; q++) {
            const int32_t v = part == 0 ? Cv[q] : (part == 1 ? (Cv[q] & 63) : (Cv[q] >> 6));
#pragma unroll
            for (int r = 0; r < 4; r++)
                cp[64 * q + r * (kMfmaCBytes - 1)] = (int8_t)v;
        }
    }

    // One K-sweep of the tile with the C' bytes now in the copies.  Lane (slice, nn) needs the
    // 16 bytes C'_{i0 .. i0+15}, i0 = t0 - 1 - nn; copy r = (i0 + 20) mod 4 holds them from a
    // dword boundary.
    __device__ __forceinline__ mfma_v4i tile() const
    {
        const int lane = this->lane;
        const int nn = lane & 15, slice = lane >> 4;
        const int kind = lane & 3, ib = (lane & 15) >> 2;
        const int r = (3 - nn) & 3;
        mfma_v4i acc = {0, 0, 0, 0};
#pragma unroll
        for (int kb = 0; kb < KB; kb++) {
            const int t0 = 16 * slice + 64 * kb;
            const uint32_t *ap = &lds->sb[kind][(t0 + 16 * ib) >> 2];
            const mfma_v4i a = {(int)ap[0], (int)ap[1], (int)ap[2], (int)ap[3]};
            const uint32_t *bp = &lds->cb[r][(t0 - 1 - nn + 20 - r) >> 2];
            const mfma_v4i b = {(int)bp[0], (int)bp[1], (int)bp[2], (int)bp[3]};
            acc = __builtin_amdgcn_mfma_i32_16x16x64_i8(a, b, acc, 0, 0, 0);
        }
        return acc;
    }

    __device__ __forceinline__ void score(int32_t (&isl_j)[G])
    {
        const int lane = this->lane;
        mfma_v4i d = tile();
        if (planes > 8) {
            // C' = 64 hi + lo: the copies held lo; the wave's LDS operations run in order, so the
            // reads above complete before the hi bytes overwrite them
            put_c(2);
            lds_fence();
            const mfma_v4i hi = tile();
            d = d + hi * 64;
        }
        // Z for h = lane sits in lane 63 - lane
        const int src = (63 - lane) << 2;
        int32_t acc[G];
        acc[0] = d[0] + __builtin_amdgcn_ds_bpermute(src, d[2]);
        acc[1] = d[1] + __builtin_amdgcn_ds_bpermute(src, d[3]);
#pragma unroll
        for (int g = 0; g < G; g++) {
            const FlipConst &f = fc[g];
            // R_j = nq - 2 rc, rc = differing bits of Wp and Wq over the both-sided shifts
            // (kappa < nq <= 63: two window words)
            const uint32_t wp0 = funnel(f.wp[1], f.wp[0], (int)f.sp);
            const uint32_t wp1 = funnel(f.wp[2], f.wp[1], (int)f.sp);
            const uint32_t wq0 = funnel(f.wq[1], f.wq[0], (int)(1u - f.sp));
            const uint32_t wq1 = funnel(f.wq[2], f.wq[1], (int)(1u - f.sp));
            uint32_t rc = bcnt_acc((wp0 ^ wq0) & low_mask(f.nq), 0u);
            rc = bcnt_acc((wp1 ^ wq1) & low_mask(f.nq - 32), rc);
            const int32_t Cd = *f.c_kd;
            const int32_t pnp = *f.psx_np, pnq = *f.psx_nq;
            const uint32_t qbit = (*f.qd_word >> f.qd_shift) & 1u;
            const uint32_t m_neg = (uint32_t)sbit[g] ^ f.m_par;
            const int j = 2 * lane + g;
            const bool centre = j == c;
            const bool qd_valid = 3 * j >= 2 * c;
            const int32_t smqd = qd_valid ? ((m_neg ^ qbit) ? -1 : 1) : 0;
            const int32_t Gg = pnp + pnq - 2 * acc[g] - (m_neg ? -Cd : Cd);
            const int32_t Hg = f.hconst - 4 * (int32_t)rc - 2 * smqd;
            const int32_t Gj = centre ? pnq - acc[g] : Gg;
            const int32_t Hj = centre ? f.nq : Hg;
            isl_j[g] = isl + (sbit[g] ? 8 * Gj : -8 * Gj) + 16 * Hj;
        }
    }

    __device__ __forceinline__ void commit(int js, int32_t isl_new)
    {
        const int lane = this->lane;
        const int32_t sjs = 1 - 2 * (int32_t)xbit_uniform(x, js);
        const int hjs = js >> 1;
        const int pis = js & 1;
        const int nps = (js == c) ? 0 : c - ((js + 1) >> 1);
        const int kds = (js == c) ? -1 : c - 1 - js;
#pragma unroll
        for (int q = 0; q < QR; q++) {
            const int kappa = lane + 64 * q;
            if (kappa < c) {
                const int ip = hjs + 1 + kappa;
                const uint32_t bp = (lds->par[pis][ip >> 5] >> (ip & 31)) & 1u;
                const int32_t pv = (kappa < nps && kappa != kds) ? 1 - 2 * (int32_t)bp : 0;
                int32_t qv = 0;
                const int iq = hjs - 1 - kappa;
                if (iq >= 0)
                    qv = 1 - 2 * (int32_t)((lds->par[pis][iq >> 5] >> (iq & 31)) & 1u);
                Cv[q] += -4 * sjs * (pv + qv);
            }
        }
        lds_fence();
        // the flipped symbol and its mirror (m = 2c - js, half index nps) in the bit strings and
        // in the byte copies (kind p at byte a, kind 2+p at byte 63 - a when a <= 63)
        if (lane < 4 && ((lane & 1) == 0 || js != c)) {
            const int a = (lane & 1) ? nps : hjs;
            if (lane < 2) {
                atomicXor(&lds->par[pis][a >> 5], 1u << (a & 31));
                const int ar = kNA - 1 - a;
                atomicXor(&lds->rev[pis][ar >> 5], 1u << (ar & 31));
                atomicXor(&lds->sb[pis][a >> 2], 1u << (8 * (a & 3)));
            } else {
                const int u = 63 - a;
                if (u >= 0)
                    atomicXor(&lds->sb[2 + pis][u >> 2], 1u << (8 * (u & 3)));
            }
        }
        lds_fence();
#pragma unroll
        for (int g = 0; g < G; g++)
            sbit[g] ^= (2 * lane + g == js) ? 1 : 0;
        xflip_uniform(x, js);
        const uint64_t z = zk[js];
        h ^= ((uint64_t)uniform((uint32_t)(z >> 32)) << 32) | uniform((uint32_t)z);
        isl = isl_new;
    }
};

} // namespace liblabs
