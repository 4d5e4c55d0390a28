// device_common.hpp -- wave-level building blocks for the gfx950 kernels of liblabs.
//
// Everything here assumes 64-wide wavefronts (gfx950 / CDNA4) and a workgroup made of whole
// waves.  Cross-lane work uses DPP row operations plus v_readlane, never LDS round trips.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace liblabs {

constexpr int kWave = 64;
constexpr int kLMax = 383;             // largest walk length
constexpr int kNMax = (kLMax + 1) / 2; // 192 free symbols
constexpr int kCMax = kNMax - 1;       // 191 even shifts k = 2..L-1
constexpr int kXWords = 6;             // 32-bit words of a free-bit vector
constexpr int kNA = 192;               // bit length of the reversed parity strings
constexpr int kParWords = 12;          // parity string words (incl. zero padding)
constexpr int kRevWords = 14;          // reversed parity string words (incl. zero padding)

// ------------------------------------------------------------------------------------------
// SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): the state advances by 0x9E3779B97F4A7C15 and
// each output is the state run through the finaliser below.  sm_at(s, i) is output i (from 0)
// of the generator started at state s.
// ------------------------------------------------------------------------------------------
__host__ __device__ inline uint64_t sm_finalise(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__host__ __device__ inline uint64_t sm_at(uint64_t state, uint64_t i)
{
    return sm_finalise(state + (i + 1ull) * 0x9E3779B97F4A7C15ull);
}

// Zobrist key of free symbol j.
__host__ __device__ inline uint64_t zobrist_key(int j)
{
    return sm_at(0x2011000068ABCDEFull, (uint64_t)j);
}

// ------------------------------------------------------------------------------------------
// Lane helpers.
// ------------------------------------------------------------------------------------------
__device__ inline int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

__device__ inline uint32_t readlane(uint32_t v, int l)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}

__device__ inline int32_t readlane_i(int32_t v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ inline uint32_t uniform(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }

__device__ inline uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// A wave-uniform value read from memory, moved to scalar registers so that the arithmetic that
// follows runs on the scalar unit (a vector load leaves even a uniform value in VGPRs).
__device__ inline uint32_t su(uint32_t v) { return uniform(v); }
__device__ inline int32_t su(int32_t v) { return (int32_t)uniform((uint32_t)v); }
__device__ inline uint64_t su(uint64_t v)
{
    return ((uint64_t)uniform((uint32_t)(v >> 32)) << 32) | uniform((uint32_t)v);
}
__device__ inline int64_t su(int64_t v) { return (int64_t)su((uint64_t)v); }

// DPP move of src into the lane layout given by CTRL (rows of 16 lanes); lanes whose source is
// outside the row (or disabled by the masks) get `old`.
template <int CTRL, int ROW_MASK = 0xf, int BANK_MASK = 0xf>
__device__ inline int32_t dpp(int32_t old, int32_t src)
{
    return __builtin_amdgcn_update_dpp(old, src, CTRL, ROW_MASK, BANK_MASK, false);
}

constexpr int kQuadSwap1 = 0xB1;     // quad_perm [1,0,3,2]
constexpr int kQuadSwap2 = 0x4E;     // quad_perm [2,3,0,1]
constexpr int kRowHalfMirror = 0x141;
constexpr int kRowMirror = 0x140;
constexpr int kRowShr1 = 0x111;
constexpr int kRowShr2 = 0x112;
constexpr int kRowShr4 = 0x114;
constexpr int kRowShr8 = 0x118;
constexpr int kRowBcast15 = 0x142;
constexpr int kRowBcast31 = 0x143;

// Wave reductions.  Each step moves the partner value with DPP and combines it; the `old`
// operand of every move is the identity of the combining operation, which lets the compiler fold
// the move into the ALU instruction (one v_<op>_dpp per step).  Rows of 16 lanes are reduced with
// quad / half-row / row mirrors; rows are then combined with row_bcast:15 and row_bcast:31, after
// which lane 63 holds the result.
template <typename Op>
__device__ inline uint32_t wave_reduce_u32(uint32_t v, uint32_t identity, Op op)
{
    const int id = (int)identity;
    v = op(v, (uint32_t)dpp<kQuadSwap1>(id, (int)v));
    v = op(v, (uint32_t)dpp<kQuadSwap2>(id, (int)v));
    v = op(v, (uint32_t)dpp<kRowHalfMirror>(id, (int)v));
    v = op(v, (uint32_t)dpp<kRowMirror>(id, (int)v));
    v = op(v, (uint32_t)dpp<kRowBcast15, 0xa>(id, (int)v));
    v = op(v, (uint32_t)dpp<kRowBcast31, 0xc>(id, (int)v));
    return readlane(v, 63);
}

struct OpMinU { __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return min(a, b); } };
struct OpOrU { __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a | b; } };
struct OpXorU { __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a ^ b; } };
struct OpAddU { __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a + b; } };

// Minimum of v over the wave (uniform result).
__device__ inline uint32_t wave_min_u32(uint32_t v) { return wave_reduce_u32(v, 0xFFFFFFFFu, OpMinU()); }

// Bitwise OR of v over the wave (uniform result).
__device__ inline uint32_t wave_or_u32(uint32_t v) { return wave_reduce_u32(v, 0u, OpOrU()); }

__device__ inline int32_t wave_sum_i32(int32_t v) { return (int32_t)wave_reduce_u32((uint32_t)v, 0u, OpAddU()); }

__device__ inline uint32_t wave_xor_u32(uint32_t v) { return wave_reduce_u32(v, 0u, OpXorU()); }

__device__ inline uint64_t wave_xor_u64(uint64_t v)
{
    uint32_t lo = wave_xor_u32((uint32_t)v);
    uint32_t hi = wave_xor_u32((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Inclusive prefix sum of v over lanes 0..63 (lane l gets v_0 + ... + v_l).
__device__ inline int32_t wave_inclusive_scan(int32_t v)
{
    v += dpp<kRowShr1>(0, v);
    v += dpp<kRowShr2>(0, v);
    v += dpp<kRowShr4>(0, v);
    v += dpp<kRowShr8>(0, v);
    v += dpp<kRowBcast15, 0xa>(0, v);
    v += dpp<kRowBcast31, 0xc>(0, v);
    return v;
}

// Low r bits set (r <= 0 -> 0, r >= 32 -> all).
__device__ inline uint32_t low_mask(int r)
{
    return r >= 32 ? 0xFFFFFFFFu : (r <= 0 ? 0u : ((1u << r) - 1u));
}

__device__ inline uint32_t funnel(uint32_t hi, uint32_t lo, int sh)
{
    return __builtin_amdgcn_alignbit(hi, lo, (uint32_t)sh);
}

__device__ inline int popc(uint32_t v) { return __builtin_popcount(v); }

// popcount(x) + acc as one v_bcnt_u32_b32; written as an instruction so that a run of them stays
// a dependent chain instead of being re-associated into separate popcounts and adds.
__device__ inline uint32_t bcnt_acc(uint32_t x, uint32_t acc)
{
    uint32_t r;
    asm("v_bcnt_u32_b32 %0, %1, %2" : "=v"(r) : "v"(x), "v"(acc));
    return r;
}

// v with lane L replaced by the wave-uniform x (one v_writelane_b32; readfirstlane, free on a value
// already in a scalar register, makes x a scalar operand, and the lane is an inline constant)
template <int L>
__device__ inline int32_t write_lane(int32_t v, int32_t x)
{
    static_assert(L >= 0 && L < 64, "a lane of the wave");
    asm("v_writelane_b32 %0, %1, %2" : "+v"(v) : "s"(__builtin_amdgcn_readfirstlane(x)), "n"(L));
    return v;
}

// a * b + acc for a, b in the signed 24-bit range, as one full-rate v_mad_i32_i24 (the generic
// 32-bit multiply is a multi-pass instruction).
__device__ inline int32_t mad24(int32_t a, int32_t b, int32_t acc)
{
    int32_t r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(acc));
    return r;
}

// the same with a wave-uniform b
__device__ inline int32_t mad24_u(int32_t a, int32_t b, int32_t acc)
{
    int32_t r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(acc));
    return r;
}

} // namespace liblabs
