// internal.hpp -- structures and launch wrappers shared by the host side of liblabs and its
// kernels (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/labs.h"
#include "device_common.hpp"

namespace liblabs {

enum : int32_t { kFresh = 0, kRunning = 1, kDone = 2 };

// Per-walk state resident in HBM between kernel launches.  The host writes the configuration
// and status = kFresh; from then on only the kernels write it.  Everything a walk needs to
// resume is here: the correlation table and bit strings are rebuilt from x at the start of
// every launch.
struct alignas(16) WalkState {
    // configuration
    int32_t L;
    int32_t table_log2;
    uint64_t seed;
    uint32_t walk_id;
    uint32_t flags;
    int64_t steps;
    int64_t restart_period;
    int64_t target_isl;
    int64_t watch_isl;
    int64_t table_offset; // first table word of this walk (64-bit words)
    int64_t trace_offset; // first trace record (2 int32) of this walk, -1 = none
    int64_t score_offset; // first score entry (int32) of this walk, -1 = none
    int64_t step_cap;     // a launch never takes the walk past this step
    // progress
    int64_t t;
    int64_t flips;
    int64_t hit_step;
    int64_t watch_step;
    int64_t best_isl;
    int64_t best_step;
    uint64_t h;
    int32_t isl;
    int32_t restart_idx;
    int32_t restarts;
    int32_t traps;
    int32_t status;
    int32_t table_epoch; // epoch of the visited table's entries, 0 = contents unknown
    uint32_t x[kXWords];
    uint32_t best_x[kXWords];
};

// Launch parameters of the walk kernel (all results are independent of them).
struct WalkLaunch {
    int32_t variant;         // LABS_VARIANT_BITSLICE or LABS_VARIANT_DIRECT
    int32_t waves_per_block; // 1, 2, 4 or 8
    int32_t probe_width;     // 1..4
    int32_t shape;           // kernel instantiation, see shape_for_length()
    int64_t chunk;           // steps per launch
    int32_t persistent;      // 1 = grid of resident waves pulling walks from a counter
    int32_t grid_waves;      // persistent: number of waves launched
};

// Kernel instantiation for length L: flip groups G = ceil(n/64), table words KW = ceil(c/32).
int shape_for_length(int L);
int shape_groups(int shape);
// Waves of the walk kernel chosen by lp that fit on the device at once (0 if unknown).
int resident_walk_waves(const WalkLaunch &lp);

// Launch wrappers (walk_kernels.hip).
hipError_t launch_walk(const WalkLaunch &lp, WalkState *states, int32_t n_walks,
                       const int32_t *order, uint64_t *tables, int32_t *trace, int32_t *scores,
                       int32_t *counter, hipStream_t stream);
hipError_t launch_reset(WalkState *states, const WalkState *pristine, int32_t n_walks,
                        int32_t *counter, hipStream_t stream);
hipError_t launch_zero_counter(int32_t *counter, hipStream_t stream);
hipError_t launch_flip_scores(int32_t variant, int L, int count, const uint32_t *x,
                              int32_t *scores, hipStream_t stream);
hipError_t launch_isl_batch(int L, int count, const int8_t *s, int64_t *isl, double *F,
                            int32_t *psl, int32_t *corr, hipStream_t stream);
hipError_t launch_enum_skew(int L, int32_t *isl, hipStream_t stream);
// LDS read-bandwidth probe (probe_kernels.hip): blocks of lds_probe_threads() threads, each
// lane reading bytes_per_lane (4, 8 or 16) bytes per read; out holds one word per thread.
int lds_probe_threads();
double lds_probe_bytes(int bytes_per_lane, int blocks, int rounds);
hipError_t launch_lds_read_probe(int bytes_per_lane, int blocks, int rounds, uint32_t *out, hipStream_t stream);
int general_shape_for_length(int L);
hipError_t launch_general_flip_scores(int L, int count, const uint32_t *x, int32_t *scores, hipStream_t stream);
constexpr int kMfmaLMax = 383;     // the matrix-core scoring covers every walk length
constexpr int kMfmaAutoLMin = 3; // the matrix-core walker was measured faster at every length
hipError_t launch_flip_scores_mfma(int L, int count, const uint32_t *x, int32_t *scores, hipStream_t stream);
size_t mfma_wave_lds_bytes(int shape); // per walk (shape < 0: mixed lengths)
hipError_t launch_walk_general(int shape, WalkState *states, int32_t count, const int32_t *order, uint64_t *tables,
                               int32_t *trace, int32_t *scores, hipStream_t stream);
hipError_t launch_pq_walk(int shape, WalkState *states, int32_t count, const int32_t *order, uint64_t *tables,
                          uint64_t *nbr_tables, int nlog2, int cap, int32_t *trace, int32_t *scores,
                          hipStream_t stream);
// first-improvement search with perturbations of P symbols (fi_walk.hip); no visited table
hipError_t launch_fi_walk(int shape, WalkState *states, int32_t count, const int32_t *order, int P, int32_t *trace,
                          int32_t *scores, hipStream_t stream);

// Running result of one grouped skew-space minimum (one slot per block, then one final slot).
struct EnumPartial {
    uint32_t min_isl; // 0xFFFFFFFF: nothing covered yet
    uint32_t reserved;
    uint64_t count;
    uint64_t first_x;
    uint64_t word_ops; // algorithmic word operations of the (sequence, lag) pairs evaluated
};
int enum_min_blocks(int L);
hipError_t launch_enum_part_init(EnumPartial *part, int count, hipStream_t stream);
hipError_t launch_enum_min(int L, uint64_t r_begin, uint64_t r_count, EnumPartial *part, int blocks,
                           hipStream_t stream);
hipError_t launch_enum_final(const EnumPartial *part, int count, EnumPartial *out, hipStream_t stream);

} // namespace liblabs
