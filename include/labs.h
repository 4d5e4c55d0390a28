/*
 * labs.h -- C ABI of liblabs, a gfx950 (MI355X) implementation of the hot path of the
 * stochastic skew-symmetric LABS search of
 *   J. Brest, B. Boskovic, "Computational Search of Long Skew-symmetric Binary Sequences with
 *   High Merit Factors", arXiv:2011.00068.
 *
 * Vocabulary (the paper's notation, 0-based indices):
 *   S = (s_0 .. s_{L-1}), s_i in {+1,-1}                                  (Section 1)
 *   C_k = sum_{i=0}^{L-k-1} s_i s_{i+k}                                   (Eq. (1))
 *   ISL = sum_{k=1}^{L-1} C_k^2                                           (Eq. (2))
 *   F   = L^2 / (2 ISL)                                                   (Eq. (3))
 *   skew-symmetric: L = 2n-1, centre c = n-1, s_{c+i} = (-1)^i s_{c-i}    (Eq. (4), re-indexed
 *   from the paper's 1-based form; Table 1's sequences satisfy this reading)
 *   free bits x: bit j (32-bit word j/32, bit j%32) is 1 <=> s_j = -1, j = 0..c (the paper's
 *   0 -> +1, 1 -> -1 convention of Section 4).
 *   flip j (0 <= j <= c): negate s_j and its mirror s_{L-1-j} (one symbol when j == c).
 *
 * Conventions for every entry point:
 *   - Return value: LABS_OK (0) or a negative LABS_E* code; nothing throws or aborts across the
 *     ABI.  labs_strerror() names a code; labs_last_error() gives a message for the calling
 *     thread's last failure.
 *   - "host" pointers are ordinary CPU memory owned by the caller; the library copies out of /
 *     into them before returning.  "device" pointers are HIP device memory (hipMalloc or a torch
 *     CUDA tensor) owned by the caller; the library only reads / writes them.
 *   - Entry points that run walks or searches take n_walks >= 1 (LABS_EINVAL for 0 or less,
 *     checked before any device work); the batched sequence entry points accept count = 0.
 *   - stream: a hipStream_t passed as void*; NULL = the default (null) stream.  Entry points
 *     whose name ends in _dev are asynchronous on that stream unless stated otherwise; all
 *     others are synchronous.
 *   - Every computation of the search runs in the library's gfx950 kernels; there is no CPU
 *     fallback.  A missing or unusable GPU returns LABS_EDEVICE.  (labs_isl_threshold, which only
 *     converts a stop parameter, and labs_from_hex / labs_to_hex, which convert sequence notation,
 *     are host code.)
 */
#ifndef LABS_H
#define LABS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LABS_OK 0
#define LABS_EINVAL (-1)     /* bad argument (size, range, symbol not +1/-1, NULL pointer) */
#define LABS_ENOTSKEW (-2)   /* a skew-only entry point got a sequence that violates Eq. (4) */
#define LABS_ENOMEM (-3)     /* device or host allocation failed, or request above a budget */
#define LABS_EPENDING (-4)   /* job not finished yet (labs_search_poll) */
#define LABS_ENOTFOUND (-5)  /* unknown job id */
#define LABS_EDEVICE (-6)    /* HIP runtime error / no usable gfx950 device */
#define LABS_EDOM (-7)       /* result undefined (F for ISL = 0, i.e. L = 1) */
#define LABS_ECANCELLED (-8) /* job was cancelled */

/* Largest L accepted by the walk entry points (n = (L+1)/2 <= 192 free symbols). */
#define LABS_WALK_L_MAX 383
/* 32-bit words of a free-bit vector in the walk structures. */
#define LABS_X_WORDS 6

const char *labs_strerror(int status);
const char *labs_last_error(void);

/* Device this library runs on: fills name (NUL-terminated, cap bytes), compute-unit count and
 * shader clock (kHz).  Returns LABS_EDEVICE when no gfx950 device is visible. */
int labs_device_info(char *name, int32_t cap, int32_t *compute_units, int32_t *clock_khz);

/* Measurement aid (no operation of the paper): the LDS read bandwidth of the device, for the LDS
 * roof of the walk kernels.  A kernel of 256-thread blocks (16 per compute unit, 64 KB of LDS
 * each) streams conflict-free reads of bytes_per_lane = 4, 8 or 16 bytes per lane out of LDS;
 * *bytes_per_s receives the bytes read per second of the fastest of five timed launches (HIP
 * events on the default stream), *ms_out (may be NULL) that launch's time.  Synchronous; allocates
 * and frees a small device buffer.  LABS_EINVAL for another width or a NULL bytes_per_s. */
int labs_probe_lds_read(int32_t bytes_per_lane, double *bytes_per_s, double *ms_out);

/* ---------------------------------------------------------------------------------------------
 * Definitions of Section 1.
 * ------------------------------------------------------------------------------------------- */

/* ISL of one sequence (Eq. (2), with C_k of Eq. (1)).  s: host, L int8 symbols, each +1 or -1
 * (else LABS_EINVAL).  Any 1 <= L <= 65535.  isl_out: host. */
int labs_isl(int32_t L, const int8_t *s, int64_t *isl_out);

/* Merit factor of one sequence (Eq. (3)).  As labs_isl; L == 1 (ISL = 0) gives LABS_EDOM. */
int labs_merit(int32_t L, const int8_t *s, double *F_out);

/* Integer form of a merit-factor threshold (Eq. (3)): F >= num/den holds at length L exactly when
 * ISL <= floor(L^2 * den / (2 * num)), since F = L^2 / (2 ISL) with ISL > 0.  Walks, searches and
 * the server compare integer ISL with this bound, never a rounded F.  Host integer arithmetic only
 * (a conversion of a stop parameter; no device work).  1 <= L <= 65535, num > 0, den > 0, else
 * LABS_EINVAL; a bound above INT64_MAX is clamped to it.  isl_out: host. */
int labs_isl_threshold(int32_t L, int64_t num, int64_t den, int64_t *isl_out);

/* Table 1's sequence notation (Section 4): each hex digit gives 4 bits, most significant first;
 * leading 0 bits are dropped down to L symbols; bit 0 is +1 and bit 1 is -1.  Host code only (a
 * conversion of inputs and outputs, no device work).
 *   labs_from_hex: hex is a NUL-terminated string of 0-9, a-f, A-F with at least L bits; every
 *     dropped bit must be 0.  s_out: host, L int8 symbols, written only on success.  LABS_EINVAL for
 *     another character, too few bits, a dropped bit 1, L outside [1, 65535] or a NULL pointer.
 *   labs_to_hex: the shortest form, ceil(L/4) upper-case digits (the first digit holds the
 *     4 ceil(L/4) - L zero pad bits), then a NUL.  out: host, cap bytes, at least ceil(L/4) + 1.
 *     LABS_EINVAL for a symbol other than +1 / -1, a short cap, L outside [1, 65535] or a NULL
 *     pointer (out's contents are then unspecified). */
int labs_from_hex(const char *hex, int32_t L, int8_t *s_out);
int labs_to_hex(int32_t L, const int8_t *s, char *out, int32_t cap);

/* Batched Eq. (1)-(3) and the PSL of Section 1 (max_{k>=1} |C_k|) for `count` sequences of
 * length L stored back to back (row r at s_dev + r*L).  Device buffers: s_dev (count*L int8),
 * isl_dev (count int64), F_dev (count double, -1.0 where ISL = 0; may be NULL), psl_dev (count
 * int32; may be NULL), corr_dev (count*L int32 holding C_0..C_{L-1}; may be NULL).  Symbols
 * outside {+1,-1} are not checked on this path (the host entry points check them); 1 <= L <=
 * 65535.  Asynchronous on stream. */
int labs_isl_batch_dev(int32_t L, int32_t count, const int8_t *s_dev, int64_t *isl_dev,
                       double *F_dev, int32_t *psl_dev, int32_t *corr_dev, void *stream);

/* Exhaustive enumeration of the 2^n skew-symmetric sequences of odd length L (Eq. (4); the
 * search-space reduction of Section 1).  isl_dev: device, 2^n int32; entry x is the ISL of the
 * sequence whose free bits are x.  Odd 3 <= L <= 47 (n <= 24).  Asynchronous on stream. */
int labs_enum_skew_dev(int32_t L, int32_t *isl_dev, void *stream);

/* Lowest ISL over the skew-symmetric sequences of odd length L, or over a block of them (Eq. (2),
 * (4); Section 1's search-space reduction), without storing per-sequence values.  Negation
 * (x -> x ^ A, A = all n free bits) and alternation s_i -> (-1)^i s_i (x -> x ^ O, O = the free
 * bits at odd positions j) preserve skew symmetry and ISL; group r (0 <= r < 2^(n-2)) is
 * {x, x^A, x^O, x^A^O} with x = r << 2, and the groups partition the 2^n sequences.  The call
 * covers groups r_begin .. r_end - 1 (r_begin = 0, r_end = 2^(n-2): the whole space) and reports
 * the lowest ISL, how many covered sequences reach it (always a multiple of 4), the lowest such
 * free-bit vector x (bit j = 1 <=> s_j = -1), the sequences covered, the device time of the
 * enumeration kernels, and the work they did: word_ops sums 3 ceil((L-k)/32) + 2 word operations
 * (funnel shift, masked xor and popcount per 32-bit word of the L-k overlapping positions, then
 * C_k^2) over the (sequence, even lag k) pairs evaluated.  The search is branch and bound: once
 * the partial ISL of every sequence of a pass exceeds the lowest ISL found, the pass's remaining
 * lags are skipped (they cannot change the minimum, its multiplicity or its lowest argument), so
 * word_ops is below the exhaustive count.  Odd 3 <= L <= 125 (n <= 63).  An empty block (r_begin
 * == r_end) gives min_isl = -1, count = first_x = states = word_ops = 0.  Blocking: the work runs
 * on `stream` (NULL = the default stream) and the call returns when it is done; it allocates and
 * frees a small device buffer (32 bytes per resident block).  LABS_EINVAL for a bad L, r_begin >
 * r_end or r_end > 2^(n-2). */
typedef struct labs_enum_min_result {
    int32_t min_isl;
    int32_t reserved;
    uint64_t count;
    uint64_t first_x;
    uint64_t states;
    double kernel_ms;
    uint64_t word_ops;
} labs_enum_min_result;

int labs_enum_skew_min(int32_t L, uint64_t r_begin, uint64_t r_end, labs_enum_min_result *out,
                       void *stream);

/* labs_enum_skew_min for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same arguments and results, except
 * kernel_ms = -1 (not timed: timing would create events).  It calls no hipMalloc, hipFree or other
 * allocating routine: its per-block partial results live in a fixed device array of 4096 slots of
 * 32 bytes (128 KiB) that each GPU the library runs on holds from the first call on it until the
 * process ends (a device with more than 4095 resident enumeration blocks runs a smaller grid; the
 * results do not depend on the grid).  Every call clears the slots it uses before it starts, so
 * nothing carries over between calls, but all calls on one GPU share the array: calls that
 * overlap in time on one GPU (from several threads or streams) race and must not be made.
 * Blocking on `stream`.  Errors as labs_enum_skew_min. */
int labs_enum_skew_min_noalloc(int32_t L, uint64_t r_begin, uint64_t r_end, labs_enum_min_result *out,
                               void *stream);

/* ---------------------------------------------------------------------------------------------
 * One-flip evaluation (Section 3; Algorithm 1's fast merit-factor step).
 * ------------------------------------------------------------------------------------------- */

/* Scores of every flip of `count` skew-symmetric states of odd length L, 3 <= L <=
 * LABS_WALK_L_MAX: scores_dev[r*n + j] = ISL of state r with flip j applied, computed from the
 * state's correlation table as the walk does.  x_dev: device, count * LABS_X_WORDS uint32
 * (bits at j >= n must be 0; not checked).  variant: LABS_VARIANT_* below (AUTO = BITSLICE
 * here).
 * Asynchronous on stream; LABS_EINVAL for a bad L, count < 0, NULL buffers with count > 0, an
 * unknown variant, or LABS_VARIANT_MFMA beyond its range. */
int labs_flip_scores_dev(int32_t L, int32_t count, const uint32_t *x_dev, int32_t *scores_dev,
                         int32_t variant, void *stream);

/* ---------------------------------------------------------------------------------------------
 * The search walk (Section 3, Algorithm 1, read as a self-avoiding walk over skew-symmetric
 * sequences): at every step score all n flips of the current state, move to the lowest-ISL flip
 * whose state is not in the walk's visited table (lowest j on ties), insert it, and keep the
 * best state.  Walks are independent (the paper's runs are, Section 4).  The readings that fix
 * what the paper leaves open (start states, table, ties, restarts, stop rules) are:
 *   - start state of restart r of walk w: free bits drawn from SplitMix64: key_w =
 *     sm(seed, walk_id), key_r = sm(key_w, r), word_i = sm(key_r, i), where sm(s, i) is the
 *     i-th output (from 0) of SplitMix64 started at state s; bit j of x = bit j%64 of word j/64.
 *   - visited table: 2^table_log2 64-bit words per walk, 0 = empty, entry = hash | 1, where
 *     hash = XOR of z_j over set free bits and z_j = sm(0x2011000068ABCDEF, j).  Slot = x read
 *     as an integer when n <= table_log2 (exact, never evicts), else the top table_log2 bits of
 *     the hash; an insert overwrites.  The start state is inserted; so is every committed state.
 *   - every step scores n flips (n flip evaluations, the paper's speed unit of Section 3); if
 *     every flip leads to a visited state the walk restarts (a trap; the step still counts).
 *   - best: strict improvement only (the first best is kept).  Every occupied state counts for
 *     best, target and watch: the initial state (step 0), each committed state, and each restart
 *     state (a restart repeats the initialisation), occupied at the step after which the restart
 *     happens (the trap step, or the step completing the period).
 *   - after a committed step t: if ISL <= target_isl the walk records hit_step = t and stops;
 *     if ISL <= watch_isl it records watch_step = t (first time) and goes on; if the budget
 *     `steps` is reached it stops; otherwise if restart_period > 0 and t % restart_period == 0
 *     it restarts, and the restart state is checked the same way at step t.  A start state
 *     (t = 0) that already meets target / watch records step 0.
 * ------------------------------------------------------------------------------------------- */

typedef struct labs_walk_cfg {
    int32_t L;              /* odd, 3 <= L <= LABS_WALK_L_MAX */
    int32_t table_log2;     /* 1..30; visited table of 2^table_log2 words (16 = 512 KiB) */
    uint64_t seed;          /* start-state generator seed */
    uint32_t walk_id;       /* start-state stream id */
    uint32_t flags;         /* 0, or LABS_TRACE and/or LABS_TRACE_SCORES */
    int64_t steps;          /* step budget, >= 0 */
    int64_t restart_period; /* 0 = never */
    int64_t target_isl;     /* -1 = none */
    int64_t watch_isl;      /* -1 = none */
} labs_walk_cfg;

#define LABS_TRACE 1u        /* record (chosen flip or -1 on a trap, ISL after the step) */
#define LABS_TRACE_SCORES 2u /* record all n flip scores of every step */

typedef struct labs_walk_result {
    int64_t best_isl;   /* lowest ISL seen */
    int64_t best_step;  /* step at which it was first reached (0 = start state) */
    int64_t steps_done; /* steps taken */
    int64_t flip_evals; /* n per step */
    int64_t hit_step;   /* first step with ISL <= target_isl, else -1 */
    int64_t watch_step; /* first step with ISL <= watch_isl, else -1 */
    int64_t final_isl;  /* ISL of the state the walk ended in */
    int32_t restarts;   /* restarts of any cause */
    int32_t traps;      /* restarts caused by an all-visited neighbourhood */
    uint32_t best_bits[LABS_X_WORDS];  /* free bits of the best state */
    uint32_t final_bits[LABS_X_WORDS]; /* free bits of the final state */
} labs_walk_result;

/* Kernel variants: results never depend on the choice. */
#define LABS_VARIANT_AUTO 0     /* autotuned (labs_autotune cache), else LABS_VARIANT_MFMA when
                                   every walk has L <= 383, else LABS_VARIANT_BITSLICE */
#define LABS_VARIANT_BITSLICE 1 /* bit-sliced correlation table, popcount scoring */
#define LABS_VARIANT_DIRECT 2   /* int8 sequence + int32 table in LDS, direct sum of squares */
#define LABS_VARIANT_MFMA 3     /* the correlation sums of every flip as int8 matrix-core tiles:
                                   one tile per step for L <= 255, two beyond (every L <= 383) */

typedef struct labs_plan_opts {
    int32_t variant;          /* LABS_VARIANT_* */
    int32_t waves_per_block;  /* walks per workgroup: 0 = auto, else 1, 2, 4 or 8 */
    int32_t probe_width;      /* visited-table probes issued together: 0 = auto, 1 or 2
                                 (3 and 4 are accepted and run as 2) */
    int32_t plain;            /* 1 = one launch per walk, serialised (comparison form) */
    int64_t steps_per_launch; /* 0 = auto; else steps each walk advances per kernel launch */
    int32_t use_graph;        /* 1 = capture the launches of a run in a hipGraph and replay it */
    int32_t persistent;       /* 0 = auto; 1 = one wave per walk (the hardware schedules the
                                 grid); 2 = a grid of resident waves that pull walks, costliest
                                 first, from a counter until none are left */
} labs_plan_opts;

/* Runs n_walks walks (cfg: host array) to completion on the GPU and copies the results to out
 * (host, n_walks entries).  trace (host, may be NULL): for each walk in order with LABS_TRACE,
 * 2*steps int32 (entries past steps_done are left 0).  scores (host, may be NULL): for each walk
 * with LABS_TRACE_SCORES, steps*n int32.  stream as above; synchronous.  Allocates and frees
 * its device state; use the plan API to keep it resident. */
int labs_walk_batch(int32_t n_walks, const labs_walk_cfg *cfg, labs_walk_result *out,
                    int32_t *trace, int32_t *scores, void *stream);

/* ---------------------------------------------------------------------------------------------
 * Best-first search with a bounded priority queue: Algorithm 1 taken literally (Section 3), and
 * optionally with the second table of evaluated neighbours of xLastovka (Section 3).  Each
 * iteration scores the n flips of the current state S; a neighbour found in the second table (as
 * it stood before the iteration) is skipped without evaluation; a neighbour in the visited table
 * is evaluated but skipped; every other neighbour is recorded in the second table (when in use;
 * of several neighbours sharing a slot the highest flip index is stored), offered to the queue
 * and compared with the best.  Then the front entry whose state is not visited becomes S and is
 * recorded as visited; an empty queue restarts the search (a trap).  The queue is ordered by
 * (ISL, iteration that generated the entry, flip index); an entry offered to a full queue
 * replaces the last entry if it precedes it, else it is dropped; entries are not de-duplicated.
 * Start states, tables, restarts, target and watch are those of the walk above, except:
 *   - best, hit_step and watch_step are taken when a neighbour is evaluated: best_step (and
 *     hit / watch) is the iteration count after the iteration that evaluated the state;
 *   - flip_evals counts n per iteration less the neighbours skipped by the second table;
 *   - trace records (j when the new S is the current state's flip-j neighbour, -2 when it is an
 *     older queue entry, -1 on a trap; ISL of the new S);
 *   - restarts clear the visited table, the second table and the queue.
 * With capacity 1 and no second table the search is exactly the walk of labs_walk_batch.
 * ------------------------------------------------------------------------------------------- */
typedef struct labs_pq_opts {
    int32_t capacity;       /* queue entries per walk, 1..64 */
    int32_t nbr_table_log2; /* 0 = no second table (impxLast); else 1..30: 2^log2 words per walk,
                               the visited table's layout and hash */
} labs_pq_opts;

/* Runs n_walks best-first searches to completion (one launch per kernel shape; steps < 2^31 per
 * walk) and copies the results to out (host).  trace / scores as for labs_walk_batch.
 * kernel_ms (may be NULL): device time of the search launches.  Synchronous on stream.
 * Allocates and frees its device state (visited and second tables: n_walks * (2^table_log2 +
 * 2^nbr_table_log2) * 8 bytes; LABS_ENOMEM if that does not fit). */
int labs_pq_walk_batch(int32_t n_walks, const labs_walk_cfg *cfg, const labs_pq_opts *opts,
                       labs_walk_result *out, int32_t *trace, int32_t *scores, double *kernel_ms,
                       void *stream);

/* ---------------------------------------------------------------------------------------------
 * First-improvement search with perturbations: the method of Dimitrov et al. as Section 2
 * describes it.  From the current skew-symmetric state the search moves at once to the first flip
 * j = 0, 1, ..., c (index order) whose ISL is strictly lower than the current ISL, and scans again
 * from the new state; when no flip improves (a local minimum of the one-flip neighbourhood) it
 * flips perturb_bits distinct free symbols drawn at random and goes on from the perturbed state,
 * whatever its ISL.  Perturbation k of a walk (k = 0, 1, ... over the whole walk) draws 64-bit
 * words sm(sm(sm(seed, walk_id), 2^32 + k), i), i = 0, 1, ... (sm as for the start states) and
 * flips j = floor((word >> 32) * n / 2^32) for each word whose j was not drawn before, until
 * perturb_bits symbols are flipped (or 65536 words are used).  There is no visited table
 * (table_log2 is checked but unused).  One step = one scan; flip_evals counts j + 1 for a move at
 * flip j and n + perturb_bits for a perturbation (the flips the sequential method evaluates);
 * traps counts the perturbations; trace records (j of the move, or -1 for a perturbation; ISL
 * after the step); scores (LABS_TRACE_SCORES) the ISL of every flip of the state each step starts
 * from.  Start states, restarts, target, watch and best follow the walk above.
 * ------------------------------------------------------------------------------------------- */
typedef struct labs_fi_opts {
    int32_t perturb_bits; /* symbols flipped by a perturbation: 1 <= perturb_bits <= min(n, 32) */
    int32_t reserved;
} labs_fi_opts;

/* Runs n_walks first-improvement searches to completion (one launch per kernel shape; steps <
 * 2^31 per walk) and copies the results to out (host).  trace / scores as for labs_walk_batch.
 * kernel_ms (may be NULL): device time of the search launches.  Synchronous on stream.  Allocates
 * and frees its device state.  LABS_EINVAL for a bad walk configuration or perturb_bits. */
int labs_fi_walk_batch(int32_t n_walks, const labs_walk_cfg *cfg, const labs_fi_opts *opts,
                       labs_walk_result *out, int32_t *trace, int32_t *scores, double *kernel_ms,
                       void *stream);

/* ---------------------------------------------------------------------------------------------
 * The walk over general (not skew-symmetric) sequences: the unrestricted problem that the
 * skew-symmetric restriction of Section 1 reduces.  Exactly the walk of labs_walk_batch with
 * n = L free symbols (bit j of x = b_j, drawn as the skew start's words over L bits), a flip
 * negating one symbol, and every shift k = 1 .. L-1 in Eq. (1)-(2); any 3 <= L <=
 * LABS_GENERAL_L_MAX, odd or even.  flip_evals counts L per step.
 * ------------------------------------------------------------------------------------------- */
#define LABS_GENERAL_L_MAX 192

/* ISL of every one-symbol flip of a batch of general sequences (Eq. (1)-(2), all shifts):
 * x_dev: device, count * LABS_X_WORDS uint32 (bit j of state r = b_j, j < L; higher bits must be 0,
 * not checked);
 * scores_dev: device, count * L int32; scores_dev[r*L + j] = ISL of state r with s_j negated.
 * 3 <= L <= LABS_GENERAL_L_MAX.  Asynchronous on stream; LABS_EINVAL for a bad L, count < 0 or
 * NULL buffers with count > 0. */
int labs_general_flip_scores_dev(int32_t L, int32_t count, const uint32_t *x_dev, int32_t *scores_dev,
                                 void *stream);

/* Runs n_walks general walks to completion (one launch per kernel shape; steps <= 2^30 per walk);
 * arguments and results as labs_pq_walk_batch (scores: steps * L int32 per walk with
 * LABS_TRACE_SCORES).  Synchronous on stream; allocates and frees its device state. */
int labs_general_walk_batch(int32_t n_walks, const labs_walk_cfg *cfg, labs_walk_result *out,
                            int32_t *trace, int32_t *scores, double *kernel_ms, void *stream);

typedef struct labs_walk_plan labs_walk_plan;

/* Allocates device state for n_walks walks (visited tables: n_walks * 2^table_log2 * 8 bytes;
 * LABS_ENOMEM if it does not fit, or if the tables, trace records or score entries of the batch
 * add up to more than 2^40 entries), uploads cfg and resolves the options (opts may be NULL =
 * all auto).  The plan owns its device memory until labs_walk_plan_destroy. */
int labs_walk_plan_create(int32_t n_walks, const labs_walk_cfg *cfg, const labs_plan_opts *opts,
                          labs_walk_plan **plan);
/* Resets every walk to its start state and runs all walks to completion, asynchronously on
 * stream (re-running gives identical results).  Not thread-safe per plan. */
int labs_walk_plan_run(labs_walk_plan *plan, void *stream);
/* Waits for the plan's last run and copies results / traces out (host buffers as in
 * labs_walk_batch; out may be NULL). */
int labs_walk_plan_results(labs_walk_plan *plan, labs_walk_result *out, int32_t *trace,
                           int32_t *scores);
/* Options the plan resolved (after autotuning). */
int labs_walk_plan_get_opts(const labs_walk_plan *plan, labs_plan_opts *opts);
/* Device time of the walk launches of the plan's last run (hipEvents recorded on the run's
 * stream after the state reset and after the last walk launch; with use_graph the events
 * bracket the whole graph, whose reset copy is a few microseconds), in milliseconds, and the
 * number of walk-kernel launches the run made.  Waits for the run to finish. */
int labs_walk_plan_last_timing(const labs_walk_plan *plan, double *ms, int32_t *launches);
void labs_walk_plan_destroy(labs_walk_plan *plan);

/* Times the kernel variants / launch shapes (variant, waves_per_block, probe_width, persistent)
 * on a short synthetic walk batch of n_walks walks at length L and stores the fastest in the
 * autotune cache (file named by $LABS_AUTOTUNE_CACHE, default ~/.cache/liblabs_autotune.txt;
 * entries keyed by device arch and L).  Plans created afterwards with automatic options take the
 * cached entry of their own L, else of the nearest L tuned for the same kernel shape (walks of
 * one length), or the entry of their own key (mixed lengths, see labs_autotune_batch).  Tuning
 * never changes results.  best (host, may be NULL) receives the winner. */
int labs_autotune(int32_t L, int32_t n_walks, labs_plan_opts *best);

/* As labs_autotune, timed on the caller's batch (cfg: host array, as for labs_walk_plan_create)
 * with every walk cut to at most 512 steps, without traces, target or watch.  A batch of mixed
 * lengths is keyed by its shortest and longest length and only plans of that same range take
 * its entry.  LABS_EINVAL for n_walks < 1, a NULL cfg or a bad walk configuration. */
int labs_autotune_batch(int32_t n_walks, const labs_walk_cfg *cfg, labs_plan_opts *best);

/* ---------------------------------------------------------------------------------------------
 * Serving: a request loop that admits search jobs by device memory for their walk state, keeps
 * every admitted walk resident across kernel launches and advances all running jobs together
 * (continuous batching; each tick is enqueued before the previous one is summarised, so the GPU
 * does not wait for the host).  A job = n_walks walks of one length; each walk's step budget is
 * floor(flip_budget / (n_walks * n)); the job stops at its budget or at the first tick
 * boundary (steps_per_tick, 2 steps_per_tick, ... logical steps) at or after the first step at
 * which some walk reached ISL <= ISL_T, where
 * ISL_T = floor(L^2 * den / (2 * num)) is the exact integer form of F >= num/den (Eq. (3)).
 * Results are a function of the request alone: they do not depend on what else runs.
 * ------------------------------------------------------------------------------------------- */

typedef struct labs_server labs_server;

typedef struct labs_server_opts {
    int64_t device_mem_bytes; /* budget for resident walk state (tables + state) */
    int32_t table_log2;       /* visited table per walk (default 16) */
    int32_t steps_per_tick;   /* logical steps every running walk advances per tick (> 0) */
    int32_t max_walks;        /* slot cap (0 = as many as the budget allows) */
    int32_t reserved;
} labs_server_opts;

typedef struct labs_search_req {
    int32_t L;             /* odd, 3 <= L <= LABS_WALK_L_MAX */
    int32_t n_walks;       /* >= 1 */
    uint64_t seed;         /* walk w of the job uses walk_id = w */
    int64_t flip_budget;   /* total flip evaluations over all walks */
    int64_t target_F_num;  /* stop threshold F >= num/den; num <= 0 = none */
    int64_t target_F_den;
} labs_search_req;

#define LABS_JOB_QUEUED 0
#define LABS_JOB_RUNNING 1
#define LABS_JOB_DONE 2
#define LABS_JOB_CANCELLED 3

typedef struct labs_search_status {
    int32_t state;        /* LABS_JOB_* */
    int32_t best_walk;    /* walk holding best_isl (lowest id on ties) */
    int64_t best_isl;
    double best_F;
    int64_t hit_step;     /* lowest step at which a walk reached ISL_T, else -1 */
    int32_t hit_walk;     /* lowest walk id reaching it at hit_step, else -1 */
    int32_t reserved;
    int64_t steps_done;   /* logical steps every walk of the job has taken */
    int64_t flip_evals;   /* sum over walks */
    double t_submit, t_admit, t_done; /* seconds on the server's monotonic clock */
    uint32_t best_bits[LABS_X_WORDS];
} labs_search_status;

/* Creates a server owning one GPU stream, its slot pool and a scheduler thread. */
int labs_server_create(const labs_server_opts *opts, labs_server **srv);
/* Queues a job (never blocks on the GPU); LABS_ENOMEM if the job could never fit the budget. */
int labs_search_submit(labs_server *srv, const labs_search_req *req, uint64_t *job_id);
/* LABS_OK with st filled when the job is done or cancelled; LABS_EPENDING with st filled
 * (state QUEUED or RUNNING) otherwise; LABS_ENOTFOUND for an unknown id.  Thread-safe. */
int labs_search_poll(labs_server *srv, uint64_t job_id, labs_search_status *st);
/* Blocks until the job is done (or timeout_ms passes: LABS_EPENDING); timeout_ms < 0 waits. */
int labs_search_wait(labs_server *srv, uint64_t job_id, int64_t timeout_ms,
                     labs_search_status *st);
/* Cancels a queued or running job; its slots are freed at the next tick.  Thread-safe. */
int labs_search_cancel(labs_server *srv, uint64_t job_id);
/* Drops the record of a finished (done or cancelled) job, so that a long-running server does not
 * keep every past job; afterwards the id is unknown (LABS_ENOTFOUND).  LABS_EPENDING if the job is
 * still queued or running.  Thread-safe. */
int labs_search_release(labs_server *srv, uint64_t job_id);
/* Server counters: ticks run, walks resident now, peak resident walks, flip evaluations done. */
int labs_server_stats(labs_server *srv, int64_t *ticks, int32_t *resident_walks,
                      int32_t *peak_walks, int64_t *flip_evals);
/* Stops the scheduler, ends every job still queued or running as cancelled, and frees everything.
 * No other call on srv may run concurrently with or after it. */
void labs_server_destroy(labs_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* LABS_H */
