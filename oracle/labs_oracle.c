/*
 * labs_oracle.c -- the oracle: a plain, slow, CPU statement of everything the GPU library
 * computes for the skew-symmetric LABS search of
 *   J. Brest, B. Boskovic, "Computational Search of Long Skew-symmetric Binary Sequences
 *   with High Merit Factors", arXiv:2011.00068.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the package smoke check and the CPU-baseline
 * leg of the benchmark load this file.  The GPU library never calls, links or includes it, and
 * the two share no code, header, table or constant generator: every constant below is written
 * out here from its published definition.
 *
 * Conventions (all 0-based, as in Eq. (1)):
 *   S = (s_0 .. s_{L-1}), s_i in {+1,-1};  bit b_i = 1  <=>  s_i = -1  (Section 4's hex rule).
 *   Skew-symmetric: L = 2n-1, centre c = n-1, s_{c+i} = (-1)^i s_{c-i} for i = 1..c (Eq. (4),
 *   re-indexed from the paper's 1-based form so that Table 1's sequences satisfy it).
 *   Free symbols s_0..s_c; "flip j" (0 <= j <= c) negates s_j and its mirror s_{L-1-j}
 *   (one symbol when j == c), which keeps the sequence skew-symmetric.
 *   Free-bit vector x: bit j (word j/64, bit j%64) = b_j, j = 0..c.
 *
 * Every accumulator is int64.
 *
 * Pins: Eq. (1)-(4), PSL, the hex codec and the one-flip evaluation are pinned by Table 1, the
 * Barker-13 worked case, numpy.correlate, brute force over all 2^L sequences and the plain
 * definition of a flipped ISL (tests/test_oracle_*.py), for skew-symmetric and general sequences; the grouped skew-space minimum by brute
 * force over all 2^L sequences and numpy on blocks up to n = 63; SplitMix64 by its published
 * first outputs.
 * Parity unpinned: ref_start_bits, ref_zobrist and the visited-table, tie and restart rules of
 * ref_walk are readings of what the paper leaves open; they are checked only for internal
 * consistency (incremental walk == recomputing walk, bounded table == exact set before any
 * eviction, no revisits, best == first minimum of the trajectory).  So are the queue order,
 * capacity and discard rules of ref_pq_walk: it is checked against ref_walk (capacity 1) and
 * against an independent Python statement of the same reading; and so are the scan order, the
 * perturbation draw and its size of ref_fi_walk: it is checked against the plain definition of
 * every flip score, an independent numpy statement of the same reading, its move and local-minimum
 * rules, the negation symmetry (a perturbation of every symbol keeps the ISL) and the uniformity
 * of the draw.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_WORDS 8 /* free-bit words (64-bit) -> n <= 512 */

/* ------------------------------------------------------------------------------------------
 * Definitions (Section 1)
 * ---------------------------------------------------------------------------------------- */

/* Eq. (1): aperiodic autocorrelation C_k = sum_{i=0}^{L-k-1} s_i s_{i+k}, k = 0..L-1. */
void ref_corr(int32_t L, const int8_t *s, int64_t *C)
{
    for (int32_t k = 0; k < L; k++) {
        int64_t acc = 0;
        for (int32_t i = 0; i + k < L; i++)
            acc += (int64_t)s[i] * (int64_t)s[i + k];
        C[k] = acc;
    }
}

/* Eq. (2): ISL = sum_{k=1}^{L-1} C_k^2 (one-sided sum of squared off-peak correlations). */
int64_t ref_isl(int32_t L, const int8_t *s)
{
    int64_t isl = 0;
    for (int32_t k = 1; k < L; k++) {
        int64_t acc = 0;
        for (int32_t i = 0; i + k < L; i++)
            acc += (int64_t)s[i] * (int64_t)s[i + k];
        isl += acc * acc;
    }
    return isl;
}

/* Eq. (3): F = L^2 / (2 ISL).  Returns -1.0 when ISL == 0 (L == 1), where F is undefined. */
double ref_merit(int32_t L, const int8_t *s)
{
    int64_t isl = ref_isl(L, s);
    if (isl == 0)
        return -1.0;
    return ((double)L * (double)L) / (2.0 * (double)isl);
}

/* Section 1: peak sidelobe level PSL = max_{k=1}^{L-1} |C_k|. */
int64_t ref_psl(int32_t L, const int8_t *s)
{
    int64_t psl = 0;
    for (int32_t k = 1; k < L; k++) {
        int64_t acc = 0;
        for (int32_t i = 0; i + k < L; i++)
            acc += (int64_t)s[i] * (int64_t)s[i + k];
        if (acc < 0)
            acc = -acc;
        if (acc > psl)
            psl = acc;
    }
    return psl;
}

/* Eq. (4), 0-based centre c = (L-1)/2: s_{c+i} = (-1)^i s_{c-i}, i = 1..c.  1 = skew. */
int ref_is_skew(int32_t L, const int8_t *s)
{
    if (L < 1 || (L % 2) == 0)
        return 0;
    int32_t c = (L - 1) / 2;
    for (int32_t i = 1; i <= c; i++) {
        int32_t want = (i % 2 == 1) ? -s[c - i] : s[c - i];
        if (s[c + i] != want)
            return 0;
    }
    return 1;
}

/* Builds the skew-symmetric sequence whose free symbols s_0..s_c carry the bits of x
 * (bit set -> -1), filling the second half by Eq. (4). */
void ref_skew_expand(int32_t L, const uint64_t *x, int8_t *s)
{
    int32_t c = (L - 1) / 2;
    for (int32_t j = 0; j <= c; j++)
        s[j] = ((x[j / 64] >> (j % 64)) & 1u) ? -1 : 1;
    for (int32_t i = 1; i <= c; i++)
        s[c + i] = (i % 2 == 1) ? (int8_t)(-s[c - i]) : s[c - i];
}

/* Inverse of ref_skew_expand on the free half: x bit j = (s_j == -1).  nwords 64-bit words. */
void ref_skew_bits(int32_t L, const int8_t *s, uint64_t *x, int32_t nwords)
{
    int32_t c = (L - 1) / 2;
    for (int32_t w = 0; w < nwords; w++)
        x[w] = 0;
    for (int32_t j = 0; j <= c; j++)
        if (s[j] == -1)
            x[j / 64] |= (uint64_t)1 << (j % 64);
}

/* ------------------------------------------------------------------------------------------
 * Section 4's hexadecimal encoding of Table 1: each hex digit is 4 bits (most significant
 * first); leading zero bits are dropped down to length L; bit 0 -> +1, bit 1 -> -1.
 * ---------------------------------------------------------------------------------------- */

static int hex_value(char ch)
{
    if (ch >= '0' && ch <= '9')
        return ch - '0';
    if (ch >= 'A' && ch <= 'F')
        return ch - 'A' + 10;
    if (ch >= 'a' && ch <= 'f')
        return ch - 'a' + 10;
    return -1;
}

/* Returns 0 on success, -1 on a bad digit, -2 if the string has fewer than L bits,
 * -3 if a dropped leading bit is 1. */
int ref_hex_decode(const char *hex, int32_t L, int8_t *s)
{
    int32_t ndig = (int32_t)strlen(hex);
    int32_t nbits = 4 * ndig;
    if (nbits < L)
        return -2;
    int32_t drop = nbits - L;
    for (int32_t b = 0; b < nbits; b++) {
        int v = hex_value(hex[b / 4]);
        if (v < 0)
            return -1;
        int bit = (v >> (3 - (b % 4))) & 1;
        if (b < drop) {
            if (bit)
                return -3;
            continue;
        }
        s[b - drop] = bit ? -1 : 1;
    }
    return 0;
}

/* Writes ceil(L/4) upper-case hex digits plus a terminating NUL into out (cap >= that + 1).
 * Returns the number of digits, or -1 if cap is too small. */
int ref_hex_encode(int32_t L, const int8_t *s, char *out, int32_t cap)
{
    int32_t ndig = (L + 3) / 4;
    if (cap < ndig + 1)
        return -1;
    int32_t pad = 4 * ndig - L;
    for (int32_t d = 0; d < ndig; d++) {
        int v = 0;
        for (int32_t q = 0; q < 4; q++) {
            int32_t b = 4 * d + q - pad; /* index into S, negative = padding zero */
            int bit = (b >= 0) ? (s[b] == -1) : 0;
            v = (v << 1) | bit;
        }
        out[d] = "0123456789ABCDEF"[v];
    }
    out[ndig] = '\0';
    return ndig;
}

/* ------------------------------------------------------------------------------------------
 * One-flip evaluation (Section 3; Algorithm 1's "fast calculate merit factor" step).
 * ---------------------------------------------------------------------------------------- */

/* Plain definition: ISL of S with s_j and its mirror negated, recomputed from Eq. (1)-(2). */
int64_t ref_flip_isl_brute(int32_t L, const int8_t *s, int32_t j)
{
    int8_t *t = (int8_t *)malloc((size_t)L);
    memcpy(t, s, (size_t)L);
    t[j] = (int8_t)(-t[j]);
    if (L - 1 - j != j)
        t[L - 1 - j] = (int8_t)(-t[L - 1 - j]);
    int64_t isl = ref_isl(L, t);
    free(t);
    return isl;
}

/*
 * Incremental evaluation from a table of the current correlations C (C[k], k = 0..L-1, as
 * produced by ref_corr).  Derived from Eq. (1): negating the symbols of a set P negates exactly
 * the products s_i s_{i+k} with one end in P, so C_k moves by -2 times their sum.  For a
 * skew-symmetric S (Eq. (4)) and even k, the mirror's products equal the primary's, so for
 * P = {j, m}, m = L-1-j, j < c, with d = m - j (the shift at which j and m pair with each
 * other, whose product is negated twice and so does not change):
 *     dC_k = -4 s_j ( s_{j+k} [j+k <= L-1, k != d] + s_{j-k} [j-k >= 0] ),
 * and for the centre (P = {c}): dC_k = -4 s_c s_{c-k} [k <= c].  Odd-k correlations are 0 on
 * every skew-symmetric sequence and stay 0.  The flipped ISL is sum over even k of
 * (C_k + dC_k)^2.  The tests pin this against ref_flip_isl_brute on every flip.
 */
int64_t ref_flip_isl_incr(int32_t L, const int8_t *s, const int64_t *C, int32_t j)
{
    int32_t c = (L - 1) / 2;
    int64_t isl = 0;
    for (int32_t k = 2; k <= L - 1; k += 2) {
        int64_t dk;
        if (j < c) {
            int32_t d = L - 1 - 2 * j;
            int64_t p = (j + k <= L - 1 && k != d) ? s[j + k] : 0;
            int64_t q = (j - k >= 0) ? s[j - k] : 0;
            dk = -4 * (int64_t)s[j] * (p + q);
        } else {
            int64_t q = (k <= c) ? s[c - k] : 0;
            dk = -4 * (int64_t)s[c] * q;
        }
        int64_t t = C[k] + dk;
        isl += t * t;
    }
    return isl;
}

/* All n = c+1 flip scores of the skew sequence with free bits x.  brute != 0 selects the plain
 * definition, otherwise the incremental evaluation. */
void ref_flip_scores(int32_t L, const uint64_t *x, int64_t *out, int brute)
{
    int8_t *s = (int8_t *)malloc((size_t)L);
    int64_t *C = (int64_t *)malloc(sizeof(int64_t) * (size_t)L);
    ref_skew_expand(L, x, s);
    ref_corr(L, s, C);
    int32_t c = (L - 1) / 2;
    for (int32_t j = 0; j <= c; j++)
        out[j] = brute ? ref_flip_isl_brute(L, s, j) : ref_flip_isl_incr(L, s, C, j);
    free(s);
    free(C);
}

/* One-flip evaluation for a general (not skew-symmetric) sequence: flip j negates s_j alone.
 * Plain definition: recompute Eq. (1)-(2) for the flipped sequence. */
int64_t ref_flip_isl_general_brute(int32_t L, const int8_t *s, int32_t j)
{
    int8_t *t = (int8_t *)malloc((size_t)L);
    memcpy(t, s, (size_t)L);
    t[j] = (int8_t)(-t[j]);
    int64_t isl = ref_isl(L, t);
    free(t);
    return isl;
}

/* Incremental form (Eq. (1)): negating s_j negates the products s_j s_{j+k} and s_{j-k} s_j, so
 *     dC_k = -2 s_j ( s_{j+k} [j+k <= L-1] + s_{j-k} [j-k >= 0] ),  k = 1 .. L-1,
 * and the flipped ISL is sum_k (C_k + dC_k)^2 over every k (odd k included). */
int64_t ref_flip_isl_general_incr(int32_t L, const int8_t *s, const int64_t *C, int32_t j)
{
    int64_t isl = 0;
    for (int32_t k = 1; k <= L - 1; k++) {
        int64_t p = (j + k <= L - 1) ? s[j + k] : 0;
        int64_t q = (j - k >= 0) ? s[j - k] : 0;
        int64_t v = C[k] - 2 * (int64_t)s[j] * (p + q);
        isl += v * v;
    }
    return isl;
}

/* ------------------------------------------------------------------------------------------
 * Counter-based random numbers: SplitMix64 (G. L. Steele, D. Lea, C. H. Flood, "Fast
 * splittable pseudorandom number generators", OOPSLA 2014), written from its published
 * definition: the state advances by the odd constant 0x9E3779B97F4A7C15 and each output is
 * the state passed through the mixing function below.  ref_sm64_at(seed, i) is the i-th output
 * (i = 0, 1, ...) of the generator started from state `seed`.
 * ---------------------------------------------------------------------------------------- */

static uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t ref_sm64_at(uint64_t seed, uint64_t i)
{
    return sm64_mix(seed + (i + 1) * 0x9E3779B97F4A7C15ULL);
}

/* Start sequence of restart r of walk w (Algorithm 1's "initialize a starting skew-symmetric
 * sequence"; the paper does not say how): free symbols i.i.d. uniform, drawn as 64-bit words
 *   key_w = sm64_at(seed, w), key_wr = sm64_at(key_w, r), word_i = sm64_at(key_wr, i),
 * bit j of x = bit (j % 64) of word_(j / 64), bits at j >= n cleared. */
static void draw_bits(int32_t n, uint64_t seed, uint32_t walk_id, uint32_t restart, uint64_t *x,
                      int32_t nwords)
{
    uint64_t kw = ref_sm64_at(seed, walk_id);
    uint64_t kr = ref_sm64_at(kw, restart);
    for (int32_t w = 0; w < nwords; w++) {
        uint64_t v = ref_sm64_at(kr, (uint64_t)w);
        int32_t lo = 64 * w;
        if (lo >= n)
            v = 0;
        else if (n - lo < 64)
            v &= (((uint64_t)1) << (n - lo)) - 1;
        x[w] = v;
    }
}

void ref_start_bits(int32_t L, uint64_t seed, uint32_t walk_id, uint32_t restart, uint64_t *x,
                    int32_t nwords)
{
    draw_bits((L + 1) / 2, seed, walk_id, restart, x, nwords);
}

/* Start sequence of a general walk (ORACLE_GENERAL): the same draw over all L symbols. */
void ref_start_bits_general(int32_t L, uint64_t seed, uint32_t walk_id, uint32_t restart, uint64_t *x,
                            int32_t nwords)
{
    draw_bits(L, seed, walk_id, restart, x, nwords);
}

/* Zobrist key of free symbol j (A. L. Zobrist, 1970): z_j = sm64_at(0x2011000068ABCDEF, j).
 * The hash of a state is the XOR of z_j over its set free bits. */
uint64_t ref_zobrist(int32_t j)
{
    return ref_sm64_at(0x2011000068ABCDEFULL, (uint64_t)j);
}

/* ------------------------------------------------------------------------------------------
 * The search walk (Section 3, Algorithm 1, in its self-avoiding-walk reading): at every step
 * score all n flips of the current state, move to the best flip whose resulting state has not
 * been visited (lowest index on ties), record it as visited, and keep the best state seen.
 * With ORACLE_GENERAL the same walk runs over general sequences of any length L >= 3 (all L
 * symbols free, a flip negates one symbol, every shift k counts): the unrestricted problem the
 * skew-symmetric restriction of Section 1 reduces.
 * ---------------------------------------------------------------------------------------- */

typedef struct {
    int32_t L;
    int32_t table_log2;     /* visited table has 2^table_log2 64-bit words */
    uint64_t seed;
    uint32_t walk_id;
    uint32_t flags;         /* ORACLE_BRUTE: score flips by the plain definition;
                               ORACLE_IDEAL: exact visited set instead of the bounded table;
                               ORACLE_GENERAL: general sequences (ref_walk only) */
    int64_t steps;          /* iteration budget */
    int64_t restart_period; /* 0 = never */
    int64_t target_isl;     /* -1 = none; else stop after the first state with ISL <= target */
    int64_t watch_isl;      /* -1 = none; else record the first step with ISL <= watch */
} ref_walk_cfg;

typedef struct {
    int64_t best_isl, best_step, steps_done, flip_evals, hit_step, watch_step, final_isl;
    int32_t restarts, traps;
    uint32_t best_bits[2 * ORACLE_MAX_WORDS];  /* 32-bit words of the free bits */
    uint32_t final_bits[2 * ORACLE_MAX_WORDS];
} ref_walk_result;

#define ORACLE_BRUTE 1u
#define ORACLE_IDEAL 2u
#define ORACLE_GENERAL 4u

/* Exact visited set used with ORACLE_IDEAL: open addressing over whole free-bit vectors. */
typedef struct {
    uint64_t *keys; /* cap * nwords words */
    uint8_t *used;
    int64_t cap, count;
    int32_t nwords;
} ideal_set;

static uint64_t ideal_hash(const uint64_t *x, int32_t nwords)
{
    uint64_t h = 0x12345678ULL;
    for (int32_t w = 0; w < nwords; w++)
        h = sm64_mix(h ^ x[w]);
    return h;
}

static void ideal_init(ideal_set *S, int32_t nwords)
{
    S->nwords = nwords;
    S->cap = 1024;
    S->count = 0;
    S->keys = (uint64_t *)calloc((size_t)S->cap * (size_t)nwords, sizeof(uint64_t));
    S->used = (uint8_t *)calloc((size_t)S->cap, 1);
}

static void ideal_free(ideal_set *S)
{
    free(S->keys);
    free(S->used);
}

static void ideal_clear(ideal_set *S)
{
    memset(S->used, 0, (size_t)S->cap);
    S->count = 0;
}

static int ideal_contains(const ideal_set *S, const uint64_t *x)
{
    int64_t i = (int64_t)(ideal_hash(x, S->nwords) & (uint64_t)(S->cap - 1));
    while (S->used[i]) {
        if (memcmp(S->keys + i * S->nwords, x, sizeof(uint64_t) * (size_t)S->nwords) == 0)
            return 1;
        i = (i + 1) & (S->cap - 1);
    }
    return 0;
}

static void ideal_insert(ideal_set *S, const uint64_t *x);

static void ideal_grow(ideal_set *S)
{
    ideal_set T;
    T.nwords = S->nwords;
    T.cap = S->cap * 2;
    T.count = 0;
    T.keys = (uint64_t *)calloc((size_t)T.cap * (size_t)T.nwords, sizeof(uint64_t));
    T.used = (uint8_t *)calloc((size_t)T.cap, 1);
    for (int64_t i = 0; i < S->cap; i++)
        if (S->used[i])
            ideal_insert(&T, S->keys + i * S->nwords);
    ideal_free(S);
    *S = T;
}

static void ideal_insert(ideal_set *S, const uint64_t *x)
{
    if (ideal_contains(S, x))
        return;
    if (2 * (S->count + 1) > S->cap)
        ideal_grow(S);
    int64_t i = (int64_t)(ideal_hash(x, S->nwords) & (uint64_t)(S->cap - 1));
    while (S->used[i])
        i = (i + 1) & (S->cap - 1);
    S->used[i] = 1;
    memcpy(S->keys + i * S->nwords, x, sizeof(uint64_t) * (size_t)S->nwords);
    S->count++;
}

/* Bounded visited table (the paper's hash table HT; its size and collision handling are not
 * stated).  Direct-mapped, one 64-bit word per slot, 0 = empty, stored word = hash | 1.
 * Slot = the state's free bits read as an integer when they fit (n <= table_log2: exact, never
 * evicts), otherwise the top table_log2 bits of the hash.  Insert overwrites. */
typedef struct {
    uint64_t *T;
    int32_t log2;
    int exact;
} bounded_table;

static uint64_t table_slot(const bounded_table *B, uint64_t h, const uint64_t *x)
{
    if (B->exact)
        return x[0];
    return h >> (64 - B->log2);
}

static void to_u32_words(const uint64_t *x, int32_t nwords, uint32_t *out)
{
    for (int32_t w = 0; w < nwords; w++) {
        out[2 * w] = (uint32_t)(x[w] & 0xFFFFFFFFu);
        out[2 * w + 1] = (uint32_t)(x[w] >> 32);
    }
}

/*
 * One walk.  trace (optional): 2 int32 per iteration, (chosen flip or -1 when trapped, ISL of
 * the state after the iteration).  score_trace (optional): n int32 per iteration, every flip's
 * ISL in index order.  Returns 0, or -1 on invalid arguments, -2 if an internal check fails.
 */
int ref_walk(const ref_walk_cfg *cfg, ref_walk_result *res, int32_t *trace, int32_t *score_trace)
{
    const int32_t L = cfg->L;
    const int general = (cfg->flags & ORACLE_GENERAL) != 0;
    if (L < 3 || (!general && (L % 2) == 0) || cfg->steps < 0 || cfg->table_log2 < 1 || cfg->table_log2 > 30)
        return -1;
    /* skew: n = c + 1 free symbols (flip j also negates the mirror L-1-j unless j = c);
     * general: all L symbols are free and a flip negates one */
    const int32_t n = general ? L : (L + 1) / 2, c = general ? -1 : n - 1;
    const int32_t nwords = (n + 63) / 64;
    if (nwords > ORACLE_MAX_WORDS)
        return -1;
    const int brute = (cfg->flags & ORACLE_BRUTE) != 0;
    const int ideal = (cfg->flags & ORACLE_IDEAL) != 0;

    int8_t *s = (int8_t *)malloc((size_t)L);
    int64_t *C = (int64_t *)malloc(sizeof(int64_t) * (size_t)L);
    int64_t *score = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    uint64_t *z = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    uint64_t x[ORACLE_MAX_WORDS], xn[ORACLE_MAX_WORDS];
    memset(x, 0, sizeof x);
    memset(xn, 0, sizeof xn);
    for (int32_t j = 0; j < n; j++)
        z[j] = ref_zobrist(j);

    bounded_table B;
    B.log2 = cfg->table_log2;
    B.exact = (n <= cfg->table_log2);
    B.T = ideal ? NULL : (uint64_t *)calloc((size_t)1 << cfg->table_log2, sizeof(uint64_t));
    ideal_set I;
    if (ideal)
        ideal_init(&I, nwords);

    int64_t isl = 0;
    uint64_t h = 0;
    uint32_t restart = 0;
    int rc = 0;

    memset(res, 0, sizeof *res);
    res->hit_step = -1;
    res->watch_step = -1;

/* (Re)start: draw the start state, compute C and ISL from scratch, clear the visited
 * record and insert the start state (Algorithm 1's initialisation). */
#define START_STATE()                                                                          \
    do {                                                                                       \
        if (general) {                                                                         \
            ref_start_bits_general(L, cfg->seed, cfg->walk_id, restart, x, nwords);            \
            for (int32_t i = 0; i < L; i++)                                                    \
                s[i] = ((x[i / 64] >> (i % 64)) & 1u) ? -1 : 1;                                \
        } else {                                                                               \
            ref_start_bits(L, cfg->seed, cfg->walk_id, restart, x, nwords);                    \
            ref_skew_expand(L, x, s);                                                          \
        }                                                                                      \
        ref_corr(L, s, C);                                                                     \
        isl = 0;                                                                               \
        for (int32_t k = 1; k < L; k++)                                                        \
            isl += C[k] * C[k];                                                                \
        h = 0;                                                                                 \
        for (int32_t j = 0; j < n; j++)                                                        \
            if ((x[j / 64] >> (j % 64)) & 1u)                                                  \
                h ^= z[j];                                                                     \
        if (ideal) {                                                                           \
            ideal_clear(&I);                                                                   \
            ideal_insert(&I, x);                                                               \
        } else {                                                                               \
            memset(B.T, 0, sizeof(uint64_t) * ((size_t)1 << B.log2));                          \
            B.T[table_slot(&B, h, x)] = h | 1u;                                                \
        }                                                                                      \
    } while (0)

/* Every state the walk occupies counts for best, hit and watch, start states included: the
 * initial state (Algorithm 1 initialises the best from it) and every restart state (a restart is
 * that same initialisation, Section 2).  t = the step after which the state is occupied. */
#define NOTE_STATE(t_)                                                                         \
    do {                                                                                       \
        if (isl < res->best_isl) {                                                             \
            res->best_isl = isl;                                                               \
            res->best_step = (t_);                                                             \
            to_u32_words(x, nwords, res->best_bits);                                           \
        }                                                                                      \
        if (cfg->target_isl >= 0 && res->hit_step < 0 && isl <= cfg->target_isl)             \
            res->hit_step = (t_);                                                              \
        if (cfg->watch_isl >= 0 && res->watch_step < 0 && isl <= cfg->watch_isl)             \
            res->watch_step = (t_);                                                            \
    } while (0)

    START_STATE();
    res->best_isl = INT64_MAX;
    NOTE_STATE(0);

    int64_t t = 0, flips = 0;
    while (t < cfg->steps && !(cfg->target_isl >= 0 && res->hit_step >= 0)) {
        /* score every flip of the current state */
        for (int32_t j = 0; j < n; j++) {
            if (general)
                score[j] = brute ? ref_flip_isl_general_brute(L, s, j) : ref_flip_isl_general_incr(L, s, C, j);
            else
                score[j] = brute ? ref_flip_isl_brute(L, s, j) : ref_flip_isl_incr(L, s, C, j);
        }
        flips += n;
        if (score_trace)
            for (int32_t j = 0; j < n; j++)
                score_trace[t * n + j] = (int32_t)score[j];

        /* best non-visited flip, lowest index on ties */
        int32_t jb = -1;
        for (int32_t j = 0; j < n; j++) {
            memcpy(xn, x, sizeof x);
            xn[j / 64] ^= (uint64_t)1 << (j % 64);
            uint64_t hn = h ^ z[j];
            int visited = ideal ? ideal_contains(&I, xn) : (B.T[table_slot(&B, hn, xn)] == (hn | 1u));
            if (visited)
                continue;
            if (jb < 0 || score[j] < score[jb])
                jb = j;
        }

        if (jb < 0) {
            /* every neighbour visited: restart from a fresh start state (the step counts) */
            res->traps++;
            res->restarts++;
            restart++;
            START_STATE();
            t++;
            if (trace) {
                trace[2 * t - 2] = -1;
                trace[2 * t - 1] = (int32_t)isl;
            }
            NOTE_STATE(t);
            continue;
        }

        /* commit the move */
        s[jb] = (int8_t)(-s[jb]);
        if (!general && jb != c)
            s[L - 1 - jb] = (int8_t)(-s[L - 1 - jb]);
        x[jb / 64] ^= (uint64_t)1 << (jb % 64);
        h ^= z[jb];
        ref_corr(L, s, C);
        isl = 0;
        for (int32_t k = 1; k < L; k++)
            isl += C[k] * C[k];
        if (isl != score[jb]) {
            rc = -2;
            break;
        }
        if (ideal)
            ideal_insert(&I, x);
        else
            B.T[table_slot(&B, h, x)] = h | 1u;
        t++;
        if (trace) {
            trace[2 * t - 2] = jb;
            trace[2 * t - 1] = (int32_t)isl;
        }
        NOTE_STATE(t);
        /* periodic restart (lssOrel-style, Section 2), only if the walk goes on */
        if (cfg->restart_period > 0 && t % cfg->restart_period == 0 && t < cfg->steps &&
            !(cfg->target_isl >= 0 && res->hit_step >= 0)) {
            res->restarts++;
            restart++;
            START_STATE();
            NOTE_STATE(t);
        }
    }
#undef NOTE_STATE
#undef START_STATE

    res->steps_done = t;
    res->flip_evals = flips;
    res->final_isl = isl;
    to_u32_words(x, nwords, res->final_bits);

    free(s);
    free(C);
    free(score);
    free(z);
    if (ideal)
        ideal_free(&I);
    else
        free(B.T);
    return rc;
}

/* ------------------------------------------------------------------------------------------
 * Exhaustive skew-symmetric enumeration (Eq. (4) leaves 2^n sequences; Section 1 notes the
 * search-space reduction).  out[x] = ISL of the sequence with free bits x, x = 0..2^n - 1.
 * ---------------------------------------------------------------------------------------- */
int ref_enum_skew(int32_t L, int64_t *out)
{
    if (L < 1 || (L % 2) == 0)
        return -1;
    int32_t n = (L + 1) / 2;
    if (n > 30)
        return -1;
    int8_t *s = (int8_t *)malloc((size_t)L);
    for (uint64_t x = 0; x < ((uint64_t)1 << n); x++) {
        uint64_t xw[1] = {x};
        ref_skew_expand(L, xw, s);
        out[x] = ref_isl(L, s);
    }
    free(s);
    return 0;
}

/* ------------------------------------------------------------------------------------------
 * Minimum over a block of the skew space, grouped by the symmetries of Section 1's search-space
 * reduction.  Negation (x -> x ^ A, A = all n free bits) and alternation s_i -> (-1)^i s_i
 * (x -> x ^ O, O = the free bits at odd positions) keep a sequence skew-symmetric and leave its
 * ISL unchanged; the four sequences {x, x^A, x^O, x^A^O} of a free-bit vector x = r << 2 (bits 0
 * and 1 clear) are distinct, and every x lies in exactly one such group.  This function covers
 * the groups of r = r_begin .. r_end - 1 by evaluating all four members of each group from the
 * definition (Eq. (2), (4)); it does not use the invariance.  Results: the lowest ISL, how many
 * of the covered sequences reach it, and the lowest such x.  n <= 63.  Returns 0, or -1 on bad
 * arguments; an empty block gives min_isl = -1, count = 0, first_x = 0.
 * ---------------------------------------------------------------------------------------- */
int ref_enum_skew_min(int32_t L, uint64_t r_begin, uint64_t r_end, int64_t *min_isl,
                      uint64_t *count, uint64_t *first_x)
{
    if (L < 3 || (L % 2) == 0)
        return -1;
    int32_t n = (L + 1) / 2;
    if (n > 63 || r_begin > r_end || r_end > ((uint64_t)1 << (n - 2)))
        return -1;
    uint64_t all = ((uint64_t)1 << n) - 1, odd = 0;
    for (int32_t j = 1; j < n; j += 2)
        odd |= (uint64_t)1 << j;
    int8_t *s = (int8_t *)malloc((size_t)L);
    int64_t best = -1;
    uint64_t cnt = 0, first = 0;
    for (uint64_t r = r_begin; r < r_end; r++) {
        uint64_t base = r << 2;
        uint64_t member[4] = {base, base ^ all, base ^ odd, base ^ all ^ odd};
        for (int m = 0; m < 4; m++) {
            uint64_t xw[1] = {member[m]};
            ref_skew_expand(L, xw, s);
            int64_t v = ref_isl(L, s);
            if (best < 0 || v < best) {
                best = v;
                cnt = 1;
                first = member[m];
            } else if (v == best) {
                cnt++;
                if (member[m] < first)
                    first = member[m];
            }
        }
    }
    free(s);
    *min_isl = best;
    *count = cnt;
    *first_x = best < 0 ? 0 : first;
    return 0;
}

/* ------------------------------------------------------------------------------------------
 * Best-first search with a bounded priority queue: Algorithm 1 taken literally (Section 3).
 * Each iteration flips every free symbol of the current state S in index order.  A flipped
 * state found in the optional second table of evaluated neighbours (the xLastovka variant
 * described in Section 3, which impxLast drops), as that table stood before the iteration, is
 * skipped without evaluation; every other one
 * counts one function evaluation and, if it is not in the visited table HT, is recorded in the
 * second table when that is in use, offered to the queue and compared with the best.  Then the front of the
 * queue is removed and becomes S, and S is recorded in HT.
 * Readings of what the paper leaves open:
 *   - queue order: ascending (ISL, iteration that generated the entry, flip index), so equal
 *     ISLs are served oldest first; capacity Q (the paper does not state it).  An entry offered
 *     to a full queue replaces the queue's last entry if it precedes it, otherwise it is dropped.
 *     Entries are not de-duplicated; a removed front entry whose state is already in HT is
 *     discarded and the next one is taken.
 *   - an empty queue (nothing left to take) restarts the search (a trap, counted like a
 *     restart); restarts clear HT, the second table and the queue.
 *   - best: strict improvement, checked when a neighbour is evaluated; best_step is the
 *     iteration count after the iteration that evaluated it.  Start states count as well (the
 *     initial one at 0, a restart state at the iteration count after which it is occupied, as
 *     in ref_walk).  hit_step / watch_step: the first iteration count after which the best ISL
 *     is <= target_isl / watch_isl (0 for the start).
 *   - flip_evals: n per iteration, less the neighbours skipped by the second table (a
 *     neighbour in HT counts, as in ref_walk).  A neighbour in HT is not recorded in the
 *     second table.
 *   - trace per iteration: (j when the new S is the current state's flip-j neighbour, -2 when it
 *     is an older queue entry, -1 on a trap restart; ISL of the new S).
 * With Q = 1 and no second table the queue holds exactly the best unvisited neighbour of the
 * current state after each iteration, so the search coincides with ref_walk.
 * The second table uses the visited table's layout and hash (own size nbr_log2; 0 = absent).
 * ---------------------------------------------------------------------------------------- */
typedef struct {
    int64_t isl;
    int64_t gen; /* iteration that generated the entry */
    int32_t j;   /* flip of the generating state */
    uint64_t x[ORACLE_MAX_WORDS];
} pq_entry;

static int pq_before(const pq_entry *a, const pq_entry *b)
{
    if (a->isl != b->isl)
        return a->isl < b->isl;
    if (a->gen != b->gen)
        return a->gen < b->gen;
    return a->j < b->j;
}

int ref_pq_walk(const ref_walk_cfg *cfg, int32_t capacity, int32_t nbr_log2, ref_walk_result *res,
                int32_t *trace, int32_t *score_trace)
{
    const int32_t L = cfg->L;
    if (L < 3 || (L % 2) == 0 || cfg->steps < 0 || cfg->table_log2 < 1 || cfg->table_log2 > 30 ||
        capacity < 1 || nbr_log2 < 0 || nbr_log2 > 30)
        return -1;
    const int32_t n = (L + 1) / 2;
    const int32_t nwords = (n + 63) / 64;
    if (nwords > ORACLE_MAX_WORDS)
        return -1;

    int8_t *s = (int8_t *)malloc((size_t)L);
    int64_t *C = (int64_t *)malloc(sizeof(int64_t) * (size_t)L);
    uint64_t *z = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    pq_entry *Q = (pq_entry *)malloc(sizeof(pq_entry) * (size_t)capacity);
    uint8_t *nbr_seen = (uint8_t *)malloc((size_t)n);
    int32_t q = 0;
    uint64_t x[ORACLE_MAX_WORDS], xn[ORACLE_MAX_WORDS];
    memset(x, 0, sizeof x);
    memset(xn, 0, sizeof xn);
    for (int32_t j = 0; j < n; j++)
        z[j] = ref_zobrist(j);

    bounded_table B, N;
    B.log2 = cfg->table_log2;
    B.exact = (n <= cfg->table_log2);
    B.T = (uint64_t *)calloc((size_t)1 << B.log2, sizeof(uint64_t));
    N.log2 = nbr_log2;
    N.exact = nbr_log2 > 0 && (n <= nbr_log2);
    N.T = nbr_log2 > 0 ? (uint64_t *)calloc((size_t)1 << nbr_log2, sizeof(uint64_t)) : NULL;

    int64_t isl = 0;
    uint64_t h = 0;
    uint32_t restart = 0;

    memset(res, 0, sizeof *res);
    res->hit_step = -1;
    res->watch_step = -1;

#define PQ_START()                                                                             \
    do {                                                                                       \
        ref_start_bits(L, cfg->seed, cfg->walk_id, restart, x, nwords);                        \
        ref_skew_expand(L, x, s);                                                              \
        isl = ref_isl(L, s);                                                                   \
        h = 0;                                                                                 \
        for (int32_t j = 0; j < n; j++)                                                        \
            if ((x[j / 64] >> (j % 64)) & 1u)                                                  \
                h ^= z[j];                                                                     \
        memset(B.T, 0, sizeof(uint64_t) * ((size_t)1 << B.log2));                              \
        B.T[table_slot(&B, h, x)] = h | 1u;                                                    \
        if (N.T)                                                                               \
            memset(N.T, 0, sizeof(uint64_t) * ((size_t)1 << N.log2));                          \
        q = 0;                                                                                 \
    } while (0)

    PQ_START();
    res->best_isl = isl;
    res->best_step = 0;
    to_u32_words(x, nwords, res->best_bits);
    if (cfg->target_isl >= 0 && isl <= cfg->target_isl)
        res->hit_step = 0;
    if (cfg->watch_isl >= 0 && isl <= cfg->watch_isl)
        res->watch_step = 0;

    int64_t t = 0, flips = 0;
    while (t < cfg->steps && !(cfg->target_isl >= 0 && res->hit_step >= 0)) {
        /* search the neighbourhood (scores by the pinned one-flip evaluation); the second table
         * is consulted as it stood before this iteration */
        ref_corr(L, s, C);
        for (int32_t j = 0; j < n; j++) {
            memcpy(xn, x, sizeof x);
            xn[j / 64] ^= (uint64_t)1 << (j % 64);
            const uint64_t hn = h ^ z[j];
            nbr_seen[j] = N.T && N.T[table_slot(&N, hn, xn)] == (hn | 1u);
        }
        for (int32_t j = 0; j < n; j++) {
            memcpy(xn, x, sizeof x);
            xn[j / 64] ^= (uint64_t)1 << (j % 64);
            const uint64_t hn = h ^ z[j];
            const int64_t v = ref_flip_isl_incr(L, s, C, j);
            if (score_trace)
                score_trace[t * n + j] = (int32_t)v;
            if (nbr_seen[j])
                continue;
            flips++;
            if (B.T[table_slot(&B, hn, xn)] == (hn | 1u))
                continue;
            if (N.T)
                N.T[table_slot(&N, hn, xn)] = hn | 1u;
            pq_entry e;
            e.isl = v;
            e.gen = t;
            e.j = j;
            memcpy(e.x, xn, sizeof e.x);
            if (q < capacity) {
                Q[q++] = e;
            } else {
                int32_t w = 0;
                for (int32_t i = 1; i < q; i++)
                    if (pq_before(&Q[w], &Q[i]))
                        w = i;
                if (pq_before(&e, &Q[w]))
                    Q[w] = e;
            }
            if (v < res->best_isl) {
                res->best_isl = v;
                res->best_step = t + 1;
                to_u32_words(xn, nwords, res->best_bits);
            }
        }
        /* take the front of the queue, skipping states visited since they were queued */
        int found = 0;
        pq_entry f;
        while (q > 0) {
            int32_t b = 0;
            for (int32_t i = 1; i < q; i++)
                if (pq_before(&Q[i], &Q[b]))
                    b = i;
            f = Q[b];
            Q[b] = Q[--q];
            uint64_t hf = 0;
            for (int32_t j = 0; j < n; j++)
                if ((f.x[j / 64] >> (j % 64)) & 1u)
                    hf ^= z[j];
            if (B.T[table_slot(&B, hf, f.x)] == (hf | 1u))
                continue;
            found = 1;
            break;
        }
        int32_t move;
        if (!found) {
            res->traps++;
            res->restarts++;
            restart++;
            PQ_START();
            move = -1;
            /* a restart state counts like the initial state (see ref_walk) */
            if (isl < res->best_isl) {
                res->best_isl = isl;
                res->best_step = t + 1;
                to_u32_words(x, nwords, res->best_bits);
            }
        } else {
            move = (f.gen == t) ? f.j : -2;
            memcpy(x, f.x, sizeof x);
            ref_skew_expand(L, x, s);
            isl = ref_isl(L, s);
            if (isl != f.isl) {
                free(s); free(C); free(z); free(Q); free(nbr_seen); free(B.T); free(N.T);
                return -2;
            }
            h = 0;
            for (int32_t j = 0; j < n; j++)
                if ((x[j / 64] >> (j % 64)) & 1u)
                    h ^= z[j];
            B.T[table_slot(&B, h, x)] = h | 1u;
        }
        t++;
        if (trace) {
            trace[2 * t - 2] = move;
            trace[2 * t - 1] = (int32_t)isl;
        }
        if (cfg->target_isl >= 0 && res->hit_step < 0 && res->best_isl <= cfg->target_isl)
            res->hit_step = t;
        if (cfg->watch_isl >= 0 && res->watch_step < 0 && res->best_isl <= cfg->watch_isl)
            res->watch_step = t;
        if (found && cfg->restart_period > 0 && t % cfg->restart_period == 0 && t < cfg->steps &&
            !(cfg->target_isl >= 0 && res->hit_step >= 0)) {
            res->restarts++;
            restart++;
            PQ_START();
            if (isl < res->best_isl) {
                res->best_isl = isl;
                res->best_step = t;
                to_u32_words(x, nwords, res->best_bits);
            }
            if (cfg->target_isl >= 0 && res->hit_step < 0 && res->best_isl <= cfg->target_isl)
                res->hit_step = t;
            if (cfg->watch_isl >= 0 && res->watch_step < 0 && res->best_isl <= cfg->watch_isl)
                res->watch_step = t;
        }
    }
#undef PQ_START

    res->steps_done = t;
    res->flip_evals = flips;
    res->final_isl = isl;
    to_u32_words(x, nwords, res->final_bits);
    free(s);
    free(C);
    free(z);
    free(Q);
    free(nbr_seen);
    free(B.T);
    free(N.T);
    return 0;
}

/* ------------------------------------------------------------------------------------------
 * First-improvement search with perturbations: the method of Dimitrov et al. as Section 2
 * describes it.  Like lssOrel it moves by single flips of the free symbols, but it moves at
 * once to the first flip that improves the merit factor and starts a new scan from that
 * sequence; when no flip improves it (a local minimum of the one-flip neighbourhood) it flips a
 * few randomly chosen symbols and goes on from there.  Merit factors of flips come from the
 * stored correlation values C_k (the one-dimensional structure Section 2 mentions).
 * Readings of what the paper leaves open:
 *   - scan order: flips j = 0 .. c in index order, from j = 0 again after every move; a flip
 *     improves when its ISL is strictly lower than the current ISL.
 *   - perturbation: P distinct free symbols (P is a parameter, 1 <= P <= min(n, 32)); the k-th
 *     perturbation of the walk (k = 0, 1, ... counted over the whole walk, restarts included)
 *     draws words u_i = sm64_at(sm64_at(sm64_at(seed, walk_id), 2^32 + k), i), i = 0, 1, ...,
 *     takes j_i = floor((u_i >> 32) * n / 2^32) and skips indices already drawn, until P are
 *     chosen (or 65536 words are drawn).  The perturbed sequence becomes the current one whatever
 *     its ISL.
 *   - one step = one scan: an improving move, or (no improving flip) a perturbation.  Function
 *     evaluations (Section 3's unit): j + 1 for a move at flip j (flips 0 .. j were evaluated), n
 *     + P for a perturbation (the n evaluated flips and the P flips applied).
 *   - no visited table; restarts (restart_period), target and watch as in ref_walk; every
 *     occupied state counts for best, hit and watch, start states included.
 *   - results as ref_walk, with traps = the number of perturbations; trace per step (j of the
 *     move, or -1 for a perturbation; ISL after the step); score trace: the ISL of every flip of
 *     the state the step started from.
 * ---------------------------------------------------------------------------------------- */

/* Free symbols flipped by perturbation k of a walk (the draw stated above), in draw order; the
 * number found (P, unless 65536 draws did not find P distinct symbols, which a uniform draw of P
 * <= n <= 192 symbols makes vanishingly unlikely; then the ones found). */
int32_t ref_perturb_indices(int32_t n, uint64_t seed, uint32_t walk_id, uint64_t k, int32_t P, int32_t *out)
{
    const uint64_t kw = ref_sm64_at(seed, walk_id);
    const uint64_t kp = ref_sm64_at(kw, ((uint64_t)1 << 32) + k);
    int32_t got = 0;
    for (uint64_t i = 0; got < P && i < 65536; i++) {
        const uint64_t u = ref_sm64_at(kp, i);
        const int32_t j = (int32_t)(((u >> 32) * (uint64_t)n) >> 32);
        int dup = 0;
        for (int32_t q = 0; q < got; q++)
            if (out[q] == j)
                dup = 1;
        if (!dup)
            out[got++] = j;
    }
    return got;
}

int ref_fi_walk(const ref_walk_cfg *cfg, int32_t perturb, ref_walk_result *res, int32_t *trace,
                int32_t *score_trace)
{
    const int32_t L = cfg->L;
    if (L < 3 || (L % 2) == 0 || cfg->steps < 0)
        return -1;
    const int32_t n = (L + 1) / 2, c = n - 1;
    const int32_t nwords = (n + 63) / 64;
    if (nwords > ORACLE_MAX_WORDS || perturb < 1 || perturb > n || perturb > 32)
        return -1;
    const int brute = (cfg->flags & ORACLE_BRUTE) != 0;

    int8_t *s = (int8_t *)malloc((size_t)L);
    int64_t *C = (int64_t *)malloc(sizeof(int64_t) * (size_t)L);
    int64_t *score = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    uint64_t x[ORACLE_MAX_WORDS];
    int32_t pick[32];
    memset(x, 0, sizeof x);
    int64_t isl = 0;
    uint32_t restart = 0;
    uint64_t kpert = 0;

    memset(res, 0, sizeof *res);
    res->hit_step = -1;
    res->watch_step = -1;
    res->best_isl = INT64_MAX;

#define FI_START()                                                                             \
    do {                                                                                       \
        ref_start_bits(L, cfg->seed, cfg->walk_id, restart, x, nwords);                        \
        ref_skew_expand(L, x, s);                                                              \
        isl = ref_isl(L, s);                                                                   \
    } while (0)
#define FI_NOTE(t_)                                                                            \
    do {                                                                                       \
        if (isl < res->best_isl) {                                                             \
            res->best_isl = isl;                                                               \
            res->best_step = (t_);                                                             \
            to_u32_words(x, nwords, res->best_bits);                                           \
        }                                                                                      \
        if (cfg->target_isl >= 0 && res->hit_step < 0 && isl <= cfg->target_isl)             \
            res->hit_step = (t_);                                                              \
        if (cfg->watch_isl >= 0 && res->watch_step < 0 && isl <= cfg->watch_isl)             \
            res->watch_step = (t_);                                                            \
    } while (0)
/* negate free symbol j (and its mirror unless j is the centre) */
#define FI_FLIP(j_)                                                                            \
    do {                                                                                       \
        s[(j_)] = (int8_t)(-s[(j_)]);                                                          \
        if ((j_) != c)                                                                         \
            s[L - 1 - (j_)] = (int8_t)(-s[L - 1 - (j_)]);                                      \
        x[(j_) / 64] ^= (uint64_t)1 << ((j_) % 64);                                            \
    } while (0)

    FI_START();
    FI_NOTE(0);
    int64_t t = 0, flips = 0;
    int rc = 0;
    while (t < cfg->steps && !(cfg->target_isl >= 0 && res->hit_step >= 0)) {
        ref_corr(L, s, C);
        for (int32_t j = 0; j < n; j++)
            score[j] = brute ? ref_flip_isl_brute(L, s, j) : ref_flip_isl_incr(L, s, C, j);
        if (score_trace)
            for (int32_t j = 0; j < n; j++)
                score_trace[t * n + j] = (int32_t)score[j];
        /* the scan: the first flip in index order that improves the current ISL */
        int32_t jb = -1;
        for (int32_t j = 0; j < n && jb < 0; j++)
            if (score[j] < isl)
                jb = j;
        int32_t move;
        if (jb >= 0) {
            FI_FLIP(jb);
            flips += jb + 1;
            isl = ref_isl(L, s);
            if (isl != score[jb]) {
                rc = -2;
                break;
            }
            move = jb;
        } else {
            /* a local minimum: perturb P randomly chosen free symbols */
            const int32_t np = ref_perturb_indices(n, cfg->seed, cfg->walk_id, kpert, perturb, pick);
            kpert++;
            for (int32_t q = 0; q < np; q++)
                FI_FLIP(pick[q]);
            flips += n + np;
            isl = ref_isl(L, s);
            res->traps++;
            move = -1;
        }
        t++;
        if (trace) {
            trace[2 * t - 2] = move;
            trace[2 * t - 1] = (int32_t)isl;
        }
        FI_NOTE(t);
        if (cfg->restart_period > 0 && t % cfg->restart_period == 0 && t < cfg->steps &&
            !(cfg->target_isl >= 0 && res->hit_step >= 0)) {
            res->restarts++;
            restart++;
            FI_START();
            FI_NOTE(t);
        }
    }
#undef FI_FLIP
#undef FI_NOTE
#undef FI_START

    res->steps_done = t;
    res->flip_evals = flips;
    res->final_isl = isl;
    to_u32_words(x, nwords, res->final_bits);
    free(s);
    free(C);
    free(score);
    return rc;
}
