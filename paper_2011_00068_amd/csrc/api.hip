// api.hip -- the C ABI of liblabs (include/labs.h): argument checking, device memory, launch
// plans, hipGraph capture and the autotuner.  No step of the search runs on the CPU: apart from
// the conversions of a stop parameter and of sequence notation (labs_isl_threshold,
// labs_from_hex, labs_to_hex), every entry point ends in the library's kernels.

#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <sys/stat.h>
#include <vector>

#include "internal.hpp"

namespace liblabs {

static thread_local char g_last_error[512] = "";

int fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof g_last_error, fmt, ap);
    va_end(ap);
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(LABS_ENOMEM, "%s: %s", what, hipGetErrorString(e));
    return fail(LABS_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                                                                           \
    do {                                                                                              \
        hipError_t e_ = (expr);                                                                       \
        if (e_ != hipSuccess)                                                                         \
            return hip_fail(e_, what);                                                                \
    } while (0)

int check_device()
{
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count <= 0)
        return fail(LABS_EDEVICE, "no HIP device visible (%s)", hipGetErrorString(e));
    return LABS_OK;
}

static std::string device_arch()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return "unknown";
    std::string a = prop.gcnArchName;
    const size_t colon = a.find(':');
    return colon == std::string::npos ? a : a.substr(0, colon);
}

int walk_cfg_check(const labs_walk_cfg &c, int idx)
{
    if (c.L < 3 || c.L > LABS_WALK_L_MAX || (c.L % 2) == 0)
        return fail(LABS_EINVAL, "walk %d: L = %d must be odd and in [3, %d]", idx, c.L, LABS_WALK_L_MAX);
    if (c.table_log2 < 1 || c.table_log2 > 30)
        return fail(LABS_EINVAL, "walk %d: table_log2 = %d must be in [1, 30]", idx, c.table_log2);
    if (c.steps < 0)
        return fail(LABS_EINVAL, "walk %d: steps < 0", idx);
    if (c.restart_period < 0)
        return fail(LABS_EINVAL, "walk %d: restart_period < 0", idx);
    if (c.target_isl < -1 || c.watch_isl < -1)
        return fail(LABS_EINVAL, "walk %d: target_isl / watch_isl must be >= -1", idx);
    if (c.flags & ~(LABS_TRACE | LABS_TRACE_SCORES))
        return fail(LABS_EINVAL, "walk %d: unknown flags 0x%x", idx, c.flags);
    if (c.steps > ((int64_t)1 << 40))
        return fail(LABS_EINVAL, "walk %d: steps above 2^40", idx);
    return LABS_OK;
}

} // namespace liblabs

using namespace liblabs;

// =============================================================================================
// Errors, device.
// =============================================================================================
extern "C" const char *labs_strerror(int status)
{
    switch (status) {
    case LABS_OK: return "ok";
    case LABS_EINVAL: return "invalid argument";
    case LABS_ENOTSKEW: return "sequence is not skew-symmetric";
    case LABS_ENOMEM: return "out of memory";
    case LABS_EPENDING: return "pending";
    case LABS_ENOTFOUND: return "not found";
    case LABS_EDEVICE: return "device error";
    case LABS_EDOM: return "undefined result";
    case LABS_ECANCELLED: return "cancelled";
    default: return "unknown status";
    }
}

extern "C" const char *labs_last_error(void) { return g_last_error; }

extern "C" int labs_device_info(char *name, int32_t cap, int32_t *compute_units, int32_t *clock_khz)
{
    int rc = check_device();
    if (rc)
        return rc;
    int dev = 0;
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    HIP_TRY(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
    if (name && cap > 0) {
        snprintf(name, (size_t)cap, "%s", prop.gcnArchName);
    }
    if (compute_units)
        *compute_units = prop.multiProcessorCount;
    if (clock_khz)
        *clock_khz = prop.clockRate;
    return LABS_OK;
}

extern "C" int labs_probe_lds_read(int32_t bytes_per_lane, double *bytes_per_s, double *ms_out)
{
    if (bytes_per_lane != 4 && bytes_per_lane != 8 && bytes_per_lane != 16)
        return fail(LABS_EINVAL, "bytes_per_lane = %d must be 4, 8 or 16", bytes_per_lane);
    if (!bytes_per_s)
        return fail(LABS_EINVAL, "NULL bytes_per_s");
    int rc = check_device();
    if (rc)
        return rc;
    int dev = 0;
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDevice(&dev), "hipGetDevice");
    HIP_TRY(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
    // 16 blocks per CU (two resident at a time: 64 KB of LDS each); 0.5-1 ms a launch
    const int blocks = 16 * std::max(1, prop.multiProcessorCount);
    const int rounds = 512;
    uint32_t *d_out = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    float best = -1.0f;
    hipError_t e = hipMalloc(&d_out, (size_t)blocks * lds_probe_threads() * sizeof(uint32_t));
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) e = launch_lds_read_probe(bytes_per_lane, blocks, rounds, d_out, nullptr);
    for (int r = 0; r < 5 && e == hipSuccess; r++) {
        e = hipEventRecord(a, nullptr);
        if (e == hipSuccess) e = launch_lds_read_probe(bytes_per_lane, blocks, rounds, d_out, nullptr);
        if (e == hipSuccess) e = hipEventRecord(b, nullptr);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (e == hipSuccess && (best < 0.0f || ms < best))
            best = ms;
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (d_out) (void)hipFree(d_out);
    if (e != hipSuccess)
        return hip_fail(e, "labs_probe_lds_read");
    if (best <= 0.0f)
        return fail(LABS_EDEVICE, "labs_probe_lds_read: no measurable time");
    *bytes_per_s = lds_probe_bytes(bytes_per_lane, blocks, rounds) / (best * 1e-3);
    if (ms_out)
        *ms_out = best;
    return LABS_OK;
}

// =============================================================================================
// Definitions: labs_isl, labs_merit, labs_isl_batch_dev, labs_enum_skew_dev.
// =============================================================================================
static int isl_one(int32_t L, const int8_t *s, int64_t *isl_out, double *F_out)
{
    if (!s || L < 1 || L > 65535)
        return fail(LABS_EINVAL, "L = %d out of [1, 65535] or NULL sequence", L);
    for (int32_t i = 0; i < L; i++)
        if (s[i] != 1 && s[i] != -1)
            return fail(LABS_EINVAL, "s[%d] = %d is not +1 or -1", i, (int)s[i]);
    int rc = check_device();
    if (rc)
        return rc;
    int8_t *d_s = nullptr;
    int64_t *d_isl = nullptr;
    double *d_F = nullptr;
    int64_t isl = 0;
    double F = 0.0;
    hipError_t e = hipMalloc(&d_s, (size_t)L);
    if (e == hipSuccess) e = hipMalloc(&d_isl, sizeof(int64_t));
    if (e == hipSuccess) e = hipMalloc(&d_F, sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(d_s, s, (size_t)L, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_isl_batch(L, 1, d_s, d_isl, d_F, nullptr, nullptr, nullptr);
    if (e == hipSuccess) e = hipMemcpy(&isl, d_isl, sizeof isl, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(&F, d_F, sizeof F, hipMemcpyDeviceToHost);
    if (d_s) (void)hipFree(d_s);
    if (d_isl) (void)hipFree(d_isl);
    if (d_F) (void)hipFree(d_F);
    if (e != hipSuccess)
        return hip_fail(e, "labs_isl");
    if (isl_out)
        *isl_out = isl;
    if (F_out) {
        if (isl == 0)
            return fail(LABS_EDOM, "F is undefined for ISL = 0 (L = %d)", L);
        *F_out = F;
    }
    return LABS_OK;
}

extern "C" int labs_isl(int32_t L, const int8_t *s, int64_t *isl_out)
{
    if (!isl_out)
        return fail(LABS_EINVAL, "NULL isl_out");
    return isl_one(L, s, isl_out, nullptr);
}

extern "C" int labs_merit(int32_t L, const int8_t *s, double *F_out)
{
    if (!F_out)
        return fail(LABS_EINVAL, "NULL F_out");
    return isl_one(L, s, nullptr, F_out);
}

extern "C" int labs_isl_threshold(int32_t L, int64_t num, int64_t den, int64_t *isl_out)
{
    if (!isl_out)
        return fail(LABS_EINVAL, "NULL isl_out");
    if (L < 1 || L > 65535 || num <= 0 || den <= 0)
        return fail(LABS_EINVAL, "labs_isl_threshold: L = %d, num = %lld, den = %lld (need 1 <= L <= 65535, "
                    "num > 0, den > 0)", L, (long long)num, (long long)den);
    // F >= num/den  <=>  L^2 / (2 ISL) >= num/den  <=>  ISL <= L^2 den / (2 num)   (Eq. (3))
    const __int128 v = (__int128)L * L * den / ((__int128)2 * num);
    *isl_out = (int64_t)std::min<__int128>(v, (__int128)INT64_MAX);
    return LABS_OK;
}

// The sequence notation of Table 1 (Section 4): hex digits, 4 bits each with the most significant
// first, leading zero bits dropped down to L symbols, bit 0 = +1 and bit 1 = -1.
extern "C" int labs_from_hex(const char *hex, int32_t L, int8_t *s_out)
{
    if (!hex || !s_out || L < 1 || L > 65535)
        return fail(LABS_EINVAL, "labs_from_hex: L = %d (need 1 <= L <= 65535) and non-NULL pointers", L);
    const size_t nd = strlen(hex);
    if (4 * (uint64_t)nd < (uint64_t)L)
        return fail(LABS_EINVAL, "labs_from_hex: %zu digits do not hold %d symbols", nd, L);
    // symbols from the last digit backwards: bit q (weight 2^q) of digit nd-1-d is symbol L-1-4d-q;
    // the first pass checks every digit and dropped bit, so that s_out is written only on success
    auto digit = [](char ch) {
        return (ch >= '0' && ch <= '9') ? ch - '0'
               : (ch >= 'a' && ch <= 'f') ? ch - 'a' + 10
               : (ch >= 'A' && ch <= 'F') ? ch - 'A' + 10 : -1;
    };
    for (int pass = 0; pass < 2; pass++) {
        for (size_t d = 0; d < nd; d++) {
            const char ch = hex[nd - 1 - d];
            const int v = digit(ch);
            if (v < 0)
                return fail(LABS_EINVAL, "labs_from_hex: '%c' is not a hex digit", ch);
            for (int q = 0; q < 4; q++) {
                const int64_t i = (int64_t)L - 1 - 4 * (int64_t)d - q;
                const int bit = (v >> q) & 1;
                if (i < 0 && bit)
                    return fail(LABS_EINVAL, "labs_from_hex: a dropped leading bit is 1 (more than %d symbols)", L);
                if (pass == 1 && i >= 0)
                    s_out[i] = (int8_t)(1 - 2 * bit);
            }
        }
    }
    return LABS_OK;
}

extern "C" int labs_to_hex(int32_t L, const int8_t *s, char *out, int32_t cap)
{
    if (!s || !out || L < 1 || L > 65535)
        return fail(LABS_EINVAL, "labs_to_hex: L = %d (need 1 <= L <= 65535) and non-NULL pointers", L);
    const int32_t nd = (L + 3) / 4;
    if (cap < nd + 1)
        return fail(LABS_EINVAL, "labs_to_hex: cap = %d, need %d", cap, nd + 1);
    for (int32_t d = 0; d < nd; d++) {
        int v = 0;
        for (int q = 0; q < 4; q++) {
            const int32_t i = L - 1 - 4 * d - q;
            if (i < 0)
                break;
            if (s[i] != 1 && s[i] != -1)
                return fail(LABS_EINVAL, "labs_to_hex: s[%d] = %d is not +1 or -1", i, s[i]);
            v |= (s[i] < 0) << q;
        }
        out[nd - 1 - d] = "0123456789ABCDEF"[v];
    }
    out[nd] = '\0';
    return LABS_OK;
}

extern "C" int labs_isl_batch_dev(int32_t L, int32_t count, const int8_t *s_dev, int64_t *isl_dev, double *F_dev,
                                  int32_t *psl_dev, int32_t *corr_dev, void *stream)
{
    if (L < 1 || L > 65535 || count < 0 || (count > 0 && (!s_dev || !isl_dev)))
        return fail(LABS_EINVAL, "labs_isl_batch_dev: bad arguments (L = %d, count = %d)", L, count);
    int rc = check_device();
    if (rc)
        return rc;
    HIP_TRY(launch_isl_batch(L, count, s_dev, isl_dev, F_dev, psl_dev, corr_dev, (hipStream_t)stream),
            "labs_isl_batch_dev");
    return LABS_OK;
}

extern "C" int labs_enum_skew_dev(int32_t L, int32_t *isl_dev, void *stream)
{
    if (L < 3 || L > 47 || (L % 2) == 0 || !isl_dev)
        return fail(LABS_EINVAL, "labs_enum_skew_dev: L = %d must be odd in [3, 47]", L);
    int rc = check_device();
    if (rc)
        return rc;
    HIP_TRY(launch_enum_skew(L, isl_dev, (hipStream_t)stream), "labs_enum_skew_dev");
    return LABS_OK;
}

extern "C" int labs_enum_skew_min(int32_t L, uint64_t r_begin, uint64_t r_end, labs_enum_min_result *out,
                                  void *stream)
{
    if (!out)
        return fail(LABS_EINVAL, "labs_enum_skew_min: NULL result");
    if (L < 3 || L > 125 || (L % 2) == 0)
        return fail(LABS_EINVAL, "labs_enum_skew_min: L = %d must be odd in [3, 125]", L);
    const int n = (L + 1) / 2;
    const uint64_t groups = 1ull << (n - 2);
    if (r_begin > r_end || r_end > groups)
        return fail(LABS_EINVAL, "labs_enum_skew_min: block [%llu, %llu) outside [0, 2^%d)",
                    (unsigned long long)r_begin, (unsigned long long)r_end, n - 2);
    memset(out, 0, sizeof *out);
    out->min_isl = -1;
    if (r_begin == r_end)
        return LABS_OK;
    int rc = check_device();
    if (rc)
        return rc;
    const int blocks = enum_min_blocks(L);
    if (blocks <= 0)
        return fail(LABS_EDEVICE, "labs_enum_skew_min: occupancy query failed");
    hipStream_t s = (hipStream_t)stream;
    // launches of at most 2^32 groups and at most 2^20 passes per lane, so that per-wave counts
    // stay far below 2^31 inside a launch
    const uint64_t cap = std::min<uint64_t>(1ull << 32, (uint64_t)blocks * 256ull * 4ull * (1ull << 20));
    EnumPartial *part = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    EnumPartial res{};
    float ms = 0.0f;
    hipError_t e = hipMalloc(&part, sizeof(EnumPartial) * (size_t)(blocks + 1));
    if (e == hipSuccess) e = hipEventCreate(&ev0);
    if (e == hipSuccess) e = hipEventCreate(&ev1);
    if (e == hipSuccess) e = launch_enum_part_init(part, blocks, s);
    if (e == hipSuccess) e = hipEventRecord(ev0, s);
    for (uint64_t r = r_begin; e == hipSuccess && r < r_end;) {
        const uint64_t cnt = std::min<uint64_t>(r_end - r, cap);
        e = launch_enum_min(L, r, cnt, part, blocks, s);
        r += cnt;
    }
    if (e == hipSuccess) e = launch_enum_final(part, blocks, part + blocks, s);
    if (e == hipSuccess) e = hipEventRecord(ev1, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&res, part + blocks, sizeof res, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev0, ev1);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (part) (void)hipFree(part);
    if (e != hipSuccess)
        return hip_fail(e, "labs_enum_skew_min");
    out->min_isl = res.min_isl == 0xFFFFFFFFu ? -1 : (int32_t)res.min_isl;
    out->count = res.count;
    out->first_x = res.min_isl == 0xFFFFFFFFu ? 0 : res.first_x;
    out->states = 4 * (r_end - r_begin);
    out->kernel_ms = (double)ms;
    out->word_ops = res.word_ops;
    return LABS_OK;
}

extern "C" int labs_flip_scores_dev(int32_t L, int32_t count, const uint32_t *x_dev, int32_t *scores_dev,
                                    int32_t variant, void *stream)
{
    if (L < 3 || L > LABS_WALK_L_MAX || (L % 2) == 0 || count < 0 || (count > 0 && (!x_dev || !scores_dev)))
        return fail(LABS_EINVAL, "labs_flip_scores_dev: bad arguments (L = %d, count = %d)", L, count);
    if (variant == LABS_VARIANT_AUTO)
        variant = LABS_VARIANT_BITSLICE;
    if (variant != LABS_VARIANT_BITSLICE && variant != LABS_VARIANT_DIRECT && variant != LABS_VARIANT_MFMA)
        return fail(LABS_EINVAL, "labs_flip_scores_dev: unknown variant %d", variant);
    if (variant == LABS_VARIANT_MFMA && L > kMfmaLMax)
        return fail(LABS_EINVAL, "labs_flip_scores_dev: the matrix-core variant needs L <= %d", kMfmaLMax);
    int rc = check_device();
    if (rc)
        return rc;
    HIP_TRY(launch_flip_scores(variant, L, count, x_dev, scores_dev, (hipStream_t)stream), "labs_flip_scores_dev");
    return LABS_OK;
}

// =============================================================================================
// Walk plans.
// =============================================================================================
struct labs_walk_plan {
    int32_t n_walks = 0;
    std::vector<labs_walk_cfg> cfg;
    std::vector<WalkState> pristine;
    labs_plan_opts opts{};
    WalkLaunch lp{};
    int64_t max_steps = 0;
    int32_t launches_per_run = 0;
    int64_t trace_records = 0; // total (int32 pairs)
    int64_t score_entries = 0;
    WalkState *d_states = nullptr;
    WalkState *d_pristine = nullptr;
    uint64_t *d_tables = nullptr;
    int32_t *d_trace = nullptr;
    int32_t *d_scores = nullptr;
    int32_t *d_counter = nullptr;
    int32_t *d_order = nullptr;
    hipEvent_t ev0 = nullptr, ev_mid = nullptr, ev1 = nullptr; // run start, walks start, run end
    hipGraphExec_t graph_exec = nullptr;
    hipStream_t graph_stream = nullptr;
    bool ran = false;
    int32_t last_launches = 0;
};

namespace liblabs {

static int resolve_opts(labs_walk_plan *p, const labs_plan_opts *in);

static void plan_free(labs_walk_plan *p)
{
    if (!p)
        return;
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev_mid) (void)hipEventDestroy(p->ev_mid);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    if (p->d_states) (void)hipFree(p->d_states);
    if (p->d_pristine) (void)hipFree(p->d_pristine);
    if (p->d_tables) (void)hipFree(p->d_tables);
    if (p->d_trace) (void)hipFree(p->d_trace);
    if (p->d_scores) (void)hipFree(p->d_scores);
    if (p->d_counter) (void)hipFree(p->d_counter);
    if (p->d_order) (void)hipFree(p->d_order);
    delete p;
}

// Enqueue one full run: reset, then the walk launches.
static hipError_t enqueue_run(labs_walk_plan *p, hipStream_t s, int32_t *launches, bool mark)
{
    hipError_t e = launch_reset(p->d_states, p->d_pristine, p->n_walks, p->d_counter, s);
    if (e != hipSuccess)
        return e;
    if (mark) {
        e = hipEventRecord(p->ev_mid, s);
        if (e != hipSuccess)
            return e;
    }
    int32_t nl = 0;
    if (p->opts.plain) {
        // comparison form: one walk per launch, serialised on the stream
        WalkLaunch lp = p->lp;
        lp.persistent = 0;
        lp.waves_per_block = 1;
        for (int32_t i = 0; i < p->n_walks; i++) {
            for (int64_t done = 0; done < p->cfg[(size_t)i].steps || done == 0; done += lp.chunk) {
                e = launch_walk(lp, p->d_states, 1, p->d_order + i, p->d_tables, p->d_trace, p->d_scores, nullptr, s);
                if (e != hipSuccess)
                    return e;
                nl++;
                if (lp.chunk <= 0)
                    break;
            }
        }
    } else {
        for (int32_t r = 0; r < p->launches_per_run; r++) {
            if (r > 0 && p->lp.persistent) {
                e = launch_zero_counter(p->d_counter, s);
                if (e != hipSuccess)
                    return e;
            }
            e = launch_walk(p->lp, p->d_states, p->n_walks, p->d_order, p->d_tables, p->d_trace, p->d_scores,
                            p->d_counter, s);
            if (e != hipSuccess)
                return e;
            nl++;
        }
    }
    *launches = nl;
    return hipSuccess;
}

} // namespace liblabs

extern "C" int labs_walk_plan_create(int32_t n_walks, const labs_walk_cfg *cfg, const labs_plan_opts *opts,
                                     labs_walk_plan **plan)
{
    if (!plan)
        return fail(LABS_EINVAL, "NULL plan");
    *plan = nullptr;
    if (n_walks < 1 || !cfg)
        return fail(LABS_EINVAL, "n_walks = %d must be >= 1 with a cfg array", n_walks);
    for (int32_t i = 0; i < n_walks; i++) {
        int rc = walk_cfg_check(cfg[i], i);
        if (rc)
            return rc;
    }
    int rc = check_device();
    if (rc)
        return rc;
    labs_walk_plan *p = new labs_walk_plan();
    p->n_walks = n_walks;
    p->cfg.assign(cfg, cfg + n_walks);
    p->pristine.resize((size_t)n_walks);
    int64_t table_words = 0;
    for (int32_t i = 0; i < n_walks; i++) {
        const labs_walk_cfg &c = cfg[i];
        WalkState w;
        memset(&w, 0, sizeof w);
        w.L = c.L;
        w.table_log2 = c.table_log2;
        w.seed = c.seed;
        w.walk_id = c.walk_id;
        w.flags = c.flags;
        w.steps = c.steps;
        w.restart_period = c.restart_period;
        w.target_isl = c.target_isl;
        w.watch_isl = c.watch_isl;
        w.table_offset = table_words;
        table_words += (int64_t)1 << c.table_log2;
        const int n = (c.L + 1) / 2;
        if (c.flags & LABS_TRACE) {
            w.trace_offset = p->trace_records;
            p->trace_records += c.steps;
        } else {
            w.trace_offset = -1;
        }
        if (c.flags & LABS_TRACE_SCORES) {
            w.score_offset = p->score_entries;
            p->score_entries += c.steps * n;
        } else {
            w.score_offset = -1;
        }
        w.step_cap = INT64_MAX;
        w.hit_step = -1;
        w.watch_step = -1;
        w.status = kFresh;
        p->pristine[(size_t)i] = w;
        p->max_steps = std::max(p->max_steps, c.steps);
        // (each term is below 2^48, so the running sums cannot overflow before this test)
        if (p->trace_records > ((int64_t)1 << 40) || p->score_entries > ((int64_t)1 << 40) ||
            table_words > ((int64_t)1 << 40)) {
            plan_free(p);
            return fail(LABS_ENOMEM, "walk %d: trace, score or table buffers above 2^40 entries", i);
        }
    }
    rc = resolve_opts(p, opts);
    if (rc) {
        plan_free(p);
        return rc;
    }
    // walk order: costliest shape first (longest-first for mixed lengths), stable by index
    std::vector<int32_t> order((size_t)n_walks);
    for (int32_t i = 0; i < n_walks; i++)
        order[(size_t)i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        return cfg[a].L > cfg[b].L;
    });
    if (p->opts.plain) {
        for (int32_t i = 0; i < n_walks; i++)
            order[(size_t)i] = i;
    }
    hipError_t e = hipMalloc(&p->d_states, sizeof(WalkState) * (size_t)n_walks);
    if (e == hipSuccess) e = hipMalloc(&p->d_pristine, sizeof(WalkState) * (size_t)n_walks);
    if (e == hipSuccess) e = hipMalloc(&p->d_tables, sizeof(uint64_t) * (size_t)table_words);
    if (e == hipSuccess && p->trace_records > 0) e = hipMalloc(&p->d_trace, sizeof(int32_t) * 2 * (size_t)p->trace_records);
    if (e == hipSuccess && p->score_entries > 0) e = hipMalloc(&p->d_scores, sizeof(int32_t) * (size_t)p->score_entries);
    if (e == hipSuccess) e = hipMalloc(&p->d_counter, sizeof(int32_t));
    if (e == hipSuccess) e = hipMalloc(&p->d_order, sizeof(int32_t) * (size_t)n_walks);
    if (e == hipSuccess) e = hipMemcpy(p->d_pristine, p->pristine.data(), sizeof(WalkState) * (size_t)n_walks, hipMemcpyHostToDevice);
    // the states too: their table epochs (0: the tables' contents are unknown) carry over runs
    if (e == hipSuccess) e = hipMemcpy(p->d_states, p->pristine.data(), sizeof(WalkState) * (size_t)n_walks, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->d_order, order.data(), sizeof(int32_t) * (size_t)n_walks, hipMemcpyHostToDevice);
    if (e == hipSuccess && p->d_trace) e = hipMemset(p->d_trace, 0, sizeof(int32_t) * 2 * (size_t)p->trace_records);
    if (e == hipSuccess && p->d_scores) e = hipMemset(p->d_scores, 0, sizeof(int32_t) * (size_t)p->score_entries);
    if (e == hipSuccess) e = hipEventCreate(&p->ev0);
    if (e == hipSuccess) e = hipEventCreate(&p->ev_mid);
    if (e == hipSuccess) e = hipEventCreate(&p->ev1);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        plan_free(p);
        return hip_fail(e, "labs_walk_plan_create");
    }
    *plan = p;
    return LABS_OK;
}

extern "C" int labs_walk_plan_run(labs_walk_plan *p, void *stream)
{
    if (!p)
        return fail(LABS_EINVAL, "NULL plan");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(hipEventRecord(p->ev0, s), "hipEventRecord");
    int32_t nl = 0;
    if (p->opts.use_graph && !p->opts.plain) {
        if (!p->graph_exec || p->graph_stream != s) {
            if (p->graph_exec) {
                (void)hipGraphExecDestroy(p->graph_exec);
                p->graph_exec = nullptr;
            }
            hipStream_t cap = s;
            hipStream_t own = nullptr;
            if (cap == nullptr) {
                HIP_TRY(hipStreamCreate(&own), "hipStreamCreate");
                cap = own;
            }
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                hipError_t e2 = enqueue_run(p, cap, &nl, false);
                e = hipStreamEndCapture(cap, &g);
                if (e2 != hipSuccess)
                    e = e2;
            }
            if (e == hipSuccess)
                e = hipGraphInstantiate(&p->graph_exec, g, nullptr, nullptr, 0);
            if (g)
                (void)hipGraphDestroy(g);
            if (own)
                (void)hipStreamDestroy(own);
            if (e != hipSuccess)
                return hip_fail(e, "graph capture");
            p->graph_stream = s;
            p->launches_per_run = nl - 0; // informational
        }
        HIP_TRY(hipEventRecord(p->ev_mid, s), "hipEventRecord");
        HIP_TRY(hipGraphLaunch(p->graph_exec, s), "hipGraphLaunch");
        nl = p->launches_per_run;
    } else {
        hipError_t e = enqueue_run(p, s, &nl, true);
        if (e != hipSuccess)
            return hip_fail(e, "walk launch");
    }
    HIP_TRY(hipEventRecord(p->ev1, s), "hipEventRecord");
    p->ran = true;
    p->last_launches = nl;
    return LABS_OK;
}

extern "C" int labs_walk_plan_results(labs_walk_plan *p, labs_walk_result *out, int32_t *trace, int32_t *scores)
{
    if (!p)
        return fail(LABS_EINVAL, "NULL plan");
    if (!p->ran)
        return fail(LABS_EINVAL, "plan has not been run");
    HIP_TRY(hipEventSynchronize(p->ev1), "hipEventSynchronize");
    if (out) {
        std::vector<WalkState> st((size_t)p->n_walks);
        HIP_TRY(hipMemcpy(st.data(), p->d_states, sizeof(WalkState) * st.size(), hipMemcpyDeviceToHost), "results copy");
        for (int32_t i = 0; i < p->n_walks; i++) {
            const WalkState &w = st[(size_t)i];
            labs_walk_result &r = out[i];
            memset(&r, 0, sizeof r);
            r.best_isl = w.best_isl;
            r.best_step = w.best_step;
            r.steps_done = w.t;
            r.flip_evals = w.flips;
            r.hit_step = w.hit_step;
            r.watch_step = w.watch_step;
            r.final_isl = w.isl;
            r.restarts = w.restarts;
            r.traps = w.traps;
            for (int k = 0; k < kXWords; k++) {
                r.best_bits[k] = w.best_x[k];
                r.final_bits[k] = w.x[k];
            }
        }
    }
    if (trace && p->trace_records > 0)
        HIP_TRY(hipMemcpy(trace, p->d_trace, sizeof(int32_t) * 2 * (size_t)p->trace_records, hipMemcpyDeviceToHost),
                "trace copy");
    if (scores && p->score_entries > 0)
        HIP_TRY(hipMemcpy(scores, p->d_scores, sizeof(int32_t) * (size_t)p->score_entries, hipMemcpyDeviceToHost),
                "score copy");
    return LABS_OK;
}

extern "C" int labs_walk_plan_get_opts(const labs_walk_plan *p, labs_plan_opts *opts)
{
    if (!p || !opts)
        return fail(LABS_EINVAL, "NULL argument");
    *opts = p->opts;
    return LABS_OK;
}

extern "C" int labs_walk_plan_last_timing(const labs_walk_plan *p, double *ms, int32_t *launches)
{
    if (!p || !p->ran)
        return fail(LABS_EINVAL, "plan has not been run");
    HIP_TRY(hipEventSynchronize(p->ev1), "hipEventSynchronize");
    float f = 0.f;
    HIP_TRY(hipEventElapsedTime(&f, p->ev_mid, p->ev1), "hipEventElapsedTime");
    if (ms)
        *ms = (double)f;
    if (launches)
        *launches = p->last_launches;
    return LABS_OK;
}

extern "C" void labs_walk_plan_destroy(labs_walk_plan *p)
{
    if (p && p->ran)
        (void)hipEventSynchronize(p->ev1);
    plan_free(p);
}

extern "C" int labs_walk_batch(int32_t n_walks, const labs_walk_cfg *cfg, labs_walk_result *out, int32_t *trace,
                               int32_t *scores, void *stream)
{
    labs_walk_plan *p = nullptr;
    int rc = labs_walk_plan_create(n_walks, cfg, nullptr, &p);
    if (rc)
        return rc;
    rc = labs_walk_plan_run(p, stream);
    if (!rc)
        rc = labs_walk_plan_results(p, out, trace, scores);
    labs_walk_plan_destroy(p);
    return rc;
}

namespace liblabs {

// The synchronous one-launch-per-shape batches: the best-first search (nlog2, cap) and the
// general walk (general = true).
// The searches run to completion by one launch per kernel shape: the best-first search (cap,
// nlog2), the general walk, the first-improvement search (cap = perturbation size, no tables).
enum BatchKind { kBatchPq, kBatchGeneral, kBatchFi };

static int batch_sync(BatchKind kind, int32_t n_walks, const labs_walk_cfg *cfg, int cap, int nlog2,
                      labs_walk_result *out, int32_t *trace, int32_t *scores, double *kernel_ms, void *stream)
{
    const bool general = kind == kBatchGeneral;
    const char *what = general ? "labs_general_walk_batch" : (kind == kBatchFi ? "labs_fi_walk_batch" : "labs_pq_walk_batch");
    int rc = check_device();
    if (rc)
        return rc;
    std::vector<WalkState> st((size_t)n_walks);
    int64_t table_words = 0, trace_records = 0, score_entries = 0;
    for (int32_t i = 0; i < n_walks; i++) {
        const labs_walk_cfg &c = cfg[i];
        const int n = general ? c.L : (c.L + 1) / 2;
        WalkState &w = st[(size_t)i];
        memset(&w, 0, sizeof w);
        w.L = c.L;
        w.table_log2 = c.table_log2;
        w.seed = c.seed;
        w.walk_id = c.walk_id;
        w.flags = c.flags;
        w.steps = c.steps;
        w.restart_period = c.restart_period;
        w.target_isl = c.target_isl;
        w.watch_isl = c.watch_isl;
        w.table_offset = table_words;
        if (kind != kBatchFi)
            table_words += (int64_t)1 << c.table_log2;
        w.trace_offset = (c.flags & LABS_TRACE) ? trace_records : -1;
        if (c.flags & LABS_TRACE)
            trace_records += c.steps;
        w.score_offset = (c.flags & LABS_TRACE_SCORES) ? score_entries : -1;
        if (c.flags & LABS_TRACE_SCORES)
            score_entries += c.steps * n;
        w.step_cap = INT64_MAX;
        w.hit_step = -1;
        w.watch_step = -1;
        w.status = kFresh;
        if (trace_records > ((int64_t)1 << 40) || score_entries > ((int64_t)1 << 40) ||
            table_words > ((int64_t)1 << 40))
            return fail(LABS_ENOMEM, "walk %d: trace, score or table buffers above 2^40 entries", i);
    }
    // one launch per kernel shape, over the walks of that shape
    auto shape_of = [&](int L) { return general ? general_shape_for_length(L) : shape_for_length(L); };
    std::vector<int32_t> order((size_t)n_walks);
    std::vector<int32_t> first(9, 0);
    {
        std::vector<int32_t> count(8, 0);
        for (int32_t i = 0; i < n_walks; i++)
            count[(size_t)shape_of(cfg[i].L)]++;
        for (int s = 0; s < 8; s++)
            first[(size_t)s + 1] = first[(size_t)s] + count[(size_t)s];
        std::vector<int32_t> fill(first.begin(), first.end() - 1);
        for (int32_t i = 0; i < n_walks; i++)
            order[(size_t)fill[(size_t)shape_of(cfg[i].L)]++] = i;
    }
    hipStream_t s = (hipStream_t)stream;
    WalkState *d_st = nullptr;
    uint64_t *d_tables = nullptr, *d_nbr = nullptr;
    int32_t *d_trace = nullptr, *d_scores = nullptr, *d_order = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    float ms = 0.0f;
    hipError_t e = hipMalloc(&d_st, sizeof(WalkState) * (size_t)n_walks);
    if (e == hipSuccess && table_words > 0) e = hipMalloc(&d_tables, sizeof(uint64_t) * (size_t)table_words);
    if (e == hipSuccess && nlog2 > 0) e = hipMalloc(&d_nbr, sizeof(uint64_t) * ((size_t)n_walks << nlog2));
    if (e == hipSuccess && trace_records > 0) e = hipMalloc(&d_trace, sizeof(int32_t) * 2 * (size_t)trace_records);
    if (e == hipSuccess && score_entries > 0) e = hipMalloc(&d_scores, sizeof(int32_t) * (size_t)score_entries);
    if (e == hipSuccess) e = hipMalloc(&d_order, sizeof(int32_t) * (size_t)n_walks);
    if (e == hipSuccess) e = hipMemcpyAsync(d_st, st.data(), sizeof(WalkState) * (size_t)n_walks, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(d_order, order.data(), sizeof(int32_t) * (size_t)n_walks, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && d_trace) e = hipMemsetAsync(d_trace, 0, sizeof(int32_t) * 2 * (size_t)trace_records, s);
    if (e == hipSuccess && d_scores) e = hipMemsetAsync(d_scores, 0, sizeof(int32_t) * (size_t)score_entries, s);
    if (e == hipSuccess) e = hipEventCreate(&ev0);
    if (e == hipSuccess) e = hipEventCreate(&ev1);
    if (e == hipSuccess) e = hipEventRecord(ev0, s);
    for (int sh = 7; e == hipSuccess && sh >= 0; sh--) {
        const int32_t cnt = first[(size_t)sh + 1] - first[(size_t)sh];
        if (cnt <= 0)
            continue;
        if (general)
            e = launch_walk_general(sh, d_st, cnt, d_order + first[(size_t)sh], d_tables, d_trace, d_scores, s);
        else if (kind == kBatchFi)
            e = launch_fi_walk(sh, d_st, cnt, d_order + first[(size_t)sh], cap, d_trace, d_scores, s);
        else
            e = launch_pq_walk(sh, d_st, cnt, d_order + first[(size_t)sh], d_tables, d_nbr, nlog2, cap, d_trace,
                               d_scores, s);
    }
    if (e == hipSuccess) e = hipEventRecord(ev1, s);
    if (e == hipSuccess) e = hipMemcpyAsync(st.data(), d_st, sizeof(WalkState) * (size_t)n_walks, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && trace && d_trace)
        e = hipMemcpyAsync(trace, d_trace, sizeof(int32_t) * 2 * (size_t)trace_records, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && scores && d_scores)
        e = hipMemcpyAsync(scores, d_scores, sizeof(int32_t) * (size_t)score_entries, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev0, ev1);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    if (d_st) (void)hipFree(d_st);
    if (d_tables) (void)hipFree(d_tables);
    if (d_nbr) (void)hipFree(d_nbr);
    if (d_trace) (void)hipFree(d_trace);
    if (d_scores) (void)hipFree(d_scores);
    if (d_order) (void)hipFree(d_order);
    if (e != hipSuccess)
        return hip_fail(e, what);
    for (int32_t i = 0; i < n_walks; i++) {
        const WalkState &w = st[(size_t)i];
        labs_walk_result &r = out[i];
        memset(&r, 0, sizeof r);
        r.best_isl = w.best_isl;
        r.best_step = w.best_step;
        r.steps_done = w.t;
        r.flip_evals = w.flips;
        r.hit_step = w.hit_step;
        r.watch_step = w.watch_step;
        r.final_isl = w.isl;
        r.restarts = w.restarts;
        r.traps = w.traps;
        for (int k = 0; k < kXWords; k++) {
            r.best_bits[k] = w.best_x[k];
            r.final_bits[k] = w.x[k];
        }
    }
    if (kernel_ms)
        *kernel_ms = (double)ms;
    return LABS_OK;
}

} // namespace liblabs

extern "C" int labs_pq_walk_batch(int32_t n_walks, const labs_walk_cfg *cfg, const labs_pq_opts *opts,
                                  labs_walk_result *out, int32_t *trace, int32_t *scores, double *kernel_ms,
                                  void *stream)
{
    if (n_walks < 1 || !cfg || !opts || !out)
        return fail(LABS_EINVAL, "labs_pq_walk_batch: n_walks = %d with cfg, opts and out required", n_walks);
    if (opts->capacity < 1 || opts->capacity > 64)
        return fail(LABS_EINVAL, "labs_pq_walk_batch: capacity = %d must be in [1, 64]", opts->capacity);
    if (opts->nbr_table_log2 < 0 || opts->nbr_table_log2 > 30)
        return fail(LABS_EINVAL, "labs_pq_walk_batch: nbr_table_log2 = %d must be in [0, 30]", opts->nbr_table_log2);
    for (int32_t i = 0; i < n_walks; i++) {
        int rc = walk_cfg_check(cfg[i], i);
        if (rc)
            return rc;
        if (cfg[i].steps >= ((int64_t)1 << 31))
            return fail(LABS_EINVAL, "labs_pq_walk_batch: walk %d: steps must be below 2^31", i);
    }
    return batch_sync(kBatchPq, n_walks, cfg, opts->capacity, opts->nbr_table_log2, out, trace, scores, kernel_ms,
                      stream);
}

extern "C" int labs_fi_walk_batch(int32_t n_walks, const labs_walk_cfg *cfg, const labs_fi_opts *opts,
                                  labs_walk_result *out, int32_t *trace, int32_t *scores, double *kernel_ms,
                                  void *stream)
{
    if (n_walks < 1 || !cfg || !opts || !out)
        return fail(LABS_EINVAL, "labs_fi_walk_batch: n_walks = %d with cfg, opts and out required", n_walks);
    for (int32_t i = 0; i < n_walks; i++) {
        int rc = walk_cfg_check(cfg[i], i);
        if (rc)
            return rc;
        if (cfg[i].steps >= ((int64_t)1 << 31))
            return fail(LABS_EINVAL, "labs_fi_walk_batch: walk %d: steps must be below 2^31", i);
        const int n = (cfg[i].L + 1) / 2;
        if (opts->perturb_bits < 1 || opts->perturb_bits > 32 || opts->perturb_bits > n)
            return fail(LABS_EINVAL, "labs_fi_walk_batch: walk %d: perturb_bits = %d must be in [1, min(n, 32)] "
                        "(n = %d)", i, opts->perturb_bits, n);
    }
    return batch_sync(kBatchFi, n_walks, cfg, opts->perturb_bits, 0, out, trace, scores, kernel_ms, stream);
}

extern "C" int labs_general_flip_scores_dev(int32_t L, int32_t count, const uint32_t *x_dev, int32_t *scores_dev,
                                            void *stream)
{
    if (L < 3 || L > LABS_GENERAL_L_MAX || count < 0 || (count > 0 && (!x_dev || !scores_dev)))
        return fail(LABS_EINVAL, "labs_general_flip_scores_dev: bad arguments (L = %d, count = %d)", L, count);
    int rc = check_device();
    if (rc)
        return rc;
    HIP_TRY(launch_general_flip_scores(L, count, x_dev, scores_dev, (hipStream_t)stream),
            "labs_general_flip_scores_dev");
    return LABS_OK;
}

extern "C" int labs_general_walk_batch(int32_t n_walks, const labs_walk_cfg *cfg, labs_walk_result *out,
                                       int32_t *trace, int32_t *scores, double *kernel_ms, void *stream)
{
    if (n_walks < 1 || !cfg || !out)
        return fail(LABS_EINVAL, "labs_general_walk_batch: n_walks = %d with cfg and out required", n_walks);
    for (int32_t i = 0; i < n_walks; i++) {
        const labs_walk_cfg &c = cfg[i];
        if (c.L < 3 || c.L > LABS_GENERAL_L_MAX)
            return fail(LABS_EINVAL, "walk %d: L = %d must be in [3, %d]", i, c.L, LABS_GENERAL_L_MAX);
        labs_walk_cfg odd = c;
        odd.L = 3; // the remaining checks do not depend on L
        int rc = walk_cfg_check(odd, i);
        if (rc)
            return rc;
        if (c.steps > ((int64_t)1 << 30))
            return fail(LABS_EINVAL, "labs_general_walk_batch: walk %d: steps must be at most 2^30", i);
    }
    return batch_sync(kBatchGeneral, n_walks, cfg, 0, 0, out, trace, scores, kernel_ms, stream);
}

// =============================================================================================
// Option resolution and the autotuner.
// =============================================================================================
namespace liblabs {

static std::mutex g_tune_mu;

static std::string cache_path()
{
    const char *env = getenv("LABS_AUTOTUNE_CACHE");
    if (env && *env)
        return env;
    const char *home = getenv("HOME");
    return std::string(home ? home : "/tmp") + "/.cache/liblabs_autotune.txt";
}

// Cache key of a batch: "<L>" when every walk has length L, "M<minL>-<maxL>" for a batch of
// mixed lengths (they run the dispatching kernel, so a single-length entry does not describe
// them).
static std::string batch_key(int minL, int maxL)
{
    return minL == maxL ? std::to_string(maxL) : "M" + std::to_string(minL) + "-" + std::to_string(maxL);
}

// cache lines: "<arch> <key> <variant> <waves_per_block> <probe_width> <persistent>".  Later
// entries win.  A single-length batch takes the entry of its own L, else that of the nearest L
// tuned for the same kernel shape; a mixed batch takes only an entry of its own key.
static bool cache_lookup(int minL, int maxL, labs_plan_opts *o)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    std::ifstream f(cache_path());
    if (!f)
        return false;
    const std::string arch = device_arch();
    const bool mixed = minL != maxL;
    const std::string want = batch_key(minL, maxL);
    const int shape = shape_for_length(maxL);
    bool found = false;
    int best_dist = 1 << 30;
    std::string line;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string a, key;
        int v, wpb, pw, pers;
        if (!(is >> a >> key >> v >> wpb >> pw >> pers) || a != arch)
            continue;
        int dist = 0;
        if (mixed) {
            if (key != want)
                continue;
        } else {
            if (key.empty() || key[0] == 'M')
                continue;
            const int l = atoi(key.c_str());
            if (l < 3 || l > LABS_WALK_L_MAX || (l % 2) == 0 || shape_for_length(l) != shape)
                continue;
            dist = l > maxL ? l - maxL : maxL - l;
        }
        if (dist <= best_dist) {
            best_dist = dist;
            o->variant = v;
            o->waves_per_block = wpb;
            o->probe_width = pw;
            o->persistent = pers;
            found = true;
        }
    }
    return found;
}

static void cache_store(const std::string &key, const labs_plan_opts &o)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const std::string path = cache_path();
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos) {
        const std::string dir = path.substr(0, slash);
        (void)mkdir(dir.c_str(), 0755); // best effort: the last component only
    }
    std::ofstream f(path, std::ios::app);
    if (!f)
        return;
    f << device_arch() << " " << key << " " << o.variant << " " << o.waves_per_block << " " << o.probe_width << " "
      << o.persistent << "\n";
}

static int resolve_opts(labs_walk_plan *p, const labs_plan_opts *in)
{
    labs_plan_opts o{};
    if (in)
        o = *in;
    int32_t persistent = 0;
    // shapes present
    int shape = -2;
    int maxL = 0, minL = 1 << 30;
    for (const labs_walk_cfg &c : p->cfg) {
        const int s = shape_for_length(c.L);
        shape = (shape == -2 || shape == s) ? s : -1;
        maxL = std::max(maxL, c.L);
        minL = std::min(minL, c.L);
    }
    labs_plan_opts tuned{};
    const bool have = cache_lookup(minL, maxL, &tuned);
    // untuned default: the matrix-core scoring (measured faster than the bit-sliced one at every
    // length it covers, L <= 383), the bit-sliced one beyond
    if (o.variant == LABS_VARIANT_AUTO)
        o.variant = have ? tuned.variant
                         : ((minL >= kMfmaAutoLMin && maxL <= kMfmaLMax) ? LABS_VARIANT_MFMA : LABS_VARIANT_BITSLICE);
    if (o.variant != LABS_VARIANT_BITSLICE && o.variant != LABS_VARIANT_DIRECT && o.variant != LABS_VARIANT_MFMA)
        return fail(LABS_EINVAL, "unknown variant %d", o.variant);
    if (o.variant == LABS_VARIANT_MFMA && maxL > kMfmaLMax)
        return fail(LABS_EINVAL, "the matrix-core variant needs L <= %d (longest walk: %d)", kMfmaLMax, maxL);
    if (o.waves_per_block == 0)
        o.waves_per_block = have ? tuned.waves_per_block : 1;
    if (o.waves_per_block != 1 && o.waves_per_block != 2 && o.waves_per_block != 4 && o.waves_per_block != 8)
        return fail(LABS_EINVAL, "waves_per_block = %d must be 0, 1, 2, 4 or 8", o.waves_per_block);
    if (o.probe_width == 0) // measured: two probes in flight pay off for the matrix-core walker only
        o.probe_width = have ? tuned.probe_width : (o.variant == LABS_VARIANT_MFMA ? 2 : 1);
    if (o.probe_width < 1 || o.probe_width > 4)
        return fail(LABS_EINVAL, "probe_width = %d must be in [0, 4]", o.probe_width);
    if (o.probe_width > 2)
        o.probe_width = 2; // the kernels are built for one or two probes in flight
    if (o.steps_per_launch < 0)
        return fail(LABS_EINVAL, "steps_per_launch < 0");
    if (o.steps_per_launch == 0)
        o.steps_per_launch = std::max<int64_t>(p->max_steps, 1);
    o.steps_per_launch = std::min<int64_t>(o.steps_per_launch, (int64_t)1 << 30); // kernel limit
    // one wave per walk, the hardware dispatching workgroups as others finish (walks in the
    // costliest-first order), measured 1-3 % faster than resident waves pulling walks from a
    // counter for the matrix-core walker, at the L = 255 headline and on the uneven batch
    if (o.persistent == 0)
        o.persistent = have ? tuned.persistent : 1;
    if (o.persistent != 1 && o.persistent != 2)
        return fail(LABS_EINVAL, "persistent = %d must be 0, 1 or 2", o.persistent);
    persistent = o.persistent == 2;
    p->opts = o;
    p->lp.variant = o.variant;
    p->lp.waves_per_block = o.waves_per_block;
    p->lp.probe_width = o.probe_width;
    p->lp.shape = shape;
    p->lp.chunk = o.steps_per_launch;
    p->lp.persistent = persistent;
    int cus = 256;
    {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
            cus = prop.multiProcessorCount;
    }
    const int resident = resident_walk_waves(p->lp);
    p->lp.grid_waves = std::min<int32_t>(p->n_walks, resident > 0 ? resident : cus * 8);
    const int64_t per = o.steps_per_launch;
    p->launches_per_run = (int32_t)std::max<int64_t>(1, (p->max_steps + per - 1) / per);
    return LABS_OK;
}

} // namespace liblabs

namespace liblabs {

// Times every candidate launch form on the batch cfg (short synthetic runs: results never depend
// on the form) and stores the fastest under key.
static int tune_batch(const std::vector<labs_walk_cfg> &cfg, int maxL, const std::string &key,
                      labs_plan_opts *best)
{
    const int32_t n_walks = (int32_t)cfg.size();
    struct Cand { labs_plan_opts o; };
    std::vector<Cand> cands;
    for (int v : {LABS_VARIANT_BITSLICE, LABS_VARIANT_DIRECT, LABS_VARIANT_MFMA})
        for (int wpb : {1, 2, 4})
            for (int pw : {1, 2})
                for (int pers : {1, 2}) {
                    if (v == LABS_VARIANT_MFMA && maxL > kMfmaLMax)
                        continue;
                    Cand c{};
                    c.o.variant = v;
                    c.o.waves_per_block = wpb;
                    c.o.probe_width = pw;
                    c.o.persistent = pers;
                    cands.push_back(c);
                }
    double best_ms = 1e30;
    Cand winner = cands[0];
    for (const Cand &c : cands) {
        labs_walk_plan *p = nullptr;
        int rc = labs_walk_plan_create(n_walks, cfg.data(), &c.o, &p);
        if (rc)
            return rc;
        double total = 0.0;
        for (int rep = 0; rep < 3; rep++) {
            rc = labs_walk_plan_run(p, nullptr);
            double ms = 0.0;
            if (!rc)
                rc = labs_walk_plan_last_timing(p, &ms, nullptr);
            if (rc) {
                labs_walk_plan_destroy(p);
                return rc;
            }
            if (rep > 0)
                total += ms;
        }
        labs_walk_plan_destroy(p);
        if (total < best_ms) {
            best_ms = total;
            winner = c;
        }
    }
    cache_store(key, winner.o);
    if (best)
        *best = winner.o;
    return LABS_OK;
}

} // namespace liblabs

extern "C" int labs_autotune(int32_t L, int32_t n_walks, labs_plan_opts *best)
{
    if (L < 3 || L > LABS_WALK_L_MAX || (L % 2) == 0 || n_walks < 1)
        return fail(LABS_EINVAL, "labs_autotune: L = %d, n_walks = %d", L, n_walks);
    int rc = check_device();
    if (rc)
        return rc;
    std::vector<labs_walk_cfg> cfg((size_t)n_walks);
    for (int32_t i = 0; i < n_walks; i++) {
        labs_walk_cfg &c = cfg[(size_t)i];
        memset(&c, 0, sizeof c);
        c.L = L;
        c.table_log2 = 16;
        c.seed = 0x7E57ull;
        c.walk_id = (uint32_t)i;
        c.steps = 512;
        c.target_isl = -1;
        c.watch_isl = -1;
    }
    return tune_batch(cfg, L, batch_key(L, L), best);
}

extern "C" int labs_autotune_batch(int32_t n_walks, const labs_walk_cfg *cfg, labs_plan_opts *best)
{
    if (n_walks < 1 || !cfg)
        return fail(LABS_EINVAL, "labs_autotune_batch: n_walks = %d with a cfg array required", n_walks);
    int minL = 1 << 30, maxL = 0;
    std::vector<labs_walk_cfg> tune((size_t)n_walks);
    for (int32_t i = 0; i < n_walks; i++) {
        int rc = walk_cfg_check(cfg[i], i);
        if (rc)
            return rc;
        minL = std::min(minL, cfg[i].L);
        maxL = std::max(maxL, cfg[i].L);
        // the batch's walks, shortened to a sample of at most 512 steps, without traces or stops
        labs_walk_cfg c = cfg[i];
        c.flags = 0;
        c.steps = std::min<int64_t>(c.steps, 512);
        c.target_isl = -1;
        c.watch_isl = -1;
        tune[(size_t)i] = c;
    }
    int rc = check_device();
    if (rc)
        return rc;
    return tune_batch(tune, maxL, batch_key(minL, maxL), best);
}
