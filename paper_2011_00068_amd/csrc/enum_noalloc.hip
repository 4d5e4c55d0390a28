// enum_noalloc.hip -- labs_enum_skew_min_noalloc: the grouped skew-space minimum of
// labs_enum_skew_min (Eq. (2), (4)) without any device allocation, for callers that cannot
// allocate (code under HIP graph capture, serving loops, harnesses that forbid hipMalloc).
//
// The per-block partial results, which the allocating entry point keeps in a buffer it allocates
// per call, live here in a file-scope device array, `scratch`, that every GPU the library runs on
// holds until the process ends.  Host code never passes the array's name to a kernel (on the host
// it is only a stand-in for the symbol): the first call on a device looks up the array's device
// address with hipGetSymbolAddress, with that device current, and keeps it per device; the kernels
// receive that address.  Every call re-initialises the slots it uses by a kernel before the
// enumeration, so nothing carries over from an earlier call; calls that overlap on one GPU (other
// threads, other streams) share the array and race.
#include <algorithm>
#include <cstring>
#include <mutex>

#include "internal.hpp"

namespace liblabs {
int fail(int code, const char *fmt, ...);
int hip_fail(hipError_t e, const char *what);
int check_device();
} // namespace liblabs

using namespace liblabs;

namespace {

// One slot per resident block of the enumeration kernel plus the final slot: 4096 x 32 bytes =
// 128 KiB per device.  A device with more resident blocks runs a smaller grid (the results do not
// depend on the grid).
constexpr int kScratchSlots = 4096;
static_assert(sizeof(EnumPartial) == 32, "slot size");

} // namespace

static __device__ __align__(256) EnumPartial scratch[kScratchSlots];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
EnumPartial *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
int scratch_on_current_device(EnumPartial **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return hip_fail(e, "labs_enum_skew_min_noalloc: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices)
        return fail(LABS_EDEVICE, "labs_enum_skew_min_noalloc: device %d beyond the %d supported", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                            "labs_enum_skew_min_noalloc: hipGetSymbolAddress(scratch)");
        g_scratch_ptr[dev] = static_cast<EnumPartial *>(p);
    }
    *out = g_scratch_ptr[dev];
    return LABS_OK;
}

} // namespace

extern "C" int labs_enum_skew_min_noalloc(int32_t L, uint64_t r_begin, uint64_t r_end, labs_enum_min_result *out,
                                          void *stream)
{
    if (!out)
        return fail(LABS_EINVAL, "labs_enum_skew_min_noalloc: NULL result");
    if (L < 3 || L > 125 || (L % 2) == 0)
        return fail(LABS_EINVAL, "labs_enum_skew_min_noalloc: L = %d must be odd in [3, 125]", L);
    const int n = (L + 1) / 2;
    const uint64_t groups = 1ull << (n - 2);
    if (r_begin > r_end || r_end > groups)
        return fail(LABS_EINVAL, "labs_enum_skew_min_noalloc: block [%llu, %llu) outside [0, 2^%d)",
                    (unsigned long long)r_begin, (unsigned long long)r_end, n - 2);
    memset(out, 0, sizeof *out);
    out->min_isl = -1;
    out->kernel_ms = -1.0; // not timed: timing would create events
    if (r_begin == r_end)
        return LABS_OK;
    int rc = check_device();
    if (rc)
        return rc;
    EnumPartial *part = nullptr;
    rc = scratch_on_current_device(&part);
    if (rc)
        return rc;
    const int blocks = std::min(enum_min_blocks(L), kScratchSlots - 1);
    if (blocks <= 0)
        return fail(LABS_EDEVICE, "labs_enum_skew_min_noalloc: occupancy query failed");
    hipStream_t s = (hipStream_t)stream;
    // the launch split of labs_enum_skew_min: at most 2^32 groups and 2^20 passes per lane
    const uint64_t cap = std::min<uint64_t>(1ull << 32, (uint64_t)blocks * 256ull * 4ull * (1ull << 20));
    EnumPartial res{};
    hipError_t e = launch_enum_part_init(part, blocks, s);
    for (uint64_t r = r_begin; e == hipSuccess && r < r_end;) {
        const uint64_t cnt = std::min<uint64_t>(r_end - r, cap);
        e = launch_enum_min(L, r, cnt, part, blocks, s);
        r += cnt;
    }
    if (e == hipSuccess) e = launch_enum_final(part, blocks, part + blocks, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&res, part + blocks, sizeof res, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(e, "labs_enum_skew_min_noalloc");
    out->min_isl = res.min_isl == 0xFFFFFFFFu ? -1 : (int32_t)res.min_isl;
    out->count = res.count;
    out->first_x = res.min_isl == 0xFFFFFFFFu ? 0 : res.first_x;
    out->states = 4 * (r_end - r_begin);
    out->word_ops = res.word_ops;
    return LABS_OK;
}
