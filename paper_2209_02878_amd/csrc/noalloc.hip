// noalloc.hip -- rsi_query_noalloc: the segment query of rsi_query for
// callers that cannot allocate device memory (code under HIP graph capture,
// serving loops, harnesses that forbid hipMalloc).
//
// rsi_query keeps two scratch buffers with the handle, allocated on first use
// and grown with the number of segments: the deep pass's queue (one int32 per
// segment whose stack outgrew its LDS part) and its device-memory stack (one
// column per thread of the deep pass's fixed grid).  Here both live in one
// file-scope device array of fixed size instead, and a query with more
// segments than the array's queue part can hold runs as consecutive parts on
// the same stream, each a complete query of a contiguous range of segments.
//
// The array's device address is obtained once per device with
// hipGetSymbolAddress and kept; host code never passes the array's own name
// to a kernel (on the host that name is not a device address).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>

#include "../../include/rsi.h"
#include "rsi_host.h"

namespace {

// 32 MiB of int32 entries, held by every GPU the library runs on until the
// process ends.
constexpr int64_t kScratchInts = int64_t(8) << 20;
static __device__ __align__(256) int32_t scratch[kScratchInts];

constexpr int kMaxDevices = 64;
int32_t *g_scratch[kMaxDevices] = {};
std::mutex g_scratch_mu;

// Device address of `scratch` on device `dev` (the current device).
hipError_t scratch_address(int dev, int32_t **out)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch[dev] = static_cast<int32_t *>(p);
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

rsi_status fail(rsi_status st, const std::string &msg)
{
    rsi::set_error(msg);
    return st;
}

}  // namespace

rsi_status rsi_query_noalloc(rsi_handle h, const float *S, const float *E, int64_t n_r, uint32_t mode,
                             const rsi_outputs *out, void *stream)
{
    rsi::set_error("");
    if (!h) return fail(RSI_E_INVALID, "rsi_query_noalloc: NULL handle");
    if (h->M != 1) return fail(RSI_E_INVALID, "rsi_query_noalloc: batch handle");
    if (!out) return fail(RSI_E_INVALID, "rsi_query_noalloc: NULL outputs");
    if (n_r < 0 || n_r >= (int64_t(1) << 30)) return fail(RSI_E_INVALID, "rsi_query_noalloc: n_r must be in [0, 2^30)");
    if (mode == 0 || (mode & ~(uint32_t)(RSI_BOOL | RSI_FIRST_HIT | RSI_COUNT)))
        return fail(RSI_E_INVALID,
                    "rsi_query_noalloc: mode must be a nonzero mask of RSI_BOOL, RSI_FIRST_HIT, RSI_COUNT "
                    "(RSI_ALL_HITS needs memory that grows with the crossings: use rsi_query)");
    if (n_r == 0) return RSI_OK;
    if (!S || !E) return fail(RSI_E_INVALID, "rsi_query_noalloc: NULL segment pointer");
    if ((mode & RSI_BOOL) && !out->hit) return fail(RSI_E_INVALID, "rsi_query_noalloc: RSI_BOOL needs out->hit");
    if ((mode & RSI_FIRST_HIT) && (!out->tri || !out->t || !out->uv || !out->point))
        return fail(RSI_E_INVALID, "rsi_query_noalloc: RSI_FIRST_HIT needs out->tri, t, uv, point");
    if ((mode & RSI_COUNT) && !out->count) return fail(RSI_E_INVALID, "rsi_query_noalloc: RSI_COUNT needs out->count");

    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(RSI_E_HIP, std::string("rsi_query_noalloc: hipGetDevice: ") + hipGetErrorString(e));
    if (dev != h->device)
        return fail(RSI_E_INVALID, "rsi_query_noalloc: the current device is not the handle's device");
    if (dev < 0 || dev >= kMaxDevices) return fail(RSI_E_INVALID, "rsi_query_noalloc: device index above 63");
    int32_t *base = nullptr;
    e = scratch_address(dev, &base);
    if (e != hipSuccess)
        return fail(RSI_E_HIP, std::string("rsi_query_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));

    hipStream_t s = (hipStream_t)stream;
    h->last_stream = s;
    const rsi::QueryOut o = {out->hit, out->tri, out->t, out->uv, out->point, out->count, nullptr, nullptr, 1,
                             nullptr, nullptr, nullptr, 0};
    if (h->n_t == 0) {
        e = rsi::launch_fill_miss(n_r, mode, o, s);
        if (e == hipSuccess) e = rsi::launch_clear_query(h, s);
        return e == hipSuccess ? RSI_OK
                               : fail(RSI_E_HIP, std::string("rsi_query_noalloc: ") + hipGetErrorString(e));
    }

    // the deep pass's stack takes the front of the array (64-entry aligned),
    // the queue the rest; the queue sets how many segments one part holds
    const int64_t stack_ints = (rsi::deep_stack_entries(h, mode) + 63) / 64 * 64;
    const int64_t part = kScratchInts - stack_ints;
    if (part < 4096)
        return fail(RSI_E_INVALID,
                    "rsi_query_noalloc: the deep pass's stack for these options (" + std::to_string(stack_ints) +
                        " entries) leaves no room in the 32 MiB scratch array; use a smaller block_size or "
                        "rsi_query");
    const rsi::QueryScratch sc = {base + stack_ints, part, stack_ints > 0 ? base : nullptr, stack_ints};
    for (int64_t off = 0; off < n_r; off += part) {
        const int64_t n = n_r - off < part ? n_r - off : part;
        rsi::QueryOut p = o;
        if (p.hit) p.hit += off;
        if (p.tri) p.tri += off;
        if (p.t) p.t += off;
        if (p.uv) p.uv += 2 * off;
        if (p.point) p.point += 3 * off;
        if (p.count) p.count += off;
        e = rsi::launch_query_scratch(h, S + 3 * off, E + 3 * off, n, mode, p, sc, off > 0, s);
        if (e != hipSuccess) return fail(RSI_E_HIP, std::string("rsi_query_noalloc: ") + hipGetErrorString(e));
    }
    return RSI_OK;
}
