// api.hip -- the extern "C" boundary declared in include/rsi.h: argument
// validation, handle lifetime, device memory, and the launch sequence.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <new>
#include <string>

#include "../../include/rsi.h"
#include "rsi_host.h"

namespace rsi {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

}  // namespace rsi

using rsi::set_error;

namespace {

rsi_status hip_fail(hipError_t e, const char *what)
{
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? RSI_E_NOMEM : RSI_E_HIP;
}

rsi_status invalid(const char *msg)
{
    set_error(msg);
    return RSI_E_INVALID;
}

template <class T>
hipError_t dalloc(T **p, int64_t n)
{
    *p = nullptr;
    if (n <= 0) n = 1;
    return hipMalloc(reinterpret_cast<void **>(p), sizeof(T) * (size_t)n);
}

void free_handle_memory(rsi_bvh *h)
{
    void *ptrs[] = {h->T, h->cent, h->keys, h->order, h->nodes, h->tris, h->arrive, h->heights, h->climb,
                    h->scalars, h->counters, h->ovf_seg, h->ovf_cnt, h->ovf_off, h->pool_ids, h->pool_ts};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    rsi::free_sort_scratch(h->sort);
    if (h->h_scalars) (void)hipHostFree(h->h_scalars);
}

// Copy the indices, run the build kernels, then wait once to read back the
// index check and the tree height (which sizes the traversal stack).
rsi_status build_into(rsi_bvh *h, const float *V, int64_t n_v, const int32_t *T, hipStream_t s)
{
    const int64_t n = h->n_t;
    h->n_v = n_v;
    hipError_t e = hipSuccess;
    if (n > 0) e = hipMemcpyAsync(h->T, T, sizeof(int32_t) * 3 * n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = rsi::launch_build(h, V, s);
    if (e == hipSuccess && n > 0)
        e = hipMemcpyAsync(h->h_scalars, h->scalars, sizeof(int32_t) * rsi::kNumScalars, hipMemcpyDeviceToHost,
                           s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "rsi_build");
    if (n > 0) {
        if (h->h_scalars[rsi::kBadIndex]) return invalid("rsi_build: triangle index outside [0, n_v)");
        h->height = h->h_scalars[rsi::kHeight];
        h->root_ref = h->h_scalars[rsi::kRootRef];
    }
    return RSI_OK;
}

}  // namespace

extern "C" {

const char *rsi_status_str(rsi_status s)
{
    switch (s) {
    case RSI_OK: return "ok";
    case RSI_E_INVALID: return "invalid argument";
    case RSI_E_NOMEM: return "out of device memory";
    case RSI_E_HIP: return "HIP runtime error";
    case RSI_E_OVERFLOW: return "buffer overflow";
    }
    return "unknown status";
}

const char *rsi_last_error(void) { return rsi::g_last_error.c_str(); }

rsi_status rsi_build(const float *V, int64_t n_v, const int32_t *T, int64_t n_t, const rsi_opts *opts,
                     void *stream, rsi_handle *out)
{
    set_error("");
    if (!out) return invalid("rsi_build: out is NULL");
    *out = nullptr;
    if (n_v < 0 || n_t < 0) return invalid("rsi_build: negative size");
    if (n_t >= (int64_t(1) << rsi::kLeafFirstBits)) return invalid("rsi_build: n_t must be below 2^27");
    if (n_t > 0 && n_v == 0) return invalid("rsi_build: triangles given without vertices");
    if ((n_v > 0 && !V) || (n_t > 0 && !T)) return invalid("rsi_build: NULL pointer with nonzero size");
    int leaf = 1, block = 128, defer = 32, refill = 32, chunk = 0;
    if (opts) {
        if (opts->leaf_size) leaf = opts->leaf_size;
        if (opts->block_size) block = opts->block_size;
        if (opts->defer_lanes) defer = opts->defer_lanes;
        if (opts->refill_lanes) refill = opts->refill_lanes;
        if (opts->chunk) chunk = opts->chunk;
    }
    if (chunk != 0 && (chunk < 64 || chunk > (1 << 20))) return invalid("rsi_build: chunk must be 0 or 64..2^20");
    if (defer < 1 || defer > 64) return invalid("rsi_build: defer_lanes must be in 1..64");
    if (refill < 1 || refill > 64) return invalid("rsi_build: refill_lanes must be in 1..64");
    if (leaf < 1 || leaf > rsi::kMaxLeafSize) return invalid("rsi_build: leaf_size must be in 1..16");
    if (block < 64 || block > 256 || block % 64) return invalid("rsi_build: block_size must be 64, 128, 192 or 256");

    rsi_bvh *h = new (std::nothrow) rsi_bvh();
    if (!h) return invalid("rsi_build: host allocation failed");
    hipStream_t s = (hipStream_t)stream;
    h->n_v = n_v;
    h->n_t = n_t;
    h->leaf_size = leaf;
    h->block_size = block;
    h->defer_lanes = defer;
    h->refill_lanes = refill;
    h->chunk = chunk;
    h->entry = n_t > 0 ? (int32_t)(n_t - 1) : 0;
    hipError_t e = hipGetDevice(&h->device);
    const int64_t n = n_t;
    if (e == hipSuccess) e = dalloc(&h->T, 3 * n);
    if (e == hipSuccess) e = dalloc(&h->cent, 3 * n);
    if (e == hipSuccess) e = dalloc(&h->keys, n);
    if (e == hipSuccess) e = dalloc(&h->order, n);
    if (e == hipSuccess) e = dalloc(&h->nodes, n);
    if (e == hipSuccess) e = dalloc(&h->tris, n);
    if (e == hipSuccess) e = dalloc(&h->arrive, n);
    if (e == hipSuccess) e = dalloc(&h->heights, 2 * n);
    if (e == hipSuccess) e = dalloc(&h->climb, 11 * n);
    if (e == hipSuccess) e = dalloc(&h->scalars, rsi::kNumScalars);
    if (e == hipSuccess) e = dalloc(&h->counters, 1);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void **>(&h->h_scalars), sizeof(int32_t) * rsi::kNumScalars);
    if (e == hipSuccess && n > 0) e = rsi::ensure_sort_scratch(h->sort, n);
    if (e != hipSuccess) {
        rsi_status st = hip_fail(e, "rsi_build");
        free_handle_memory(h);
        delete h;
        return st;
    }
    rsi_status st = build_into(h, V, n_v, T, s);
    if (st != RSI_OK) {
        free_handle_memory(h);
        delete h;
        return st;
    }
    *out = h;
    return RSI_OK;
}

rsi_status rsi_rebuild(rsi_handle h, const float *V, int64_t n_v, const int32_t *T, void *stream)
{
    set_error("");
    if (!h) return invalid("rsi_rebuild: NULL handle");
    if (n_v < 0) return invalid("rsi_rebuild: negative n_v");
    if (h->n_t > 0 && n_v == 0) return invalid("rsi_rebuild: triangles given without vertices");
    if (h->n_t > 0 && (!V || !T)) return invalid("rsi_rebuild: NULL pointer with nonzero size");
    return build_into(h, V, n_v, T, (hipStream_t)stream);
}

rsi_status rsi_refit(rsi_handle h, const float *V, void *stream)
{
    set_error("");
    if (!h) return invalid("rsi_refit: NULL handle");
    if (h->n_t > 0 && !V) return invalid("rsi_refit: NULL vertices");
    hipError_t e = rsi::launch_refit(h, V, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "rsi_refit");
    return RSI_OK;
}

static hipError_t ensure_ovf(rsi_bvh *h, int64_t n_r)
{
    if (h->ovf_cap >= n_r) return hipSuccess;
    if (h->ovf_seg) (void)hipFree(h->ovf_seg);
    if (h->ovf_cnt) (void)hipFree(h->ovf_cnt);
    if (h->ovf_off) (void)hipFree(h->ovf_off);
    h->ovf_seg = nullptr;
    h->ovf_cnt = nullptr;
    h->ovf_off = nullptr;
    h->ovf_cap = 0;
    hipError_t e = dalloc(&h->ovf_seg, n_r);
    if (e == hipSuccess) e = dalloc(&h->ovf_cnt, n_r);
    if (e == hipSuccess) e = dalloc(&h->ovf_off, n_r);
    if (e == hipSuccess) h->ovf_cap = n_r;
    return e;
}

static hipError_t ensure_pool(rsi_bvh *h, int64_t n)
{
    if (h->pool_cap >= n) return hipSuccess;
    if (h->pool_ids) (void)hipFree(h->pool_ids);
    if (h->pool_ts) (void)hipFree(h->pool_ts);
    h->pool_ids = nullptr;
    h->pool_ts = nullptr;
    h->pool_cap = 0;
    const int64_t want = n + n / 4;
    hipError_t e = dalloc(&h->pool_ids, want);
    if (e == hipSuccess) e = dalloc(&h->pool_ts, want);
    if (e == hipSuccess) h->pool_cap = want;
    return e;
}

rsi_status rsi_query(rsi_handle h, const float *S, const float *E, int64_t n_r, uint32_t mode,
                     const rsi_outputs *out, void *stream)
{
    set_error("");
    if (!h) return invalid("rsi_query: NULL handle");
    if (!out) return invalid("rsi_query: NULL outputs");
    if (n_r < 0) return invalid("rsi_query: negative n_r");
    if (mode == 0 || (mode & ~(uint32_t)(RSI_BOOL | RSI_FIRST_HIT | RSI_ALL_HITS)))
        return invalid("rsi_query: mode must be a nonzero mask of RSI_BOOL, RSI_FIRST_HIT, RSI_ALL_HITS");
    if (n_r == 0) return RSI_OK;  // nothing to read or write; output pointers may be NULL
    if (!S || !E) return invalid("rsi_query: NULL segment pointer");
    if ((mode & RSI_BOOL) && !out->hit) return invalid("rsi_query: RSI_BOOL needs out->hit");
    if ((mode & RSI_FIRST_HIT) && (!out->tri || !out->t || !out->uv || !out->point))
        return invalid("rsi_query: RSI_FIRST_HIT needs out->tri, t, uv, point");
    if (mode & RSI_ALL_HITS) {
        if (!out->count || !out->ids || !out->ts) return invalid("rsi_query: RSI_ALL_HITS needs out->count, ids, ts");
        if (out->capacity < 1) return invalid("rsi_query: capacity must be >= 1");
    }
    if (n_r >= (int64_t(1) << 30)) return invalid("rsi_query: n_r must be below 2^30");
    hipStream_t s = (hipStream_t)stream;
    rsi::QueryOut o = {out->hit, out->tri, out->t, out->uv, out->point, out->count, out->ids, out->ts,
                       out->capacity};
    h->last_ovf_segs = 0;
    h->last_ovf_total = 0;
    hipError_t e;
    if (h->n_t == 0) {
        e = rsi::launch_fill_miss(n_r, mode, o, s);
        return e == hipSuccess ? RSI_OK : hip_fail(e, "rsi_query");
    }
    if (mode & RSI_ALL_HITS) {
        e = ensure_ovf(h, n_r);
        if (e != hipSuccess) return hip_fail(e, "rsi_query: overflow list");
    }
    e = rsi::launch_query(h, S, E, n_r, mode, o, s);
    if (e != hipSuccess) return hip_fail(e, "rsi_query");
    if (mode & RSI_ALL_HITS) {
        // size the spill pool: one read-back of the overflow totals
        e = hipMemcpyAsync(h->h_scalars + rsi::kOvfSegs, h->scalars + rsi::kOvfSegs, 3 * sizeof(int32_t),
                           hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "rsi_query: overflow read-back");
        const int64_t nseg = h->h_scalars[rsi::kOvfSegs];
        uint64_t tot = (uint32_t)h->h_scalars[rsi::kOvfTotalLo] | ((uint64_t)(uint32_t)h->h_scalars[rsi::kOvfTotalHi] << 32);
        h->last_ovf_segs = nseg;
        h->last_ovf_total = (int64_t)tot;
        if (nseg > 0) {
            e = ensure_pool(h, (int64_t)tot);
            if (e != hipSuccess) return hip_fail(e, "rsi_query: spill pool");
            e = rsi::launch_spill(h, S, E, mode, o, s);
            if (e != hipSuccess) return hip_fail(e, "rsi_query: spill pass");
        }
    }
    return RSI_OK;
}

rsi_status rsi_first_hit_backward(rsi_handle h, const float *V, const float *S, const float *E, int64_t n_r,
                                  const int32_t *tri, const float *g_t, const float *g_uv, const float *g_point,
                                  float *dV, float *dS, float *dE, void *stream)
{
    set_error("");
    if (!h) return invalid("rsi_first_hit_backward: NULL handle");
    if (n_r < 0 || n_r >= (int64_t(1) << 30)) return invalid("rsi_first_hit_backward: n_r must be in [0, 2^30)");
    if (n_r == 0) return RSI_OK;
    if (!S || !E || !tri) return invalid("rsi_first_hit_backward: NULL S, E or tri");
    if (h->n_t > 0 && (!V || !dV)) return invalid("rsi_first_hit_backward: NULL V or dV");
    hipError_t e = rsi::launch_first_hit_adjoint(h, V, S, E, n_r, tri, g_t, g_uv, g_point, dV, dS, dE,
                                                 (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "rsi_first_hit_backward");
    return RSI_OK;
}

rsi_status rsi_spill_info(rsi_handle h, int64_t *n_segments, int64_t *n_crossings)
{
    set_error("");
    if (!h || !n_segments || !n_crossings) return invalid("rsi_spill_info: NULL argument");
    *n_segments = h->last_ovf_segs;
    *n_crossings = h->last_ovf_total;
    return RSI_OK;
}

rsi_status rsi_spill_read(rsi_handle h, int32_t *seg, int64_t *offset, int32_t *count, int32_t *ids, float *ts,
                          void *stream)
{
    set_error("");
    if (!h) return invalid("rsi_spill_read: NULL handle");
    const int64_t n = h->last_ovf_segs, m = h->last_ovf_total;
    if (n == 0) return RSI_OK;
    if (!seg || !offset || !count || !ids || !ts) return invalid("rsi_spill_read: NULL buffer");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(seg, h->ovf_seg, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(offset, h->ovf_off, sizeof(int64_t) * n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(count, h->ovf_cnt, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(ids, h->pool_ids, sizeof(int32_t) * m, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(ts, h->pool_ts, sizeof(float) * m, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "rsi_spill_read");
    return RSI_OK;
}

rsi_status rsi_set_counting(rsi_handle h, int enable)
{
    set_error("");
    if (!h) return invalid("rsi_set_counting: NULL handle");
    h->counting = enable != 0;
    return RSI_OK;
}

rsi_status rsi_get_counters(rsi_handle h, rsi_counters *out)
{
    set_error("");
    if (!h || !out) return invalid("rsi_get_counters: NULL argument");
    rsi::Counters c;
    hipError_t e = hipMemcpy(&c, h->counters, sizeof(c), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "rsi_get_counters");
    out->node_visits = c.node_visits;
    out->box_tests = c.box_tests;
    out->tri_tests = c.tri_tests;
    out->segments = c.segments;
    return RSI_OK;
}

rsi_status rsi_get_tree_info(rsi_handle h, rsi_tree_info *out)
{
    set_error("");
    if (!h || !out) return invalid("rsi_get_tree_info: NULL argument");
    memset(out, 0, sizeof(*out));
    out->n_t = h->n_t;
    out->n_nodes = h->n_t;
    out->height = h->height;
    out->leaf_size = h->leaf_size;
    out->entry = h->entry;
    return RSI_OK;
}

rsi_status rsi_export_tree(rsi_handle h, float *boxes, int32_t *refs, int32_t *order, uint64_t *keys)
{
    set_error("");
    if (!h) return invalid("rsi_export_tree: NULL handle");
    const int64_t n = h->n_t;
    if (n == 0) return RSI_OK;
    hipError_t e = hipDeviceSynchronize();
    rsi::Node *tmp = nullptr;
    if (e == hipSuccess && (boxes || refs)) {
        tmp = new (std::nothrow) rsi::Node[(size_t)n];
        if (!tmp) return invalid("rsi_export_tree: host allocation failed");
        e = hipMemcpy(tmp, h->nodes, sizeof(rsi::Node) * (size_t)n, hipMemcpyDeviceToHost);
        if (e == hipSuccess) {
            for (int64_t k = 0; k < n; ++k) {
                if (boxes) memcpy(boxes + 12 * k, tmp[k].f, 12 * sizeof(float));
                if (refs) {
                    refs[2 * k] = tmp[k].ref[0];
                    refs[2 * k + 1] = tmp[k].ref[1];
                }
            }
        }
        delete[] tmp;
    }
    if (e == hipSuccess && order) e = hipMemcpy(order, h->order, sizeof(int32_t) * n, hipMemcpyDeviceToHost);
    if (e == hipSuccess && keys) e = hipMemcpy(keys, h->keys, sizeof(uint64_t) * n, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "rsi_export_tree");
    return RSI_OK;
}

void rsi_destroy(rsi_handle h)
{
    if (!h) return;
    (void)hipDeviceSynchronize();
    free_handle_memory(h);
    delete h;
}

}  // extern "C"
