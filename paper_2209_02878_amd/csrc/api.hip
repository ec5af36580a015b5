// api.hip -- the extern "C" boundary declared in include/rsi.h: argument
// validation, handle lifetime, device memory, and the launch sequences.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

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
    if (h->graph) (void)hipGraphExecDestroy(h->graph);
    if (h->capture_stream) (void)hipStreamDestroy(h->capture_stream);
    void *ptrs[] = {h->rank, h->adj_vals, h->seg_keys, h->adj_rec, h->adj_rec_v, h->tri_sum, h->adj_part, h->adj_cell_first, h->inc_first, h->inc_keys,
                    h->inc_vals, h->compact_counts, h->nodes4, h->aux_E, h->aux_count,
                    h->retry_q, h->retry_stack, h->arena, h->T, h->V_all, h->src_V, h->src_T, h->cent, h->keys,
                    h->order, h->nodes, h->tris, h->arrive, h->heights, h->climb, h->split_prefix, h->scalars,
                    h->counters, h->ovf_seg, h->ovf_cnt, h->ovf_list, h->ovf_off, h->ovf_part, h->pool_ids, h->pool_ts, h->tri_off,
                    h->vert_off, h->mesh_bounds, h->mesh_height, h->mesh_root, h->mesh_entry};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    rsi::BatchTables *tabs[] = {&h->bt, &h->bt_graph};
    for (rsi::BatchTables *t : tabs) {
        void *tp[] = {t->seg_off, t->S, t->E, t->hit, t->tri, t->t, t->uv, t->point, t->count, t->ids, t->ts,
                      t->spill_off};
        for (void *p : tp)
            if (p) (void)hipFree(p);
    }
    rsi::free_sort_scratch(h->sort);
    rsi::free_sort_scratch(h->seg_sort);
    if (h->h_scalars) (void)hipHostFree(h->h_scalars);
}

void destroy_handle(rsi_bvh *h)
{
    free_handle_memory(h);
    delete h;
}

// Apply the nonzero fields of `opts` on top of the handle's current values.
rsi_status read_opts(const rsi_opts *opts, rsi_bvh *h)
{
    int leaf = h->leaf_size, block = h->block_size, defer = h->defer_lanes, refill = h->refill_lanes;
    int chunk = h->chunk, stack = h->stack_cap, width = h->width;
    if (opts) {
        if (opts->branching) width = opts->branching;
        if (opts->leaf_size) leaf = opts->leaf_size;
        if (opts->block_size) block = opts->block_size;
        if (opts->defer_lanes) defer = opts->defer_lanes;
        if (opts->refill_lanes) refill = opts->refill_lanes;
        if (opts->chunk) chunk = opts->chunk;
        if (opts->stack_depth) stack = opts->stack_depth;
    }
    if (stack < 0 || stack > 255) return invalid("stack_depth must be in 1..255");
    if (leaf < 1 || leaf > rsi::kMaxLeafSize) return invalid("leaf_size must be in 1..16");
    if (block < 64 || block > 256 || block % 64) return invalid("block_size must be 64, 128, 192 or 256");
    if (defer < 1 || defer > 64) return invalid("defer_lanes must be in 1..64");
    if (refill < 1 || refill > 64) return invalid("refill_lanes must be in 1..64");
    if (chunk != 0 && (chunk < 64 || chunk > (1 << 20))) return invalid("chunk must be 0 or 64..2^20");
    if (width != 2 && width != 4) return invalid("branching must be 2 or 4");
    h->leaf_size = leaf;
    h->block_size = block;
    h->defer_lanes = defer;
    h->refill_lanes = refill;
    h->chunk = chunk;
    h->stack_cap = stack;
    h->width = width;
    return RSI_OK;
}

hipError_t alloc_tables(rsi::BatchTables &t, int32_t M)
{
    hipError_t e = dalloc(&t.seg_off, M + 1);
    if (e == hipSuccess) e = dalloc(&t.S, M);
    if (e == hipSuccess) e = dalloc(&t.E, M);
    if (e == hipSuccess) e = dalloc(&t.hit, M);
    if (e == hipSuccess) e = dalloc(&t.tri, M);
    if (e == hipSuccess) e = dalloc(&t.t, M);
    if (e == hipSuccess) e = dalloc(&t.uv, M);
    if (e == hipSuccess) e = dalloc(&t.point, M);
    if (e == hipSuccess) e = dalloc(&t.count, M);
    if (e == hipSuccess) e = dalloc(&t.ids, M);
    if (e == hipSuccess) e = dalloc(&t.ts, M);
    if (e == hipSuccess) e = dalloc(&t.spill_off, M);
    return e;
}

// Allocate a handle for M meshes with the given vertex and triangle counts.
rsi_status alloc_handle(int32_t M, const int64_t *n_v, const int64_t *n_t, const rsi_opts *opts, bool batch,
                        rsi_bvh **out)
{
    rsi_bvh *h = new (std::nothrow) rsi_bvh();
    if (!h) return invalid("host allocation failed");
    rsi_status st = read_opts(opts, h);
    if (st != RSI_OK) {
        delete h;
        return st;
    }
    h->M = M;
    h->h_tri_off.assign(M + 1, 0);
    h->h_vert_off.assign(M + 1, 0);
    for (int32_t m = 0; m < M; ++m) {
        h->h_tri_off[m + 1] = h->h_tri_off[m] + n_t[m];
        h->h_vert_off[m + 1] = h->h_vert_off[m] + n_v[m];
    }
    h->n_t = h->h_tri_off[M];
    h->n_v = h->h_vert_off[M];
    // A radix-tree node's split has a longer common key prefix than its
    // parent's, and prefix lengths take at most 63 values for distinct
    // 63-bit keys plus 27 for equal keys split by a (27-bit) index, so no
    // path holds more than 90 internal nodes (nor more than n - 1).
    for (int32_t m = 0; m < M; ++m) {
        const int64_t hb = n_t[m] - 1 < 90 ? n_t[m] - 1 : 90;
        if (hb > h->height_bound) h->height_bound = (int32_t)hb;
    }
    if (h->n_t >= (int64_t(1) << rsi::kLeafFirstBits)) {
        delete h;
        return invalid("total triangle count must be below 2^27");
    }
    std::vector<int32_t> entry(M);
    for (int32_t m = 0; m < M; ++m) entry[m] = n_t[m] > 0 ? (int32_t)(h->h_tri_off[m + 1] - 1) : -1;

    const int64_t n = h->n_t;
    hipError_t e = hipGetDevice(&h->device);
    if (e == hipSuccess) e = dalloc(&h->T, 3 * n);
    if (e == hipSuccess && batch) e = dalloc(&h->V_all, 3 * h->n_v);
    if (e == hipSuccess && batch) e = dalloc(&h->src_V, M);
    if (e == hipSuccess && batch) e = dalloc(&h->src_T, M);
    if (e == hipSuccess) e = dalloc(&h->cent, 3 * n);
    if (e == hipSuccess) e = dalloc(&h->keys, n);
    if (e == hipSuccess) e = dalloc(&h->order, n);
    if (e == hipSuccess) e = dalloc(&h->rank, n);
    if (e == hipSuccess) e = dalloc(&h->nodes, n);
    if (e == hipSuccess && h->width == 4) e = dalloc(&h->nodes4, n);
    if (e == hipSuccess) e = dalloc(&h->tris, n);
    if (e == hipSuccess) e = dalloc(&h->arrive, n);
    if (e == hipSuccess) e = dalloc(&h->heights, 2 * n);
    if (e == hipSuccess) e = dalloc(&h->climb, 11 * n);
    if (e == hipSuccess) e = dalloc(&h->split_prefix, n);
    if (e == hipSuccess) e = dalloc(&h->scalars, rsi::kNumScalars);
    if (e == hipSuccess) e = dalloc(&h->counters, 1);
    if (e == hipSuccess) e = dalloc(&h->tri_off, M + 1);
    if (e == hipSuccess) e = dalloc(&h->vert_off, M + 1);
    if (e == hipSuccess) e = dalloc(&h->mesh_bounds, 6 * M);
    if (e == hipSuccess) e = dalloc(&h->mesh_height, M);
    if (e == hipSuccess) e = dalloc(&h->mesh_root, M);
    if (e == hipSuccess) e = dalloc(&h->mesh_entry, M);
    if (e == hipSuccess && batch) e = alloc_tables(h->bt, M);
    if (e == hipSuccess && batch) e = alloc_tables(h->bt_graph, M);
    if (e == hipSuccess)
        e = hipHostMalloc(reinterpret_cast<void **>(&h->h_scalars), sizeof(int32_t) * rsi::kNumScalars);
    if (e == hipSuccess && n > 0) e = rsi::ensure_sort_scratch(h->sort, n);
    // device flags and counters start clear (a fresh handle reports nothing)
    if (e == hipSuccess) e = hipMemset(h->scalars, 0, sizeof(int32_t) * rsi::kNumScalars);
    if (e == hipSuccess) e = hipMemset(h->counters, 0, sizeof(rsi::Counters));
    if (e == hipSuccess)
        e = hipMemcpy(h->tri_off, h->h_tri_off.data(), sizeof(int64_t) * (M + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(h->vert_off, h->h_vert_off.data(), sizeof(int64_t) * (M + 1), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h->mesh_entry, entry.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        st = hip_fail(e, "handle allocation");
        destroy_handle(h);
        return st;
    }
    *out = h;
    return RSI_OK;
}

// A build is stream-ordered: nothing is read back.  Index checks stay in
// device flags that rsi_query_stats reports; the traversal needs no tree
// height on the host (its deep pass is sized from a bound).
rsi_status finish_build(rsi_bvh *h, hipStream_t s, const char *who)
{
    h->last_stream = s;
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? RSI_OK : hip_fail(e, who);
}

// Wait for the handle's last work and read every mesh's tree height.
bool read_heights(rsi_bvh *h, std::vector<int32_t> &hts)
{
    hts.assign(h->M, 0);
    hipError_t e = hipStreamSynchronize(h->last_stream);
    if (e == hipSuccess && h->n_t > 0)
        e = hipMemcpy(hts.data(), h->mesh_height, sizeof(int32_t) * h->M, hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
        hip_fail(e, "tree heights");
        return false;
    }
    return true;
}

// Wait for the handle's last enqueued work and copy its device scalars.
hipError_t read_scalars(rsi_bvh *h)
{
    hipError_t e = hipStreamSynchronize(h->last_stream);
    if (e == hipSuccess)
        e = hipMemcpy(h->h_scalars, h->scalars, sizeof(int32_t) * rsi::kNumScalars, hipMemcpyDeviceToHost);
    return e;
}

// Single mesh: copy the indices and run the build kernels.
hipError_t enqueue_build_single(rsi_bvh *h, const float *V, const int32_t *T, hipStream_t s)
{
    hipError_t e = hipSuccess;
    h->inc_valid = false;  // new triangles, new Morton order: the adjoint's incidence table is stale
    if (h->n_t > 0) e = hipMemcpyAsync(h->T, T, sizeof(int32_t) * 3 * h->n_t, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = rsi::launch_build(h, V, s);
    return e;
}

// Batch: gather the meshes into the concatenated arrays and build.
hipError_t enqueue_build_batch(rsi_bvh *h, hipStream_t s)
{
    hipError_t e = rsi::launch_gather(h, s);
    if (e == hipSuccess) e = rsi::launch_build(h, h->V_all, s);
    return e;
}

bool valid_mode(uint32_t mode)
{
    return mode != 0 && !(mode & ~(uint32_t)(RSI_BOOL | RSI_FIRST_HIT | RSI_ALL_HITS | RSI_COUNT));
}

// Validate a batch query and write its tables; returns the total segment count.
rsi_status set_batch_tables(rsi_bvh *h, rsi::BatchTables &bt, const float *const *S, const float *const *E,
                            const int64_t *n_r, uint32_t mode, const rsi_outputs *outs, hipStream_t s,
                            int64_t *total, int32_t *cap)
{
    const int32_t M = h->M;
    if (!S || !E || !n_r || !outs) return invalid("rsi_batch_query: NULL table");
    if (mode == 0 || (mode & ~(uint32_t)(RSI_BOOL | RSI_FIRST_HIT | RSI_ALL_HITS)))
        return invalid("rsi_batch_query: mode must be a nonzero mask of RSI_BOOL, RSI_FIRST_HIT and RSI_ALL_HITS");
    constexpr int kTabs = 11;
    std::vector<int64_t> off(M + 1, 0);
    std::vector<const void *> tab(kTabs * (size_t)M, nullptr);
    int32_t K = 0;
    for (int32_t m = 0; m < M; ++m) {
        if (n_r[m] < 0) return invalid("rsi_batch_query: negative segment count");
        off[m + 1] = off[m] + n_r[m];
        if (n_r[m] > 0) {
            if (!S[m] || !E[m]) return invalid("rsi_batch_query: NULL segment pointer");
            if ((mode & RSI_BOOL) && !outs[m].hit) return invalid("rsi_batch_query: RSI_BOOL needs hit");
            if ((mode & RSI_FIRST_HIT) && (!outs[m].tri || !outs[m].t || !outs[m].uv || !outs[m].point))
                return invalid("rsi_batch_query: RSI_FIRST_HIT needs tri, t, uv, point");
            if (mode & RSI_ALL_HITS) {
                if (!outs[m].count || !outs[m].ids || !outs[m].ts)
                    return invalid("rsi_batch_query: RSI_ALL_HITS needs count, ids, ts");
                if (outs[m].capacity < 1 || (K && outs[m].capacity != K))
                    return invalid("rsi_batch_query: RSI_ALL_HITS needs one capacity >= 1 for every mesh");
                K = outs[m].capacity;
            }
        }
        const void *row[kTabs] = {S[m], E[m], outs[m].hit, outs[m].tri, outs[m].t, outs[m].uv, outs[m].point,
                                  outs[m].count, outs[m].ids, outs[m].ts, outs[m].spill_off};
        for (int k = 0; k < kTabs; ++k) tab[(size_t)k * M + m] = row[k];
    }
    if (off[M] >= (int64_t(1) << 30)) return invalid("rsi_batch_query: total segments must be below 2^30");
    void *dst[kTabs] = {bt.S, bt.E, bt.hit, bt.tri, bt.t, bt.uv, bt.point, bt.count, bt.ids, bt.ts, bt.spill_off};
    hipError_t e = hipMemcpyAsync(bt.seg_off, off.data(), sizeof(int64_t) * (M + 1), hipMemcpyHostToDevice, s);
    for (int k = 0; k < kTabs && e == hipSuccess; ++k)
        e = hipMemcpyAsync(dst[k], tab.data() + (size_t)k * M, sizeof(void *) * M, hipMemcpyHostToDevice, s);
    // the host vectors go out of scope on return: wait for the copies
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "rsi_batch_query: tables");
    *total = off[M];
    *cap = K ? K : 1;
    return RSI_OK;
}

// Device memory of a batched query (before any capture: nothing may be
// allocated inside one).
rsi_status prepare_batch_memory(rsi_bvh *h, int64_t total, uint32_t mode)
{
    const bool all = (mode & RSI_ALL_HITS) != 0;
    hipError_t e = rsi::ensure_query_memory(h, total, all);
    if (e == hipSuccess && all) {
        const int64_t dflt = total / 4 > (1 << 20) ? total / 4 : (1 << 20);
        e = rsi::ensure_pool(h, h->pool_want > dflt ? h->pool_want : dflt);
        h->last_pool_ids = h->pool_ids;
        h->last_pool_ts = h->pool_ts;
        h->last_pool_cap = h->pool_cap;
    }
    return e == hipSuccess ? RSI_OK : hip_fail(e, "batched query: scratch");
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
    rsi_bvh *h = nullptr;
    rsi_status st = alloc_handle(1, &n_v, &n_t, opts, false, &h);
    if (st != RSI_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = enqueue_build_single(h, V, T, s);
    st = e == hipSuccess ? finish_build(h, s, "rsi_build") : hip_fail(e, "rsi_build");
    if (st != RSI_OK) {
        destroy_handle(h);
        return st;
    }
    *out = h;
    return RSI_OK;
}

rsi_status rsi_rebuild(rsi_handle h, const float *V, int64_t n_v, const int32_t *T, void *stream)
{
    set_error("");
    if (!h) return invalid("rsi_rebuild: NULL handle");
    if (h->M != 1) return invalid("rsi_rebuild: batch handle (use rsi_batch_rebuild)");
    if (n_v < 0) return invalid("rsi_rebuild: negative n_v");
    if (h->n_t > 0 && n_v == 0) return invalid("rsi_rebuild: triangles given without vertices");
    if (h->n_t > 0 && (!V || !T)) return invalid("rsi_rebuild: NULL pointer with nonzero size");
    h->n_v = n_v;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = enqueue_build_single(h, V, T, s);
    if (e != hipSuccess) return hip_fail(e, "rsi_rebuild");
    return finish_build(h, s, "rsi_rebuild");
}

rsi_status rsi_refit(rsi_handle h, const float *V, int64_t n_v, void *stream)
{
    set_error("");
    if (!h) return invalid("rsi_refit: NULL handle");
    if (h->M != 1) return invalid("rsi_refit: batch handle");
    if (n_v != h->n_v) return invalid("rsi_refit: n_v differs from the vertex count of the last build");
    if (h->n_t > 0 && !V) return invalid("rsi_refit: NULL vertices");
    hipError_t e = rsi::launch_refit(h, V, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "rsi_refit");
    return RSI_OK;
}

rsi_status rsi_query(rsi_handle h, const float *S, const float *E, int64_t n_r, uint32_t mode,
                     const rsi_outputs *out, void *stream)
{
    set_error("");
    if (!h) return invalid("rsi_query: NULL handle");
    if (h->M != 1) return invalid("rsi_query: batch handle (use rsi_batch_query)");
    if (!out) return invalid("rsi_query: NULL outputs");
    if (n_r < 0) return invalid("rsi_query: negative n_r");
    if (!valid_mode(mode))
        return invalid("rsi_query: mode must be a nonzero mask of RSI_BOOL, RSI_FIRST_HIT, RSI_ALL_HITS, RSI_COUNT");
    if (mode & RSI_ALL_HITS) mode &= ~(uint32_t)RSI_COUNT;  // the all-hits pass writes the count anyway
    if (n_r == 0) return RSI_OK;  // nothing to read or write; output pointers may be NULL
    if (!S || !E) return invalid("rsi_query: NULL segment pointer");
    if ((mode & RSI_BOOL) && !out->hit) return invalid("rsi_query: RSI_BOOL needs out->hit");
    if ((mode & RSI_FIRST_HIT) && (!out->tri || !out->t || !out->uv || !out->point))
        return invalid("rsi_query: RSI_FIRST_HIT needs out->tri, t, uv, point");
    if (mode & RSI_ALL_HITS) {
        if (!out->count || !out->ids || !out->ts) return invalid("rsi_query: RSI_ALL_HITS needs out->count, ids, ts");
        if (out->capacity < 1) return invalid("rsi_query: capacity must be >= 1");
    }
    if ((mode & RSI_COUNT) && !out->count) return invalid("rsi_query: RSI_COUNT needs out->count");
    if (n_r >= (int64_t(1) << 30)) return invalid("rsi_query: n_r must be below 2^30");
    hipStream_t s = (hipStream_t)stream;
    rsi::QueryOut o = {out->hit, out->tri, out->t, out->uv, out->point, out->count, out->ids, out->ts,
                       out->capacity, nullptr, nullptr, nullptr, 0};
    h->last_stream = s;
    hipError_t e;
    if (mode & RSI_ALL_HITS) {
        o.spill_off = out->spill_off;
        if (out->spill_ids || out->spill_ts || out->spill_cap) {
            if (!out->spill_ids || !out->spill_ts || out->spill_cap < 1)
                return invalid("rsi_query: a caller spill pool needs spill_ids, spill_ts and spill_cap >= 1");
            o.pool_ids = out->spill_ids;
            o.pool_ts = out->spill_ts;
            o.pool_cap = out->spill_cap;
        } else {
            const int64_t dflt = n_r / 4 > (1 << 20) ? n_r / 4 : (1 << 20);
            e = rsi::ensure_pool(h, h->pool_want > dflt ? h->pool_want : dflt);
            if (e != hipSuccess) return hip_fail(e, "rsi_query: spill pool");
            o.pool_ids = h->pool_ids;
            o.pool_ts = h->pool_ts;
            o.pool_cap = h->pool_cap;
        }
        h->last_pool_ids = o.pool_ids;
        h->last_pool_ts = o.pool_ts;
        h->last_pool_cap = o.pool_cap;
    }
    if (h->n_t == 0) {
        e = rsi::launch_fill_miss(n_r, mode, o, s);
        if (e == hipSuccess) e = rsi::launch_clear_query(h, s);
        return e == hipSuccess ? RSI_OK : hip_fail(e, "rsi_query");
    }
    e = rsi::ensure_query_memory(h, n_r, (mode & RSI_ALL_HITS) != 0);
    if (e != hipSuccess) return hip_fail(e, "rsi_query: scratch");
    e = rsi::launch_query(h, S, E, n_r, mode, o, s);
    if (e != hipSuccess) return hip_fail(e, "rsi_query");
    return RSI_OK;
}

rsi_status rsi_inside(rsi_handle h, const float *P, int64_t n_p, uint8_t *inside, int32_t *count, float *E,
                      void *stream)
{
    set_error("");
    if (!h) return invalid("rsi_inside: NULL handle");
    if (h->M != 1) return invalid("rsi_inside: batch handle");
    if (n_p < 0) return invalid("rsi_inside: negative n_p");
    if (n_p == 0) return RSI_OK;
    if (!P || !inside) return invalid("rsi_inside: NULL point or output pointer");
    if (n_p >= (int64_t(1) << 30)) return invalid("rsi_inside: n_p must be below 2^30");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if ((!E || !count) && h->aux_cap < n_p) {
        if (h->aux_E) (void)hipFree(h->aux_E);
        if (h->aux_count) (void)hipFree(h->aux_count);
        h->aux_E = nullptr;
        h->aux_count = nullptr;
        h->aux_cap = 0;
        e = hipMalloc(reinterpret_cast<void **>(&h->aux_E), sizeof(float) * 3 * (size_t)n_p);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&h->aux_count), sizeof(int32_t) * (size_t)n_p);
        if (e != hipSuccess) return hip_fail(e, "rsi_inside: scratch");
        h->aux_cap = n_p;
    }
    float *ends = E ? E : h->aux_E;
    int32_t *cnt = count ? count : h->aux_count;
    rsi_outputs o = {};
    o.count = cnt;
    if (h->n_t == 0) {
        // no surface: every point is outside; the ends are the points themselves
        e = hipMemcpyAsync(ends, P, sizeof(float) * 3 * (size_t)n_p, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemsetAsync(cnt, 0, sizeof(int32_t) * (size_t)n_p, s);
        if (e == hipSuccess) e = rsi::launch_parity(cnt, n_p, inside, s);
        return e == hipSuccess ? RSI_OK : hip_fail(e, "rsi_inside");
    }
    e = rsi::launch_inside_ends(h, P, n_p, ends, s);
    if (e != hipSuccess) return hip_fail(e, "rsi_inside: segment ends");
    const rsi_status st = rsi_query(h, P, ends, n_p, RSI_COUNT, &o, stream);
    if (st != RSI_OK) return st;
    e = rsi::launch_parity(cnt, n_p, inside, s);
    return e == hipSuccess ? RSI_OK : hip_fail(e, "rsi_inside: parity");
}

rsi_status rsi_segment_order(rsi_handle h, const float *S, const float *E, int64_t n_r, int32_t *order,
                             void *stream)
{
    set_error("");
    if (!h) return invalid("rsi_segment_order: NULL handle");
    if (n_r < 0 || n_r >= (int64_t(1) << 31)) return invalid("rsi_segment_order: n_r must be in [0, 2^31)");
    if (n_r == 0) return RSI_OK;
    if (!S || !E || !order) return invalid("rsi_segment_order: NULL pointer");
    hipError_t e = rsi::launch_segment_order(h, S, E, n_r, order, (hipStream_t)stream);
    return e == hipSuccess ? RSI_OK : hip_fail(e, "rsi_segment_order");
}

rsi_status rsi_gather_segments(rsi_handle h, const float *S, const float *E, const int32_t *order, int64_t n_r,
                               float *S_out, float *E_out, void *stream)
{
    set_error("");
    if (!h) return invalid("rsi_gather_segments: NULL handle");
    if (n_r < 0 || n_r >= (int64_t(1) << 31)) return invalid("rsi_gather_segments: n_r must be in [0, 2^31)");
    if (n_r == 0) return RSI_OK;
    if (!S || !E || !order || !S_out || !E_out) return invalid("rsi_gather_segments: NULL pointer");
    hipError_t e = rsi::launch_gather_segments(h, S, E, order, n_r, S_out, E_out, (hipStream_t)stream);
    return e == hipSuccess ? RSI_OK : hip_fail(e, "rsi_gather_segments");
}

rsi_status rsi_compact(rsi_handle h, const uint8_t *hit, const int32_t *tri, const float *t, const float *point,
                       const float *S, const float *E, int64_t n_r, int32_t *ids, float *dist, int32_t *tri_out,
                       float *point_out, int64_t *n_out, void *stream)
{
    set_error("");
    if (!h || !n_out) return invalid("rsi_compact: NULL handle or count pointer");
    *n_out = 0;
    if (n_r < 0 || n_r >= (int64_t(1) << 31)) return invalid("rsi_compact: n_r must be in [0, 2^31)");
    if (n_r == 0) return RSI_OK;
    if (!ids) return invalid("rsi_compact: NULL ids");
    if (hit) {
        if (dist || tri_out || point_out) return invalid("rsi_compact: boolean selection gives ids only");
    } else {
        if (!tri) return invalid("rsi_compact: pass hit (boolean) or tri (first hit)");
        if (dist && (!t || !S || !E)) return invalid("rsi_compact: distances need t, S and E");
        if (point_out && !point) return invalid("rsi_compact: points need point");
    }
    hipError_t e = rsi::launch_compact(h, hit, S, E, tri, t, point, n_r, ids, dist, tri_out, point_out, n_out,
                                       (hipStream_t)stream);
    return e == hipSuccess ? RSI_OK : hip_fail(e, "rsi_compact");
}

rsi_status rsi_first_hit_backward(rsi_handle h, const float *V, int64_t n_v, const float *S, const float *E,
                                  int64_t n_r, const int32_t *tri, const float *g_t, const float *g_uv,
                                  const float *g_point, float *dV, float *dS, float *dE, void *stream)
{
    set_error("");
    if (!h) return invalid("rsi_first_hit_backward: NULL handle");
    if (h->M != 1) return invalid("rsi_first_hit_backward: batch handle");
    if (n_v != h->n_v)
        return invalid("rsi_first_hit_backward: n_v differs from the vertex count of the last build");
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
    hipError_t e = read_scalars(h);
    if (e != hipSuccess) return hip_fail(e, "rsi_spill_info");
    const int64_t ne = h->h_scalars[rsi::kOvfSegs];
    const uint64_t tot = (uint32_t)h->h_scalars[rsi::kOvfTotalLo] |
                         ((uint64_t)(uint32_t)h->h_scalars[rsi::kOvfTotalHi] << 32);
    *n_segments = ne < h->ovf_cap ? ne : h->ovf_cap;
    *n_crossings = (int64_t)tot < h->last_pool_cap ? (int64_t)tot : h->last_pool_cap;
    return RSI_OK;
}

rsi_status rsi_spill_read(rsi_handle h, int32_t *seg, int64_t *offset, int32_t *count, int32_t *ids, float *ts,
                          void *stream)
{
    set_error("");
    if (!h) return invalid("rsi_spill_read: NULL handle");
    int64_t n = 0, m = 0;
    rsi_status st = rsi_spill_info(h, &n, &m);
    if (st != RSI_OK) return st;
    if (n == 0) return RSI_OK;
    if (!seg || !offset || !count || (m > 0 && (!ids || !ts))) return invalid("rsi_spill_read: NULL buffer");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(seg, h->ovf_seg, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(offset, h->ovf_off, sizeof(int64_t) * n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(count, h->ovf_cnt, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && m > 0)
        e = hipMemcpyAsync(ids, h->last_pool_ids, sizeof(int32_t) * m, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess && m > 0)
        e = hipMemcpyAsync(ts, h->last_pool_ts, sizeof(float) * m, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "rsi_spill_read");
    return RSI_OK;
}

rsi_status rsi_query_stats(rsi_handle h, rsi_stats *out)
{
    set_error("");
    if (!h || !out) return invalid("rsi_query_stats: NULL argument");
    memset(out, 0, sizeof(*out));
    hipError_t e = read_scalars(h);
    if (e != hipSuccess) return hip_fail(e, "rsi_query_stats");
    const int32_t *c = h->h_scalars;
    auto u64 = [&](int lo, int hi) { return (int64_t)((uint32_t)c[lo] | ((uint64_t)(uint32_t)c[hi] << 32)); };
    out->bad_index = (c[rsi::kBadIndex] & 1) || (h->src_V && c[rsi::kBadGather]) ? 1 : 0;
    out->build_inconsistent = (c[rsi::kBadIndex] & 2) ? 1 : 0;
    out->walk_cut = c[rsi::kWalkCut] != 0;
    out->stack_dropped = c[rsi::kStackDropped] != 0;
    out->deep_segments = c[rsi::kRetryN];
    out->overflow_segments = c[rsi::kOvfUsed];
    out->overflow_crossings = u64(rsi::kOvfTotalLo, rsi::kOvfTotalHi);
    out->arena_records = c[rsi::kArenaUsed];
    // records handed out (in blocks; the arena must hold them all)
    const int64_t arena_claimed = u64(rsi::kArenaLo, rsi::kArenaHi);
    out->pool_capacity = h->last_pool_cap;
    out->overflow_full = (c[rsi::kOvfFull] != 0 || c[rsi::kRetryLost] != 0) ? 1 : 0;
    if (out->overflow_full) {
        // the next all-hits query gets a pool and an arena that hold this one
        int64_t want = out->overflow_crossings > arena_claimed ? out->overflow_crossings : arena_claimed;
        want += want / 4;
        if (want > h->pool_want) h->pool_want = want;
    }
    if (out->bad_index) return invalid("triangle index outside [0, n_v)");
    if (out->build_inconsistent) return invalid("inconsistent build state (report this)");
    if (out->overflow_full) {
        set_error("all-hits spill pool or arena too small for the last query (counts are exact; query again: "
                  "the library pool has grown, a caller pool needs overflow_crossings entries)");
        return RSI_E_OVERFLOW;
    }
    return RSI_OK;
}

// ------------------------------------------------------------- batches ---

rsi_status rsi_batch_create(int32_t n_meshes, const float *const *V, const int64_t *n_v, const int32_t *const *T,
                            const int64_t *n_t, const rsi_opts *opts, void *stream, rsi_handle *out)
{
    set_error("");
    if (!out) return invalid("rsi_batch_create: out is NULL");
    *out = nullptr;
    if (n_meshes < 1 || n_meshes > 65535) return invalid("rsi_batch_create: n_meshes must be in 1..65535");
    if (!V || !n_v || !T || !n_t) return invalid("rsi_batch_create: NULL table");
    for (int32_t m = 0; m < n_meshes; ++m) {
        if (n_v[m] < 0 || n_t[m] < 0) return invalid("rsi_batch_create: negative size");
        if (n_t[m] > 0 && n_v[m] == 0) return invalid("rsi_batch_create: triangles given without vertices");
        if ((n_v[m] > 0 && !V[m]) || (n_t[m] > 0 && !T[m])) return invalid("rsi_batch_create: NULL pointer");
    }
    rsi_bvh *h = nullptr;
    rsi_status st = alloc_handle(n_meshes, n_v, n_t, opts, true, &h);
    if (st != RSI_OK) return st;
    hipError_t e = hipMemcpy(h->src_V, V, sizeof(float *) * n_meshes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(h->src_T, T, sizeof(int32_t *) * n_meshes, hipMemcpyHostToDevice);
    hipStream_t s = (hipStream_t)stream;
    if (e == hipSuccess) e = enqueue_build_batch(h, s);
    st = e == hipSuccess ? finish_build(h, s, "rsi_batch_create") : hip_fail(e, "rsi_batch_create");
    if (st != RSI_OK) {
        destroy_handle(h);
        return st;
    }
    *out = h;
    return RSI_OK;
}

rsi_status rsi_batch_rebuild(rsi_handle h, void *stream)
{
    set_error("");
    if (!h) return invalid("rsi_batch_rebuild: NULL handle");
    if (!h->src_V) return invalid("rsi_batch_rebuild: not a batch handle");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = enqueue_build_batch(h, s);
    if (e != hipSuccess) return hip_fail(e, "rsi_batch_rebuild");
    return finish_build(h, s, "rsi_batch_rebuild");
}

rsi_status rsi_batch_query(rsi_handle h, const float *const *S, const float *const *E, const int64_t *n_r,
                           uint32_t mode, const rsi_outputs *outs, void *stream)
{
    set_error("");
    if (!h) return invalid("rsi_batch_query: NULL handle");
    if (!h->src_V) return invalid("rsi_batch_query: not a batch handle");
    hipStream_t s = (hipStream_t)stream;
    int64_t total = 0;
    int32_t cap = 1;
    rsi_status st = set_batch_tables(h, h->bt, S, E, n_r, mode, outs, s, &total, &cap);
    if (st != RSI_OK) return st;
    st = prepare_batch_memory(h, total, mode);
    if (st != RSI_OK) return st;
    h->last_stream = s;
    hipError_t e = rsi::launch_batch_query(h, h->bt, total, mode, cap, s);
    if (e != hipSuccess) return hip_fail(e, "rsi_batch_query");
    return RSI_OK;
}

rsi_status rsi_batch_capture(rsi_handle h, const float *const *S, const float *const *E, const int64_t *n_r,
                             uint32_t mode, const rsi_outputs *outs, int rebuild, void *stream)
{
    set_error("");
    if (!h) return invalid("rsi_batch_capture: NULL handle");
    if (!h->src_V) return invalid("rsi_batch_capture: not a batch handle");
    hipStream_t s = (hipStream_t)stream;
    int64_t total = 0;
    if (h->graph) {
        // the old graph reads bt_graph, which is about to be rewritten
        hipError_t w = hipDeviceSynchronize();
        if (w != hipSuccess) return hip_fail(w, "rsi_batch_capture: wait for replays");
        (void)hipGraphExecDestroy(h->graph);
        h->graph = nullptr;
    }
    int32_t cap = 1;
    rsi_status st = set_batch_tables(h, h->bt_graph, S, E, n_r, mode, outs, s, &total, &cap);
    if (st != RSI_OK) return st;
    st = prepare_batch_memory(h, total, mode);  // no allocation may happen inside the capture
    if (st != RSI_OK) return st;
    hipError_t e = hipSuccess;
    if (!h->capture_stream) e = hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "rsi_batch_capture: stream");
    hipGraph_t g = nullptr;
    e = hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "rsi_batch_capture: begin");
    hipError_t ek = hipSuccess;
    if (rebuild) ek = enqueue_build_batch(h, h->capture_stream);
    if (ek == hipSuccess) ek = rsi::launch_batch_query(h, h->bt_graph, total, mode, cap, h->capture_stream);
    e = hipStreamEndCapture(h->capture_stream, &g);
    if (ek != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(ek, "rsi_batch_capture: enqueue");
    }
    if (e != hipSuccess) return hip_fail(e, "rsi_batch_capture: end");
    e = hipGraphInstantiate(&h->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        h->graph = nullptr;
        return hip_fail(e, "rsi_batch_capture: instantiate");
    }
    return RSI_OK;
}

rsi_status rsi_batch_replay(rsi_handle h, void *stream)
{
    set_error("");
    if (!h) return invalid("rsi_batch_replay: NULL handle");
    if (!h->graph) return invalid("rsi_batch_replay: nothing captured");
    h->last_stream = (hipStream_t)stream;
    hipError_t e = hipGraphLaunch(h->graph, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "rsi_batch_replay");
    return RSI_OK;
}

// --------------------------------------------------------------- tuning ---

// A captured graph froze the launch shape of the old options: drop it.
static rsi_status drop_graph(rsi_bvh *h)
{
    if (!h->graph) return RSI_OK;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "waiting for graph replays");
    (void)hipGraphExecDestroy(h->graph);
    h->graph = nullptr;
    return RSI_OK;
}

// Lay out the four-way view for the current tree when branching 4 is asked
// for and the tree was built without it (synchronous: a short device pass).
rsi_status apply_width(rsi_bvh *h, hipStream_t s)
{
    if (h->width == 2) {
        h->width_built = 2;
        return RSI_OK;
    }
    if (h->width_built == 4) return RSI_OK;
    hipError_t e = hipSuccess;
    if (!h->nodes4) e = dalloc(&h->nodes4, h->n_t);
    if (e == hipSuccess) e = rsi::launch_widen(h, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? RSI_OK : hip_fail(e, "branching 4: four-way layout");
}

rsi_status rsi_set_opts(rsi_handle h, const rsi_opts *opts)
{
    set_error("");
    if (!h) return invalid("rsi_set_opts: NULL handle");
    rsi_status st = drop_graph(h);
    if (st != RSI_OK) return st;
    st = read_opts(opts, h);
    if (st != RSI_OK) return st;
    return apply_width(h, nullptr);
}

rsi_status rsi_get_opts(rsi_handle h, rsi_opts *out)
{
    set_error("");
    if (!h || !out) return invalid("rsi_get_opts: NULL argument");
    memset(out, 0, sizeof(*out));
    out->leaf_size = h->leaf_size;
    out->block_size = h->block_size;
    out->defer_lanes = h->defer_lanes;
    out->refill_lanes = h->refill_lanes;
    out->chunk = h->chunk;
    out->stack_depth = h->stack_cap;
    out->branching = h->width;
    return RSI_OK;
}

static rsi_status tune_rebuild(rsi_bvh *h, const rsi_tune_job *job, hipStream_t s)
{
    if (h->src_V) return rsi_batch_rebuild(h, s);
    if (h->n_t > 0 && (!job->V || !job->T)) return invalid("rsi_tune: V and T are needed to try leaf sizes");
    return rsi_rebuild(h, job->V, job->n_v, job->T, s);
}

static rsi_status tune_run(rsi_bvh *h, const rsi_tune_job *job, hipStream_t s)
{
    if (h->src_V) return rsi_batch_query(h, job->bS, job->bE, job->b_nr, job->mode, job->b_outs, s);
    return rsi_query(h, job->S, job->E, job->n_r, job->mode, job->out, s);
}

rsi_status rsi_tune(rsi_handle h, const rsi_tune_job *job, const rsi_opts *cand, int32_t n_cand, int32_t reps,
                    float *ms, int32_t *best, void *stream)
{
    set_error("");
    if (!h || !job || !cand || n_cand < 1 || reps < 1 || !best) return invalid("rsi_tune: bad argument");
    {
        rsi_status dg = drop_graph(h);
        if (dg != RSI_OK) return dg;
    }
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return hip_fail(e, "rsi_tune: events");
    // options before tuning (set directly: a zero field in rsi_opts means "keep")
    const int32_t o_leaf = h->leaf_size, o_block = h->block_size, o_defer = h->defer_lanes;
    const int32_t o_refill = h->refill_lanes, o_chunk = h->chunk, o_stack = h->stack_cap, o_width = h->width;
    auto restore = [&]() {
        h->width = o_width;
        h->leaf_size = o_leaf;
        h->block_size = o_block;
        h->defer_lanes = o_defer;
        h->refill_lanes = o_refill;
        h->chunk = o_chunk;
        h->stack_cap = o_stack;
    };
    rsi_status st = RSI_OK;
    float best_ms = 0.0f;
    int32_t best_i = -1;
    std::vector<float> t((size_t)reps);
    for (int32_t c = 0; c < n_cand && st == RSI_OK; ++c) {
        const int32_t old_leaf = h->leaf_size;
        restore();  // each candidate starts from the original options
        st = read_opts(&cand[c], h);
        if (st == RSI_OK && h->leaf_size != old_leaf) st = tune_rebuild(h, job, s);
        if (st == RSI_OK) st = apply_width(h, s);
        if (st == RSI_OK) st = tune_run(h, job, s);  // warm-up
        for (int32_t r = 0; r < reps && st == RSI_OK; ++r) {
            e = hipEventRecord(e0, s);
            if (e == hipSuccess) st = tune_run(h, job, s);
            if (st == RSI_OK && e == hipSuccess) e = hipEventRecord(e1, s);
            if (st == RSI_OK && e == hipSuccess) e = hipEventSynchronize(e1);
            if (st == RSI_OK && e == hipSuccess) e = hipEventElapsedTime(&t[(size_t)r], e0, e1);
            if (e != hipSuccess) st = hip_fail(e, "rsi_tune: timing");
        }
        if (st != RSI_OK) break;
        std::vector<float> sorted = t;
        for (size_t x = 1; x < sorted.size(); ++x)
            for (size_t y = x; y > 0 && sorted[y] < sorted[y - 1]; --y) std::swap(sorted[y], sorted[y - 1]);
        const float med = sorted[sorted.size() / 2];
        if (ms) ms[c] = med;
        if (best_i < 0 || med < best_ms) {
            best_ms = med;
            best_i = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != RSI_OK) {
        const int32_t cur_leaf = h->leaf_size;
        restore();
        if (h->leaf_size != cur_leaf) (void)tune_rebuild(h, job, s);
        (void)apply_width(h, s);
        return st;
    }
    const int32_t old_leaf = h->leaf_size;
    restore();
    st = read_opts(&cand[best_i], h);
    if (st == RSI_OK && h->leaf_size != old_leaf) st = tune_rebuild(h, job, s);
    if (st == RSI_OK) st = apply_width(h, s);
    *best = best_i;
    return st;
}

// --------------------------------------------------------------- status ---

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
    out->wave_loops = c.wave_loops;
    out->wave_node_steps = c.wave_node_steps;
    out->wave_leaf_phases = c.wave_leaf_phases;
    out->wave_refills = c.wave_refills;
    out->lanes_blocked = c.lanes_blocked;
    out->lanes_waiting = c.lanes_waiting;
    out->wave_leaf_rounds = c.wave_leaf_rounds;
    out->leaf_lanes = c.leaf_lanes;
    return RSI_OK;
}

rsi_status rsi_get_tree_info(rsi_handle h, rsi_tree_info *out)
{
    set_error("");
    if (!h || !out) return invalid("rsi_get_tree_info: NULL argument");
    memset(out, 0, sizeof(*out));
    std::vector<int32_t> hts;
    if (!read_heights(h, hts)) return RSI_E_HIP;
    int32_t mx = 0;
    for (int32_t x : hts) mx = x > mx ? x : mx;
    out->n_t = h->n_t;
    out->n_nodes = h->n_t;
    out->height = mx;
    out->leaf_size = h->leaf_size;
    out->entry = h->n_t > 0 ? (int32_t)(h->h_tri_off[1] - 1) : 0;
    out->n_meshes = h->M;
    return RSI_OK;
}

rsi_status rsi_get_mesh_info(rsi_handle h, int32_t mesh, int64_t *tri_offset, int64_t *n_t, int32_t *height)
{
    set_error("");
    if (!h) return invalid("rsi_get_mesh_info: NULL handle");
    if (mesh < 0 || mesh >= h->M) return invalid("rsi_get_mesh_info: mesh out of range");
    if (tri_offset) *tri_offset = h->h_tri_off[mesh];
    if (n_t) *n_t = h->h_tri_off[mesh + 1] - h->h_tri_off[mesh];
    if (height) {
        std::vector<int32_t> hts;
        if (!read_heights(h, hts)) return RSI_E_HIP;
        *height = hts[mesh];
    }
    return RSI_OK;
}

rsi_status rsi_export_tree(rsi_handle h, float *boxes, int32_t *refs, int32_t *order, uint64_t *keys)
{
    set_error("");
    if (!h) return invalid("rsi_export_tree: NULL handle");
    const int64_t n = h->n_t;
    if (n == 0) return RSI_OK;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess && (boxes || refs)) {
        rsi::Node *tmp = new (std::nothrow) rsi::Node[(size_t)n];
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
    destroy_handle(h);
}

}  // extern "C"
