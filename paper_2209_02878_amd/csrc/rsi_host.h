// rsi_host.h -- host-side handle and the internal launch functions shared by
// the ABI layer (api.hip) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "rsi_device.h"

namespace rsi {

// Device scalars of a handle (one small array, read back when needed).
enum Scalar {
    kBadIndex = 6,     // nonzero if a triangle index was out of range (1) or the build state was inconsistent (2)
    kBadGather = 7,    // nonzero if a batch gather met a triangle index outside its mesh
    kOvfTotalLo = 10,  // 64-bit total crossings of those segments: pool entries reserved (lo, hi words)
    kOvfTotalHi = 11,
    kWalkCut = 13,     // walks stopped by the node-visit bound (damaged tree)
    kSegBounds = 16,   // 6 ordered ints: bounding box of segment midpoints (segment order)
    kRetryN = 22,      // segments whose stack outgrew its LDS part, queued for the deep pass
    kWorkRetry = 23,   // next unclaimed item of the deep pass
    kRetryLost = 24,   // retry queue full (cannot happen with a queue of one entry per segment)
    kStackDropped = 25,  // pushes dropped by the deep pass (only a damaged tree is that deep)
    kOvfFull = 26,     // the overflow table, arena or pool was too small: lists incomplete
    kOvfUsed = 27,     // all hits: overflow-table entries in use (segments with more crossings than slots)
    kArenaUsed = 28,   // all hits: arena records placed into the pool (crossings past the slots)
    kOvfValid = 29,    // all hits: overflow-table entries that are not void (listed in table order)
    kWorkXcd = 32,     // 8 counters, kWorkStride ints (128 bytes) apart: items claimed from each
                       // eighth of the main query pass's items
    kWorkStride = 32,
    // the all-hits block counters, each on its own 128-byte line (waves claim
    // blocks from them throughout the walk)
    kOvfSegs = kWorkXcd + 8 * kWorkStride,  // overflow-table entries handed out (in blocks; unused ones are void)
    kArenaLo = kOvfSegs + kWorkStride,      // 64-bit count of arena records handed out during the walk, in
    kArenaHi = kArenaLo + 1,                // blocks (lo, hi words)
    kNumScalars = kArenaLo + kWorkStride
};

struct Counters {
    unsigned long long node_visits, box_tests, tri_tests, segments;
    // per wave: loop iterations, iterations with a node step, with a leaf
    // phase, with a refill
    unsigned long long wave_loops, wave_node_steps, wave_leaf_phases, wave_refills;
    unsigned long long lanes_blocked, lanes_waiting;
    // leaf phases: rounds (one leaf test per lane and round), lanes testing
    unsigned long long wave_leaf_rounds, leaf_lanes;
};

// Radix-sort scratch sized for n elements.
struct SortScratch {
    uint64_t *keys_alt = nullptr;
    uint32_t *vals_alt = nullptr;
    uint32_t *hist = nullptr;
    int64_t cap = 0;
    int64_t hist_cap = 0;
};

// Per-mesh tables of a batched query (device arrays, one entry per mesh).
struct BatchTables {
    int64_t *seg_off = nullptr;        // [M+1] segment offsets of the work items
    const float **S = nullptr;         // [M] segment starts of each mesh
    const float **E = nullptr;
    uint8_t **hit = nullptr;
    int32_t **tri = nullptr;
    float **t = nullptr;
    float **uv = nullptr;
    float **point = nullptr;
    int32_t **count = nullptr;
    int32_t **ids = nullptr;
    float **ts = nullptr;
    int64_t **spill_off = nullptr;
};

}  // namespace rsi

// A handle owns the trees of M >= 1 meshes in concatenated arrays: mesh m
// owns triangles, sorted leaves and node records [tri_off[m], tri_off[m+1]).
struct rsi_bvh {
    int device = 0;
    int32_t M = 1;
    int64_t n_v = 0, n_t = 0;      // totals over all meshes
    int32_t leaf_size = 1;
    int32_t block_size = 128;
    int32_t defer_lanes = 32;
    int32_t refill_lanes = 32;
    int32_t chunk = 0;             // 0: sized per launch
    int32_t stack_cap = 0;         // LDS stack entries per lane of the main pass (0: default)
    bool counting = false;
    std::vector<int64_t> h_tri_off, h_vert_off;  // host copies of the offsets

    // mesh tables (device)
    int64_t *tri_off = nullptr;    // [M+1]
    int64_t *vert_off = nullptr;   // [M+1]
    int32_t *mesh_bounds = nullptr;  // [6M]
    int32_t *mesh_height = nullptr;  // [M]
    int32_t *mesh_root = nullptr;    // [M]
    int32_t *mesh_entry = nullptr;   // [M] entry node per mesh, -1 for an empty mesh

    // geometry and tree (device)
    int32_t *T = nullptr;          // index triplets with global vertex indices [n_t*3]
    float *V_all = nullptr;        // concatenated vertices (batches only) [n_v*3]
    const float **src_V = nullptr; // batches: the caller's per-mesh vertex pointers [M]
    const int32_t **src_T = nullptr;
    float *cent = nullptr;         // centroids SoA [3*n_t]
    uint64_t *keys = nullptr;      // Morton codes, sorted in place [n_t]
    uint32_t *order = nullptr;     // original triangle per sorted position [n_t]
    int32_t *rank = nullptr;       // sorted position of each triangle (inverse of order) [n_t]
    rsi::Node *nodes = nullptr;    // [max(n_t, 1)]; each mesh's last record is its entry node
    rsi::Tri *tris = nullptr;      // [n_t] in sorted order
    int32_t *arrive = nullptr;     // arrival counters [n_t]
    int32_t *heights = nullptr;    // child heights [2*n_t]
    int32_t *climb = nullptr;      // climbs handed from the local to the global build pass [11*n_t]
    uint8_t *split_prefix = nullptr;  // common-prefix length at each sorted split [n_t]
    int32_t *scalars = nullptr;    // rsi::Scalar
    rsi::Counters *counters = nullptr;
    rsi::SortScratch sort;

    // all-hits lists beyond the slots (device): the overflow table (one
    // entry per overflowed segment: work item, count, pool offset), the arena
    // of (entry, rank, sorted position) records written during the walk, and
    // the library's pool of full lists (used when the caller passes none)
    int32_t *ovf_seg = nullptr;
    int32_t *ovf_cnt = nullptr;
    int32_t *ovf_list = nullptr;  // the entries that are not void, in table order
    int64_t *ovf_off = nullptr;
    int64_t ovf_cap = 0;
    int4 *arena = nullptr;
    int64_t arena_cap = 0;
    unsigned long long *ovf_part = nullptr;  // part sums of the pool-offset scan
    int64_t ovf_part_cap = 0;
    int32_t *pool_ids = nullptr;
    float *pool_ts = nullptr;
    int64_t pool_cap = 0;
    int64_t pool_want = 0;         // pool entries the last overflowing query needed (grown to on the next query)
    int32_t *last_pool_ids = nullptr;  // pool of the last all-hits query (the caller's or the library's)
    float *last_pool_ts = nullptr;
    int64_t last_pool_cap = 0;

    // walks whose stack outgrew its LDS part: queue of work items and the
    // device-memory stack of the deep pass (a small fixed grid)
    int32_t *retry_q = nullptr;
    int64_t retry_cap = 0;
    int32_t *retry_stack = nullptr;
    int64_t retry_stack_cap = 0;
    int32_t height_bound = 0;      // bound on any tree height of the handle's meshes (sizes the deep pass)
    hipStream_t last_stream = nullptr;  // stream of the last enqueued call (waited on by rsi_query_stats)

    // batched queries (device tables, sized for M meshes): `bt` serves the
    // eager calls, `bt_graph` belongs to the captured graph, so an eager call
    // never rewrites what a replay reads
    rsi::BatchTables bt;
    rsi::BatchTables bt_graph;
    hipGraphExec_t graph = nullptr;
    hipStream_t capture_stream = nullptr;

    // four-way view of the tree (branching 4): requested width, and the width
    // the current tree was laid out for
    int32_t width = 4;
    int32_t width_built = 2;
    rsi::Node4 *nodes4 = nullptr;

    // segment order (and the adjoint's cell grouping): keys, values and sort
    // scratch sized for the segments
    uint64_t *seg_keys = nullptr;
    int64_t seg_key_cap = 0;
    uint32_t *adj_vals = nullptr;
    int64_t adj_val_cap = 0;
    rsi::SortScratch seg_sort;
    // first-hit adjoint: per-segment records, per-triangle sums (FP64) and
    // the vertex incidence table of the current topology
    float4 *adj_rec = nullptr;
    int64_t adj_rec_cap = 0;
    float2 *adj_rec_v = nullptr;
    int64_t adj_rec_v_cap = 0;
    double *tri_sum = nullptr;
    int64_t tri_sum_cap = 0;
    double *adj_part = nullptr;  // per (cell, chunk, cell triangle): partial sums
    int64_t adj_part_cap = 0;
    int64_t *adj_cell_first = nullptr;  // first sorted pair of every cell
    int64_t adj_cell_first_cap = 0;
    int64_t *inc_first = nullptr;       // first incidence-table entry of every vertex
    int64_t inc_first_cap = 0;
    uint64_t *inc_keys = nullptr;
    uint32_t *inc_vals = nullptr;
    int64_t inc_cap = 0;
    bool inc_valid = false;

    // stream compaction: per-block counts and their scan (+ total)
    int32_t *compact_counts = nullptr;
    int64_t compact_cap = 0;

    // inside test: far ends and counts when the caller passes none
    float *aux_E = nullptr;
    int32_t *aux_count = nullptr;
    int64_t aux_cap = 0;

    // pinned host mirror of `scalars`
    int32_t *h_scalars = nullptr;
};

namespace rsi {

// error plumbing (api.hip)
void set_error(const std::string &msg);

// build.hip
hipError_t launch_gather(rsi_bvh *h, hipStream_t s);
hipError_t launch_build(rsi_bvh *h, const float *V, hipStream_t s);
hipError_t launch_refit(rsi_bvh *h, const float *V, hipStream_t s);

// sort.hip: stable LSD radix sort of (key, value) pairs by key bits
// [first_bit, key_bits), in place; with mesh_off (M > 1) the mesh of each
// value is the most significant digit.  With kres and vres the result may
// be left in the scratch buffers instead of being copied back: *kres, *vres
// then name the arrays that hold it.
hipError_t radix_sort_pairs(uint64_t *keys, uint32_t *vals, int64_t n, int key_bits, SortScratch &scratch,
                            hipStream_t s, const int64_t *mesh_off = nullptr, int32_t M = 1, int first_bit = 0,
                            uint64_t **kres = nullptr, uint32_t **vres = nullptr);
hipError_t ensure_sort_scratch(SortScratch &scratch, int64_t n);
void free_sort_scratch(SortScratch &scratch);

// query.hip
struct QueryOut {
    uint8_t *hit;
    int32_t *tri;
    float *t, *uv, *point;
    int32_t *count, *ids;
    float *ts;
    int32_t cap;
    int64_t *spill_off;  // optional: per segment, offset of its full list in the pool (-1: none)
    int32_t *pool_ids;   // pool of the full lists of overflowed segments (caller's or the library's)
    float *pool_ts;
    int64_t pool_cap;
};
hipError_t launch_query(rsi_bvh *h, const float *S, const float *E, int64_t n_r, uint32_t mode,
                        const QueryOut &o, hipStream_t s);
// The deep pass's queue (one entry per segment) and device-memory stack.
struct QueryScratch {
    int32_t *retry_q;
    int64_t retry_cap;
    int32_t *gstack;
    int64_t gstack_cap;
};
// launch_query with the deep pass's memory given by the caller; keep_flags
// (a later part of a query split into parts) keeps the damaged-tree flags
// and work counters of the earlier parts
hipError_t launch_query_scratch(rsi_bvh *h, const float *S, const float *E, int64_t n_r, uint32_t mode,
                                const QueryOut &o, const QueryScratch &sc, bool keep_flags, hipStream_t s);
// stack entries (int32) the deep pass of a query in `mode` needs
int64_t deep_stack_entries(const rsi_bvh *h, uint32_t mode);
hipError_t launch_fill_miss(int64_t n_r, uint32_t mode, const QueryOut &o, hipStream_t s);
// zero the per-query device scalars (a query that launches no walk)
hipError_t launch_clear_query(rsi_bvh *h, hipStream_t s);
hipError_t launch_widen(rsi_bvh *h, hipStream_t s);
hipError_t launch_segment_order(rsi_bvh *h, const float *S, const float *E, int64_t n, int32_t *order,
                                hipStream_t s);
hipError_t launch_gather_segments(rsi_bvh *h, const float *S, const float *E, const int32_t *order, int64_t n,
                                  float *So, float *Eo, hipStream_t s);
hipError_t launch_compact(rsi_bvh *h, const uint8_t *hit, const float *S, const float *E, const int32_t *tri,
                          const float *t, const float *point, int64_t n, int32_t *ids, float *dist,
                          int32_t *tri_out, float *point_out, int64_t *n_out, hipStream_t s);
hipError_t launch_inside_ends(const rsi_bvh *h, const float *P, int64_t n, float *E, hipStream_t s);
hipError_t launch_parity(const int32_t *count, int64_t n, uint8_t *inside, hipStream_t s);
hipError_t launch_batch_query(rsi_bvh *h, const BatchTables &bt, int64_t n_total, uint32_t mode, int32_t cap,
                              hipStream_t s);
// device memory of a query over n work items: retry queue, deep-pass stack
// and, for all hits, the overflow table and arena (call outside capture)
hipError_t ensure_query_memory(rsi_bvh *h, int64_t n, bool all_hits);
// size the library's pool of full lists for at least n entries
hipError_t ensure_pool(rsi_bvh *h, int64_t n);

// adjoint.hip
hipError_t launch_first_hit_adjoint(rsi_bvh *h, const float *V, const float *S, const float *E, int64_t n_r,
                                    const int32_t *tri, const float *g_t, const float *g_uv, const float *g_p,
                                    float *dV, float *dS, float *dE, hipStream_t s);

}  // namespace rsi
