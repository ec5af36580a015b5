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
    kOvfSegs = 9,      // overflowed segments of the last all-hits pass
    kOvfTotalLo = 10,  // 64-bit total crossings of those segments (lo, hi words)
    kOvfTotalHi = 11,
    kWorkNext = 12,    // next unclaimed work item of the running query kernel
    kSegBounds = 16,   // 6 ordered ints: bounding box of segment midpoints (segment order)
    kNumScalars = 32
};

struct Counters {
    unsigned long long node_visits, box_tests, tri_tests, segments;
    // per wave: loop iterations, iterations with a node step, with a leaf
    // phase, with a refill
    unsigned long long wave_loops, wave_node_steps, wave_leaf_phases, wave_refills;
    unsigned long long lanes_blocked, lanes_waiting;
};

// Radix-sort scratch sized for n elements.
struct SortScratch {
    uint64_t *keys_alt = nullptr;
    uint32_t *vals_alt = nullptr;
    uint32_t *hist = nullptr;
    uint32_t *h_word = nullptr;  // pinned host word: a read-back of the sort
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
    int32_t stack_cap = 0;         // LDS part of the traversal stack (0: the whole stack)
    int32_t height = 0;            // largest tree height over the meshes
    bool counting = false;
    std::vector<int64_t> h_tri_off, h_vert_off;  // host copies of the offsets
    std::vector<int32_t> h_height;

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

    // all-hits overflow (device)
    int32_t *ovf_seg = nullptr;    // overflowed segment ids
    int32_t *ovf_cnt = nullptr;    // their counts
    int64_t *ovf_off = nullptr;    // their offsets into the pool
    int64_t ovf_cap = 0;
    int32_t *pool_ids = nullptr;
    float *pool_ts = nullptr;
    int64_t pool_cap = 0;
    int64_t last_ovf_segs = 0;
    int64_t last_ovf_total = 0;

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

    // global part of the traversal stack when stack_cap is below the height
    int32_t *gstack = nullptr;
    int64_t gstack_cap = 0;

    // segment order (and the adjoint's hit order): keys, values and sort
    // scratch sized for the segments
    uint64_t *seg_keys = nullptr;
    int64_t seg_key_cap = 0;
    uint32_t *adj_vals = nullptr;
    int64_t adj_val_cap = 0;
    rsi::SortScratch seg_sort;

    // stream compaction: per-block counts and their scan (+ total)
    int32_t *compact_counts = nullptr;
    int64_t compact_cap = 0;

    // inside test: far ends and counts when the caller passes none
    float *aux_E = nullptr;
    int32_t *aux_count = nullptr;
    int64_t aux_cap = 0;

    // pinned host mirror of `scalars`
    int32_t *h_scalars = nullptr;
    // pinned host block that k_publish fills after a build: the two index
    // flags, then the M tree heights; d_pub is its device-side address
    int32_t *h_pub = nullptr;
    int32_t *d_pub = nullptr;
};

namespace rsi {

// error plumbing (api.hip)
void set_error(const std::string &msg);

// build.hip
hipError_t launch_gather(rsi_bvh *h, hipStream_t s);
hipError_t launch_build(rsi_bvh *h, const float *V, hipStream_t s);
hipError_t launch_refit(rsi_bvh *h, const float *V, hipStream_t s);
hipError_t launch_publish(rsi_bvh *h, hipStream_t s);

// sort.hip: stable LSD radix sort of 63-bit keys with 32-bit values, in
// place; with mesh_off (M > 1) the mesh of each value is the most
// significant digit
hipError_t radix_sort_pairs(uint64_t *keys, uint32_t *vals, int64_t n, int key_bits, SortScratch &scratch,
                            hipStream_t s, const int64_t *mesh_off = nullptr, int32_t M = 1);
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
};
hipError_t launch_query(rsi_bvh *h, const float *S, const float *E, int64_t n_r, uint32_t mode,
                        const QueryOut &o, hipStream_t s);
hipError_t launch_spill(rsi_bvh *h, const float *S, const float *E, uint32_t mode, const QueryOut &o,
                        hipStream_t s);
hipError_t launch_fill_miss(int64_t n_r, uint32_t mode, const QueryOut &o, hipStream_t s);
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
hipError_t launch_batch_query(rsi_bvh *h, const BatchTables &bt, int64_t n_total, uint32_t mode, hipStream_t s);
// size the global part of the traversal stack (call outside graph capture)
hipError_t ensure_gstack(rsi_bvh *h);

// adjoint.hip
hipError_t launch_first_hit_adjoint(rsi_bvh *h, const float *V, const float *S, const float *E, int64_t n_r,
                                    const int32_t *tri, const float *g_t, const float *g_uv, const float *g_p,
                                    float *dV, float *dS, float *dE, hipStream_t s);

}  // namespace rsi
