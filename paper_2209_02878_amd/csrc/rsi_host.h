// rsi_host.h -- host-side handle and the internal launch functions shared by
// the ABI layer (api.hip) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "rsi_device.h"

namespace rsi {

// Device scalars written by the build (one small array, read back once).
enum Scalar {
    kBoundLo = 0,      // 3 ordered-int centroid minima
    kBoundHi = 3,      // 3 ordered-int centroid maxima
    kBadIndex = 6,     // nonzero if a triangle index was out of range
    kHeight = 7,       // levels of internal nodes below the entry node
    kRootRef = 8,      // reference of the root (internal index or leaf ref)
    kOvfSegs = 9,      // overflowed segments of the last all-hits pass
    kOvfTotalLo = 10,  // 64-bit total crossings of those segments (lo, hi words)
    kOvfTotalHi = 11,
    kWorkNext = 12,    // next unclaimed work item of the running query kernel
    kNumScalars = 16
};

struct Counters {
    unsigned long long node_visits, box_tests, tri_tests, segments;
};

// Radix-sort scratch sized for n elements.
struct SortScratch {
    uint64_t *keys_alt = nullptr;
    uint32_t *vals_alt = nullptr;
    uint32_t *hist = nullptr;
    int64_t cap = 0;
    int64_t hist_cap = 0;
};

}  // namespace rsi

struct rsi_bvh {
    int device = 0;
    int64_t n_v = 0, n_t = 0;
    int32_t leaf_size = 1;
    int32_t block_size = 256;
    int32_t defer_lanes = 32;
    int32_t refill_lanes = 32;
    int32_t chunk = 0;  // 0: sized per launch
    int32_t height = 0;
    int32_t root_ref = 0;
    int32_t entry = 0;
    bool counting = false;

    // geometry and tree (device)
    int32_t *T = nullptr;          // copy of the index triplets [n_t*3]
    float *cent = nullptr;         // centroids SoA [3*n_t]
    uint64_t *keys = nullptr;      // Morton codes, sorted in place [n_t]
    uint32_t *order = nullptr;     // original id per sorted position [n_t]
    rsi::Node *nodes = nullptr;    // [max(n_t, 1)]; node n_t-1 is the entry node
    rsi::Tri *tris = nullptr;      // [n_t] in sorted order
    int32_t *arrive = nullptr;     // arrival counters [n_t]
    int32_t *heights = nullptr;    // child heights [2*n_t]
    int32_t *climb = nullptr;      // climbs handed from the local to the global build pass [11*n_t]
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

    // pinned host mirror of `scalars`
    int32_t *h_scalars = nullptr;
};

namespace rsi {

// error plumbing (api.hip)
void set_error(const std::string &msg);

// build.hip
hipError_t launch_build(rsi_bvh *h, const float *V, hipStream_t s);
hipError_t launch_refit(rsi_bvh *h, const float *V, hipStream_t s);

// sort.hip: stable LSD radix sort of 63-bit keys with 32-bit values, in place
hipError_t radix_sort_pairs(uint64_t *keys, uint32_t *vals, int64_t n, int key_bits,
                            SortScratch &scratch, hipStream_t s);
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

// adjoint.hip
hipError_t launch_first_hit_adjoint(rsi_bvh *h, const float *V, const float *S, const float *E, int64_t n_r,
                                    const int32_t *tri, const float *g_t, const float *g_uv, const float *g_p,
                                    float *dV, float *dS, float *dE, hipStream_t s);

}  // namespace rsi
