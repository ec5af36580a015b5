// compact.hip -- stream compaction of query results into the paper's compact
// outputs (Section 2.4, extended usage): the ids of the segments that cross
// the mesh, and with them the first-hit distance, triangle and point
// (`barycentric`: intersecting rays, distances, intersecting triangles,
// intersecting points).
//
// Three launches: per-block counts of selected segments (1024 per block,
// wave64 ballots), one workgroup's exclusive scan of the block counts, and a
// scatter in which every block recomputes its selection, ranks it with
// ballots and writes in increasing segment order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rsi_host.h"

namespace rsi {
namespace {

constexpr int kCThreads = 256;
constexpr int kCItems = 4;
constexpr int kCBlock = kCThreads * kCItems;

// Selection: hit[i] != 0 (boolean output) or tri[i] >= 0 (first-hit output).
struct Select {
    const uint8_t *hit;
    const int32_t *tri;
    __device__ inline bool operator()(int64_t i) const { return hit ? hit[i] != 0 : tri[i] >= 0; }
};

__global__ __launch_bounds__(kCThreads) void k_block_counts(Select sel, int64_t n, int32_t *__restrict__ counts)
{
    __shared__ int32_t wsum[kCThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kCBlock;
    int32_t c = 0;
#pragma unroll
    for (int r = 0; r < kCItems; ++r) {
        const int64_t i = base + r * kCThreads + threadIdx.x;
        const bool f = i < n && sel(i);
        c += (int32_t)__popcll(__ballot(f));
    }
    if (__lane_id() == 0) wsum[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int w = 0; w < kCThreads / 64; ++w) t += wsum[w];
        counts[blockIdx.x] = t;
    }
}

// Exclusive scan of nb counts in place (one workgroup of 1024 threads, each
// owning a contiguous chunk); the total goes to counts[nb].
__global__ __launch_bounds__(1024) void k_scan_counts(int32_t *__restrict__ counts, int64_t nb)
{
    __shared__ int64_t part[1024];
    const int tid = threadIdx.x;
    const int64_t chunk = (nb + 1023) / 1024;
    const int64_t lo = tid * chunk, hi = lo + chunk < nb ? lo + chunk : nb;
    int64_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += counts[i];
    part[tid] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int64_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int64_t run = tid ? part[tid - 1] : 0;
    for (int64_t i = lo; i < hi; ++i) {
        const int32_t v = counts[i];
        counts[i] = (int32_t)run;
        run += v;
    }
    if (tid == 1023) counts[nb] = (int32_t)part[1023];
}

struct FirstHit {
    const float *S, *E, *t, *point;
    const int32_t *tri;
    float *dist;       // may be null
    int32_t *tri_out;  // may be null
    float *point_out;  // may be null
};

__global__ __launch_bounds__(kCThreads) void k_compact_scatter(Select sel, int64_t n,
                                                               const int32_t *__restrict__ offs,
                                                               int32_t *__restrict__ ids, FirstHit fh)
{
    __shared__ int32_t wcnt[kCItems][kCThreads / 64];
    const int64_t base = (int64_t)blockIdx.x * kCBlock;
    const int wave = threadIdx.x >> 6;
    bool f[kCItems];
    uint32_t below[kCItems];
    const uint64_t lt = threadIdx.x & 63 ? (~0ull >> (64 - (threadIdx.x & 63))) : 0ull;
#pragma unroll
    for (int r = 0; r < kCItems; ++r) {
        const int64_t i = base + r * kCThreads + threadIdx.x;
        f[r] = i < n && sel(i);
        const uint64_t m = __ballot(f[r]);
        below[r] = (uint32_t)__popcll(m & lt);
        if (__lane_id() == 0) wcnt[r][wave] = (int32_t)__popcll(m);
    }
    __syncthreads();
    // order inside the block: round r, then wave, then lane (= segment order)
#pragma unroll
    for (int r = 0; r < kCItems; ++r) {
        if (!f[r]) continue;
        int32_t k = offs[blockIdx.x];
        for (int q = 0; q < r; ++q)
            for (int w = 0; w < kCThreads / 64; ++w) k += wcnt[q][w];
        for (int w = 0; w < wave; ++w) k += wcnt[r][w];
        k += (int32_t)below[r];
        const int64_t i = base + r * kCThreads + threadIdx.x;
        ids[k] = (int32_t)i;
        if (fh.dist) {
            const float dx = fh.E[3 * i] - fh.S[3 * i], dy = fh.E[3 * i + 1] - fh.S[3 * i + 1];
            const float dz = fh.E[3 * i + 2] - fh.S[3 * i + 2];
            fh.dist[k] = fh.t[i] * sqrtf(dx * dx + dy * dy + dz * dz);
        }
        if (fh.tri_out) fh.tri_out[k] = fh.tri[i];
        if (fh.point_out) {
            fh.point_out[3 * k] = fh.point[3 * i];
            fh.point_out[3 * k + 1] = fh.point[3 * i + 1];
            fh.point_out[3 * k + 2] = fh.point[3 * i + 2];
        }
    }
}

}  // namespace

hipError_t launch_compact(rsi_bvh *h, const uint8_t *hit, const float *S, const float *E, const int32_t *tri,
                          const float *t, const float *point, int64_t n, int32_t *ids, float *dist,
                          int32_t *tri_out, float *point_out, int64_t *n_out, hipStream_t s)
{
    *n_out = 0;
    if (n == 0) return hipSuccess;
    const int64_t nb = (n + kCBlock - 1) / kCBlock;
    hipError_t e = hipSuccess;
    if (h->compact_cap < nb + 1) {
        if (h->compact_counts) (void)hipFree(h->compact_counts);
        h->compact_counts = nullptr;
        h->compact_cap = 0;
        e = hipMalloc(reinterpret_cast<void **>(&h->compact_counts), sizeof(int32_t) * (size_t)(nb + 1));
        if (e != hipSuccess) return e;
        h->compact_cap = nb + 1;
    }
    const Select sel = {hit, hit ? nullptr : tri};
    hipLaunchKernelGGL(k_block_counts, dim3((unsigned)nb), dim3(kCThreads), 0, s, sel, n, h->compact_counts);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, s, h->compact_counts, nb);
    const FirstHit fh = {S, E, t, point, tri, dist, tri_out, point_out};
    hipLaunchKernelGGL(k_compact_scatter, dim3((unsigned)nb), dim3(kCThreads), 0, s, sel, n, h->compact_counts,
                       ids, fh);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int32_t total = 0;
    e = hipMemcpyAsync(&total, h->compact_counts + nb, sizeof(int32_t), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    *n_out = total;
    return e;
}

}  // namespace rsi
