// build.hip -- linear BVH construction on the GPU (paper Section 2 and
// Section 3.1; the steps are those timed in the paper's Table 2).
//
//   k_init       reset the build scalars and the per-node arrival counters
//   k_centroids  c_j = (v_a + v_b + v_c) / 3 per triangle, index validation,
//                and the support interval of the centroids (block min/max
//                in LDS, then one ordered-int atomic per block and axis)
//   k_morton     quantise c_j to 2^21 levels per axis inside that interval
//                and interleave the three 21-bit integers into a 63-bit key
//   (sort.hip)   stable radix sort of (key, triangle id)
//   k_lbvh       agglomerative single-pass construction over the sorted
//                keys (Apetrei's scheme, as the paper follows): every leaf
//                climbs; at each step the node joins the neighbour across the
//                split whose key distance is smaller, writes its box and
//                reference into its parent, and the parent's arrival counter
//                lets only the second child continue -- so the parent's box
//                is formed exactly once, from both children.  Ranges with at
//                most `leaf_size` triangles become leaves.
//
// The entry node is record n_t - 1 (unused by the n_t - 1 internal nodes
// 0 .. n_t - 2): its left child is the root and its right child an empty far
// box, which mirrors the paper's convention of keeping the root as the left
// child of internalNodes[N_t - 1] and also covers n_t == 1.
#include <hip/hip_runtime.h>
#include <float.h>
#include <stdint.h>

#include "rsi_host.h"

namespace rsi {
namespace {

__global__ void k_init(int32_t *__restrict__ scalars, int32_t *__restrict__ arrive, int64_t n_arrive)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        for (int k = 0; k < 3; ++k) {
            scalars[kBoundLo + k] = float_to_ordered(FLT_MAX);
            scalars[kBoundHi + k] = float_to_ordered(-FLT_MAX);
        }
        scalars[kBadIndex] = 0;
        scalars[kHeight] = 0;
        scalars[kRootRef] = 0;
    }
    if (i < n_arrive) arrive[i] = 0;
}

__global__ __launch_bounds__(256) void k_centroids(const float *__restrict__ V, int64_t n_v,
                                                   const int32_t *__restrict__ T, int64_t n_t,
                                                   float *__restrict__ cent, int32_t *__restrict__ scalars)
{
    __shared__ int32_t lo[3], hi[3];
    const int tid = threadIdx.x;
    if (tid < 3) {
        lo[tid] = float_to_ordered(FLT_MAX);
        hi[tid] = float_to_ordered(-FLT_MAX);
    }
    __syncthreads();
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + tid;
    if (j < n_t) {
        int32_t a = T[3 * j], b = T[3 * j + 1], c = T[3 * j + 2];
        bool ok = a >= 0 && a < n_v && b >= 0 && b < n_v && c >= 0 && c < n_v;
        if (!ok) {
            atomicOr(&scalars[kBadIndex], 1);
            a = b = c = 0;
        }
        float cx = (V[3 * a] + V[3 * b] + V[3 * c]) * (1.0f / 3.0f);
        float cy = (V[3 * a + 1] + V[3 * b + 1] + V[3 * c + 1]) * (1.0f / 3.0f);
        float cz = (V[3 * a + 2] + V[3 * b + 2] + V[3 * c + 2]) * (1.0f / 3.0f);
        cent[j] = cx;
        cent[n_t + j] = cy;
        cent[2 * n_t + j] = cz;
        atomicMin(&lo[0], float_to_ordered(cx));
        atomicMin(&lo[1], float_to_ordered(cy));
        atomicMin(&lo[2], float_to_ordered(cz));
        atomicMax(&hi[0], float_to_ordered(cx));
        atomicMax(&hi[1], float_to_ordered(cy));
        atomicMax(&hi[2], float_to_ordered(cz));
    }
    __syncthreads();
    if (tid < 3) {
        atomicMin(&scalars[kBoundLo + tid], lo[tid]);
        atomicMax(&scalars[kBoundHi + tid], hi[tid]);
    }
}

// Spread the low 21 bits of x so that bit k moves to bit 3k.
__device__ inline uint64_t spread3(uint32_t v)
{
    uint64_t x = v & 0x1FFFFFu;
    x = (x | (x << 32)) & 0x001F00000000FFFFull;
    x = (x | (x << 16)) & 0x001F0000FF0000FFull;
    x = (x | (x << 8)) & 0x100F00F00F00F00Full;
    x = (x | (x << 4)) & 0x10C30C30C30C30C3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ inline uint32_t quantise21(float c, float lo, float ext)
{
    // floor((c - lo) / ext * 2^21), clamped to [0, 2^21 - 1]; a flat axis maps to 0
    if (!(ext > 0.0f)) return 0u;
    float q = (c - lo) / ext * 2097152.0f;
    q = fminf(fmaxf(q, 0.0f), 2097151.0f);
    return (uint32_t)q;
}

__global__ void k_morton(const float *__restrict__ cent, int64_t n_t, const int32_t *__restrict__ scalars,
                         uint64_t *__restrict__ keys, uint32_t *__restrict__ ids)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_t) return;
    const float lx = ordered_to_float(scalars[kBoundLo]), ly = ordered_to_float(scalars[kBoundLo + 1]),
                lz = ordered_to_float(scalars[kBoundLo + 2]);
    const float hx = ordered_to_float(scalars[kBoundHi]), hy = ordered_to_float(scalars[kBoundHi + 1]),
                hz = ordered_to_float(scalars[kBoundHi + 2]);
    const uint32_t qx = quantise21(cent[j], lx, hx - lx);
    const uint32_t qy = quantise21(cent[n_t + j], ly, hy - ly);
    const uint32_t qz = quantise21(cent[2 * n_t + j], lz, hz - lz);
    keys[j] = (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
    ids[j] = (uint32_t)j;
}

// Key distance between sorted neighbours k and k+1, compared
// lexicographically as (key xor, index xor): equal keys are split by index,
// so duplicate codes still form a valid radix tree.
__device__ inline bool dist_less(const uint64_t *__restrict__ keys, int a, int b)
{
    const uint64_t xa = keys[a] ^ keys[a + 1];
    const uint64_t xb = keys[b] ^ keys[b + 1];
    if (xa != xb) return xa < xb;
    return (uint32_t)(a ^ (a + 1)) < (uint32_t)(b ^ (b + 1));
}

__device__ inline void write_child(Node *__restrict__ p, int side, const float bx[6], int32_t ref)
{
    float *f = p->f + 6 * side;
#pragma unroll
    for (int k = 0; k < 6; ++k) f[k] = bx[k];
    p->ref[side] = ref;
}

__global__ __launch_bounds__(256) void k_lbvh(int32_t n, const uint64_t *__restrict__ keys,
                                              const uint32_t *__restrict__ order, const float *__restrict__ V,
                                              int64_t n_v, const int32_t *__restrict__ T, Node *__restrict__ nodes,
                                              Tri *__restrict__ tris, int32_t *__restrict__ arrive,
                                              int32_t *__restrict__ heights, int32_t leaf_size,
                                              int32_t *__restrict__ scalars)
{
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;

    // leaf i: pack the triangle in sorted order and form its box
    int32_t id = (int32_t)order[i];
    if (id < 0 || id >= n) {  // cannot happen after a correct sort; never read outside T
        atomicOr(&scalars[kBadIndex], 2);
        id = 0;
    }
    int32_t a = T[3 * id], b = T[3 * id + 1], c = T[3 * id + 2];
    // an out-of-range index is reported by k_centroids; read vertex 0 instead
    // so that no access leaves the vertex array
    if (a < 0 || a >= n_v) a = 0;
    if (b < 0 || b >= n_v) b = 0;
    if (c < 0 || c >= n_v) c = 0;
    const float v0x = V[3 * a], v0y = V[3 * a + 1], v0z = V[3 * a + 2];
    const float v1x = V[3 * b], v1y = V[3 * b + 1], v1z = V[3 * b + 2];
    const float v2x = V[3 * c], v2y = V[3 * c + 1], v2z = V[3 * c + 2];
    Tri tr;
    tr.a = make_float4(v0x, v0y, v0z, v1x);
    tr.b = make_float4(v1y, v1z, v2x, v2y);
    tr.c = make_float4(v2z, __int_as_float(id), 0.0f, 0.0f);
    tris[i] = tr;

    float box[6] = {fminf(v0x, fminf(v1x, v2x)), fminf(v0y, fminf(v1y, v2y)), fminf(v0z, fminf(v1z, v2z)),
                    fmaxf(v0x, fmaxf(v1x, v2x)), fmaxf(v0y, fmaxf(v1y, v2y)), fmaxf(v0z, fmaxf(v1z, v2z))};
    int32_t l = i, r = i;
    int32_t ref = leaf_ref(i, 1);
    int32_t h = 0;

    // every step strictly widens [l, r], so at most n - 1 steps are needed
    for (int32_t step = 0; !(l == 0 && r == n - 1); ++step) {
        if (step >= n || l < 0 || r > n - 1 || l > r) {  // inconsistent state: report, do not wander
            atomicOr(&scalars[kBadIndex], 2);
            return;
        }
        int32_t parent;
        int side;  // 0: this node is the parent's left child, 1: right child
        if (l == 0 || (r != n - 1 && dist_less(keys, r, l - 1))) {
            parent = r;
            side = 0;
        } else {
            parent = l - 1;
            side = 1;
        }
        Node *p = nodes + parent;
        write_child(p, side, box, ref);
        p->aux[side] = side ? r : l;
        heights[2 * parent + side] = h;
        // release our writes / acquire the sibling's, at device scope: the
        // eight XCDs have separate L2s, so both halves are needed
        const int32_t prev =
            __hip_atomic_fetch_add(&arrive[parent], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == 0) return;  // the sibling finishes this parent
        const int other = 1 - side;
        if (side == 0) r = p->aux[1];
        else l = p->aux[0];
        const float *g = p->f + 6 * other;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            box[k] = fminf(box[k], g[k]);
            box[3 + k] = fmaxf(box[3 + k], g[3 + k]);
        }
        const int32_t ho = heights[2 * parent + other];
        h = 1 + (h > ho ? h : ho);
        ref = (r - l + 1 <= leaf_size) ? leaf_ref(l, r - l + 1) : parent;
        if (ref < 0) h = 0;  // a collapsed range is a leaf
    }
    // only the thread that completed the root gets here (or the single leaf)
    Node *e = nodes + (n - 1);
    write_child(e, 0, box, ref);
    const float far[6] = {FLT_MAX, FLT_MAX, FLT_MAX, FLT_MAX, FLT_MAX, FLT_MAX};
    write_child(e, 1, far, leaf_ref(0, 1));
    e->aux[0] = 0;
    e->aux[1] = n - 1;
    scalars[kHeight] = h;
    scalars[kRootRef] = ref;
}

}  // namespace

static hipError_t run_lbvh(rsi_bvh *h, const float *V, hipStream_t s)
{
    const int32_t n = (int32_t)h->n_t;
    const int blk = 256;
    hipLaunchKernelGGL(k_init, dim3((unsigned)((n + blk - 1) / blk)), dim3(blk), 0, s, h->scalars, h->arrive,
                       (int64_t)n);
    hipLaunchKernelGGL(k_lbvh, dim3((unsigned)((n + blk - 1) / blk)), dim3(blk), 0, s, n, h->keys, h->order, V,
                       h->n_v, h->T, h->nodes, h->tris, h->arrive, h->heights, h->leaf_size, h->scalars);
    return hipGetLastError();
}

hipError_t launch_build(rsi_bvh *h, const float *V, hipStream_t s)
{
    const int64_t n = h->n_t;
    if (n == 0) return hipSuccess;
    const int blk = 256;
    const unsigned grid = (unsigned)((n + blk - 1) / blk);
    hipLaunchKernelGGL(k_init, dim3(grid), dim3(blk), 0, s, h->scalars, h->arrive, n);
    hipLaunchKernelGGL(k_centroids, dim3(grid), dim3(blk), 0, s, V, h->n_v, h->T, n, h->cent, h->scalars);
    hipLaunchKernelGGL(k_morton, dim3(grid), dim3(blk), 0, s, h->cent, n, h->scalars, h->keys, h->order);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = radix_sort_pairs(h->keys, h->order, n, 63, h->sort, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_lbvh, dim3(grid), dim3(blk), 0, s, (int32_t)n, h->keys, h->order, V, h->n_v, h->T, h->nodes,
                       h->tris, h->arrive, h->heights, h->leaf_size, h->scalars);
    return hipGetLastError();
}

hipError_t launch_refit(rsi_bvh *h, const float *V, hipStream_t s)
{
    if (h->n_t == 0) return hipSuccess;
    return run_lbvh(h, V, s);
}

}  // namespace rsi
