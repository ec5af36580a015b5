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
//   k_lbvh_*     agglomerative single-pass construction over the sorted
//                keys (Apetrei's scheme, as the paper follows): every leaf
//                climbs; at each step the node joins the neighbour across the
//                split whose key distance is smaller, writes its box and
//                reference into its parent, and the parent's arrival counter
//                lets only the second child continue -- so the parent's box
//                is formed exactly once, from both children.  Ranges with at
//                most `leaf_size` triangles become leaves.  The climb runs in
//                two passes: subtrees inside a block of 256 sorted leaves
//                finish in LDS (k_lbvh_local), the few that cross block
//                boundaries finish with device-scope counters
//                (k_lbvh_global), so only those pay for cross-XCD ordering.
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

// State of one climbing node: its box, leaf range [l, r], reference and
// height (internal levels below it).
struct Climb {
    float box[6];
    int32_t l, r, ref, h;
};

// The neighbour to join: across the split with the smaller key distance.
// Returns the parent index (= that split position) and our side in it
// (0: left child, 1: right child).
__device__ inline int32_t choose_parent(const uint64_t *__restrict__ keys, int32_t n, int32_t l, int32_t r,
                                        int &side)
{
    if (l == 0 || (r != n - 1 && dist_less(keys, r, l - 1))) {
        side = 0;
        return r;
    }
    side = 1;
    return l - 1;
}

__device__ inline void merge(Climb &c, const float *g, int32_t other_bound, int32_t other_h, int side,
                             int32_t parent, int32_t leaf_size)
{
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        c.box[k] = fminf(c.box[k], g[k]);
        c.box[3 + k] = fmaxf(c.box[3 + k], g[3 + k]);
    }
    if (side == 0) c.r = other_bound;
    else c.l = other_bound;
    c.h = 1 + (c.h > other_h ? c.h : other_h);
    c.ref = (c.r - c.l + 1 <= leaf_size) ? leaf_ref(c.l, c.r - c.l + 1) : parent;
    if (c.ref < 0) c.h = 0;  // a collapsed range is a leaf
}

// Entry node n-1: the root as its left child (the paper keeps the root as the
// left child of its last internal node record), an empty far box on the right.
__device__ inline void write_entry(Node *__restrict__ nodes, int32_t n, const Climb &c, int32_t *scalars)
{
    Node *e = nodes + (n - 1);
    write_child(e, 0, c.box, c.ref);
    const float far[6] = {FLT_MAX, FLT_MAX, FLT_MAX, FLT_MAX, FLT_MAX, FLT_MAX};
    write_child(e, 1, far, leaf_ref(0, 1));
    e->aux[0] = 0;
    e->aux[1] = n - 1;
    scalars[kHeight] = c.h;
    scalars[kRootRef] = c.ref;
}

constexpr int kLocal = 256;   // leaves per workgroup in the local pass
constexpr int kClimbWords = 11;

// Local pass: each workgroup owns kLocal consecutive sorted leaves.  A node
// whose leaf range lies inside that block has its whole subtree inside it,
// so these subtrees are completed here with the arrival counters and child
// records in LDS.  A climb that reaches a split outside the block (its parent
// range crosses the block boundary) is saved for the global pass.
__global__ __launch_bounds__(kLocal) void k_lbvh_local(int32_t n, const uint64_t *__restrict__ keys,
                                                       const uint32_t *__restrict__ order,
                                                       const float *__restrict__ V, int64_t n_v,
                                                       const int32_t *__restrict__ T, Node *__restrict__ nodes,
                                                       Tri *__restrict__ tris, int32_t *__restrict__ arrive,
                                                       int32_t *__restrict__ heights, int32_t leaf_size,
                                                       int32_t *__restrict__ scalars, int32_t *__restrict__ climb)
{
    __shared__ int32_t lflag[kLocal];
    __shared__ float lbox[kLocal][12];
    __shared__ int32_t lref[kLocal][2];
    __shared__ int32_t lbound[kLocal][2];
    __shared__ int32_t lh[kLocal][2];
    const int tid = threadIdx.x;
    const int32_t B0 = (int32_t)blockIdx.x * kLocal;
    const int32_t B1 = (B0 + kLocal < n ? B0 + kLocal : n) - 1;  // last leaf of this block
    lflag[tid] = 0;
    __syncthreads();

    const int32_t i = B0 + tid;
    bool active = i < n;
    Climb c;
    if (active) {
        // leaf i: pack the triangle in sorted order and form its box
        int32_t id = (int32_t)order[i];
        if (id < 0 || id >= n) {  // cannot happen after a correct sort; never read outside T
            atomicOr(&scalars[kBadIndex], 2);
            id = 0;
        }
        int32_t a = T[3 * id], b = T[3 * id + 1], d = T[3 * id + 2];
        // an out-of-range index is reported by k_centroids; read vertex 0
        // instead so that no access leaves the vertex array
        if (a < 0 || a >= n_v) a = 0;
        if (b < 0 || b >= n_v) b = 0;
        if (d < 0 || d >= n_v) d = 0;
        const float v0x = V[3 * a], v0y = V[3 * a + 1], v0z = V[3 * a + 2];
        const float v1x = V[3 * b], v1y = V[3 * b + 1], v1z = V[3 * b + 2];
        const float v2x = V[3 * d], v2y = V[3 * d + 1], v2z = V[3 * d + 2];
        Tri tr;
        tr.a = make_float4(v0x, v0y, v0z, v1x);
        tr.b = make_float4(v1y, v1z, v2x, v2y);
        tr.c = make_float4(v2z, __int_as_float(id), 0.0f, 0.0f);
        tris[i] = tr;
        c.box[0] = fminf(v0x, fminf(v1x, v2x));
        c.box[1] = fminf(v0y, fminf(v1y, v2y));
        c.box[2] = fminf(v0z, fminf(v1z, v2z));
        c.box[3] = fmaxf(v0x, fmaxf(v1x, v2x));
        c.box[4] = fmaxf(v0y, fmaxf(v1y, v2y));
        c.box[5] = fmaxf(v0z, fmaxf(v1z, v2z));
        c.l = c.r = i;
        c.ref = leaf_ref(i, 1);
        c.h = 0;
        climb[kClimbWords * (int64_t)i] = 0;  // no saved climb for this leaf unless set below
    }
    // a climb inside the block takes fewer than kLocal steps
    for (int step = 0; active; ++step) {
        if (c.l == 0 && c.r == n - 1) {  // the whole tree fits in this block
            write_entry(nodes, n, c, scalars);
            break;
        }
        int side;
        const int32_t parent = choose_parent(keys, n, c.l, c.r, side);
        if (parent < B0 || parent >= B1 || step >= kLocal) {
            // the parent's range crosses the block boundary: hand over
            int32_t *st = climb + kClimbWords * (int64_t)i;
            st[0] = 1;
            st[1] = c.l;
            st[2] = c.r;
            st[3] = c.ref;
            st[4] = c.h;
#pragma unroll
            for (int k = 0; k < 6; ++k) st[5 + k] = __float_as_int(c.box[k]);
            break;
        }
        const int slot = parent - B0;
#pragma unroll
        for (int k = 0; k < 6; ++k) lbox[slot][6 * side + k] = c.box[k];
        lref[slot][side] = c.ref;
        lbound[slot][side] = side ? c.r : c.l;
        lh[slot][side] = c.h;
        const int32_t prev =
            __hip_atomic_fetch_add(&lflag[slot], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (prev == 0) break;  // the sibling finishes this parent
        const int other = 1 - side;
        merge(c, &lbox[slot][6 * other], lbound[slot][other], lh[slot][other], side, parent, leaf_size);
    }
    __syncthreads();
    // publish the block's internal node records (splits B0 .. B1-1)
    if (tid < B1 - B0 && lflag[tid] > 0) {
        const int32_t p = B0 + tid;
        Node *q = nodes + p;
#pragma unroll
        for (int k = 0; k < 12; ++k) q->f[k] = lbox[tid][k];
        q->ref[0] = lref[tid][0];
        q->ref[1] = lref[tid][1];
        q->aux[0] = lbound[tid][0];
        q->aux[1] = lbound[tid][1];
        heights[2 * p] = lh[tid][0];
        heights[2 * p + 1] = lh[tid][1];
        arrive[p] = lflag[tid];
    }
}

// Global pass: continue the climbs saved by the local pass.  Their parents
// are shared between workgroups, so the arrival counter works at device
// scope (the XCDs have separate L2 caches: release our writes, acquire the
// sibling's).  Only the few subtrees that cross block boundaries remain.
__global__ __launch_bounds__(256) void k_lbvh_global(int32_t n, const uint64_t *__restrict__ keys,
                                                     Node *__restrict__ nodes, int32_t *__restrict__ arrive,
                                                     int32_t *__restrict__ heights, int32_t leaf_size,
                                                     int32_t *__restrict__ scalars,
                                                     const int32_t *__restrict__ climb)
{
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    const int32_t *st = climb + kClimbWords * (int64_t)i;
    if (st[0] == 0) return;
    Climb c;
    c.l = st[1];
    c.r = st[2];
    c.ref = st[3];
    c.h = st[4];
#pragma unroll
    for (int k = 0; k < 6; ++k) c.box[k] = __int_as_float(st[5 + k]);
    // every step strictly widens [l, r], so at most n - 1 steps are needed
    for (int32_t step = 0; !(c.l == 0 && c.r == n - 1); ++step) {
        if (step >= n || c.l < 0 || c.r > n - 1 || c.l > c.r) {  // inconsistent: report, do not wander
            atomicOr(&scalars[kBadIndex], 2);
            return;
        }
        int side;
        const int32_t parent = choose_parent(keys, n, c.l, c.r, side);
        Node *p = nodes + parent;
        write_child(p, side, c.box, c.ref);
        p->aux[side] = side ? c.r : c.l;
        heights[2 * parent + side] = c.h;
        const int32_t prev =
            __hip_atomic_fetch_add(&arrive[parent], 1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == 0) return;  // the sibling finishes this parent
        const int other = 1 - side;
        merge(c, p->f + 6 * other, p->aux[other], heights[2 * parent + other], side, parent, leaf_size);
    }
    write_entry(nodes, n, c, scalars);
}

}  // namespace

static hipError_t run_hierarchy(rsi_bvh *h, const float *V, hipStream_t s)
{
    const int32_t n = (int32_t)h->n_t;
    const unsigned nb = (unsigned)((n + kLocal - 1) / kLocal);
    hipLaunchKernelGGL(k_lbvh_local, dim3(nb), dim3(kLocal), 0, s, n, h->keys, h->order, V, h->n_v, h->T,
                       h->nodes, h->tris, h->arrive, h->heights, h->leaf_size, h->scalars, h->climb);
    if (nb > 1)
        hipLaunchKernelGGL(k_lbvh_global, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, h->keys,
                           h->nodes, h->arrive, h->heights, h->leaf_size, h->scalars, h->climb);
    return hipGetLastError();
}

static hipError_t run_lbvh(rsi_bvh *h, const float *V, hipStream_t s)
{
    const int32_t n = (int32_t)h->n_t;
    const int blk = 256;
    hipLaunchKernelGGL(k_init, dim3((unsigned)((n + blk - 1) / blk)), dim3(blk), 0, s, h->scalars, h->arrive,
                       (int64_t)n);
    return run_hierarchy(h, V, s);
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
    return run_hierarchy(h, V, s);
}

hipError_t launch_refit(rsi_bvh *h, const float *V, hipStream_t s)
{
    if (h->n_t == 0) return hipSuccess;
    return run_lbvh(h, V, s);
}

}  // namespace rsi
