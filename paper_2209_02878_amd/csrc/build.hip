// build.hip -- linear BVH construction on the GPU (paper Section 2 and
// Section 3.1; the steps are those timed in the paper's Table 2), for one
// mesh or for a batch of meshes in the same launches.
//
// All meshes of a handle share concatenated arrays: mesh m owns triangles,
// sorted leaves and node records [off[m], off[m+1]).  A single mesh is the
// case M = 1.
//
//   k_gather     (batches) copy every mesh's vertices and triangles into the
//                concatenated arrays, offsetting the vertex indices
//   k_init       reset per-mesh bounds, heights, roots and arrival counters
//   k_centroids  c_j = (v_a + v_b + v_c) / 3 per triangle, index validation,
//                and the support interval of each mesh's centroids (block
//                min/max in LDS, then one ordered-int atomic per block, mesh
//                and axis)
//   k_morton     quantise c_j to 2^21 levels per axis inside its mesh's
//                interval and interleave the three 21-bit integers into a
//                63-bit key
//   (sort.hip)   stable radix sort of (key, triangle id); with M > 1 a final
//                stable pass on the mesh id groups each mesh's leaves again
//   k_lbvh_*     agglomerative single-pass construction over the sorted
//                keys (Apetrei's scheme, as the paper follows): every leaf
//                climbs; at each step the node joins the neighbour across the
//                split whose key distance is smaller, writes its box and
//                reference into its parent, and the parent's arrival counter
//                lets only the second child continue -- so the parent's box
//                is formed exactly once, from both children.  Ranges with at
//                most `leaf_size` triangles become leaves.  The climb runs in
//                two passes: subtrees inside a block of 2048 sorted leaves
//                finish in LDS (k_lbvh_local), the few that cross block
//                boundaries finish in k_lbvh_global, which exchanges the
//                climb data through memory past the per-XCD caches, so only
//                those pay for cross-XCD ordering.
//
// The entry node of mesh m is its last record off[m+1] - 1 (unused by its
// n - 1 internal nodes): its left child is the root and its right child an
// empty far box, which mirrors the paper's convention of keeping the root as
// the left child of internalNodes[N_t - 1] and also covers n = 1.
#include <hip/hip_runtime.h>
#include <float.h>
#include <stdint.h>

#include "rsi_host.h"

namespace rsi {
namespace {

struct BuildArgs {
    int32_t M;
    const int64_t *off;    // [M+1] triangle offsets
    const float *V;        // vertices, global indexing
    int64_t n_v;
    const int32_t *T;      // triangles with global vertex indices
    int64_t n_t;
    float *cent;
    uint64_t *keys;
    uint32_t *order;
    int32_t *rank;
    Node *nodes;
    Tri *tris;
    int32_t *arrive;
    int32_t *heights;
    int32_t *climb;
    uint8_t *prefix;       // [n_t] common-prefix length at sorted split k
    int32_t *bounds;       // [6M] ordered-int centroid bounds per mesh
    int32_t *mesh_height;  // [M]
    int32_t *mesh_root;    // [M]
    int32_t *scalars;
    int32_t leaf_size;
};

__global__ void k_gather(int32_t M, const float *const *__restrict__ Vp, const int32_t *const *__restrict__ Tp,
                         const int64_t *__restrict__ voff, const int64_t *__restrict__ toff, float *__restrict__ V,
                         int32_t *__restrict__ T, int32_t *__restrict__ scalars)
{
    const int64_t nv = voff[M], nt = toff[M];
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nv + nt; k += stride) {
        if (k < nv) {
            const int32_t m = mesh_of(voff, M, k);
            const int64_t loc = k - voff[m];
            V[3 * k] = Vp[m][3 * loc];
            V[3 * k + 1] = Vp[m][3 * loc + 1];
            V[3 * k + 2] = Vp[m][3 * loc + 2];
        } else {
            const int64_t j = k - nv;
            const int32_t m = mesh_of(toff, M, j);
            const int64_t loc = j - toff[m];
            const int64_t nvm = voff[m + 1] - voff[m];
            for (int c = 0; c < 3; ++c) {
                int32_t x = Tp[m][3 * loc + c];
                if (x < 0 || x >= nvm) {  // reported; a valid index keeps later reads inside V
                    atomicOr(&scalars[kBadGather], 1);
                    x = 0;
                }
                T[3 * j + c] = (int32_t)(x + voff[m]);
            }
        }
    }
}

__global__ void k_clear_gather_flag(int32_t *scalars) { scalars[kBadGather] = 0; }

__global__ void k_init(BuildArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < a.M) {
        for (int k = 0; k < 3; ++k) {
            a.bounds[6 * i + k] = float_to_ordered(FLT_MAX);
            a.bounds[6 * i + 3 + k] = float_to_ordered(-FLT_MAX);
        }
        a.mesh_height[i] = 0;
        a.mesh_root[i] = 0;
    }
    if (i == 0) a.scalars[kBadIndex] = 0;
    if (i < a.n_t) a.arrive[i] = 0;
}

constexpr int kCentBlock = 256;
constexpr int kCentMeshes = 4;  // meshes per block reduced in LDS; the rest go straight to global

__global__ __launch_bounds__(kCentBlock) void k_centroids(BuildArgs a)
{
    __shared__ int32_t lb[kCentMeshes][6];
    const int tid = threadIdx.x;
    if (tid < kCentMeshes * 6) {
        lb[tid / 6][tid % 6] = float_to_ordered((tid % 6) < 3 ? FLT_MAX : -FLT_MAX);
    }
    const int64_t j0 = (int64_t)blockIdx.x * kCentBlock;
    const int32_t m0 = mesh_of(a.off, a.M, j0 < a.n_t ? j0 : a.n_t - 1);
    __syncthreads();
    const int64_t j = j0 + tid;
    if (j < a.n_t) {
        int32_t va = a.T[3 * j], vb = a.T[3 * j + 1], vc = a.T[3 * j + 2];
        const bool ok = va >= 0 && va < a.n_v && vb >= 0 && vb < a.n_v && vc >= 0 && vc < a.n_v;
        if (!ok) {
            atomicOr(&a.scalars[kBadIndex], 1);
            va = vb = vc = 0;
        }
        const float cx = (a.V[3 * va] + a.V[3 * vb] + a.V[3 * vc]) * (1.0f / 3.0f);
        const float cy = (a.V[3 * va + 1] + a.V[3 * vb + 1] + a.V[3 * vc + 1]) * (1.0f / 3.0f);
        const float cz = (a.V[3 * va + 2] + a.V[3 * vb + 2] + a.V[3 * vc + 2]) * (1.0f / 3.0f);
        a.cent[j] = cx;
        a.cent[a.n_t + j] = cy;
        a.cent[2 * a.n_t + j] = cz;
        const int32_t m = mesh_of(a.off, a.M, j);
        const int32_t q[3] = {float_to_ordered(cx), float_to_ordered(cy), float_to_ordered(cz)};
        if (m - m0 < kCentMeshes) {
            int32_t *l = lb[m - m0];
            for (int k = 0; k < 3; ++k) {
                atomicMin(&l[k], q[k]);
                atomicMax(&l[3 + k], q[k]);
            }
        } else {
            for (int k = 0; k < 3; ++k) {
                atomicMin(&a.bounds[6 * m + k], q[k]);
                atomicMax(&a.bounds[6 * m + 3 + k], q[k]);
            }
        }
    }
    __syncthreads();
    if (tid < kCentMeshes * 6) {
        const int32_t m = m0 + tid / 6, k = tid % 6;
        const int32_t v = lb[tid / 6][k];
        if (m < a.M && v != float_to_ordered(k < 3 ? FLT_MAX : -FLT_MAX)) {
            if (k < 3) atomicMin(&a.bounds[6 * m + k], v);
            else atomicMax(&a.bounds[6 * m + k], v);
        }
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

__global__ void k_morton(BuildArgs a)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= a.n_t) return;
    const int32_t *b = a.bounds + 6 * mesh_of(a.off, a.M, j);
    const float lx = ordered_to_float(b[0]), ly = ordered_to_float(b[1]), lz = ordered_to_float(b[2]);
    const float hx = ordered_to_float(b[3]), hy = ordered_to_float(b[4]), hz = ordered_to_float(b[5]);
    const uint32_t qx = quantise21(a.cent[j], lx, hx - lx);
    const uint32_t qy = quantise21(a.cent[a.n_t + j], ly, hy - ly);
    const uint32_t qz = quantise21(a.cent[2 * a.n_t + j], lz, hz - lz);
    a.keys[j] = (spread3(qx) << 2) | (spread3(qy) << 1) | spread3(qz);
    a.order[j] = (uint32_t)j;
}

// Common-prefix length of the augmented keys (key, index) of the sorted
// neighbours k and k+1: the leading equal key bits while the keys differ,
// else 64 plus the leading equal index bits, so equal keys are split by index
// and duplicate codes still form a valid radix tree.  A longer prefix is a
// smaller key distance.
__device__ inline uint8_t split_prefix(const uint64_t *__restrict__ keys, int32_t k)
{
    const uint64_t x = keys[k] ^ keys[k + 1];
    if (x) return (uint8_t)__clzll((long long)x);
    return (uint8_t)(64 + __clz((int)((uint32_t)k ^ (uint32_t)(k + 1))));
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

// The neighbour to join, within the mesh's leaf range [lo, hi]: across the
// split with the longer common prefix (smaller key distance; the two splits
// around a node of the radix tree never tie).  `prefix(k)` is the prefix
// length at split k.  Returns the parent index (= that split position) and
// our side in it (0: left child, 1: right child).
template <typename Prefix>
__device__ inline int32_t choose_parent(Prefix prefix, int32_t lo, int32_t hi, int32_t l, int32_t r, int &side)
{
    if (l == lo || (r != hi && prefix(r) > prefix(l - 1))) {
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

// Entry node `hi` (the mesh's last record): the root as its left child (the
// paper keeps the root as the left child of its last internal node record),
// an empty far box on the right.
__device__ inline void write_entry(const BuildArgs &a, int32_t m, int32_t lo, int32_t hi, const Climb &c)
{
    Node *e = a.nodes + hi;
    write_child(e, 0, c.box, c.ref);
    const float far[6] = {FLT_MAX, FLT_MAX, FLT_MAX, FLT_MAX, FLT_MAX, FLT_MAX};
    write_child(e, 1, far, leaf_ref(lo, 1));
    e->aux[0] = lo;
    e->aux[1] = hi;
    a.mesh_height[m] = c.h;
    a.mesh_root[m] = c.ref;
}

constexpr int kClimbWords = 11;

// Local pass: each workgroup owns kLocal consecutive sorted leaves (2048 with
// 1024 threads, whose 152 KiB of LDS node slots fit gfx950's 160 KiB; or 512
// with 256 threads).  A node whose leaf range lies inside that block has its
// whole subtree inside it, so these subtrees are completed here with the
// arrival counters and child records in LDS.  A climb that reaches a split
// outside the block (its parent range crosses the block boundary) is saved
// for the global pass.
template <int kLocal, int kLocalThreads>
__global__ __launch_bounds__(kLocalThreads) void k_lbvh_local(BuildArgs a)
{
    constexpr int kPer = kLocal / kLocalThreads;  // leaves per thread
    __shared__ int32_t lflag[kLocal];
    __shared__ float lbox[kLocal][12];
    __shared__ int32_t lref[kLocal][2];
    __shared__ int32_t lbound[kLocal][2];
    __shared__ int32_t lh[kLocal][2];
    __shared__ uint8_t lpre[kLocal + 1];  // prefix length at split k, k = B0-1 .. B1
    const int32_t n = (int32_t)a.n_t;
    const int32_t B0 = (int32_t)blockIdx.x * kLocal;
    const int32_t B1 = (B0 + kLocal < n ? B0 + kLocal : n) - 1;  // last leaf of this block
    // split prefixes of the block (and the split before it) into LDS; each
    // split is also stored once for the global pass
    for (int t = threadIdx.x; t <= kLocal; t += kLocalThreads) {
        const int32_t k = B0 - 1 + t;
        if (k >= 0 && k <= B1 && k < n - 1) {
            const uint8_t p = split_prefix(a.keys, k);
            lpre[t] = p;
            if (t > 0) a.prefix[k] = p;
        }
        if (t < kLocal) lflag[t] = 0;
    }
    __syncthreads();
    const auto prefix = [&](int32_t k) { return (int32_t)lpre[k - B0 + 1]; };

    // leaf set-up for all of this thread's leaves first (their loads overlap)
    Climb cl[kPer];
    int32_t lo_[kPer], hi_[kPer], m_[kPer];
    bool act[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int32_t i = B0 + (int32_t)threadIdx.x + q * kLocalThreads;
        act[q] = i < n;
        m_[q] = lo_[q] = hi_[q] = 0;
        if (!act[q]) continue;
        Climb &c = cl[q];
        const int32_t m = mesh_of(a.off, a.M, i);
        const int32_t lo = (int32_t)a.off[m];
        const int32_t hi = (int32_t)a.off[m + 1] - 1;
        m_[q] = m;
        lo_[q] = lo;
        hi_[q] = hi;
        // leaf i: pack the triangle in sorted order and form its box
        int32_t id = (int32_t)a.order[i];
        if (id < lo || id > hi) {  // cannot happen after a correct sort; never read outside T
            atomicOr(&a.scalars[kBadIndex], 2);
            id = lo;
        }
        a.rank[id] = i;
        int32_t va = a.T[3 * id], vb = a.T[3 * id + 1], vd = a.T[3 * id + 2];
        // an out-of-range index is reported by k_centroids; read vertex 0
        // instead so that no access leaves the vertex array, and mark the
        // record (the adjoint skips it)
        const bool bad = va < 0 || va >= a.n_v || vb < 0 || vb >= a.n_v || vd < 0 || vd >= a.n_v;
        if (va < 0 || va >= a.n_v) va = 0;
        if (vb < 0 || vb >= a.n_v) vb = 0;
        if (vd < 0 || vd >= a.n_v) vd = 0;
        const float v0x = a.V[3 * va], v0y = a.V[3 * va + 1], v0z = a.V[3 * va + 2];
        const float v1x = a.V[3 * vb], v1y = a.V[3 * vb + 1], v1z = a.V[3 * vb + 2];
        const float v2x = a.V[3 * vd], v2y = a.V[3 * vd + 1], v2z = a.V[3 * vd + 2];
        Tri tr;
        tr.a = make_float4(v0x, v0y, v0z, v1x);
        tr.b = make_float4(v1y, v1z, v2x, v2y);
        tr.c = make_float4(v2z, __int_as_float(id - lo), 0.0f, bad ? 1.0f : 0.0f);  // id within its mesh
        a.tris[i] = tr;
        c.box[0] = fminf(v0x, fminf(v1x, v2x));
        c.box[1] = fminf(v0y, fminf(v1y, v2y));
        c.box[2] = fminf(v0z, fminf(v1z, v2z));
        c.box[3] = fmaxf(v0x, fmaxf(v1x, v2x));
        c.box[4] = fmaxf(v0y, fmaxf(v1y, v2y));
        c.box[5] = fmaxf(v0z, fmaxf(v1z, v2z));
        c.l = c.r = i;
        c.ref = leaf_ref(i, 1);
        c.h = 0;
        a.climb[kClimbWords * (int64_t)i] = 0;  // no saved climb for this leaf unless set below
    }

    // each thread climbs from its leaves one after the other; a climb that
    // arrives first at a node stops, so no thread ever waits
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
    const int32_t i = B0 + (int32_t)threadIdx.x + q * kLocalThreads;
    Climb &c = cl[q];
    const int32_t m = m_[q], lo = lo_[q], hi = hi_[q];
    // a climb inside the block takes fewer than kLocal steps
    for (int step = 0; act[q]; ++step) {
        if (c.l == lo && c.r == hi) {  // the whole mesh fits in this block
            write_entry(a, m, lo, hi, c);
            break;
        }
        int side;
        // inside the block [l, r] lies in [B0, B1], so both splits are in lpre
        const int32_t parent = choose_parent(prefix, lo, hi, c.l, c.r, side);
        if (parent < B0 || parent >= B1 || step >= kLocal) {
            // the parent's range crosses the block boundary: hand over
            int32_t *st = a.climb + kClimbWords * (int64_t)i;
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
        // A wave's LDS operations are performed in the order it issues them,
        // so the child data above is in place before the counter moves, and
        // the sibling's data read right after the counter update (before its
        // result is known; unused if we arrive first) is complete whenever
        // the counter shows that the sibling arrived.  The signal fences
        // keep the compiler from moving LDS accesses across the update; one
        // wait then covers the update and the reads.
        const int other = 1 - side;
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        const int32_t prev = __hip_atomic_fetch_add(&lflag[slot], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        float g[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) g[k] = lbox[slot][6 * other + k];
        const int32_t ob = lbound[slot][other], oh = lh[slot][other];
        // an empty statement that uses the loaded values keeps the compiler
        // from sinking the reads below the branch (it emits no instruction)
        asm volatile("" : : "v"(g[0]), "v"(g[1]), "v"(g[2]), "v"(g[3]), "v"(g[4]), "v"(g[5]), "v"(ob), "v"(oh));
        if (prev == 0) break;  // the sibling finishes this parent
        merge(c, g, ob, oh, side, parent, a.leaf_size);
    }
    }
    __syncthreads();
    // publish the block's internal node records (splits B0 .. B1-1)
    for (int tid = threadIdx.x; tid < kLocal; tid += kLocalThreads) {
    if (tid < B1 - B0 && lflag[tid] > 0) {
        const int32_t p = B0 + tid;
        Node *q = a.nodes + p;
#pragma unroll
        for (int k = 0; k < 12; ++k) q->f[k] = lbox[tid][k];
        q->ref[0] = lref[tid][0];
        q->ref[1] = lref[tid][1];
        q->aux[0] = lbound[tid][0];
        q->aux[1] = lbound[tid][1];
        a.heights[2 * p] = lh[tid][0];
        a.heights[2 * p + 1] = lh[tid][1];
        a.arrive[p] = lflag[tid];
    }
    }
}

// Global pass: continue the climbs saved by the local pass.  Their parents
// are shared between workgroups on different XCDs, whose L2 caches are not
// coherent with each other.  Release/acquire ordering at device scope would
// write back and invalidate a whole L2 at every level of every climb;
// instead the few words a sibling needs are written and read with
// system-coherent accesses (past the per-XCD caches), the writes complete
// before the arrival counter moves, and the counter is a system-coherent
// atomic.  Only the subtrees that cross block boundaries remain.
__global__ __launch_bounds__(256) void k_lbvh_global(BuildArgs a)
{
    const int32_t n = (int32_t)a.n_t;
    const int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i >= n) return;
    const int32_t *st = a.climb + kClimbWords * (int64_t)i;
    if (st[0] == 0) return;
    const int32_t m = mesh_of(a.off, a.M, i);
    const int32_t lo = (int32_t)a.off[m], hi = (int32_t)a.off[m + 1] - 1;
    Climb c;
    c.l = st[1];
    c.r = st[2];
    c.ref = st[3];
    c.h = st[4];
#pragma unroll
    for (int k = 0; k < 6; ++k) c.box[k] = __int_as_float(st[5 + k]);
    // every step strictly widens [l, r], so at most n - 1 steps are needed
    for (int32_t step = 0; !(c.l == lo && c.r == hi); ++step) {
        if (step >= n || c.l < lo || c.r > hi || c.l > c.r) {  // inconsistent: report, do not wander
            atomicOr(&a.scalars[kBadIndex], 2);
            return;
        }
        int side;
        const int32_t parent =
            choose_parent([&](int32_t k) { return a.prefix[k]; }, lo, hi, c.l, c.r, side);
        Node *p = a.nodes + parent;
        // child data with system-coherent stores (they bypass the per-XCD
        // caches), completed before the counter moves; the sibling reads
        // them back with system-coherent loads, so no cache-wide write-back
        // or invalidation is needed at any level
        for (int k = 0; k < 6; ++k)
            __hip_atomic_store(&p->f[6 * side + k], c.box[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&p->ref[side], c.ref, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&p->aux[side], side ? c.r : c.l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&a.heights[2 * parent + side], c.h, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __builtin_amdgcn_s_waitcnt(0);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        const int32_t prev = __hip_atomic_fetch_add(&a.arrive[parent], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __atomic_signal_fence(__ATOMIC_SEQ_CST);
        if (prev == 0) return;  // the sibling finishes this parent
        const int other = 1 - side;
        float g[6];
        for (int k = 0; k < 6; ++k)
            g[k] = __hip_atomic_load(&p->f[6 * other + k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        const int32_t ob = __hip_atomic_load(&p->aux[other], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        const int32_t oh = __hip_atomic_load(&a.heights[2 * parent + other], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        merge(c, g, ob, oh, side, parent, a.leaf_size);
    }
    write_entry(a, m, lo, hi, c);
}

// Four-way view: record n lists the boxes and references of n's
// grandchildren (a leaf child stands for itself), read from n's record and
// its internal children's records, quantised inside their union box.
// Every record is rewritten, including ones no traversal reaches (inside
// collapsed leaves), so references are range-checked before use.
//
// Grid step per axis: the smallest power of two 2^e with 255 * 2^e >= the
// box extent (with a 2^-40 relative margin over the FP64 extent); planes are
// placed in FP64, where the offset from the corner carries at most 2^-45
// steps of rounding error, and rounded outward with a 2^-40-step margin, so
// corner + q * step bounds the exact plane on the safe side.
__device__ inline int quant_exponent(double ext)
{
    const double x = ext * (1.0 + 0x1p-40) / 255.0;
    if (!(x > 0x1p-126)) return -126;
    int k = 0;
    const double m = frexp(x, &k);  // x = m 2^k, m in [0.5, 1)
    const int e = (m == 0.5) ? k - 1 : k;
    return e > 127 ? 127 : e;
}

// `inv_step` is 1 / step, a power of two, so the scaling is exact
__device__ inline uint32_t quant_down(double off, double inv_step)
{
    const double q = floor(off * inv_step - 0x1p-40);
    return (uint32_t)fmin(fmax(q, 0.0), 255.0);
}

__device__ inline uint32_t quant_up(double off, double inv_step)
{
    const double q = ceil(off * inv_step + 0x1p-40);
    return (uint32_t)fmin(fmax(q, 0.0), 255.0);
}

__global__ __launch_bounds__(256) void k_widen(const Node *__restrict__ nodes, int64_t n, Node4 *__restrict__ out)
{
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const Node nd = nodes[j];
    float box[4][6];
    int32_t ref[4];
    int k = 0;
    for (int side = 0; side < 2; ++side) {
        const int32_t c = nd.ref[side];
        if (c >= 0 && c < n) {
            const Node ch = nodes[c];
            for (int g = 0; g < 2; ++g) {
                for (int q = 0; q < 6; ++q) box[k][q] = ch.f[6 * g + q];
                ref[k++] = ch.ref[g];
            }
        } else {
            // the entry record's far box (all FLT_MAX) is no child: the slot
            // stays empty
            bool far = true;
            for (int q = 0; q < 6; ++q) far = far && nd.f[6 * side + q] == FLT_MAX;
            if (far) continue;
            for (int q = 0; q < 6; ++q) box[k][q] = nd.f[6 * side + q];
            ref[k++] = c < 0 ? c : leaf_ref(0, 1);
        }
    }
    // union box of the used slots
    float lo[3] = {FLT_MAX, FLT_MAX, FLT_MAX}, hi[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
    for (int s = 0; s < k; ++s)
        for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], box[s][a]);
            hi[a] = fmaxf(hi[a], box[s][3 + a]);
        }
    Node4 w;
    double inv_step[3];
    float step[3];
    for (int a = 0; a < 3; ++a) {
        const int e = quant_exponent((double)hi[a] - (double)lo[a]);
        inv_step[a] = ldexp(1.0, -e);
        step[a] = ldexpf(1.0f, e);  // a normal float for e in [-126, 127]
    }
    w.ox = lo[0];
    w.oy = lo[1];
    w.oz = lo[2];
    w.sx = step[0];
    w.sy = step[1];
    w.sz = step[2];
    for (int a = 0; a < 3; ++a) {
        uint32_t ql = 0, qh = 0;
        for (int s = 0; s < 4; ++s) {
            uint32_t l = 255u, h = 0u;  // unused slot: never read (kEmptySlot)
            if (s < k) {
                l = quant_down((double)box[s][a] - (double)lo[a], inv_step[a]);
                h = quant_up((double)box[s][3 + a] - (double)lo[a], inv_step[a]);
            }
            ql |= l << (8 * s);
            qh |= h << (8 * s);
        }
        w.lo[a] = ql;
        w.hi[a] = qh;
    }
    for (int s = 0; s < 4; ++s) w.ref[s] = s < k ? ref[s] : kEmptySlot;
    out[j] = w;
}

BuildArgs make_build_args(rsi_bvh *h, const float *V)
{
    BuildArgs a;
    a.M = h->M;
    a.off = h->tri_off;
    a.V = V;
    a.n_v = h->n_v;
    a.T = h->T;
    a.n_t = h->n_t;
    a.cent = h->cent;
    a.keys = h->keys;
    a.order = h->order;
    a.rank = h->rank;
    a.nodes = h->nodes;
    a.tris = h->tris;
    a.arrive = h->arrive;
    a.heights = h->heights;
    a.climb = h->climb;
    a.prefix = h->split_prefix;
    a.bounds = h->mesh_bounds;
    a.mesh_height = h->mesh_height;
    a.mesh_root = h->mesh_root;
    a.scalars = h->scalars;
    a.leaf_size = h->leaf_size;
    return a;
}

hipError_t run_hierarchy(const BuildArgs &a, hipStream_t s)
{
    const int32_t n = (int32_t)a.n_t;
    // Blocks of 2048 leaves: one block holds a small mesh whole (no global
    // pass), and a large one needs few device-wide climbs.  Between the two,
    // blocks of 512 spread the local pass over four times as many CUs (the
    // 29,768-triangle rebuild: 0.119 -> 0.109 ms; the trees are the same).
    unsigned nb;
    if (n > 2048 && n <= 131072) {
        nb = (unsigned)((n + 511) / 512);
        hipLaunchKernelGGL((k_lbvh_local<512, 256>), dim3(nb), dim3(256), 0, s, a);
    } else {
        nb = (unsigned)((n + 2047) / 2048);
        hipLaunchKernelGGL((k_lbvh_local<2048, 1024>), dim3(nb), dim3(1024), 0, s, a);
    }
    if (nb > 1) hipLaunchKernelGGL(k_lbvh_global, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

unsigned init_grid(const BuildArgs &a)
{
    const int64_t n = a.n_t > a.M ? a.n_t : a.M;
    return (unsigned)((n + 255) / 256);
}

}  // namespace

hipError_t launch_gather(rsi_bvh *h, hipStream_t s)
{
    const int64_t total = h->n_v + h->n_t;
    if (total == 0) return hipSuccess;
    int64_t grid = (total + 255) / 256;
    if (grid > 65536) grid = 65536;
    hipLaunchKernelGGL(k_clear_gather_flag, dim3(1), dim3(1), 0, s, h->scalars);
    hipLaunchKernelGGL(k_gather, dim3((unsigned)grid), dim3(256), 0, s, h->M, h->src_V, h->src_T, h->vert_off,
                       h->tri_off, h->V_all, h->T, h->scalars);
    return hipGetLastError();
}

hipError_t launch_widen(rsi_bvh *h, hipStream_t s)
{
    if (h->width != 4 || h->n_t == 0 || !h->nodes4) {
        h->width_built = 2;
        return hipSuccess;
    }
    hipLaunchKernelGGL(k_widen, dim3((unsigned)((h->n_t + 255) / 256)), dim3(256), 0, s, h->nodes, h->n_t,
                       h->nodes4);
    h->width_built = 4;
    return hipGetLastError();
}

hipError_t launch_build(rsi_bvh *h, const float *V, hipStream_t s)
{
    const int64_t n = h->n_t;
    if (n == 0) return hipSuccess;
    const BuildArgs a = make_build_args(h, V);
    hipLaunchKernelGGL(k_init, dim3(init_grid(a)), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_centroids, dim3((unsigned)((n + kCentBlock - 1) / kCentBlock)), dim3(kCentBlock), 0, s,
                       a);
    hipLaunchKernelGGL(k_morton, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = radix_sort_pairs(h->keys, h->order, n, 63, h->sort, s, h->M > 1 ? h->tri_off : nullptr, h->M);
    if (e != hipSuccess) return e;
    e = run_hierarchy(a, s);
    if (e != hipSuccess) return e;
    return launch_widen(h, s);
}

hipError_t launch_refit(rsi_bvh *h, const float *V, hipStream_t s)
{
    if (h->n_t == 0) return hipSuccess;
    const BuildArgs a = make_build_args(h, V);
    hipLaunchKernelGGL(k_init, dim3(init_grid(a)), dim3(256), 0, s, a);
    hipError_t e = run_hierarchy(a, s);
    if (e != hipSuccess) return e;
    return launch_widen(h, s);
}

}  // namespace rsi
