// query.hip -- segment queries against the linear BVH (paper Section 3.2,
// the traversal and candidate testing, and Section 3.3, the query kernel).
//
// One lane per segment.  A lane walks the tree from the entry node with a
// short stack kept in LDS (laid out [depth][lane] so a wave's pushes and pops
// hit distinct banks).  Each step loads one 64-byte node, tests the segment
// against both child boxes, runs the Moller-Trumbore test on the triangles of
// any leaf child whose box it touches, then descends into the nearer internal
// child that it touches and pushes the other.  The paper's bounded candidate
// list with resume (Section 3.2) is not needed: candidates are tested as soon
// as they are found, so the only bounded buffers left are the stack, sized
// from the tree height at build time so it cannot overflow, and the per-
// segment crossing slots of the all-hits mode, whose overflow is detected and
// retried into a pool sized on the host.
//
// Modes
//   bool only   stop at the first crossing (any-hit, Section 3.2)
//   first hit   keep the crossing with the smallest (t, id) and prune boxes
//               that start beyond it
//   all hits    count every crossing, keep the first K found in slots; the
//               epilogue re-solves them in FP64, orders them by (t, id), and
//               appends segments with more than K crossings to an overflow
//               list for the spill pass
#include <hip/hip_runtime.h>
#include <float.h>
#include <math.h>
#include <stdint.h>

#include "../../include/rsi.h"
#include "rsi_host.h"

namespace rsi {
namespace {

enum : uint32_t { M_BOOL = RSI_BOOL, M_FIRST = RSI_FIRST_HIT, M_ALL = RSI_ALL_HITS };

struct QArgs {
    const Node *nodes;
    const Tri *tris;
    int32_t entry;
    const float *S;
    const float *E;
    int64_t n_r;
    QueryOut o;
    // overflow list (all-hits)
    int32_t *ovf_seg;
    int32_t *ovf_cnt;
    int64_t *ovf_off;
    int64_t ovf_cap;
    int32_t *scalars;
    // spill pass
    int32_t *pool_ids;
    float *pool_ts;
    int64_t n_items;  // spill: number of overflow entries
    Counters *counters;
    int32_t depth;       // stack entries per lane (tree height + 1)
    int32_t max_steps;   // node visits never exceed the node count
};

__device__ inline void wave_add_u64(unsigned long long *dst, unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (__lane_id() == 0) atomicAdd(dst, v);
}

// Per-lane traversal state for one segment.
struct Lane {
    Seg seg;
    float tlim;     // MT / box limit on t: 1, or slightly above the best t (first hit)
    float best_t;
    int32_t best_id;
    int32_t best_pos;
    int32_t count;  // crossings found (all hits)
    int32_t spill_cap;  // pool entries reserved for this segment (spill pass)
    bool found;
    uint32_t visits, boxes, tests;
};

// Process the triangles of one leaf; returns true when the lane may stop.
template <uint32_t MODE, bool SPILL, bool COUNT>
__device__ inline bool visit_leaf(const QArgs &a, Lane &L, int32_t ref, int64_t seg_i, int64_t slot_base)
{
    const int32_t first = leaf_first(ref);
    const int32_t cnt = leaf_count(ref);
    for (int32_t k = 0; k < cnt; ++k) {
        const int32_t pos = first + k;
        float v[9];
        int32_t id;
        tri_load(a.tris, pos, v, id);
        if (COUNT) ++L.tests;
        const float lim = (MODE & M_ALL) ? 1.0f : L.tlim;
        const MTHit h = mt_test(L.seg, v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], v[8], lim);
        if (!h.hit) continue;
        L.found = true;
        if (MODE == M_BOOL) return true;
        const float t = h.tn / h.det;
        if (MODE & M_FIRST) {
            if (t < L.best_t || (t == L.best_t && id < L.best_id)) {
                L.best_t = t;
                L.best_id = id;
                L.best_pos = pos;
                if (!(MODE & M_ALL)) L.tlim = fminf(1.0f, t * (1.0f + 0x1p-20f));
            }
        }
        if (MODE & M_ALL) {
            const int32_t c = L.count++;
            if (SPILL) {
                // the spill pass repeats the first pass's decisions; the
                // bound only keeps a mismatch from writing past the segment
                if (c < L.spill_cap) a.pool_ids[slot_base + c] = pos;
            } else if (c < a.o.cap) {
                a.o.ids[slot_base + c] = pos;
            }
        }
    }
    return false;
}

// Stack traversal of one segment.
template <uint32_t MODE, bool SPILL, bool COUNT>
__device__ inline void traverse(const QArgs &a, Lane &L, int32_t *stk, int stride, int64_t seg_i,
                                int64_t slot_base)
{
    int32_t node = a.entry;
    int sp = 0;
    // A traversal visits each node at most once and the stack never holds
    // more than the tree height; both bounds are checked so that a damaged
    // tree can only produce wrong answers, never a hang or a stray access.
    for (int32_t step = 0; step < a.max_steps; ++step) {
        const float4 *q = reinterpret_cast<const float4 *>(a.nodes + node);
        const float4 q0 = q[0], q1 = q[1], q2 = q[2];
        const int4 q3 = reinterpret_cast<const int4 *>(a.nodes + node)[3];
        const float lim = (MODE & M_ALL) ? 1.0f : L.tlim;
        float tl, tr;
        const bool hl = slab_hit(L.seg, q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, lim, tl);
        const bool hr = slab_hit(L.seg, q1.z, q1.w, q2.x, q2.y, q2.z, q2.w, lim, tr);
        if (COUNT) {
            ++L.visits;
            L.boxes += 2;
        }
        const int32_t cl = q3.x, cr = q3.y;
        if (hl && cl < 0) {
            if (visit_leaf<MODE, SPILL, COUNT>(a, L, cl, seg_i, slot_base)) return;
        }
        if (hr && cr < 0) {
            if (visit_leaf<MODE, SPILL, COUNT>(a, L, cr, seg_i, slot_base)) return;
        }
        const bool gl = hl && cl >= 0;
        const bool gr = hr && cr >= 0;
        if (gl && gr && sp < a.depth) {
            const bool left_first = tl <= tr;
            stk[sp * stride] = left_first ? cr : cl;
            ++sp;
            node = left_first ? cl : cr;
        } else if (gl) {
            node = cl;
        } else if (gr) {
            node = cr;
        } else {
            if (sp == 0) return;
            --sp;
            node = stk[sp * stride];
        }
    }
}

// Orders entries [0, n) of a (t, id) list in place by (t, id); insertion sort
// because lists are short.
__device__ inline void sort_slots(int32_t *ids, float *ts, int n)
{
    for (int x = 1; x < n; ++x) {
        const float kt = ts[x];
        const int32_t ki = ids[x];
        int y = x - 1;
        while (y >= 0 && (ts[y] > kt || (ts[y] == kt && ids[y] > ki))) {
            ts[y + 1] = ts[y];
            ids[y + 1] = ids[y];
            --y;
        }
        ts[y + 1] = kt;
        ids[y + 1] = ki;
    }
}

// Replace sorted positions by original ids and FP32 t by the FP64 re-solve.
__device__ inline void refine_list(const QArgs &a, double sx, double sy, double sz, double ex, double ey,
                                   double ez, int32_t *ids, float *ts, int n)
{
    for (int c = 0; c < n; ++c) {
        float v[9];
        int32_t id;
        tri_load(a.tris, ids[c], v, id);
        double t, u, w;
        mt_refine64(sx, sy, sz, ex, ey, ez, v, t, u, w);
        ids[c] = id;
        ts[c] = (float)t;
    }
}

template <uint32_t MODE, bool COUNT>
__global__ __launch_bounds__(1024) void k_query(QArgs a)
{
    extern __shared__ int32_t lds_stack[];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    Lane L;
    L.visits = L.boxes = L.tests = 0;
    if (i < a.n_r) {
        const float sx = a.S[3 * i], sy = a.S[3 * i + 1], sz = a.S[3 * i + 2];
        const float ex = a.E[3 * i], ey = a.E[3 * i + 1], ez = a.E[3 * i + 2];
        L.seg = make_seg(sx, sy, sz, ex, ey, ez);
        L.tlim = 1.0f;
        L.best_t = INFINITY;
        L.best_id = 0x7FFFFFFF;
        L.best_pos = -1;
        L.count = 0;
        L.spill_cap = 0;
        L.found = false;
        const int64_t slot_base = (MODE & M_ALL) ? i * (int64_t)a.o.cap : 0;
        traverse<MODE, false, COUNT>(a, L, lds_stack + threadIdx.x, blockDim.x, i, slot_base);

        if (MODE & M_BOOL) a.o.hit[i] = L.found ? 1 : 0;
        if (MODE & M_FIRST) {
            if (L.best_pos >= 0) {
                float v[9];
                int32_t id;
                tri_load(a.tris, L.best_pos, v, id);
                double t, u, w;
                mt_refine64(sx, sy, sz, ex, ey, ez, v, t, u, w);
                a.o.tri[i] = id;
                a.o.t[i] = (float)t;
                a.o.uv[2 * i] = (float)u;
                a.o.uv[2 * i + 1] = (float)w;
                a.o.point[3 * i] = (float)((double)sx + t * ((double)ex - (double)sx));
                a.o.point[3 * i + 1] = (float)((double)sy + t * ((double)ey - (double)sy));
                a.o.point[3 * i + 2] = (float)((double)sz + t * ((double)ez - (double)sz));
            } else {
                a.o.tri[i] = -1;
                a.o.t[i] = INFINITY;
                a.o.uv[2 * i] = 0.0f;
                a.o.uv[2 * i + 1] = 0.0f;
                a.o.point[3 * i] = 0.0f;
                a.o.point[3 * i + 1] = 0.0f;
                a.o.point[3 * i + 2] = 0.0f;
            }
        }
        if (MODE & M_ALL) {
            const int K = a.o.cap;
            a.o.count[i] = L.count;
            int32_t *ids = a.o.ids + slot_base;
            float *ts = a.o.ts + slot_base;
            const int n_in = L.count < K ? L.count : K;
            if (L.count <= K) {
                refine_list(a, sx, sy, sz, ex, ey, ez, ids, ts, n_in);
                sort_slots(ids, ts, n_in);
            }
            for (int c = n_in; c < K; ++c) {
                ids[c] = -1;
                ts[c] = INFINITY;
            }
            if (L.count > K) {
                const int32_t e = atomicAdd(&a.scalars[kOvfSegs], 1);
                const unsigned long long off =
                    atomicAdd(reinterpret_cast<unsigned long long *>(&a.scalars[kOvfTotalLo]),
                              (unsigned long long)L.count);
                if (e < a.ovf_cap) {
                    a.ovf_seg[e] = (int32_t)i;
                    a.ovf_cnt[e] = L.count;
                    a.ovf_off[e] = (int64_t)off;
                }
            }
        }
    }
    if (COUNT) {
        wave_add_u64(&a.counters->node_visits, L.visits);
        wave_add_u64(&a.counters->box_tests, L.boxes);
        wave_add_u64(&a.counters->tri_tests, L.tests);
        wave_add_u64(&a.counters->segments, i < a.n_r ? 1ull : 0ull);
    }
}

// Spill pass: one lane per overflowed segment traverses again and writes all
// of its crossings to the pool, then orders them and refreshes its K slots.
template <uint32_t MODE>
__global__ __launch_bounds__(1024) void k_spill(QArgs a)
{
    extern __shared__ int32_t lds_stack[];
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.n_items) return;
    const int64_t i = a.ovf_seg[e];
    const int64_t off = a.ovf_off[e];
    const float sx = a.S[3 * i], sy = a.S[3 * i + 1], sz = a.S[3 * i + 2];
    const float ex = a.E[3 * i], ey = a.E[3 * i + 1], ez = a.E[3 * i + 2];
    Lane L;
    L.seg = make_seg(sx, sy, sz, ex, ey, ez);
    L.tlim = 1.0f;
    L.best_t = INFINITY;
    L.best_id = 0x7FFFFFFF;
    L.best_pos = -1;
    L.count = 0;
    L.spill_cap = a.ovf_cnt[e];
    L.found = false;
    L.visits = L.boxes = L.tests = 0;
    traverse<M_ALL, true, false>(a, L, lds_stack + threadIdx.x, blockDim.x, i, off);
    const int n = L.count < L.spill_cap ? L.count : L.spill_cap;
    int32_t *ids = a.pool_ids + off;
    float *ts = a.pool_ts + off;
    refine_list(a, sx, sy, sz, ex, ey, ez, ids, ts, n);
    sort_slots(ids, ts, n);
    const int K = a.o.cap;
    int32_t *sid = a.o.ids + i * (int64_t)K;
    float *sts = a.o.ts + i * (int64_t)K;
    for (int c = 0; c < K; ++c) {
        sid[c] = ids[c];
        sts[c] = ts[c];
    }
}

__global__ void k_fill_miss(int64_t n_r, uint32_t mode, QueryOut o)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_r) return;
    if (mode & M_BOOL) o.hit[i] = 0;
    if (mode & M_FIRST) {
        o.tri[i] = -1;
        o.t[i] = INFINITY;
        o.uv[2 * i] = o.uv[2 * i + 1] = 0.0f;
        o.point[3 * i] = o.point[3 * i + 1] = o.point[3 * i + 2] = 0.0f;
    }
    if (mode & M_ALL) {
        o.count[i] = 0;
        for (int c = 0; c < o.cap; ++c) {
            o.ids[i * (int64_t)o.cap + c] = -1;
            o.ts[i * (int64_t)o.cap + c] = INFINITY;
        }
    }
}

__global__ void k_reset_ovf(int32_t *scalars)
{
    scalars[kOvfSegs] = 0;
    scalars[kOvfTotalLo] = 0;
    scalars[kOvfTotalHi] = 0;
}

__global__ void k_zero_counters(Counters *c)
{
    c->node_visits = c->box_tests = c->tri_tests = c->segments = 0;
}

template <uint32_t MODE, bool COUNT>
void launch_mode(const QArgs &a, int block, size_t lds, hipStream_t s)
{
    const unsigned grid = (unsigned)((a.n_r + block - 1) / block);
    hipLaunchKernelGGL((k_query<MODE, COUNT>), dim3(grid), dim3(block), lds, s, a);
}

template <bool COUNT>
hipError_t dispatch(uint32_t mode, const QArgs &a, int block, size_t lds, hipStream_t s)
{
    // RSI_BOOL is derived for free whenever a full pass runs
    switch (mode) {
    case M_BOOL: launch_mode<M_BOOL, COUNT>(a, block, lds, s); break;
    case M_FIRST: launch_mode<M_FIRST, COUNT>(a, block, lds, s); break;
    case M_FIRST | M_BOOL: launch_mode<M_FIRST | M_BOOL, COUNT>(a, block, lds, s); break;
    case M_ALL: launch_mode<M_ALL, COUNT>(a, block, lds, s); break;
    case M_ALL | M_BOOL: launch_mode<M_ALL | M_BOOL, COUNT>(a, block, lds, s); break;
    case M_ALL | M_FIRST: launch_mode<M_ALL | M_FIRST, COUNT>(a, block, lds, s); break;
    case M_ALL | M_FIRST | M_BOOL: launch_mode<M_ALL | M_FIRST | M_BOOL, COUNT>(a, block, lds, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// Largest multiple of 64 not above `want` whose stack fits in 64 KiB of LDS.
int fit_block(int want, int depth)
{
    int b = want;
    while (b > 64 && (size_t)b * depth * sizeof(int32_t) > 65536) b -= 64;
    return b;
}

QArgs make_args(rsi_bvh *h, const float *S, const float *E, int64_t n_r, const QueryOut &o)
{
    QArgs a;
    a.nodes = h->nodes;
    a.tris = h->tris;
    a.entry = h->entry;
    a.S = S;
    a.E = E;
    a.n_r = n_r;
    a.o = o;
    a.ovf_seg = h->ovf_seg;
    a.ovf_cnt = h->ovf_cnt;
    a.ovf_off = h->ovf_off;
    a.ovf_cap = h->ovf_cap;
    a.scalars = h->scalars;
    a.pool_ids = h->pool_ids;
    a.pool_ts = h->pool_ts;
    a.n_items = 0;
    a.counters = h->counters;
    a.depth = h->height + 1;
    a.max_steps = (int32_t)(h->n_t + 1);
    return a;
}

}  // namespace

hipError_t launch_query(rsi_bvh *h, const float *S, const float *E, int64_t n_r, uint32_t mode,
                        const QueryOut &o, hipStream_t s)
{
    if (n_r == 0) return hipSuccess;
    const int depth = h->height + 1;
    const int block = fit_block(h->block_size, depth);
    const size_t lds = (size_t)block * depth * sizeof(int32_t);
    QArgs a = make_args(h, S, E, n_r, o);
    if (mode & M_ALL) hipLaunchKernelGGL(k_reset_ovf, dim3(1), dim3(1), 0, s, h->scalars);
    if (h->counting) {
        hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(1), 0, s, h->counters);
        return dispatch<true>(mode, a, block, lds, s);
    }
    return dispatch<false>(mode, a, block, lds, s);
}

hipError_t launch_spill(rsi_bvh *h, const float *S, const float *E, uint32_t mode, const QueryOut &o,
                        hipStream_t s)
{
    (void)mode;
    const int64_t n = h->last_ovf_segs;
    if (n == 0) return hipSuccess;
    const int depth = h->height + 1;
    const int block = fit_block(h->block_size, depth);
    const size_t lds = (size_t)block * depth * sizeof(int32_t);
    QArgs a = make_args(h, S, E, 0, o);
    a.n_items = n;
    const unsigned grid = (unsigned)((n + block - 1) / block);
    hipLaunchKernelGGL(k_spill<M_ALL>, dim3(grid), dim3(block), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_fill_miss(int64_t n_r, uint32_t mode, const QueryOut &o, hipStream_t s)
{
    if (n_r == 0) return hipSuccess;
    const int blk = 256;
    hipLaunchKernelGGL(k_fill_miss, dim3((unsigned)((n_r + blk - 1) / blk)), dim3(blk), 0, s, n_r, mode, o);
    return hipGetLastError();
}

}  // namespace rsi
