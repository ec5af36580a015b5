// adjoint.hip -- gradient of the first hit with respect to the mesh vertices
// and both segment ends (an extension of the paper's `barycentric` mode,
// Section 2.4, which returns the crossing point and triangle).
//
// A hit solves  S + t d = v0 + u e1 + v e2  (d = E - S, e1 = v1 - v0,
// e2 = v2 - v0), i.e.  M x = S - v0  with  M = [-d | e1 | e2], x = (t, u, v),
// and reports P = S + t d.  Given upstream gradients (tbar, ubar, vbar, Pbar),
// fold P into t (tbar += Pbar . d) and solve the transposed system
//   M^T lambda = (tbar, ubar, vbar);
// then, by the implicit-function rule,
//   dL/dS  = (1 - t) (lambda + Pbar),    dL/dE = t (lambda + Pbar),
//   dL/dv0 = -(1 - u - v) lambda,  dL/dv1 = -u lambda,  dL/dv2 = -v lambda.
// (t, u, v) and the solve are recomputed in FP64 from the FP32 inputs.
//
// The vertex gradient sums over every segment whose first hit is a triangle
// around the vertex.  It is formed without any atomic operation, in a fixed
// order, so every call gives the same bits:
//   k_adj_solve   one lane per segment, in input order (coalesced): the
//                 solve, dS and dE, and a record of lambda and the three
//                 corner weights (1 - u - v, u, v) with the
//                 sort pair (Morton position of the hit triangle, segment)
//   (sort.hip)    one stable pass per 8 bits of the cell index (position >>
//                 10): the pairs of each cell of 1,024 consecutive
//                 triangles become contiguous, in input order within a cell
//   k_adj_tri     one workgroup per 256 triangles of a cell: it walks its
//                 cell's pairs in tiles, ranks the tile's own pairs stably by
//                 triangle in LDS, and thread t adds the records of triangle
//                 t in that order, in FP64, to nine running sums (three
//                 corners x three axes), stored per triangle at the end
//   k_adj_vertex  one lane per vertex: the sums of the (triangle, corner)
//                 pairs incident to it (a table sorted by vertex, built once
//                 per topology), added to dV
// A miss (tri < 0), an invalid triangle or a singular solve contributes
// nothing; such segments get zero dS and dE.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rsi_host.h"
#include "rsi_rank.h"

namespace rsi {
namespace {

using rank::kThreads;
using rank::kWaves;
using rank::kRadix;

constexpr int kCellBits = 10;                    // triangles per cell: 1,024
constexpr int kGroupBits = 8;                    // triangles per k_adj_tri workgroup: 256
constexpr int kGroupsPerCell = 1 << (kCellBits - kGroupBits);
constexpr int kTriItems = 4;                     // pairs per thread per tile of k_adj_tri
constexpr int kTriTile = kThreads * kTriItems;

struct AdjArgs {
    const float *V;
    int64_t n_v;
    const int32_t *T;
    int64_t n_t;
    const int32_t *rank;  // sorted (Morton) position of each triangle
    const float *S;
    const float *E;
    int64_t n_r;
    const int32_t *tri;
    const float *g_t;
    const float *g_uv;
    const float *g_p;
    float *dV;
    float *dS;
    float *dE;
    float4 *rec;          // per segment, 32 bytes (one line to gather): lambda.x, lambda.y,
                          // lambda.z, 1 - u - v, then u, v and two unused words
    uint64_t *keys;       // per segment: sorted position of the hit triangle, n_t when none
    uint32_t *vals;       // per segment: its index
    double *tri_sum;      // per sorted triangle: 3 corners x 3 axes
};

struct d3 {
    double x, y, z;
};
__device__ inline d3 mk(double x, double y, double z) { return {x, y, z}; }
__device__ inline d3 sub(d3 a, d3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline double dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline d3 cross(d3 a, d3 b)
{
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// First pass: one lane per segment in input order.
__global__ __launch_bounds__(256) void k_adj_solve(AdjArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n_r) return;
    double gs[3] = {0.0, 0.0, 0.0}, ge[3] = {0.0, 0.0, 0.0};
    float4 r = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float2 rv = make_float2(0.0f, 0.0f);
    uint64_t key = (uint64_t)a.n_t;
    const int32_t j = a.tri[i];
    if (j >= 0 && j < a.n_t) {
        const int32_t ia = a.T[3 * (int64_t)j], ib = a.T[3 * (int64_t)j + 1], ic = a.T[3 * (int64_t)j + 2];
        if (ia >= 0 && ia < a.n_v && ib >= 0 && ib < a.n_v && ic >= 0 && ic < a.n_v) {
            const d3 s = mk(a.S[3 * i], a.S[3 * i + 1], a.S[3 * i + 2]);
            const d3 e = mk(a.E[3 * i], a.E[3 * i + 1], a.E[3 * i + 2]);
            const d3 v0 = mk(a.V[3 * ia], a.V[3 * ia + 1], a.V[3 * ia + 2]);
            const d3 v1 = mk(a.V[3 * ib], a.V[3 * ib + 1], a.V[3 * ib + 2]);
            const d3 v2 = mk(a.V[3 * ic], a.V[3 * ic + 1], a.V[3 * ic + 2]);
            const d3 d = sub(e, s), e1 = sub(v1, v0), e2 = sub(v2, v0), q = sub(s, v0);
            const d3 md = {-d.x, -d.y, -d.z};
            // forward values by Cramer's rule on the columns of M
            const d3 c12 = cross(e1, e2);
            const double det = dot(md, c12);
            if (det != 0.0) {
                const double inv = 1.0 / det;
                const double t = dot(q, c12) * inv;
                const double u = dot(md, cross(q, e2)) * inv;
                const double v = dot(md, cross(e1, q)) * inv;
                const d3 pb = a.g_p ? mk(a.g_p[3 * i], a.g_p[3 * i + 1], a.g_p[3 * i + 2]) : mk(0, 0, 0);
                const double tb = (a.g_t ? (double)a.g_t[i] : 0.0) + dot(pb, d);
                const double ub = a.g_uv ? (double)a.g_uv[2 * i] : 0.0;
                const double vb = a.g_uv ? (double)a.g_uv[2 * i + 1] : 0.0;
                // M^T lambda = (tb, ub, vb): rows of M^T are -d, e1, e2, so
                // lambda = (tb (e1 x e2) + ub (e2 x -d) + vb (-d x e1)) / det
                const d3 c20 = cross(e2, md), c01 = cross(md, e1);
                const d3 lam = {(tb * c12.x + ub * c20.x + vb * c01.x) * inv,
                                (tb * c12.y + ub * c20.y + vb * c01.y) * inv,
                                (tb * c12.z + ub * c20.z + vb * c01.z) * inv};
                const d3 w = {lam.x + pb.x, lam.y + pb.y, lam.z + pb.z};
                gs[0] = (1.0 - t) * w.x;
                gs[1] = (1.0 - t) * w.y;
                gs[2] = (1.0 - t) * w.z;
                ge[0] = t * w.x;
                ge[1] = t * w.y;
                ge[2] = t * w.z;
                // the three corner weights are rounded separately from their
                // FP64 values: 1 - u - v formed later from rounded u and v
                // would lose its relative accuracy near the edge v1 v2
                r = make_float4((float)lam.x, (float)lam.y, (float)lam.z, (float)(1.0 - u - v));
                rv = make_float2((float)u, (float)v);
                key = (uint64_t)a.rank[j];
            }
        }
    }
    if (a.dS) {
        a.dS[3 * i] = (float)gs[0];
        a.dS[3 * i + 1] = (float)gs[1];
        a.dS[3 * i + 2] = (float)gs[2];
    }
    if (a.dE) {
        a.dE[3 * i] = (float)ge[0];
        a.dE[3 * i + 1] = (float)ge[1];
        a.dE[3 * i + 2] = (float)ge[2];
    }
    a.rec[2 * i] = r;
    a.rec[2 * i + 1] = make_float4(rv.x, rv.y, 0.0f, 0.0f);
    a.keys[i] = key;
    a.vals[i] = (uint32_t)i;
}

// First index k in [lo, hi) with (keys[k] >> shift) >= x (keys ordered by that field).
__device__ inline int64_t lower_bound_field(const uint64_t *keys, int64_t lo, int64_t hi, uint64_t x, int shift)
{
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((keys[mid] >> shift) < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// One workgroup per 256 consecutive sorted triangles (quarter q of cell g).
// keys/vals: the pairs ordered by cell (stable, so input order within a cell).
__global__ __launch_bounds__(kThreads) void k_adj_tri(AdjArgs a, const uint64_t *__restrict__ keys,
                                                      const uint32_t *__restrict__ vals, int64_t n)
{
    __shared__ uint32_t wcnt[kTriItems * kWaves * kRadix];
    __shared__ uint32_t run[kRadix], start[kRadix];
    __shared__ float4 srec[kTriTile];
    __shared__ float2 srv[kTriTile];
    __shared__ int64_t range[2];
    const int tid = threadIdx.x;
    const int64_t g = blockIdx.x / kGroupsPerCell;
    const int32_t group = (int32_t)blockIdx.x;  // == (position >> kGroupBits) of its triangles
    if (tid == 0) {
        range[0] = lower_bound_field(keys, 0, n, (uint64_t)g, kCellBits);
        range[1] = lower_bound_field(keys, range[0], n, (uint64_t)g + 1, kCellBits);
    }
    __syncthreads();
    const int64_t lo = range[0], hi = range[1];
    double acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] = 0.0;
    for (int64_t c0 = lo; c0 < hi; c0 += kTriTile) {
        uint32_t dig[kTriItems], pos[kTriItems], seg[kTriItems];
        bool sel[kTriItems];
#pragma unroll
        for (int r = 0; r < kTriItems; ++r) {
            const int64_t k = c0 + r * kThreads + tid;
            const uint64_t key = k < hi ? keys[k] : ~0ull;
            sel[r] = k < hi && key < (uint64_t)a.n_t && (int32_t)(key >> kGroupBits) == group;
            dig[r] = sel[r] ? (uint32_t)(key & (kRadix - 1)) : 0u;
            seg[r] = sel[r] ? vals[k] : 0u;
        }
        // a tile without pairs of this group is skipped (segments in Morton
        // order put most of a cell's tiles in one or two of its groups)
        bool any = false;
#pragma unroll
        for (int r = 0; r < kTriItems; ++r) any = any || sel[r];
        if (!__syncthreads_or(any)) continue;
        rank::rank_tile<kTriItems>(dig, sel, pos, wcnt, run, start);
#pragma unroll
        for (int r = 0; r < kTriItems; ++r) {
            if (sel[r]) {
                const float4 *rp = a.rec + 2 * (int64_t)seg[r];
                srec[pos[r]] = rp[0];
                const float4 b = rp[1];
                srv[pos[r]] = make_float2(b.x, b.y);
            }
        }
        __syncthreads();
        // triangle tid: its records of this tile, in input order
        const uint32_t b = start[tid], e = b + run[tid];
        for (uint32_t p = b; p < e; ++p) {
            const float4 rr = srec[p];
            const float2 uv = srv[p];
            const double w[3] = {-(double)rr.w, -(double)uv.x, -(double)uv.y};
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                acc[3 * c] += w[c] * (double)rr.x;
                acc[3 * c + 1] += w[c] * (double)rr.y;
                acc[3 * c + 2] += w[c] * (double)rr.z;
            }
        }
        __syncthreads();
    }
    const int64_t t = (int64_t)group * kRadix + tid;
    if (t < a.n_t) {
        double *o = a.tri_sum + 9 * t;
#pragma unroll
        for (int q = 0; q < 9; ++q) o[q] = acc[q];
    }
}

// Incidence table of a topology: pairs (vertex, 3 * sorted position + corner).
__global__ __launch_bounds__(256) void k_adj_incidence(const int32_t *__restrict__ T, int64_t n_t,
                                                       const int32_t *__restrict__ rank, int64_t n_v,
                                                       uint64_t *__restrict__ keys, uint32_t *__restrict__ vals)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 3 * n_t) return;
    const int64_t j = k / 3;
    const int c = (int)(k - 3 * j);
    const int32_t vtx = T[k];
    keys[k] = (vtx >= 0 && vtx < n_v) ? (uint64_t)vtx : (uint64_t)n_v;  // an invalid index sorts last, unused
    vals[k] = (uint32_t)(3 * (int64_t)rank[j] + c);
}

// One lane per vertex: its incident (triangle, corner) sums, in table order.
__global__ __launch_bounds__(256) void k_adj_vertex(AdjArgs a, const uint64_t *__restrict__ inc_keys,
                                                    const uint32_t *__restrict__ inc_vals, int64_t n_inc)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= a.n_v) return;
    const int64_t b = lower_bound_field(inc_keys, 0, n_inc, (uint64_t)v, 0);
    double x = 0.0, y = 0.0, z = 0.0;
    for (int64_t k = b; k < n_inc && inc_keys[k] == (uint64_t)v; ++k) {
        const uint32_t tc = inc_vals[k];
        const double *s = a.tri_sum + 9 * (int64_t)(tc / 3) + 3 * (tc % 3);
        x += s[0];
        y += s[1];
        z += s[2];
    }
    float *d = a.dV + 3 * v;
    d[0] = (float)((double)d[0] + x);
    d[1] = (float)((double)d[1] + y);
    d[2] = (float)((double)d[2] + z);
}

template <class T>
hipError_t grow(T **p, int64_t &cap, int64_t want)
{
    if (cap >= want) return hipSuccess;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    cap = 0;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(p), sizeof(T) * (size_t)(want > 0 ? want : 1));
    if (e == hipSuccess) cap = want;
    return e;
}

int bits_for(int64_t x)  // bits of the largest value x
{
    int b = 1;
    while (b < 63 && ((int64_t)1 << b) <= x) ++b;
    return b;
}

}  // namespace

hipError_t launch_first_hit_adjoint(rsi_bvh *h, const float *V, const float *S, const float *E, int64_t n_r,
                                    const int32_t *tri, const float *g_t, const float *g_uv, const float *g_p,
                                    float *dV, float *dS, float *dE, hipStream_t s)
{
    if (n_r == 0) return hipSuccess;
    hipError_t e = hipSuccess;
    AdjArgs a = {};
    a.V = V;
    a.n_v = h->n_v;
    a.T = h->T;
    a.n_t = h->n_t;
    a.rank = h->rank;
    a.S = S;
    a.E = E;
    a.n_r = n_r;
    a.tri = tri;
    a.g_t = g_t;
    a.g_uv = g_uv;
    a.g_p = g_p;
    a.dV = dV;
    a.dS = dS;
    a.dE = dE;
    if (h->n_t == 0) {
        // no triangle: every segment misses (zero dS, dE), dV unchanged
        if (dS && (e = hipMemsetAsync(dS, 0, sizeof(float) * 3 * (size_t)n_r, s)) != hipSuccess) return e;
        if (dE && (e = hipMemsetAsync(dE, 0, sizeof(float) * 3 * (size_t)n_r, s)) != hipSuccess) return e;
        return hipSuccess;
    }
    if ((e = grow(&h->seg_keys, h->seg_key_cap, n_r)) != hipSuccess) return e;
    if ((e = grow(&h->adj_vals, h->adj_val_cap, n_r)) != hipSuccess) return e;
    if ((e = grow(&h->adj_rec, h->adj_rec_cap, 2 * n_r)) != hipSuccess) return e;
    const int64_t n_groups = (h->n_t + (1 << kGroupBits) - 1) >> kGroupBits;
    const int64_t n_cells = (n_groups + kGroupsPerCell - 1) / kGroupsPerCell;
    if ((e = grow(&h->tri_sum, h->tri_sum_cap, 9 * n_cells * (1 << kCellBits))) != hipSuccess) return e;
    // incidence table of the current topology (kept until a build changes it)
    if (!h->inc_valid) {
        const int64_t n_inc = 3 * h->n_t;
        if (h->inc_cap < n_inc) {
            // keys and values share one capacity: it holds once both grew
            int64_t ck = 0, cv = 0;
            h->inc_cap = 0;
            if ((e = grow(&h->inc_keys, ck, n_inc)) != hipSuccess) return e;
            if ((e = grow(&h->inc_vals, cv, n_inc)) != hipSuccess) return e;
            h->inc_cap = n_inc;
        }
        hipLaunchKernelGGL(k_adj_incidence, dim3((unsigned)((n_inc + 255) / 256)), dim3(256), 0, s, h->T, h->n_t,
                           h->rank, h->n_v, h->inc_keys, h->inc_vals);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        e = radix_sort_pairs(h->inc_keys, h->inc_vals, n_inc, bits_for(h->n_v), h->seg_sort, s);
        if (e != hipSuccess) return e;
        h->inc_valid = true;
    }
    a.rec = h->adj_rec;
    a.keys = h->seg_keys;
    a.vals = h->adj_vals;
    a.tri_sum = h->tri_sum;
    const unsigned grid = (unsigned)((n_r + 255) / 256);
    hipLaunchKernelGGL(k_adj_solve, dim3(grid), dim3(256), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // group the pairs by cell (keys in [0, n_t]; cell = key >> kCellBits)
    uint64_t *ks = h->seg_keys;
    uint32_t *vs = h->adj_vals;
    e = radix_sort_pairs(h->seg_keys, h->adj_vals, n_r, bits_for(h->n_t), h->seg_sort, s, nullptr, 1, kCellBits, &ks,
                         &vs);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_tri, dim3((unsigned)(n_cells * kGroupsPerCell)), dim3(kThreads), 0, s, a, ks, vs, n_r);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (dV) {
        hipLaunchKernelGGL(k_adj_vertex, dim3((unsigned)((h->n_v + 255) / 256)), dim3(256), 0, s, a, h->inc_keys,
                           h->inc_vals, 3 * h->n_t);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace rsi
