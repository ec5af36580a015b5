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
//   k_adj_tri     four workgroups per cell, each taking a quarter of the
//                 cell's pairs in order: tiles of 512 pairs are ranked
//                 stably by (cell triangle mod 256) in LDS, and thread t adds
//                 the records of its four triangles (t + 256 j) in that order,
//                 in FP64, to nine running sums per triangle (three corners x
//                 three axes); each quarter's sums are stored
//   k_adj_combine one lane per triangle: the four quarters' sums, in order
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
constexpr int kCellTris = 1 << kCellBits;
constexpr int kTriPerThread = kCellTris / kThreads;  // 4: thread t owns cell triangles t + 256 j
constexpr int kChunks = 4;                       // k_adj_tri workgroups per cell (each a quarter of its pairs)
constexpr int kTriItems = 2;                     // pairs per thread per tile of k_adj_tri
constexpr int kTriTile = kThreads * kTriItems;

struct AdjArgs {
    const float *V;
    int64_t n_v;
    const int32_t *T;
    int64_t n_t;
    const int32_t *rank;  // sorted (Morton) position of each triangle
    const Tri *tris;      // the tree's triangle records (vertices of the last build or refit), sorted
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
    float4 *rec;          // per segment: lambda.x, lambda.y, lambda.z, 1 - u - v
    float2 *rec_v;        // per segment: u, v
    uint64_t *keys;       // per segment: sorted position of the hit triangle, n_t when none
    uint32_t *vals;       // per segment: its index
    double *tri_sum;      // per sorted triangle: 3 corners x 3 axes
    double *part;         // per (cell, chunk, cell triangle): the chunk's 9 sums
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
    // the hit triangle's vertices from its record in the tree (copied from
    // V at the last build or refit, which is the V this call is given): one
    // gather of 48 contiguous bytes at its sorted position instead of an
    // index row and three vertex rows
    const int32_t pos = (j >= 0 && j < a.n_t) ? a.rank[j] : -1;
    if (pos >= 0 && pos < a.n_t) {
        const float4 ta = a.tris[pos].a, tb4 = a.tris[pos].b, tc = a.tris[pos].c;
        if (tc.w == 0.0f) {
            const d3 s = mk(a.S[3 * i], a.S[3 * i + 1], a.S[3 * i + 2]);
            const d3 e = mk(a.E[3 * i], a.E[3 * i + 1], a.E[3 * i + 2]);
            const d3 v0 = mk(ta.x, ta.y, ta.z);
            const d3 v1 = mk(ta.w, tb4.x, tb4.y);
            const d3 v2 = mk(tb4.z, tb4.w, tc.x);
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
                key = (uint64_t)pos;
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
    a.rec[i] = r;
    a.rec_v[i] = rv;
    a.keys[i] = key;
    a.vals[i] = (uint32_t)i;
}

// Bucket starts of keys ordered by the field (key >> shift): for b in
// [0, nb], first[b] = the first index whose field is >= b (n if none).  One
// thread per key writes the starts of the buckets between its predecessor's
// field and its own, so a single coalesced pass fills every entry, empty
// buckets included.
__global__ __launch_bounds__(256) void k_bucket_starts(const uint64_t *__restrict__ keys, int64_t n, int shift,
                                                       int64_t nb, int64_t *__restrict__ first)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k > n) return;
    // k is the first index of every bucket b with field(k - 1) < b <= field(k)
    // (field(-1) = -1, field(n) = nb + 1)
    const int64_t cur = k < n ? (int64_t)(keys[k] >> shift) : nb + 1;
    const int64_t prev = k > 0 ? (int64_t)(keys[k - 1] >> shift) : -1;
    for (int64_t b = prev + 1; b <= cur && b <= nb; ++b) first[b] = k;
}

// One workgroup per (cell g, chunk c): the c-th quarter of the cell's pairs
// (in order).  keys/vals: the pairs ordered by cell (stable, so input order
// within a cell).  Thread t owns the cell's triangles t + 256 j (j < 4); the
// tile's pairs are ranked stably by (cell triangle mod 256), so thread t
// meets the records of its four triangles in tile order and adds each to
// its triangle's nine FP64 sums.  Every pair is ranked once; the chunk's
// sums of all 1,024 triangles go to `part`, which k_adj_combine adds up in
// chunk order.
__global__ __launch_bounds__(kThreads) void k_adj_tri(AdjArgs a, const uint64_t *__restrict__ keys,
                                                      const uint32_t *__restrict__ vals,
                                                      const int64_t *__restrict__ cell_first)
{
    __shared__ uint32_t wcnt[kTriItems * kWaves * kRadix];
    __shared__ uint32_t run[kRadix], start[kRadix];
    __shared__ float4 srec[kTriTile];
    __shared__ float2 srv[kTriTile];
    __shared__ uint8_t sj[kTriTile];
    __shared__ int64_t range[2];
    const int tid = threadIdx.x;
    const int64_t g = blockIdx.x / kChunks;
    const int chunk = (int)(blockIdx.x % kChunks);
    if (tid == 0) {
        const int64_t clo = cell_first[g];
        const int64_t chi = cell_first[g + 1];
        const int64_t len = chi - clo;
        range[0] = clo + len * chunk / kChunks;
        range[1] = clo + len * (chunk + 1) / kChunks;
    }
    __syncthreads();
    const int64_t lo = range[0], hi = range[1];
    double acc[kTriPerThread][9];
#pragma unroll
    for (int j = 0; j < kTriPerThread; ++j)
#pragma unroll
        for (int q = 0; q < 9; ++q) acc[j][q] = 0.0;
    for (int64_t c0 = lo; c0 < hi; c0 += kTriTile) {
        uint32_t dig[kTriItems], pos[kTriItems], seg[kTriItems], jj[kTriItems];
        bool sel[kTriItems];
#pragma unroll
        for (int r = 0; r < kTriItems; ++r) {
            const int64_t k = c0 + r * kThreads + tid;
            const uint64_t key = k < hi ? keys[k] : ~0ull;
            sel[r] = k < hi && key < (uint64_t)a.n_t;  // misses sort last (key n_t), past every cell
            const uint32_t local = (uint32_t)(key & (kCellTris - 1));
            dig[r] = sel[r] ? (local & (kRadix - 1)) : 0u;
            jj[r] = local >> 8;
            seg[r] = sel[r] ? vals[k] : 0u;
        }
        rank::rank_tile<kTriItems>(dig, sel, pos, wcnt, run, start);
#pragma unroll
        for (int r = 0; r < kTriItems; ++r) {
            if (sel[r]) {
                srec[pos[r]] = a.rec[seg[r]];
                srv[pos[r]] = a.rec_v[seg[r]];
                sj[pos[r]] = (uint8_t)jj[r];
            }
        }
        __syncthreads();
        // the records of this thread's four triangles, in tile order: one
        // sweep of the run per triangle, adding the records that belong to it
        const uint32_t b = start[tid], e = b + run[tid];
#pragma unroll
        for (int jt = 0; jt < kTriPerThread; ++jt) {
            for (uint32_t p = b; p < e; ++p) {
                if (sj[p] != jt) continue;
                const float4 rr = srec[p];
                const float2 uv = srv[p];
                const double w[3] = {-(double)rr.w, -(double)uv.x, -(double)uv.y};
                const double l[3] = {(double)rr.x, (double)rr.y, (double)rr.z};
#pragma unroll
                for (int c = 0; c < 3; ++c)
#pragma unroll
                    for (int d = 0; d < 3; ++d) acc[jt][3 * c + d] += w[c] * l[d];
            }
        }
        __syncthreads();
    }
    double *o = a.part + ((g * kChunks + chunk) * kCellTris) * 9;
#pragma unroll
    for (int j = 0; j < kTriPerThread; ++j)
#pragma unroll
        for (int q = 0; q < 9; ++q) o[(j * kThreads + tid) * 9 + q] = acc[j][q];
}

// Per sorted triangle: its chunks' sums, added in chunk order.
__global__ __launch_bounds__(256) void k_adj_combine(AdjArgs a)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.n_t) return;
    const int64_t g = t >> kCellBits, local = t & (kCellTris - 1);
    double s[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) s[q] = 0.0;
    for (int c = 0; c < kChunks; ++c) {
        const double *p = a.part + ((g * kChunks + c) * kCellTris + local) * 9;
#pragma unroll
        for (int q = 0; q < 9; ++q) s[q] += p[q];
    }
    double *o = a.tri_sum + 9 * t;
#pragma unroll
    for (int q = 0; q < 9; ++q) o[q] = s[q];
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
                                                    const uint32_t *__restrict__ inc_vals, int64_t n_inc,
                                                    const int64_t *__restrict__ inc_first)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= a.n_v) return;
    const int64_t b = inc_first[v];
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
    a.tris = h->tris;
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
    if ((e = grow(&h->adj_rec, h->adj_rec_cap, n_r)) != hipSuccess) return e;
    if ((e = grow(&h->adj_rec_v, h->adj_rec_v_cap, n_r)) != hipSuccess) return e;
    const int64_t n_cells = (h->n_t + kCellTris - 1) >> kCellBits;
    if ((e = grow(&h->tri_sum, h->tri_sum_cap, 9 * h->n_t)) != hipSuccess) return e;
    if ((e = grow(&h->adj_part, h->adj_part_cap, 9 * n_cells * kChunks * kCellTris)) != hipSuccess) return e;
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
        // first table entry of every vertex (CSR starts; an invalid index sorts last, at n_v)
        if ((e = grow(&h->inc_first, h->inc_first_cap, h->n_v + 2)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_bucket_starts, dim3((unsigned)((n_inc + 1 + 255) / 256)), dim3(256), 0, s, h->inc_keys,
                           n_inc, 0, h->n_v, h->inc_first);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        h->inc_valid = true;
    }
    a.rec = h->adj_rec;
    a.rec_v = h->adj_rec_v;
    a.keys = h->seg_keys;
    a.vals = h->adj_vals;
    a.tri_sum = h->tri_sum;
    a.part = h->adj_part;
    const unsigned grid = (unsigned)((n_r + 255) / 256);
    hipLaunchKernelGGL(k_adj_solve, dim3(grid), dim3(256), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // group the pairs by cell (keys in [0, n_t]; cell = key >> kCellBits)
    uint64_t *ks = h->seg_keys;
    uint32_t *vs = h->adj_vals;
    e = radix_sort_pairs(h->seg_keys, h->adj_vals, n_r, bits_for(h->n_t), h->seg_sort, s, nullptr, 1, kCellBits, &ks,
                         &vs);
    if (e != hipSuccess) return e;
    // pairs of cell g: [cell_first[g], cell_first[g + 1]); misses (key n_t) sort last
    if ((e = grow(&h->adj_cell_first, h->adj_cell_first_cap, n_cells + 2)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_bucket_starts, dim3((unsigned)((n_r + 1 + 255) / 256)), dim3(256), 0, s, ks, n_r, kCellBits,
                       n_cells, h->adj_cell_first);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_tri, dim3((unsigned)(n_cells * kChunks)), dim3(kThreads), 0, s, a, ks, vs,
                       h->adj_cell_first);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_adj_combine, dim3((unsigned)((h->n_t + 255) / 256)), dim3(256), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (dV) {
        hipLaunchKernelGGL(k_adj_vertex, dim3((unsigned)((h->n_v + 255) / 256)), dim3(256), 0, s, a, h->inc_keys,
                           h->inc_vals, 3 * h->n_t, h->inc_first);
        e = hipGetLastError();
    }
    return e;
}

}  // namespace rsi
