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
// One lane per segment.  (t, u, v) and the solve are recomputed in FP64 from
// the FP32 inputs; dS and dE are stores, the nine vertex components go to dV
// by FP32 atomic adds (a vertex is shared by the hits of many segments).
// Device-wide atomics dominate the cost, so large batches are first ordered
// by the Morton position of the hit triangle (the build's radix sort) and
// each wave sums the contributions of its runs of equal triangles before
// adding them.  A miss (tri < 0) contributes nothing and gets zero dS, dE.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rsi_host.h"

namespace rsi {
namespace {

struct AdjArgs {
    const float *V;
    int64_t n_v;
    const int32_t *T;
    int64_t n_t;
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

// One segment's adjoint: dS, dE and the three vertex contributions
// (wv[3 * corner + axis]).  tri_ok: the hit triangle and its vertex indices
// are valid (ia, ib, ic set); valid: also a nonsingular solve (the
// contributions are nonzero only then).
struct AdjOut {
    double gs[3], ge[3];
    float wv[9];
    int32_t ia, ib, ic;
    bool tri_ok, valid;
};

__device__ inline AdjOut adjoint_of(const AdjArgs &a, int64_t i)
{
    AdjOut o;
    for (int k = 0; k < 3; ++k) o.gs[k] = o.ge[k] = 0.0;
    for (int k = 0; k < 9; ++k) o.wv[k] = 0.0f;
    o.ia = o.ib = o.ic = 0;
    o.tri_ok = o.valid = false;
    const int32_t j = a.tri[i];
    if (j < 0 || j >= a.n_t) return o;
    const int32_t ia = a.T[3 * (int64_t)j], ib = a.T[3 * (int64_t)j + 1], ic = a.T[3 * (int64_t)j + 2];
    if (ia < 0 || ia >= a.n_v || ib < 0 || ib >= a.n_v || ic < 0 || ic >= a.n_v) return o;
    o.ia = ia;
    o.ib = ib;
    o.ic = ic;
    o.tri_ok = true;
    const d3 s = mk(a.S[3 * i], a.S[3 * i + 1], a.S[3 * i + 2]);
    const d3 e = mk(a.E[3 * i], a.E[3 * i + 1], a.E[3 * i + 2]);
    const d3 v0 = mk(a.V[3 * ia], a.V[3 * ia + 1], a.V[3 * ia + 2]);
    const d3 v1 = mk(a.V[3 * ib], a.V[3 * ib + 1], a.V[3 * ib + 2]);
    const d3 v2 = mk(a.V[3 * ic], a.V[3 * ic + 1], a.V[3 * ic + 2]);
    const d3 d = sub(e, s), e1 = sub(v1, v0), e2 = sub(v2, v0), r = sub(s, v0);
    const d3 md = {-d.x, -d.y, -d.z};
    // forward values by Cramer's rule on the columns of M
    const d3 c12 = cross(e1, e2);
    const double det = dot(md, c12);
    if (det == 0.0) return o;
    const double inv = 1.0 / det;
    const double t = dot(r, c12) * inv;
    const double u = dot(md, cross(r, e2)) * inv;
    const double v = dot(md, cross(e1, r)) * inv;
    const d3 pb = a.g_p ? mk(a.g_p[3 * i], a.g_p[3 * i + 1], a.g_p[3 * i + 2]) : mk(0, 0, 0);
    const double tb = (a.g_t ? (double)a.g_t[i] : 0.0) + dot(pb, d);
    const double ub = a.g_uv ? (double)a.g_uv[2 * i] : 0.0;
    const double vb = a.g_uv ? (double)a.g_uv[2 * i + 1] : 0.0;
    // M^T lambda = (tb, ub, vb): rows of M^T are -d, e1, e2, so
    // lambda = (tb (e1 x e2) + ub (e2 x -d) + vb (-d x e1)) / det
    const d3 c20 = cross(e2, md), c01 = cross(md, e1);
    const d3 lam = {(tb * c12.x + ub * c20.x + vb * c01.x) * inv, (tb * c12.y + ub * c20.y + vb * c01.y) * inv,
                    (tb * c12.z + ub * c20.z + vb * c01.z) * inv};
    const d3 q = {lam.x + pb.x, lam.y + pb.y, lam.z + pb.z};
    o.gs[0] = (1.0 - t) * q.x;
    o.gs[1] = (1.0 - t) * q.y;
    o.gs[2] = (1.0 - t) * q.z;
    o.ge[0] = t * q.x;
    o.ge[1] = t * q.y;
    o.ge[2] = t * q.z;
    const double w[3] = {-(1.0 - u - v), -u, -v};
    for (int c = 0; c < 3; ++c) {
        o.wv[3 * c] = (float)(w[c] * lam.x);
        o.wv[3 * c + 1] = (float)(w[c] * lam.y);
        o.wv[3 * c + 2] = (float)(w[c] * lam.z);
    }
    o.valid = true;
    return o;
}

__device__ inline void store_ends(const AdjArgs &a, int64_t i, const AdjOut &o)
{
    if (a.dS) {
        a.dS[3 * i] = (float)o.gs[0];
        a.dS[3 * i + 1] = (float)o.gs[1];
        a.dS[3 * i + 2] = (float)o.gs[2];
    }
    if (a.dE) {
        a.dE[3 * i] = (float)o.ge[0];
        a.dE[3 * i + 1] = (float)o.ge[1];
        a.dE[3 * i + 2] = (float)o.ge[2];
    }
}

__device__ inline void add_vertices(const AdjArgs &a, const AdjOut &o, const float *wv)
{
    const int32_t vi[3] = {o.ia, o.ib, o.ic};
    for (int c = 0; c < 3; ++c) {
        float *dv = a.dV + 3 * (int64_t)vi[c];
        unsafeAtomicAdd(dv + 0, wv[3 * c]);
        unsafeAtomicAdd(dv + 1, wv[3 * c + 1]);
        unsafeAtomicAdd(dv + 2, wv[3 * c + 2]);
    }
}

// Small inputs: one lane per segment in input order, nine atomics per hit.
__global__ __launch_bounds__(256) void k_first_hit_adjoint(AdjArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n_r) return;
    const AdjOut o = adjoint_of(a, i);
    if (o.valid) add_vertices(a, o, o.wv);
    store_ends(a, i, o);
}

// Hit-order keys: the sorted (Morton) position of the hit triangle, misses
// last; values: segment indices.
__global__ __launch_bounds__(256) void k_adj_keys(const int32_t *__restrict__ tri, int64_t n_r,
                                                  const int32_t *__restrict__ rank, int32_t n_t,
                                                  uint64_t *__restrict__ keys, uint32_t *__restrict__ vals)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_r) return;
    const int32_t j = tri[i];
    keys[i] = (j >= 0 && j < n_t) ? (uint64_t)rank[j] : (uint64_t)n_t;
    vals[i] = (uint32_t)i;
}

// Segments in hit-triangle order: lanes of a wave that hit the same
// triangle form runs; a segmented sum over each run (shuffles up the wave)
// leaves the run's total in its last lane, which alone adds it to dV.
// Consecutive segments share a triangle about N_r / N_t times, so this cuts
// the device-wide atomics by about that factor.
__global__ __launch_bounds__(256) void k_first_hit_adjoint_sorted(AdjArgs a, const uint64_t *__restrict__ keys,
                                                                  const uint32_t *__restrict__ vals)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = k < a.n_r;
    const int64_t i = in ? (int64_t)vals[k] : 0;
    // lanes past the end get a key no real segment has
    const uint64_t key = in ? keys[k] : ~0ull;
    AdjOut o;
    if (in) {
        o = adjoint_of(a, i);
        store_ends(a, i, o);
    } else {
        for (int q = 0; q < 9; ++q) o.wv[q] = 0.0f;
        o.tri_ok = o.valid = false;
    }
    float acc[9];
    for (int q = 0; q < 9; ++q) acc[q] = o.wv[q];
    const int lane = (int)__lane_id();
    const uint32_t klo = (uint32_t)key, khi = (uint32_t)(key >> 32);
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t ulo = __shfl_up(klo, off, 64), uhi = __shfl_up(khi, off, 64);
        const bool same = lane >= off && ulo == klo && uhi == khi;
        for (int q = 0; q < 9; ++q) {
            const float up = __shfl_up(acc[q], off, 64);
            acc[q] += same ? up : 0.0f;
        }
    }
    const uint32_t nlo = __shfl_down(klo, 1, 64), nhi = __shfl_down(khi, 1, 64);
    const bool last = lane == 63 || nlo != klo || nhi != khi;
    // every lane of a run hit the same triangle, so the last lane's indices
    // serve the run (its own solve may have been singular)
    if (in && o.tri_ok && last) add_vertices(a, o, acc);
}

}  // namespace

hipError_t launch_first_hit_adjoint(rsi_bvh *h, const float *V, const float *S, const float *E, int64_t n_r,
                                    const int32_t *tri, const float *g_t, const float *g_uv, const float *g_p,
                                    float *dV, float *dS, float *dE, hipStream_t s)
{
    if (n_r == 0) return hipSuccess;
    AdjArgs a = {V, h->n_v, h->T, h->n_t, S, E, n_r, tri, g_t, g_uv, g_p, dV, dS, dE};
    const int blk = 256;
    const unsigned grid = (unsigned)((n_r + blk - 1) / blk);
    // few hits per triangle (or a tiny batch): nothing to combine
    if (h->n_t == 0 || n_r < 4 * h->n_t || n_r < 65536) {
        hipLaunchKernelGGL(k_first_hit_adjoint, dim3(grid), dim3(blk), 0, s, a);
        return hipGetLastError();
    }
    hipError_t e = hipSuccess;
    if (h->seg_key_cap < n_r) {
        if (h->seg_keys) (void)hipFree(h->seg_keys);
        h->seg_keys = nullptr;
        h->seg_key_cap = 0;
        if ((e = hipMalloc(reinterpret_cast<void **>(&h->seg_keys), sizeof(uint64_t) * (size_t)n_r)) != hipSuccess)
            return e;
        h->seg_key_cap = n_r;
    }
    if (h->adj_val_cap < n_r) {
        if (h->adj_vals) (void)hipFree(h->adj_vals);
        h->adj_vals = nullptr;
        h->adj_val_cap = 0;
        if ((e = hipMalloc(reinterpret_cast<void **>(&h->adj_vals), sizeof(uint32_t) * (size_t)n_r)) != hipSuccess)
            return e;
        h->adj_val_cap = n_r;
    }
    hipLaunchKernelGGL(k_adj_keys, dim3(grid), dim3(blk), 0, s, tri, n_r, h->rank, (int32_t)h->n_t, h->seg_keys,
                       h->adj_vals);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    int bits = 1;
    while (bits < 63 && ((int64_t)1 << bits) <= h->n_t) ++bits;  // keys in [0, n_t]
    e = radix_sort_pairs(h->seg_keys, h->adj_vals, n_r, bits, h->seg_sort, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_first_hit_adjoint_sorted, dim3(grid), dim3(blk), 0, s, a, h->seg_keys, h->adj_vals);
    return hipGetLastError();
}

}  // namespace rsi
