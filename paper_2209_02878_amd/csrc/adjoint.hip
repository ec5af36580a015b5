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
// the FP32 inputs; the nine vertex components go to dV by FP32 atomic adds
// (a vertex is shared by the hits of many segments), dS and dE are stores.
// A miss (tri < 0) contributes nothing and gets zero dS, dE.
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

__global__ __launch_bounds__(256) void k_first_hit_adjoint(AdjArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n_r) return;
    const int32_t j = a.tri[i];
    double gs[3] = {0, 0, 0}, ge[3] = {0, 0, 0};
    if (j >= 0 && j < a.n_t) {
        int32_t ia = a.T[3 * (int64_t)j], ib = a.T[3 * (int64_t)j + 1], ic = a.T[3 * (int64_t)j + 2];
        if (ia >= 0 && ia < a.n_v && ib >= 0 && ib < a.n_v && ic >= 0 && ic < a.n_v) {
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
            if (det != 0.0) {
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
                const d3 lam = {(tb * c12.x + ub * c20.x + vb * c01.x) * inv,
                                (tb * c12.y + ub * c20.y + vb * c01.y) * inv,
                                (tb * c12.z + ub * c20.z + vb * c01.z) * inv};
                const d3 q = {lam.x + pb.x, lam.y + pb.y, lam.z + pb.z};
                gs[0] = (1.0 - t) * q.x;
                gs[1] = (1.0 - t) * q.y;
                gs[2] = (1.0 - t) * q.z;
                ge[0] = t * q.x;
                ge[1] = t * q.y;
                ge[2] = t * q.z;
                const double w0 = -(1.0 - u - v), w1 = -u, w2 = -v;
                float *dv0 = a.dV + 3 * (int64_t)ia;
                float *dv1 = a.dV + 3 * (int64_t)ib;
                float *dv2 = a.dV + 3 * (int64_t)ic;
                unsafeAtomicAdd(dv0 + 0, (float)(w0 * lam.x));
                unsafeAtomicAdd(dv0 + 1, (float)(w0 * lam.y));
                unsafeAtomicAdd(dv0 + 2, (float)(w0 * lam.z));
                unsafeAtomicAdd(dv1 + 0, (float)(w1 * lam.x));
                unsafeAtomicAdd(dv1 + 1, (float)(w1 * lam.y));
                unsafeAtomicAdd(dv1 + 2, (float)(w1 * lam.z));
                unsafeAtomicAdd(dv2 + 0, (float)(w2 * lam.x));
                unsafeAtomicAdd(dv2 + 1, (float)(w2 * lam.y));
                unsafeAtomicAdd(dv2 + 2, (float)(w2 * lam.z));
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
}

}  // namespace

hipError_t launch_first_hit_adjoint(rsi_bvh *h, const float *V, const float *S, const float *E, int64_t n_r,
                                    const int32_t *tri, const float *g_t, const float *g_uv, const float *g_p,
                                    float *dV, float *dS, float *dE, hipStream_t s)
{
    if (n_r == 0) return hipSuccess;
    AdjArgs a = {V, h->n_v, h->T, h->n_t, S, E, n_r, tri, g_t, g_uv, g_p, dV, dS, dE};
    const int blk = 256;
    hipLaunchKernelGGL(k_first_hit_adjoint, dim3((unsigned)((n_r + blk - 1) / blk)), dim3(blk), 0, s, a);
    return hipGetLastError();
}

}  // namespace rsi
