// rsi_device.h -- device-side records and predicates shared by the build and
// query kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsi {

// ---------------------------------------------------------------- records --
//
// Node: one 64-byte record per internal node holding the bounding boxes of
// BOTH children next to their references, so a traversal step fetches the
// two boxes it tests with four 16-byte loads from one line.  This replaces
// the paper's per-node BVHNode with raw child pointers (Section 3.1): boxes
// move up into the parent, pointers become 32-bit indices, and a leaf is
// encoded in the reference itself.
//
//   f[0..5]   left child  lo.x lo.y lo.z hi.x hi.y hi.z
//   f[6..11]  right child lo.x lo.y lo.z hi.x hi.y hi.z
//   ref[0..1] left / right child reference
//   aux[0..1] build scratch: index-range bounds written by the children
//
// Child reference: >= 0 internal node index; < 0 leaf with
//   first sorted triangle = ref & 0x07FFFFFF, count = ((ref >> 27) & 15) + 1.
struct alignas(64) Node {
    float f[12];
    int32_t ref[2];
    int32_t aux[2];
};
static_assert(sizeof(Node) == 64, "Node must be 64 bytes");

// Node4 (64 bytes, four 16-byte loads like a binary step): the four-way
// view of binary node n, whose children are n's grandchildren (a child that
// is a leaf stands for itself), with the child boxes quantised to 8 bits per
// plane on a grid anchored at the lower corner of n's box.  Record n of the
// Node4 array belongs to binary node n, so a child reference (an internal
// grandchild's index, or a leaf) is valid in both arrays.
//
//   ox, oy, oz   lower corner of n's box (exact)
//   sx, sy, sz   grid steps, powers of two (2^-126 .. 2^122) with 255
//                steps spanning n's box on that axis
//   lo[a]        byte c: child c's lower plane on axis a in grid steps,
//                rounded down;  hi[a] likewise for the upper plane, rounded
//                up -- every quantised box contains its exact child box
//   ref[c]       child reference, kEmptySlot for an unused slot
//
// With exact boxes the four-way record would need 128 bytes; 64 bytes halve
// the vector-cache lookups per visited box, which bound the binary walk.  Any finite
// box is representable.
constexpr int32_t kEmptySlot = 0x7FFFFFFF;
struct alignas(64) Node4 {
    float ox, oy, oz, sz;
    uint32_t lo[3];
    uint32_t hi[3];
    float sx, sy;
    int32_t ref[4];
};
static_assert(sizeof(Node4) == 64, "Node4 must be 64 bytes");

// Tri: the three FP32 vertices of a triangle in Morton (sorted) order plus
// its original id, 48 bytes = three 16-byte loads.  Storing the vertices
// themselves (rather than edges) keeps the FP64 re-solve of reported hits
// exact with respect to the FP32 inputs.
struct alignas(16) Tri {
    float4 a;  // v0.x v0.y v0.z v1.x
    float4 b;  // v1.y v1.z v2.x v2.y
    float4 c;  // v2.z, id (int bits), 0, 1 when a vertex index was out of range (else 0)
};
static_assert(sizeof(Tri) == 48, "Tri must be 48 bytes");

constexpr int kLeafFirstBits = 27;
constexpr int32_t kLeafFirstMask = (1 << kLeafFirstBits) - 1;
constexpr int kMaxLeafSize = 16;

__host__ __device__ inline int32_t leaf_ref(int32_t first, int32_t count)
{
    return (int32_t)(0x80000000u | ((uint32_t)(count - 1) << kLeafFirstBits) | (uint32_t)first);
}
__host__ __device__ inline bool ref_is_leaf(int32_t r) { return r < 0; }
__host__ __device__ inline int32_t leaf_first(int32_t r) { return r & kLeafFirstMask; }
__host__ __device__ inline int32_t leaf_count(int32_t r) { return ((r >> kLeafFirstBits) & 15) + 1; }

// ---------------------------------------------------------------- segment --
//
// Per-lane segment state: origin o = S, direction d = E - S (t in [0, 1]
// spans the segment) and the guarded reciprocal of d for the slab test.
struct Seg {
    float ox, oy, oz;
    float dx, dy, dz;
    float ix, iy, iz;
};

__device__ inline float guarded_rcp(float d)
{
    // Components below the smallest normal FP32 value 2^-126 in magnitude
    // (zero included) use +-2^-126, so the reciprocal is finite (at most
    // 2^126) and every slab parameter is finite or +-inf, never NaN.  The
    // capped reciprocal keeps the box decision exact while every nonzero
    // coordinate difference is a normal number: then |(plane - o) * 2^126|
    // >= 1 lies outside [0, 1] on the same side as the exact parameter.
    // Only differences in the subnormal range (coordinates below about
    // 2^-102) fall short of that.  (plane == o with d == 0 is a segment
    // lying in a box face, which meets the triangles inside only on their
    // boundary.)  The hardware reciprocal is within 1 ulp, which the slack
    // of slab_hit covers.
    const float tiny = 0x1p-126f;
    const float g = fabsf(d) < tiny ? copysignf(tiny, d) : d;
    return __builtin_amdgcn_rcpf(g);
}

__device__ inline Seg make_seg(float sx, float sy, float sz, float ex, float ey, float ez)
{
    Seg r;
    r.ox = sx; r.oy = sy; r.oz = sz;
    r.dx = ex - sx; r.dy = ey - sy; r.dz = ez - sz;
    r.ix = guarded_rcp(r.dx);
    r.iy = guarded_rcp(r.dy);
    r.iz = guarded_rcp(r.dz);
    return r;
}

// Conservative segment / box test (slab method).  Each slab parameter is
// (plane - o) * (1/d): a subtraction, a reciprocal within 1 ulp and a
// product, so its relative error is at most about 4 ulp (2^-22) with no
// absolute term; accepting when near <= far * (1 + 2^-20) therefore never
// rejects a box that the exact segment touches within [0, tmax].  Returns
// the entry parameter in `tnear`.
__device__ inline bool slab_hit(const Seg &s, float lx, float ly, float lz,
                                float hx, float hy, float hz, float tmax, float &tnear)
{
    float t0x = (lx - s.ox) * s.ix, t1x = (hx - s.ox) * s.ix;
    float t0y = (ly - s.oy) * s.iy, t1y = (hy - s.oy) * s.iy;
    float t0z = (lz - s.oz) * s.iz, t1z = (hz - s.oz) * s.iz;
    float n = fmaxf(fmaxf(fminf(t0x, t1x), fminf(t0y, t1y)), fmaxf(fminf(t0z, t1z), 0.0f));
    float f = fminf(fminf(fmaxf(t0x, t1x), fmaxf(t0y, t1y)), fminf(fmaxf(t0z, t1z), tmax));
    tnear = n;
    return n <= f * (1.0f + 0x1p-20f);
}

// Conservative segment / quantised-box test for the four-way view.  Per
// node and axis the caller forms D = corner - o, the margin
// eps = (255 step + |D|) 2^-19 and the parameter of grid plane q
// as one fused multiply-add, fma(q, a, b), with a = step * (1/d) and
// b = (D -+ eps) * (1/d): the lower sign for the plane the segment meets
// first on that axis (the lower plane when the direction component is
// non-negative -- 1/d keeps the sign of d, zero included), the upper sign
// for the other one; qn and qf are those planes' quantised values as floats.
// step is a power of two, so a is exact (barring underflow, i.e. |d| near
// the FP32 range).  The roundings of D, of D -+ eps, of b and of the fma, and
// the reciprocal's own error (within 1 ulp), add up to at most
// 6 * 2^-24 (|D| + 255 step) in plane-offset units, under a fifth of eps: a
// first plane's parameter never exceeds, and an other plane's never falls
// below, that of the exact quantised plane, so the tested box contains the
// quantised box, which contains the child box.  No per-axis min/max is
// needed, and no further slack on the far side.  A product that leaves the
// FP32 range makes the parameter an infinity with the sign of the exact
// one, which then lies far outside [0, 1], or NaN (an exactly zero offset
// with d near zero), which fmaxf / fminf skip with the bounds 0 and tmax_s
// still in place, so such a plane never rejects a box that the exact test
// accepts.  `tmax_s` is the segment's upper parameter with the slack that
// covers the FP32 error of a first-hit bound.
__device__ inline bool qslab_hit(float ax, float ay, float az, float bnx, float bny, float bnz, float bfx,
                                 float bfy, float bfz, float qnx, float qny, float qnz, float qfx, float qfy,
                                 float qfz, float tmax_s, float &tnear)
{
    const float nx = fmaf(qnx, ax, bnx), fx = fmaf(qfx, ax, bfx);
    const float ny = fmaf(qny, ay, bny), fy = fmaf(qfy, ay, bfy);
    const float nz = fmaf(qnz, az, bnz), fz = fmaf(qfz, az, bfz);
    const float n = fmaxf(fmaxf(nx, ny), fmaxf(nz, 0.0f));
    const float f = fminf(fminf(fx, fy), fminf(fz, tmax_s));
    tnear = n;
    return n <= f;
}

// Moller-Trumbore segment / triangle test in FP32, division-free decision
// (paper Section 2 names the test: one division, four dot and two cross
// products at worst).  With e1 = v1 - v0, e2 = v2 - v0, p = d x e2,
// det = e1 . p, s = o - v0, q = s x e1:  u = s.p / det, v = d.q / det,
// t = e2.q / det.  The decision compares the numerators against |det| after
// moving det's sign onto them, so only an accepted hit pays the division.
// Closed triangle and closed segment: u >= 0, v >= 0, u + v <= 1,
// 0 <= t <= tmax; det == 0 (parallel or degenerate triangle) never hits.
struct MTHit {
    bool hit;
    float tn;   // t numerator (sign-normalised)
    float det;  // |det|
};

__device__ inline MTHit mt_test(const Seg &s, float v0x, float v0y, float v0z,
                                float v1x, float v1y, float v1z,
                                float v2x, float v2y, float v2z, float tmax)
{
    // Every fused multiply-add is written out (the library is compiled with
    // contraction off), so the decision is bit-identical in every mode.
    float e1x = v1x - v0x, e1y = v1y - v0y, e1z = v1z - v0z;
    float e2x = v2x - v0x, e2y = v2y - v0y, e2z = v2z - v0z;
    float px = fmaf(s.dy, e2z, -(s.dz * e2y));
    float py = fmaf(s.dz, e2x, -(s.dx * e2z));
    float pz = fmaf(s.dx, e2y, -(s.dy * e2x));
    float det = fmaf(e1x, px, fmaf(e1y, py, e1z * pz));
    float sx = s.ox - v0x, sy = s.oy - v0y, sz = s.oz - v0z;
    float un = fmaf(sx, px, fmaf(sy, py, sz * pz));
    float qx = fmaf(sy, e1z, -(sz * e1y));
    float qy = fmaf(sz, e1x, -(sx * e1z));
    float qz = fmaf(sx, e1y, -(sy * e1x));
    float vn = fmaf(s.dx, qx, fmaf(s.dy, qy, s.dz * qz));
    float tn = fmaf(e2x, qx, fmaf(e2y, qy, e2z * qz));
    float ad = fabsf(det);
    if (det < 0.0f) { un = -un; vn = -vn; tn = -tn; }
    MTHit h;
    h.hit = (det != 0.0f) & (un >= 0.0f) & (vn >= 0.0f) & (un + vn <= ad) & (tn >= 0.0f) &
            (tn <= ad * tmax);
    h.tn = tn;
    h.det = ad;
    return h;
}

__device__ inline void tri_load(const Tri *__restrict__ tris, int32_t k, float v[9], int32_t &id)
{
    float4 a = tris[k].a, b = tris[k].b, c = tris[k].c;
    v[0] = a.x; v[1] = a.y; v[2] = a.z;
    v[3] = a.w; v[4] = b.x; v[5] = b.y;
    v[6] = b.z; v[7] = b.w; v[8] = c.x;
    id = __float_as_int(c.y);
}

// FP64 re-solve of a reported crossing (same Moller-Trumbore algebra in
// double precision on the FP32 inputs promoted exactly).  The FP32 test
// decides WHETHER a crossing exists; this only sharpens t, u, v.
__device__ inline void mt_refine64(double sx, double sy, double sz, double ex, double ey, double ez,
                                   const float v[9], double &t, double &u, double &w)
{
    double dx = ex - sx, dy = ey - sy, dz = ez - sz;
    double v0x = v[0], v0y = v[1], v0z = v[2];
    double e1x = (double)v[3] - v0x, e1y = (double)v[4] - v0y, e1z = (double)v[5] - v0z;
    double e2x = (double)v[6] - v0x, e2y = (double)v[7] - v0y, e2z = (double)v[8] - v0z;
    double px = dy * e2z - dz * e2y;
    double py = dz * e2x - dx * e2z;
    double pz = dx * e2y - dy * e2x;
    double det = e1x * px + e1y * py + e1z * pz;
    double ox = sx - v0x, oy = sy - v0y, oz = sz - v0z;
    double qx = oy * e1z - oz * e1y;
    double qy = oz * e1x - ox * e1z;
    double qz = ox * e1y - oy * e1x;
    double inv = 1.0 / det;
    u = (ox * px + oy * py + oz * pz) * inv;
    w = (dx * qx + dy * qy + dz * qz) * inv;
    t = (e2x * qx + e2y * qy + e2z * qz) * inv;
}

// Index of the segment of a partition that holds item j: the largest m with
// off[m] <= j, for a table of M + 1 nondecreasing offsets (meshes of a batch
// over triangles, nodes or segments).
__device__ inline int32_t mesh_of(const int64_t *__restrict__ off, int32_t M, int64_t j)
{
    int32_t lo = 0, hi = M - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= j) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Order-preserving int encoding of floats for atomic min / max.
__device__ inline int32_t float_to_ordered(float f)
{
    int32_t i = __float_as_int(f);
    return i >= 0 ? i : i ^ 0x7FFFFFFF;
}
__host__ __device__ inline float ordered_to_float(int32_t i)
{
    int32_t b = i >= 0 ? i : i ^ 0x7FFFFFFF;
    union { int32_t i; float f; } u;
    u.i = b;
    return u.f;
}

}  // namespace rsi
