/*
 * rsi_oracle.c -- FP64 brute-force oracle for line-segment / triangle-mesh
 * crossing queries.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library path links, loads or calls
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline
 * leg do.  It shares no code, header or constant with the GPU implementation.
 *
 * What it computes (Section 1 of the paper states the problem): for every
 * segment l_i = (r_start, r_end) and every triangle t_j = (v_a, v_b, v_c) of
 * the mesh, whether the closed segment meets the closed triangle in a single
 * point.  The BVH of Section 2 / Section 3 only changes how fast this set is
 * found, never the set itself, so the oracle visits every (segment, triangle)
 * pair.  From the set of crossings X_i = {(j, t, u, v)} it derives
 *   - the boolean flag of Section 1 (|X_i| >= 1),
 *   - the crossing count of the `intercept_count` mode (Section 2.4),
 *   - the first hit (smallest t, ties to the smallest triangle id), which is
 *     our reading of the `barycentric` mode of Section 2.4,
 *   - the crossing list ordered by (t, id).
 *
 * Formulation.  Deliberately not Moller-Trumbore (the GPU predicate named in
 * Section 2): the decision uses signed tetrahedron volumes (the sign test of
 * Segura-Feito, one of the alternatives listed in Section 2), evaluated in
 * FP64.  Inputs are FP64 arrays; FP32 data is promoted exactly by the caller.
 *   oS = orient(v0, v1, v2, S), oE = orient(v0, v1, v2, E):
 *     both strictly of one sign -> no crossing; both zero -> coplanar, no
 *     crossing (a coplanar segment never yields a single crossing point).
 *   w0 = orient(S, E, v0, v1), w1 = orient(S, E, v1, v2),
 *   w2 = orient(S, E, v2, v0): the line through S, E passes through the
 *     closed triangle iff the three are all >= 0 or all <= 0.
 * The crossing parameters follow from the same volumes:
 *   t = oS / (oS - oE)      (fraction of the segment, S + t (E - S)),
 *   u = w2 / (w0+w1+w2)     (weight of v1),  v = w0 / (w0+w1+w2) (weight of v2),
 * i.e. P = (1-u-v) v0 + u v1 + v v2.
 *
 * A pair whose segment box and triangle box do not overlap is skipped before
 * the volumes are taken; that reject uses comparisons only and cannot change
 * the result.
 *
 * The degeneracy classifier marks segments whose answer is not decided
 * robustly by any finite-precision method: within delta of a triangle edge
 * (segment-to-segment distance), an endpoint within delta of a triangle
 * (point-to-triangle distance), or two crossings closer than delta along the
 * segment.
 *
 * The first-hit gradient is the adjoint of the crossing point of the linear
 * system S + t d = v0 + u e1 + v e2 (d = E - S, e1 = v1 - v0, e2 = v2 - v0)
 * with respect to every input coordinate, written as the inverse-transpose
 * solve of that 3x3 system.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct { double x, y, z; } dv3;

static dv3 ld(const double *p) { dv3 r = {p[0], p[1], p[2]}; return r; }
static dv3 sub(dv3 a, dv3 b) { dv3 r = {a.x - b.x, a.y - b.y, a.z - b.z}; return r; }
static dv3 add(dv3 a, dv3 b) { dv3 r = {a.x + b.x, a.y + b.y, a.z + b.z}; return r; }
static dv3 scl(dv3 a, double s) { dv3 r = {a.x * s, a.y * s, a.z * s}; return r; }
static double dot(dv3 a, dv3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static dv3 cross(dv3 a, dv3 b)
{
    dv3 r = {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
    return r;
}
/* 6 x signed volume of tetrahedron (a, b, c, d): det[b-a, c-a, d-a]. */
static double orient(dv3 a, dv3 b, dv3 c, dv3 d)
{
    return dot(sub(d, a), cross(sub(b, a), sub(c, a)));
}

/* One (segment, triangle) pair.  Returns 1 on a crossing and its t, u, v. */
static int pair_crossing(dv3 s, dv3 e, dv3 v0, dv3 v1, dv3 v2,
                         double *t, double *u, double *v)
{
    double oS = orient(v0, v1, v2, s);
    double oE = orient(v0, v1, v2, e);
    if ((oS > 0 && oE > 0) || (oS < 0 && oE < 0)) return 0;
    if (oS == 0 && oE == 0) return 0;
    double w0 = orient(s, e, v0, v1);
    double w1 = orient(s, e, v1, v2);
    double w2 = orient(s, e, v2, v0);
    int all_pos = (w0 >= 0) && (w1 >= 0) && (w2 >= 0);
    int all_neg = (w0 <= 0) && (w1 <= 0) && (w2 <= 0);
    if (!all_pos && !all_neg) return 0;
    double sw = w0 + w1 + w2;
    if (sw == 0 || oS == oE) return 0;
    *t = oS / (oS - oE);
    *u = w2 / sw;
    *v = w0 / sw;
    return 1;
}

typedef struct { double lo[3], hi[3]; } box;

static box tri_box(dv3 a, dv3 b, dv3 c)
{
    box r;
    double pa[3] = {a.x, a.y, a.z}, pb[3] = {b.x, b.y, b.z}, pc[3] = {c.x, c.y, c.z};
    for (int k = 0; k < 3; ++k) {
        r.lo[k] = fmin(pa[k], fmin(pb[k], pc[k]));
        r.hi[k] = fmax(pa[k], fmax(pb[k], pc[k]));
    }
    return r;
}

static box seg_box(dv3 s, dv3 e, double pad)
{
    box r;
    double ps[3] = {s.x, s.y, s.z}, pe[3] = {e.x, e.y, e.z};
    for (int k = 0; k < 3; ++k) {
        r.lo[k] = fmin(ps[k], pe[k]) - pad;
        r.hi[k] = fmax(ps[k], pe[k]) + pad;
    }
    return r;
}

static int boxes_overlap(const box *a, const box *b)
{
    for (int k = 0; k < 3; ++k)
        if (a->hi[k] < b->lo[k] || b->hi[k] < a->lo[k]) return 0;
    return 1;
}

typedef struct { double t, u, v; int32_t tri; } xing;

static int xing_less(const xing *a, const xing *b)
{
    if (a->t != b->t) return a->t < b->t;
    return a->tri < b->tri;
}

/* insertion sort by (t, id): lists are short */
static void sort_xings(xing *x, int n)
{
    for (int i = 1; i < n; ++i) {
        xing k = x[i];
        int j = i - 1;
        while (j >= 0 && xing_less(&k, &x[j])) { x[j + 1] = x[j]; --j; }
        x[j + 1] = k;
    }
}

typedef struct { xing *a; int n, cap; } xlist;

static void xpush(xlist *l, xing x)
{
    if (l->n == l->cap) {
        l->cap = l->cap ? 2 * l->cap : 16;
        l->a = (xing *)realloc(l->a, sizeof(xing) * (size_t)l->cap);
    }
    l->a[l->n++] = x;
}

static int check_indices(const int32_t *T, int64_t nt, int64_t nv)
{
    for (int64_t j = 0; j < 3 * nt; ++j)
        if (T[j] < 0 || T[j] >= nv) return -1;
    return 0;
}

static box *make_boxes(const double *V, const int32_t *T, int64_t nt)
{
    box *b = (box *)malloc(sizeof(box) * (size_t)(nt > 0 ? nt : 1));
    for (int64_t j = 0; j < nt; ++j)
        b[j] = tri_box(ld(V + 3 * T[3 * j]), ld(V + 3 * T[3 * j + 1]), ld(V + 3 * T[3 * j + 2]));
    return b;
}

/* All crossings of segment (s, e) against the mesh, sorted by (t, id). */
static void segment_crossings(dv3 s, dv3 e, const double *V, const int32_t *T, int64_t nt,
                              const box *tb, xlist *out)
{
    out->n = 0;
    box sb = seg_box(s, e, 0.0);
    for (int64_t j = 0; j < nt; ++j) {
        if (!boxes_overlap(&sb, &tb[j])) continue;
        double t, u, v;
        dv3 v0 = ld(V + 3 * T[3 * j]), v1 = ld(V + 3 * T[3 * j + 1]), v2 = ld(V + 3 * T[3 * j + 2]);
        if (pair_crossing(s, e, v0, v1, v2, &t, &u, &v)) {
            xing x = {t, u, v, (int32_t)j};
            xpush(out, x);
        }
    }
    sort_xings(out->a, out->n);
}

int rsi_oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Crossing query over every (segment, triangle) pair.
 *   V [nv*3] f64, T [nt*3] i32, S, E [nr*3] f64.
 *   count [nr]            number of crossings (nullable)
 *   first_tri [nr]        triangle id of the first hit, -1 on a miss (nullable)
 *   first_tuv [nr*3]      (t, u, v) of the first hit, (inf, 0, 0) on a miss (nullable)
 *   first_p [nr*3]        hit point S + t (E - S), 0 on a miss (nullable)
 *   list_tri, list_t [nr*cap]  the first `cap` crossings by (t, id); -1 / inf padding
 *   nthreads <= 0 uses the OpenMP default.
 * Returns 0, or -1 when a triangle index is out of range.
 */
int rsi_oracle_query(const double *V, int64_t nv, const int32_t *T, int64_t nt,
                     const double *S, const double *E, int64_t nr, int32_t cap,
                     int32_t *count, int32_t *first_tri, double *first_tuv, double *first_p,
                     int32_t *list_tri, double *list_t, int32_t nthreads)
{
    if (check_indices(T, nt, nv)) return -1;
    box *tb = make_boxes(V, T, nt);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        xlist xl = {0, 0, 0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < nr; ++i) {
            dv3 s = ld(S + 3 * i), e = ld(E + 3 * i);
            segment_crossings(s, e, V, T, nt, tb, &xl);
            if (count) count[i] = xl.n;
            if (first_tri) first_tri[i] = xl.n ? xl.a[0].tri : -1;
            if (first_tuv) {
                first_tuv[3 * i + 0] = xl.n ? xl.a[0].t : INFINITY;
                first_tuv[3 * i + 1] = xl.n ? xl.a[0].u : 0.0;
                first_tuv[3 * i + 2] = xl.n ? xl.a[0].v : 0.0;
            }
            if (first_p) {
                dv3 p = {0, 0, 0};
                if (xl.n) p = add(s, scl(sub(e, s), xl.a[0].t));
                first_p[3 * i + 0] = p.x;
                first_p[3 * i + 1] = p.y;
                first_p[3 * i + 2] = p.z;
            }
            if (list_tri && list_t) {
                for (int k = 0; k < cap; ++k) {
                    list_tri[(int64_t)cap * i + k] = k < xl.n ? xl.a[k].tri : -1;
                    list_t[(int64_t)cap * i + k] = k < xl.n ? xl.a[k].t : INFINITY;
                }
            }
        }
        free(xl.a);
    }
    free(tb);
    return 0;
}

/* ------------------------------------------------------------ distances -- */

/* Squared distance from p to the closed segment [a, b]. */
static double pt_seg_d2(dv3 p, dv3 a, dv3 b)
{
    dv3 ab = sub(b, a);
    double L2 = dot(ab, ab);
    double s = 0.0;
    if (L2 > 0) {
        s = dot(sub(p, a), ab) / L2;
        s = s < 0 ? 0 : (s > 1 ? 1 : s);
    }
    dv3 q = add(a, scl(ab, s));
    dv3 r = sub(p, q);
    return dot(r, r);
}

/* Squared distance between closed segments [p1, q1] and [p2, q2]: the minimum
 * is reached either at an interior pair of the two carrier lines (when both
 * line parameters fall inside [0, 1]) or with one end of a segment, so it is
 * the least of those candidates. */
static double seg_seg_d2(dv3 p1, dv3 q1, dv3 p2, dv3 q2)
{
    double best = pt_seg_d2(p1, p2, q2);
    double c;
    if ((c = pt_seg_d2(q1, p2, q2)) < best) best = c;
    if ((c = pt_seg_d2(p2, p1, q1)) < best) best = c;
    if ((c = pt_seg_d2(q2, p1, q1)) < best) best = c;
    dv3 d1 = sub(q1, p1), d2 = sub(q2, p2), r = sub(p1, p2);
    double a = dot(d1, d1), b = dot(d1, d2), e = dot(d2, d2);
    double f = dot(d1, r), g = dot(d2, r);
    double den = a * e - b * b;
    if (a > 0 && e > 0 && den > 0) {
        /* stationary point of |p1 + s d1 - p2 - t d2|^2 */
        double s = (b * g - e * f) / den;
        double t = (a * g - b * f) / den;
        if (s >= 0 && s <= 1 && t >= 0 && t <= 1) {
            dv3 w = sub(add(p1, scl(d1, s)), add(p2, scl(d2, t)));
            if ((c = dot(w, w)) < best) best = c;
        }
    }
    return best;
}

/* Squared distance from p to the closed triangle (a, b, c): the distance to
 * the plane when the foot of the perpendicular falls inside the triangle,
 * else the distance to the nearest edge. */
static double pt_tri_d2(dv3 p, dv3 a, dv3 b, dv3 c)
{
    dv3 e1 = sub(b, a), e2 = sub(c, a);
    dv3 n = cross(e1, e2);
    double nn = dot(n, n);
    if (nn > 0) {
        /* foot of the perpendicular: f = p - n ((p - a).n) / |n|^2 */
        dv3 f = sub(p, scl(n, dot(sub(p, a), n) / nn));
        /* f - a = u e1 + v e2 with u = ((f-a) x e2).n / |n|^2, v = (e1 x (f-a)).n / |n|^2 */
        double u = dot(cross(sub(f, a), e2), n) / nn;
        double v = dot(cross(e1, sub(f, a)), n) / nn;
        if (u >= 0 && v >= 0 && u + v <= 1) {
            dv3 fp = sub(p, f);
            return dot(fp, fp);
        }
    }
    double best = pt_seg_d2(p, a, b), d;
    if ((d = pt_seg_d2(p, b, c)) < best) best = d;
    if ((d = pt_seg_d2(p, c, a)) < best) best = d;
    return best;
}

/* Exported for the distance pins in the tests. */
double rsi_oracle_seg_seg_dist(const double *p1, const double *q1, const double *p2, const double *q2)
{
    dv3 a = {p1[0], p1[1], p1[2]}, b = {q1[0], q1[1], q1[2]};
    dv3 c = {p2[0], p2[1], p2[2]}, d = {q2[0], q2[1], q2[2]};
    return sqrt(seg_seg_d2(a, b, c, d));
}

double rsi_oracle_pt_tri_dist(const double *p, const double *a, const double *b, const double *c)
{
    dv3 P = {p[0], p[1], p[2]}, A = {a[0], a[1], a[2]}, B = {b[0], b[1], b[2]}, C = {c[0], c[1], c[2]};
    return sqrt(pt_tri_d2(P, A, B, C));
}

/*
 * Degeneracy flags per segment (bit mask):
 *   1  some triangle edge lies within delta of the segment,
 *   2  an endpoint lies within delta of some triangle,
 *   4  two crossings lie within delta of each other along the segment.
 * Returns 0, or -1 on an out-of-range index.
 */
int rsi_oracle_degenerate(const double *V, int64_t nv, const int32_t *T, int64_t nt,
                          const double *S, const double *E, int64_t nr, double delta,
                          uint8_t *flags, int32_t nthreads)
{
    if (check_indices(T, nt, nv)) return -1;
    box *tb = make_boxes(V, T, nt);
    double d2 = delta * delta;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        xlist xl = {0, 0, 0};
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < nr; ++i) {
            dv3 s = ld(S + 3 * i), e = ld(E + 3 * i);
            box sb = seg_box(s, e, delta);
            uint8_t f = 0;
            for (int64_t j = 0; j < nt && f != 3; ++j) {
                if (!boxes_overlap(&sb, &tb[j])) continue;
                dv3 v0 = ld(V + 3 * T[3 * j]), v1 = ld(V + 3 * T[3 * j + 1]), v2 = ld(V + 3 * T[3 * j + 2]);
                if (!(f & 1)) {
                    if (seg_seg_d2(s, e, v0, v1) <= d2 || seg_seg_d2(s, e, v1, v2) <= d2 ||
                        seg_seg_d2(s, e, v2, v0) <= d2)
                        f |= 1;
                }
                if (!(f & 2)) {
                    if (pt_tri_d2(s, v0, v1, v2) <= d2 || pt_tri_d2(e, v0, v1, v2) <= d2) f |= 2;
                }
            }
            segment_crossings(s, e, V, T, nt, tb, &xl);
            double len = sqrt(dot(sub(e, s), sub(e, s)));
            for (int k = 1; k < xl.n; ++k)
                if ((xl.a[k].t - xl.a[k - 1].t) * len <= delta) f |= 4;
            flags[i] = f;
        }
        free(xl.a);
    }
    free(tb);
    return 0;
}

/* ------------------------------------------------------------ gradient -- */

/* Solve A x = b for a 3x3 matrix given by columns c0, c1, c2 (Cramer). */
static int solve3(dv3 c0, dv3 c1, dv3 c2, dv3 b, dv3 *x)
{
    double D = dot(c0, cross(c1, c2));
    if (D == 0) return 0;
    x->x = dot(b, cross(c1, c2)) / D;
    x->y = dot(c0, cross(b, c2)) / D;
    x->z = dot(c0, cross(c1, b)) / D;
    return 1;
}

/* Solve A^T y = g with A = [c0 | c1 | c2]: the rows of A^T are c0, c1, c2. */
static int solve3_transpose(dv3 c0, dv3 c1, dv3 c2, dv3 g, dv3 *y)
{
    /* A^T has columns (c0.x, c1.x, c2.x), (c0.y, c1.y, c2.y), (c0.z, c1.z, c2.z) */
    dv3 k0 = {c0.x, c1.x, c2.x}, k1 = {c0.y, c1.y, c2.y}, k2 = {c0.z, c1.z, c2.z};
    return solve3(k0, k1, k2, g, y);
}

/*
 * First-hit adjoint.  For each segment i with first hit on triangle
 * tri[i] (-1: miss, contributes nothing), given upstream gradients
 *   g_t [nr], g_uv [nr*2], g_p [nr*3]  (each nullable = zero),
 * accumulates dL/dV into dV [nv*3] and writes dL/dS, dL/dE [nr*3]; dV_abs
 * (nullable) accumulates the absolute value of every contribution.
 * The hit solves M x = S - v0, M = [-d | e1 | e2], x = (t, u, v),
 * d = E - S, e1 = v1 - v0, e2 = v2 - v0, and P = S + t d.
 * With tbar the gradient on t after folding P in (tbar += Pbar.d) and
 *   lambda = M^{-T} (tbar, ubar, vbar),
 * the implicit-function rule on M x - (S - v0) = 0 gives
 *   dL/dS  = (1 - t) (lambda + Pbar),   dL/dE = t (lambda + Pbar),
 *   dL/dv0 += -(1 - u - v) lambda,  dL/dv1 += -u lambda,  dL/dv2 += -v lambda.
 * Serial over segments so that dV is summed in a fixed order.
 */
int rsi_oracle_first_hit_grad(const double *V, int64_t nv, const int32_t *T, int64_t nt,
                              const double *S, const double *E, int64_t nr,
                              const int32_t *tri, const double *tuv,
                              const double *g_t, const double *g_uv, const double *g_p,
                              double *dV, double *dS, double *dE, double *dV_abs)
{
    if (check_indices(T, nt, nv)) return -1;
    for (int64_t i = 0; i < nr; ++i) {
        dv3 zero = {0, 0, 0};
        dv3 gs = zero, ge = zero;
        int32_t j = tri[i];
        if (j >= 0 && j < nt) {
            dv3 s = ld(S + 3 * i), e = ld(E + 3 * i);
            dv3 v0 = ld(V + 3 * T[3 * j]), v1 = ld(V + 3 * T[3 * j + 1]), v2 = ld(V + 3 * T[3 * j + 2]);
            dv3 d = sub(e, s), e1 = sub(v1, v0), e2 = sub(v2, v0);
            double t = tuv[3 * i], u = tuv[3 * i + 1], v = tuv[3 * i + 2];
            dv3 pbar = g_p ? (dv3){g_p[3 * i], g_p[3 * i + 1], g_p[3 * i + 2]} : zero;
            /* P = S + t d: fold its gradient into t, S and d */
            double tbar = (g_t ? g_t[i] : 0.0) + dot(pbar, d);
            double ubar = g_uv ? g_uv[2 * i] : 0.0;
            double vbar = g_uv ? g_uv[2 * i + 1] : 0.0;
            dv3 dbar = scl(pbar, t);
            gs = pbar;
            dv3 xbar = {tbar, ubar, vbar};
            dv3 lam;
            dv3 md = scl(d, -1.0);
            if (solve3_transpose(md, e1, e2, xbar, &lam)) {
                /* residual r(x, inputs) = M x - (S - v0) = 0
                 * d x = -M^{-1} (dM x - dS + dv0); L-bar on inputs = -lam^T (dM x - dS + dv0) */
                gs = add(gs, lam);                       /* rhs S */
                dv3 v0bar = scl(lam, -1.0);              /* rhs -v0 */
                /* dM x = -dd t + de1 u + de2 v */
                dbar = add(dbar, scl(lam, t));           /* -(-t) lam */
                dv3 e1bar = scl(lam, -u);
                dv3 e2bar = scl(lam, -v);
                /* e1 = v1 - v0, e2 = v2 - v0 */
                v0bar = sub(v0bar, add(e1bar, e2bar));
                dv3 v1bar = e1bar, v2bar = e2bar;
                int32_t a = T[3 * j], b = T[3 * j + 1], c = T[3 * j + 2];
                dV[3 * a] += v0bar.x; dV[3 * a + 1] += v0bar.y; dV[3 * a + 2] += v0bar.z;
                dV[3 * b] += v1bar.x; dV[3 * b + 1] += v1bar.y; dV[3 * b + 2] += v1bar.z;
                dV[3 * c] += v2bar.x; dV[3 * c + 1] += v2bar.y; dV[3 * c + 2] += v2bar.z;
                if (dV_abs) {  /* sum of |contribution| per element: the scale of its rounding */
                    dV_abs[3 * a] += fabs(v0bar.x); dV_abs[3 * a + 1] += fabs(v0bar.y); dV_abs[3 * a + 2] += fabs(v0bar.z);
                    dV_abs[3 * b] += fabs(v1bar.x); dV_abs[3 * b + 1] += fabs(v1bar.y); dV_abs[3 * b + 2] += fabs(v1bar.z);
                    dV_abs[3 * c] += fabs(v2bar.x); dV_abs[3 * c + 1] += fabs(v2bar.y); dV_abs[3 * c + 2] += fabs(v2bar.z);
                }
            }
            /* d = E - S */
            ge = dbar;
            gs = sub(gs, dbar);
        }
        if (dS) { dS[3 * i] = gs.x; dS[3 * i + 1] = gs.y; dS[3 * i + 2] = gs.z; }
        if (dE) { dE[3 * i] = ge.x; dE[3 * i + 1] = ge.y; dE[3 * i + 2] = ge.z; }
    }
    return 0;
}
