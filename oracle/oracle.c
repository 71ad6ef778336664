/*
 * oracle.c -- plain, slow, FP64 reference for compressed-BVH collision
 * detection and proximity queries (Tan, Weller, Zachmann, "Compressed
 * Bounding Volume Hierarchies for Collision Detection & Proximity Query").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may call, link or
 * load this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the GPU path.
 *
 * What is here, and the passage each part follows:
 *   - Simultaneous recursive BVH traversal exactly in the shape of the
 *     paper's Algorithm 1 (BVHtraversal(a, b): both leaves -> check the
 *     primitives; one leaf -> recurse over the other node's children whose
 *     BV intersects it; otherwise recurse over every intersecting child
 *     pair), over the oracle's own uncompressed FP64 binary AABB tree.
 *     The root pair is tested before the first call (the algorithm starts
 *     inside an already-overlapping pair).
 *   - BV overlap and BV distance lower bound ("faster overlap or separation
 *     distance test", Introduction): A's box placed by the pose is an
 *     oriented box in B's frame; the 15-axis separating-axis test decides
 *     overlap, the largest gap over the same axes bounds the distance.
 *   - checkPrimitives: closed triangle-triangle intersection, three
 *     independent FP64 formulations (separating axes, edge-pierces-triangle,
 *     intervals on the planes' intersection line), and triangle-triangle
 *     distance (6 point-triangle + 9 segment-segment closest-point problems).
 *   - Proximity query as branch-and-bound over Algorithm 1: a child pair is
 *     visited only while its BV lower bound is below the best distance.
 *   - Input validity: penetration depth over the 11 separating axes, and the
 *     margin classification used to reject near-contact poses.
 *   - An independent parser/decoder of the compressed BVH blob (quantized
 *     BV descriptors predicted from the decoded parent, the paper's
 *     "predictor-corrector" compression with predictors from the chain of
 *     ancestors, section III; treelet tops stored absolute) and checks of
 *     its invariants.
 *
 * Build: gcc -O2 -std=c11 -fPIC -shared -ffp-contract=off -fno-fast-math -pthread
 */
#define _GNU_SOURCE
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define EXPORT __attribute__((visibility("default")))

/* ------------------------------------------------------------------ */
/* small FP64 vector helpers                                           */
/* ------------------------------------------------------------------ */
typedef double v3[3];

static inline void vsub(const double *a, const double *b, double *o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static inline void vadd(const double *a, const double *b, double *o) { o[0] = a[0] + b[0]; o[1] = a[1] + b[1]; o[2] = a[2] + b[2]; }
static inline void vscale(const double *a, double s, double *o) { o[0] = a[0] * s; o[1] = a[1] * s; o[2] = a[2] * s; }
static inline double vdot(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static inline void vcross(const double *a, const double *b, double *o)
{
    double x = a[1] * b[2] - a[2] * b[1];
    double y = a[2] * b[0] - a[0] * b[2];
    double z = a[0] * b[1] - a[1] * b[0];
    o[0] = x; o[1] = y; o[2] = z;
}
static inline double vnorm2(const double *a) { return vdot(a, a); }
static inline double dmin(double a, double b) { return a < b ? a : b; }
static inline double dmax(double a, double b) { return a > b ? a : b; }
static inline double clamp01(double x) { return x < 0.0 ? 0.0 : (x > 1.0 ? 1.0 : x); }

/* the pose [R | t] (row-major float32 3x4) promoted to FP64 */
typedef struct { double R[3][3]; double t[3]; } pose_t;

static void pose_from(const float *p, pose_t *o)
{
    for (int i = 0; i < 3; i++) {
        for (int j = 0; j < 3; j++) o->R[i][j] = (double)p[4 * i + j];
        o->t[i] = (double)p[4 * i + 3];
    }
}

static inline void pose_apply(const pose_t *P, const double *x, double *o)
{
    double r[3];
    for (int i = 0; i < 3; i++) r[i] = P->R[i][0] * x[0] + P->R[i][1] * x[1] + P->R[i][2] * x[2] + P->t[i];
    o[0] = r[0]; o[1] = r[1]; o[2] = r[2];
}

/* ------------------------------------------------------------------ */
/* triangle-triangle intersection, formulation 1: separating axes      */
/* ------------------------------------------------------------------ */
/* Closed triangles are disjoint iff some axis among the two face normals,
 * the 9 edge-edge cross products and the 6 in-plane edge normals separates
 * their projections.  Axes that degenerate (parallel edges) are skipped. */
static int axis_separates(const v3 *a, const v3 *b, const double *L)
{
    double pa0 = vdot(a[0], L), pa1 = vdot(a[1], L), pa2 = vdot(a[2], L);
    double pb0 = vdot(b[0], L), pb1 = vdot(b[1], L), pb2 = vdot(b[2], L);
    double amin = dmin(pa0, dmin(pa1, pa2)), amax = dmax(pa0, dmax(pa1, pa2));
    double bmin = dmin(pb0, dmin(pb1, pb2)), bmax = dmax(pb0, dmax(pb1, pb2));
    return amax < bmin || bmax < amin;
}

static int degenerate_axis(const double *L, double ref2)
{
    return vnorm2(L) <= 1e-24 * ref2;
}

EXPORT int orc_tt_sat(const double *a9, const double *b9)
{
    const v3 *a = (const v3 *)a9, *b = (const v3 *)b9;
    v3 ea[3], eb[3], na, nb, L;
    for (int i = 0; i < 3; i++) { vsub(a[(i + 1) % 3], a[i], ea[i]); vsub(b[(i + 1) % 3], b[i], eb[i]); }
    vcross(ea[0], ea[1], na);
    vcross(eb[0], eb[1], nb);
    if (!degenerate_axis(na, vnorm2(ea[0]) * vnorm2(ea[1])) && axis_separates(a, b, na)) return 0;
    if (!degenerate_axis(nb, vnorm2(eb[0]) * vnorm2(eb[1])) && axis_separates(a, b, nb)) return 0;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            vcross(ea[i], eb[j], L);
            if (!degenerate_axis(L, vnorm2(ea[i]) * vnorm2(eb[j])) && axis_separates(a, b, L)) return 0;
        }
    for (int i = 0; i < 3; i++) {
        vcross(na, ea[i], L);
        if (!degenerate_axis(L, vnorm2(na) * vnorm2(ea[i])) && axis_separates(a, b, L)) return 0;
        vcross(nb, eb[i], L);
        if (!degenerate_axis(L, vnorm2(nb) * vnorm2(eb[i])) && axis_separates(a, b, L)) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------ */
/* formulation 2: some edge of one triangle meets the other triangle   */
/* ------------------------------------------------------------------ */
static double orient3(const double *a, const double *b, const double *c, const double *d)
{
    v3 u, v, w, n;
    vsub(b, a, u); vsub(c, a, v); vsub(d, a, w);
    vcross(u, v, n);
    return vdot(n, w);
}

static double orient2(const double *a, const double *b, const double *c)
{
    return (b[0] - a[0]) * (c[1] - a[1]) - (b[1] - a[1]) * (c[0] - a[0]);
}

static int seg_seg_2d(const double *p, const double *q, const double *r, const double *s)
{
    double o1 = orient2(p, q, r), o2 = orient2(p, q, s), o3 = orient2(r, s, p), o4 = orient2(r, s, q);
    if (((o1 > 0 && o2 < 0) || (o1 < 0 && o2 > 0)) && ((o3 > 0 && o4 < 0) || (o3 < 0 && o4 > 0))) return 1;
    /* collinear touching cases: an endpoint lies on the other segment */
#define ONSEG(a, b, c) (dmin(a[0], b[0]) <= c[0] && c[0] <= dmax(a[0], b[0]) && dmin(a[1], b[1]) <= c[1] && c[1] <= dmax(a[1], b[1]))
    if (o1 == 0 && ONSEG(p, q, r)) return 1;
    if (o2 == 0 && ONSEG(p, q, s)) return 1;
    if (o3 == 0 && ONSEG(r, s, p)) return 1;
    if (o4 == 0 && ONSEG(r, s, q)) return 1;
#undef ONSEG
    return 0;
}

static int point_in_tri_2d(const double *p, const double *a, const double *b, const double *c)
{
    double d1 = orient2(a, b, p), d2 = orient2(b, c, p), d3 = orient2(c, a, p);
    int neg = (d1 < 0) || (d2 < 0) || (d3 < 0);
    int pos = (d1 > 0) || (d2 > 0) || (d3 > 0);
    return !(neg && pos);
}

/* drop the coordinate of largest |n| component */
static void project2(const double *x, int drop, double *o)
{
    int i0 = drop == 0 ? 1 : 0, i1 = drop == 2 ? 1 : 2;
    o[0] = x[i0]; o[1] = x[i1];
}

static int dominant_axis(const double *n)
{
    double ax = fabs(n[0]), ay = fabs(n[1]), az = fabs(n[2]);
    return (ax >= ay && ax >= az) ? 0 : (ay >= az ? 1 : 2);
}

static int seg_tri_3d(const double *p, const double *q, const v3 *t)
{
    double dp = orient3(t[0], t[1], t[2], p), dq = orient3(t[0], t[1], t[2], q);
    if ((dp > 0 && dq > 0) || (dp < 0 && dq < 0)) return 0;
    if (dp == 0 && dq == 0) {
        v3 e1, e2, n;
        vsub(t[1], t[0], e1); vsub(t[2], t[0], e2); vcross(e1, e2, n);
        int d = dominant_axis(n);
        double p2[2], q2[2], a2[2], b2[2], c2[2];
        project2(p, d, p2); project2(q, d, q2); project2(t[0], d, a2); project2(t[1], d, b2); project2(t[2], d, c2);
        if (point_in_tri_2d(p2, a2, b2, c2) || point_in_tri_2d(q2, a2, b2, c2)) return 1;
        return seg_seg_2d(p2, q2, a2, b2) || seg_seg_2d(p2, q2, b2, c2) || seg_seg_2d(p2, q2, c2, a2);
    }
    double s1 = orient3(p, q, t[0], t[1]), s2 = orient3(p, q, t[1], t[2]), s3 = orient3(p, q, t[2], t[0]);
    return (s1 >= 0 && s2 >= 0 && s3 >= 0) || (s1 <= 0 && s2 <= 0 && s3 <= 0);
}

EXPORT int orc_tt_segtri(const double *a9, const double *b9)
{
    const v3 *a = (const v3 *)a9, *b = (const v3 *)b9;
    for (int i = 0; i < 3; i++) {
        if (seg_tri_3d(a[i], a[(i + 1) % 3], b)) return 1;
        if (seg_tri_3d(b[i], b[(i + 1) % 3], a)) return 1;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* formulation 3: intervals on the line where the two planes meet      */
/* ------------------------------------------------------------------ */
static int coplanar_tri_tri(const double *n, const v3 *a, const v3 *b)
{
    int d = dominant_axis(n);
    double A[3][2], B[3][2];
    for (int i = 0; i < 3; i++) { project2(a[i], d, A[i]); project2(b[i], d, B[i]); }
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            if (seg_seg_2d(A[i], A[(i + 1) % 3], B[j], B[(j + 1) % 3])) return 1;
    if (point_in_tri_2d(A[0], B[0], B[1], B[2])) return 1;
    if (point_in_tri_2d(B[0], A[0], A[1], A[2])) return 1;
    return 0;
}

/* Parameter interval where a triangle with projections pr[] onto the line
 * direction and signed plane distances dd[] (of the other plane) meets that
 * plane.  Exactly one vertex lies on its own side (or the only non-zero). */
static void line_interval(const double *pr, const double *dd, double *lo, double *hi)
{
    int k;
    if (dd[0] * dd[1] > 0) k = 2;
    else if (dd[0] * dd[2] > 0) k = 1;
    else if (dd[1] * dd[2] > 0 || dd[0] != 0) k = 0;
    else if (dd[1] != 0) k = 1;
    else k = 2;
    int i = (k + 1) % 3, j = (k + 2) % 3;
    double t0 = pr[k] + (pr[i] - pr[k]) * dd[k] / (dd[k] - dd[i]);
    double t1 = pr[k] + (pr[j] - pr[k]) * dd[k] / (dd[k] - dd[j]);
    if (dd[k] - dd[i] == 0) t0 = pr[i];
    if (dd[k] - dd[j] == 0) t1 = pr[j];
    *lo = dmin(t0, t1);
    *hi = dmax(t0, t1);
}

EXPORT int orc_tt_interval(const double *a9, const double *b9)
{
    const v3 *a = (const v3 *)a9, *b = (const v3 *)b9;
    v3 e1, e2, na, nb, D;
    vsub(b[1], b[0], e1); vsub(b[2], b[0], e2); vcross(e1, e2, nb);
    double da[3];
    for (int i = 0; i < 3; i++) { v3 w; vsub(a[i], b[0], w); da[i] = vdot(nb, w); }
    if ((da[0] > 0 && da[1] > 0 && da[2] > 0) || (da[0] < 0 && da[1] < 0 && da[2] < 0)) return 0;
    vsub(a[1], a[0], e1); vsub(a[2], a[0], e2); vcross(e1, e2, na);
    double db[3];
    for (int i = 0; i < 3; i++) { v3 w; vsub(b[i], a[0], w); db[i] = vdot(na, w); }
    if ((db[0] > 0 && db[1] > 0 && db[2] > 0) || (db[0] < 0 && db[1] < 0 && db[2] < 0)) return 0;
    if (da[0] == 0 && da[1] == 0 && da[2] == 0) return coplanar_tri_tri(na, a, b);
    vcross(na, nb, D);
    double pa[3], pb[3];
    for (int i = 0; i < 3; i++) { pa[i] = vdot(D, a[i]); pb[i] = vdot(D, b[i]); }
    double alo, ahi, blo, bhi;
    line_interval(pa, da, &alo, &ahi);
    line_interval(pb, db, &blo, &bhi);
    return !(ahi < blo || bhi < alo);
}

/* ------------------------------------------------------------------ */
/* triangle-triangle distance                                          */
/* ------------------------------------------------------------------ */
/* closest point of triangle t to p: classify p against the Voronoi regions
 * of the vertices, edges and face (barycentric region tests); the textbook
 * method of Ericson, Real-Time Collision Detection (2005), section 5.1.5 */
static void closest_pt_tri(const double *p, const v3 *t, double *out)
{
    v3 ab, ac, ap, bp, cp;
    vsub(t[1], t[0], ab); vsub(t[2], t[0], ac); vsub(p, t[0], ap);
    double d1 = vdot(ab, ap), d2 = vdot(ac, ap);
    if (d1 <= 0 && d2 <= 0) { memcpy(out, t[0], sizeof(v3)); return; }
    vsub(p, t[1], bp);
    double d3 = vdot(ab, bp), d4 = vdot(ac, bp);
    if (d3 >= 0 && d4 <= d3) { memcpy(out, t[1], sizeof(v3)); return; }
    double vc = d1 * d4 - d3 * d2;
    if (vc <= 0 && d1 >= 0 && d3 <= 0) {
        double v = d1 / (d1 - d3);
        for (int k = 0; k < 3; k++) out[k] = t[0][k] + v * ab[k];
        return;
    }
    vsub(p, t[2], cp);
    double d5 = vdot(ab, cp), d6 = vdot(ac, cp);
    if (d6 >= 0 && d5 <= d6) { memcpy(out, t[2], sizeof(v3)); return; }
    double vb = d5 * d2 - d1 * d6;
    if (vb <= 0 && d2 >= 0 && d6 <= 0) {
        double w = d2 / (d2 - d6);
        for (int k = 0; k < 3; k++) out[k] = t[0][k] + w * ac[k];
        return;
    }
    double va = d3 * d6 - d5 * d4;
    if (va <= 0 && (d4 - d3) >= 0 && (d5 - d6) >= 0) {
        double w = (d4 - d3) / ((d4 - d3) + (d5 - d6));
        for (int k = 0; k < 3; k++) out[k] = t[1][k] + w * (t[2][k] - t[1][k]);
        return;
    }
    double den = 1.0 / (va + vb + vc);
    double v = vb * den, w = vc * den;
    for (int k = 0; k < 3; k++) out[k] = t[0][k] + ab[k] * v + ac[k] * w;
}

EXPORT double orc_pt_tri_dist(const double *p, const double *t9)
{
    v3 c, d;
    closest_pt_tri(p, (const v3 *)t9, c);
    vsub(p, c, d);
    return sqrt(vnorm2(d));
}

/* squared distance between segments p1q1 and p2q2 (minimise the convex
 * quadratic |P(s) - Q(t)|^2 over [0,1]^2: interior stationary point when the
 * segments are not parallel, then clamp and re-solve for the other
 * parameter; Ericson, Real-Time Collision Detection, section 5.1.9) */
static double seg_seg_dist2(const double *p1, const double *q1, const double *p2, const double *q2)
{
    v3 d1, d2, r;
    vsub(q1, p1, d1); vsub(q2, p2, d2); vsub(p1, p2, r);
    double a = vdot(d1, d1), e = vdot(d2, d2), f = vdot(d2, r);
    double s, t;
    if (a <= 1e-300 && e <= 1e-300) { return vnorm2(r); }
    if (a <= 1e-300) { s = 0; t = clamp01(f / e); }
    else {
        double c = vdot(d1, r);
        if (e <= 1e-300) { t = 0; s = clamp01(-c / a); }
        else {
            double b = vdot(d1, d2), den = a * e - b * b;
            s = den > 0 ? clamp01((b * f - c * e) / den) : 0.0;
            t = (b * s + f) / e;
            if (t < 0) { t = 0; s = clamp01(-c / a); }
            else if (t > 1) { t = 1; s = clamp01((b - c) / a); }
        }
    }
    v3 c1, c2, w;
    for (int k = 0; k < 3; k++) { c1[k] = p1[k] + d1[k] * s; c2[k] = p2[k] + d2[k] * t; }
    vsub(c1, c2, w);
    return vnorm2(w);
}

EXPORT double orc_seg_seg_dist(const double *p1, const double *q1, const double *p2, const double *q2)
{
    return sqrt(seg_seg_dist2(p1, q1, p2, q2));
}

/* distance between closed triangles: 0 if they intersect, else the smallest
 * of the 6 vertex-to-triangle and 9 edge-to-edge distances */
EXPORT double orc_tt_dist(const double *a9, const double *b9)
{
    const v3 *a = (const v3 *)a9, *b = (const v3 *)b9;
    if (orc_tt_sat(a9, b9)) return 0.0;
    double best = INFINITY;
    for (int i = 0; i < 3; i++) {
        best = dmin(best, orc_pt_tri_dist(a[i], b9));
        best = dmin(best, orc_pt_tri_dist(b[i], a9));
    }
    double best2 = best * best;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            best2 = dmin(best2, seg_seg_dist2(a[i], a[(i + 1) % 3], b[j], b[(j + 1) % 3]));
    return sqrt(best2);
}

/* penetration depth of intersecting triangles: smallest translation overlap
 * over the unit face normals and unit edge-edge cross products */
EXPORT double orc_tt_pd(const double *a9, const double *b9)
{
    const v3 *a = (const v3 *)a9, *b = (const v3 *)b9;
    v3 ea[3], eb[3], ax[11];
    int n = 0;
    for (int i = 0; i < 3; i++) { vsub(a[(i + 1) % 3], a[i], ea[i]); vsub(b[(i + 1) % 3], b[i], eb[i]); }
    vcross(ea[0], ea[1], ax[n]); if (!degenerate_axis(ax[n], vnorm2(ea[0]) * vnorm2(ea[1]))) n++;
    vcross(eb[0], eb[1], ax[n]); if (!degenerate_axis(ax[n], vnorm2(eb[0]) * vnorm2(eb[1]))) n++;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            vcross(ea[i], eb[j], ax[n]);
            if (!degenerate_axis(ax[n], vnorm2(ea[i]) * vnorm2(eb[j]))) n++;
        }
    double pd = INFINITY;
    for (int k = 0; k < n; k++) {
        double inv = 1.0 / sqrt(vnorm2(ax[k]));
        double amin = INFINITY, amax = -INFINITY, bmin = INFINITY, bmax = -INFINITY;
        for (int i = 0; i < 3; i++) {
            double pa = vdot(a[i], ax[k]) * inv, pb = vdot(b[i], ax[k]) * inv;
            amin = dmin(amin, pa); amax = dmax(amax, pa); bmin = dmin(bmin, pb); bmax = dmax(bmax, pb);
        }
        pd = dmin(pd, dmin(amax - bmin, bmax - amin));
    }
    return pd;
}

/* signed separation: distance if disjoint, minus penetration depth if not */
EXPORT double orc_tt_signed(const double *a9, const double *b9)
{
    if (orc_tt_sat(a9, b9)) return -orc_tt_pd(a9, b9);
    return orc_tt_dist(a9, b9);
}

/* ------------------------------------------------------------------ */
/* the oracle's own BVH: binary AABB tree in FP64, one triangle per leaf */
/* ------------------------------------------------------------------ */
typedef struct {
    double lo[3], hi[3];
    int32_t left, right; /* children; left < 0 marks a leaf holding triangle -left-1 */
} onode_t;

typedef struct {
    uint32_t nt;
    double *tri;      /* [nt][9], FP64 copy of the input triangles */
    onode_t *node;
    int32_t nnode;
} omesh_t;

typedef struct { double key; uint32_t idx; } keyidx_t;

static int cmp_keyidx(const void *x, const void *y)
{
    const keyidx_t *a = x, *b = y;
    if (a->key < b->key) return -1;
    if (a->key > b->key) return 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

static int32_t build_rec(omesh_t *m, uint32_t *idx, uint32_t n, keyidx_t *tmp)
{
    int32_t me = m->nnode++;
    onode_t *nd = &m->node[me];
    for (int k = 0; k < 3; k++) { nd->lo[k] = INFINITY; nd->hi[k] = -INFINITY; }
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t i = 0; i < n; i++) {
        const double *t = &m->tri[9 * (size_t)idx[i]];
        for (int v = 0; v < 3; v++)
            for (int k = 0; k < 3; k++) {
                nd->lo[k] = dmin(nd->lo[k], t[3 * v + k]);
                nd->hi[k] = dmax(nd->hi[k], t[3 * v + k]);
            }
        for (int k = 0; k < 3; k++) {
            double c = (t[k] + t[3 + k] + t[6 + k]) / 3.0;
            clo[k] = dmin(clo[k], c); chi[k] = dmax(chi[k], c);
        }
    }
    if (n == 1) { nd->left = -1 - (int32_t)idx[0]; nd->right = -1; return me; }
    int ax = 0;
    for (int k = 1; k < 3; k++) if (chi[k] - clo[k] > chi[ax] - clo[ax]) ax = k;
    for (uint32_t i = 0; i < n; i++) {
        const double *t = &m->tri[9 * (size_t)idx[i]];
        tmp[i].key = t[ax] + t[3 + ax] + t[6 + ax];
        tmp[i].idx = idx[i];
    }
    qsort(tmp, n, sizeof(keyidx_t), cmp_keyidx);
    for (uint32_t i = 0; i < n; i++) idx[i] = tmp[i].idx;
    uint32_t h = n / 2;
    int32_t l = build_rec(m, idx, h, tmp);
    int32_t r = build_rec(m, idx + h, n - h, tmp);
    m->node[me].left = l;
    m->node[me].right = r;
    return me;
}

EXPORT void *orc_mesh_new(const float *V, uint32_t nv, const uint32_t *T, uint32_t nt)
{
    if (nt == 0) return NULL;
    for (uint32_t i = 0; i < 3 * nt; i++) if (T[i] >= nv) return NULL;
    omesh_t *m = calloc(1, sizeof(omesh_t));
    m->nt = nt;
    m->tri = malloc(sizeof(double) * 9 * (size_t)nt);
    for (uint32_t i = 0; i < nt; i++)
        for (int v = 0; v < 3; v++)
            for (int k = 0; k < 3; k++) m->tri[9 * (size_t)i + 3 * v + k] = (double)V[3 * (size_t)T[3 * (size_t)i + v] + k];
    m->node = malloc(sizeof(onode_t) * (2 * (size_t)nt));
    uint32_t *idx = malloc(sizeof(uint32_t) * nt);
    keyidx_t *tmp = malloc(sizeof(keyidx_t) * nt);
    for (uint32_t i = 0; i < nt; i++) idx[i] = i;
    build_rec(m, idx, nt, tmp);
    free(idx); free(tmp);
    return m;
}

EXPORT void orc_mesh_free(void *p)
{
    omesh_t *m = p;
    if (!m) return;
    free(m->tri); free(m->node); free(m);
}

/* ------------------------------------------------------------------ */
/* BV tests: A's box as an oriented box in B's frame vs B's box         */
/* ------------------------------------------------------------------ */
typedef struct {
    double gap;   /* largest normalised gap over the 15 axes (<= 0: no axis separates) */
} boxsep_t;

/* largest separation along the 15 candidate axes (face axes of both boxes
 * and their 9 cross products), normalised by the axis length */
static double box_gap(const pose_t *P, const onode_t *a, const onode_t *b)
{
    double ca[3], ea[3], cb[3], eb[3], c[3], T[3];
    for (int k = 0; k < 3; k++) {
        ca[k] = 0.5 * (a->lo[k] + a->hi[k]); ea[k] = 0.5 * (a->hi[k] - a->lo[k]);
        cb[k] = 0.5 * (b->lo[k] + b->hi[k]); eb[k] = 0.5 * (b->hi[k] - b->lo[k]);
    }
    pose_apply(P, ca, c);
    vsub(c, cb, T);
    /* columns of R are A's axes expressed in B's frame */
    double ax[3][3];
    for (int j = 0; j < 3; j++) for (int i = 0; i < 3; i++) ax[j][i] = P->R[i][j];
    double best = -INFINITY;
    double L[3];
    for (int n = 0; n < 15; n++) {
        if (n < 3) { L[0] = L[1] = L[2] = 0; L[n] = 1; }
        else if (n < 6) { memcpy(L, ax[n - 3], sizeof L); }
        else { double e[3] = {0, 0, 0}; e[(n - 6) / 3] = 1; vcross(e, ax[(n - 6) % 3], L); }
        double len = sqrt(vnorm2(L));
        if (len < 1e-12) continue;
        double rb = eb[0] * fabs(L[0]) + eb[1] * fabs(L[1]) + eb[2] * fabs(L[2]);
        double ra = ea[0] * fabs(vdot(ax[0], L)) + ea[1] * fabs(vdot(ax[1], L)) + ea[2] * fabs(vdot(ax[2], L));
        double g = (fabs(vdot(T, L)) - ra - rb) / len;
        if (g > best) best = g;
    }
    return best;
}

/* relative slack so that rounding in the FP64 box test never culls a
 * touching pair: scale of the coordinates involved x 1e-9 */
static double box_slack(const pose_t *P, const onode_t *a, const onode_t *b)
{
    double s = fabs(P->t[0]) + fabs(P->t[1]) + fabs(P->t[2]);
    for (int k = 0; k < 3; k++) s += fabs(a->lo[k]) + fabs(a->hi[k]) + fabs(b->lo[k]) + fabs(b->hi[k]);
    return 1e-9 * s;
}

static inline int bv_overlap(const pose_t *P, const onode_t *a, const onode_t *b, double dilate)
{
    return box_gap(P, a, b) <= dilate + box_slack(P, a, b);
}

/* distance lower bound of two boxes: the larger of the largest axis gap and
 * the gap between their circumscribed spheres (both are lower bounds) */
static inline double bv_lower_bound(const pose_t *P, const onode_t *a, const onode_t *b)
{
    double ca[3], cb[3], c[3], d[3], ra = 0, rb = 0;
    for (int k = 0; k < 3; k++) {
        ca[k] = 0.5 * (a->lo[k] + a->hi[k]); cb[k] = 0.5 * (b->lo[k] + b->hi[k]);
        ra += 0.25 * (a->hi[k] - a->lo[k]) * (a->hi[k] - a->lo[k]);
        rb += 0.25 * (b->hi[k] - b->lo[k]) * (b->hi[k] - b->lo[k]);
    }
    pose_apply(P, ca, c);
    vsub(c, cb, d);
    double gs = sqrt(vnorm2(d)) - sqrt(ra) - sqrt(rb);
    double g = dmax(box_gap(P, a, b), gs) - box_slack(P, a, b);
    return g > 0 ? g : 0.0;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1 for collision                                            */
/* ------------------------------------------------------------------ */
typedef struct {
    const omesh_t *A, *B;
    pose_t P;
    int early_exit;
    int hit;
    uint32_t *pairs; uint64_t cap, n;
    uint64_t bv_tests, tri_tests;
} cstate_t;

static int is_leaf(const onode_t *n) { return n->left < 0; }

static void check_primitives(cstate_t *s, const onode_t *a, const onode_t *b)
{
    uint32_t ia = (uint32_t)(-1 - a->left), ib = (uint32_t)(-1 - b->left);
    double ta[9], *tb = &s->B->tri[9 * (size_t)ib];
    for (int v = 0; v < 3; v++) pose_apply(&s->P, &s->A->tri[9 * (size_t)ia + 3 * v], &ta[3 * v]);
    s->tri_tests++;
    if (orc_tt_sat(ta, tb)) {
        s->hit = 1;
        if (s->pairs && s->n < s->cap) { s->pairs[2 * s->n] = ia; s->pairs[2 * s->n + 1] = ib; }
        s->n++;
    }
}

static int intersect(cstate_t *s, const onode_t *a, const onode_t *b)
{
    s->bv_tests++;
    return bv_overlap(&s->P, a, b, 0.0);
}

static void bvh_traversal(cstate_t *s, int32_t ia, int32_t ib)
{
    if (s->early_exit && s->hit) return;
    const onode_t *a = &s->A->node[ia], *b = &s->B->node[ib];
    if (is_leaf(a) && is_leaf(b)) {
        check_primitives(s, a, b);
    } else if (is_leaf(a)) {
        int32_t ch[2] = {b->left, b->right};
        for (int j = 0; j < 2; j++)
            if (intersect(s, a, &s->B->node[ch[j]])) bvh_traversal(s, ia, ch[j]);
    } else if (is_leaf(b)) {
        int32_t ch[2] = {a->left, a->right};
        for (int i = 0; i < 2; i++)
            if (intersect(s, &s->A->node[ch[i]], b)) bvh_traversal(s, ch[i], ib);
    } else {
        int32_t ca[2] = {a->left, a->right}, cb[2] = {b->left, b->right};
        for (int i = 0; i < 2; i++)
            for (int j = 0; j < 2; j++)
                if (intersect(s, &s->A->node[ca[i]], &s->B->node[cb[j]])) bvh_traversal(s, ca[i], cb[j]);
    }
}

/* returns 1 if any triangle pair intersects; with pairs != NULL all
 * intersecting (triA, triB) input-index pairs are written (up to cap) and
 * *n_pairs receives the total count */
EXPORT int orc_collide(const void *A, const void *B, const float *pose, int early_exit,
                       uint32_t *pairs, uint64_t cap, uint64_t *n_pairs, uint64_t *counters)
{
    cstate_t s;
    memset(&s, 0, sizeof s);
    s.A = A; s.B = B; s.early_exit = early_exit && !pairs; s.pairs = pairs; s.cap = cap;
    pose_from(pose, &s.P);
    if (intersect(&s, &s.A->node[0], &s.B->node[0])) bvh_traversal(&s, 0, 0);
    if (n_pairs) *n_pairs = s.n;
    if (counters) { counters[0] += s.bv_tests; counters[1] += s.tri_tests; }
    return s.hit;
}

/* ------------------------------------------------------------------ */
/* Algorithm 1 as branch-and-bound for the minimum distance             */
/* ------------------------------------------------------------------ */
typedef struct {
    const omesh_t *A, *B;
    pose_t P;
    double best;
    uint64_t bv_tests, tri_tests;
} dstate_t;

typedef struct { double lb; int32_t a, b; } cand_t;

static int cmp_cand(const void *x, const void *y)
{
    const cand_t *p = x, *q = y;
    return (p->lb > q->lb) - (p->lb < q->lb);
}

static void dist_traversal(dstate_t *s, int32_t ia, int32_t ib)
{
    const onode_t *a = &s->A->node[ia], *b = &s->B->node[ib];
    if (is_leaf(a) && is_leaf(b)) {
        uint32_t ta_i = (uint32_t)(-1 - a->left), tb_i = (uint32_t)(-1 - b->left);
        double ta[9];
        for (int v = 0; v < 3; v++) pose_apply(&s->P, &s->A->tri[9 * (size_t)ta_i + 3 * v], &ta[3 * v]);
        s->tri_tests++;
        double d = orc_tt_dist(ta, &s->B->tri[9 * (size_t)tb_i]);
        if (d < s->best) s->best = d;
        return;
    }
    cand_t c[4];
    int n = 0;
    int32_t ca[2] = {ia, ia}, cb[2] = {ib, ib};
    int na = 1, nb = 1;
    if (!is_leaf(a)) { ca[0] = a->left; ca[1] = a->right; na = 2; }
    if (!is_leaf(b)) { cb[0] = b->left; cb[1] = b->right; nb = 2; }
    for (int i = 0; i < na; i++)
        for (int j = 0; j < nb; j++) {
            s->bv_tests++;
            c[n].lb = bv_lower_bound(&s->P, &s->A->node[ca[i]], &s->B->node[cb[j]]);
            c[n].a = ca[i]; c[n].b = cb[j]; n++;
        }
    qsort(c, n, sizeof(cand_t), cmp_cand);
    for (int k = 0; k < n; k++)
        if (c[k].lb < s->best) dist_traversal(s, c[k].a, c[k].b);
}

EXPORT double orc_distance(const void *A, const void *B, const float *pose, uint64_t *counters)
{
    dstate_t s;
    memset(&s, 0, sizeof s);
    s.A = A; s.B = B; s.best = INFINITY;
    pose_from(pose, &s.P);
    dist_traversal(&s, 0, 0);
    if (counters) { counters[0] += s.bv_tests; counters[1] += s.tri_tests; }
    return s.best;
}

/* ------------------------------------------------------------------ */
/* brute force over all triangle pairs (for tiny meshes)                */
/* ------------------------------------------------------------------ */
EXPORT uint64_t orc_brute_collide(const void *Ap, const void *Bp, const float *pose, uint32_t *pairs, uint64_t cap)
{
    const omesh_t *A = Ap, *B = Bp;
    pose_t P;
    pose_from(pose, &P);
    uint64_t n = 0;
    double ta[9];
    for (uint32_t i = 0; i < A->nt; i++) {
        for (int v = 0; v < 3; v++) pose_apply(&P, &A->tri[9 * (size_t)i + 3 * v], &ta[3 * v]);
        for (uint32_t j = 0; j < B->nt; j++)
            if (orc_tt_sat(ta, &B->tri[9 * (size_t)j])) {
                if (pairs && n < cap) { pairs[2 * n] = i; pairs[2 * n + 1] = j; }
                n++;
            }
    }
    return n;
}

EXPORT double orc_brute_distance(const void *Ap, const void *Bp, const float *pose)
{
    const omesh_t *A = Ap, *B = Bp;
    pose_t P;
    pose_from(pose, &P);
    double best = INFINITY, ta[9];
    for (uint32_t i = 0; i < A->nt; i++) {
        for (int v = 0; v < 3; v++) pose_apply(&P, &A->tri[9 * (size_t)i + 3 * v], &ta[3 * v]);
        for (uint32_t j = 0; j < B->nt; j++) best = dmin(best, orc_tt_dist(ta, &B->tri[9 * (size_t)j]));
    }
    return best;
}

/* ------------------------------------------------------------------ */
/* input validity: penetration / separation margin                      */
/* ------------------------------------------------------------------ */
enum { CLS_SEPARATED = 0, CLS_COLLIDING = 1, CLS_MARGINAL = 2 };

typedef struct {
    const omesh_t *A, *B;
    pose_t P;
    double m;
    int pair_level;
    int robust_hit, marginal, any_hit;
} mstate_t;

static void margin_traversal(mstate_t *s, int32_t ia, int32_t ib)
{
    if (!s->pair_level && s->robust_hit) return;
    const onode_t *a = &s->A->node[ia], *b = &s->B->node[ib];
    if (is_leaf(a) && is_leaf(b)) {
        uint32_t ta_i = (uint32_t)(-1 - a->left), tb_i = (uint32_t)(-1 - b->left);
        double ta[9];
        for (int v = 0; v < 3; v++) pose_apply(&s->P, &s->A->tri[9 * (size_t)ta_i + 3 * v], &ta[3 * v]);
        double sep = orc_tt_signed(ta, &s->B->tri[9 * (size_t)tb_i]);
        if (sep <= 0 && orc_tt_sat(ta, &s->B->tri[9 * (size_t)tb_i])) s->any_hit = 1;
        if (sep <= -s->m) s->robust_hit = 1;
        else if (sep < s->m) s->marginal = 1;
        return;
    }
    int32_t ca[2] = {ia, ia}, cb[2] = {ib, ib};
    int na = 1, nb = 1;
    if (!is_leaf(a)) { ca[0] = a->left; ca[1] = a->right; na = 2; }
    if (!is_leaf(b)) { cb[0] = b->left; cb[1] = b->right; nb = 2; }
    for (int i = 0; i < na; i++)
        for (int j = 0; j < nb; j++)
            if (bv_overlap(&s->P, &s->A->node[ca[i]], &s->B->node[cb[j]], s->m)) margin_traversal(s, ca[i], cb[j]);
}

/* Pose-level (pair_level = 0): COLLIDING if some pair penetrates by >= m,
 * else SEPARATED if every pair is >= m apart, else MARGINAL.
 * Pair-level (pair_level = 1): MARGINAL if any pair has signed separation
 * in (-m, m), else COLLIDING / SEPARATED by whether any pair intersects. */
EXPORT int orc_classify(const void *A, const void *B, const float *pose, double m, int pair_level)
{
    mstate_t s;
    memset(&s, 0, sizeof s);
    s.A = A; s.B = B; s.m = m; s.pair_level = pair_level;
    pose_from(pose, &s.P);
    if (bv_overlap(&s.P, &s.A->node[0], &s.B->node[0], m)) margin_traversal(&s, 0, 0);
    if (pair_level) {
        if (s.marginal) return CLS_MARGINAL;
        return (s.robust_hit || s.any_hit) ? CLS_COLLIDING : CLS_SEPARATED;
    }
    if (s.robust_hit) return CLS_COLLIDING;
    return s.marginal ? CLS_MARGINAL : CLS_SEPARATED;
}

/* ------------------------------------------------------------------ */
/* batches over poses on a pthread pool                                 */
/* ------------------------------------------------------------------ */
typedef struct {
    int kind; /* 0 collide (bool, early exit), 1 distance, 2 classify, 3 count colliding pairs */
    const void *A, *B;
    const float *poses;
    uint64_t n;
    double m; int pair_level;
    uint8_t *u8_out; double *f64_out; uint64_t *u64_out;
    uint64_t next;
    pthread_mutex_t mu;
    uint64_t counters[2];
} batch_t;

static void *batch_worker(void *arg)
{
    batch_t *b = arg;
    uint64_t cnt[2] = {0, 0};
    for (;;) {
        pthread_mutex_lock(&b->mu);
        uint64_t i = b->next++;
        pthread_mutex_unlock(&b->mu);
        if (i >= b->n) break;
        const float *p = b->poses + 12 * i;
        if (b->kind == 0) b->u8_out[i] = (uint8_t)orc_collide(b->A, b->B, p, 1, NULL, 0, NULL, cnt);
        else if (b->kind == 1) b->f64_out[i] = orc_distance(b->A, b->B, p, cnt);
        else if (b->kind == 2) b->u8_out[i] = (uint8_t)orc_classify(b->A, b->B, p, b->m, b->pair_level);
        else orc_collide(b->A, b->B, p, 0, NULL, 0, &b->u64_out[i], cnt);
    }
    pthread_mutex_lock(&b->mu);
    b->counters[0] += cnt[0]; b->counters[1] += cnt[1];
    pthread_mutex_unlock(&b->mu);
    return NULL;
}

static void run_batch(batch_t *b, int nthreads, uint64_t *counters)
{
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    b->next = 0;
    pthread_mutex_init(&b->mu, NULL);
    for (int i = 0; i < nthreads; i++) pthread_create(&th[i], NULL, batch_worker, b);
    for (int i = 0; i < nthreads; i++) pthread_join(th[i], NULL);
    pthread_mutex_destroy(&b->mu);
    if (counters) { counters[0] = b->counters[0]; counters[1] = b->counters[1]; }
}

EXPORT void orc_collide_batch(const void *A, const void *B, const float *poses, uint64_t n, int nthreads,
                              uint8_t *hit, uint64_t *counters)
{
    batch_t b;
    memset(&b, 0, sizeof b);
    b.kind = 0; b.A = A; b.B = B; b.poses = poses; b.n = n; b.u8_out = hit;
    run_batch(&b, nthreads, counters);
}

EXPORT void orc_distance_batch(const void *A, const void *B, const float *poses, uint64_t n, int nthreads,
                               double *dist, uint64_t *counters)
{
    batch_t b;
    memset(&b, 0, sizeof b);
    b.kind = 1; b.A = A; b.B = B; b.poses = poses; b.n = n; b.f64_out = dist;
    run_batch(&b, nthreads, counters);
}

/* number of intersecting triangle pairs per pose (the full enumeration of
 * Algorithm 1 without early exit, as for pair lists) */
EXPORT void orc_pair_count_batch(const void *A, const void *B, const float *poses, uint64_t n, int nthreads,
                                 uint64_t *count, uint64_t *counters)
{
    batch_t b;
    memset(&b, 0, sizeof b);
    b.kind = 3; b.A = A; b.B = B; b.poses = poses; b.n = n; b.u64_out = count;
    run_batch(&b, nthreads, counters);
}

EXPORT void orc_classify_batch(const void *A, const void *B, const float *poses, uint64_t n, double m,
                               int pair_level, int nthreads, uint8_t *cls)
{
    batch_t b;
    memset(&b, 0, sizeof b);
    b.kind = 2; b.A = A; b.B = B; b.poses = poses; b.n = n; b.m = m; b.pair_level = pair_level; b.u8_out = cls;
    run_batch(&b, nthreads, NULL);
}

/* ------------------------------------------------------------------ */
/* compressed BVH blob: independent parser, decoder and invariants      */
/* ------------------------------------------------------------------ */
/* Byte layout (little endian), as produced by the library's builder:
 *   header (128 B): "CBVH", version 1, bv, K, bits, branching, leaf_size,
 *     n_nodes, n_tris, n_abs, n_treelets, code_stride, depth,
 *     treelet_bytes, then u64 offsets of topo, codes, abs, tris, perm,
 *     treelets, and the total size; f32 max |coordinate|.
 *   topo[n]: u32; bit31 leaf, bit30 absolute, bits27-29 count-1,
 *     bits0-26 first child node (inner) or first leaf-order triangle (leaf).
 *   codes[n][code_stride]: per slab (lo code, hi code), u8 or u16; with
 *     bits = 0, (lo, hi) as f32; with bits = 0x8010, (lo, hi) as IEEE
 *     binary16 (the half-precision descriptors of section III.A of the
 *     paper, rounded outward).  Absolute nodes keep a u32 index into abs.
 *   abs[n_abs][2K]: f32 (lo, hi) per slab.
 *   Oriented boxes (bv 2, K 3; the OBBs the paper names among BV types and
 *     as future work for its layout): a node is {o + u0 a0 + u1 a1 + u2 a2 :
 *     lo_k <= u_k <= hi_k}, its slabs the intervals of the frame
 *     coordinates u.  Its descriptor is 20 f32: lo0 hi0 lo1 hi1 lo2 hi2, 0,
 *     eps, o[3], a0[3], a1[3], a2[3], with eps >= max |a_i.a_j - [i==j]|.
 *     Absolute nodes (all nodes when bits = 0) store the whole descriptor
 *     (abs[] entries, or the code slot: stride 80); relative nodes code their
 *     intervals against the parent's like fixed slabs and keep its frame.
 *   tris[n_tris][9]: f32 in leaf order;  perm[n_tris]: u32 input index.
 *   treelets[n_treelets+1]: u32 first node of each treelet.
 * Decoding a relative node from its decoded parent interval [Pl, Ph] with
 * b-bit codes (ql, qh):  E = Ph - Pl (float),  s = E * 2^-b (0 if
 * E < 2^-100),  lo = fma(ql, s, Pl),  hi = fma(-qh, s, Ph)  (float fma). */
typedef struct {
    uint32_t bv, K, bits, branching, leaf_size, n_nodes, n_tris, n_abs, n_treelets, code_stride, depth, treelet_bytes;
    uint64_t off_topo, off_codes, off_abs, off_tris, off_perm, off_treelets, total;
    float max_abs_coord;
} ohdr_t;

static uint32_t rd32(const uint8_t *p) { return (uint32_t)p[0] | (uint32_t)p[1] << 8 | (uint32_t)p[2] << 16 | (uint32_t)p[3] << 24; }
static uint64_t rd64(const uint8_t *p) { return (uint64_t)rd32(p) | (uint64_t)rd32(p + 4) << 32; }
static float rdf32(const uint8_t *p) { uint32_t u = rd32(p); float f; memcpy(&f, &u, 4); return f; }
static uint16_t rd16(const uint8_t *p) { return (uint16_t)(p[0] | p[1] << 8); }

#define BITS_FP16 0x8010u
static int bits_codes(uint32_t b) { return b == 8 || b == 16; }
/* IEEE binary16 -> float, exactly: subnormals m * 2^-24, normals
 * (1024 + m) * 2^(e - 25); exponent 31 (inf / NaN) is not a valid bound */
static int half_finite(uint16_t h) { return ((h >> 10) & 31) != 31; }
static float half_value(uint16_t h)
{
    int e = (h >> 10) & 31, m = h & 1023;
    float v = e == 0 ? ldexpf((float)m, -24) : ldexpf((float)(m | 1024), e - 25);
    return (h & 0x8000) ? -v : v;
}
/* neighbouring binary16 values towards +inf / -inf */
static uint16_t half_next_up(uint16_t h) { return h == 0x8000 ? 0x0001 : (h & 0x8000) ? (uint16_t)(h - 1) : (uint16_t)(h + 1); }
static uint16_t half_next_down(uint16_t h) { return h == 0x0000 ? 0x8001 : (h & 0x8000) ? (uint16_t)(h + 1) : (uint16_t)(h - 1); }

/* f32 words per decoded node: the bounds, or an OBB's whole descriptor */
#define OBB_WORDS 20
static uint32_t desc_words(const ohdr_t *h) { return h->bv == 2 ? OBB_WORDS : 2 * h->K; }

static int parse_header(const uint8_t *blob, size_t n, ohdr_t *h, char *msg, size_t ml)
{
    if (n < 128 || memcmp(blob, "CBVH", 4) != 0) { snprintf(msg, ml, "bad magic/size"); return -1; }
    if (rd32(blob + 4) != 1) { snprintf(msg, ml, "bad version"); return -1; }
    h->bv = rd32(blob + 8); h->K = rd32(blob + 12); h->bits = rd32(blob + 16); h->branching = rd32(blob + 20);
    h->leaf_size = rd32(blob + 24); h->n_nodes = rd32(blob + 28); h->n_tris = rd32(blob + 32); h->n_abs = rd32(blob + 36);
    h->n_treelets = rd32(blob + 40); h->code_stride = rd32(blob + 44); h->depth = rd32(blob + 48); h->treelet_bytes = rd32(blob + 52);
    h->off_topo = rd64(blob + 56); h->off_codes = rd64(blob + 64); h->off_abs = rd64(blob + 72); h->off_tris = rd64(blob + 80);
    h->off_perm = rd64(blob + 88); h->off_treelets = rd64(blob + 96); h->total = rd64(blob + 104); h->max_abs_coord = rdf32(blob + 112);
    if (!((h->bv == 0 && h->K == 3) || (h->bv == 1 && h->K == 9) || (h->bv == 2 && h->K == 3))) { snprintf(msg, ml, "bad bv/K"); return -1; }
    if (!(h->bits == 0 || bits_codes(h->bits) || h->bits == BITS_FP16)) { snprintf(msg, ml, "bad bits"); return -1; }
    if (h->bv == 2 && h->bits == BITS_FP16) { snprintf(msg, ml, "FP16 OBB blob"); return -1; }
    uint32_t want = h->bits == 0 ? (h->bv == 2 ? 80 : 8 * h->K) : h->bits == BITS_FP16 ? 4 * h->K : (h->bits / 8) * 2 * h->K;
    if (h->code_stride != want) { snprintf(msg, ml, "bad code stride"); return -1; }
    if (h->total != n) { snprintf(msg, ml, "size mismatch"); return -1; }
#define FITS(off, bytes) ((off) <= n && (uint64_t)(bytes) <= n - (off))
    if (!FITS(h->off_topo, 4ull * h->n_nodes) || !FITS(h->off_codes, (uint64_t)h->code_stride * h->n_nodes) ||
        !FITS(h->off_abs, 4ull * desc_words(h) * h->n_abs) || !FITS(h->off_tris, 36ull * h->n_tris) ||
        !FITS(h->off_perm, 4ull * h->n_tris) || !FITS(h->off_treelets, 4ull * (h->n_treelets + 1))) {
        snprintf(msg, ml, "section out of range"); return -1;
    }
#undef FITS
    return 0;
}

/* decode every node's bounds, top-down; out[n][2K] as (lo, hi) per slab
 * (OBB blobs: out[n][20], each node's descriptor with its frame) */
static int decode_all(const uint8_t *blob, const ohdr_t *h, float *out, int32_t *parent, char *msg, size_t ml)
{
    const uint32_t K2 = 2 * h->K, DW = desc_words(h);
    for (uint32_t i = 0; i < h->n_nodes; i++) parent[i] = -2;
    parent[0] = -1;
    for (uint32_t i = 0; i < h->n_nodes; i++) {
        uint32_t tw = rd32(blob + h->off_topo + 4ull * i);
        const uint8_t *code = blob + h->off_codes + (uint64_t)h->code_stride * i;
        if (parent[i] == -2) { snprintf(msg, ml, "node %u unreachable or out of order", i); return -1; }
        int absolute = (tw >> 30) & 1;
        float *o = &out[DW * (size_t)i];
        if (h->bits == 0) {
            for (uint32_t k = 0; k < DW; k++) o[k] = rdf32(code + 4 * k);
        } else if (h->bits == BITS_FP16) {
            if (absolute) { snprintf(msg, ml, "absolute flag in an FP16 blob"); return -1; }
            for (uint32_t k = 0; k < K2; k++) {
                uint16_t hv = rd16(code + 2 * k);
                if (!half_finite(hv)) { snprintf(msg, ml, "non-finite FP16 bound at node %u", i); return -1; }
                o[k] = half_value(hv);
            }
        } else if (absolute || parent[i] < 0) {
            if (!absolute) { snprintf(msg, ml, "root not absolute"); return -1; }
            uint32_t ai = rd32(code);
            if (ai >= h->n_abs) { snprintf(msg, ml, "abs index out of range"); return -1; }
            for (uint32_t k = 0; k < DW; k++) o[k] = rdf32(blob + h->off_abs + 4ull * (DW * (size_t)ai + k));
        } else {
            const float *P = &out[DW * (size_t)parent[i]];
            for (uint32_t k = K2; k < DW; k++) o[k] = P[k]; /* an OBB keeps its parent's frame */
            for (uint32_t k = 0; k < h->K; k++) {
                uint32_t ql, qh;
                if (h->bits == 8) { ql = code[2 * k]; qh = code[2 * k + 1]; }
                else { ql = rd16(code + 4 * k); qh = rd16(code + 4 * k + 2); }
                float Pl = P[2 * k], Ph = P[2 * k + 1];
                float E = Ph - Pl;
                float s = (E >= 0x1p-100f) ? ldexpf(E, -(int)h->bits) : 0.0f;
                o[2 * k] = fmaf((float)ql, s, Pl);
                o[2 * k + 1] = fmaf(-(float)qh, s, Ph);
            }
        }
        if (!((tw >> 31) & 1)) {
            uint32_t first = tw & 0x07FFFFFFu, cnt = ((tw >> 27) & 7u) + 1;
            if (first <= i || first + cnt > h->n_nodes) { snprintf(msg, ml, "bad child range at %u", i); return -1; }
            for (uint32_t c = 0; c < cnt; c++) {
                if (parent[first + c] != -2) { snprintf(msg, ml, "node %u has two parents", first + c); return -1; }
                parent[first + c] = (int32_t)i;
            }
        }
    }
    return 0;
}

EXPORT int orc_blob_info(const uint8_t *blob, size_t n, uint32_t *info /* 12 */)
{
    ohdr_t h;
    char msg[128];
    if (parse_header(blob, n, &h, msg, sizeof msg)) return -1;
    uint32_t v[12] = {h.bv, h.K, h.bits, h.branching, h.leaf_size, h.n_nodes, h.n_tris, h.n_abs, h.n_treelets, h.code_stride, h.depth, h.treelet_bytes};
    memcpy(info, v, sizeof v);
    return 0;
}

EXPORT int orc_blob_decode(const uint8_t *blob, size_t n, float *out, char *msg, size_t ml)
{
    ohdr_t h;
    if (parse_header(blob, n, &h, msg, ml)) return -1;
    int32_t *parent = malloc(sizeof(int32_t) * h.n_nodes);
    int rc = decode_all(blob, &h, out, parent, msg, ml);
    free(parent);
    return rc;
}

/* Exact comparisons of a float f against x + y (x, y floats): with
 * s = fl64(x + y) and e = (x + y) - s exactly (two-sum), f <= x + y iff
 * f < s, or f == s and e >= 0.  Exact because f and s are doubles and |e|
 * is below half the spacing of doubles around s. */
typedef struct { double s, e; } dd_t;

static dd_t dd_sum(double x, double y)
{
    dd_t r;
    r.s = x + y;
    double bp = r.s - x, ap = r.s - bp;
    r.e = (x - ap) + (y - bp);
    return r;
}
static int dd_lt(dd_t a, dd_t b) { return a.s < b.s || (a.s == b.s && a.e < b.e); }
static int f_le_dd(double f, dd_t v) { return f < v.s || (f == v.s && v.e >= 0); }
static int f_ge_dd(double f, dd_t v) { return f > v.s || (f == v.s && v.e <= 0); }

/* slab directions: AABB x, y, z; 18-DOP adds x+y, x+z, y+z, x-y, x-z, y-z */
static dd_t slab_value(const float *p, int k)
{
    switch (k) {
    case 0: return dd_sum(p[0], 0.0);
    case 1: return dd_sum(p[1], 0.0);
    case 2: return dd_sum(p[2], 0.0);
    case 3: return dd_sum(p[0], p[1]);
    case 4: return dd_sum(p[0], p[2]);
    case 5: return dd_sum(p[1], p[2]);
    case 6: return dd_sum(p[0], -(double)p[1]);
    case 7: return dd_sum(p[0], -(double)p[2]);
    default: return dd_sum(p[1], -(double)p[2]);
    }
}

/* Frame coordinates of x in the frame (o, a0, a1, a2): the solution of
 * u0 a0 + u1 a1 + u2 a2 = x - o by Cramer's rule in FP64.  Returns a bound
 * on the evaluation's error (for axes within 2^-6 of orthonormal the
 * determinant is near 1 and every rounding is relative to |x - o|). */
static double frame_coords(const float *f, const double *x, double *u)
{
    double a[3][3], d[3];
    for (int j = 0; j < 3; j++)
        for (int k = 0; k < 3; k++) a[j][k] = f[11 + 3 * j + k];
    for (int k = 0; k < 3; k++) d[k] = x[k] - (double)f[8 + k];
    double det;
    {
        double c[3];
        vcross(a[1], a[2], c);
        det = vdot(a[0], c);
    }
    double c12[3], c20[3], c01[3];
    vcross(a[1], a[2], c12);
    vcross(a[2], a[0], c20);
    vcross(a[0], a[1], c01);
    u[0] = vdot(d, c12) / det;
    u[1] = vdot(d, c20) / det;
    u[2] = vdot(d, c01) / det;
    return 0x1p-44 * (fabs(d[0]) + fabs(d[1]) + fabs(d[2]));
}

/* OBB blob invariants: every frame's eps bounds its axes' orthonormality
 * defect (and is below 2^-6); every node's intervals are ordered, lie in its
 * parent's where the two share a frame, and enclose the frame coordinates of
 * every vertex of the node's triangles (beyond the FP64 evaluation error). */
static int obb_check(const uint8_t *blob, const ohdr_t *h, const float *dec, const int32_t *parent, char *msg,
                     size_t ml)
{
    uint32_t *stack = malloc(sizeof(uint32_t) * (h->n_nodes + 1));
    int rc = -1;
    for (uint32_t i = 0; i < h->n_nodes; i++) {
        const float *f = &dec[OBB_WORDS * (size_t)i];
        uint32_t tw = rd32(blob + h->off_topo + 4ull * i);
        int absolute = (tw >> 30) & 1;
        for (int k = 7; k < OBB_WORDS; k++)
            if (!isfinite(f[k])) { snprintf(msg, ml, "node %u frame not finite", i); goto out; }
        double defect = 0.0;
        for (int p = 0; p < 3; p++)
            for (int q = p; q < 3; q++) {
                double g = 0.0;
                for (int k = 0; k < 3; k++) g += (double)f[11 + 3 * p + k] * (double)f[11 + 3 * q + k];
                defect = dmax(defect, fabs(g - (p == q ? 1.0 : 0.0)));
            }
        if (!((double)f[7] >= defect + 0x1p-50) || f[7] > 0x1p-6f) { snprintf(msg, ml, "node %u eps does not bound its frame", i); goto out; }
        for (int k = 0; k < 3; k++)
            if (!(f[2 * k] <= f[2 * k + 1])) { snprintf(msg, ml, "node %u slab %d empty", i, k); goto out; }
        int same_frame = parent[i] >= 0 && bits_codes(h->bits) && !absolute;
        if (same_frame) {
            const float *P = &dec[OBB_WORDS * (size_t)parent[i]];
            for (int k = 0; k < 3; k++)
                if (f[2 * k] < P[2 * k] || f[2 * k + 1] > P[2 * k + 1]) { snprintf(msg, ml, "node %u slab %d outside parent", i, k); goto out; }
        }
        /* every vertex under the node */
        uint32_t sp = 0;
        stack[sp++] = i;
        while (sp) {
            uint32_t x = stack[--sp], w = rd32(blob + h->off_topo + 4ull * x);
            uint32_t first = w & 0x07FFFFFFu, cnt = ((w >> 27) & 7u) + 1;
            if (!((w >> 31) & 1)) {
                for (uint32_t c = 0; c < cnt; c++) stack[sp++] = first + c;
                continue;
            }
            for (uint32_t t = first; t < first + cnt; t++)
                for (int v = 0; v < 3; v++) {
                    double p[3], u[3];
                    for (int c = 0; c < 3; c++) p[c] = rdf32(blob + h->off_tris + 4ull * (9 * (size_t)t + 3 * v + c));
                    double e = frame_coords(f, p, u);
                    for (int k = 0; k < 3; k++)
                        if (!((double)f[2 * k] <= u[k] - e && u[k] + e <= (double)f[2 * k + 1])) {
                            snprintf(msg, ml, "node %u slab %d does not enclose triangle %u", i, k, t);
                            goto out;
                        }
                }
        }
    }
    rc = 0;
out:
    free(stack);
    return rc;
}

/* Invariant check of a blob against the mesh it was built from:
 *  (1) leaf-order triangles equal the input triangles under perm, perm is a
 *      permutation and the leaves' triangle ranges partition it;
 *  (2) every decoded bound encloses the exact slab of the node's triangles;
 *  (3) every decoded child lies inside its decoded parent;
 *  (4) codes are tight: the next code would no longer enclose;
 *  (5) absolute nodes are exactly the first nodes of treelets' top groups
 *      and treelets are contiguous node ranges closed under parent links.
 * Returns 0 if all hold, else -1 with a message. */
EXPORT int orc_blob_check(const uint8_t *blob, size_t n, const float *V, uint32_t nv, const uint32_t *T, uint32_t nt,
                          char *msg, size_t ml)
{
    ohdr_t h;
    if (parse_header(blob, n, &h, msg, ml)) return -1;
    if (h.n_tris != nt) { snprintf(msg, ml, "triangle count mismatch"); return -1; }
    const uint32_t K2 = 2 * h.K;
    int rc = -1;
    float *dec = malloc(sizeof(float) * desc_words(&h) * (size_t)h.n_nodes);
    int32_t *parent = malloc(sizeof(int32_t) * h.n_nodes);
    dd_t *exlo = malloc(sizeof(dd_t) * h.K * (size_t)h.n_nodes), *exhi = malloc(sizeof(dd_t) * h.K * (size_t)h.n_nodes);
    uint8_t *seen = calloc(nt, 1);
    uint32_t *treelet_of = malloc(sizeof(uint32_t) * h.n_nodes);
    if (decode_all(blob, &h, dec, parent, msg, ml)) goto done;
    /* (1) triangles and perm */
    for (uint32_t i = 0; i < nt; i++) {
        uint32_t p = rd32(blob + h.off_perm + 4ull * i);
        if (p >= nt || seen[p]) { snprintf(msg, ml, "perm not a permutation"); goto done; }
        seen[p] = 1;
        for (int v = 0; v < 3; v++) {
            uint32_t vi = T[3 * (size_t)p + v];
            if (vi >= nv) { snprintf(msg, ml, "bad index"); goto done; }
            for (int k = 0; k < 3; k++) {
                float a = rdf32(blob + h.off_tris + 4ull * (9 * (size_t)i + 3 * v + k));
                if (memcmp(&a, &V[3 * (size_t)vi + k], 4) != 0) { snprintf(msg, ml, "leaf triangle %u differs from input", i); goto done; }
            }
        }
    }
    memset(seen, 0, nt);
    /* exact slabs bottom-up (children have larger indices than parents) */
    for (int64_t i = (int64_t)h.n_nodes - 1; i >= 0; i--) {
        uint32_t tw = rd32(blob + h.off_topo + 4ull * (size_t)i);
        uint32_t first = tw & 0x07FFFFFFu, cnt = ((tw >> 27) & 7u) + 1;
        int leaf = (tw >> 31) & 1;
        if (leaf && cnt > h.leaf_size) { snprintf(msg, ml, "leaf %lld exceeds leaf size", (long long)i); goto done; }
        if (!leaf && (cnt < 2 || cnt > h.branching)) { snprintf(msg, ml, "bad child count at %lld", (long long)i); goto done; }
        for (uint32_t k = 0; k < h.K; k++) {
            dd_t lo = {INFINITY, 0}, hi = {-INFINITY, 0};
            if (leaf) {
                if (first + cnt > nt) { snprintf(msg, ml, "leaf range out of bounds"); goto done; }
                for (uint32_t t = first; t < first + cnt; t++) {
                    if (k == 0) {
                        if (seen[t]) { snprintf(msg, ml, "leaf ranges overlap"); goto done; }
                        seen[t] = 1;
                    }
                    for (int v = 0; v < 3; v++) {
                        float p[3];
                        for (int c = 0; c < 3; c++) p[c] = rdf32(blob + h.off_tris + 4ull * (9 * (size_t)t + 3 * v + c));
                        dd_t x = slab_value(p, (int)k);
                        if (dd_lt(x, lo)) lo = x;
                        if (dd_lt(hi, x)) hi = x;
                    }
                }
            } else {
                for (uint32_t c = first; c < first + cnt; c++) {
                    if (dd_lt(exlo[h.K * (size_t)c + k], lo)) lo = exlo[h.K * (size_t)c + k];
                    if (dd_lt(hi, exhi[h.K * (size_t)c + k])) hi = exhi[h.K * (size_t)c + k];
                }
            }
            exlo[h.K * (size_t)i + k] = lo;
            exhi[h.K * (size_t)i + k] = hi;
        }
    }
    for (uint32_t t = 0; t < nt; t++) if (!seen[t]) { snprintf(msg, ml, "triangle %u in no leaf", t); goto done; }
    if (h.bv == 2) {
        /* oriented boxes: frames, enclosure in frame coordinates, nesting */
        if (obb_check(blob, &h, dec, parent, msg, ml)) goto done;
        goto treelets;
    }
    /* (2)-(4) */
    for (uint32_t i = 0; i < h.n_nodes; i++) {
        uint32_t tw = rd32(blob + h.off_topo + 4ull * i);
        int absolute = (tw >> 30) & 1;
        const uint8_t *code = blob + h.off_codes + (uint64_t)h.code_stride * i;
        for (uint32_t k = 0; k < h.K; k++) {
            float lo = dec[K2 * (size_t)i + 2 * k], hi = dec[K2 * (size_t)i + 2 * k + 1];
            dd_t el = exlo[h.K * (size_t)i + k], eh = exhi[h.K * (size_t)i + k];
            if (!f_le_dd(lo, el) || !f_ge_dd(hi, eh)) { snprintf(msg, ml, "node %u slab %u does not enclose", i, k); goto done; }
            if (h.bits == BITS_FP16) {
                /* binary16 bounds: tightest halves, i.e. the next half inward fails */
                float lo2 = half_value(half_next_up(rd16(code + 4 * k))), hi2 = half_value(half_next_down(rd16(code + 4 * k + 2)));
                if (f_le_dd(lo2, el) || f_ge_dd(hi2, eh)) { snprintf(msg, ml, "node %u slab %u FP16 bound not tight", i, k); goto done; }
            } else if (h.bits == 0 || absolute) {
                /* absolute bounds: tightest floats, i.e. the next float inward fails */
                float lo2 = nextafterf(lo, INFINITY), hi2 = nextafterf(hi, -INFINITY);
                if (f_le_dd(lo2, el) || f_ge_dd(hi2, eh)) { snprintf(msg, ml, "node %u slab %u absolute bound not tight", i, k); goto done; }
            }
            if (parent[i] >= 0) {
                const float *P = &dec[K2 * (size_t)parent[i]];
                if (lo < P[2 * k] || hi > P[2 * k + 1]) { snprintf(msg, ml, "node %u slab %u outside parent", i, k); goto done; }
                if (bits_codes(h.bits) && !absolute) {
                    uint32_t ql, qh, Q = (1u << h.bits) - 1;
                    if (h.bits == 8) { ql = code[2 * k]; qh = code[2 * k + 1]; }
                    else { ql = rd16(code + 4 * k); qh = rd16(code + 4 * k + 2); }
                    float E = P[2 * k + 1] - P[2 * k];
                    float s = (E >= 0x1p-100f) ? ldexpf(E, -(int)h.bits) : 0.0f;
                    if (s > 0 && ql < Q && f_le_dd(fmaf((float)(ql + 1), s, P[2 * k]), el)) { snprintf(msg, ml, "node %u slab %u lo code not tight", i, k); goto done; }
                    if (s > 0 && qh < Q && f_ge_dd(fmaf(-(float)(qh + 1), s, P[2 * k + 1]), eh)) { snprintf(msg, ml, "node %u slab %u hi code not tight", i, k); goto done; }
                    if (s == 0 && (ql || qh)) { snprintf(msg, ml, "node %u zero-scale slab with non-zero code", i); goto done; }
                }
            }
        }
    }
    /* (5) treelets */
treelets:
    {
        uint32_t prev = 0;
        if (h.n_treelets < 1 || rd32(blob + h.off_treelets) != 0 || rd32(blob + h.off_treelets + 4ull * h.n_treelets) != h.n_nodes) {
            snprintf(msg, ml, "bad treelet table"); goto done;
        }
        for (uint32_t t = 0; t < h.n_treelets; t++) {
            uint32_t a = rd32(blob + h.off_treelets + 4ull * t), b = rd32(blob + h.off_treelets + 4ull * (t + 1));
            if (a != prev || b <= a) { snprintf(msg, ml, "treelets not contiguous"); goto done; }
            for (uint32_t i = a; i < b; i++) treelet_of[i] = t;
            prev = b;
        }
        uint32_t n_abs = 0;
        for (uint32_t i = 0; i < h.n_nodes; i++) {
            uint32_t tw = rd32(blob + h.off_topo + 4ull * i);
            int absolute = (tw >> 30) & 1;
            int top = parent[i] < 0 || treelet_of[parent[i]] != treelet_of[i];
            if (!bits_codes(h.bits)) { if (absolute) { snprintf(msg, ml, "absolute flag in a blob without codes"); goto done; } continue; }
            if (absolute != top) { snprintf(msg, ml, "node %u absolute flag %d but treelet top %d", i, absolute, top); goto done; }
            n_abs += (uint32_t)absolute;
        }
        if (bits_codes(h.bits) && n_abs != h.n_abs) { snprintf(msg, ml, "n_abs mismatch"); goto done; }
    }
    rc = 0;
done:
    free(dec); free(parent); free(exlo); free(exhi); free(seen); free(treelet_of);
    return rc;
}
