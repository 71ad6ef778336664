// Geometry of the leaf tests (checkPrimitives of Algorithm 1): closed
// triangle-triangle intersection and distance, in FP32 with certified error
// bounds and in FP64 for re-decision / refinement.  Device code; the same
// functions also compile as plain host C++ (no HIP), so that CPU tests can
// drive them against the oracle.
#pragma once
#if defined(__HIP__)
#include <hip/hip_runtime.h>
#define CBVH_GEOM __host__ __device__
#define CBVH_GEOM_INLINE __host__ __device__ __forceinline__
#else
#include <math.h>

#include <cmath>
#define CBVH_GEOM
#define CBVH_GEOM_INLINE inline __attribute__((always_inline))
#endif

namespace cbvh {
#if !defined(__HIP__)
using std::fabs;
using std::fma;
using std::fmax;
using std::fmin;
using std::sqrt;
#endif

template <typename T>
struct V3 {
    T x, y, z;
};

template <typename T>
CBVH_GEOM_INLINE V3<T> vsub(V3<T> a, V3<T> b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <typename T>
CBVH_GEOM_INLINE V3<T> vneg(V3<T> a) { return {-a.x, -a.y, -a.z}; }
template <typename T>
CBVH_GEOM_INLINE T vdot(V3<T> a, V3<T> b) { return fma(a.x, b.x, fma(a.y, b.y, a.z * b.z)); }
template <typename T>
CBVH_GEOM_INLINE V3<T> vcross(V3<T> a, V3<T> b)
{
    return {fma(a.y, b.z, -(a.z * b.y)), fma(a.z, b.x, -(a.x * b.z)), fma(a.x, b.y, -(a.y * b.x))};
}
template <typename T>
CBVH_GEOM_INLINE T vmaxabs(V3<T> a) { return fmax(fabs(a.x), fmax(fabs(a.y), fabs(a.z))); }
template <typename T>
CBVH_GEOM_INLINE V3<T> vmad(V3<T> a, T s, V3<T> b) { return {fma(a.x, s, b.x), fma(a.y, s, b.y), fma(a.z, s, b.z)}; }

// ---------------------------------------------------------------------------
// FP32 separating-axis test with certified decisions for the given float
// triangles.  Candidate axes: both face normals, the 9 edge-edge cross
// products, the 6 in-plane edge normals.  Edges are differences of the
// given coordinates (one rounding each: error <= u |edge|, u = 2^-24), so
// an axis from edges with largest components m1, m2 is within 7 u m1 m2 of
// the exact one (in-plane normals n x e: 24 u m1 m2 m3).  Projections use
// coordinates relative to a0 (one rounding each, error <= u R, R the
// largest relative coordinate).  Per endpoint, the computed projection is
// within 24 u R m1 m2 (48 u R m1 m2 m3) of the exact projection of the
// exact vertices on the computed axis, and the exact projections on the
// computed and on the exact axis differ by at most 21 u R m1 m2
// (72 u R m1 m2 m3).  Hence a computed gap above E = 128 u R m1 m2
// (512 u R m1 m2 m3) proves the triangles separated along the computed
// axis, and overlaps beyond E on every axis prove that no exact candidate
// axis separates them (both need at most 96 resp. 240 of those units).
// Returns 0 = disjoint, 1 = intersecting, 2 = undecided.
// ---------------------------------------------------------------------------
CBVH_GEOM inline int tri_tri_f32(const V3<float> *a, const V3<float> *b)
{
    const float u = 0x1p-24f;
    V3<float> ea[3] = {vsub(a[1], a[0]), vsub(a[2], a[1]), vsub(a[0], a[2])};
    V3<float> eb[3] = {vsub(b[1], b[0]), vsub(b[2], b[1]), vsub(b[0], b[2])};
    // a1 - a0 and a2 - a0 are edges of A (the second exactly negated)
    V3<float> A1 = ea[0], A2 = vneg(ea[2]);
    V3<float> B0 = vsub(b[0], a[0]), B1 = vsub(b[1], a[0]), B2 = vsub(b[2], a[0]);
    float R = fmaxf(fmaxf(vmaxabs(A1), vmaxabs(A2)), fmaxf(vmaxabs(B0), fmaxf(vmaxabs(B1), vmaxabs(B2))));
    float ma[3] = {vmaxabs(ea[0]), vmaxabs(ea[1]), vmaxabs(ea[2])};
    float mb[3] = {vmaxabs(eb[0]), vmaxabs(eb[1]), vmaxabs(eb[2])};
    bool undecided = false;
    auto separates = [&](V3<float> L, float E) -> bool {
        float p1 = vdot(A1, L), p2 = vdot(A2, L);
        float amin = fminf(0.0f, fminf(p1, p2)), amax = fmaxf(0.0f, fmaxf(p1, p2));
        float q0 = vdot(B0, L), q1 = vdot(B1, L), q2 = vdot(B2, L);
        float bmin = fminf(q0, fminf(q1, q2)), bmax = fmaxf(q0, fmaxf(q1, q2));
        float gap = fmaxf(bmin - amax, amin - bmax);
        if (gap > E) return true;
        if (gap >= -E) undecided = true;
        return false;
    };
    const float c2 = 128.0f * u * R, c3 = 512.0f * u * R;
    V3<float> na = vcross(ea[0], ea[1]);
    if (separates(na, c2 * ma[0] * ma[1])) return 0;
    V3<float> nb = vcross(eb[0], eb[1]);
    if (separates(nb, c2 * mb[0] * mb[1])) return 0;
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++)
            if (separates(vcross(ea[i], eb[j]), c2 * ma[i] * mb[j])) return 0;
#pragma unroll
    for (int i = 0; i < 3; i++) {
        if (separates(vcross(na, ea[i]), c3 * ma[0] * ma[1] * ma[i])) return 0;
        if (separates(vcross(nb, eb[i]), c3 * mb[0] * mb[1] * mb[i])) return 0;
    }
    return undecided ? 2 : 1;
}

// FP64 separating-axis test (used when the FP32 decision is not certified);
// axes whose squared length is below 1e-24 of the product of the squared
// edge lengths are parallel-edge degeneracies and are skipped.
CBVH_GEOM inline bool tri_tri_f64(const V3<double> *a, const V3<double> *b)
{
    V3<double> ea[3] = {vsub(a[1], a[0]), vsub(a[2], a[1]), vsub(a[0], a[2])};
    V3<double> eb[3] = {vsub(b[1], b[0]), vsub(b[2], b[1]), vsub(b[0], b[2])};
    auto separates = [&](V3<double> L, double ref2) -> bool {
        if (vdot(L, L) <= 1e-24 * ref2) return false;
        double p0 = vdot(a[0], L), p1 = vdot(a[1], L), p2 = vdot(a[2], L);
        double q0 = vdot(b[0], L), q1 = vdot(b[1], L), q2 = vdot(b[2], L);
        double amin = fmin(p0, fmin(p1, p2)), amax = fmax(p0, fmax(p1, p2));
        double bmin = fmin(q0, fmin(q1, q2)), bmax = fmax(q0, fmax(q1, q2));
        return amax < bmin || bmax < amin;
    };
    double la[3] = {vdot(ea[0], ea[0]), vdot(ea[1], ea[1]), vdot(ea[2], ea[2])};
    double lb[3] = {vdot(eb[0], eb[0]), vdot(eb[1], eb[1]), vdot(eb[2], eb[2])};
    V3<double> na = vcross(ea[0], ea[1]), nb = vcross(eb[0], eb[1]);
    double lna = vdot(na, na), lnb = vdot(nb, nb);
    if (separates(na, la[0] * la[1])) return false;
    if (separates(nb, lb[0] * lb[1])) return false;
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++)
            if (separates(vcross(ea[i], eb[j]), la[i] * lb[j])) return false;
    for (int i = 0; i < 3; i++) {
        if (separates(vcross(na, ea[i]), lna * la[i])) return false;
        if (separates(vcross(nb, eb[i]), lnb * lb[i])) return false;
    }
    return true;
}

// squared distance from p to triangle t (Voronoi-region classification by
// barycentric sign tests; Ericson, Real-Time Collision Detection, 5.1.5)
template <typename T>
CBVH_GEOM inline T pt_tri_dist2(V3<T> p, const V3<T> *t)
{
    V3<T> ab = vsub(t[1], t[0]), ac = vsub(t[2], t[0]), ap = vsub(p, t[0]);
    T d1 = vdot(ab, ap), d2 = vdot(ac, ap);
    V3<T> c;
    if (d1 <= T(0) && d2 <= T(0)) {
        c = t[0];
    } else {
        V3<T> bp = vsub(p, t[1]);
        T d3 = vdot(ab, bp), d4 = vdot(ac, bp);
        V3<T> cp = vsub(p, t[2]);
        T d5 = vdot(ab, cp), d6 = vdot(ac, cp);
        T vc = d1 * d4 - d3 * d2, vb = d5 * d2 - d1 * d6, va = d3 * d6 - d5 * d4;
        if (d3 >= T(0) && d4 <= d3) {
            c = t[1];
        } else if (d6 >= T(0) && d5 <= d6) {
            c = t[2];
        } else if (vc <= T(0) && d1 >= T(0) && d3 <= T(0)) {
            c = vmad(ab, d1 / (d1 - d3), t[0]);
        } else if (vb <= T(0) && d2 >= T(0) && d6 <= T(0)) {
            c = vmad(ac, d2 / (d2 - d6), t[0]);
        } else if (va <= T(0) && (d4 - d3) >= T(0) && (d5 - d6) >= T(0)) {
            c = vmad(vsub(t[2], t[1]), (d4 - d3) / ((d4 - d3) + (d5 - d6)), t[1]);
        } else {
            T den = T(1) / (va + vb + vc);
            c = vmad(ac, vc * den, vmad(ab, vb * den, t[0]));
        }
    }
    V3<T> d = vsub(p, c);
    return vdot(d, d);
}

// squared distance between segments p1-q1 and p2-q2: stationary point of
// the convex quadratic, clamped, then the other parameter re-solved
// (Ericson, Real-Time Collision Detection, 5.1.9)
template <typename T>
CBVH_GEOM inline T seg_seg_dist2(V3<T> p1, V3<T> q1, V3<T> p2, V3<T> q2)
{
    V3<T> d1 = vsub(q1, p1), d2 = vsub(q2, p2), r = vsub(p1, p2);
    T a = vdot(d1, d1), e = vdot(d2, d2), f = vdot(d2, r);
    T s, t;
    const T tiny = T(1e-30);
    if (a <= tiny && e <= tiny) {
        s = T(0); t = T(0);
    } else if (a <= tiny) {
        s = T(0);
        t = fmin(fmax(f / e, T(0)), T(1));
    } else {
        T c = vdot(d1, r);
        if (e <= tiny) {
            t = T(0);
            s = fmin(fmax(-c / a, T(0)), T(1));
        } else {
            T b = vdot(d1, d2), den = a * e - b * b;
            s = den > T(0) ? fmin(fmax((b * f - c * e) / den, T(0)), T(1)) : T(0);
            t = (b * s + f) / e;
            if (t < T(0)) {
                t = T(0);
                s = fmin(fmax(-c / a, T(0)), T(1));
            } else if (t > T(1)) {
                t = T(1);
                s = fmin(fmax((b - c) / a, T(0)), T(1));
            }
        }
    }
    V3<T> w = vsub(vmad(d1, s, p1), vmad(d2, t, p2));
    return vdot(w, w);
}

// squared distance between disjoint triangles: 6 vertex-triangle and 9
// edge-edge closest-point problems
template <typename T>
CBVH_GEOM inline T tri_tri_dist2(const V3<T> *a, const V3<T> *b)
{
    T best = pt_tri_dist2(a[0], b);
    best = fmin(best, pt_tri_dist2(a[1], b));
    best = fmin(best, pt_tri_dist2(a[2], b));
    best = fmin(best, pt_tri_dist2(b[0], a));
    best = fmin(best, pt_tri_dist2(b[1], a));
    best = fmin(best, pt_tri_dist2(b[2], a));
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int j = 0; j < 3; j++) best = fmin(best, seg_seg_dist2(a[i], a[(i + 1) % 3], b[j], b[(j + 1) % 3]));
    return best;
}

// ---------------------------------------------------------------------------
// Placement of A's vertices by a pose, and the FP32 leaf distance
// ---------------------------------------------------------------------------
struct Pose {
    float R[9], t[3];  // row-major rotation part and translation of [R | t]
};

CBVH_GEOM_INLINE V3<float> xform_f32(const Pose &P, V3<float> x)
{
    return {__builtin_fmaf(P.R[0], x.x, __builtin_fmaf(P.R[1], x.y, __builtin_fmaf(P.R[2], x.z, P.t[0]))),
            __builtin_fmaf(P.R[3], x.x, __builtin_fmaf(P.R[4], x.y, __builtin_fmaf(P.R[5], x.z, P.t[1]))),
            __builtin_fmaf(P.R[6], x.x, __builtin_fmaf(P.R[7], x.y, __builtin_fmaf(P.R[8], x.z, P.t[2])))};
}
CBVH_GEOM_INLINE V3<double> xform_f64(const Pose &P, V3<float> x)
{
    double X = x.x, Y = x.y, Z = x.z;
    return {fma((double)P.R[0], X, fma((double)P.R[1], Y, fma((double)P.R[2], Z, (double)P.t[0]))),
            fma((double)P.R[3], X, fma((double)P.R[4], Y, fma((double)P.R[5], Z, (double)P.t[1]))),
            fma((double)P.R[6], X, fma((double)P.R[7], Y, fma((double)P.R[8], Z, (double)P.t[2])))};
}
CBVH_GEOM_INLINE V3<double> to64(V3<float> x) { return {(double)x.x, (double)x.y, (double)x.z}; }

// FP32 distance of two disjoint triangles (A placed by the pose in FP32),
// evaluated on coordinates relative to A's first vertex.
CBVH_GEOM_INLINE float tri_dist_f32(const V3<float> *a, const V3<float> *b)
{
    V3<float> ar[3], br[3];
#pragma unroll
    for (int v = 0; v < 3; v++) {
        ar[v] = vsub(a[v], a[0]);
        br[v] = vsub(b[v], a[0]);
    }
    return sqrtf(tri_tri_dist2(ar, br));
}

// Distance queries: bound e on the error of an FP32 leaf distance (placement
// by the pose in FP32 plus the closest-point evaluation) for a pose with
// translation t and models whose coordinates are at most maxA and maxB in
// magnitude: every coordinate in B's frame is below |t| + 3 maxA + maxB, the
// placement errs by at most about 5u (|t| + 3 maxA) and the relative
// coordinates and closest points by a few tens of u times that scale; 256 u
// (|t| + 3.5 (maxA + maxB)) covers the sum several times over.  The
// traversal and the FP64 stage evaluate it identically.
CBVH_GEOM_INLINE float dist_err_abs(const float *pose, float maxA, float maxB)
{
    const float tx = pose[3], ty = pose[7], tz = pose[11];
    const float tnorm = sqrtf(tx * tx + ty * ty + tz * tz);
    return 256.0f * 0x1p-24f * (tnorm + 3.5f * (maxA + maxB));
}

// ---------------------------------------------------------------------------
// Oriented boxes (OBB models)
// ---------------------------------------------------------------------------
// A node's descriptor d (20 floats): (lo, hi) of its three frame
// coordinates, a word the traversal uses for the topology, eps, the frame's
// origin o and axes a0, a1, a2.  The box is {o + u0 a0 + u1 a1 + u2 a2 : u in
// the intervals}, i.e. {x_c + sum_j s_j r_j a_j : |s_j| <= 1} with centre
// x_c = o + sum_j m_j a_j, m_j and r_j the intervals' midpoints and
// half-lengths.

// Allowances of the OBB test for a pose [R | t] whose columns' Gram matrix is
// within rot_eps of the identity (so |R| <= rho = 1 + 1.5 rot_eps) and models
// whose coordinates are at most maxA and maxB in magnitude:
//   al[0] e_obb:  rounding of the centres and of D along B's unit-ish axes.
//     Every centre coordinate and frame coordinate is below about 12 max in
//     magnitude; placing A's centre, forming d = c - c_B and one dot product
//     err by a few hundred u (rho maxA + |t| + maxB); 2^-14 covers it twice;
//   al[1] e_obbA: the same along A's placed axes (length up to rho);
//   al[2] delta_C: rounding of C_kj = b_k . g_j and of the placed axes g_j,
//     per unit of extent (about 10 u rho |R|; 2^-18 rho max(1, rho));
//   al[3] eta_R = 3.1 rot_eps: (R a_i).(R a_j) - a_i.a_j is at most
//     |R^T R - I| |a_i| |a_j| <= 3 rot_eps (1 + eps)^2.
CBVH_GEOM_INLINE void obb_allowances(const float *pose, float rot_eps, float maxA, float maxB, float *al)
{
    const float rho = 1.0f + 1.5f * rot_eps;
    const float e = 0x1p-14f * (rho * maxA + maxB + fabsf(pose[3]) + fabsf(pose[7]) + fabsf(pose[11]));
    al[0] = e;
    al[1] = e * rho * 1.0625f;
    al[2] = 0x1p-18f * rho * fmaxf(1.0f, rho);
    al[3] = 3.1f * rot_eps;
}

// A's box placed by the pose, in generator form:
//   out[0..2] centre c = R x_c + t, out[3] = r0 + r1 + r2;
//   out[4 + 4j .. 6 + 4j] g_j = R a_j, out[7 + 4j] = r_j   (j = 0, 1, 2);
//   out[16] eta = eps + eta_R, a bound on |(R a_i).(R a_j) - [i == j]|;
//   out[17] radius of the placed box's circumscribed sphere (the Gram matrix
//     of the placed axes has its largest eigenvalue below 1 + 3 eta);
//   out[18], out[19] = 0.
CBVH_GEOM_INLINE void obb_place(const Pose &P, const float *d, float eta_R, float *out)
{
    const float m0 = 0.5f * (d[0] + d[1]), m1 = 0.5f * (d[2] + d[3]), m2 = 0.5f * (d[4] + d[5]);
    const float r0 = 0.5f * (d[1] - d[0]), r1 = 0.5f * (d[3] - d[2]), r2 = 0.5f * (d[5] - d[4]);
    const float *o = d + 8, *a = d + 11;
    V3<float> xc;
    xc.x = __builtin_fmaf(m2, a[6], __builtin_fmaf(m1, a[3], __builtin_fmaf(m0, a[0], o[0])));
    xc.y = __builtin_fmaf(m2, a[7], __builtin_fmaf(m1, a[4], __builtin_fmaf(m0, a[1], o[1])));
    xc.z = __builtin_fmaf(m2, a[8], __builtin_fmaf(m1, a[5], __builtin_fmaf(m0, a[2], o[2])));
    const V3<float> c = xform_f32(P, xc);
    out[0] = c.x, out[1] = c.y, out[2] = c.z, out[3] = r0 + r1 + r2;
    const float r[3] = {r0, r1, r2};
#pragma unroll
    for (int j = 0; j < 3; j++) {
        const float ax = a[3 * j], ay = a[3 * j + 1], az = a[3 * j + 2];
        out[4 + 4 * j] = __builtin_fmaf(P.R[0], ax, __builtin_fmaf(P.R[1], ay, P.R[2] * az));
        out[5 + 4 * j] = __builtin_fmaf(P.R[3], ax, __builtin_fmaf(P.R[4], ay, P.R[5] * az));
        out[6 + 4 * j] = __builtin_fmaf(P.R[6], ax, __builtin_fmaf(P.R[7], ay, P.R[8] * az));
        out[7 + 4 * j] = r[j];
    }
    const float eta = d[7] + eta_R;
    out[16] = eta;
    out[17] = sqrtf(__builtin_fmaf(r0, r0, __builtin_fmaf(r1, r1, r2 * r2))) * (1.0f + 0x1p-20f + 2.0f * eta);
    out[18] = 0.0f;
    out[19] = 0.0f;
}

// A's placed box pa (from obb_place) against B's box (descriptor bB).  Along
// any direction n the two are disjoint if
//   |n.(c - c_B)| > sum_j r_j |n.g_j| + sum_k rb_k |n.b_k|.
// The six face axes n = b_k and n = g_j give, with C_kj = |b_k . g_j|,
// D_k = b_k . d, D'_j = g_j . d and d = c - c_B,
//   gap_k  = |D_k|  - rb_k - sum_j C_kj r_j,
//   gap'_j = |D'_j| - r_j  - sum_k C_kj rb_k,
// where rb_k and r_j stand for each box's support along its own axes, exact
// for orthonormal axes.  Allowances: eps_B sum(rb) and eta sum(r) for axes
// that are not orthonormal, delta_C per unit of extent for the rounding of C
// and of the placed axes, e_obb and e_obbA for the rounding of the centres
// and of D, and 2^-20 of the large terms for the rounding of the sums.  The
// nine edge-edge axes of the full separating-axis test are left out: a
// subset of the axes never separates boxes that overlap, so the test stays
// conservative.  *sep > 0 proves the boxes disjoint.  With DIST, *lb is a
// lower bound on their distance: each gap times a lower bound on 1 / |n|
// (|b_k| <= 1 + eps_B, |g_j| <= 1 + eta + delta_C), and the gap of the
// circumscribed spheres; negative where the boxes may overlap.
template <bool DIST>
CBVH_GEOM_INLINE void obb_gap(const float *pa, const float *bB, const float *al, float *sep_out, float *lb_out)
{
    const float e_obb = al[0], e_obbA = al[1], dC = al[2];
    const float *o = bB + 8, *bk = bB + 11;
    const float epsB = bB[7], etaA = pa[16];
    float mb[3], rb[3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        mb[k] = 0.5f * (bB[2 * k] + bB[2 * k + 1]);
        rb[k] = 0.5f * (bB[2 * k + 1] - bB[2 * k]);
    }
    const float rsumB = rb[0] + rb[1] + rb[2], rsumA = pa[3];
    const float dx = pa[0] - __builtin_fmaf(mb[2], bk[6], __builtin_fmaf(mb[1], bk[3], __builtin_fmaf(mb[0], bk[0], o[0])));
    const float dy = pa[1] - __builtin_fmaf(mb[2], bk[7], __builtin_fmaf(mb[1], bk[4], __builtin_fmaf(mb[0], bk[1], o[1])));
    const float dz = pa[2] - __builtin_fmaf(mb[2], bk[8], __builtin_fmaf(mb[1], bk[5], __builtin_fmaf(mb[0], bk[2], o[2])));
    float C[3][3];
#pragma unroll
    for (int k = 0; k < 3; k++)
#pragma unroll
        for (int j = 0; j < 3; j++)
            C[k][j] = fabsf(__builtin_fmaf(bk[3 * k], pa[4 + 4 * j],
                                           __builtin_fmaf(bk[3 * k + 1], pa[5 + 4 * j], bk[3 * k + 2] * pa[6 + 4 * j])));
    const float allowB = __builtin_fmaf(epsB, rsumB, __builtin_fmaf(dC, rsumA, e_obb));
    const float allowA = __builtin_fmaf(etaA + dC, rsumA, __builtin_fmaf(dC, rsumB, e_obbA));
    float sep = -INFINITY, lb = -INFINITY;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const float D = __builtin_fmaf(bk[3 * k], dx, __builtin_fmaf(bk[3 * k + 1], dy, bk[3 * k + 2] * dz));
        const float S = __builtin_fmaf(C[k][0], pa[7], __builtin_fmaf(C[k][1], pa[11], __builtin_fmaf(C[k][2], pa[15], rb[k])));
        const float g = __builtin_fmaf(fabsf(D), 1.0f - 0x1p-20f, -S * (1.0f + 0x1p-20f)) - allowB;
        sep = fmaxf(sep, g);
        if (DIST) lb = fmaxf(lb, g * (1.0f - epsB - 0x1p-20f));
    }
#pragma unroll
    for (int j = 0; j < 3; j++) {
        const float D = __builtin_fmaf(pa[4 + 4 * j], dx, __builtin_fmaf(pa[5 + 4 * j], dy, pa[6 + 4 * j] * dz));
        const float S = __builtin_fmaf(C[0][j], rb[0], __builtin_fmaf(C[1][j], rb[1], __builtin_fmaf(C[2][j], rb[2], pa[7 + 4 * j])));
        const float g = __builtin_fmaf(fabsf(D), 1.0f - 0x1p-20f, -S * (1.0f + 0x1p-20f)) - allowA;
        sep = fmaxf(sep, g);
        if (DIST) lb = fmaxf(lb, g * (1.0f - etaA - dC - 0x1p-20f));
    }
    if (DIST) {
        const float radB = sqrtf(__builtin_fmaf(rb[0], rb[0], __builtin_fmaf(rb[1], rb[1], rb[2] * rb[2]))) *
                           (1.0f + 0x1p-20f + 2.0f * epsB);
        const float gs = sqrtf(__builtin_fmaf(dx, dx, __builtin_fmaf(dy, dy, dz * dz))) * (1.0f - 0x1p-20f) - pa[17] -
                         radB - 2.0f * e_obb;
        lb = fmaxf(lb, gs);
        // The gap along one direction found by alternating projections: B's
        // point nearest to A's centre, A's point nearest to that, B's point
        // nearest to that, each taken in the boxes' own axes as if they were
        // orthonormal (any direction is valid; this only picks a good one).
        // Along n the supports are exactly sum_j r_j |n.g_j| + sum_k rb_k |n.b_k|
        // for the boxes in generator form, so only rounding needs allowances:
        // delta_C per unit of extent for the placed axes and the dot
        // products, 2 e_obb for the centres, 2^-20 for the sums.
        const float cbx = pa[0] - dx, cby = pa[1] - dy, cbz = pa[2] - dz;  // B's centre
        // u: B's point nearest to A's centre, as an offset from B's centre
        float ux = 0.0f, uy = 0.0f, uz = 0.0f;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const float t = __builtin_fmaf(bk[3 * k], dx, __builtin_fmaf(bk[3 * k + 1], dy, bk[3 * k + 2] * dz));
            const float tc = fminf(fmaxf(t, -rb[k]), rb[k]);
            ux = __builtin_fmaf(tc, bk[3 * k], ux);
            uy = __builtin_fmaf(tc, bk[3 * k + 1], uy);
            uz = __builtin_fmaf(tc, bk[3 * k + 2], uz);
        }
        // A's point nearest to it (offset from A's centre)
        const float ex = cbx + ux - pa[0], ey = cby + uy - pa[1], ez = cbz + uz - pa[2];
        float vx = 0.0f, vy = 0.0f, vz = 0.0f;
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const float gx = pa[4 + 4 * j], gy = pa[5 + 4 * j], gz = pa[6 + 4 * j], r = pa[7 + 4 * j];
            const float t = __builtin_fmaf(gx, ex, __builtin_fmaf(gy, ey, gz * ez));
            const float tc = fminf(fmaxf(t, -r), r);
            vx = __builtin_fmaf(tc, gx, vx);
            vy = __builtin_fmaf(tc, gy, vy);
            vz = __builtin_fmaf(tc, gz, vz);
        }
        // B's point nearest to that one; n points from A's point towards it
        const float fx = pa[0] + vx - cbx, fy = pa[1] + vy - cby, fz = pa[2] + vz - cbz;
        float wx = 0.0f, wy = 0.0f, wz = 0.0f;
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const float t = __builtin_fmaf(bk[3 * k], fx, __builtin_fmaf(bk[3 * k + 1], fy, bk[3 * k + 2] * fz));
            const float tc = fminf(fmaxf(t, -rb[k]), rb[k]);
            wx = __builtin_fmaf(tc, bk[3 * k], wx);
            wy = __builtin_fmaf(tc, bk[3 * k + 1], wy);
            wz = __builtin_fmaf(tc, bk[3 * k + 2], wz);
        }
        const float nx = wx - fx, ny = wy - fy, nz = wz - fz;
        const float nn = __builtin_fmaf(nx, nx, __builtin_fmaf(ny, ny, nz * nz));
        if (nn > 0x1p-100f) {
            // n.(c_B - c) minus both supports along n
            float S = 0.0f;
#pragma unroll
            for (int j = 0; j < 3; j++)
                S = __builtin_fmaf(pa[7 + 4 * j],
                                   fabsf(__builtin_fmaf(nx, pa[4 + 4 * j], __builtin_fmaf(ny, pa[5 + 4 * j], nz * pa[6 + 4 * j]))), S);
#pragma unroll
            for (int k = 0; k < 3; k++)
                S = __builtin_fmaf(rb[k], fabsf(__builtin_fmaf(nx, bk[3 * k], __builtin_fmaf(ny, bk[3 * k + 1], nz * bk[3 * k + 2]))), S);
            const float D = -__builtin_fmaf(nx, dx, __builtin_fmaf(ny, dy, nz * dz));
            const float gn = __builtin_fmaf(D, 1.0f - 0x1p-20f, -S * (1.0f + 0x1p-20f)) * (1.0f / sqrtf(nn)) * (1.0f - 0x1p-20f);
            lb = fmaxf(lb, gn - __builtin_fmaf(dC, rsumA + rsumB, 2.0f * e_obb));
        }
    }
    *sep_out = sep;
    *lb_out = lb;
}

}  // namespace cbvh
