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

}  // namespace cbvh
