// Host (CPU) build of the leaf geometry that the traversal kernels run
// (paper_2012_05348_amd/csrc/geom.h, compiled here as plain C++), so that
// tests can drive the FP32 certified intersection test, the FP32 leaf
// distance and the OBB box test with adversarial inputs and compare them
// with exact references.
// Built by the tests with g++ -O2 -ffp-contract=off (IEEE single precision,
// fused multiply-adds only where the source writes them, as on the GPU).
#include "../paper_2012_05348_amd/csrc/geom.h"

using namespace cbvh;

namespace {
void tri(const float *p, V3<float> t[3])
{
    for (int v = 0; v < 3; v++) t[v] = {p[3 * v], p[3 * v + 1], p[3 * v + 2]};
}
Pose pose(const float *p)
{
    Pose P;
    for (int i = 0; i < 3; i++) {
        for (int j = 0; j < 3; j++) P.R[3 * i + j] = p[4 * i + j];
        P.t[i] = p[4 * i + 3];
    }
    return P;
}
}  // namespace

extern "C" {

// 0 disjoint, 1 intersecting, 2 undecided, for the float triangles as given
int gh_tri_tri_f32(const float *a9, const float *b9)
{
    V3<float> a[3], b[3];
    tri(a9, a);
    tri(b9, b);
    return tri_tri_f32(a, b);
}

// A's triangle (its own frame) placed by the pose in FP32, as the traversal does
void gh_place_f32(const float *pose12, const float *a9, float *out9)
{
    const Pose P = pose(pose12);
    V3<float> a[3];
    tri(a9, a);
    for (int v = 0; v < 3; v++) {
        const V3<float> x = xform_f32(P, a[v]);
        out9[3 * v] = x.x;
        out9[3 * v + 1] = x.y;
        out9[3 * v + 2] = x.z;
    }
}

// the traversal's leaf step for a distance query: FP32 placement, the
// certified test, and the FP32 distance when the pair is not certified
// intersecting (then *res receives the test's answer)
float gh_leaf_dist_f32(const float *pose12, const float *a9, const float *b9, int *res)
{
    const Pose P = pose(pose12);
    V3<float> a0[3], a[3], b[3];
    tri(a9, a0);
    tri(b9, b);
    for (int v = 0; v < 3; v++) a[v] = xform_f32(P, a0[v]);
    *res = tri_tri_f32(a, b);
    return *res != 1 ? tri_dist_f32(a, b) : 0.0f;
}

float gh_dist_err(const float *pose12, float maxA, float maxB) { return dist_err_abs(pose12, maxA, maxB); }

// the OBB test of the traversal: allowances of a pose, A's box placed by it,
// and the gap test against B's box (sep > 0 proves them disjoint; lb is the
// distance lower bound of distance queries)
void gh_obb_test(const float *pose12, float rot_eps, float maxA, float maxB, const float *descA, const float *descB,
                 float *sep, float *lb)
{
    const Pose P = pose(pose12);
    float al[4], pa[20], s0, l0;
    obb_allowances(pose12, rot_eps, maxA, maxB, al);
    obb_place(P, descA, al[3], pa);
    obb_gap<false>(pa, descB, al, sep, &l0);
    obb_gap<true>(pa, descB, al, &s0, lb);
}

}  // extern "C"
