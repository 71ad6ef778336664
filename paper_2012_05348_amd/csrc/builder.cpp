// Host-side BVH construction, predictor-corrector compression and treelet
// layout (the paper's section III: quantized BV descriptors coded relative to
// the parent, BVH clustered into treelets), and validation of serialized
// models.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>
#include <vector>

#include "format.h"
#include "model.h"

namespace cbvh {
namespace {

// An exact real number s + e with |e| below half the spacing of doubles at s
// (the two-sum of two doubles).  Slab values x, x+y, x-y of float
// coordinates are represented exactly this way.
struct Exact {
    double s, e;
};

inline Exact two_sum(double x, double y)
{
    Exact r;
    r.s = x + y;
    double bp = r.s - x, ap = r.s - bp;
    r.e = (x - ap) + (y - bp);
    return r;
}
inline bool exact_lt(const Exact &a, const Exact &b) { return a.s < b.s || (a.s == b.s && a.e < b.e); }
// float f <= exact value v (f and v.s are doubles; |v.e| < half spacing at v.s)
inline bool f_le(float f, const Exact &v) { double d = f; return d < v.s || (d == v.s && v.e >= 0.0); }
inline bool f_ge(float f, const Exact &v) { double d = f; return d > v.s || (d == v.s && v.e <= 0.0); }

// slab directions: x, y, z, then (18-DOP) x+y, x+z, y+z, x-y, x-z, y-z
inline Exact slab_value(const float *p, int k)
{
    switch (k) {
    case 0: return {p[0], 0.0};
    case 1: return {p[1], 0.0};
    case 2: return {p[2], 0.0};
    case 3: return two_sum(p[0], p[1]);
    case 4: return two_sum(p[0], p[2]);
    case 5: return two_sum(p[1], p[2]);
    case 6: return two_sum(p[0], -(double)p[1]);
    case 7: return two_sum(p[0], -(double)p[2]);
    default: return two_sum(p[1], -(double)p[2]);
    }
}

// largest float <= v, smallest float >= v
float round_down(const Exact &v)
{
    float f = (float)v.s;
    while (!f_le(f, v)) f = std::nextafter(f, -INFINITY);
    while (f_le(std::nextafter(f, INFINITY), v)) f = std::nextafter(f, INFINITY);
    return f;
}
float round_up(const Exact &v)
{
    float f = (float)v.s;
    while (!f_ge(f, v)) f = std::nextafter(f, INFINITY);
    while (f_ge(std::nextafter(f, -INFINITY), v)) f = std::nextafter(f, -INFINITY);
    return f;
}

struct TmpNode {
    bool leaf = false;
    uint32_t begin = 0, end = 0;     // triangle range of the subtree in `order`
    std::vector<uint32_t> children;  // indices into the temporary node array
    uint32_t depth = 0;
    Exact lo[9], hi[9];
};

struct Builder {
    const BuildParams &p;
    uint32_t K;
    std::vector<float> tri;          // [nt][9] input order
    std::vector<double> centroid;    // [nt][3] (sum of the three vertices)
    std::vector<uint32_t> order;     // triangle indices; leaves own contiguous ranges
    std::vector<TmpNode> nodes;

    explicit Builder(const BuildParams &pp) : p(pp), K(bv_slabs(pp.bv)) {}

    // one binary median split of order[b, e): longest axis of the centroid
    // bounds, sort by (centroid, input index), left part keeps full leaves
    uint32_t split(uint32_t b, uint32_t e)
    {
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (uint32_t i = b; i < e; i++)
            for (int k = 0; k < 3; k++) {
                double c = centroid[3 * (size_t)order[i] + k];
                lo[k] = std::min(lo[k], c);
                hi[k] = std::max(hi[k], c);
            }
        int ax = 0;
        for (int k = 1; k < 3; k++)
            if (hi[k] - lo[k] > hi[ax] - lo[ax]) ax = k;
        std::sort(order.begin() + b, order.begin() + e, [&](uint32_t x, uint32_t y) {
            double cx = centroid[3 * (size_t)x + ax], cy = centroid[3 * (size_t)y + ax];
            return cx < cy || (cx == cy && x < y);
        });
        uint32_t n = e - b, L = p.leaf_size;
        uint32_t leaves = (n + L - 1) / L;
        uint32_t left = L * ((leaves + 1) / 2);
        return b + left;
    }

    uint32_t build(uint32_t b, uint32_t e, uint32_t depth)
    {
        uint32_t me = (uint32_t)nodes.size();
        nodes.emplace_back();
        nodes[me].depth = depth;
        nodes[me].begin = b;
        nodes[me].end = e;
        if (e - b <= p.leaf_size) {
            nodes[me].leaf = true;
            return me;
        }
        std::vector<std::pair<uint32_t, uint32_t>> parts{{b, e}};
        for (uint32_t width = 1; width < p.branching; width *= 2) {
            std::vector<std::pair<uint32_t, uint32_t>> next;
            for (auto &r : parts) {
                if (r.second - r.first > p.leaf_size) {
                    uint32_t m = split(r.first, r.second);
                    next.push_back({r.first, m});
                    next.push_back({m, r.second});
                } else {
                    next.push_back(r);
                }
            }
            parts.swap(next);
        }
        std::vector<uint32_t> ch;
        for (auto &r : parts) ch.push_back(build(r.first, r.second, depth + 1));
        nodes[me].children = ch;
        return me;
    }

    void exact_slabs(uint32_t i)
    {
        TmpNode &n = nodes[i];
        for (uint32_t k = 0; k < K; k++) {
            n.lo[k] = {INFINITY, 0.0};
            n.hi[k] = {-INFINITY, 0.0};
        }
        if (n.leaf) {
            for (uint32_t t = n.begin; t < n.end; t++)
                for (int v = 0; v < 3; v++)
                    for (uint32_t k = 0; k < K; k++) {
                        Exact x = slab_value(&tri[9 * (size_t)order[t] + 3 * v], (int)k);
                        if (exact_lt(x, n.lo[k])) n.lo[k] = x;
                        if (exact_lt(n.hi[k], x)) n.hi[k] = x;
                    }
            return;
        }
        for (uint32_t c : n.children) {
            exact_slabs(c);
            for (uint32_t k = 0; k < K; k++) {
                if (exact_lt(nodes[c].lo[k], n.lo[k])) n.lo[k] = nodes[c].lo[k];
                if (exact_lt(n.hi[k], nodes[c].hi[k])) n.hi[k] = nodes[c].hi[k];
            }
        }
    }
};

// ---- oriented boxes ----
// A frame: origin o and axes a[k] (float32, the values the descriptor
// stores), eps >= max |a_i . a_j - [i == j]|, and M^-1 (FP64) for the
// frame coordinates u = M^-1 (x - o), M = [a0 a1 a2] by columns.
struct Frame {
    float o[3], a[3][3], eps;
    double inv[3][3];
    double pad;  // outward pad of every interval coded in this frame
};

// eigenvectors of a symmetric 3x3 matrix (cyclic Jacobi rotations), as the
// rows of V, ordered by decreasing eigenvalue
void sym_eigen3(double A[3][3], double V[3][3])
{
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) V[i][j] = i == j ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 64; sweep++) {
        double off = std::fabs(A[0][1]) + std::fabs(A[0][2]) + std::fabs(A[1][2]);
        double scale = std::fabs(A[0][0]) + std::fabs(A[1][1]) + std::fabs(A[2][2]);
        if (off <= 1e-30 * scale || off == 0.0) break;
        for (int p = 0; p < 2; p++)
            for (int q = p + 1; q < 3; q++) {
                if (A[p][q] == 0.0) continue;
                double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < 3; k++) {  // A <- J^T A J
                    double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - sn * akq;
                    A[k][q] = sn * akp + c * akq;
                }
                for (int k = 0; k < 3; k++) {
                    double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - sn * aqk;
                    A[q][k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < 3; k++) {  // rows of V are eigenvectors
                    double vp = V[p][k], vq = V[q][k];
                    V[p][k] = c * vp - sn * vq;
                    V[q][k] = sn * vp + c * vq;
                }
            }
    }
    int ord[3] = {0, 1, 2};
    std::sort(ord, ord + 3, [&](int x, int y) { return A[x][x] > A[y][y] || (A[x][x] == A[y][y] && x < y); });
    double W[3][3];
    for (int i = 0; i < 3; i++)
        for (int k = 0; k < 3; k++) W[i][k] = V[ord[i]][k];
    memcpy(V, W, sizeof W);
}

// largest float <= x, smallest float >= x (x a double)
float f32_down(double x)
{
    float f = (float)x;
    while ((double)f > x) f = std::nextafter(f, -INFINITY);
    return f;
}
float f32_up(double x)
{
    float f = (float)x;
    while ((double)f < x) f = std::nextafter(f, INFINITY);
    return f;
}

// The frame of an absolute OBB node: principal axes of the vertices of its
// triangles (order[b, e) of the builder), origin at their mean.
Frame fit_frame(const std::vector<float> &tri, const std::vector<uint32_t> &order, uint32_t b, uint32_t e)
{
    double mean[3] = {0, 0, 0};
    const double nv = 3.0 * (double)(e - b);
    for (uint32_t i = b; i < e; i++)
        for (int v = 0; v < 3; v++)
            for (int k = 0; k < 3; k++) mean[k] += tri[9 * (size_t)order[i] + 3 * v + k];
    for (int k = 0; k < 3; k++) mean[k] /= nv;
    double C[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (uint32_t i = b; i < e; i++)
        for (int v = 0; v < 3; v++) {
            double d[3];
            for (int k = 0; k < 3; k++) d[k] = tri[9 * (size_t)order[i] + 3 * v + k] - mean[k];
            for (int r = 0; r < 3; r++)
                for (int c = 0; c < 3; c++) C[r][c] += d[r] * d[c];
        }
    double V[3][3];
    sym_eigen3(C, V);
    // a right-handed frame (the third axis the cross product of the first two)
    V[2][0] = V[0][1] * V[1][2] - V[0][2] * V[1][1];
    V[2][1] = V[0][2] * V[1][0] - V[0][0] * V[1][2];
    V[2][2] = V[0][0] * V[1][1] - V[0][1] * V[1][0];
    Frame f;
    for (int k = 0; k < 3; k++) f.o[k] = (float)mean[k];
    for (int i = 0; i < 3; i++)
        for (int k = 0; k < 3; k++) f.a[i][k] = (float)V[i][k];
    // orthonormality defect of the stored axes (products of floats are exact
    // in FP64; the two additions of each entry round by at most 2^-52 of 3)
    double dev = 0.0;
    for (int i = 0; i < 3; i++)
        for (int j = i; j < 3; j++) {
            double g = 0.0;
            for (int k = 0; k < 3; k++) g += (double)f.a[i][k] * (double)f.a[j][k];
            dev = std::max(dev, std::fabs(g - (i == j ? 1.0 : 0.0)));
        }
    f.eps = f32_up(dev + 0x1p-48);
    // M^-1 = adj(M) / det(M), M[r][c] = a[c][r]
    double M[3][3];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) M[r][c] = f.a[c][r];
    double adj[3][3];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) {
            int r1 = (c + 1) % 3, r2 = (c + 2) % 3, c1 = (r + 1) % 3, c2 = (r + 2) % 3;
            adj[r][c] = M[r1][c1] * M[r2][c2] - M[r1][c2] * M[r2][c1];
        }
    double det = M[0][0] * adj[0][0] + M[0][1] * adj[1][0] + M[0][2] * adj[2][0];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) f.inv[r][c] = adj[r][c] / det;
    // the FP64 evaluation of u (a few roundings of terms bounded by |x - o|
    // times entries of M^-1 near 1) errs by far less than 2^-40 |x - o|_1:
    // intervals are widened by that much, the same in every node of the frame
    double ext = 0.0;
    for (uint32_t i = b; i < e; i++)
        for (int v = 0; v < 3; v++) {
            double s1 = 0.0;
            for (int k = 0; k < 3; k++) s1 += std::fabs((double)tri[9 * (size_t)order[i] + 3 * v + k] - (double)f.o[k]);
            ext = std::max(ext, s1);
        }
    f.pad = 0x1p-40 * ext + 0x1p-1000;
    return f;
}

// frame-coordinate intervals of the vertices of order[b, e), widened by the
// frame's pad
void frame_bounds(const Frame &f, const std::vector<float> &tri, const std::vector<uint32_t> &order, uint32_t b,
                  uint32_t e, Exact lo[3], Exact hi[3])
{
    double l[3] = {INFINITY, INFINITY, INFINITY}, h[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t i = b; i < e; i++)
        for (int v = 0; v < 3; v++) {
            double d[3];
            for (int k = 0; k < 3; k++) d[k] = (double)tri[9 * (size_t)order[i] + 3 * v + k] - (double)f.o[k];
            for (int k = 0; k < 3; k++) {
                double u = f.inv[k][0] * d[0] + f.inv[k][1] * d[1] + f.inv[k][2] * d[2];
                l[k] = std::min(l[k], u);
                h[k] = std::max(h[k], u);
            }
        }
    for (int k = 0; k < 3; k++) {
        lo[k] = {l[k] - f.pad, 0.0};
        hi[k] = {h[k] + f.pad, 0.0};
    }
}

// binary16 helpers for the half-precision descriptors: finite halves in
// value order are ranks 0 .. 2*0x7C00-1 (negatives from -65504 up to -0,
// then +0 up to +65504)
constexpr uint32_t kHalfRanks = 2u * 0x7C00u;
uint16_t half_of_rank(uint32_t r) { return r < 0x7C00u ? (uint16_t)(0x8000u | (0x7BFFu - r)) : (uint16_t)(r - 0x7C00u); }
double half_value(uint16_t h)
{
    const int e = (h >> 10) & 0x1F, m = h & 0x3FF;
    const double v = e == 0 ? std::ldexp((double)m, -24) : std::ldexp((double)(m | 0x400), e - 25);
    return (h & 0x8000u) ? -v : v;
}
inline bool d_le(double d, const Exact &v) { return d < v.s || (d == v.s && v.e >= 0.0); }
inline bool d_ge(double d, const Exact &v) { return d > v.s || (d == v.s && v.e <= 0.0); }
// largest half <= v, smallest half >= v (v within the finite half range)
uint16_t half_down(const Exact &v)
{
    uint32_t lo = 0, hi = kHalfRanks - 1;  // invariant: value(lo) <= v
    while (lo < hi) {
        uint32_t mid = (lo + hi + 1) / 2;
        if (d_le(half_value(half_of_rank(mid)), v)) lo = mid; else hi = mid - 1;
    }
    return half_of_rank(lo);
}
uint16_t half_up(const Exact &v)
{
    uint32_t lo = 0, hi = kHalfRanks - 1;  // invariant: value(hi) >= v
    while (lo < hi) {
        uint32_t mid = (lo + hi) / 2;
        if (d_ge(half_value(half_of_rank(mid)), v)) hi = mid; else lo = mid + 1;
    }
    return half_of_rank(hi);
}

// b-bit corrector codes of one slab relative to the decoded parent
// [Pl, Ph]: the largest codes whose decoded bounds still enclose [cl, ch]
void encode_slab(float Pl, float Ph, const Exact &cl, const Exact &ch, uint32_t bits, uint32_t *ql, uint32_t *qh,
                 float *lo, float *hi)
{
    const uint32_t Q = (1u << bits) - 1u;
    float E = Ph - Pl;
    float s = (E >= 0x1p-100f) ? std::ldexp(E, -(int)bits) : 0.0f;
    if (s == 0.0f) {
        *ql = *qh = 0;
        *lo = Pl;
        *hi = Ph;
        return;
    }
    auto dec_lo = [&](uint32_t q) { return std::fma((float)q, s, Pl); };
    auto dec_hi = [&](uint32_t q) { return std::fma(-(float)q, s, Ph); };
    auto clampq = [&](double x) -> uint32_t { return x <= 0 ? 0u : (x >= (double)Q ? Q : (uint32_t)x); };
    uint32_t a = clampq(std::floor((cl.s - (double)Pl) / (double)s));
    while (a > 0 && !f_le(dec_lo(a), cl)) a--;
    while (a < Q && f_le(dec_lo(a + 1), cl)) a++;
    uint32_t b = clampq(std::floor(((double)Ph - ch.s) / (double)s));
    while (b > 0 && !f_ge(dec_hi(b), ch)) b--;
    while (b < Q && f_ge(dec_hi(b + 1), ch)) b++;
    *ql = a;
    *qh = b;
    *lo = dec_lo(a);
    *hi = dec_hi(b);
}

inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

}  // namespace

std::string build_model(const float *V, uint32_t nv, const uint32_t *T, uint32_t nt, const BuildParams &p,
                        cbvh_model *m)
{
    Builder B(p);
    const uint32_t K = B.K;
    B.tri.resize(9 * (size_t)nt);
    B.centroid.resize(3 * (size_t)nt);
    float max_abs = 0.0f;
    for (uint32_t i = 0; i < nt; i++)
        for (int v = 0; v < 3; v++) {
            uint32_t vi = T[3 * (size_t)i + v];
            if (vi >= nv) return "triangle index out of range";
            for (int k = 0; k < 3; k++) {
                float x = V[3 * (size_t)vi + k];
                if (!std::isfinite(x) || std::fabs(x) >= 0x1p60f) return "vertex coordinate not finite or too large";
                B.tri[9 * (size_t)i + 3 * v + k] = x;
                max_abs = std::max(max_abs, std::fabs(x));
            }
        }
    for (uint32_t i = 0; i < nt; i++)
        for (int k = 0; k < 3; k++)
            B.centroid[3 * (size_t)i + k] = (double)B.tri[9 * (size_t)i + k] + (double)B.tri[9 * (size_t)i + 3 + k] +
                                            (double)B.tri[9 * (size_t)i + 6 + k];
    B.order.resize(nt);
    std::iota(B.order.begin(), B.order.end(), 0u);
    B.nodes.reserve(2 * (size_t)nt / std::max(1u, p.leaf_size) + 8);
    B.build(0, nt, 0);
    const bool obb = p.bv == kBvObb;
    if (obb && !(p.bits == 0 || bits_are_codes(p.bits))) return "OBB models take bits 0, 8 or 16";
    if (!obb) B.exact_slabs(0);

    const uint32_t stride = code_stride_for(K, p.bits, p.bv);
    const uint32_t n_nodes = (uint32_t)B.nodes.size();
    if (n_nodes > kIndexMask) return "too many nodes";

    // ---- treelets: bounded-size connected parts of the tree of sibling groups ----
    // A group is the children of one node (or the root alone).  Bottom-up,
    // every group accumulates the bytes of its subtree; whenever that exceeds
    // the budget, its heaviest child subtrees are cut off until it fits (the
    // greedy that minimizes the number of parts of a tree under a size bound).
    // Every cut group becomes the top group of its own treelet and stores its
    // bounds absolute; the budget of the relative parts leaves room for that.
    const uint64_t rel_node = 4 + stride;
    const bool codes_mode = bits_are_codes(p.bits);
    if (p.bits == kBitsFp16 && max_abs * (K == 9 ? 2.0f : 1.0f) >= 32768.0f)
        return "FP16 descriptors need |coordinate| < 32768 (16384 for 18-DOPs)";
    const uint64_t abs_node = codes_mode ? 4 + stride + 4 * (uint64_t)abs_words(K, p.bv) : 4 + stride;
    std::vector<std::vector<uint32_t>> groups;   // node ids per group, breadth-first
    std::vector<std::vector<uint32_t>> kids;     // child groups of each group
    groups.push_back({0u});
    kids.emplace_back();
    for (size_t g = 0; g < groups.size(); g++)
        for (uint32_t x : groups[g])
            if (!B.nodes[x].leaf) {
                uint32_t cg = (uint32_t)groups.size();
                groups.push_back(B.nodes[x].children);
                kids.emplace_back();
                kids[g].push_back(cg);
            }
    const uint64_t extra = (uint64_t)p.branching * (abs_node - rel_node);
    const uint64_t budget = p.treelet_bytes > extra + rel_node * p.branching ? p.treelet_bytes - extra
                                                                             : rel_node * p.branching;
    std::vector<uint64_t> weight(groups.size(), 0);
    std::vector<uint8_t> cut(groups.size(), 0);
    for (size_t gi = groups.size(); gi-- > 0;) {
        uint64_t total = rel_node * groups[gi].size();
        std::vector<uint32_t> ch = kids[gi];
        for (uint32_t c : ch) total += weight[c];
        std::sort(ch.begin(), ch.end(), [&](uint32_t x, uint32_t y) { return weight[x] > weight[y] || (weight[x] == weight[y] && x < y); });
        for (size_t k = 0; k < ch.size() && total > budget; k++) {
            cut[ch[k]] = 1;
            total -= weight[ch[k]];
        }
        weight[gi] = total;
    }
    std::vector<std::vector<uint32_t>> treelet_groups_flat;  // per treelet: node ids, groups concatenated
    std::vector<uint8_t> is_top(n_nodes, 0);
    {
        std::vector<uint32_t> tops{0u};
        for (size_t ti = 0; ti < tops.size(); ti++) {
            std::vector<uint32_t> nodes_in;
            std::vector<uint32_t> q{tops[ti]};
            for (uint32_t x : groups[tops[ti]]) is_top[x] = 1;
            for (size_t qi = 0; qi < q.size(); qi++) {
                uint32_t g = q[qi];
                for (uint32_t x : groups[g]) nodes_in.push_back(x);
                for (uint32_t c : kids[g]) {
                    if (cut[c]) tops.push_back(c);
                    else q.push_back(c);
                }
            }
            treelet_groups_flat.push_back(nodes_in);
        }
    }
    const uint32_t n_treelets = (uint32_t)treelet_groups_flat.size();

    // ---- final numbering ----
    std::vector<uint32_t> newid(n_nodes), oldid(n_nodes);
    std::vector<uint32_t> treelet_first(n_treelets + 1);
    {
        uint32_t c = 0;
        for (uint32_t t = 0; t < n_treelets; t++) {
            treelet_first[t] = c;
            for (uint32_t x : treelet_groups_flat[t]) {
                newid[x] = c;
                oldid[c] = x;
                c++;
            }
        }
        treelet_first[n_treelets] = c;
        if (c != n_nodes) return "internal error: treelet numbering";
    }

    // leaf-order triangles follow the leaves in node order
    std::vector<uint32_t> perm;
    perm.reserve(nt);
    std::vector<uint32_t> topo(n_nodes);
    uint32_t n_abs = 0, depth = 0, n_inner = 0, n_leaves = 0;
    std::vector<uint32_t> abs_index(n_nodes, 0xFFFFFFFFu);
    for (uint32_t i = 0; i < n_nodes; i++) {
        const TmpNode &nd = B.nodes[oldid[i]];
        depth = std::max(depth, nd.depth);
        bool absolute = codes_mode && is_top[oldid[i]];
        if (absolute) abs_index[i] = n_abs++;
        if (nd.leaf) {
            uint32_t first = (uint32_t)perm.size();
            for (uint32_t t = nd.begin; t < nd.end; t++) perm.push_back(B.order[t]);
            topo[i] = make_topo(first, nd.end - nd.begin, true, absolute);
            n_leaves++;
        } else {
            uint32_t first = newid[nd.children[0]];
            for (size_t c = 1; c < nd.children.size(); c++)
                if (newid[nd.children[c]] != first + c) return "internal error: sibling group not contiguous";
            topo[i] = make_topo(first, (uint32_t)nd.children.size(), false, absolute);
            n_inner++;
        }
    }

    // ---- oriented boxes: frames of the absolute nodes (every node without
    // codes), inherited by relative nodes; intervals in the node's frame ----
    std::vector<uint32_t> frame_of(obb ? n_nodes : 0);
    std::vector<Frame> frames;
    if (obb) {
        for (uint32_t i = 0; i < n_nodes; i++) {
            TmpNode &nd = B.nodes[oldid[i]];
            if (p.bits == 0 || topo_abs(topo[i])) {
                frame_of[i] = (uint32_t)frames.size();
                frames.push_back(fit_frame(B.tri, B.order, nd.begin, nd.end));
            } else if (i == 0) {
                return "internal error: relative root";
            }
            if (!topo_leaf(topo[i]))
                for (uint32_t c = 0; c < topo_count(topo[i]); c++) {
                    const uint32_t ch = topo_first(topo[i]) + c;
                    if (!(p.bits == 0 || topo_abs(topo[ch]))) frame_of[ch] = frame_of[i];
                }
            frame_bounds(frames[frame_of[i]], B.tri, B.order, nd.begin, nd.end, nd.lo, nd.hi);
        }
    }
    auto put_frame = [&](float *w, uint32_t i) {
        const Frame &f = frames[frame_of[i]];
        w[6] = 0.0f;
        w[kObbEps] = f.eps;
        for (int k = 0; k < 3; k++) w[kObbOrigin + k] = f.o[k];
        for (int a = 0; a < 3; a++)
            for (int k = 0; k < 3; k++) w[kObbAxes + 3 * a + k] = f.a[a][k];
    };

    // ---- encode, top-down (parents precede children in node order) ----
    std::vector<uint8_t> codes((size_t)n_nodes * stride, 0);
    const uint32_t AW = abs_words(K, p.bv);
    std::vector<float> absb((size_t)n_abs * AW);
    std::vector<float> dec((size_t)n_nodes * 2 * K);
    std::vector<uint32_t> parent(n_nodes, 0xFFFFFFFFu);
    for (uint32_t i = 0; i < n_nodes; i++)
        if (!topo_leaf(topo[i]))
            for (uint32_t c = 0; c < topo_count(topo[i]); c++) parent[topo_first(topo[i]) + c] = i;
    const uint32_t Kc = K;
    for (uint32_t i = 0; i < n_nodes; i++) {
        const TmpNode &nd = B.nodes[oldid[i]];
        float *d = &dec[(size_t)i * 2 * Kc];
        uint8_t *code = &codes[(size_t)i * stride];
        if (p.bits == kBitsFp16) {
            for (uint32_t k = 0; k < Kc; k++) {
                uint16_t a = half_down(nd.lo[k]), b = half_up(nd.hi[k]);
                memcpy(code + 4 * k, &a, 2);
                memcpy(code + 4 * k + 2, &b, 2);
                d[2 * k] = (float)half_value(a);
                d[2 * k + 1] = (float)half_value(b);
            }
            continue;
        }
        if (p.bits == 0 || topo_abs(topo[i])) {
            for (uint32_t k = 0; k < Kc; k++) {
                d[2 * k] = round_down(nd.lo[k]);
                d[2 * k + 1] = round_up(nd.hi[k]);
            }
            float wds[kObbWords];
            memcpy(wds, d, 8 * (size_t)Kc);
            if (obb) put_frame(wds, i);
            if (p.bits == 0) {
                memcpy(code, wds, 4 * (size_t)AW);
            } else {
                uint32_t ai = abs_index[i];
                memcpy(code, &ai, 4);
                memcpy(&absb[(size_t)ai * AW], wds, 4 * (size_t)AW);
            }
            continue;
        }
        if (parent[i] == 0xFFFFFFFFu) return "internal error: relative node without parent";
        const float *P = &dec[(size_t)parent[i] * 2 * Kc];
        for (uint32_t k = 0; k < Kc; k++) {
            uint32_t ql, qh;
            encode_slab(P[2 * k], P[2 * k + 1], nd.lo[k], nd.hi[k], p.bits, &ql, &qh, &d[2 * k], &d[2 * k + 1]);
            if (p.bits == 8) {
                code[2 * k] = (uint8_t)ql;
                code[2 * k + 1] = (uint8_t)qh;
            } else {
                uint16_t a = (uint16_t)ql, b = (uint16_t)qh;
                memcpy(code + 4 * k, &a, 2);
                memcpy(code + 4 * k + 2, &b, 2);
            }
        }
    }

    // ---- serialize ----
    BlobHeader h;
    memset(&h, 0, sizeof h);
    h.magic = kMagic;
    h.version = kVersion;
    h.bv = p.bv;
    h.K = K;
    h.bits = p.bits;
    h.branching = p.branching;
    h.leaf_size = p.leaf_size;
    h.n_nodes = n_nodes;
    h.n_tris = nt;
    h.n_abs = n_abs;
    h.n_treelets = n_treelets;
    h.code_stride = stride;
    h.depth = depth;
    h.treelet_bytes = p.treelet_bytes;
    h.max_abs_coord = max_abs;
    uint64_t cur = kHeaderBytes;
    auto place = [&](uint64_t bytes) {
        cur = align_up(cur, kSectionAlign);
        uint64_t o = cur;
        cur += bytes;
        return o;
    };
    h.off_topo = place(4ull * n_nodes);
    h.off_codes = place((uint64_t)stride * n_nodes);
    h.off_abs = place(4ull * absb.size());
    h.off_tris = place(36ull * nt);
    h.off_perm = place(4ull * nt);
    h.off_treelets = place(4ull * (n_treelets + 1));
    h.total = align_up(cur, kSectionAlign);
    m->blob.assign(h.total, 0);
    uint8_t *o = m->blob.data();
    memcpy(o, &h, sizeof h);
    memcpy(o + h.off_topo, topo.data(), 4ull * n_nodes);
    memcpy(o + h.off_codes, codes.data(), codes.size());
    if (!absb.empty()) memcpy(o + h.off_abs, absb.data(), 4 * absb.size());
    for (uint32_t i = 0; i < nt; i++) memcpy(o + h.off_tris + 36ull * i, &B.tri[9 * (size_t)perm[i]], 36);
    memcpy(o + h.off_perm, perm.data(), 4ull * nt);
    memcpy(o + h.off_treelets, treelet_first.data(), 4ull * (n_treelets + 1));
    m->hdr = h;
    m->n_inner = n_inner;
    m->n_leaves = n_leaves;
    m->descriptor_bytes = (uint64_t)stride * n_nodes + 4ull * absb.size();
    return std::string();
}

std::string validate_blob(const uint8_t *blob, size_t n, BlobHeader *hp, uint32_t *n_inner, uint32_t *n_leaves)
{
    if (!blob || n < kHeaderBytes) return "blob too small";
    BlobHeader h;
    memcpy(&h, blob, sizeof h);
    if (h.magic != kMagic || h.version != kVersion) return "bad magic or version";
    if (!((h.bv == kBvAabb && h.K == 3) || (h.bv == kBvDop18 && h.K == 9) || (h.bv == kBvObb && h.K == 3)))
        return "bad BV type";
    if (!(h.bits == 0 || bits_are_codes(h.bits) || h.bits == kBitsFp16)) return "bad code width";
    if (h.bv == kBvObb && h.bits == kBitsFp16) return "OBB models take bits 0, 8 or 16";
    if (!(h.branching == 2 || h.branching == 4 || h.branching == 8)) return "bad branching factor";
    if (h.leaf_size < 1 || h.leaf_size > kMaxLeaf) return "bad leaf size";
    if (h.code_stride != code_stride_for(h.K, h.bits, h.bv)) return "bad code stride";
    if (h.n_nodes < 1 || h.n_nodes > kIndexMask || h.n_tris < 1 || h.n_tris > kIndexMask) return "bad counts";
    if (h.total != n) return "size mismatch";
    auto fits = [&](uint64_t off, uint64_t bytes) { return off >= kHeaderBytes && off <= n && bytes <= n - off; };
    if (!fits(h.off_topo, 4ull * h.n_nodes) || !fits(h.off_codes, (uint64_t)h.code_stride * h.n_nodes) ||
        !fits(h.off_abs, 4ull * abs_words(h.K, h.bv) * h.n_abs) || !fits(h.off_tris, 36ull * h.n_tris) ||
        !fits(h.off_perm, 4ull * h.n_tris) || !fits(h.off_treelets, 4ull * ((uint64_t)h.n_treelets + 1)))
        return "section out of range";
    if (h.off_topo % 4 || h.off_codes % 4 || h.off_abs % 4 || h.off_tris % 4 || h.off_perm % 4) return "misaligned section";
    const uint32_t *topo = (const uint32_t *)(blob + h.off_topo);
    std::vector<uint32_t> depth(h.n_nodes, 0xFFFFFFFFu);
    std::vector<uint8_t> tri_seen(h.n_tris, 0);
    depth[0] = 0;
    uint32_t max_depth = 0, inner = 0, leaves = 0;
    for (uint32_t i = 0; i < h.n_nodes; i++) {
        if (depth[i] == 0xFFFFFFFFu) return "node without parent";
        uint32_t w = topo[i];
        max_depth = std::max(max_depth, depth[i]);
        if (topo_abs(w)) {
            if (!bits_are_codes(h.bits)) return "absolute flag in a model without codes";
            uint32_t ai;
            memcpy(&ai, blob + h.off_codes + (uint64_t)h.code_stride * i, 4);
            if (ai >= h.n_abs) return "absolute index out of range";
        } else if (i == 0 && bits_are_codes(h.bits)) {
            return "root not absolute";
        }
        uint32_t first = topo_first(w), cnt = topo_count(w);
        if (topo_leaf(w)) {
            leaves++;
            if (cnt > h.leaf_size || (uint64_t)first + cnt > h.n_tris) return "bad leaf range";
            for (uint32_t t = first; t < first + cnt; t++) {
                if (tri_seen[t]) return "leaf ranges overlap";
                tri_seen[t] = 1;
            }
        } else {
            inner++;
            if (cnt < 2 || cnt > h.branching || first <= i || (uint64_t)first + cnt > h.n_nodes) return "bad child range";
            for (uint32_t c = first; c < first + cnt; c++) {
                if (depth[c] != 0xFFFFFFFFu) return "node with two parents";
                depth[c] = depth[i] + 1;
            }
        }
    }
    for (uint32_t t = 0; t < h.n_tris; t++)
        if (!tri_seen[t]) return "triangle in no leaf";
    if (max_depth != h.depth) return "depth mismatch";
    const uint32_t *perm = (const uint32_t *)(blob + h.off_perm);
    std::fill(tri_seen.begin(), tri_seen.end(), 0);
    for (uint32_t t = 0; t < h.n_tris; t++) {
        if (perm[t] >= h.n_tris || tri_seen[perm[t]]) return "perm is not a permutation";
        tri_seen[perm[t]] = 1;
    }
    *hp = h;
    *n_inner = inner;
    *n_leaves = leaves;
    return std::string();
}

}  // namespace cbvh
