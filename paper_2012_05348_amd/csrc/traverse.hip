// Simultaneous traversal of two compressed BVHs on gfx950 (Algorithm 1 of
// Tan, Weller, Zachmann, "Compressed Bounding Volume Hierarchies for
// Collision Detection & Proximity Query"), one wavefront per pose.
//
// Per wave, in LDS:
//   records  decoded BVs (topology word + 2K float bounds; an OBB's whole
//            descriptor with its frame) grouped in LIFO frames; a frame
//            holds the children decoded by one node step and is the
//            predictor for the next level's codes;
//   entries  pending node pairs (A record, B record, frame id), LIFO;
//   leafq    pending leaf pairs (two leaf topology words);
//   ta       A's records of the current frame moved into B's frame (OBB
//            models: A's boxes placed by the pose, in tsph);
//   pose     the current pose and its rounding allowances; statistics.
//
// Node step: pop up to 8 entries whose child-pair tests fit in 64 lanes,
// decode the children (one lane per child) into a new frame, transform A's
// children with the pose's support-function coefficients, test every child
// pair in its own lane (Algorithm 1's "a_i and b_j intersect", or a BV
// distance lower bound), and compact the survivors with ballot + mbcnt into
// the entry stack (inner pairs; the most promising one on top) or the leaf
// queue (leaf pairs).
// Leaf step: up to 64 triangle pairs, one per lane (checkPrimitives);
// pairs that FP32 cannot decide go to a separate FP64 kernel.
//
// A pose whose next node step would not fit its LDS state hands all of its
// pending pairs to the device-wide item queue (other waves finish them);
// if the queue cannot take them (helpers have left, or it is full) the pose
// is flagged CBVH_POSE_STACK_OVERFLOW.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#include <mutex>

#include "format.h"
#include "geom.h"
#include "kernels.h"

namespace cbvh {
namespace {

constexpr int WAVE = 64;
constexpr uint32_t kMaxWavesPerGroup = 4;            // waves per workgroup (the launch's workgroup shape), most
constexpr int PMAX = 8;                              // entries popped by one node step (most)
constexpr uint32_t TMAX = 64;                        // child-pair tests of one node step (most): one pass
constexpr uint32_t AMAX = 32;                        // A records of one node step (most)
constexpr int TA_MAX = (int)AMAX;                    // A records transformed per step
constexpr int MAX_FRAMES = 64;
constexpr uint32_t REC_BITS = 13;                    // entry: recA | recB << 13 | frame << 26
constexpr uint32_t REC_MASK = (1u << REC_BITS) - 1u;

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}
__device__ __forceinline__ uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
// square root for the BV bounds: the hardware instruction (within 1 ulp),
// whose error the bounds' 2^-20 relative factors cover, instead of the
// correctly rounded expansion (about 15 instructions)
__device__ __forceinline__ float bound_sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ uint32_t lane_of(uint32_t x, int l) { return __builtin_amdgcn_readlane(x, l); }
// a float not below the exact sum a + b, for a + b >= 0 (distances plus
// error allowances): the sum rounded to nearest, then the next float up
// (the same as nextafterf(a + b, INFINITY) there, in two instructions
// instead of a library call; an infinite sum is kept)
__device__ __forceinline__ float add_up(float a, float b)
{
    const float x = a + b;
    return x < INFINITY ? __uint_as_float(__float_as_uint(x) + 1u) : x;
}
__device__ __forceinline__ uint32_t mbcnt(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
// DPP move with an identity for lanes that have no source (or sit in a row
// the row mask leaves out): GFX9 controls row_shr:n = 0x110 + n,
// row_bcast:15 = 0x142 (lane 15 of each row to the next row), row_bcast:31
// = 0x143 (lane 31 to rows 2 and 3).
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_or(uint32_t identity, uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)identity, (int)v, CTRL, ROWS, 0xF, false);
}
// minimum over the wave (all lanes active): a min-scan inside each row of 16
// lanes, then the row results carried across rows; lane 63 ends with the
// wave's minimum.  All register-to-register (no LDS round trips).
__device__ __forceinline__ float wave_min(float v)
{
    // on keys that order as the floats do (sign bit flipped for positive
    // values, every bit for negative ones), so that each step is an integer
    // minimum the DPP move folds into
    const uint32_t b = __float_as_uint(v);
    uint32_t k = b ^ ((uint32_t)((int32_t)b >> 31) | 0x80000000u);
    const uint32_t top = 0xFFFFFFFFu;
    k = min(k, dpp_or<0x111, 0xF>(top, k));
    k = min(k, dpp_or<0x112, 0xF>(top, k));
    k = min(k, dpp_or<0x114, 0xF>(top, k));
    k = min(k, dpp_or<0x118, 0xF>(top, k));
    k = min(k, dpp_or<0x142, 0xA>(top, k));
    k = min(k, dpp_or<0x143, 0xC>(top, k));
    k = __builtin_amdgcn_readlane(k, 63);
    return __uint_as_float(k ^ ((k & 0x80000000u) ? 0x80000000u : 0xFFFFFFFFu));
}
// DPP row shifts (within each row of 16 lanes; 0 where there is no source lane)
template <int N>
__device__ __forceinline__ uint32_t row_shr(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x110 | N, 0xF, 0xF, true);
}
template <int N>
__device__ __forceinline__ uint32_t row_shl(uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x100 | N, 0xF, 0xF, true);
}
// value of x in lane src (all lanes must be active)
__device__ __forceinline__ uint32_t gather(uint32_t x, uint32_t src)
{
    return (uint32_t)__builtin_amdgcn_ds_bpermute((int)(src << 2), (int)x);
}
// inclusive prefix sum over the wave (all lanes active), with DPP: a scan
// inside each row of 16 lanes, then row totals carried to the later rows
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, uint32_t)
{
    v += dpp_or<0x111, 0xF>(0u, v);
    v += dpp_or<0x112, 0xF>(0u, v);
    v += dpp_or<0x114, 0xF>(0u, v);
    v += dpp_or<0x118, 0xF>(0u, v);
    v += dpp_or<0x142, 0xA>(0u, v);
    v += dpp_or<0x143, 0xC>(0u, v);
    return v;
}

// ---------------------------------------------------------------------------
// per-wave state layout (identical on host and device)
// ---------------------------------------------------------------------------
// A record is one decoded BV: 2K bounds (lo, hi per slab), its topology word
// and one pad word, 16-byte aligned so that it moves in 16-byte LDS accesses.
// An OBB record is its node's whole descriptor (frame included), with the
// topology word in the descriptor's word 6.
__host__ __device__ constexpr uint32_t rec_words(uint32_t K, bool obb = false) { return obb ? kObbWords : 2 * K + 2; }
// words a decode produces per node: the bounds, or an OBB's whole descriptor
__host__ __device__ constexpr uint32_t dec_words(uint32_t K, bool obb) { return obb ? kObbWords : 2 * K; }
// Collision queries keep both topology words in each pending entry (one LDS
// access pops an entry); distance queries, whose stacks are far deeper, read
// them from the records.
__host__ __device__ constexpr bool topo_in_entry(int mode) { return mode != MODE_DIST; }

struct Layout {
    uint32_t ctr, pz, xf, rec, ta, ta_topo, tsph, ent, ent_tp, ent_lb, lq, lq_lb, lscan, total;
};

__host__ __device__ inline Layout make_layout(uint32_t K, int mode, StackLimits lim, bool obb)
{
    Layout L;
    uint32_t o = 0;
    auto take = [&](uint32_t bytes) {
        uint32_t r = o;
        o += (bytes + 15u) & ~15u;
        return r;
    };
    L.ctr = take(8 * C_NUM);
    L.pz = take(80);
    L.xf = take(32 * K);
    L.rec = take(4 * rec_words(K, obb) * lim.records);
    // AABB distance tests and OBB tests read no support-function transform
    L.ta = ((mode == MODE_DIST && K == 3) || obb) ? o : take(4 * rec_words(K) * TA_MAX);
    L.ta_topo = take(4 * TA_MAX);
    // A's records placed by the pose: sphere and half extents (2 float4), or
    // the placed OBB (5 float4)
    L.tsph = obb ? take(80 * TA_MAX) : (mode == MODE_DIST || K == 3) ? take(32 * TA_MAX) : o;
    L.ent = take(4 * lim.entries);
    L.ent_tp = topo_in_entry(mode) ? take(8 * lim.entries) : o;
    L.ent_lb = mode == MODE_DIST ? take(4 * lim.entries) : o;
    L.lq = take(8 * lim.leafq);
    L.lq_lb = mode == MODE_DIST ? take(4 * lim.leafq) : o;
    L.lscan = take(4 * WAVE);
    L.total = o;
    return L;
}

// slab directions of the AABB (first 3) and the 18-DOP (all 9)
__device__ __forceinline__ void slab_dir(int k, int v[3])
{
    // x, y, z, x+y, x+z, y+z, x-y, x-z, y-z
    v[0] = (k == 0 || k == 3 || k == 4 || k == 6 || k == 7) ? 1 : 0;
    v[1] = (k == 1 || k == 3 || k == 5) ? 1 : (k == 6 ? -1 : (k == 8 ? 1 : 0));
    v[2] = (k == 2 || k == 4 || k == 5) ? 1 : ((k == 7 || k == 8) ? -1 : 0);
}

// u = sum alpha_m * sign_m * n(axis_m) with alpha >= 0 over three normals
// of the fan of the 18 DOP normals {+-x, +-y, +-z, +-(x+-y), +-(x+-z),
// +-(y+-z)}: the fan splits every octant into 4 triangular cones (a corner
// cone per axis and the middle cone of the three diagonals).
__device__ inline void dop18_cone(const double u[3], double alpha[3], int axis[3], int sgn[3])
{
    int sx = u[0] >= 0 ? 1 : -1, sy = u[1] >= 0 ? 1 : -1, sz = u[2] >= 0 ? 1 : -1;
    double a = fabs(u[0]), b = fabs(u[1]), c = fabs(u[2]);
    int gxy = sx * sy > 0 ? 3 : 6, gxz = sx * sz > 0 ? 4 : 7, gyz = sy * sz > 0 ? 5 : 8;
    if (a >= b + c) {
        alpha[0] = a - b - c; axis[0] = 0; sgn[0] = sx;
        alpha[1] = b; axis[1] = gxy; sgn[1] = sx;
        alpha[2] = c; axis[2] = gxz; sgn[2] = sx;
    } else if (b >= a + c) {
        alpha[0] = b - a - c; axis[0] = 1; sgn[0] = sy;
        alpha[1] = a; axis[1] = gxy; sgn[1] = sx;
        alpha[2] = c; axis[2] = gyz; sgn[2] = sy;
    } else if (c >= a + b) {
        alpha[0] = c - a - b; axis[0] = 2; sgn[0] = sz;
        alpha[1] = a; axis[1] = gxz; sgn[1] = sx;
        alpha[2] = b; axis[2] = gyz; sgn[2] = sy;
    } else {
        alpha[0] = 0.5 * (a + b - c); axis[0] = gxy; sgn[0] = sx;
        alpha[1] = 0.5 * (a + c - b); axis[1] = gxz; sgn[1] = sx;
        alpha[2] = 0.5 * (b + c - a); axis[2] = gyz; sgn[2] = sy;
    }
}

// Per-pose setup (lanes 0..K-1, one slab axis v_k of B each).  The result
// for slab k is two float4: (c_0, c_1, c_2, packed generator indices) and
// (vtU, vtL, 0, 0), read back with two 16-byte LDS loads.  A's node
// polytope {x : lo_j <= n_j.x <= hi_j} moved by the pose projects onto v_k
// inside [L_k, U_k] with
//   U_k = v_k.t + sum_m alpha_m d_m   (support function bound: any alpha >= 0
//   with sum alpha_m n_m = R^T v_k bounds the support of the polytope),
// d_m the bound of generator m (hi for +n, -lo for -n).  Written as
//   U_k = vtU_k + sum_m c_m b[up_m],  L_k = vtL_k + sum_m c_m b[up_m ^ 1]
// with c_m = sign_m alpha_m and b the record's (lo, hi) array.  vtU/vtL
// carry a pad covering every FP32 rounding of the bound's evaluation.
template <int K>
__device__ void pose_setup(const float *P, float maxA, float4 *xf, uint32_t lane)
{
    if (lane >= (uint32_t)K) return;
    double R[3][3], t[3];
#pragma unroll
    for (int i = 0; i < 3; i++) {
#pragma unroll
        for (int j = 0; j < 3; j++) R[i][j] = (double)P[4 * i + j];
        t[i] = (double)P[4 * i + 3];
    }
    int v[3];
    slab_dir((int)lane, v);
    double u[3];
    for (int j = 0; j < 3; j++) u[j] = R[0][j] * v[0] + R[1][j] * v[1] + R[2][j] * v[2];
    double vt = t[0] * v[0] + t[1] * v[1] + t[2] * v[2];
    double alpha[3];
    int axis[3], sgn[3];
    if (K == 3) {
        for (int m = 0; m < 3; m++) {
            alpha[m] = fabs(u[m]);
            axis[m] = m;
            sgn[m] = u[m] >= 0 ? 1 : -1;
        }
    } else {
        dop18_cone(u, alpha, axis, sgn);
    }
    double asum = alpha[0] + alpha[1] + alpha[2];
    double tmax = fmax(fabs(t[0]), fmax(fabs(t[1]), fabs(t[2])));
    double vn1 = fabs((double)v[0]) + fabs((double)v[1]) + fabs((double)v[2]);
    double SA = (K == 9 ? 2.0 : 1.0) * (double)maxA * (1.0 + 0x1p-20);
    double pad = 8.0 * 0x1p-24 * (vn1 * tmax + asum * SA) + 0x1p-120;
    uint32_t packed = 0;
    float c[3];
    for (int m = 0; m < 3; m++) {
        c[m] = (float)(sgn[m] * alpha[m]);
        packed |= (uint32_t)(2 * axis[m] + (sgn[m] > 0 ? 1 : 0)) << (8 * m);
    }
    xf[2 * lane] = make_float4(c[0], c[1], c[2], __uint_as_float(packed));
    xf[2 * lane + 1] = make_float4(__double2float_ru(vt + pad), __double2float_rd(vt - pad), 0.0f, 0.0f);
}

// Reads of model data through global-address-space pointers: the model
// pointers reach the kernel through structures in memory (and through
// selects between the two models), so the compiler would otherwise emit
// flat loads, whose waits also drain every outstanding LDS access.
template <typename T>
__device__ __forceinline__ T gload(const void *p)
{
    return *(const __attribute__((address_space(1))) T *)p;
}

// Raw descriptor words of one node: K 16-bit code pairs (one word each),
// K 8-bit code pairs (one 16-bit load each), K binary16 pairs, or 2K FP32
// bounds.  All of them are read up front, before the topology word is
// known, so that a node costs one memory round trip.
template <int K, int BITS, bool OBB = false>
struct NodeWords {
    static constexpr int N = BITS == 0 ? (int)dec_words(K, OBB) : K;
    uint32_t w[N];
};

template <int K, int BITS, bool OBB = false>
__device__ __forceinline__ void load_node(const DevModel &M, uint32_t node, uint32_t &topo, NodeWords<K, BITS, OBB> &nw)
{
    topo = gload<uint32_t>(M.topo + node);
    const uint8_t *code = M.codes + (size_t)node * M.stride;
#pragma unroll
    for (int k = 0; k < NodeWords<K, BITS, OBB>::N; k++)
        nw.w[k] = BITS == 8 ? (uint32_t)gload<uint16_t>(code + 2 * k) : gload<uint32_t>(code + 4 * k);
}

// Decode one node's 2K bounds (lo, hi per slab) from its parent's decoded
// bounds: E = Ph - Pl, s = E * 2^-BITS (0 if E < 2^-100), lo = fma(ql, s, Pl),
// hi = fma(-qh, s, Ph).  Absolute nodes (treelet tops) and uncompressed
// models read FP32 bounds instead, half-precision models binary16 bounds.
// An OBB node decoded from codes keeps its parent's frame (words 2K on).
template <int K, int BITS, bool OBB = false>
__device__ __forceinline__ void decode_rel(const NodeWords<K, BITS, OBB> &nw, const float *parent,
                                           float out[dec_words(K, OBB)])
{
    if constexpr (BITS == (int)kBitsFp16) {
        // binary16 absolute bounds, widened exactly
#pragma unroll
        for (int k = 0; k < K; k++) {
            out[2 * k] = (float)__builtin_bit_cast(_Float16, (uint16_t)(nw.w[k] & 0xFFFFu));
            out[2 * k + 1] = (float)__builtin_bit_cast(_Float16, (uint16_t)(nw.w[k] >> 16));
        }
    } else if constexpr (BITS == 0) {
#pragma unroll
        for (int k = 0; k < (int)dec_words(K, OBB); k++) out[k] = __uint_as_float(nw.w[k]);
    } else {
        if constexpr (OBB) {
#pragma unroll
            for (int k = 2 * K; k < (int)kObbWords; k++) out[k] = parent[k];
        }
        const float scale = 1.0f / (float)(1u << (BITS & 31));
#pragma unroll
        for (int k = 0; k < K; k++) {
            const uint32_t w = nw.w[k];
            const uint32_t ql = BITS == 8 ? (w & 0xFFu) : (w & 0xFFFFu);
            const uint32_t qh = BITS == 8 ? (w >> 8) : (w >> 16);
            float Pl = parent[2 * k], Ph = parent[2 * k + 1];
            float E = Ph - Pl;
            float s = E >= 0x1p-100f ? E * scale : 0.0f;
            out[2 * k] = __builtin_fmaf((float)ql, s, Pl);
            out[2 * k + 1] = __builtin_fmaf(-(float)qh, s, Ph);
        }
    }
}

// an absolute node of a coded model: the first four code bytes hold its
// index in the FP32 table
template <int K, int BITS, bool OBB = false>
__device__ __forceinline__ void decode_abs(const DevModel &M, const NodeWords<K, BITS, OBB> &nw,
                                           float out[dec_words(K, OBB)])
{
    constexpr uint32_t DW = dec_words(K, OBB);
    const uint32_t ai = BITS == 8 ? (nw.w[0] | (nw.w[1] << 16)) : nw.w[0];
    const uint64_t *c = (const uint64_t *)(M.absb + (size_t)ai * DW);
#pragma unroll
    for (int k = 0; k < (int)DW / 2; k++) {
        const uint64_t w = gload<uint64_t>(c + k);
        out[2 * k] = __uint_as_float((uint32_t)w);
        out[2 * k + 1] = __uint_as_float((uint32_t)(w >> 32));
    }
}

template <int K, int BITS, bool OBB = false, typename ParentPtr>
__device__ __forceinline__ void decode_words(const DevModel &M, uint32_t topo, const NodeWords<K, BITS, OBB> &nw,
                                             ParentPtr parent, float out[dec_words(K, OBB)])
{
    if (bits_are_codes((uint32_t)BITS) && topo_abs(topo)) decode_abs<K, BITS, OBB>(M, nw, out);
    else decode_rel<K, BITS, OBB>(nw, parent, out);
}

// The traversal's decode of a child whose parent bounds are at hand: the
// relative decode always runs (so the code words are consumed before any
// branch and their loads travel together with the topology word's), and
// the rare treelet tops then read their absolute bounds.
template <int K, int BITS, bool OBB = false>
__device__ __forceinline__ void decode_child(const DevModel &M, uint32_t topo, const NodeWords<K, BITS, OBB> &nw,
                                             const float *parent, float out[dec_words(K, OBB)])
{
    decode_rel<K, BITS, OBB>(nw, parent, out);
    if (bits_are_codes((uint32_t)BITS) && topo_abs(topo)) decode_abs<K, BITS, OBB>(M, nw, out);
}

template <int K, int BITS, bool OBB = false, typename ParentPtr>
__device__ __forceinline__ void decode_node(const DevModel &M, uint32_t node, ParentPtr parent,
                                            float out[dec_words(K, OBB)])
{
    NodeWords<K, BITS, OBB> nw;
    uint32_t topo;
    load_node<K, BITS, OBB>(M, node, topo, nw);
    decode_words<K, BITS, OBB>(M, topo, nw, parent, out);
}

__device__ __forceinline__ void load_tri(const float *tris, uint32_t i, V3<float> t[3])
{
    const float *p = tris + 9 * (size_t)i;
#pragma unroll
    for (int v = 0; v < 3; v++)
        t[v] = {gload<float>(p + 3 * v), gload<float>(p + 3 * v + 1), gload<float>(p + 3 * v + 2)};
}


// Lower bound on the distance between A's box placed by the pose and B's
// axis-aligned box: their gap along one direction n, from a point of A's
// placed box to the point of B's box nearest to it (one round of alternating
// projections started at A's centre).  For separated boxes this is close to
// their true distance, where gaps along fixed axes can fall short by up to a
// factor sqrt(3).  A's extent along n is its support function through the
// pose's matrix, which holds for any matrix, so the allowance `e` covers FP32
// rounding only.  Inputs: R the matrix (row-major), c A's centre placed by the
// pose, ea A's half extents in its own frame, b B's x, y, z slabs (lo, hi),
// d = c - B's centre, h B's half extents.  Returns -inf when the chosen
// point lies in B's box (the boxes overlap).
__device__ __forceinline__ float dir_gap(const float *R, float4 c, float4 ea, const float *b, float dx, float dy,
                                         float dz, float hx, float hy, float hz, float e)
{
    // B's point nearest to A's centre, as an offset from it, taken into A's
    // frame by the matrix's transpose and clamped to A's box
    const float ox = __builtin_amdgcn_fmed3f(c.x, b[0], b[1]) - c.x;
    const float oy = __builtin_amdgcn_fmed3f(c.y, b[2], b[3]) - c.y;
    const float oz = __builtin_amdgcn_fmed3f(c.z, b[4], b[5]) - c.z;
    const float u0 = __builtin_amdgcn_fmed3f(__builtin_fmaf(R[0], ox, __builtin_fmaf(R[3], oy, R[6] * oz)), -ea.x, ea.x);
    const float u1 = __builtin_amdgcn_fmed3f(__builtin_fmaf(R[1], ox, __builtin_fmaf(R[4], oy, R[7] * oz)), -ea.y, ea.y);
    const float u2 = __builtin_amdgcn_fmed3f(__builtin_fmaf(R[2], ox, __builtin_fmaf(R[5], oy, R[8] * oz)), -ea.z, ea.z);
    // that point of A's placed box, and n towards B's point nearest to it
    const float px = __builtin_fmaf(R[0], u0, __builtin_fmaf(R[1], u1, __builtin_fmaf(R[2], u2, c.x)));
    const float py = __builtin_fmaf(R[3], u0, __builtin_fmaf(R[4], u1, __builtin_fmaf(R[5], u2, c.y)));
    const float pz = __builtin_fmaf(R[6], u0, __builtin_fmaf(R[7], u1, __builtin_fmaf(R[8], u2, c.z)));
    const float nx = __builtin_amdgcn_fmed3f(px, b[0], b[1]) - px;
    const float ny = __builtin_amdgcn_fmed3f(py, b[2], b[3]) - py;
    const float nz = __builtin_amdgcn_fmed3f(pz, b[4], b[5]) - pz;
    // min over B of n.y minus max over placed A of n.x
    const float m0 = __builtin_fmaf(R[0], nx, __builtin_fmaf(R[3], ny, R[6] * nz));
    const float m1 = __builtin_fmaf(R[1], nx, __builtin_fmaf(R[4], ny, R[7] * nz));
    const float m2 = __builtin_fmaf(R[2], nx, __builtin_fmaf(R[5], ny, R[8] * nz));
    const float ext = __builtin_fmaf(
        ea.x, fabsf(m0),
        __builtin_fmaf(ea.y, fabsf(m1),
                       __builtin_fmaf(ea.z, fabsf(m2),
                                      __builtin_fmaf(hx, fabsf(nx), __builtin_fmaf(hy, fabsf(ny), hz * fabsf(nz))))));
    const float gap = -__builtin_fmaf(nx, dx, __builtin_fmaf(ny, dy, nz * dz)) - ext;
    const float nn = __builtin_fmaf(nx, nx, __builtin_fmaf(ny, ny, nz * nz));
    return nn > 0x1p-100f ? gap * __builtin_amdgcn_rsqf(nn) * (1.0f - 0x1p-20f) - e : -INFINITY;
}

// 16-bit reciprocal for n in [1, 8]: (x * r) >> 16 == x / n for x < 64
__device__ __forceinline__ uint32_t recip16(uint32_t n) { return (65536u + n - 1u) / n; }

// An entry popped by a node step, as its tests see it: first A record and
// first B record (relative to the frame), B's child count, first test.
__device__ __forceinline__ uint32_t meta_word(uint32_t aoff, uint32_t boff, uint32_t nb, uint32_t tpre)
{
    return aoff | (boff << 8) | (nb << 16) | (tpre << 24);
}

// A donated work item: a node pair that passed its BV test, with both
// nodes' decoded bounds so that it is self-contained, or a leaf pair.
//   u32 pose, u32 topo A, u32 topo B, f32 lower bound, f32 A[2K], f32 B[2K]
// (OBB models: each node's whole decoded descriptor, 20 words)
__host__ __device__ constexpr uint32_t words_of_item(uint32_t K, bool obb = false) { return 4u + 2u * dec_words(K, obb); }

// Queue accesses between waves on different XCDs go through read-modify-write
// atomics at device scope: they are performed at the device's coherence
// point, where every XCD sees them in one order, whatever its own L2 holds.
__device__ __forceinline__ uint32_t rmw_add(uint32_t *p, uint32_t v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t rmw_read(uint32_t *p) { return rmw_add(p, 0u); }
__device__ __forceinline__ uint32_t rmw_xchg(uint32_t *p, uint32_t v)
{
    return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Polling reads are device-scope atomic loads: coherent like the RMWs but
// served without the per-address serialization of RMWs, which thousands of
// waves polling one word would otherwise queue behind.
__device__ __forceinline__ uint32_t poll(uint32_t *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ __forceinline__ unsigned long long poll64(unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// A device-scope atomic exchange whose old value is not needed: issued in
// the form that returns nothing, so that many of them travel at once (the
// returning form would make each wait for its reply before the next).
__device__ __forceinline__ void rmw_put(uint32_t *p, uint32_t v)
{
    (void)__hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Wait until every vector memory operation this wave issued has completed
// (atomics performed at the coherence point included); the memory clobber
// keeps the compiler from moving memory operations across.
__device__ __forceinline__ void wait_mem() { asm volatile("s_waitcnt vmcnt(0)" : : : "memory"); }


// node steps between two looks at the queue (for waiting waves to feed;
// distance queries look less often, below)
constexpr uint32_t kDonatePeriod = 8;
// steps between refreshes of the shared per-pose answer (hit flag or best distance)
constexpr uint32_t kSyncPeriod = 4;
// distance queries between 18-DOP models with multi-triangle leaves: triangle
// pairs screened per leaf step (by the distance of their boxes) before the
// survivors get the full FP32 test, and how many times the usual number of
// leaf pairs a leaf step waits for
constexpr uint32_t kScreenMax = 256;
constexpr uint32_t kScreenTrigMult = 4;
// most items one balancing donation hands out
constexpr uint32_t kMaxDonate = 32;
// a unit hands work over only while it holds at least this many entries
constexpr uint32_t kDonateMinTop = 2;
// steps after which a collision unit looks at the item queue every other step
constexpr uint32_t kOldSteps = 48;
// pose word of a queue slot that holds no work
constexpr uint32_t kVoidItem = 0xFFFFFFFFu;

// ---------------------------------------------------------------------------
// The traversal kernel: persistent waves.  Each wave takes poses from a queue
// and traverses one pose at a time (a work unit).  Once the pose queue is
// empty a wave takes the next slot of the item queue and waits for it to be
// filled; busy waves look at the queue every few node steps and, while
// slots wait, hand the bottom entries of their stack (the pairs nearest the
// roots, i.e. the largest pending subtrees) to the waiting slots as items.
// A unit whose next node step does not fit its LDS state hands over all of
// its pending pairs and ends.  `pending` counts the poses and published items
// not finished yet: it reaches zero exactly when no work is left, which
// is when waiting waves exit.  Per-pose answers (hit flag, best distances)
// are merged in device memory, so results do not depend on the split.
// ---------------------------------------------------------------------------
// Collision modes and distance queries of AABB models fit 3 waves per SIMD
// (168 VGPRs); distance queries of 18-DOP or OBB models need more.  OBB
// selects oriented boxes (K == 3 slabs in per-node frames).
template <int K, int BITS, int MODE, bool OBB>
__global__ __launch_bounds__(kMaxWavesPerGroup * WAVE)
__attribute__((amdgpu_waves_per_eu((MODE == MODE_DIST && (K == 9 || OBB)) ? 2 : 3)))
void traverse_kernel(QueryArgs q, StackLimits lim)
{
    static_assert(!OBB || (K == 3 && BITS != (int)kBitsFp16), "OBB models: 3 slabs, bits 0, 8 or 16");
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const uint32_t lane = __lane_id();
    const Layout LY = make_layout(K, MODE, lim, OBB);
    // a workgroup holds one or more independent waves (the launch's
    // workgroup shape); each has its own slice of LDS
    const uint32_t wave_in_group = uni(threadIdx.x / WAVE), waves_per_group = blockDim.x / WAVE;
    const uint32_t wave_id = blockIdx.x * waves_per_group + wave_in_group;
    const uint32_t n_waves = gridDim.x * waves_per_group;
    unsigned char *base = lds_raw + (size_t)wave_in_group * LY.total;
    constexpr uint32_t RW = rec_words(K, OBB);  // floats per record
    constexpr uint32_t RV = RW / 4;             // float4 per record
    constexpr uint32_t DW = dec_words(K, OBB);  // decoded words per node
    constexpr uint32_t TW = rec_words(K);       // floats per transformed A record
    constexpr bool kTopoEnt = topo_in_entry(MODE);
    float4 *xf = (float4 *)(base + LY.xf);
    // the current pose and its error allowances, kept in LDS (read where
    // needed, so that they hold no scalar registers across the traversal):
    // rows (R_i0, R_i1, R_i2, t_i), then (e_abs, e_sph, e_dir, rot_eps), then
    // the OBB test's allowances (e_obb, e_obbA, delta_C, eta_R)
    float4 *pz = (float4 *)(base + LY.pz);
    auto pose_of = [&]() -> Pose {
        Pose P;
#pragma unroll
        for (int i = 0; i < 3; i++) {
            const float4 r = pz[i];
            P.R[3 * i] = r.x, P.R[3 * i + 1] = r.y, P.R[3 * i + 2] = r.z, P.t[i] = r.w;
        }
        return P;
    };
    float *rec = (float *)(base + LY.rec);
    float *ta = (float *)(base + LY.ta);
    uint32_t *ta_topo = (uint32_t *)(base + LY.ta_topo);
    float4 *tsph = (float4 *)(base + LY.tsph);
    uint32_t *ent = (uint32_t *)(base + LY.ent);      // recA | recB << 13 | frame level << 26
    uint2 *ent_tp = (uint2 *)(base + LY.ent_tp);      // collision queries: both nodes' topology words
    float *ent_lb = (float *)(base + LY.ent_lb);
    uint2 *lq = (uint2 *)(base + LY.lq);
    float *lq_lb = (float *)(base + LY.lq_lb);
    uint32_t *lscan = (uint32_t *)(base + LY.lscan);  // leaf step: prefix sums of the taken leaf pairs
    auto rec_topo_ref = [&](uint32_t r) -> uint32_t & { return ((uint32_t *)rec)[(size_t)r * RW + 2 * K]; };

    constexpr uint32_t IW = words_of_item(K, OBB);  // dwords per item
    constexpr uint32_t CPL = (uint32_t)WAVE / (uint32_t)K;  // records per transform pass
    constexpr uint32_t IPI = (uint32_t)WAVE / IW;   // items written per wave instruction
    const DevModel &MA = q.A;
    DevModel MB = q.B;  // the fixed model of the current unit (per pose in batched queries)
    WsHeader *hdr = q.ws.hdr;
    // this wave's statistics counters (C_* rows), kept in LDS so that they
    // hold no registers; lane 0 updates them with LDS atomics
    unsigned long long *ctr = (unsigned long long *)(base + LY.ctr);
    if (lane < (uint32_t)C_NUM) ctr[lane] = (lane == C_T_START || lane == C_T_DRAIN) ? ~0ull : 0ull;
    auto ctr_add = [&](int c, unsigned long long v) {
        __hip_atomic_fetch_add(&ctr[c], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    auto ctr_max = [&](int c, unsigned long long v) {
        __hip_atomic_fetch_max(&ctr[c], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    };
    uint32_t lq_trigger_full = (uint32_t)(WAVE / (MA.leaf_size * MB.leaf_size));
    const uint32_t code_bytes_A = 4 + MA.stride;
    uint32_t code_bytes_B = 4 + MB.stride;
    const bool can_donate = !q.no_split;

    // the two topology words of entry i
    auto entry_topo = [&](uint32_t i, uint32_t e) -> uint2 {
        if constexpr (kTopoEnt) return ent_tp[i];
        else return make_uint2(rec_topo_ref(e & REC_MASK), rec_topo_ref((e >> REC_BITS) & REC_MASK));
    };

    // Publish items: reserve n slots of the item queue, fill them from
    // entries [0, n_ent) and leaf pairs [0, n - n_ent), then mark them
    // ready.  Returns the number of items published (n, or 0 if the queue
    // is full; the slots reserved below its end are then published void).
    auto publish = [&](uint32_t pose, uint32_t n, uint32_t n_ent, float best) -> uint32_t {
        uint32_t first = 0, ok = 0, left = 0;
        // once helpers have begun to leave, a claimed slot may have nobody
        // behind it: publish nothing (this unit's own count in `pending`
        // keeps any helper from leaving while it publishes)
        if (lane == 0) left = rmw_read(&hdr->gone);
        if (uni(left)) return 0u;
        if (lane == 0) {
            first = rmw_add(&hdr->q_tail, n);
            ok = first + n <= q.ws.item_cap && first + n >= first;
            if (ok) {
                (void)rmw_add(&hdr->pending, n);
                if (MODE == MODE_DIST && best < INFINITY)
                    (void)__hip_atomic_fetch_min(&q.ws.best32[pose], __float_as_uint(best), __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            }
        }
        ok = uni(ok);
        first = uni(first);
        if (!ok) {
            for (uint32_t i = lane; i < n && first + i < q.ws.item_cap; i += WAVE)
                rmw_put(&q.ws.items[(size_t)(first + i) * IW], kVoidItem);
        } else {
            for (uint32_t i0 = 0; i0 < n; i0 += IPI) {
                const uint32_t i = i0 + lane / IW, w = lane % IW;
                if (lane < IPI * IW && i < n) {
                    uint32_t val = 0;
                    bool write = true;
                    if (i < n_ent) {
                        const uint32_t ee = ent[i];
                        const uint32_t rA = ee & REC_MASK, rB = (ee >> REC_BITS) & REC_MASK;
                        if (w == 0) val = pose;
                        else if (w == 1) val = entry_topo(i, ee).x;
                        else if (w == 2) val = entry_topo(i, ee).y;
                        else if (w == 3) val = MODE == MODE_DIST ? __float_as_uint(ent_lb[i]) : 0u;
                        else if (w < 4 + DW) val = __float_as_uint(rec[(size_t)rA * RW + (w - 4)]);
                        else val = __float_as_uint(rec[(size_t)rB * RW + (w - 4 - DW)]);
                    } else {
                        const uint32_t j = i - n_ent;
                        const uint2 le = lq[j];
                        if (w == 0) val = pose;
                        else if (w == 1) val = le.x;
                        else if (w == 2) val = le.y;
                        else if (w == 3) val = MODE == MODE_DIST ? __float_as_uint(lq_lb[j]) : 0u;
                        else write = false;  // a leaf pair needs no bounds
                    }
                    if (write) rmw_put(&q.ws.items[(size_t)(first + i) * IW + w], val);
                }
            }
        }
        // every payload word and the pending count are in place before any
        // ready flag is set
        wait_mem();
        for (uint32_t i = lane; i < n && first + i < q.ws.item_cap; i += WAVE) rmw_put(&q.ws.ready[first + i], 1u);
        return ok ? n : 0u;
    };

    // An A record of the current frame (index c within it, lane holding its
    // bounds and topology word) prepared for the child-pair tests: its
    // topology word beside the transformed records, and for AABB models or
    // distance queries its circumscribed sphere (centre placed by the pose)
    // and half extents in its own frame.
    auto prep_A = [&](uint32_t c, const float *b, uint32_t topo) {
        ta_topo[c] = topo;
        if constexpr (OBB) {
            // the box placed by the pose, in generator form
            float pl[20];
            obb_place(pose_of(), b, pz[4].w, pl);
            float4 *d = tsph + 5 * c;
#pragma unroll
            for (int v = 0; v < 5; v++) d[v] = make_float4(pl[4 * v], pl[4 * v + 1], pl[4 * v + 2], pl[4 * v + 3]);
        } else if constexpr (MODE == MODE_DIST || K == 3) {
            const Pose P = pose_of();
            const float rot_eps = pz[3].w;
            V3<float> cc = {0.5f * (b[0] + b[1]), 0.5f * (b[2] + b[3]), 0.5f * (b[4] + b[5])};
            float hx = 0.5f * (b[1] - b[0]), hy = 0.5f * (b[3] - b[2]), hz = 0.5f * (b[5] - b[4]);
            // the map stretches lengths by at most 1 + 1.5 rot_eps
            float r = bound_sqrt(hx * hx + hy * hy + hz * hz) * (1.0f + 0x1p-20f + 2.0f * rot_eps);
            V3<float> cw = xform_f32(P, cc);
            tsph[2 * c] = make_float4(cw.x, cw.y, cw.z, r);
            tsph[2 * c + 1] = make_float4(hx, hy, hz, hx + hy + hz);  // A-frame half extents
        }
    };
    auto store_rec = [&](uint32_t r, const float *b, uint32_t topo) {
        float t[RW];
#pragma unroll
        for (uint32_t k = 0; k < DW; k++) t[k] = b[k];
        t[2 * K] = __uint_as_float(topo);
        if constexpr (!OBB) t[2 * K + 1] = 0.0f;
        float4 *dst = (float4 *)(rec + (size_t)r * RW);
#pragma unroll
        for (uint32_t v = 0; v < RV; v++) dst[v] = make_float4(t[4 * v], t[4 * v + 1], t[4 * v + 2], t[4 * v + 3]);
    };
    auto load_rec = [&](uint32_t r, float *b) {
        const float4 *src = (const float4 *)(rec + (size_t)r * RW);
#pragma unroll
        for (uint32_t v = 0; v < RV; v++) {
            const float4 x = src[v];
            b[4 * v] = x.x;
            b[4 * v + 1] = x.y;
            b[4 * v + 2] = x.z;
            b[4 * v + 3] = x.w;
        }
    };

    bool poses_left = true, first_claim = true;
    // A wave with a pose to run counts as work that may still publish items
    // until it finds the pose queue empty; a wave that starts late, after
    // helpers left, therefore never waits on them and never hands work to
    // them.  (The count is not waited for here: the wave's first memory
    // waits complete it long before it could publish.)  A wave whose block
    // index is past the poses gets none from the queue either: it holds no
    // count and goes straight to helping or exits.
    const bool counted = can_donate && wave_id < q.n_poses;
    if (counted && lane == 0) rmw_add(&hdr->pending, 1u);
    uint32_t cur_pose = 0xFFFFFFFFu;
    // this lane's slab (lane mod K) of the pose's support-function transform,
    // kept in registers for the whole pose
    const uint32_t my_k = lane % (uint32_t)K;
    float4 xf0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float xfU = 0.0f, xfL = 0.0f;
    const float w_diag = 0.70710676f;  // <= 1/sqrt(2): unit-length correction of diagonal slabs

    for (;;) {
        // ---- next work unit: a pose, or once they are gone a donated item ----
        uint32_t pose = 0;
        bool from_item = false;
        uint32_t it_tA = 0, it_tB = 0;
        float it_lb = 0.0f;
        if (poses_left) {
            // a wave's first pose is its block index; later ones come from
            // the queue (no burst of atomics on one line at the start)
            uint32_t p = wave_id;
            if (lane == 0) {
                if (first_claim) ctr[C_T_START] = wall_clock64();
                else p = n_waves + atomicAdd(&hdr->pose_next, 1u);
            }
            first_claim = false;
            // (queue claims start at the grid size, past any block index)
            pose = uni(p);
            if (pose >= q.n_poses) {
                poses_left = false;
                if (lane == 0) ctr[C_T_DRAIN] = wall_clock64();
                // this wave starts no more poses: it no longer counts as work
                // that could still publish items
                if (counted && lane == 0) rmw_add(&hdr->pending, 0xFFFFFFFFu);
            }
        }
        if (!poses_left) {
            if (!can_donate) break;
            // the waves of the workgroups with the lowest indices (spread
            // over the XCDs and CUs by the dispatcher) stay as helpers, all
            // waves of a workgroup together: a workgroup's LDS is held
            // until its last wave exits, so a lone helper wave would pin
            // its partners' LDS too; the others exit
            if (wave_id >= q.max_helpers) break;
            uint32_t slot = 0;
            if (lane == 0) slot = rmw_add(&hdr->q_head, 1u);
            slot = uni(slot);
            // wait until the slot is filled or no work is left anywhere,
            // backing off so that thousands of waiting waves leave the
            // memory system to the busy ones
            const unsigned long long t0 = wall_clock64();
            uint32_t got = 0;
            for (uint32_t spin = 0;; spin++) {
                uint32_t r = 0, pend = 1;
                if (lane == 0) {
                    if (slot < q.ws.item_cap) r = poll(&q.ws.ready[slot]);
                    if (!r && (spin & 7) == 7) pend = poll(&hdr->pending);
                }
                if (uni(r)) {
                    got = 1;
                    break;
                }
                if (uni(pend) == 0) {
                    // nothing runs: stop all hand-over for good, then leave
                    // unless some wave started meanwhile
                    uint32_t again = 0;
                    if (lane == 0) {
                        rmw_xchg(&hdr->gone, 1u);
                        again = rmw_read(&hdr->pending);
                    }
                    if (uni(again) == 0) break;
                }
                if (wall_clock64() - t0 > q.wait_limit) {
                    if (lane == 0) {
                        rmw_xchg(&hdr->error, 1u);
                        rmw_xchg(&hdr->gone, 1u);
                    }
                    break;
                }
                if (spin < 4) __builtin_amdgcn_s_sleep(8);
                else if (spin < 16) __builtin_amdgcn_s_sleep(32);
                else __builtin_amdgcn_s_sleep(96);
            }
            if (!got) break;
            uint32_t v = 0;
            if (lane < IW) v = rmw_read(&q.ws.items[(size_t)slot * IW + lane]);
            pose = lane_of(v, 0);
            if (pose == kVoidItem) continue;  // a slot of a donation that found the queue full
            it_tA = lane_of(v, 1);
            it_tB = lane_of(v, 2);
            it_lb = __uint_as_float(lane_of(v, 3));
            // records 0 and 1 hold the item's two decoded BVs
            if (lane >= 4 && lane < 4 + DW) rec[lane - 4] = __uint_as_float(v);
            if (lane >= 4 + DW && lane < IW) rec[RW + (lane - 4 - DW)] = __uint_as_float(v);
            from_item = true;
            if (MODE == MODE_BOOL) {
                uint32_t decided = 0;
                if (lane == 0) decided = poll(&q.ws.hitw[pose]);
                if (uni(decided)) {  // another unit of this pose already found a collision
                    if (lane == 0) rmw_add(&hdr->pending, 0xFFFFFFFFu);
                    continue;
                }
            }
        }
        if (pose != cur_pose) {
            if (q.pose_obj) {
                // batched query: this pose's fixed model
                const uint32_t obj = uni(q.pose_obj[pose]);
                if (obj >= q.n_obj) {
                    if (lane == 0) q.status[pose] = 4;  // CBVH_POSE_BAD_OBSTACLE
                    continue;
                }
                MB = q.Btab[obj];
                lq_trigger_full = (uint32_t)(WAVE / (MA.leaf_size * MB.leaf_size));
                code_bytes_B = 4 + MB.stride;
            }
            cur_pose = pose;
            {
                Pose P;
#pragma unroll
                for (int i = 0; i < 3; i++) {
#pragma unroll
                    for (int j = 0; j < 3; j++) P.R[3 * i + j] = q.poses[12 * (size_t)pose + 4 * i + j];
                    P.t[i] = q.poses[12 * (size_t)pose + 4 * i + 3];
                }
                if constexpr (!OBB) pose_setup<K>(&q.poses[12 * (size_t)pose], MA.max_abs, xf, lane);
                // distance: FP32 leaf-distance error bound, and the absolute
                // rounding allowance of the sphere bound
                const float e_abs = dist_err_abs(&q.poses[12 * (size_t)pose], MA.max_abs, MB.max_abs);
                const float e_sph = 64.0f * 0x1p-24f *
                                    (fabsf(P.t[0]) + fabsf(P.t[1]) + fabsf(P.t[2]) + 4.0f * (MA.max_abs + MB.max_abs));
                float rot_eps;
                {
                    // how far the rotation's columns are from orthonormal (their
                    // Gram matrix minus the identity, largest entry, in FP64):
                    // the gaps along A's axes below allow for it
                    double dev = 0.0;
#pragma unroll
                    for (int i = 0; i < 3; i++) {
#pragma unroll
                        for (int j = i; j < 3; j++) {
                            double g = 0.0;
#pragma unroll
                            for (int k = 0; k < 3; k++) g += (double)P.R[3 * k + i] * (double)P.R[3 * k + j];
                            dev = fmax(dev, fabs(g - (i == j ? 1.0 : 0.0)));
                        }
                    }
                    rot_eps = __double2float_ru(dev) + 0x1p-22f;
                }
                // rounding allowance of the directional gap below: the sphere
                // bound's, grown with the matrix's largest stretch
                const float e_dir = __builtin_fmaf(2.0f * rot_eps, e_sph, e_sph);
                if (lane == 0) {
#pragma unroll
                    for (int i = 0; i < 3; i++) pz[i] = make_float4(P.R[3 * i], P.R[3 * i + 1], P.R[3 * i + 2], P.t[i]);
                    pz[3] = make_float4(e_abs, e_sph, e_dir, rot_eps);
                    if constexpr (OBB) {
                        float al[4];
                        obb_allowances(&q.poses[12 * (size_t)pose], rot_eps, MA.max_abs, MB.max_abs, al);
                        pz[4] = make_float4(al[0], al[1], al[2], al[3]);
                    }
                }
            }
            wave_sync();
            // this lane's slab of the support-function transform
            const float4 x0 = xf[2 * my_k], x1 = xf[2 * my_k + 1];
            xf0 = x0;
            xfU = x1.x;
            xfL = x1.y;
        }

        // ---- initial state ----
        // current frame: the records decoded by the last node step, waiting
        // for their child-pair tests (f_ns entries, described in f_meta)
        uint32_t f_base = 0, f_nA = 1, f_ns = 1, f_tasks = 1, f_level = 0;
        uint32_t f_meta = meta_word(0, 1, 1, 0);  // lane s: entry s of the frame
        // lane l: end of the frame of level l (frames are stacked in record space)
        uint32_t fe_v = lane == 0 ? 2u : 0u;
        bool have_frame;
        uint32_t top = 0, lq_count = 0;
        bool hit = false, overflow = false, pair_overflow = false, fix_overflow = false;
        // shared: other units of this pose may exist, so the per-pose answer
        // in device memory is read and merged while traversing
        bool shared = from_item;
        float best32 = INFINITY;
        double best64 = INFINITY;
        uint32_t next_look = kDonatePeriod, next_sync = kSyncPeriod;
        // this unit's node-step statistics, added to the wave's counters when it ends
        uint32_t st_tests = 0, st_exp = 0, st_steps = 0, st_max_ent = 0, st_max_rec = 0;
        unsigned long long st_bytes = 0;
        if (!from_item) {
            // root frame: record 0 = A's root, record 1 = B's root; the root pair is tested first
            if (lane < 2) {
                const DevModel &M = lane == 0 ? MA : MB;
                NodeWords<K, BITS, OBB> nw;
                uint32_t tw;
                load_node<K, BITS, OBB>(M, 0, tw, nw);
                float bnd[DW];
                decode_words<K, BITS, OBB>(M, tw, nw, (const float *)nullptr, bnd);
                store_rec(lane, bnd, tw);
                if (lane == 0) prep_A(0, bnd, tw);
            }
            have_frame = true;
        } else {
            // the item's pair already passed its BV test: records 0 and 1 hold it
            if (lane == 0) {
                rec_topo_ref(0) = it_tA;
                rec_topo_ref(1) = it_tB;
            }
            if (topo_leaf(it_tA) && topo_leaf(it_tB)) {
                if (lane == 0) {
                    lq[0] = make_uint2(it_tA, it_tB);
                    if (MODE == MODE_DIST) lq_lb[0] = it_lb;
                }
                lq_count = 1;
            } else {
                if (lane == 0) {
                    ent[0] = 0u | (1u << REC_BITS);
                    if constexpr (kTopoEnt) ent_tp[0] = make_uint2(it_tA, it_tB);
                    if (MODE == MODE_DIST) ent_lb[0] = it_lb;
                }
                top = 1;
            }
            if (MODE == MODE_DIST) {
                uint32_t g = 0;
                if (lane == 0) g = poll(&q.ws.best32[pose]);
                best32 = __uint_as_float(uni(g));
            }
            have_frame = false;
        }
        wave_sync();

        uint32_t steps = 0;
        for (;;) {
            steps++;
            // long units are the critical path of the batch: they get issue
            // priority over the short ones sharing their SIMD
            if (q.prio_steps && steps % q.prio_steps == 0) {
                const uint32_t lvl = steps / q.prio_steps;
                if (lvl == 1) __builtin_amdgcn_s_setprio(1);
                else if (lvl == 2) __builtin_amdgcn_s_setprio(2);
                else if (lvl == 3) __builtin_amdgcn_s_setprio(3);
            }
            if (have_frame) {
                have_frame = false;
                // -------- transform A's records of the frame into B's frame --------
                // lane = (record c, slab my_k), CPL records per pass; each
                // generator reads its slab's (lo, hi) pair at once (distance
                // tests of AABB models read only the spheres prepared at decode)
                if constexpr ((MODE != MODE_DIST || K != 3) && !OBB) {
                    const uint32_t up = __float_as_uint(xf0.w);
                    const uint32_t a0 = (up & 0xFFu) >> 1, a1 = ((up >> 8) & 0xFFu) >> 1, a2 = ((up >> 16) & 0xFFu) >> 1;
                    const bool h0 = (up & 1u) != 0, h1 = (up & 0x100u) != 0, h2 = (up & 0x10000u) != 0;
                    const uint32_t my_c = lane / (uint32_t)K;
                    for (uint32_t c0 = 0; c0 < f_nA; c0 += CPL) {
                        const uint32_t ca = c0 + my_c;
                        if (lane < CPL * (uint32_t)K && ca < f_nA) {
                            const float2 *b = (const float2 *)(rec + (size_t)(f_base + ca) * RW);
                            const float2 p0 = b[a0], p1 = b[a1], p2 = b[a2];
                            // U takes each generator's hi for + signs (lo for -), L the other bound
                            const float U = __builtin_fmaf(xf0.z, h2 ? p2.y : p2.x,
                                                           __builtin_fmaf(xf0.y, h1 ? p1.y : p1.x, __builtin_fmaf(xf0.x, h0 ? p0.y : p0.x, xfU)));
                            const float L = __builtin_fmaf(xf0.z, h2 ? p2.x : p2.y,
                                                           __builtin_fmaf(xf0.y, h1 ? p1.x : p1.y, __builtin_fmaf(xf0.x, h0 ? p0.x : p0.y, xfL)));
                            *(float2 *)(ta + (size_t)ca * TW + 2 * my_k) = make_float2(L, U);
                        }
                    }
                    wave_sync();
                }
                // -------- child-pair tests, one per lane --------
                const float tau = MODE == MODE_DIST ? add_up(best32, pz[3].x) : 0.0f;
                bool survive = false;
                float lb = 0.0f;
                uint32_t recA = 0, recB = 0, tA_w = 0, tB_w = 0;
                if (lane < f_tasks) {
                    // the task's entry: the last one whose first task is <= lane
                    // (culled entries of distance queries have no tasks and are
                    // passed over)
                    uint32_t w = lane_of(f_meta, 0);
                    if (f_ns > 1) {
#pragma unroll
                        for (int s = 1; s < PMAX; s++) {
                            if ((uint32_t)s < f_ns) {
                                const uint32_t ws = lane_of(f_meta, s);
                                if ((ws >> 24) <= lane) w = ws;
                            }
                        }
                    }
                    const uint32_t aoff = w & 0xFFu, boff = (w >> 8) & 0xFFu, nb = (w >> 16) & 0xFFu;
                    const uint32_t local = lane - (w >> 24);
                    // local / nb (local < 64, nb <= 8): the half offset keeps the
                    // product away from integers, so one rounding cannot move it
                    const uint32_t i = (uint32_t)(((float)local + 0.5f) * __builtin_amdgcn_rcpf((float)nb));
                    const uint32_t j = local - i * nb;
                    const uint32_t ia = aoff + i;
                    recA = f_base + ia;
                    recB = f_base + boff + j;
                    tA_w = ta_topo[ia];
                    float bB[RW];
                    load_rec(recB, bB);
                    tB_w = __float_as_uint(bB[2 * K]);
                    if constexpr (OBB) {
                        float pa[20], sep;
#pragma unroll
                        for (int v = 0; v < 5; v++) {
                            const float4 x = tsph[5 * ia + v];
                            pa[4 * v] = x.x, pa[4 * v + 1] = x.y, pa[4 * v + 2] = x.z, pa[4 * v + 3] = x.w;
                        }
                        const float4 a4 = pz[4];
                        const float al[4] = {a4.x, a4.y, a4.z, a4.w};
                        obb_gap<MODE == MODE_DIST>(pa, bB, al, &sep, &lb);
                        if constexpr (MODE == MODE_DIST) {
                            survive = lb <= tau;
                        } else {
                            lb = sep;
                            survive = !(sep > 0.0f);
                        }
                    } else if constexpr (MODE == MODE_DIST) {
                        // A lower bound on the distance of the two BVs (the largest of
                        // the ones below); where the boxes overlap it is negative, and
                        // then its value orders the traversal: the most deeply
                        // overlapping pair goes first, which reaches close triangle
                        // pairs (or an intersection, distance 0, which ends the pose)
                        // sooner than taking overlapping pairs in lane order.
                        // First: gaps of the 18-DOP slabs (AABB models skip them: beside
                        // the directional gap below they pruned no more and cost time)
                        float g = -INFINITY;
                        if constexpr (K != 3) {
                            float tA[RW];
                            {
                                const float4 *src = (const float4 *)(ta + (size_t)ia * TW);
#pragma unroll
                                for (uint32_t v = 0; v < RV; v++) {
                                    const float4 x = src[v];
                                    tA[4 * v] = x.x, tA[4 * v + 1] = x.y, tA[4 * v + 2] = x.z, tA[4 * v + 3] = x.w;
                                }
                            }
#pragma unroll
                            for (int k = 0; k < K; k++) {
                                float gk = fmaxf(tA[2 * k] - bB[2 * k + 1], bB[2 * k] - tA[2 * k + 1]);
                                gk *= (k < 3 ? 1.0f : w_diag);
                                g = fmaxf(g, gk);
                            }
                        }
                        // second lower bound: distance of the circumscribed spheres
                        const float4 sa = tsph[2 * ia];
                        const float cx = 0.5f * (bB[0] + bB[1]), cy = 0.5f * (bB[2] + bB[3]), cz = 0.5f * (bB[4] + bB[5]);
                        const float hx = 0.5f * (bB[1] - bB[0]), hy = 0.5f * (bB[3] - bB[2]), hz = 0.5f * (bB[5] - bB[4]);
                        const float rb = bound_sqrt(hx * hx + hy * hy + hz * hz) * (1.0f + 0x1p-20f);
                        const float dx = sa.x - cx, dy = sa.y - cy, dz = sa.z - cz;
                        const float4 ez = pz[3];
                        const float gs = bound_sqrt(dx * dx + dy * dy + dz * dz) * (1.0f - 0x1p-20f) - sa.w - rb - ez.y;
                        // third lower bound: the gap along one well-chosen direction
                        // (gaps along A's own axes, tried beside it, pruned no more)
                        const Pose P = pose_of();
                        const float gd = dir_gap(P.R, sa, tsph[2 * ia + 1], bB, dx, dy, dz, hx, hy, hz, ez.z);
                        lb = fmaxf(fmaxf(g * (1.0f - 0x1p-20f), gs), gd);  // g is -inf for AABB models
                        survive = lb <= tau;
                    } else {
                        // the largest gap between A's moved slab interval and B's:
                        // positive separates; otherwise its value (minus the
                        // translation that separates the pair along its best
                        // slab) orders the traversal, the deepest overlap first
                        float tA[RW];
                        {
                            const float4 *src = (const float4 *)(ta + (size_t)ia * TW);
#pragma unroll
                            for (uint32_t v = 0; v < RV; v++) {
                                const float4 x = src[v];
                                tA[4 * v] = x.x, tA[4 * v + 1] = x.y, tA[4 * v + 2] = x.z, tA[4 * v + 3] = x.w;
                            }
                        }
                        float g = -INFINITY;
#pragma unroll
                        for (int k = 0; k < K; k++)
                            g = fmaxf(g, fmaxf(tA[2 * k] - bB[2 * k + 1], bB[2 * k] - tA[2 * k + 1]));
                        bool sep = g > 0.0f;
                        if constexpr (K == 3) {
                            // separating axes along A's own axes (the rotation's
                            // columns): A's record as a box in its frame, B's as an
                            // axis-aligned box; separated only beyond the allowances
                            // for non-orthonormal columns and FP32 rounding (AABB
                            // models only: an 18-DOP's diagonal slabs already cut
                            // what these axes would, and the test costs more than
                            // it saves there)
                            const float4 sa = tsph[2 * ia], ea = tsph[2 * ia + 1];
                            const float dx = 0.5f * (bB[0] + bB[1]) - sa.x, dy = 0.5f * (bB[2] + bB[3]) - sa.y,
                                        dz = 0.5f * (bB[4] + bB[5]) - sa.z;
                            const float hx = 0.5f * (bB[1] - bB[0]), hy = 0.5f * (bB[3] - bB[2]),
                                        hz = 0.5f * (bB[5] - bB[4]);
                            const Pose P = pose_of();
                            const float4 ez = pz[3];
                            float ga = -INFINITY;
#pragma unroll
                            for (int a = 0; a < 3; a++) {
                                const float c0 = P.R[a], c1 = P.R[3 + a], c2 = P.R[6 + a];
                                const float p = __builtin_fmaf(c0, dx, __builtin_fmaf(c1, dy, c2 * dz));
                                const float rbi =
                                    __builtin_fmaf(fabsf(c0), hx, __builtin_fmaf(fabsf(c1), hy, fabsf(c2) * hz));
                                ga = fmaxf(ga, fabsf(p) - (a == 0 ? ea.x : a == 1 ? ea.y : ea.z) - rbi);
                            }
                            ga = __builtin_fmaf(-ez.w, ea.w, ga) * (1.0f - 0x1p-20f - ez.w) - ez.y;
                            sep |= ga > 0.0f;
                        }
                        survive = !sep;
                        lb = g;
                    }
                }
                // -------- compaction: leaf pairs -> leaf queue, others -> entries --------
                const bool ll = topo_leaf(tA_w) && topo_leaf(tB_w);
                const bool nd = survive && !ll;
                const uint64_t m_ll = __ballot(survive && ll), m_nd = __ballot(nd);
                const uint32_t n_ll = __popcll(m_ll), n_nd = __popcll(m_nd);
                if (survive && ll) {
                    const uint32_t slot = lq_count + mbcnt(m_ll);
                    lq[slot] = make_uint2(tA_w, tB_w);
                    if (MODE == MODE_DIST) lq_lb[slot] = lb;
                }
                // the most promising new node pair, the closest (distance) or
                // the most deeply overlapping (collision), goes on top of the
                // stack: it is expanded next
                uint64_t win = 0;
                if ((MODE == MODE_DIST || MODE == MODE_BOOL) && n_nd > 1) {
                    const float mlb = wave_min(nd ? lb : INFINITY);
                    const uint64_t cand = __ballot(nd && lb == mlb);
                    win = cand & (~cand + 1ull);
                }
                const uint32_t my_packed = recA | (recB << REC_BITS) | (f_level << (2 * REC_BITS));
                if (nd) {
                    const uint32_t slot =
                        ((win >> lane) & 1ull) ? top + n_nd - 1u : top + mbcnt(m_nd & ~win);
                    ent[slot] = my_packed;
                    if constexpr (kTopoEnt) ent_tp[slot] = make_uint2(tA_w, tB_w);
                    if (MODE == MODE_DIST) ent_lb[slot] = lb;
                }
                lq_count += n_ll;
                top += n_nd;
                st_tests += f_tasks;
                st_max_ent = max(st_max_ent, top);
                wave_sync();
            }
            if (MODE == MODE_BOOL && hit) break;
            if (MODE == MODE_DIST && best64 == 0.0) break;

            // -------- shared answer of the pose: stop or tighten --------
            if (shared && steps >= next_sync) {
                next_sync = steps + kSyncPeriod;
                if (MODE == MODE_BOOL) {
                    uint32_t d = 0;
                    if (lane == 0) d = poll(&q.ws.hitw[pose]);
                    if (uni(d)) break;
                } else if (MODE == MODE_DIST) {
                    uint32_t g = 0;
                    if (lane == 0) g = poll(&q.ws.best32[pose]);
                    best32 = fminf(best32, __uint_as_float(uni(g)));
                }
            }

            // -------- leaf step --------
            // distance queries whose leaves hold several triangles each screen
            // the triangle pairs first (18-DOP models: the screening buffer
            // shares LDS with the transformed records, which are dead here)
            constexpr bool kScreens = MODE == MODE_DIST && K == 9;
            const bool screen = kScreens && lq_trigger_full < (uint32_t)WAVE;
            uint32_t trig = lq_trigger_full < 1 ? 1 : lq_trigger_full;
            if (screen) trig = min(trig * kScreenTrigMult, lim.leafq / 2u);
            if (MODE == MODE_DIST && best32 == INFINITY) trig = 1;
            if (lq_count > 0 && (lq_count >= trig || top == 0)) {
                const Pose P = pose_of();
                const float e_abs = pz[3].x;
                const float tau = MODE == MODE_DIST ? add_up(best32, e_abs) : 0.0f;
                uint32_t n_avail = min(lq_count, (uint32_t)WAVE);
                uint32_t tasks = 0;
                uint2 e = make_uint2(0, 0);
                if (lane < n_avail) {
                    uint32_t slot = lq_count - 1 - lane;
                    e = lq[slot];
                    tasks = topo_count(e.x) * topo_count(e.y);
                    if (MODE == MODE_DIST && lq_lb[slot] > tau) tasks = 0;
                }
                uint32_t incl = wave_incl_scan(tasks, lane);
                uint64_t m_take = __ballot(lane < n_avail && incl <= (screen ? kScreenMax : (uint32_t)WAVE));
                uint32_t n_take = __popcll(m_take);
                uint32_t total = n_take ? lane_of(incl, (int)n_take - 1) : 0u;
                if (lane < n_take) lscan[lane] = incl;
                wave_sync();
                const uint32_t lq_old = lq_count;
                lq_count -= n_take;
                // triangle pair number t of the taken leaf pairs
                auto pair_of = [&](uint32_t t, uint32_t &tA, uint32_t &tB) {
                    // its leaf pair: the first taken entry with incl > t
                    uint32_t lo = 0, hi = n_take - 1;
                    while (lo < hi) {
                        uint32_t mid = (lo + hi) >> 1;
                        if (lscan[mid] > t) hi = mid; else lo = mid + 1;
                    }
                    uint32_t excl = lo ? lscan[lo - 1] : 0u;
                    uint2 le = lq[lq_old - 1 - lo];
                    uint32_t local = t - excl, nb = topo_count(le.y);
                    uint32_t ia = (local * recip16(nb)) >> 16, ib = local - ia * nb;
                    tA = topo_first(le.x) + ia;
                    tB = topo_first(le.y) + ib;
                };
                uint32_t n_full = total;
                uint2 *tq = (uint2 *)ta;
                static_assert(8 * 9 * TA_MAX >= 8 * (int)kScreenMax, "the screening buffer fits the transformed records");
                if (screen) {
                    // screening: a pair whose boxes (A's triangle placed by the
                    // pose, in FP32) are farther apart than the bound cannot be
                    // the closest one; e_abs covers the FP32 placement
                    n_full = 0;
                    for (uint32_t c0 = 0; c0 < total; c0 += WAVE) {
                        const uint32_t t = c0 + lane;
                        bool keep = false;
                        uint32_t tA = 0, tB = 0;
                        if (t < total) {
                            pair_of(t, tA, tB);
                            V3<float> a0[3], bb[3];
                            load_tri(MA.tris, tA, a0);
                            load_tri(MB.tris, tB, bb);
                            float g2 = 0.0f;
                            {
                                const V3<float> p0 = xform_f32(P, a0[0]), p1 = xform_f32(P, a0[1]), p2 = xform_f32(P, a0[2]);
                                const float ga = fmaxf(fminf(fminf(p0.x, p1.x), p2.x) - fmaxf(fmaxf(bb[0].x, bb[1].x), bb[2].x),
                                                       fminf(fminf(bb[0].x, bb[1].x), bb[2].x) - fmaxf(fmaxf(p0.x, p1.x), p2.x));
                                const float gb = fmaxf(fminf(fminf(p0.y, p1.y), p2.y) - fmaxf(fmaxf(bb[0].y, bb[1].y), bb[2].y),
                                                       fminf(fminf(bb[0].y, bb[1].y), bb[2].y) - fmaxf(fmaxf(p0.y, p1.y), p2.y));
                                const float gc = fmaxf(fminf(fminf(p0.z, p1.z), p2.z) - fmaxf(fmaxf(bb[0].z, bb[1].z), bb[2].z),
                                                       fminf(fminf(bb[0].z, bb[1].z), bb[2].z) - fmaxf(fmaxf(p0.z, p1.z), p2.z));
                                const float x = fmaxf(ga, 0.0f), y = fmaxf(gb, 0.0f), z = fmaxf(gc, 0.0f);
                                g2 = __builtin_fmaf(x, x, __builtin_fmaf(y, y, z * z));
                            }
                            keep = bound_sqrt(g2) * (1.0f - 0x1p-20f) - e_abs <= tau;
                        }
                        const uint64_t mk = __ballot(keep);
                        if (keep) tq[n_full + mbcnt(mk)] = make_uint2(tA, tB);
                        n_full += __popcll(mk);
                    }
                    if (lane == 0) ctr_add(C_TRI_BYTES, 72ull * total);
                    wave_sync();
                }
                for (uint32_t p0 = 0; p0 < n_full; p0 += WAVE) {
                    int res = 0;
                    float dres = INFINITY;
                    const uint32_t n_pass = min(n_full - p0, (uint32_t)WAVE);
                    bool active = lane < n_pass;
                    uint32_t triA = 0, triB = 0;
                    V3<float> a[3], b[3];
                    if (active) {
                        if (screen) {
                            const uint2 pr = tq[p0 + lane];
                            triA = pr.x;
                            triB = pr.y;
                        } else {
                            pair_of(lane, triA, triB);
                        }
                        V3<float> a0[3];
                        load_tri(MA.tris, triA, a0);
                        load_tri(MB.tris, triB, b);
#pragma unroll
                        for (int v = 0; v < 3; v++) a[v] = xform_f32(P, a0[v]);
                        // 0 disjoint, 1 intersecting, 2 undecided in FP32 (decided by the FP64 stage)
                        res = tri_tri_f32(a, b);
                        if (MODE == MODE_DIST) {
                            // undecided pairs also get their FP32 feature distance:
                            // it is accurate if they are disjoint and too large
                            // (never too small) if they intersect, so the running
                            // bound stays safe; the FP64 stage decides them
                            dres = res != 1 ? tri_dist_f32(a, b) : 0.0f;
                        }
                    }
                    if (lane == 0) {
                        ctr_add(C_TRI_TESTS, n_pass);
                        ctr_add(C_LEAF_STEPS, 1);
                        if (!screen) ctr_add(C_TRI_BYTES, 72ull * n_pass);
                    }
                    // leaf pairs for the FP64 stage: undecided intersections, and
                    // distances that could be the minimum
                    bool defer;
                    if (MODE == MODE_BOOL || MODE == MODE_PAIRS) {
                        bool h = active && res == 1;
                        defer = active && res == 2;
                        uint64_t mh = __ballot(h);
                        if (mh) {
                            hit = true;
                            if (lane == 0) {
                                q.hit[pose] = 1;
                                if (MODE == MODE_BOOL && shared) rmw_xchg(&q.ws.hitw[pose], 1u);
                            }
                        }
                        if (MODE == MODE_PAIRS && mh) {
                            uint32_t nh = __popcll(mh);
                            uint32_t b0 = 0;
                            if (lane == 0) b0 = atomicAdd(&hdr->pair_count, nh);
                            b0 = uni(b0);
                            if (h) {
                                uint32_t idx = b0 + mbcnt(mh);
                                if (idx < q.pair_cap)
                                    q.ws.pair_raw[idx] = make_uint4(pose, MA.perm[triA], MB.perm[triB], 0u);
                            }
                            if (b0 + nh > q.pair_cap) pair_overflow = true;
                        }
                    } else {
                        // a certified intersection is distance 0: the pose is done
                        if (__ballot(active && res == 1)) {
                            best64 = 0.0;
                            dres = 0.0f;
                        }
                        float wmin = wave_min(dres);
                        if (wmin < best32) {
                            best32 = wmin;
                            if (shared && lane == 0)
                                __hip_atomic_fetch_min(&q.ws.best32[pose], __float_as_uint(best32), __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
                        }
                        defer = active && (res == 2 || (res == 0 && dres <= add_up(best32, 2.0f * e_abs)));
                    }
                    const uint64_t md = __ballot(defer);
                    if (md) {
                        const uint32_t nd = __popcll(md);
                        uint32_t f0 = 0;
                        if (lane == 0) f0 = atomicAdd(&hdr->fix_count, nd);
                        f0 = uni(f0);
                        if (defer) {
                            const uint32_t idx = f0 + mbcnt(md);
                            // an undecided pair is stored with distance 0, which the
                            // FP64 stage's final-bound filter always keeps
                            const uint32_t dw = res == 2 ? 0u : __float_as_uint(dres);
                            if (idx < q.ws.fix_cap) q.ws.fix[idx] = make_uint4(pose, triA, triB, dw);
                        }
                        if (f0 + nd > q.ws.fix_cap) fix_overflow = true;
                        if (lane == 0) ctr_add(C_TRI_FP64, nd);
                    }
                    if constexpr (!kScreens) break;  // one pass: at most 64 pairs were taken
                }
                wave_sync();
                continue;
            }
            if (top == 0) break;

            // -------- feed waiting waves with the bottom of the stack --------
            if (can_donate && top >= q.donate_min_top && steps >= next_look && steps >= q.donate_min_steps) {
                // collision queries: a unit that has run long looks every other
                // step, so the long units (the batch's critical path) win the
                // waiting helpers more often (distance queries lose by it)
                next_look = steps + ((MODE != MODE_DIST && steps >= kOldSteps) ? 2u : q.donate_period);
                uint32_t want = 0;
                if (lane == 0) {
                    unsigned long long ht = poll64((unsigned long long *)&hdr->q_head);
                    uint32_t h = (uint32_t)ht, t = (uint32_t)(ht >> 32);
                    const uint32_t share = q.donate_keep ? (top > q.donate_keep ? top - q.donate_keep : 0u) : top / 2;
                    // waiting helpers (claimed slots not yet filled) take what they claimed
                    want = h > t ? min(h - t, min(share, q.max_donate)) : 0u;
                }
                want = uni(want);
                if (want && publish(pose, want, want, best32) == want) {
                    if (lane == 0) ctr_add(C_DONATED, want);
                    shared = true;
                    // the remaining entries move down (their records stay put)
                    const uint32_t rem = top - want;
                    for (uint32_t b0 = 0; b0 < rem; b0 += WAVE) {
                        const uint32_t i = b0 + lane;
                        uint32_t ev = 0;
                        uint2 tv = make_uint2(0, 0);
                        float lv = 0.0f;
                        if (i < rem) {
                            ev = ent[want + i];
                            if constexpr (kTopoEnt) tv = ent_tp[want + i];
                            if (MODE == MODE_DIST) lv = ent_lb[want + i];
                        }
                        wave_sync();
                        if (i < rem) {
                            ent[i] = ev;
                            if constexpr (kTopoEnt) ent_tp[i] = tv;
                            if (MODE == MODE_DIST) ent_lb[i] = lv;
                        }
                        wave_sync();
                    }
                    top = rem;
                }
            }


            // -------- node step: pop the top entries whose children fit one decode pass --------
            const float tau = MODE == MODE_DIST ? add_up(best32, pz[3].x) : 0.0f;
            // lane l <= PMAX reads the (l+1)-th entry from the top, with both
            // topology words (collision queries keep them in the entry)
            uint32_t my_e = 0, my_tA = 0, my_tB = 0, my_na = 0, my_nb = 0;
            if (lane <= (uint32_t)PMAX && lane < top) {
                const uint32_t idx = top - 1 - lane;
                my_e = ent[idx];
                const uint2 tp = entry_topo(idx, my_e);
                my_tA = tp.x;
                my_tB = tp.y;
                my_na = topo_leaf(my_tA) ? 1u : topo_count(my_tA);
                my_nb = topo_leaf(my_tB) ? 1u : topo_count(my_tB);
                if (MODE == MODE_DIST && ent_lb[idx] > tau) my_na = my_nb = 0;  // culled
            }
            const uint32_t my_tk = my_na * my_nb;
            // the newest live frame (the top entry's) ends last: its end bounds
            // where any new frame can start
            const uint32_t f_top_end = lane_of(fe_v, (int)(uni(my_e) >> (2 * REC_BITS)));
            // proximity queries dive one expansion at a time until a first leaf
            // distance exists: without a bound nothing is culled
            const bool dive = MODE == MODE_DIST && best32 == INFINITY;
            // One entry goes alone when no second one could join it (its tests
            // fill the pass, as with two branching-factor-8 nodes, or the
            // stack holds one entry): the fit checks then run on uniform values
            // and the scan over the popped lanes is skipped.
            const uint32_t tk0 = lane_of(my_tk, 0);
            const bool single = tk0 > 0 && (dive || q.max_pop == 1 || top == 1 || tk0 + lane_of(my_tk, 1) > TMAX);
            uint32_t n_pop, nA_tot, total_rec, tasks_tot, new_id, new_meta, pk = 0, my_pk = 0;
            if (single) {
                const uint32_t na0 = lane_of(my_na, 0), nb0 = lane_of(my_nb, 0), rem = top - 1u;
                new_id = rem > 0 ? (lane_of(my_e, 1) >> (2 * REC_BITS)) + 1u : 0u;
                const uint32_t nbase0 = rem > 0 ? f_top_end : 0u;
                const bool ok0 = na0 <= AMAX && na0 + nb0 <= (uint32_t)WAVE && tk0 <= TMAX &&
                                 rem + tk0 <= lim.entries && lq_count + tk0 <= lim.leafq &&
                                 new_id < (uint32_t)MAX_FRAMES && nbase0 + na0 + nb0 <= lim.records &&
                                 nbase0 + na0 + nb0 <= REC_MASK + 1u;
                n_pop = ok0 ? 1u : 0u;
                nA_tot = na0;
                total_rec = na0 + nb0;
                tasks_tot = tk0;
                new_meta = meta_word(0u, na0, nb0, 0u);
            } else {
                // inclusive prefix over lanes 0..PMAX-1 of (A records, B records,
                // tests, expanded entries), packed in one word (8, 8, 10 and 6 bits)
                my_pk = lane < (uint32_t)PMAX ? (my_na | (my_nb << 8) | (my_tk << 16) | ((my_tk > 0 ? 1u : 0u) << 26))
                                              : 0u;
                pk = my_pk;
                static_assert(PMAX == 8, "the scan covers 8 lanes");
                pk += row_shr<1>(pk);
                pk += row_shr<2>(pk);
                pk += row_shr<4>(pk);
                const uint32_t inA = pk & 0xFFu, inB = (pk >> 8) & 0xFFu, inT = (pk >> 16) & 0x3FFu, inX = pk >> 26;
                // with lane+1 entries popped the new frame sits on top of the frame
                // of the next remaining entry (lane+1 read it): its level is one more
                const uint32_t nx_e = row_shl<1>(my_e);
                const uint32_t rem_l = top - 1u - lane;
                const uint32_t nid_l = rem_l > 0 ? (nx_e >> (2 * REC_BITS)) + 1u : 0u;
                const uint32_t nbase_l = rem_l > 0 ? f_top_end : 0u;
                // A frame stays live while any of its entries is pending, so a
                // wider frame pins records for its whole subtree.  Where the record
                // space cannot hold a full-depth descent (the host decides), more
                // than one entry is popped only while the new frame leaves room for
                // a frame of the top entry's size at every level a descent below
                // it can still take (the two trees' depths minus the new frame's level).
                const uint32_t levels = MA.depth + MB.depth;
                const uint32_t reserve = (lane == 0 || !q.pop_reserve)
                                             ? 0u
                                             : lane_of(my_na + my_nb, 0) * (levels > nid_l ? levels - nid_l : 0u);
                // culled entries (distance queries) cost nothing and may always go
                const bool ok = lane < (uint32_t)PMAX && inX <= q.max_pop && lane < top && (!dive || lane == 0) &&
                                inA <= AMAX && inA + inB <= (uint32_t)WAVE && inT <= TMAX &&
                                rem_l + inT <= lim.entries && lq_count + inT <= lim.leafq &&
                                nid_l < (uint32_t)MAX_FRAMES && nbase_l + inA + inB + reserve <= lim.records &&
                                nbase_l + inA + inB <= REC_MASK + 1u;
                n_pop = (uint32_t)__builtin_ctzll(~__ballot(ok));  // leading lanes that fit
                const int last = n_pop > 0 ? (int)n_pop - 1 : 0;
                nA_tot = lane_of(inA, last);
                total_rec = nA_tot + lane_of(inB, last);
                tasks_tot = lane_of(inT, last);
                static_assert(TMAX < 1024u && PMAX < 64, "packed prefix fields");
                new_id = lane_of(nid_l, last);
                // the new frame's entries (culled ones stay, with no tasks): first
                // A record and first B record in the frame, B's child count, first task
                const uint32_t ex = pk - my_pk;  // exclusive prefix
                new_meta = meta_word(ex & 0xFFu, nA_tot + ((ex >> 8) & 0xFFu), my_nb, (ex >> 16) & 0x3FFu);
            }
            if (n_pop == 0) {
                // not even the top entry fits the LDS state: hand every pending
                // pair (node pairs with their decoded bounds, and queued leaf
                // pairs) to the item queue; the unit ends here
                const uint32_t n_items = top + lq_count;
                if (can_donate && publish(pose, n_items, top, best32) == n_items) {
                    if (lane == 0) ctr_add(C_DONATED, n_items);
                    shared = true;
                } else {
                    overflow = true;
                }
                break;
            }
            top -= n_pop;
            // the new frame starts where the frame of the next remaining entry ends
            const uint32_t new_base = top > 0 ? lane_of(fe_v, (int)new_id - 1) : 0u;
            const uint32_t ns = single ? 1u : __popcll(__ballot(lane < n_pop && my_tk > 0));
            if (ns == 0) continue;
            // decode: one lane per new record, A records first, then B records.
            // A record's entry is the popped lane whose run of records holds
            // it (with one popped entry, lane 0's, uniform); its parent data
            // comes across lanes.
            const bool sideA = lane < nA_tot;
            const uint32_t r = sideA ? lane : lane - nA_tot;
            uint32_t g_e, g_pA, g_pB, off = 0;
            if (n_pop == 1) {
                g_e = uni(my_e);
                g_pA = uni(my_tA);
                g_pB = uni(my_tB);
            } else {
                uint32_t e = 0;
                const uint32_t sh = sideA ? 0u : 8u;  // A's or B's record count in the packed prefix
#pragma unroll
                // (the last popped entry's run ends past every record of its
                // side, so only the first n_pop - 1 ends are compared)
                for (int s = 0; s < PMAX - 1; s++) {
                    if ((uint32_t)s + 1u >= n_pop) break;
                    const uint32_t w = lane_of(pk, s);
                    const uint32_t end = (w >> sh) & 0xFFu;
                    if (end <= r) {
                        e = (uint32_t)s + 1u;
                        off = end;
                    }
                }
                e = min(e, (uint32_t)PMAX - 1u);
                g_e = gather(my_e, e);
                g_pA = gather(my_tA, e);
                g_pB = gather(my_tB, e);
            }
            uint32_t my_topo = 0;
            float my_b[DW];
            const bool dec = lane < total_rec;
            {
                // algorithmic bytes: topology word and codes of every decoded child
                const bool from_node = dec && !topo_leaf(sideA ? g_pA : g_pB);
                st_bytes += (unsigned long long)__popcll(__ballot(from_node && sideA)) * code_bytes_A +
                            (unsigned long long)__popcll(__ballot(from_node && !sideA)) * code_bytes_B;
            }
            if (dec) {
                const uint32_t c = r - off;
                const uint32_t prec = sideA ? (g_e & REC_MASK) : ((g_e >> REC_BITS) & REC_MASK);
                const uint32_t ptopo = sideA ? g_pA : g_pB;
                float pb[RW];
                if (topo_leaf(ptopo)) {
                    // a leaf against an inner node: the leaf itself joins the frame
                    load_rec(prec, pb);
                    my_topo = ptopo;
#pragma unroll
                    for (int k = 0; k < (int)DW; k++) my_b[k] = pb[k];
                } else {
                    const DevModel &M = sideA ? MA : MB;
                    NodeWords<K, BITS, OBB> nw;
                    load_node<K, BITS, OBB>(M, topo_first(ptopo) + c, my_topo, nw);
                    load_rec(prec, pb);
                    decode_child<K, BITS, OBB>(M, my_topo, nw, pb, my_b);
                }
                // the new frame may overwrite records that other decoding
                // lanes read above: the wave's LDS accesses run in program
                // order, so only the compiler must keep the stores below
                // the reads (one block, so the decoded bounds need no copies
                // for the lanes that decode nothing)
                wave_sync();
                store_rec(new_base + lane, my_b, my_topo);
                if (sideA) prep_A(lane, my_b, my_topo);
            }
            if (lane == new_id) fe_v = new_base + total_rec;
            st_exp += ns;
            st_steps++;
            st_max_rec = max(st_max_rec, new_base + total_rec);
            wave_sync();
            // the new frame becomes the current one
            f_base = new_base;
            f_nA = nA_tot;
            f_ns = n_pop;
            f_tasks = tasks_tot;
            f_level = new_id;
            f_meta = new_meta;
            have_frame = true;
        }
        if (lane == 0) {
            ctr_max(C_MAX_POSE_STEPS, steps);
            ctr_add(C_BV_TESTS, st_tests);
            ctr_max(C_MAX_ENTRIES, st_max_ent);
            ctr_add(C_NODE_BYTES, st_bytes);
            ctr_add(C_EXPANSIONS, st_exp);
            ctr_add(C_NODE_STEPS, st_steps);
            ctr_max(C_MAX_RECORDS, st_max_rec);
        }
        if (q.prio_steps && steps >= q.prio_steps) __builtin_amdgcn_s_setprio(0);

        // ---- results of this unit ----
        if (lane == 0) {
            if (overflow) q.status[pose] = 1;            // CBVH_POSE_STACK_OVERFLOW
            else if (fix_overflow) q.status[pose] = 3;   // CBVH_POSE_FP64_OVERFLOW
            else if (pair_overflow) q.status[pose] = 2;  // CBVH_POSE_PAIR_OVERFLOW
            if (MODE == MODE_DIST) {
                if (best32 < INFINITY)
                    __hip_atomic_fetch_min(&q.ws.best32[pose], __float_as_uint(best32), __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
                if (best64 < INFINITY)
                    __hip_atomic_fetch_min(&q.ws.best64[pose], (unsigned long long)__double_as_longlong(best64),
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (from_item) rmw_add(&hdr->pending, 0xFFFFFFFFu);  // this item is finished
        }
        wave_sync();
    }
    // ---- this wave's counter row (plain stores: thousands of waves exit
    // at about the same time, and atomics on one line would serialise) ----
    if (wave_id == 0 && lane == 0) hdr->n_waves = n_waves;
    const unsigned long long t_exit = wall_clock64();
    wave_sync();
    if (lane < (uint32_t)C_NUM) {
        unsigned long long v = ctr[lane];
        if (lane == C_T_END) v = t_exit;
        q.ws.wave_ctr[(size_t)wave_id * C_NUM + lane] = v;
    }
}
// ---------------------------------------------------------------------------
// workspace init, distance output, pair-list finalize
// ---------------------------------------------------------------------------
__global__ void init_kernel(WsHeader *hdr, uint8_t *hit, uint8_t *status, unsigned int *best32,
                            unsigned long long *best64, uint32_t *pair_cnt, uint32_t *pair_cursor, uint32_t *hitw,
                            uint32_t *ready, uint32_t n_ready, uint32_t n, uint32_t pending0)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < sizeof(WsHeader) / 4) {
        uint32_t v = 0;
        if (i == offsetof(WsHeader, pending) / 4) v = pending0;  // waves add themselves when they start
        ((uint32_t *)hdr)[i] = v;
    }
    if (i < n_ready) ready[i] = 0;
    if (i < n) {
        status[i] = 0;
        if (hit) hit[i] = 0;
        if (hitw) hitw[i] = 0;
        if (best32) {
            best32[i] = 0x7F800000u;                 // +inf
            best64[i] = 0x7FF0000000000000ull;       // +inf
        }
        if (pair_cnt) {
            pair_cnt[i] = 0;
            pair_cursor[i] = 0;
        }
    }
}

// FP64 stage, one thread per deferred leaf pair: decides the intersections
// that FP32 left undecided, and refines every distance within the final
// FP32 bound's reach (2 e of the pose's best FP32 distance) exactly.
template <int MODE>
__global__ __launch_bounds__(256) void fix_kernel(QueryArgs q)
{
    const uint32_t total = min(q.ws.hdr->fix_count, q.ws.fix_cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const uint4 f = q.ws.fix[i];
        const uint32_t pose = f.x;
        if (MODE == MODE_BOOL && q.hit[pose]) continue;
        const float *pp = q.poses + 12 * (size_t)pose;
        const DevModel &B = q.pose_obj ? q.Btab[q.pose_obj[pose]] : q.B;  // validated by the traversal
        if (MODE == MODE_DIST) {
            const float e = dist_err_abs(pp, q.A.max_abs, B.max_abs);
            if (__uint_as_float(f.w) > add_up(__uint_as_float(q.ws.best32[pose]), 2.0f * e)) continue;
        }
        Pose P;
#pragma unroll
        for (int r = 0; r < 3; r++) {
#pragma unroll
            for (int c = 0; c < 3; c++) P.R[3 * r + c] = pp[4 * r + c];
            P.t[r] = pp[4 * r + 3];
        }
        V3<float> a0[3], b0[3];
        load_tri(q.A.tris, f.y, a0);
        load_tri(B.tris, f.z, b0);
        V3<double> a64[3], b64[3];
#pragma unroll
        for (int v = 0; v < 3; v++) {
            a64[v] = xform_f64(P, a0[v]);
            b64[v] = to64(b0[v]);
        }
        const bool inter = tri_tri_f64(a64, b64);
        if (MODE == MODE_BOOL) {
            if (inter) q.hit[pose] = 1;
        } else if (MODE == MODE_PAIRS) {
            if (inter) {
                q.hit[pose] = 1;
                const uint32_t idx = atomicAdd(&q.ws.hdr->pair_count, 1u);
                if (idx < q.pair_cap) q.ws.pair_raw[idx] = make_uint4(pose, q.A.perm[f.y], B.perm[f.z], 0u);
                else if (q.status[pose] == 0) q.status[pose] = 2;  // CBVH_POSE_PAIR_OVERFLOW
            }
        } else {
            double d = 0.0;
            if (!inter) {
                V3<double> ar[3], br[3];
#pragma unroll
                for (int v = 0; v < 3; v++) {
                    ar[v] = vsub(a64[v], a64[0]);
                    br[v] = vsub(b64[v], a64[0]);
                }
                d = sqrt(tri_tri_dist2(ar, br));
            }
            atomicMin(&q.ws.best64[pose], (unsigned long long)__double_as_longlong(d));
        }
    }
}

// After a wave gave up waiting for an item (the wait limit), work handed to
// the queue may never have run: every pose of the query is flagged
// CBVH_POSE_INCOMPLETE unless it already carries a failure of its own.
__global__ void incomplete_kernel(const WsHeader *hdr, uint8_t *status, uint32_t n)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && hdr->error && status[i] == 0) status[i] = 5;  // CBVH_POSE_INCOMPLETE
}

__global__ void dist_out_kernel(const unsigned long long *best64, float *dist, uint32_t n)
{
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dist[i] = (float)__longlong_as_double((long long)best64[i]);
}

__global__ void pair_count_kernel(const WsHeader *hdr, const uint4 *raw, uint32_t cap, uint32_t *cnt)
{
    uint32_t total = min(hdr->pair_count, cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x)
        atomicAdd(&cnt[raw[i].x], 1u);
}

// exclusive scan of n counts by one workgroup of 1024 threads
__global__ __launch_bounds__(1024) void pair_scan_kernel(const uint32_t *cnt, uint32_t *offsets, uint32_t n)
{
    __shared__ uint32_t part[1024];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint32_t b = 0; b < n; b += 1024) {
        uint32_t i = b + threadIdx.x;
        uint32_t v = i < n ? cnt[i] : 0u;
        part[threadIdx.x] = v;
        __syncthreads();
        for (uint32_t o = 1; o < 1024; o <<= 1) {
            uint32_t t = threadIdx.x >= o ? part[threadIdx.x - o] : 0u;
            __syncthreads();
            part[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < n) offsets[i] = carry + part[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 0) carry += part[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) offsets[n] = carry;
}

__global__ void pair_scatter_kernel(const WsHeader *hdr, const uint4 *raw, uint32_t cap, const uint32_t *offsets,
                                    uint32_t *cursor, unsigned long long *keys)
{
    uint32_t total = min(hdr->pair_count, cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        uint4 r = raw[i];
        uint32_t pos = offsets[r.x] + atomicAdd(&cursor[r.x], 1u);
        keys[pos] = ((unsigned long long)r.y << 32) | r.z;
    }
}

// sort each pose's keys (triA << 32 | triB) and write (pose, triA, triB);
// bitonic sort in LDS for segments up to 4096 keys, else in global memory
constexpr uint32_t SORT_LDS = 4096;
__global__ __launch_bounds__(256) void pair_sort_kernel(const uint32_t *offsets, unsigned long long *keys,
                                                        uint32_t *out, uint32_t n)
{
    __shared__ unsigned long long sk[SORT_LDS];
    for (uint32_t pose = blockIdx.x; pose < n; pose += gridDim.x) {
        uint32_t b = offsets[pose], e = offsets[pose + 1], len = e - b;
        if (len == 0) continue;
        uint32_t p2 = 1;
        while (p2 < len) p2 <<= 1;
        unsigned long long *arr = keys + b;
        if (p2 <= SORT_LDS) {
            for (uint32_t i = threadIdx.x; i < p2; i += blockDim.x) sk[i] = i < len ? arr[i] : ~0ull;
            __syncthreads();
            for (uint32_t k = 2; k <= p2; k <<= 1)
                for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                    for (uint32_t i = threadIdx.x; i < p2; i += blockDim.x) {
                        uint32_t l = i ^ j;
                        if (l > i) {
                            bool up = (i & k) == 0;
                            unsigned long long x = sk[i], y = sk[l];
                            if ((x > y) == up) {
                                sk[i] = y;
                                sk[l] = x;
                            }
                        }
                    }
                    __syncthreads();
                }
            for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) arr[i] = sk[i];
            __syncthreads();
        } else {
            // odd-even transposition in global memory (large segments are rare)
            for (uint32_t round = 0; round < len; round++) {
                for (uint32_t i = 2 * threadIdx.x + (round & 1); i + 1 < len; i += 2 * blockDim.x) {
                    unsigned long long x = arr[i], y = arr[i + 1];
                    if (x > y) {
                        arr[i] = y;
                        arr[i + 1] = x;
                    }
                }
                __threadfence_block();
                __syncthreads();
            }
        }
        for (uint32_t i = threadIdx.x; i < len; i += blockDim.x) {
            unsigned long long k = arr[i];
            out[3 * (size_t)(b + i)] = pose;
            out[3 * (size_t)(b + i) + 1] = (uint32_t)(k >> 32);
            out[3 * (size_t)(b + i) + 2] = (uint32_t)k;
        }
        __syncthreads();
    }
}

// decode every node: one thread per treelet walks its nodes in order (the
// top group is absolute, every other node's parent lies earlier in the
// same treelet), the random access that treelets give
template <int K, int BITS, bool OBB = false>
__global__ void decode_all_kernel(DevModel M, float *out)
{
    // per node: its bounds (lo, hi per slab), or an OBB's whole descriptor
    constexpr uint32_t DW = dec_words(K, OBB);
    uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (!bits_are_codes((uint32_t)BITS)) {
        // absolute descriptors (FP32 or FP16): one thread per node
        for (uint32_t i = t; i < M.n_nodes; i += gridDim.x * blockDim.x) {
            float b[DW];
            decode_node<K, BITS, OBB>(M, i, (const float *)nullptr, b);
            for (uint32_t k = 0; k < DW; k++) out[(size_t)i * DW + k] = b[k];
        }
        return;
    }
    if (t >= M.n_treelets) return;
    uint32_t first = M.treelets[t], end = M.treelets[t + 1];
    for (uint32_t i = first; i < end; i++) {
        uint32_t w = M.topo[i];
        if (topo_abs(w)) {
            float b[DW];
            decode_node<K, BITS, OBB>(M, i, (const float *)nullptr, b);
            for (uint32_t k = 0; k < DW; k++) out[(size_t)i * DW + k] = b[k];
        }
        if (!topo_leaf(w)) {
            uint32_t c0 = topo_first(w), nc = topo_count(w);
            if (c0 >= end) continue;  // children start another treelet (absolute there)
            for (uint32_t c = 0; c < nc; c++) {
                uint32_t node = c0 + c;
                float b[DW];
                decode_node<K, BITS, OBB>(M, node, out + (size_t)i * DW, b);
                for (uint32_t k = 0; k < DW; k++) out[(size_t)node * DW + k] = b[k];
            }
        }
    }
}

// Launch knobs (for the tuner; defaults when unset or 0): CBVH_WAVES_PER_CU,
// CBVH_MAX_POP (entries per node step), CBVH_DONATE_MIN_STEPS,
// CBVH_MAX_HELPERS.
//
// Once the pose queue is empty only some waves stay to take donated work:
// every wave that stays competes for issue slots with the long units on the
// critical path, and units feed them only after some steps, so that units
// about to finish do not split needlessly.  Early-exit collision queries
// have short tails (one helper per CU), pair lists longer ones (two), and
// branch-and-bound distance queries the longest (four).  Distance units run
// thousands of steps, so they start feeding later and look at the queue less
// often (every 32 steps after 32: about 6 % faster than every 8 after 16).
// Measured on MI355X over the collision, pair-list and proximity workloads.
constexpr uint32_t donate_min_steps(int mode) { return mode == MODE_DIST ? 32u : 16u; }
constexpr uint32_t donate_period(int mode) { return mode == MODE_DIST ? 32u : kDonatePeriod; }
constexpr uint32_t helpers_per_cu(int mode) { return mode == MODE_DIST ? 4u : mode == MODE_PAIRS ? 2u : 1u; }
uint32_t env_u32(const char *name, uint32_t dflt)
{
    const char *v = getenv(name);
    if (!v || !*v) return dflt;
    unsigned long x = strtoul(v, nullptr, 10);
    return x ? (uint32_t)x : dflt;
}

template <int K, int BITS, int MODE, bool OBB>
hipError_t launch_traverse(const QueryArgs &q, const StackLimits &lim, hipStream_t s)
{
    Layout L = make_layout(K, MODE, lim, OBB);
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (cus < 1) cus = 256;
    // as many waves as fit on a CU at once (registers and LDS): the waves
    // are persistent, so every one of them must be resident
    auto waves_fitting = [&](uint32_t wpg) -> uint32_t {
        int occ = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, reinterpret_cast<const void *>(traverse_kernel<K, BITS, MODE, OBB>),
                                                         WAVE * wpg, L.total * wpg) != hipSuccess || occ < 1) {
            (void)hipGetLastError();  // clear a failed query's error; fall back to the LDS bound
            occ = (int)(160u * 1024u / (L.total * wpg + 256u));
        }
        return (uint32_t)max(occ, 1) * wpg;
    };
    // workgroup shape: waves per workgroup (independent waves; 1, 2 or 4).
    // Distance queries take two where that keeps as many waves resident (5 %
    // faster on the AABB proximity query, 1.5 % on 18-DOP models, in paired
    // runs; OBB models, whose larger LDS state then fits fewer waves, were
    // 24 % slower), collision queries one.
    uint32_t wpg = env_u32("CBVH_WAVES_PER_GROUP", 0u);
    if (wpg == 0) wpg = (MODE == MODE_DIST && waves_fitting(2) >= waves_fitting(1)) ? 2u : 1u;
    wpg = wpg >= 4 ? 4u : wpg >= 2 ? 2u : 1u;
    const uint32_t occ = waves_fitting(wpg) / wpg;
    uint32_t per_cu = min((uint32_t)occ * wpg, env_u32("CBVH_WAVES_PER_CU", 32u));
    if (per_cu > 32) per_cu = 32;
    per_cu = max(per_cu / wpg, 1u) * wpg;
    uint32_t waves = (uint32_t)cus * per_cu;
    // without donation a wave beyond the pose count has nothing to do
    if (q.no_split && waves > q.n_poses) waves = q.n_poses;
    if (waves > kMaxWaves) waves = kMaxWaves;  // rows of per-wave counters in the workspace
    const uint32_t grid = (waves + wpg - 1) / wpg;  // (kMaxWaves is a multiple of every group size)
    {
        // workspace init: header (no pending work: each wave adds itself
        // when it starts), per-pose outputs, and the item queue's ready
        // flags (its slots are numbered from 0 in every query)
        const uint32_t n = q.n_poses;
        const bool dist = q.mode == MODE_DIST, pairs = q.mode == MODE_PAIRS;
        const uint32_t n_ready = q.no_split ? 0u : q.ws.item_cap;
        uint32_t threads = 256, items = max(max(n, n_ready), (uint32_t)(sizeof(WsHeader) / 4));
        hipLaunchKernelGGL(init_kernel, dim3((items + threads - 1) / threads), dim3(threads), 0, s, q.ws.hdr,
                           dist ? nullptr : q.hit, q.status, dist ? q.ws.best32 : nullptr,
                           dist ? q.ws.best64 : nullptr, pairs ? q.ws.pair_cnt : nullptr,
                           pairs ? q.ws.pair_cursor : nullptr, q.mode == MODE_BOOL ? q.ws.hitw : nullptr, q.ws.ready,
                           n_ready, n, 0u);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    QueryArgs qq = q;
    // Multi-entry node steps pop freely where the record space holds one
    // expansion frame (both branching factors) at every level of the two
    // trees; elsewhere each such step keeps room for the rest of a descent.
    const uint32_t full_descent = 2u + (q.A.depth + q.B.depth) * (q.A.branching + q.B.branching);
    qq.pop_reserve = lim.records >= full_descent ? 0u : 1u;
    qq.max_pop = min(env_u32("CBVH_MAX_POP", (uint32_t)PMAX), (uint32_t)PMAX);
    qq.donate_min_steps = env_u32("CBVH_DONATE_MIN_STEPS", donate_min_steps(MODE));
    qq.max_helpers = env_u32("CBVH_MAX_HELPERS", (uint32_t)cus * helpers_per_cu(MODE));
    qq.donate_period = env_u32("CBVH_DONATE_PERIOD", donate_period(MODE));
    qq.donate_keep = env_u32("CBVH_DONATE_KEEP", 1u) == 1u ? 0u : env_u32("CBVH_DONATE_KEEP", 1u);
    qq.donate_min_top = max(env_u32("CBVH_DONATE_MIN_TOP", kDonateMinTop), 2u);
    qq.max_donate = max(min(env_u32("CBVH_MAX_DONATE", kMaxDonate), kMaxDonate), 1u);
    // collision queries: units past 16 steps get issue priority (about 2 % on
    // the scaled workload); distance queries gain nothing from it
    qq.prio_steps = env_u32("CBVH_PRIO_STEPS", MODE == MODE_DIST ? 0u : 16u);
    hipLaunchKernelGGL((traverse_kernel<K, BITS, MODE, OBB>), dim3(grid), dim3(WAVE * wpg), L.total * wpg, s, qq, lim);
    return hipGetLastError();
}

template <int K, int BITS, bool OBB = false>
hipError_t launch_mode(const QueryArgs &q, const StackLimits &lim, hipStream_t s)
{
    switch (q.mode) {
    case MODE_BOOL: return launch_traverse<K, BITS, MODE_BOOL, OBB>(q, lim, s);
    case MODE_PAIRS: return launch_traverse<K, BITS, MODE_PAIRS, OBB>(q, lim, s);
    default: return launch_traverse<K, BITS, MODE_DIST, OBB>(q, lim, s);
    }
}

hipError_t launch_any(const QueryArgs &q, const StackLimits &lim, hipStream_t s)
{
    uint32_t K = q.A.K, bits = q.A.bits;
    constexpr int F16 = (int)kBitsFp16;
    if (q.A.bv == kBvObb) {
        if (bits == 0) return launch_mode<3, 0, true>(q, lim, s);
        if (bits == 8) return launch_mode<3, 8, true>(q, lim, s);
        if (bits == 16) return launch_mode<3, 16, true>(q, lim, s);
        return hipErrorInvalidValue;  // rejected by the builder and the loader
    }
    if (K == 3) {
        if (bits == 0) return launch_mode<3, 0>(q, lim, s);
        if (bits == 8) return launch_mode<3, 8>(q, lim, s);
        if (bits == kBitsFp16) return launch_mode<3, F16>(q, lim, s);
        return launch_mode<3, 16>(q, lim, s);
    }
    if (bits == 0) return launch_mode<9, 0>(q, lim, s);
    if (bits == 8) return launch_mode<9, 8>(q, lim, s);
    if (bits == kBitsFp16) return launch_mode<9, F16>(q, lim, s);
    return launch_mode<9, 16>(q, lim, s);
}

}  // namespace

// Workspace of the allocation-free query entry point: a fixed device array
// that every call on a GPU shares (each GPU holds its own copy).  Host code
// never uses the array's name as an address: its device address comes from
// hipGetSymbolAddress, once per device, with that device current.
static __device__ __align__(256) unsigned char scratch[kStaticWorkspaceBytes];

hipError_t static_workspace(void **out)
{
    static std::mutex mu;
    static void *ptr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        ptr[dev] = p;
    }
    *out = ptr[dev];
    return hipSuccess;
}

size_t wave_state_bytes(uint32_t bv, int mode, const StackLimits &lim)
{
    return make_layout(bv_slabs(bv), mode, lim, bv == kBvObb).total;
}

StackLimits default_limits(uint32_t bv, int mode, uint32_t branching)
{
    // branch-and-bound keeps many more pairs pending than collision queries;
    // the sizes let 10 waves (AABB) or 8 waves (18-DOP, the most its
    // registers allow) fit a CU, about 5 % faster than 8 and 7 waves with
    // the larger stacks used before (768 and 512 entries).  OBB records are
    // as large as 18-DOP records: OBB models of branching factor 8 take the
    // 18-DOP sizes, narrower ones (deeper trees, whose descents need more
    // records) the AABB sizes.
    const bool big = bv == kBvDop18 || (bv == kBvObb && branching >= 8);
    if (mode == MODE_DIST) return big ? StackLimits{136, 448, 128} : StackLimits{256, 512, 128};
    return big ? StackLimits{80, 160, 128} : StackLimits{160, 384, 128};
}

uint32_t item_words(uint32_t bv) { return words_of_item(bv_slabs(bv), bv == kBvObb); }

hipError_t launch_query(const QueryArgs &q, const StackLimits &lim, hipStream_t s, uint32_t *pair_out,
                        uint32_t *pair_offsets)
{
    const uint32_t n = q.n_poses;
    const bool dist = q.mode == MODE_DIST, pairs = q.mode == MODE_PAIRS;
    // workspace init and the traversal (the init needs the traversal's grid)
    hipError_t e = launch_any(q, lim, s);
    if (e != hipSuccess) return e;
    {
        // the FP64 stage: its pair count is known on the device only, so a
        // fixed grid strides over it
        dim3 grid(1024), block(256);
        if (q.mode == MODE_BOOL) hipLaunchKernelGGL(fix_kernel<MODE_BOOL>, grid, block, 0, s, q);
        else if (q.mode == MODE_PAIRS) hipLaunchKernelGGL(fix_kernel<MODE_PAIRS>, grid, block, 0, s, q);
        else hipLaunchKernelGGL(fix_kernel<MODE_DIST>, grid, block, 0, s, q);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(incomplete_kernel, dim3((n + 255) / 256), dim3(256), 0, s, q.ws.hdr, q.status, n);
    if (dist) {
        hipLaunchKernelGGL(dist_out_kernel, dim3((n + 255) / 256), dim3(256), 0, s, q.ws.best64, q.dist, n);
    } else if (pairs) {
        hipLaunchKernelGGL(pair_count_kernel, dim3(256), dim3(256), 0, s, q.ws.hdr, q.ws.pair_raw, q.pair_cap,
                           q.ws.pair_cnt);
        hipLaunchKernelGGL(pair_scan_kernel, dim3(1), dim3(1024), 0, s, q.ws.pair_cnt, pair_offsets, n);
        hipLaunchKernelGGL(pair_scatter_kernel, dim3(256), dim3(256), 0, s, q.ws.hdr, q.ws.pair_raw, q.pair_cap,
                           pair_offsets, q.ws.pair_cursor, q.ws.pair_keys);
        uint32_t g = n < 2048 ? n : 2048;
        if (g < 1) g = 1;
        hipLaunchKernelGGL(pair_sort_kernel, dim3(g), dim3(256), 0, s, pair_offsets, q.ws.pair_keys, pair_out, n);
    }
    return hipGetLastError();
}

hipError_t launch_decode_all(const DevModel &m, float *out, hipStream_t s)
{
    uint32_t threads = 64;
    uint32_t items = bits_are_codes(m.bits) ? m.n_treelets : m.n_nodes;
    constexpr int F16 = (int)kBitsFp16;
    dim3 grid((items + threads - 1) / threads);
    if (m.bv == kBvObb) {
        if (m.bits == 0) hipLaunchKernelGGL((decode_all_kernel<3, 0, true>), grid, dim3(threads), 0, s, m, out);
        else if (m.bits == 8) hipLaunchKernelGGL((decode_all_kernel<3, 8, true>), grid, dim3(threads), 0, s, m, out);
        else if (m.bits == 16) hipLaunchKernelGGL((decode_all_kernel<3, 16, true>), grid, dim3(threads), 0, s, m, out);
        else return hipErrorInvalidValue;
    } else if (m.K == 3) {
        if (m.bits == 0) hipLaunchKernelGGL((decode_all_kernel<3, 0>), grid, dim3(threads), 0, s, m, out);
        else if (m.bits == 8) hipLaunchKernelGGL((decode_all_kernel<3, 8>), grid, dim3(threads), 0, s, m, out);
        else if (m.bits == kBitsFp16) hipLaunchKernelGGL((decode_all_kernel<3, F16>), grid, dim3(threads), 0, s, m, out);
        else hipLaunchKernelGGL((decode_all_kernel<3, 16>), grid, dim3(threads), 0, s, m, out);
    } else {
        if (m.bits == 0) hipLaunchKernelGGL((decode_all_kernel<9, 0>), grid, dim3(threads), 0, s, m, out);
        else if (m.bits == 8) hipLaunchKernelGGL((decode_all_kernel<9, 8>), grid, dim3(threads), 0, s, m, out);
        else if (m.bits == kBitsFp16) hipLaunchKernelGGL((decode_all_kernel<9, F16>), grid, dim3(threads), 0, s, m, out);
        else hipLaunchKernelGGL((decode_all_kernel<9, 16>), grid, dim3(threads), 0, s, m, out);
    }
    return hipGetLastError();
}

}  // namespace cbvh
