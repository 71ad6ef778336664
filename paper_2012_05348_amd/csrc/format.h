// Byte layout of a compressed BVH ("blob"), shared by the host builder and
// the device kernels.  One contiguous little-endian buffer, uploaded once:
//
//   header (128 B) | topo[n] u32 | codes[n][stride] | abs[n_abs][2K or 20] f32 |
//   tris[n_tris][9] f32 | perm[n_tris] u32 | treelets[n_treelets+1] u32
//
// Sections start at 256-byte boundaries.  Nodes are numbered treelet by
// treelet; inside a treelet sibling groups follow breadth-first order, and
// the children of a node are always one contiguous group.
//
// Topology word: bit31 leaf, bit30 absolute (bounds stored in abs[], the
// code slot holds the abs index), bits27-29 count-1 (children, or triangles
// for a leaf), bits0-26 first child node / first leaf-order triangle.
//
// Codes per slab k (slab directions: x, y, z for AABB; plus x+y, x+z, y+z,
// x-y, x-z, y-z for the 18-DOP): (lo code, hi code) as u8 or u16; with
// bits == 0 the slot holds absolute (lo, hi) float32 bounds instead, and
// with bits == kBitsFp16 absolute (lo, hi) binary16 bounds rounded outward
// (the half-precision descriptors of the paper's section III.A).
//
// Oriented boxes (bv == 2, K == 3): a node is the parallelepiped
// {o + u0 a0 + u1 a1 + u2 a2 : lo_k <= u_k <= hi_k} spanned by a frame, i.e.
// an origin o and three nearly orthonormal float32 axes a_k, and its three
// slabs are the (lo, hi) intervals of the frame coordinates u_k.  Absolute
// nodes store their own frame; a relative node keeps its parent's frame and
// codes its frame-coordinate intervals against the parent's exactly as the
// fixed slabs of the other BV types are coded.  An OBB descriptor (an abs[]
// entry, or a node's code slot when bits == 0) is kObbWords float32:
//   lo0 hi0 lo1 hi1 lo2 hi2 | 0 | eps | o.x o.y o.z | a0 | a1 | a2
// with eps >= max |a_i . a_j - [i == j]| (how far the axes are from
// orthonormal).  OBB models take bits 0, 8 or 16.
//
// Decode of a relative node from its decoded parent [Pl, Ph] (per slab):
//   E = Ph - Pl (float32),  s = (E >= 2^-100) ? E * 2^-bits : 0,
//   lo = fmaf(q_lo, s, Pl),  hi = fmaf(-q_hi, s, Ph).
// q = 0 reproduces the parent bound, so decoded children always lie inside
// their decoded parent; the builder picks the largest codes that still
// enclose the exact child slab.
#pragma once
#include <stdint.h>

// the same inline helpers serve host C++ translation units and HIP kernels
#if defined(__HIP__)
#define CBVH_HD __host__ __device__
#else
#define CBVH_HD
#endif

namespace cbvh {

constexpr uint32_t kMagic = 0x48564243u;  // "CBVH"
constexpr uint32_t kVersion = 1;
constexpr uint32_t kHeaderBytes = 128;
constexpr uint32_t kSectionAlign = 256;
constexpr uint32_t kMaxBranching = 8;
constexpr uint32_t kMaxLeaf = 8;
constexpr uint32_t kIndexMask = 0x07FFFFFFu;
constexpr uint32_t kLeafBit = 0x80000000u;
constexpr uint32_t kAbsBit = 0x40000000u;

struct BlobHeader {
    uint32_t magic, version, bv, K, bits, branching, leaf_size, n_nodes;
    uint32_t n_tris, n_abs, n_treelets, code_stride, depth, treelet_bytes;
    uint64_t off_topo, off_codes, off_abs, off_tris, off_perm, off_treelets, total;
    float max_abs_coord;
    uint32_t reserved[3];
};
static_assert(sizeof(BlobHeader) == kHeaderBytes, "header is 128 bytes");

CBVH_HD inline bool topo_leaf(uint32_t w) { return (w & kLeafBit) != 0; }
CBVH_HD inline bool topo_abs(uint32_t w) { return (w & kAbsBit) != 0; }
CBVH_HD inline uint32_t topo_count(uint32_t w) { return ((w >> 27) & 7u) + 1u; }
CBVH_HD inline uint32_t topo_first(uint32_t w) { return w & kIndexMask; }
CBVH_HD inline uint32_t make_topo(uint32_t first, uint32_t count, bool leaf, bool absolute)
{
    return (first & kIndexMask) | ((count - 1u) << 27) | (absolute ? kAbsBit : 0u) | (leaf ? kLeafBit : 0u);
}

// `bits` value of models with binary16 absolute descriptors
constexpr uint32_t kBitsFp16 = 0x8010u;
// integer corrector codes relative to the parent (8 or 16 bits)?
CBVH_HD inline bool bits_are_codes(uint32_t bits) { return bits == 8u || bits == 16u; }

// BV types
constexpr uint32_t kBvAabb = 0, kBvDop18 = 1, kBvObb = 2;
// float32 words of an OBB descriptor (and of a decoded OBB node)
constexpr uint32_t kObbWords = 20;
// word offsets inside it
constexpr uint32_t kObbEps = 7, kObbOrigin = 8, kObbAxes = 11;

CBVH_HD inline uint32_t bv_slabs(uint32_t bv) { return bv == kBvDop18 ? 9u : 3u; }

inline uint32_t code_stride_for(uint32_t K, uint32_t bits, uint32_t bv = kBvAabb)
{
    if (bv == kBvObb && bits == 0) return 4u * kObbWords;
    return bits == 0 ? 8u * K : bits == kBitsFp16 ? 4u * K : (bits / 8u) * 2u * K;
}
// float32 words of one abs[] entry
inline uint32_t abs_words(uint32_t K, uint32_t bv) { return bv == kBvObb ? kObbWords : 2u * K; }

}  // namespace cbvh
