// Launch interface between the C ABI (capi.cpp) and the HIP kernels
// (traverse.hip).  Internal; not part of the public header.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "format.h"

namespace cbvh {

enum QueryMode : int { MODE_BOOL = 0, MODE_PAIRS = 1, MODE_DIST = 2 };

// Device view of an uploaded model: pointers into the blob copy.
struct DevModel {
    const uint32_t *topo;
    const uint8_t *codes;
    const float *absb;
    const float *tris;
    const uint32_t *perm;
    const uint32_t *treelets;
    uint32_t n_nodes, n_tris, n_treelets, stride, bits, K, leaf_size, depth;
    float max_abs;
};

// Counters kept in the workspace header (order matches cbvh_stats_t).
enum Counter : int {
    C_BV_TESTS = 0,
    C_TRI_TESTS,
    C_TRI_FP64,
    C_EXPANSIONS,
    C_NODE_BYTES,
    C_TRI_BYTES,
    C_FALLBACK_POSES,
    C_MAX_ENTRIES,
    C_MAX_RECORDS,
    C_NUM = 16
};

// Start of every workspace.
struct WsHeader {
    unsigned long long counters[C_NUM];
    uint32_t pose_next;       // persistent-wave pose queue (main pass)
    uint32_t fallback_count;  // poses queued for the global-stack pass
    uint32_t fallback_next;   // fallback-pass queue
    uint32_t pair_count;      // pairs appended (may exceed capacity)
    uint32_t pad[60];
};
static_assert(sizeof(WsHeader) == 384, "workspace header size");

// Limits of one wave's traversal state.
struct StackLimits {
    uint32_t records;  // decoded-BV records (frames)
    uint32_t entries;  // pending node pairs
    uint32_t leafq;    // pending leaf pairs
};

struct Workspace {
    WsHeader *hdr;
    uint32_t *fallback_list;  // [n]
    uint8_t *fell_back;       // [n]
    uint4 *pair_raw;          // [pair_capacity] (pose | pass << 31, triA, triB, 0)
    uint32_t *pair_cnt;       // [n]
    uint32_t *pair_cursor;    // [n]
    unsigned long long *pair_keys;  // [pair_capacity]
    uint8_t *garena;          // fallback stacks
    size_t garena_stride;     // bytes per fallback wave
    uint32_t garena_waves;
};

struct QueryArgs {
    DevModel A, B;
    const float *poses;
    uint32_t n_poses;
    int mode;
    uint8_t *hit;
    float *dist;
    uint8_t *status;
    uint32_t pair_cap;
    uint32_t no_fallback;
    Workspace ws;
};

// Bytes of one wave's traversal state for K slabs, a mode and limits.
size_t wave_state_bytes(uint32_t K, int mode, const StackLimits &lim);
StackLimits default_limits(uint32_t K);
StackLimits fallback_limits(uint32_t K);
uint32_t fallback_waves();

// Enqueue the whole query on `stream` (init, main pass, fallback pass, and
// for pair lists the count / scan / scatter / sort finalize).
hipError_t launch_query(const QueryArgs &q, const StackLimits &lim, hipStream_t stream, uint32_t *pair_out,
                        uint32_t *pair_offsets);

hipError_t launch_decode_all(const DevModel &m, float *out, hipStream_t stream);

}  // namespace cbvh
