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
    uint32_t n_nodes, n_tris, n_treelets, stride, bits, K, leaf_size, depth, branching;
    uint32_t bv;  // kBvAabb, kBvDop18 or kBvObb
    float max_abs;
};

// Per-wave counters (order matches cbvh_stats_t); each wave writes its own
// row once, when it exits, and the host reduces the rows.
enum Counter : int {
    C_BV_TESTS = 0,
    C_TRI_TESTS,
    C_TRI_FP64,
    C_EXPANSIONS,
    C_NODE_BYTES,
    C_TRI_BYTES,
    C_DONATED,         // work items handed from a busy wave to idle ones
    C_MAX_ENTRIES,
    C_MAX_RECORDS,
    C_T_START,         // min wall clock (100 MHz) of a wave's first pose
    C_T_DRAIN,         // min wall clock at which a wave found the pose queue empty
    C_T_END,           // max wall clock of a wave's exit
    C_MAX_POSE_STEPS,  // most node + leaf steps one work unit used
    C_NODE_STEPS,      // node steps (each decodes one frame of children)
    C_LEAF_STEPS,      // leaf steps (each tests up to 64 triangle pairs)
    C_NUM = 16
};

// Most waves one traversal launch may have (rows of per-wave counters).
constexpr uint32_t kMaxWaves = 8192;

// Start of every workspace.  The queue words that many waves hammer at
// once sit on cache lines of their own; the per-wave counter rows
// (kMaxWaves x C_NUM u64) follow the header.
struct WsHeader {
    uint32_t pose_next;   // persistent-wave pose queue
    uint32_t pair_count;  // pairs appended (may exceed capacity)
    uint32_t error;       // a wave gave up waiting for an item: every pose is then flagged incomplete
    uint32_t fix_count;   // leaf pairs handed to the FP64 stage (may exceed capacity)
    uint32_t n_waves;     // waves of the traversal launch (rows of per-wave counters)
    uint32_t pad0[27];
    uint32_t q_head;      // next item slot to claim (8-byte aligned: read together with q_tail)
    uint32_t q_tail;      // next item slot to reserve
    uint32_t pad1[30];
    uint32_t pending;     // started waves that may still start poses + published items not yet finished
    uint32_t gone;        // set once helpers began to leave: no unit hands work over after that
    uint32_t pad2[30];
    uint32_t pad3[32];
};
static_assert(sizeof(WsHeader) == 512, "workspace header size");

// Limits of one wave's traversal state (LDS).
struct StackLimits {
    uint32_t records;  // decoded-BV records (frames)
    uint32_t entries;  // pending node pairs
    uint32_t leafq;    // pending leaf pairs
};

struct Workspace {
    WsHeader *hdr;
    unsigned long long *wave_ctr;  // [kMaxWaves][C_NUM] per-wave counters
    uint32_t *items;          // donated work items, item_words dwords each
    uint32_t *ready;          // [item_cap] non-zero once an item is published
    uint32_t item_cap;        // item slots (slot indices are never reused within a query)
    uint32_t item_words;      // dwords per item
    uint32_t *hitw;           // [n] collision found (read and written with atomics)
    uint4 *fix;               // [fix_cap] (pose, triA, triB, FP32 distance bits) for the FP64 stage
    uint32_t fix_cap;
    unsigned int *best32;     // [n] distance: FP32 bits of the best leaf distance so far
    unsigned long long *best64;  // [n] distance: FP64 bits of the best refined distance
    uint4 *pair_raw;          // [pair_capacity] (pose, triA, triB, 0)
    uint32_t *pair_cnt;       // [n]
    uint32_t *pair_cursor;    // [n]
    unsigned long long *pair_keys;  // [pair_capacity]
};

struct QueryArgs {
    DevModel A, B;
    // batched queries over several fixed models: pose i is tested against
    // Btab[pose_obj[i]] (pose_obj == nullptr: every pose against B)
    const DevModel *Btab;
    const uint32_t *pose_obj;
    uint32_t n_obj;
    const float *poses;
    uint32_t n_poses;
    int mode;
    uint8_t *hit;
    float *dist;
    uint8_t *status;
    uint32_t pair_cap;
    uint32_t no_split;  // never donate work; exhausting the LDS stack then fails the pose
    uint32_t max_pop;   // entries one node step may pop (1..8)
    uint32_t pop_reserve;  // multi-entry steps must leave room for the rest of a descent
    uint32_t donate_min_steps;  // a unit feeds waiting waves only after this many steps
    uint32_t max_helpers;       // waves (the lowest block indices) that stay to take items once the poses are gone
    uint32_t donate_period;     // node steps between two looks at the item queue
    uint32_t donate_keep;       // entries a donor keeps at least (0 = half of its stack)
    uint32_t donate_min_top;    // a unit feeds waiting waves only with at least this many entries
    uint32_t max_donate;        // entries one look at the item queue may hand over
    uint32_t prio_steps;        // a unit's issue priority rises by one every this many steps (0: never)
    unsigned long long wait_limit;  // 100 MHz ticks a waiting wave waits for an item before it gives up
    Workspace ws;
};

// Bytes of one wave's traversal state for a BV type, a mode and limits.
size_t wave_state_bytes(uint32_t bv, int mode, const StackLimits &lim);
// default limits for a BV type, a mode and the models' largest branching factor
StackLimits default_limits(uint32_t bv, int mode, uint32_t branching);
uint32_t item_words(uint32_t bv);

// Enqueue the whole query on `stream`: init, the traversal, and the finalize
// (distances, or count / scan / scatter / sort of pair lists).
hipError_t launch_query(const QueryArgs &q, const StackLimits &lim, hipStream_t stream, uint32_t *pair_out,
                        uint32_t *pair_offsets);

hipError_t launch_decode_all(const DevModel &m, float *out, hipStream_t stream);

// The allocation-free query entry point's workspace: a fixed device array of
// this many bytes per GPU (held until the process ends), shared by every
// such call on that GPU.
constexpr size_t kStaticWorkspaceBytes = 32ull << 20;
constexpr int kMaxDevices = 64;
// Device address of the current device's array (looked up once per device).
hipError_t static_workspace(void **out);

}  // namespace cbvh
