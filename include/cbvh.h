/*
 * cbvh.h -- compressed bounding volume hierarchies for collision detection
 * and proximity queries between rigid triangle meshes, on AMD Instinct
 * MI355X (gfx950).
 *
 * The method follows Tan, Weller and Zachmann, "Compressed Bounding Volume
 * Hierarchies for Collision Detection & Proximity Query":
 *   - BV descriptors (axis-aligned boxes or 18-DOPs, Table I) are quantized
 *     to 8- or 16-bit integer codes relative to the decoded parent BV, i.e.
 *     each node is predicted from the chain of BVs above it and the code is
 *     the corrector (abstract; section III.B "predictors based on the delta
 *     to the parent nodes"; conclusion);
 *   - the BVH is clustered into treelets, contiguous groups of sibling
 *     groups whose top group stores absolute bounds, so any node can be
 *     decoded from its treelet without the whole ancestor chain (abstract,
 *     section III.B "cluster BVHs into a smaller parts");
 *   - two BVHs are traversed simultaneously (Algorithm 1) for a collision
 *     answer per pose, all colliding triangle pairs, or the minimum
 *     separation distance (Introduction: collision detection and proximity
 *     query between a sampled configuration and obstacles).
 *
 * Conventions for every function below:
 *   - Functions return cbvh_status and never abort or throw across the ABI;
 *     cbvh_last_error() gives a thread-local message for the last failure.
 *   - Host models (cbvh_model) are owned by the library, immutable after
 *     build/load, and safe to share between threads.
 *   - All device memory is owned by the caller (e.g. torch tensors); the
 *     query functions allocate no device memory of their own.
 *   - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *     Device work is enqueued asynchronously on it; argument and format
 *     errors are reported synchronously, before anything is enqueued.
 *   - A pose is float32 [3][4] row-major [R | t]; a point x of model A is
 *     placed in model B's frame as R x + t.  R should be a rotation.
 *   - Triangle indices in outputs are the caller's input indices.
 */
#ifndef CBVH_H
#define CBVH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CBVH_OK = 0,
    CBVH_E_INVALID = 1,     /* bad argument (NULL pointer, size, parameter, mesh) */
    CBVH_E_NOMEM = 2,       /* host allocation failed */
    CBVH_E_DEVICE = 3,      /* a HIP call failed (message has the HIP error string) */
    CBVH_E_CAPACITY = 4,    /* a caller-provided buffer or workspace is too small */
    CBVH_E_UNSUPPORTED = 5, /* valid but unsupported combination (e.g. models of different BV type) */
    CBVH_E_FORMAT = 6       /* a serialized model failed validation */
} cbvh_status;

/* BV types.  CBVH_OBB (oriented boxes, named among the BV types of the
 * paper's section I and as future work for this layout in section V): an
 * absolute node stores its own frame (origin and three float32 axes from a
 * principal-axis fit of its triangles) and three frame-coordinate intervals;
 * relative nodes keep their parent's frame and code their intervals against
 * the parent's like the fixed slabs of the other types.  Frames change only
 * at absolute nodes (treelet tops; every node when bits == 0).  OBB models
 * take bits 0, 8 or 16. */
typedef enum { CBVH_AABB = 0, CBVH_DOP18 = 1, CBVH_OBB = 2 } cbvh_bv;

/* `bits` value selecting absolute binary16 descriptors, each bound rounded
 * outward (lo down, hi up): the half-precision BVs of section III.A of the
 * paper, a third comparison point beside FP32 and the corrector codes.
 * Needs every |coordinate| < 32768 (18-DOP: < 16384); 4 bytes per slab. */
#define CBVH_BITS_FP16 0x8010u

/* Build parameters.  Table I of the paper lists the descriptor sizes
 * (AABB 6 floats, k-DOP k floats); `bits` selects the quantized width. */
typedef struct {
    uint32_t size;          /* = sizeof(cbvh_build_params) */
    uint32_t bv;            /* CBVH_AABB (3 slabs), CBVH_DOP18 (9 slabs) or CBVH_OBB (3 slabs in a frame) */
    uint32_t branching;     /* children per inner node: 2, 4 or 8 */
    uint32_t leaf_size;     /* triangles per leaf: 1..8 */
    uint32_t bits;          /* 0 = FP32 descriptors (uncompressed), 8 or 16 = quantized codes,
                               CBVH_BITS_FP16 = half-precision descriptors */
    uint32_t treelet_bytes; /* byte budget of one treelet; 0 = default (8192); >= 256 otherwise */
} cbvh_build_params;

typedef struct cbvh_model cbvh_model;

typedef struct {
    uint32_t bv, slabs, bits, branching, leaf_size;
    uint32_t n_nodes, n_inner, n_leaves, n_tris, n_abs, n_treelets, depth;
    uint64_t blob_bytes;       /* whole serialized model (= device bytes) */
    uint64_t descriptor_bytes; /* bytes of BV descriptors: codes + absolute bounds */
    uint64_t topology_bytes;   /* 4 bytes per node */
    uint64_t triangle_bytes;   /* 36 bytes per triangle */
} cbvh_model_info;

/* Build a compressed BVH from a triangle mesh (host only).
 * V: nv x 3 float32 vertex coordinates; T: nt x 3 uint32 vertex indices.
 * Both are borrowed for the duration of the call and copied.  Fails with
 * CBVH_E_INVALID for nt == 0, nt >= 2^27, an index >= nv, or a
 * non-finite / |x| >= 2^60 coordinate.  Topology: median splits, log2(BF)
 * binary rounds per node on the longest axis of the centroid bounds, leaves
 * kept full; identical for every `bv` and `bits` so compressed and
 * uncompressed models share it. */
cbvh_status cbvh_build(const float *V, uint32_t nv, const uint32_t *T, uint32_t nt,
                       const cbvh_build_params *params, cbvh_model **out);

/* Release a host model (NULL is ignored).  Device copies are not affected. */
void cbvh_free(cbvh_model *m);

/* Borrowed view of the serialized model: the exact bytes that cbvh_upload
 * copies to the device.  Valid until cbvh_free(m). */
cbvh_status cbvh_blob(const cbvh_model *m, const void **bytes, size_t *n);

/* Re-create a model from serialized bytes (copied); validates every offset,
 * index and range so that device traversal of the result stays in bounds.
 * CBVH_E_FORMAT on any inconsistency. */
cbvh_status cbvh_load(const void *bytes, size_t n, cbvh_model **out);

cbvh_status cbvh_info(const cbvh_model *m, cbvh_model_info *out);

/* Device bytes needed by cbvh_upload (the blob size). */
size_t cbvh_device_bytes(const cbvh_model *m);

/* Copy the model into caller-owned device memory `dev` (>= cbvh_device_bytes,
 * 256-byte aligned), asynchronously on `stream`.  The host model must stay
 * alive until the copy has completed. */
cbvh_status cbvh_upload(const cbvh_model *m, void *dev, size_t capacity, void *stream);

/* Query flags */
#define CBVH_EARLY_EXIT 0x1u /* collide: stop a pose at its first colliding triangle pair */
#define CBVH_PAIRS 0x2u      /* collide: report every colliding triangle pair */
#define CBVH_NO_SPLIT 0x4u   /* keep every pose in one wavefront: never hand pending work to other wavefronts */

/* Per-pose status bytes written by the queries */
#define CBVH_POSE_OK 0u
#define CBVH_POSE_STACK_OVERFLOW 1u /* traversal state exhausted and nobody to hand it to; results invalid */
#define CBVH_POSE_PAIR_OVERFLOW 2u  /* pair buffer full; this pose's pair list is incomplete */
#define CBVH_POSE_FP64_OVERFLOW 3u  /* workspace buffer of leaf pairs for FP64 re-evaluation full; results invalid */
#define CBVH_POSE_BAD_OBSTACLE 4u   /* batched queries: the pose's obstacle index is out of range; results invalid */
#define CBVH_POSE_INCOMPLETE 5u     /* a wavefront gave up waiting for handed-over work (the wait limit), so work
                                       of this query may have been lost; set on every pose that has no other
                                       failure; results invalid (the query's wait_timeouts counter is 1) */

/* Workspace bytes (device, caller-owned, 256-byte aligned) for a query on
 * models a and b with n poses. */
size_t cbvh_workspace_bytes(const cbvh_model *a, const cbvh_model *b, uint32_t n_poses, uint32_t flags,
                            uint32_t pair_capacity);

/* How a query runs: one launch of persistent wavefronts.  Each takes poses
 * from a queue and traverses one pose at a time.  Once no pose is left, some
 * wavefronts wait for work items: busy wavefronts hand the pending node
 * pairs nearest their roots (with their decoded bounds) to waiting ones, and
 * a pose whose traversal state would overflow LDS hands over all of its
 * pending pairs.  Per-pose answers are merged in device memory, so results
 * do not depend on how the work was split.  Waiting wavefronts leave once no
 * started wavefront can hand over work any more; a wavefront that starts
 * after that (possible when other launches hold the GPU) runs its poses
 * alone.  The workspace holds the queue: calls that share a workspace must
 * not overlap in time; calls on different workspaces may.
 *
 * Collision detection for a batch of poses (Algorithm 1; leaf test is the
 * closed triangle-triangle intersection, touching counts).
 *   a, a_dev: moving model and its uploaded copy; b, b_dev: fixed model.
 *   poses:    device float32 [n][3][4].
 *   hit:      device uint8 [n]: 1 if any triangle pair intersects.
 *   With CBVH_PAIRS: pairs = device uint32 [pair_capacity][3] receives
 *   (pose, triA, triB) sorted by pose, then triA, then triB; pair_offsets =
 *   device uint32 [n+1] receives each pose's start (pair_offsets[n] = number
 *   stored).  CBVH_PAIRS and CBVH_EARLY_EXIT are mutually exclusive.
 *   pose_status: device uint8 [n] (CBVH_POSE_*).
 *   workspace: device, >= cbvh_workspace_bytes(a, b, n, flags, pair_capacity).
 * Models must have the same BV type.  n == 0 is a no-op. */
cbvh_status cbvh_collide(const cbvh_model *a, const void *a_dev, const cbvh_model *b, const void *b_dev,
                         const float *poses, uint32_t n, uint32_t flags, uint8_t *hit, uint32_t *pairs,
                         uint32_t pair_capacity, uint32_t *pair_offsets, uint8_t *pose_status, void *workspace,
                         size_t workspace_bytes, void *stream);

/* Minimum separation distance per pose (proximity query; 0 if the meshes
 * intersect).  dist: device float32 [n].  Leaf distances run in FP32 and
 * every leaf pair whose FP32 distance could be the minimum is re-evaluated
 * in FP64; the result is the FP64 minimum rounded to float32. */
cbvh_status cbvh_distance(const cbvh_model *a, const void *a_dev, const cbvh_model *b, const void *b_dev,
                          const float *poses, uint32_t n, uint32_t flags, float *dist, uint8_t *pose_status,
                          void *workspace, size_t workspace_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): collision
 * booleans as cbvh_collide with CBVH_EARLY_EXIT (flags: CBVH_EARLY_EXIT,
 * CBVH_NO_SPLIT), but with no workspace argument.  The workspace is a fixed
 * device array of 32 MiB inside the library, one per GPU, held until the
 * process ends; this call allocates nothing (no hipMalloc, no library
 * allocation).  n <= CBVH_STATIC_MAX_POSES, else CBVH_E_CAPACITY before
 * anything is enqueued.  Every call on a GPU shares that GPU's array, which
 * keeps the last call's contents (each call clears what must start at zero):
 * calls that overlap in time on one GPU race and must not be made (serialize
 * them, e.g. on one stream).  The caller still passes inputs and outputs. */
#define CBVH_STATIC_MAX_POSES 262144u
cbvh_status cbvh_collide_static(const cbvh_model *a, const void *a_dev, const cbvh_model *b, const void *b_dev,
                                const float *poses, uint32_t n, uint32_t flags, uint8_t *hit, uint8_t *pose_status,
                                void *stream);

/* ---- batched queries: many fixed models ("obstacles") in one launch ----
 *
 * The batched form of the queries above (section I's use case: test
 * sampled configurations of one moving body against many obstacles): each
 * pose names the obstacle it is tested against, and poses for obstacles
 * of very different sizes share one persistent launch and its work queue.
 * Answers are identical to running each obstacle's poses through
 * cbvh_collide / cbvh_distance on their own.
 *
 * An obstacle set records the uploaded models' device views in a
 * caller-owned device table (cbvh_obstacles_device_bytes(n) bytes,
 * 256-byte aligned).  All models of a set must share BV type and code
 * width with each other and with the moving model.  The set is host
 * memory owned by the library; the uploaded models and the table must
 * stay alive and unchanged while the set is used.  The query functions
 * copy nothing from the host, so a stream capture of them into a HIP
 * graph replays correctly. */
typedef struct cbvh_obstacles cbvh_obstacles;

size_t cbvh_obstacles_device_bytes(uint32_t n);

/* Build a set from n models and their uploaded copies (host arrays of
 * length n, borrowed for the call) and copy its table to `table`.
 * Synchronizes `stream`.  CBVH_E_UNSUPPORTED for mixed BV types or code
 * widths; CBVH_E_CAPACITY if `capacity` is too small. */
cbvh_status cbvh_obstacles_create(const cbvh_model *const *models, const void *const *devs, uint32_t n, void *table,
                                  size_t capacity, void *stream, cbvh_obstacles **out);

/* Release a set (NULL is ignored); the table is the caller's. */
void cbvh_obstacles_free(cbvh_obstacles *set);

/* Collision booleans for poses[i] (moving model a) against obstacle
 * pose_obstacle[i] of the set (device uint32 [n]; an index >= the set's
 * size sets CBVH_POSE_BAD_OBSTACLE).  Flags: CBVH_EARLY_EXIT,
 * CBVH_NO_SPLIT.  The workspace is sized by cbvh_workspace_bytes(a, a, n,
 * flags, 0); other arguments as for cbvh_collide. */
cbvh_status cbvh_collide_batch(const cbvh_model *a, const void *a_dev, const cbvh_obstacles *obstacles,
                               const float *poses, const uint32_t *pose_obstacle, uint32_t n, uint32_t flags,
                               uint8_t *hit, uint8_t *pose_status, void *workspace, size_t workspace_bytes,
                               void *stream);

/* Minimum separation distance per pose against its obstacle; as
 * cbvh_distance otherwise (workspace: cbvh_workspace_bytes(a, a, n, 0, 0)). */
cbvh_status cbvh_distance_batch(const cbvh_model *a, const void *a_dev, const cbvh_obstacles *obstacles,
                                const float *poses, const uint32_t *pose_obstacle, uint32_t n, uint32_t flags,
                                float *dist, uint8_t *pose_status, void *workspace, size_t workspace_bytes,
                                void *stream);

/* Decode every node's bounds on the device: out = device float32
 * [n_nodes][2*slabs] as (lo, hi) per slab; OBB models: [n_nodes][20], each
 * node's whole descriptor (lo0 hi0 lo1 hi1 lo2 hi2, 0, eps, origin, three
 * axes).  Parity tool for the decoder. */
cbvh_status cbvh_decode_all(const cbvh_model *m, const void *m_dev, float *out, void *stream);

/* Counters of the last query that used this workspace.  Synchronizes
 * `stream` and copies them to the host. */
typedef struct {
    uint64_t bv_tests;       /* BV-pair overlap / lower-bound evaluations (Algorithm 1 "intersect") */
    uint64_t tri_tests;      /* triangle-pair tests (FP32) */
    uint64_t tri_fp64;       /* triangle pairs handed to the FP64 stage (undecided in FP32, or distance candidates) */
    uint64_t expansions;     /* node-pair expansions (children fetched and decoded) */
    uint64_t node_bytes;     /* descriptor + topology bytes the expansions fetched */
    uint64_t tri_bytes;      /* triangle bytes the leaf tests fetched */
    uint64_t donated_items;  /* pending node/leaf pairs handed from a busy wavefront to waiting ones */
    uint64_t max_entries;    /* deepest traversal stack seen (entries) */
    uint64_t max_records;    /* most decoded-BV records live at once */
    uint64_t t_start;        /* device wall clock (100 MHz ticks) when the first wave took a pose */
    uint64_t t_drain;        /* ... when a wave first found the pose queue empty */
    uint64_t t_end;          /* ... when the last wave exited */
    uint64_t max_pose_steps; /* most traversal steps (node + leaf) one work unit needed */
    uint64_t wait_timeouts;  /* 1 if a wavefront gave up waiting for work (never expected; every pose is then
                                CBVH_POSE_INCOMPLETE unless flagged otherwise) */
    uint64_t node_steps;     /* node steps: one frame of children decoded and tested (up to 64 records) */
    uint64_t leaf_steps;     /* leaf steps: up to 64 triangle pairs tested */
    uint64_t waves;          /* wavefronts of the traversal launch (resident at once when the GPU is idle) */
} cbvh_stats_t;

cbvh_status cbvh_stats(const void *workspace, size_t workspace_bytes, cbvh_stats_t *out, void *stream);

/* Test hook: cap the per-wavefront (LDS) traversal state at `entries`
 * pending node pairs (0 or >= 72) and `records` decoded BVs (0 or >= 20);
 * 0 restores the defaults.  Lets tests force the donation path from the
 * host.  Affects subsequent queries of this process. */
cbvh_status cbvh_set_stack_limits(uint32_t entries, uint32_t records);

/* How long a wavefront waiting for handed-over work waits before it gives
 * up, in ticks of the 100 MHz device clock (0 restores the default, 10 s;
 * at most 1000 s).  A query in which any wavefront gave up flags its poses
 * CBVH_POSE_INCOMPLETE; every kernel still exits.  Waiting normally ends
 * within microseconds; the limit guards against a stalled device, and a
 * tiny value lets tests force the incomplete path from the host.  Affects
 * subsequent queries of this process. */
cbvh_status cbvh_set_wait_limit(uint64_t ticks);

/* Thread-local message describing the last failure (never NULL). */
const char *cbvh_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CBVH_H */
