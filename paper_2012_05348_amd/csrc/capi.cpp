// The C ABI of include/cbvh.h: argument validation, model lifetime, device
// views of uploaded models, workspace carving and kernel dispatch.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <new>
#include <string>
#include <vector>

#include "../../include/cbvh.h"
#include "format.h"
#include "kernels.h"
#include "model.h"

// A set of fixed models for batched queries: their device views, copied to
// a caller-owned device table.
struct cbvh_obstacles {
    uint32_t n, bv, bits;
    const cbvh::DevModel *dev_table;
    std::vector<cbvh::DevModel> host;
};

namespace {

thread_local std::string g_err;

cbvh_status fail(cbvh_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

cbvh_status fail_hip(hipError_t e, const char *what)
{
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return CBVH_E_DEVICE;
}

std::atomic<uint32_t> g_limit_entries{0}, g_limit_records{0};
// fewest item-queue slots the allocation-free entry point accepts
constexpr uint64_t kStaticMinItems = 65536;
// how long a waiting wave waits for a work item before it gives up and the
// query's poses are flagged incomplete: 10 s of the 100 MHz device clock
constexpr uint64_t kDefaultWaitTicks = 1000000000ull;
std::atomic<uint64_t> g_wait_ticks{kDefaultWaitTicks};

inline uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }
inline bool aligned(const void *p, uintptr_t a) { return ((uintptr_t)p % a) == 0; }

cbvh::DevModel dev_view(const cbvh_model *m, const void *dev)
{
    const uint8_t *b = (const uint8_t *)dev;
    const cbvh::BlobHeader &h = m->hdr;
    cbvh::DevModel d;
    d.topo = (const uint32_t *)(b + h.off_topo);
    d.codes = b + h.off_codes;
    d.absb = (const float *)(b + h.off_abs);
    d.tris = (const float *)(b + h.off_tris);
    d.perm = (const uint32_t *)(b + h.off_perm);
    d.treelets = (const uint32_t *)(b + h.off_treelets);
    d.n_nodes = h.n_nodes;
    d.n_tris = h.n_tris;
    d.n_treelets = h.n_treelets;
    d.stride = h.code_stride;
    d.bits = h.bits;
    d.K = h.K;
    d.bv = h.bv;
    d.leaf_size = h.leaf_size;
    d.depth = h.depth;
    d.branching = h.branching;
    d.max_abs = h.max_abs_coord;
    return d;
}

cbvh::StackLimits current_limits(uint32_t bv, int mode, uint32_t branching)
{
    cbvh::StackLimits l = cbvh::default_limits(bv, mode, branching);
    uint32_t e = g_limit_entries.load(), r = g_limit_records.load();
    if (e) l.entries = e;
    if (r) l.records = r;
    return l;
}

// workspace carving: [header | item queue | per-pose answers | pair buffers]
struct WsPlan {
    uint64_t hdr, wave_ctr, items, ready, hitw, fix, best32, best64, pair_raw, pair_cnt, pair_cursor, pair_keys, total;
    uint32_t item_cap, item_words, fix_cap;
};

WsPlan plan_workspace(uint32_t bv, int mode, uint32_t n, uint32_t pair_cap, uint64_t item_cap_max = 1ull << 24)
{
    WsPlan p;
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t r = o;
        o = align_up(o + bytes, 256);
        return r;
    };
    p.item_words = cbvh::item_words(bv);
    // donated work items (slots are not reused within a query): four per
    // pose plus slack; a donation that finds the queue full is not made
    uint64_t cap = 4ull * n + 262144ull;
    if (cap > item_cap_max) cap = item_cap_max;
    p.item_cap = (uint32_t)cap;
    bool dist = mode == cbvh::MODE_DIST, pairs = mode == cbvh::MODE_PAIRS;
    p.hdr = take(sizeof(cbvh::WsHeader));
    p.wave_ctr = take(8ull * cbvh::C_NUM * cbvh::kMaxWaves);
    p.items = take((uint64_t)p.item_cap * p.item_words * 4ull);
    p.ready = take(4ull * p.item_cap);
    p.hitw = take(mode == cbvh::MODE_BOOL ? 4ull * n : 0);
    // leaf pairs for the FP64 stage: undecided intersections are rare;
    // distance candidates (within 2 e of a running minimum) number about a
    // hundred per pose on near-contact workloads
    uint64_t fcap = dist ? 256ull * n + (1ull << 20) : n + 65536ull;
    if (fcap > (1ull << 26)) fcap = 1ull << 26;
    p.fix_cap = (uint32_t)fcap;
    p.fix = take(16ull * p.fix_cap);
    p.best32 = take(dist ? 4ull * n : 0);
    p.best64 = take(dist ? 8ull * n : 0);
    p.pair_raw = take(pairs ? 16ull * pair_cap : 0);
    p.pair_cnt = take(pairs ? 4ull * n : 0);
    p.pair_cursor = take(pairs ? 4ull * n : 0);
    p.pair_keys = take(pairs ? 8ull * pair_cap : 0);
    p.total = o;
    return p;
}

cbvh_status check_pair(const cbvh_model *a, const void *a_dev, const cbvh_model *b, const void *b_dev)
{
    if (!a || !b) return fail(CBVH_E_INVALID, "model is NULL");
    if (!a_dev || !b_dev) return fail(CBVH_E_INVALID, "device model pointer is NULL");
    if (!aligned(a_dev, 256) || !aligned(b_dev, 256)) return fail(CBVH_E_INVALID, "device model not 256-byte aligned");
    if (a->hdr.bv != b->hdr.bv) return fail(CBVH_E_UNSUPPORTED, "models have different BV types");
    if (a->hdr.bits != b->hdr.bits) return fail(CBVH_E_UNSUPPORTED, "models have different code widths");
    return CBVH_OK;
}

cbvh_status run_query(const cbvh_model *a, const void *a_dev, const cbvh_model *b, const void *b_dev,
                      const float *poses, uint32_t n, int mode, uint32_t flags, uint8_t *hit, float *dist,
                      uint32_t *pairs, uint32_t pair_cap, uint32_t *pair_offsets, uint8_t *status, void *ws,
                      size_t ws_bytes, void *stream, const cbvh_obstacles *obs = nullptr,
                      const uint32_t *pose_obj = nullptr, uint64_t item_cap_max = 1ull << 24)
{
    cbvh_status st;
    if (obs) {
        if (!a || !a_dev) return fail(CBVH_E_INVALID, "model is NULL");
        if (!aligned(a_dev, 256)) return fail(CBVH_E_INVALID, "device model not 256-byte aligned");
        if (a->hdr.bv != obs->bv) return fail(CBVH_E_UNSUPPORTED, "models have different BV types");
        if (a->hdr.bits != obs->bits) return fail(CBVH_E_UNSUPPORTED, "models have different code widths");
        if (n && !pose_obj) return fail(CBVH_E_INVALID, "pose_obstacle is NULL");
        if (!aligned(pose_obj, 4)) return fail(CBVH_E_INVALID, "pose_obstacle not 4-byte aligned");
    } else {
        st = check_pair(a, a_dev, b, b_dev);
        if (st != CBVH_OK) return st;
    }
    if (n == 0) return CBVH_OK;
    if (!poses || !status) return fail(CBVH_E_INVALID, "poses or pose_status is NULL");
    if (mode == cbvh::MODE_DIST ? !dist : !hit) return fail(CBVH_E_INVALID, "output array is NULL");
    if (!aligned(poses, 4)) return fail(CBVH_E_INVALID, "poses not 4-byte aligned");
    if (mode == cbvh::MODE_PAIRS) {
        if (!pairs || !pair_offsets) return fail(CBVH_E_INVALID, "pairs or pair_offsets is NULL");
        if (pair_cap == 0) return fail(CBVH_E_INVALID, "pair_capacity is 0");
        if (pair_cap > (1u << 30)) return fail(CBVH_E_INVALID, "pair_capacity too large");
    }
    if (n > (1u << 30)) return fail(CBVH_E_INVALID, "too many poses");
    if (!ws) return fail(CBVH_E_INVALID, "workspace is NULL");
    if (!aligned(ws, 256)) return fail(CBVH_E_INVALID, "workspace not 256-byte aligned");
    WsPlan plan = plan_workspace(a->hdr.bv, mode, n, pair_cap, item_cap_max);
    if (ws_bytes < plan.total) return fail(CBVH_E_CAPACITY, "workspace too small");
    uint8_t *w = (uint8_t *)ws;
    cbvh::QueryArgs q;
    memset(&q, 0, sizeof q);
    q.A = dev_view(a, a_dev);
    if (obs) {
        q.B = obs->host[0];
        // launch decisions that depend on the fixed model use the set's largest
        // depth and branching factor (each unit loads its own model's view)
        for (const cbvh::DevModel &d : obs->host) {
            q.B.depth = d.depth > q.B.depth ? d.depth : q.B.depth;
            q.B.branching = d.branching > q.B.branching ? d.branching : q.B.branching;
        }
        q.Btab = obs->dev_table;
        q.pose_obj = pose_obj;
        q.n_obj = obs->n;
    } else {
        q.B = dev_view(b, b_dev);
    }
    q.poses = poses;
    q.n_poses = n;
    q.mode = mode;
    q.hit = hit;
    q.dist = dist;
    q.status = status;
    q.pair_cap = pair_cap;
    q.no_split = (flags & CBVH_NO_SPLIT) ? 1u : 0u;
    q.wait_limit = g_wait_ticks.load();
    q.ws.hdr = (cbvh::WsHeader *)(w + plan.hdr);
    q.ws.wave_ctr = (unsigned long long *)(w + plan.wave_ctr);
    q.ws.items = (uint32_t *)(w + plan.items);
    q.ws.ready = (uint32_t *)(w + plan.ready);
    q.ws.item_cap = plan.item_cap;
    q.ws.item_words = plan.item_words;
    q.ws.hitw = (uint32_t *)(w + plan.hitw);
    q.ws.fix = (uint4 *)(w + plan.fix);
    q.ws.fix_cap = plan.fix_cap;
    q.ws.best32 = (unsigned int *)(w + plan.best32);
    q.ws.best64 = (unsigned long long *)(w + plan.best64);
    q.ws.pair_raw = (uint4 *)(w + plan.pair_raw);
    q.ws.pair_cnt = (uint32_t *)(w + plan.pair_cnt);
    q.ws.pair_cursor = (uint32_t *)(w + plan.pair_cursor);
    q.ws.pair_keys = (unsigned long long *)(w + plan.pair_keys);
    cbvh::StackLimits lim = current_limits(a->hdr.bv, mode, q.A.branching > q.B.branching ? q.A.branching : q.B.branching);
    hipError_t e = cbvh::launch_query(q, lim, (hipStream_t)stream, pairs, pair_offsets);
    if (e != hipSuccess) return fail_hip(e, "kernel launch");
    return CBVH_OK;
}

}  // namespace

extern "C" {

cbvh_status cbvh_build(const float *V, uint32_t nv, const uint32_t *T, uint32_t nt, const cbvh_build_params *params,
                       cbvh_model **out)
{
    try {
        if (!out) return fail(CBVH_E_INVALID, "out is NULL");
        *out = nullptr;
        if (!V || !T || !params) return fail(CBVH_E_INVALID, "V, T or params is NULL");
        if (params->size != sizeof(cbvh_build_params)) return fail(CBVH_E_INVALID, "params.size mismatch");
        if (nt == 0 || nt > cbvh::kIndexMask) return fail(CBVH_E_INVALID, "triangle count out of range");
        if (nv == 0) return fail(CBVH_E_INVALID, "no vertices");
        if (params->bv != CBVH_AABB && params->bv != CBVH_DOP18 && params->bv != CBVH_OBB)
            return fail(CBVH_E_INVALID, "bad bv");
        if (params->bv == CBVH_OBB && params->bits == CBVH_BITS_FP16)
            return fail(CBVH_E_INVALID, "OBB models take bits 0, 8 or 16");
        if (!(params->branching == 2 || params->branching == 4 || params->branching == 8))
            return fail(CBVH_E_INVALID, "branching must be 2, 4 or 8");
        if (params->leaf_size < 1 || params->leaf_size > cbvh::kMaxLeaf) return fail(CBVH_E_INVALID, "leaf_size must be 1..8");
        if (!(params->bits == 0 || params->bits == 8 || params->bits == 16 || params->bits == CBVH_BITS_FP16))
            return fail(CBVH_E_INVALID, "bits must be 0, 8, 16 or CBVH_BITS_FP16");
        uint32_t tb = params->treelet_bytes ? params->treelet_bytes : 8192u;
        if (tb < 256) return fail(CBVH_E_INVALID, "treelet_bytes must be 0 or >= 256");
        cbvh::BuildParams p{params->bv, params->branching, params->leaf_size, params->bits, tb};
        cbvh_model *m = new cbvh_model();
        std::string msg = cbvh::build_model(V, nv, T, nt, p, m);
        if (!msg.empty()) {
            delete m;
            return fail(CBVH_E_INVALID, msg);
        }
        *out = m;
        return CBVH_OK;
    } catch (const std::bad_alloc &) {
        return fail(CBVH_E_NOMEM, "out of host memory");
    } catch (...) {
        return fail(CBVH_E_INVALID, "unexpected error in build");
    }
}

void cbvh_free(cbvh_model *m) { delete m; }

cbvh_status cbvh_blob(const cbvh_model *m, const void **bytes, size_t *n)
{
    if (!m || !bytes || !n) return fail(CBVH_E_INVALID, "NULL argument");
    *bytes = m->blob.data();
    *n = m->blob.size();
    return CBVH_OK;
}

cbvh_status cbvh_load(const void *bytes, size_t n, cbvh_model **out)
{
    try {
        if (!out) return fail(CBVH_E_INVALID, "out is NULL");
        *out = nullptr;
        if (!bytes) return fail(CBVH_E_INVALID, "bytes is NULL");
        cbvh::BlobHeader h;
        uint32_t ni = 0, nl = 0;
        std::string msg = cbvh::validate_blob((const uint8_t *)bytes, n, &h, &ni, &nl);
        if (!msg.empty()) return fail(CBVH_E_FORMAT, msg);
        cbvh_model *m = new cbvh_model();
        m->blob.assign((const uint8_t *)bytes, (const uint8_t *)bytes + n);
        m->hdr = h;
        m->n_inner = ni;
        m->n_leaves = nl;
        m->descriptor_bytes = (uint64_t)h.code_stride * h.n_nodes + 8ull * h.K * h.n_abs;
        *out = m;
        return CBVH_OK;
    } catch (const std::bad_alloc &) {
        return fail(CBVH_E_NOMEM, "out of host memory");
    } catch (...) {
        return fail(CBVH_E_FORMAT, "unexpected error in load");
    }
}

cbvh_status cbvh_info(const cbvh_model *m, cbvh_model_info *o)
{
    if (!m || !o) return fail(CBVH_E_INVALID, "NULL argument");
    const cbvh::BlobHeader &h = m->hdr;
    memset(o, 0, sizeof *o);
    o->bv = h.bv;
    o->slabs = h.K;
    o->bits = h.bits;
    o->branching = h.branching;
    o->leaf_size = h.leaf_size;
    o->n_nodes = h.n_nodes;
    o->n_inner = m->n_inner;
    o->n_leaves = m->n_leaves;
    o->n_tris = h.n_tris;
    o->n_abs = h.n_abs;
    o->n_treelets = h.n_treelets;
    o->depth = h.depth;
    o->blob_bytes = m->blob.size();
    o->descriptor_bytes = m->descriptor_bytes;
    o->topology_bytes = 4ull * h.n_nodes;
    o->triangle_bytes = 36ull * h.n_tris;
    return CBVH_OK;
}

size_t cbvh_device_bytes(const cbvh_model *m) { return m ? m->blob.size() : 0; }

cbvh_status cbvh_upload(const cbvh_model *m, void *dev, size_t capacity, void *stream)
{
    if (!m || !dev) return fail(CBVH_E_INVALID, "NULL argument");
    if (!aligned(dev, 256)) return fail(CBVH_E_INVALID, "device buffer not 256-byte aligned");
    if (capacity < m->blob.size()) return fail(CBVH_E_CAPACITY, "device buffer too small");
    hipError_t e = hipMemcpyAsync(dev, m->blob.data(), m->blob.size(), hipMemcpyHostToDevice, (hipStream_t)stream);
    if (e != hipSuccess) return fail_hip(e, "hipMemcpyAsync");
    return CBVH_OK;
}

size_t cbvh_workspace_bytes(const cbvh_model *a, const cbvh_model *b, uint32_t n_poses, uint32_t flags,
                            uint32_t pair_capacity)
{
    if (!a || !b) return 0;
    int mode = (flags & CBVH_PAIRS) ? cbvh::MODE_PAIRS : cbvh::MODE_BOOL;
    size_t x = plan_workspace(a->hdr.bv, mode, n_poses, pair_capacity).total;
    size_t y = plan_workspace(a->hdr.bv, cbvh::MODE_DIST, n_poses, 0).total;
    return x > y ? x : y;
}

cbvh_status cbvh_collide(const cbvh_model *a, const void *a_dev, const cbvh_model *b, const void *b_dev,
                         const float *poses, uint32_t n, uint32_t flags, uint8_t *hit, uint32_t *pairs,
                         uint32_t pair_capacity, uint32_t *pair_offsets, uint8_t *pose_status, void *workspace,
                         size_t workspace_bytes, void *stream)
{
    if ((flags & CBVH_PAIRS) && (flags & CBVH_EARLY_EXIT))
        return fail(CBVH_E_INVALID, "CBVH_PAIRS and CBVH_EARLY_EXIT are exclusive");
    if (flags & ~(CBVH_EARLY_EXIT | CBVH_PAIRS | CBVH_NO_SPLIT)) return fail(CBVH_E_INVALID, "unknown flag");
    int mode = (flags & CBVH_PAIRS) ? cbvh::MODE_PAIRS : cbvh::MODE_BOOL;
    return run_query(a, a_dev, b, b_dev, poses, n, mode, flags, hit, nullptr, pairs, pair_capacity, pair_offsets,
                     pose_status, workspace, workspace_bytes, stream);
}

cbvh_status cbvh_distance(const cbvh_model *a, const void *a_dev, const cbvh_model *b, const void *b_dev,
                          const float *poses, uint32_t n, uint32_t flags, float *dist, uint8_t *pose_status,
                          void *workspace, size_t workspace_bytes, void *stream)
{
    if (flags & ~CBVH_NO_SPLIT) return fail(CBVH_E_INVALID, "unknown flag");
    return run_query(a, a_dev, b, b_dev, poses, n, cbvh::MODE_DIST, flags, nullptr, dist, nullptr, 0, nullptr,
                     pose_status, workspace, workspace_bytes, stream);
}

cbvh_status cbvh_collide_static(const cbvh_model *a, const void *a_dev, const cbvh_model *b, const void *b_dev,
                                const float *poses, uint32_t n, uint32_t flags, uint8_t *hit, uint8_t *pose_status,
                                void *stream)
{
    if (flags & ~(CBVH_EARLY_EXIT | CBVH_NO_SPLIT)) return fail(CBVH_E_INVALID, "unknown or unsupported flag");
    if (n > CBVH_STATIC_MAX_POSES)
        return fail(CBVH_E_CAPACITY, "more than " + std::to_string(CBVH_STATIC_MAX_POSES) +
                                         " poses for the fixed workspace of cbvh_collide_static");
    if (!a || !b) return fail(CBVH_E_INVALID, "model is NULL");
    if (n == 0) return check_pair(a, a_dev, b, b_dev);
    // the item queue takes whatever the fixed array leaves after the rest of
    // the workspace (the donation path refuses items beyond it)
    const WsPlan fixed = plan_workspace(a->hdr.bv, cbvh::MODE_BOOL, n, 0, 0);
    const uint64_t per_item = 4ull * cbvh::item_words(a->hdr.bv) + 4ull, slack = 1024;
    if (fixed.total + slack + per_item * kStaticMinItems > cbvh::kStaticWorkspaceBytes)
        return fail(CBVH_E_CAPACITY, "the fixed workspace of cbvh_collide_static is too small for this batch");
    const uint64_t cap = (cbvh::kStaticWorkspaceBytes - fixed.total - slack) / per_item;
    void *ws = nullptr;
    hipError_t e = cbvh::static_workspace(&ws);
    if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress");
    return run_query(a, a_dev, b, b_dev, poses, n, cbvh::MODE_BOOL, flags, hit, nullptr, nullptr, 0, nullptr,
                     pose_status, ws, cbvh::kStaticWorkspaceBytes, stream, nullptr, nullptr, cap);
}

size_t cbvh_obstacles_device_bytes(uint32_t n) { return (size_t)align_up((uint64_t)n * sizeof(cbvh::DevModel), 256); }

cbvh_status cbvh_obstacles_create(const cbvh_model *const *models, const void *const *devs, uint32_t n, void *table,
                                  size_t capacity, void *stream, cbvh_obstacles **out)
{
    if (!out) return fail(CBVH_E_INVALID, "out is NULL");
    *out = nullptr;
    if (!models || !devs || !table || n == 0) return fail(CBVH_E_INVALID, "NULL argument or no models");
    if (n > (1u << 24)) return fail(CBVH_E_INVALID, "too many models");
    if (!aligned(table, 256)) return fail(CBVH_E_INVALID, "table not 256-byte aligned");
    if (capacity < cbvh_obstacles_device_bytes(n)) return fail(CBVH_E_CAPACITY, "table too small");
    try {
        cbvh_obstacles *o = new cbvh_obstacles();
        o->n = n;
        o->host.reserve(n);
        for (uint32_t i = 0; i < n; i++) {
            if (!models[i] || !devs[i] || !aligned(devs[i], 256)) {
                delete o;
                return fail(CBVH_E_INVALID, "model " + std::to_string(i) + " NULL or device copy not 256-byte aligned");
            }
            if (i == 0) {
                o->bv = models[0]->hdr.bv;
                o->bits = models[0]->hdr.bits;
            } else if (models[i]->hdr.bv != o->bv || models[i]->hdr.bits != o->bits) {
                delete o;
                return fail(CBVH_E_UNSUPPORTED, "models of one set must share BV type and code width");
            }
            o->host.push_back(dev_view(models[i], devs[i]));
        }
        o->dev_table = (const cbvh::DevModel *)table;
        hipError_t e = hipMemcpyAsync(table, o->host.data(), sizeof(cbvh::DevModel) * (size_t)n, hipMemcpyHostToDevice,
                                      (hipStream_t)stream);
        if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
        if (e != hipSuccess) {
            delete o;
            return fail_hip(e, "model table copy");
        }
        *out = o;
        return CBVH_OK;
    } catch (const std::bad_alloc &) {
        return fail(CBVH_E_NOMEM, "out of host memory");
    }
}

void cbvh_obstacles_free(cbvh_obstacles *o) { delete o; }

cbvh_status cbvh_collide_batch(const cbvh_model *a, const void *a_dev, const cbvh_obstacles *obstacles,
                               const float *poses, const uint32_t *pose_obstacle, uint32_t n, uint32_t flags,
                               uint8_t *hit, uint8_t *pose_status, void *workspace, size_t workspace_bytes,
                               void *stream)
{
    if (!obstacles) return fail(CBVH_E_INVALID, "obstacles is NULL");
    if (flags & ~(CBVH_EARLY_EXIT | CBVH_NO_SPLIT)) return fail(CBVH_E_INVALID, "unknown or unsupported flag");
    return run_query(a, a_dev, nullptr, nullptr, poses, n, cbvh::MODE_BOOL, flags, hit, nullptr, nullptr, 0, nullptr,
                     pose_status, workspace, workspace_bytes, stream, obstacles, pose_obstacle);
}

cbvh_status cbvh_distance_batch(const cbvh_model *a, const void *a_dev, const cbvh_obstacles *obstacles,
                                const float *poses, const uint32_t *pose_obstacle, uint32_t n, uint32_t flags,
                                float *dist, uint8_t *pose_status, void *workspace, size_t workspace_bytes,
                                void *stream)
{
    if (!obstacles) return fail(CBVH_E_INVALID, "obstacles is NULL");
    if (flags & ~CBVH_NO_SPLIT) return fail(CBVH_E_INVALID, "unknown flag");
    return run_query(a, a_dev, nullptr, nullptr, poses, n, cbvh::MODE_DIST, flags, nullptr, dist, nullptr, 0, nullptr,
                     pose_status, workspace, workspace_bytes, stream, obstacles, pose_obstacle);
}

cbvh_status cbvh_decode_all(const cbvh_model *m, const void *m_dev, float *out, void *stream)
{
    if (!m || !m_dev || !out) return fail(CBVH_E_INVALID, "NULL argument");
    if (!aligned(m_dev, 256)) return fail(CBVH_E_INVALID, "device model not 256-byte aligned");
    if (!aligned(out, 4)) return fail(CBVH_E_INVALID, "out not 4-byte aligned");
    hipError_t e = cbvh::launch_decode_all(dev_view(m, m_dev), out, (hipStream_t)stream);
    if (e != hipSuccess) return fail_hip(e, "decode launch");
    return CBVH_OK;
}

cbvh_status cbvh_stats(const void *workspace, size_t workspace_bytes, cbvh_stats_t *out, void *stream)
{
    if (!workspace || !out) return fail(CBVH_E_INVALID, "NULL argument");
    const size_t row_bytes = 8ull * cbvh::C_NUM, rows_at = align_up(sizeof(cbvh::WsHeader), 256);
    if (workspace_bytes < rows_at) return fail(CBVH_E_CAPACITY, "workspace too small");
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
    cbvh::WsHeader h;
    e = hipMemcpy(&h, workspace, sizeof h, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail_hip(e, "hipMemcpy");
    memset(out, 0, sizeof *out);
    out->wait_timeouts = h.error;
    const uint32_t nw = h.n_waves;
    if (nw == 0) return CBVH_OK;  // no traversal launch has run on this workspace
    if (nw > cbvh::kMaxWaves || workspace_bytes < rows_at + nw * row_bytes)
        return fail(CBVH_E_CAPACITY, "workspace too small for the launch's counter rows");
    std::vector<unsigned long long> rows((size_t)nw * cbvh::C_NUM);
    e = hipMemcpy(rows.data(), (const char *)workspace + rows_at, rows.size() * 8, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail_hip(e, "hipMemcpy");
    unsigned long long c[cbvh::C_NUM];
    for (int k = 0; k < cbvh::C_NUM; k++) {
        const bool is_min = k == cbvh::C_T_START || k == cbvh::C_T_DRAIN;
        const bool is_max = k == cbvh::C_MAX_ENTRIES || k == cbvh::C_MAX_RECORDS || k == cbvh::C_MAX_POSE_STEPS ||
                            k == cbvh::C_T_END;
        unsigned long long v = is_min ? ~0ull : 0ull;
        for (uint32_t w = 0; w < nw; w++) {
            const unsigned long long x = rows[(size_t)w * cbvh::C_NUM + k];
            v = is_min ? std::min(v, x) : is_max ? std::max(v, x) : v + x;
        }
        c[k] = v;
    }
    out->bv_tests = c[cbvh::C_BV_TESTS];
    out->tri_tests = c[cbvh::C_TRI_TESTS];
    out->tri_fp64 = c[cbvh::C_TRI_FP64];
    out->expansions = c[cbvh::C_EXPANSIONS];
    out->node_bytes = c[cbvh::C_NODE_BYTES];
    out->tri_bytes = c[cbvh::C_TRI_BYTES];
    out->donated_items = c[cbvh::C_DONATED];
    out->max_entries = c[cbvh::C_MAX_ENTRIES];
    out->max_records = c[cbvh::C_MAX_RECORDS];
    out->t_start = c[cbvh::C_T_START];
    out->t_drain = c[cbvh::C_T_DRAIN];
    out->t_end = c[cbvh::C_T_END];
    out->max_pose_steps = c[cbvh::C_MAX_POSE_STEPS];
    out->node_steps = c[cbvh::C_NODE_STEPS];
    out->leaf_steps = c[cbvh::C_LEAF_STEPS];
    out->waves = nw;
    return CBVH_OK;
}

cbvh_status cbvh_set_stack_limits(uint32_t entries, uint32_t records)
{
    if (entries > 16384 || records > 8192) return fail(CBVH_E_INVALID, "limit too large");
    // one expansion of a single pair must always fit: up to 64 new entries and 16 records
    if ((entries && entries < 72) || (records && records < 20)) return fail(CBVH_E_INVALID, "limit too small");
    g_limit_entries.store(entries);
    g_limit_records.store(records);
    return CBVH_OK;
}

cbvh_status cbvh_set_wait_limit(uint64_t ticks)
{
    if (ticks > 100ull * kDefaultWaitTicks) return fail(CBVH_E_INVALID, "wait limit above 1000 s");
    g_wait_ticks.store(ticks ? ticks : kDefaultWaitTicks);
    return CBVH_OK;
}

const char *cbvh_last_error(void) { return g_err.c_str(); }

}  // extern "C"
