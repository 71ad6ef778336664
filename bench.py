"""Benchmark: collision queries on the scaled workload (two 100k-triangle noisy
tori, 18-DOP BVHs, branching 8, leaf size 4, 16-bit predictor-corrector codes,
16,384 seeded rigid poses, boolean answers with early exit) on one GPU.

One step = one cbvh_collide call over the whole pose batch (per-pose setup,
traversal, leaf tests, outputs).  Inputs are resident in HBM before timing.
The K timed steps are spread over --streams HIP streams (8 by default), each
with its own workspace and outputs, so that several batches are in flight:
the headline value is that whole-job rate; the same K steps one at a time
are reported beside it ("sequential"), and every stream's answers must
equal the one-at-a-time run's.  Prints one JSON line.  The uncompressed (FP32 descriptor) twin, the tiny
pair-list workload and the proximity (distance) workload are timed after the
main measurement and reported as extra fields.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
# HIP maps streams onto hardware queues (4 per process by default, one of
# them the null stream's) and runs the launches of streams that share a
# queue one after the other; the pipelined legs below keep up to 8 launches
# in flight, each stream on a queue of its own.  Set before HIP starts.
if int(os.environ.get("GPU_MAX_HW_QUEUES") or 0) < 16:
    os.environ["GPU_MAX_HW_QUEUES"] = "16"

import numpy as np  # noqa: E402

METRIC = "poses/sec + BV-pair tests/sec (compressed vs uncompressed BVH); p99 latency"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ["paper_2012_05348_amd/csrc/traverse.hip", "paper_2012_05348_amd/csrc/geom.h",
                  "paper_2012_05348_amd/csrc/format.h", "paper_2012_05348_amd/csrc/kernels.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_collide_dop18_16bit_torus100k.json")
COUNTERS_FILE = os.path.join(ROOT, "profiles", "counters_collide_dop18_16bit_torus100k.json")
# VALU issue capacity: one wave64 FP32 VALU instruction per 4 cycles per SIMD, 1,024 SIMDs at 2.4 GHz
VALU_ISSUE_PEAK = 1024 * 2.4e9 / 4


def kernel_hash():
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _models(cb, w, bits, dev, bv=None):
    (va, ta), (vb, tb) = w.meshes()
    if bv is None:
        bv = cb.AABB if w.bv == "aabb" else cb.DOP18
    ma = cb.Model.build(va, ta, bv=bv, branching=w.branching, leaf_size=w.leaf_size, bits=bits).to(dev)
    mb = cb.Model.build(vb, tb, bv=bv, branching=w.branching, leaf_size=w.leaf_size, bits=bits).to(dev)
    return ma, mb


T0 = time.perf_counter()


def progress(msg):
    print(f"[bench {time.perf_counter() - T0:7.1f}s] {msg}", file=sys.stderr, flush=True)


def time_steps(fn, steps, warmup):
    """W untimed steps, then K steps between synchronizations; per-step events
    on the launching (current) stream give the per-call device time."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dev_ms = [a.elapsed_time(b) for a, b in evs]
    return wall, dev_ms


# launch knobs of the pipelined collision legs: with 8 launches in flight
# the other launches fill a launch's tail, so a few helper waves for the whole
# GPU beat one per CU (8 streams: 0.168-0.177 ms per step with 8-64 helpers,
# 0.21-0.22 with 256, 0.34 with 512), and each launch taking half of a CU's
# wave slots lets two run side by side (32 helpers: 0.151-0.153 ms per step
# with 6 waves per CU, 0.163-0.164 with 8 or 10, 0.173 with all 12)
PIPE_COLLIDE_CFG = {"max_helpers": 32, "waves_per_cu": 6}
# and of the pipelined distance leg: one helper per CU (the four of a lone
# distance launch hold slots the other launches need) and 6 of a CU's 10
# wave slots per launch (4 streams: 3.73 ms per batch, against 3.83 with 8
# waves per CU and 3.94 with 10 on 2 streams)
PIPE_DIST_CFG = {"helpers_per_cu": 1, "waves_per_cu": 6}
_STREAMS = []


def pipe_streams(n):
    """The first n of one pool of streams made once per process (new streams
    beyond the hardware queues would share a queue with an earlier one)."""
    import torch
    while len(_STREAMS) < n:
        _STREAMS.append(torch.cuda.Stream())
    return _STREAMS[:n]


def time_pipelined(fns, steps, warmup, cfg=None):
    """K calls spread round-robin over S HIP streams, one per entry of `fns`
    (each with its own workspace and outputs), after W untimed calls: the
    wall clock between synchronizations.  Each call still covers the whole
    batch; several batches are in flight at once, so one launch's tail (its
    last long poses) overlaps the next launches' bulk.  cfg: launch knobs
    (autotune.launch_env) for these calls."""
    import torch
    from paper_2012_05348_amd import autotune
    streams = pipe_streams(len(fns))
    for s_ in streams:
        s_.wait_stream(torch.cuda.current_stream())

    def call(i):
        with torch.cuda.stream(streams[i % len(fns)]):
            fns[i % len(fns)]()

    with autotune.launch_env(cfg):
        # (every stream runs at least one untimed call: a stream's first
        # launch also sets up its hardware queue)
        for i in range(max(warmup, len(fns))):
            call(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            call(i)
        torch.cuda.synchronize()
        return time.perf_counter() - t0


def traversal_kernel_ms(cb, step, ws, calls):
    """Duration of the traversal kernel alone, measured on the device: each
    call's workspace records the device wall clock (100 MHz) when its first
    wave started and when its last wave exited."""
    import torch
    out = []
    for _ in range(calls):
        step()
        s = cb.cbvh_stats(ws)
        out.append((s["t_end"] - s["t_start"]) / 1e5)
    torch.cuda.synchronize()
    return out


def run_collide(cb, w, bits, dev, steps, warmup, flags, pair_capacity=0, bv=None, pipeline=0):
    import torch
    ma, mb = _models(cb, w, bits, dev, bv)
    P = torch.from_numpy(w.raw_poses()).to(dev)
    n = P.shape[0]
    ws = cb.workspace(ma, mb, n, flags, pair_capacity, dev)
    hit = torch.empty(n, dtype=torch.uint8, device=dev)
    st = torch.empty(n, dtype=torch.uint8, device=dev)
    pairs = offs = None
    if flags & cb.PAIRS:
        pairs = torch.empty((pair_capacity, 3), dtype=torch.int32, device=dev)
        offs = torch.empty(n + 1, dtype=torch.int32, device=dev)

    def step():
        cb.cbvh_collide(ma.handle, ma.dev, mb.handle, mb.dev, P, n, flags, hit, pairs, pair_capacity, offs, st, ws.buf)

    progress(f"collide {w.name.split(':')[0]} bits={bits} n={n}: warmup")
    wall, dev_ms = time_steps(step, steps, warmup)
    stats = cb.cbvh_stats(ws.buf)
    status_ok = bool((st == 0).all().item())
    progress(f"  {steps} steps, {np.mean(dev_ms):.3f} ms/call, stats {stats}")
    kern_ms = traversal_kernel_ms(cb, step, ws.buf, min(steps, 10))
    info = ma.info()
    pipe = None
    if pipeline:
        # the same batch on `pipeline` streams at once; every stream's answers
        # must equal the one-at-a-time run's
        sets = [(cb.workspace(ma, mb, n, flags, pair_capacity, dev), torch.empty(n, dtype=torch.uint8, device=dev),
                 torch.empty(n, dtype=torch.uint8, device=dev)) for _ in range(pipeline)]
        fns = [lambda s_=s_: cb.cbvh_collide(ma.handle, ma.dev, mb.handle, mb.dev, P, n, flags, s_[1], None, 0, None,
                                             s_[2], s_[0].buf) for s_ in sets]
        progress(f"  pipelined: {pipeline} streams")
        pwall = time_pipelined(fns, steps, warmup, cfg=PIPE_COLLIDE_CFG)
        pipe = {"streams": pipeline, **PIPE_COLLIDE_CFG, "wall": pwall, "poses_per_sec": n * steps / pwall,
                "ms_per_step": pwall / steps * 1e3,
                "hits_equal": all(bool(torch.equal(h_, hit)) for _, h_, _ in sets),
                "status_ok": all(bool((st_ == 0).all().item()) for _, _, st_ in sets)}
        progress(f"  pipelined: {pipe['ms_per_step']:.3f} ms/step, answers equal {pipe['hits_equal']}")
    return dict(n=n, wall=wall, dev_ms=dev_ms, stats=stats, ok=status_ok, hits=int(hit.sum().item()),
                hit=hit.cpu().numpy(), pipe=pipe,
                info=info, descriptor_bytes=info["descriptor_bytes"] + mb.info()["descriptor_bytes"], kern_ms=kern_ms)


def run_distance(cb, w, bits, dev, steps, warmup, flags=0, bv=None, pipeline=0):
    import torch
    ma, mb = _models(cb, w, bits, dev, bv)
    P = torch.from_numpy(w.raw_poses()).to(dev)
    n = P.shape[0]
    ws = cb.workspace(ma, mb, n, 0, 0, dev)
    d = torch.empty(n, dtype=torch.float32, device=dev)
    st = torch.empty(n, dtype=torch.uint8, device=dev)

    def step():
        cb.cbvh_distance(ma.handle, ma.dev, mb.handle, mb.dev, P, n, flags, d, st, ws.buf)

    progress(f"distance {w.name.split(':')[0]} bits={bits} n={n}: warmup")
    wall, dev_ms = time_steps(step, steps, warmup)
    stats = cb.cbvh_stats(ws.buf)
    progress(f"  {steps} steps, {np.mean(dev_ms):.3f} ms/call, stats {stats}")
    kern_ms = traversal_kernel_ms(cb, step, ws.buf, min(steps, 10))
    pipe = None
    if pipeline:
        # several batches in flight (PIPE_DIST_CFG); distances must be
        # bit-identical to the one-at-a-time run's
        sets = [(cb.workspace(ma, mb, n, 0, 0, dev), torch.empty(n, dtype=torch.float32, device=dev),
                 torch.empty(n, dtype=torch.uint8, device=dev)) for _ in range(pipeline)]
        fns = [lambda s_=s_: cb.cbvh_distance(ma.handle, ma.dev, mb.handle, mb.dev, P, n, flags, s_[1], s_[2],
                                              s_[0].buf) for s_ in sets]
        progress(f"  pipelined: {pipeline} streams")
        pwall = time_pipelined(fns, steps, warmup, cfg=PIPE_DIST_CFG)
        pipe = {"streams": pipeline, **PIPE_DIST_CFG, "wall": pwall, "poses_per_sec": n * steps / pwall,
                "ms_per_step": pwall / steps * 1e3,
                "distances_equal": all(bool(torch.equal(d_.view(torch.int32), d.view(torch.int32))) for _, d_, _ in sets),
                "status_ok": all(bool((st_ == 0).all().item()) for _, _, st_ in sets)}
        progress(f"  pipelined: {pipe['ms_per_step']:.3f} ms/step, answers equal {pipe['distances_equal']}")
    return dict(n=n, wall=wall, dev_ms=dev_ms, stats=stats, ok=bool((st == 0).all().item()), dist=d.cpu().numpy(),
                pipe=pipe,
                descriptor_bytes=ma.info()["descriptor_bytes"] + mb.info()["descriptor_bytes"], kern_ms=kern_ms)


def summarize(r, steps):
    ms = float(np.mean(r["dev_ms"]))
    s = r["stats"]
    per_launch_bytes = s["node_bytes"] + s["tri_bytes"]
    return {
        "poses_per_sec": r["n"] * steps / r["wall"],
        "bv_tests_per_sec": s["bv_tests"] / (ms * 1e-3),
        "traversal_kernel_ms": float(np.mean(r["kern_ms"])),
        "ms_per_call_median": float(np.median(r["dev_ms"])),
        "ms_per_call_p99": float(np.percentile(r["dev_ms"], 99)),
        "ms_per_call_min": float(np.min(r["dev_ms"])),
        "bv_tests_per_call": s["bv_tests"],
        "tri_tests_per_call": s["tri_tests"],
        "tri_fp64_per_call": s["tri_fp64"],
        "expansions_per_call": s["expansions"],
        "algorithmic_bytes_per_call": per_launch_bytes,
        "bw_equivalent_GBs": per_launch_bytes / (ms * 1e-3) / 1e9,
        "descriptor_bytes": r["descriptor_bytes"],
        "donated_items": s["donated_items"],
        "max_unit_steps": s["max_pose_steps"],
        "node_steps_per_call": s["node_steps"],
        "leaf_steps_per_call": s["leaf_steps"],
        "status_ok": r["ok"],
        **({"pipelined": {k: v for k, v in r["pipe"].items() if k != "wall"}} if r.get("pipe") else {}),
    }


def run_treelet_sweep(cb, w, dev, sizes, calls=10):
    """The scaled workload's models built with treelets of each size (bytes;
    the largest holds the whole tree): descriptor bytes, absolute treelet
    tops, traversal kernel time, answers against the first size."""
    import torch
    from paper_2012_05348_amd import autotune
    (va, ta), (vb, tb) = w.meshes()
    P = torch.from_numpy(w.raw_poses()).to(dev)
    n = P.shape[0]
    out, ref = [], None
    for tb_ in sizes:
        progress(f"treelet sweep: {tb_} bytes")
        kw = dict(bv=cb.DOP18, branching=w.branching, leaf_size=w.leaf_size, bits=w.bits, treelet_bytes=tb_)
        ma, mb = cb.Model.build(va, ta, **kw).to(dev), cb.Model.build(vb, tb, **kw).to(dev)
        ws = cb.workspace(ma, mb, n, cb.EARLY_EXIT, 0, dev)
        hit = torch.empty(n, dtype=torch.uint8, device=dev)
        st = torch.empty(n, dtype=torch.uint8, device=dev)

        def step():
            cb.cbvh_collide(ma.handle, ma.dev, mb.handle, mb.dev, P, n, cb.EARLY_EXIT, hit, None, 0, None, st, ws.buf)

        traversal_kernel_ms(cb, step, ws.buf, 3)
        k = traversal_kernel_ms(cb, step, ws.buf, calls)
        h = hit.cpu().numpy()
        ref = h if ref is None else ref
        info = ma.info()
        out.append({"treelet_bytes": "whole tree" if tb_ == autotune.WHOLE_TREE else tb_,
                    "treelets": info["n_treelets"], "absolute_nodes": info["n_abs"],
                    "descriptor_bytes": info["descriptor_bytes"], "kernel_ms_median": float(np.median(k)),
                    "hits_equal": bool(np.array_equal(h, ref)), "status_ok": bool((st == 0).all().item())})
    return out


def run_batched(cb, dev, steps, warmup):
    """The batched workload: a 20k-triangle link against 64 obstacles of uneven
    size (1k-200k triangles) in one launch, against the plain kernel run once
    per obstacle (the fallback), and as a replayed HIP graph."""
    import torch
    from synth import configs
    w = configs.BATCHED
    kw = dict(bv=cb.DOP18, branching=w.branching, leaf_size=w.leaf_size, bits=w.bits)
    progress(f"batched: building {w.n_obstacles} obstacle models")
    link_mesh = w.link_mesh()
    obs_meshes = [w.obstacle_mesh(i) for i in range(w.n_obstacles)]
    link = cb.Model.build(*link_mesh, **kw).to(dev)
    obs = [cb.Model.build(*m, **kw).to(dev) for m in obs_meshes]
    oset = cb.Obstacles(obs, dev)
    P, obj = w.raw_poses()
    n = len(P)
    Pd, od = torch.from_numpy(P).to(dev), torch.from_numpy(obj).to(dev)
    ws = cb.workspace(link, link, n, cb.EARLY_EXIT, 0, dev)
    hit = torch.empty(n, dtype=torch.uint8, device=dev)
    st = torch.empty(n, dtype=torch.uint8, device=dev)

    def step():
        cb.cbvh_collide_batch(link.handle, link.dev, oset.handle, Pd, od, n, cb.EARLY_EXIT, hit, st, ws.buf)

    progress(f"batched: {n} poses in {len(w.batches())} batches")
    wall, dev_ms = time_steps(step, steps, warmup)
    stats = cb.cbvh_stats(ws.buf)
    ok = bool((st == 0).all().item())
    hits = hit.clone()
    # eight launches in flight on eight streams
    sets = [(cb.workspace(link, link, n, cb.EARLY_EXIT, 0, dev), torch.empty(n, dtype=torch.uint8, device=dev),
             torch.empty(n, dtype=torch.uint8, device=dev)) for _ in range(8)]
    fns = [lambda s_=s_: cb.cbvh_collide_batch(link.handle, link.dev, oset.handle, Pd, od, n, cb.EARLY_EXIT, s_[1], s_[2],
                                               s_[0].buf) for s_ in sets]
    psteps = 6 * len(sets)  # several rounds over the streams (the first and last run partly alone)
    pwall = time_pipelined(fns, psteps, len(sets), cfg=PIPE_COLLIDE_CFG)
    pipelined = {"streams": len(sets), **PIPE_COLLIDE_CFG, "steps": psteps, "poses_per_sec": n * psteps / pwall,
                 "ms_per_step": pwall / psteps * 1e3,
                 "hits_equal": all(bool(torch.equal(h_, hits)) for _, h_, _ in sets),
                 "status_ok": all(bool((st_ == 0).all().item()) for _, _, st_ in sets)}
    progress(f"  batched pipelined: {pipelined['ms_per_step']:.3f} ms/step")
    # the plain kernel, one launch per obstacle (poses grouped by obstacle)
    groups = []
    for k in range(w.n_obstacles):
        idx = np.nonzero(obj == k)[0]
        if len(idx):
            groups.append((obs[k], torch.from_numpy(P[idx]).to(dev), torch.from_numpy(idx).to(dev),
                           cb.workspace(link, obs[k], len(idx), cb.EARLY_EXIT, 0, dev),
                           torch.empty(len(idx), dtype=torch.uint8, device=dev),
                           torch.empty(len(idx), dtype=torch.uint8, device=dev)))
    hit_plain = torch.empty(n, dtype=torch.uint8, device=dev)

    def plain_step():
        for m, Pk, ik, wsk, hk, sk in groups:
            cb.cbvh_collide(link.handle, link.dev, m.handle, m.dev, Pk, len(Pk), cb.EARLY_EXIT, hk, None, 0, None, sk,
                            wsk.buf)

    pwall, pdev_ms = time_steps(plain_step, steps, warmup)
    for m, Pk, ik, wsk, hk, sk in groups:
        hit_plain[ik] = hk
    torch.cuda.synchronize()
    # the batched query captured once and replayed
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        cb.cbvh_collide_batch(link.handle, link.dev, oset.handle, Pd, od, n, cb.EARLY_EXIT, hit, st, ws.buf, stream=s)
    gwall, gdev_ms = time_steps(g.replay, steps, warmup)
    graph_equal = bool(torch.equal(hit, hits))
    progress(f"  batched {np.mean(dev_ms):.3f} ms, plain x{len(groups)} {np.mean(pdev_ms):.3f} ms, "
             f"graph {np.mean(gdev_ms):.3f} ms")
    # autotuner over branching factor, treelet size (2, 8, 32 KiB and one
    # treelet for the whole tree), waves per CU and waves per workgroup
    # (answers must not change); the pick is stored, then applied: models
    # rebuilt with its build parameters, launches with its launch knobs
    from paper_2012_05348_amd import autotune
    progress("batched: autotune (branching 4/8, treelets 2/8/32 KiB and whole tree, waves per CU, per workgroup)")
    tuned = autotune.tune(link_mesh, obs_meshes, P, obj, bits=w.bits, leaf_size=w.leaf_size, branchings=(4, 8),
                          treelet_bytes=(2048, 8192, 32768, autotune.WHOLE_TREE), waves_per_cu=(0, 8),
                          waves_per_group=(1, 2, 4), steps=5, warmup=2, device=dev)
    applied = None
    if tuned["best"]:
        cache = autotune.save(w.name, tuned["best"])
        cfg = autotune.load(w.name)
        kw_t = dict(bv=cb.DOP18, leaf_size=w.leaf_size, bits=w.bits, **autotune.build_kwargs(cfg))
        link_t = cb.Model.build(*link_mesh, **kw_t).to(dev)
        oset_t = cb.Obstacles([cb.Model.build(*m, **kw_t).to(dev) for m in obs_meshes], dev)
        hit_t = torch.empty(n, dtype=torch.uint8, device=dev)

        def tuned_step():
            cb.cbvh_collide_batch(link_t.handle, link_t.dev, oset_t.handle, Pd, od, n, cb.EARLY_EXIT, hit_t, st, ws.buf)

        with autotune.launch_env(cfg):
            twall, tdev_ms = time_steps(tuned_step, steps, warmup)
        applied = {"config": cfg, "cache": cache, "poses_per_sec": n * steps / twall,
                   "ms_per_call_median": float(np.median(tdev_ms)), "hits_equal": bool(torch.equal(hit_t, hits)),
                   "status_ok": bool((st == 0).all().item())}
        progress(f"  tuned pick {cfg}: {applied['ms_per_call_median']:.3f} ms")
    return {
        "autotune": tuned, "tuned_applied": applied,
        "workload": w.name, "poses": n, "batches": len(w.batches()), "obstacles": w.n_obstacles,
        "obstacle_triangles": int(sum(s_.n_tris for s_ in w.obstacle_specs())),
        "poses_per_sec": n * steps / wall, "ms_per_call_median": float(np.median(dev_ms)),
        "ms_per_call_p99": float(np.percentile(dev_ms, 99)), "bv_tests_per_call": stats["bv_tests"],
        "pipelined": pipelined,
        "status_ok": ok, "hits": int(hits.sum().item()),
        "plain_per_obstacle": {"launches": len(groups), "poses_per_sec": n * steps / pwall,
                               "ms_per_step_median": float(np.median(pdev_ms)),
                               "hits_equal": bool(torch.equal(hit_plain, hits))},
        "graph_replay": {"poses_per_sec": n * steps / gwall, "ms_per_call_median": float(np.median(gdev_ms)),
                         "hits_equal": graph_equal},
    }


def run_serving(cb, dev, n_requests=1500):
    """The serving workload: 32 resident obstacles (1k-200k triangles), requests
    of 1-4096 random-walk poses against a uniform obstacle, 70 % collision and
    30 % distance.  First the saturation rate (every request available at
    once), then Poisson arrivals at 50/80/95 % of it with p50/p99 latency."""
    from paper_2012_05348_amd import serve
    from synth import configs
    w = configs.SERVING
    kw = dict(bv=cb.DOP18, branching=w.branching, leaf_size=w.leaf_size, bits=w.bits)
    # the serving loop's own launch defaults (one wave per workgroup): the
    # batched workload's tuned pick (one launch at a time) made its latencies
    # worse where launches share the GPU, so it is not applied here
    cfg = None
    progress(f"serving: building {w.n_obstacles} resident obstacle models")
    link = cb.Model.build(*w.link_mesh(), **kw).to(dev)
    oset = cb.Obstacles([cb.Model.build(*w.obstacle_mesh(i), **kw).to(dev) for i in range(w.n_obstacles)], dev)
    srv = serve.Server(link, oset, dev, launch_cfg=cfg)
    rng = configs.rng_for(4, 2)
    warm = serve.make_requests(200, np.inf, w.n_obstacles, rng)
    srv.run(warm, realtime=False)
    sat_req = serve.make_requests(n_requests, np.inf, w.n_obstacles, rng)
    sat = srv.run(sat_req, realtime=False)
    rate = sat["requests_per_sec"]
    out = {"obstacles": w.n_obstacles, "max_poses_per_launch": srv.max_poses, "requests": n_requests,
           "saturation": {k: sat[k] for k in ("poses_per_sec", "requests_per_sec", "launches", "retry_launches",
                                              "p50_ms", "p99_ms")}}
    out["saturation"]["status_ok"] = bool((sat["status"] == 0).all())
    out["saturation"]["status_counts"] = np.bincount(sat["status"], minlength=6).tolist()
    # each served request against its plain query run alone (the judge of the batched path)
    progress("serving: every request of the saturation run against its plain query")
    import torch
    equal = True
    for r in range(len(sat_req)):
        sl = slice(sat_req.first[r], sat_req.first[r] + sat_req.count[r])
        Pr = torch.from_numpy(sat_req.poses[sl]).to(dev)
        m = oset.models[int(sat_req.obstacle[r])]
        if sat_req.kind[r] == serve.COLLIDE:
            h, _ = cb.collide(link, m, Pr)
            equal &= bool(np.array_equal(h.cpu().numpy(), sat["hit"][sl]))
        else:
            d, _ = cb.distance(link, m, Pr)
            equal &= bool(np.array_equal(d.cpu().numpy().view(np.uint32), sat["dist"][sl].view(np.uint32)))
    out["saturation"]["answers_equal_plain_queries"] = equal
    progress(f"serving: saturation {sat['poses_per_sec']:.3g} poses/s, {rate:.0f} requests/s")
    for frac in (0.5, 0.8, 0.95):
        req = serve.make_requests(n_requests, frac * rate, w.n_obstacles, rng)
        r = srv.run(req, realtime=True)
        ok = bool((r["status"] == 0).all())
        out[f"load_{int(frac * 100)}"] = {"offered_requests_per_sec": frac * rate, "poses_per_sec": r["poses_per_sec"],
                                          "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"], "launches": r["launches"],
                                          "retry_launches": r["retry_launches"], "status_ok": ok,
                                          "status_counts": np.bincount(r["status"], minlength=6).tolist()}
        progress(f"  load {frac:.0%}: p50 {r['p50_ms']:.2f} ms, p99 {r['p99_ms']:.2f} ms")
    return out


def run_large_obstacle_set(cb, dev, n_obstacles=192, n_poses=32768, calls=9):
    """Descriptor formats on a working set beyond the Infinity Cache: one
    20k-triangle link against n_obstacles separate device copies of a
    200k-triangle 18-DOP obstacle (about 11 MB each with triangles), poses
    spread uniformly over them; kernel time per format, answers compared."""
    import torch
    from synth import meshes, poses
    rng = np.random.default_rng(4242)
    obs_mesh = meshes.torus(*meshes.torus_grid_for(200000), 1.0, 0.3, 0.02, rng)
    link_mesh = meshes.torus(*meshes.torus_grid_for(20000), 1.0, 0.3, 0.02, rng)
    P = poses.compose(poses.uniform_rotations(n_poses, rng), poses.box_translations(n_poses, 1.5, rng))
    obj = rng.integers(0, n_obstacles, n_poses).astype(np.uint32)
    Pd, od = torch.from_numpy(P).to(dev), torch.from_numpy(obj).to(dev)
    out, ref = {"obstacles": n_obstacles, "poses": n_poses}, None
    for bits, key in ((16, "codes16"), (cb.BITS_FP16, "fp16"), (0, "fp32")):
        progress(f"large obstacle set: {n_obstacles} copies, {key}")
        kw = dict(bv=cb.DOP18, branching=8, leaf_size=4, bits=bits)
        link = cb.Model.build(*link_mesh, **kw).to(dev)
        base = cb.Model.build(*obs_mesh, **kw)
        blob = base.blob()
        obs = [cb.Model.load(blob).to(dev) for _ in range(n_obstacles)]
        oset = cb.Obstacles(obs, dev)
        ws = cb.workspace(link, link, n_poses, cb.EARLY_EXIT, 0, dev)
        hit = torch.empty(n_poses, dtype=torch.uint8, device=dev)
        st = torch.empty(n_poses, dtype=torch.uint8, device=dev)

        def step():
            cb.cbvh_collide_batch(link.handle, link.dev, oset.handle, Pd, od, n_poses, cb.EARLY_EXIT, hit, st, ws.buf)

        traversal_kernel_ms(cb, step, ws.buf, 2)
        k = traversal_kernel_ms(cb, step, ws.buf, calls)
        h = hit.cpu().numpy()
        ref = h if ref is None else ref
        out[key] = {"descriptor_bytes_total": base.info()["descriptor_bytes"] * n_obstacles,
                    "kernel_ms_median": float(np.median(k)), "kernel_ms_min": float(np.min(k)),
                    "hits_equal": bool(np.array_equal(h, ref)), "status_ok": bool((st == 0).all().item())}
        del link, obs, oset, ws, base
        torch.cuda.empty_cache()
    return out


def host_cpus():
    """The host CPU as this process sees it: model, nproc, the CPUs it may run
    on, the cgroup's CPU quota, and the thread count the oracle uses (the
    smallest of those and OMP_NUM_THREADS, the per-GPU CPU share where set)."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0))
    quota = None
    try:
        with open("/sys/fs/cgroup/cpu.max") as f:
            q, per = f.read().split()
            if q != "max":
                quota = max(1, int(int(q) / int(per)))
    except (OSError, ValueError):
        pass
    omp = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or None
    threads = min(x for x in (os.cpu_count() or 1, aff, quota, omp) if x)
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cpus": aff, "cgroup_cpus": quota,
            "omp_num_threads": omp, "threads_used": threads}


def time_oracle(run, n, threads, budget_s):
    """Oracle poses/s over a bounded sample: run(k, threads) runs the first k
    poses.  A short probe sizes the sample to about budget_s seconds; fast
    workloads repeat passes over all n poses until budget_s has elapsed (at
    most 512); one thread runs a prefix of about budget_s / 4 seconds."""
    k0 = min(n, 64)
    t0 = time.perf_counter()
    run(k0, threads)
    per_pose = (time.perf_counter() - t0) / k0
    k = int(min(n, max(k0, budget_s / max(per_pose, 1e-9))))
    passes = 0
    t0 = time.perf_counter()
    while True:
        run(k, threads)
        passes += 1
        dt = time.perf_counter() - t0
        if k < n or dt >= budget_s or passes >= 512:
            break
    k1 = int(min(n, max(16, budget_s / 4 / max(per_pose * threads, 1e-9))))
    t1 = time.perf_counter()
    run(k1, 1)
    dt1 = time.perf_counter() - t1
    return {"value": passes * k / dt, "unit": "poses/s", "cores": threads, "kind": "oracle",
            "sample": f"{passes} pass(es) over the first {k} of the {n} poses ({dt:.1f} s)",
            "single_thread": {"value": k1 / dt1, "unit": "poses/s", "sample": f"the first {k1} poses ({dt1:.1f} s)"}}


def cpu_baseline(w, threads, budget_s=10.0):
    """The FP64 oracle (Algorithm 1 over its own binary AABB tree, early exit
    per pose) on the scaled workload's poses, timed on the host."""
    import oracle
    progress("cpu baseline (oracle): scaled")
    (va, ta), (vb, tb) = w.meshes()
    A, B = oracle.Mesh(va, ta), oracle.Mesh(vb, tb)
    P = w.raw_poses()
    r = time_oracle(lambda k, t: oracle.collide_batch(A, B, P[:k], threads=t), len(P), threads, budget_s)
    r["sample"] += "; FP64 Algorithm 1 on the oracle's own binary AABB tree, early exit per pose"
    progress(f"  oracle: {r['value']:.4g} poses/s on {threads} threads, {r['single_thread']['value']:.4g} on one")
    return r


def cpu_baselines_other(threads, budget_s=6.0):
    """The oracle on the tiny (pair lists: full enumeration per pose),
    proximity (branch-and-bound distance) and batched (per-obstacle early-exit
    booleans) workloads, each on the same raw poses as the GPU run."""
    import oracle
    from synth import configs
    out = {}
    w0, w2 = configs.WORKLOADS[0], configs.WORKLOADS[2]
    for key, w, fn in (("tiny_pairs", w0, oracle.pair_count_batch), ("proximity", w2, oracle.distance_batch)):
        progress(f"cpu baseline (oracle): {key}")
        (va, ta), (vb, tb) = w.meshes()
        A, B = oracle.Mesh(va, ta), oracle.Mesh(vb, tb)
        P = w.raw_poses()
        out[key] = time_oracle(lambda k, t: fn(A, B, P[:k], threads=t), len(P), threads, budget_s)
    progress("cpu baseline (oracle): batched")
    wb = configs.BATCHED
    P, obj = wb.raw_poses()
    link = oracle.Mesh(*wb.link_mesh())
    obs = {}

    def run_batched(k, t):
        for o in np.unique(obj[:k]):
            if o not in obs:
                obs[o] = oracle.Mesh(*wb.obstacle_mesh(int(o)))
            idx = np.nonzero(obj[:k] == o)[0]
            oracle.collide_batch(link, obs[o], P[idx], threads=t)

    # oracle trees of the obstacles are built outside the timed passes
    for o in np.unique(obj):
        obs[o] = oracle.Mesh(*wb.obstacle_mesh(int(o)))
    out["batched"] = time_oracle(run_batched, len(P), threads, budget_s)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--streams", type=int, default=8,
                    help="HIP streams the timed steps are spread over (batches in flight at once; 1 = one at a time)")
    ap.add_argument("--no-extra", action="store_true", help="skip the uncompressed twin and the other workloads")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--large-obstacle-set", type=int, default=0, metavar="N",
                    help="also time the descriptor formats on N device copies of a 200k-triangle obstacle")
    ap.add_argument("--proximity-only", action="store_true",
                    help="time only the proximity distance workload (for kernel traces of the distance kernel)")
    ap.add_argument("--proximity-dop18-only", action="store_true",
                    help="time only the proximity workload's meshes as 18-DOP models (BF 8, leaf 4, 16-bit): "
                         "the 18-DOP distance kernel, for its kernel traces and counters")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (HBM counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the query batch is sharded by poses across GPUs with no exchange "
              "beyond gathering outputs; run it with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2012_05348_amd as cb
    from synth import configs

    dev = torch.device("cuda:0")
    if args.proximity_only:
        w2 = configs.WORKLOADS[2]
        pr = run_distance(cb, w2, w2.bits, dev, args.steps, args.warmup)
        print(json.dumps({"workload": w2.name, "steps": args.steps, "warmup": args.warmup,
                          "proximity": summarize(pr, args.steps)}), flush=True)
        return
    if args.proximity_dop18_only:
        w2 = dataclasses.replace(configs.WORKLOADS[2], bv="dop18", branching=8, leaf_size=4, bits=16)
        pr = run_distance(cb, w2, w2.bits, dev, args.steps, args.warmup)
        print(json.dumps({"workload": w2.name + " (as 18-DOP models, BF 8, leaf 4, 16-bit codes)",
                          "steps": args.steps, "warmup": args.warmup, "proximity_dop18": summarize(pr, args.steps)}),
              flush=True)
        return
    w = configs.WORKLOADS[1]
    streams = max(1, args.streams)
    main_r = run_collide(cb, w, w.bits, dev, args.steps, args.warmup, cb.EARLY_EXIT,
                         pipeline=streams if streams > 1 else 0)
    main_s = summarize(main_r, args.steps)
    # the headline: K steps with `streams` batches in flight (one at a time
    # when streams = 1); the one-at-a-time run is reported beside it
    pipe = main_r["pipe"]
    value = pipe["poses_per_sec"] if pipe else main_s["poses_per_sec"]
    ms_per_step = (pipe["wall"] if pipe else main_r["wall"]) / args.steps * 1e3
    # the dominant kernel's average duration, measured live on the device
    kavg_ms = float(np.mean(main_r["kern_ms"]))
    algo_bytes = main_s["algorithmic_bytes_per_call"]
    achieved = algo_bytes / (kavg_ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_hash") == kernel_hash():
            traffic = tr.get("hbm_bytes_per_launch")
    # the secondary ceiling, VALU issue, from the committed SQ counters of the same kernel source
    valu = None
    if os.path.exists(COUNTERS_FILE):
        with open(COUNTERS_FILE) as f:
            ct = json.load(f)
        if ct.get("kernel_hash") == kernel_hash():
            rate = ct["valu_insts_per_dispatch"] / (kavg_ms * 1e-3)
            valu = {"insts_per_launch": ct["valu_insts_per_dispatch"], "achieved_per_s": rate,
                    "peak_per_s": VALU_ISSUE_PEAK, "frac": rate / VALU_ISSUE_PEAK}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "poses/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "scaled collision: noisy torus 100k tri vs noisy torus 100k tri, 18-DOP BF8 leaf 4, "
                        "16-bit predictor-corrector codes, 16384 poses, booleans with early exit",
            "poses": main_r["n"], "bv": "dop18", "branching": 8, "leaf_size": 4, "bits": 16,
            "parallelism": "one wavefront per pose; pending node pairs handed to helper waves; "
                           f"{streams} batches in flight on {streams} HIP streams",
            "streams": streams,
        },
        "sequential": {"poses_per_sec": main_s["poses_per_sec"], "ms_per_step": main_r["wall"] / args.steps * 1e3,
                       "ms_per_call_median": main_s["ms_per_call_median"], "ms_per_call_p99": main_s["ms_per_call_p99"]},
        "answers_equal_across_streams": pipe["hits_equal"] if pipe else True,
        "bv_tests_per_sec": main_s["bv_tests_per_sec"],
        "compressed": main_s,
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic, "kernel": "traverse_kernel<9,16,bool>", "kernel_avg_ms": kavg_ms,
            "call_avg_ms": float(np.mean(main_r["dev_ms"])), "algorithmic_bytes_per_launch": algo_bytes,
            "valu_issue": valu,
            # the same bytes per step over the pipelined step time (several
            # launches overlap, so this is a whole-job rate, not one kernel's)
            "per_step_pipelined": ({"achieved": algo_bytes / (ms_per_step * 1e-3) / 1e9,
                                    "frac": algo_bytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS}
                                   if pipe else None),
        },
    }
    if not args.no_extra:
        unc = run_collide(cb, w, 0, dev, args.steps, args.warmup, cb.EARLY_EXIT, pipeline=streams if streams > 1 else 0)
        out["uncompressed"] = summarize(unc, args.steps)
        out["uncompressed"]["hits_equal"] = bool(np.array_equal(unc["hit"], main_r["hit"]))
        out["compression"] = {
            "descriptor_bytes_compressed": main_s["descriptor_bytes"],
            "descriptor_bytes_fp32": out["uncompressed"]["descriptor_bytes"],
            "ratio": out["uncompressed"]["descriptor_bytes"] / main_s["descriptor_bytes"],
            "bv_test_inflation": main_s["bv_tests_per_call"] / max(1, out["uncompressed"]["bv_tests_per_call"]),
            "speedup_vs_fp32": main_s["poses_per_sec"] / out["uncompressed"]["poses_per_sec"],
        }
        if pipe and unc["pipe"]:
            out["compression"]["speedup_vs_fp32_pipelined"] = pipe["poses_per_sec"] / unc["pipe"]["poses_per_sec"]
        # the paper's half-precision descriptors (section III.A), a third point
        f16 = run_collide(cb, w, cb.BITS_FP16, dev, args.steps, args.warmup, cb.EARLY_EXIT)
        out["fp16"] = summarize(f16, args.steps)
        out["fp16"]["hits_equal"] = bool(np.array_equal(f16["hit"], main_r["hit"]))
        out["compression"]["descriptor_bytes_fp16"] = out["fp16"]["descriptor_bytes"]
        out["compression"]["bv_test_inflation_fp16"] = (out["fp16"]["bv_tests_per_call"] /
                                                        max(1, out["uncompressed"]["bv_tests_per_call"]))
        w0, w2 = configs.WORKLOADS[0], configs.WORKLOADS[2]
        tiny = run_collide(cb, w0, w0.bits, dev, 10, 2, cb.PAIRS, pair_capacity=1 << 20)
        out["tiny_pairs"] = summarize(tiny, 10)
        prox = {}
        for bits, key in ((w2.bits, "proximity"), (0, "proximity_fp32"), (cb.BITS_FP16, "proximity_fp16")):
            k_ = 20 if key == "proximity" else 5
            prox[key] = run_distance(cb, w2, bits, dev, k_, 2, pipeline=4 if key == "proximity" else 0)
            out[key] = summarize(prox[key], k_)
        # oriented boxes in the same layout (the paper's future work): the
        # scaled collision workload and the proximity workload as OBB models
        # with the same trees and code widths
        obb = run_collide(cb, w, w.bits, dev, args.steps, args.warmup, cb.EARLY_EXIT, bv=cb.OBB)
        out["obb"] = summarize(obb, args.steps)
        out["obb"]["hits_equal"] = bool(np.array_equal(obb["hit"], main_r["hit"]))
        pobb = run_distance(cb, w2, w2.bits, dev, 5, 1, bv=cb.OBB)
        out["proximity_obb"] = summarize(pobb, 5)
        out["proximity_obb"]["distances_equal"] = bool(np.array_equal(pobb["dist"].view(np.uint32),
                                                                      prox["proximity"]["dist"].view(np.uint32)))
        from paper_2012_05348_amd import autotune
        out["treelet_sweep_scaled"] = run_treelet_sweep(cb, w, dev, (2048, 8192, 32768, autotune.WHOLE_TREE))
        out["batched"] = run_batched(cb, dev, 10, 2)
        out["serving"] = run_serving(cb, dev)
    if args.large_obstacle_set:
        out["large_obstacle_set"] = run_large_obstacle_set(cb, dev, args.large_obstacle_set)
    if not args.no_cpu:
        host = host_cpus()
        out["cpu_baseline"] = cpu_baseline(w, threads=host["threads_used"])
        out["cpu_baseline"]["host"] = host
        out["cpu_baseline"]["gpu_over_oracle"] = out["value"] / out["cpu_baseline"]["value"]
        if not args.no_extra:
            other = cpu_baselines_other(host["threads_used"])
            gpu = {"tiny_pairs": out["tiny_pairs"]["poses_per_sec"], "proximity": out["proximity"]["poses_per_sec"],
                   "batched": out["batched"]["poses_per_sec"]}
            for k, r in other.items():
                r["gpu_poses_per_sec"] = gpu[k]
                r["gpu_over_oracle"] = gpu[k] / r["value"]
            out["cpu_baseline"]["other_workloads"] = other
    if args.calibrate_copy_mib:
        n = args.calibrate_copy_mib << 20
        src = torch.empty(n, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["calibration_copy_bytes"] = n
    print(json.dumps(out))


if __name__ == "__main__":
    main()
