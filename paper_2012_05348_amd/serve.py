"""Serving loop with continuous batching for collision and distance requests
against resident obstacle models (the motion-planning use case of the
paper's introduction: configurations sampled by a planner are tested
against a fixed set of obstacles as they arrive).

A request is a batch of poses of the moving model against one obstacle,
either a collision query (booleans) or a distance query.  The loop keeps a
few launch slots per query kind, each with its own HIP stream, device
buffers and workspace, sized so that all slots fit a device-memory budget.
Whenever a slot is free it admits every request that has arrived and fits
(one batched launch covers requests for different obstacles), and
completions are polled without blocking, so requests that arrive while
others run are admitted as slots and memory free up, and work of different
requests overlaps on the device.  Results are per pose and do not depend
on what else shares the launch.
"""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

from . import (EARLY_EXIT, NO_SPLIT, POSE_INCOMPLETE, POSE_STACK_OVERFLOW, Model, Obstacles, cbvh_collide_batch,
               cbvh_distance_batch, cbvh_workspace_bytes, _aligned_empty)

# times a pose flagged CBVH_POSE_STACK_OVERFLOW is run again before its flag is kept
RETRIES = 2

COLLIDE, DISTANCE = 0, 1


@dataclass
class Requests:
    """Requests in arrival order; request r owns poses[first[r] : first[r] + count[r]]."""
    arrival: np.ndarray   # float64 [R], seconds after the start
    kind: np.ndarray      # uint8 [R], COLLIDE or DISTANCE
    obstacle: np.ndarray  # uint32 [R]
    first: np.ndarray     # int64 [R]
    count: np.ndarray     # int64 [R]
    poses: np.ndarray     # float32 [N, 3, 4]

    def __len__(self):
        return len(self.arrival)


def _qmul(a, b):
    aw, ax, ay, az = a[..., 0], a[..., 1], a[..., 2], a[..., 3]
    bw, bx, by, bz = b[..., 0], b[..., 1], b[..., 2], b[..., 3]
    return np.stack([aw * bw - ax * bx - ay * by - az * bz, aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx, aw * bz + ax * by - ay * bx + az * bw], axis=-1)


def _unit(rng, n):
    v = rng.normal(size=(n, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def make_requests(n_requests, rate, n_obstacles, rng, batch_min=1, batch_max=4096, collide_frac=0.7,
                  rot_step=0.05, trans_step=0.02, box=2.5):
    """Poisson arrivals at `rate` requests/s (rate = inf: all at time 0), batch
    sizes log-uniform in [batch_min, batch_max], obstacles uniform, a
    collide/distance mix, and each request's poses a random walk: a uniform
    start (rotation uniform, translation uniform in [-box, box]^3), then steps
    rotating by an angle in [0, rot_step] about a uniform axis and moving by
    a length in [0, trans_step] along a uniform direction."""
    R = n_requests
    gaps = np.zeros(R) if not np.isfinite(rate) else rng.exponential(1.0 / rate, R)
    arrival = np.cumsum(gaps) - (gaps[0] if R else 0.0)
    kind = np.where(rng.random(R) < collide_frac, COLLIDE, DISTANCE).astype(np.uint8)
    obstacle = rng.integers(0, n_obstacles, R).astype(np.uint32)
    count = np.floor(np.exp(rng.uniform(np.log(batch_min), np.log(batch_max + 1), R))).astype(np.int64)
    count = np.clip(count, batch_min, batch_max)
    first = np.concatenate([[0], np.cumsum(count)[:-1]]).astype(np.int64)
    N = int(count.sum())
    # start poses: Shoemake uniform quaternions, uniform translations
    u1, u2, u3 = rng.random(R), rng.random(R), rng.random(R)
    q = np.stack([np.sqrt(1 - u1) * np.sin(2 * np.pi * u2), np.sqrt(1 - u1) * np.cos(2 * np.pi * u2),
                  np.sqrt(u1) * np.sin(2 * np.pi * u3), np.sqrt(u1) * np.cos(2 * np.pi * u3)], axis=1)
    t = rng.uniform(-box, box, size=(R, 3))
    Q = np.empty((N, 4))
    T = np.empty((N, 3))
    for s in range(int(count.max()) if R else 0):
        act = np.nonzero(count > s)[0]
        if s > 0:
            ang = rng.uniform(0.0, rot_step, len(act))
            ax = _unit(rng, len(act))
            dq = np.concatenate([np.cos(ang / 2)[:, None], np.sin(ang / 2)[:, None] * ax], axis=1)
            q[act] = _qmul(dq, q[act])
            q[act] /= np.linalg.norm(q[act], axis=1, keepdims=True)
            t[act] += _unit(rng, len(act)) * rng.uniform(0.0, trans_step, len(act))[:, None]
        Q[first[act] + s] = q[act]
        T[first[act] + s] = t[act]
    w, x, y, z = Q[:, 0], Q[:, 1], Q[:, 2], Q[:, 3]
    M = np.empty((N, 3, 4))
    M[:, 0, 0], M[:, 0, 1], M[:, 0, 2] = 1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)
    M[:, 1, 0], M[:, 1, 1], M[:, 1, 2] = 2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)
    M[:, 2, 0], M[:, 2, 1], M[:, 2, 2] = 2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)
    M[:, :, 3] = T
    return Requests(arrival, kind, obstacle, first, count, M.astype(np.float32))


class _Slot:
    def __init__(self, link, kind, max_poses, device, small_max):
        import torch
        self.kind = kind
        self.small_max = small_max  # admits only requests of at most this many poses (None: any)
        self.stream = torch.cuda.Stream(device=device)
        self.P = torch.empty((max_poses, 3, 4), dtype=torch.float32, device=device)
        self.obj = torch.empty(max_poses, dtype=torch.int32, device=device)
        self.out = torch.empty(max_poses, dtype=torch.uint8 if kind == COLLIDE else torch.float32, device=device)
        self.status = torch.empty(max_poses, dtype=torch.uint8, device=device)
        self.ws = _aligned_empty(cbvh_workspace_bytes(link.handle, link.handle, max_poses,
                                                      EARLY_EXIT if kind == COLLIDE else 0, 0), device)
        # pinned staging: the admitted requests' poses gathered in launch order, results back
        self.hP = torch.empty((max_poses, 3, 4), dtype=torch.float32).pin_memory()
        self.hobj = torch.empty(max_poses, dtype=torch.int32).pin_memory()
        self.hout = torch.empty(max_poses, dtype=self.out.dtype).pin_memory()
        self.hstatus = torch.empty(max_poses, dtype=torch.uint8).pin_memory()
        self.event = torch.cuda.Event()
        # while a launch is in flight: the global pose index of each of its
        # poses, in launch order, and how many times they have been retried
        self.busy = None
        self.gidx = None
        self.tries = 0


class Server:
    """Continuous-batching request loop over a resident obstacle set.

    Each query kind has `slots_per_kind` launch slots.  With two or more, the
    first slot of a kind only admits small requests (at most `small_max`
    poses), so that they never wait behind a launch that carries a request of
    thousands of poses; the other slots admit any request, in arrival order."""

    def __init__(self, link: Model, obstacles: Obstacles, device="cuda", slots_per_kind=2,
                 memory_budget=2 << 30, max_poses=None, launch_cap=16384, distance_cap=None, small_max=256,
                 launch_cfg=None, first_flags=0):
        self.link, self.obstacles, self.device = link, obstacles, device
        # extra query flags of a pose's first launch (CBVH_NO_SPLIT keeps it in
        # one wavefront); a pose run again after a stack overflow always may
        # hand work over
        self.first_flags = first_flags
        # launch knobs (autotune.launch_env), applied to every launch.  By
        # default two waves per workgroup and one helper wave per CU: the
        # slots' launches share the GPU, and the four helpers per CU of a
        # lone distance launch wait holding CU slots the other launches
        # need (measured in paired runs: saturation 4.74-4.75 M poses/s and
        # p99 126 ms, against 4.47 M and 157 ms with the library's defaults
        # and 4.39-4.64 M with one wave per workgroup)
        self.launch_cfg = {"waves_per_group": 2, "helpers_per_cu": 1} if launch_cfg is None else launch_cfg
        # the largest launch that lets every slot's workspace fit the budget
        if max_poses is None:
            lo, hi = 4096, 1 << 22
            while lo < hi:
                mid = (lo + hi + 1) // 2
                need = slots_per_kind * sum(cbvh_workspace_bytes(link.handle, link.handle, mid, f, 0)
                                            for f in (EARLY_EXIT, 0))
                if need <= memory_budget:
                    lo = mid
                else:
                    hi = mid - 1
            # larger launches add latency and little throughput
            max_poses = min(lo, launch_cap)
        self.max_poses = max_poses
        # distance launches cost far more per pose: a smaller cap keeps them
        # short, so that requests behind them wait less
        self.cap = {COLLIDE: max_poses, DISTANCE: min(max_poses, distance_cap or max_poses)}
        self.slots = []
        for k in (COLLIDE, DISTANCE):
            for i in range(slots_per_kind):
                small = small_max if (slots_per_kind > 1 and i == 0 and small_max) else None
                self.slots.append(_Slot(link, k, self.cap[k], device, small))

    def run(self, req: Requests, realtime=True):
        """Serve every request; returns per-request latencies (s), per-pose results
        (booleans and distances in request pose order) and throughput."""
        from .autotune import launch_env
        with launch_env(self.launch_cfg):
            return self._run(req, realtime)

    def _run(self, req, realtime):
        import torch
        R, N = len(req), len(req.poses)
        for k in (COLLIDE, DISTANCE):
            m = req.kind == k
            if m.any() and int(req.count[m].max()) > self.cap[k]:
                raise ValueError(f"a request of {int(req.count[m].max())} poses exceeds the {self.cap[k]} poses one "
                                 "launch holds; raise launch_cap, distance_cap or memory_budget")
        hit = np.zeros(N, dtype=np.uint8)
        dist = np.full(N, np.nan, dtype=np.float32)
        status = np.zeros(N, dtype=np.uint8)
        req_of = np.repeat(np.arange(R), req.count)  # request of each global pose
        pending = req.count.astype(np.int64).copy()  # poses of each request without a final answer
        # per kind: its requests in arrival order, which are admitted, and the first not yet admitted
        queue = {k: {"rs": np.nonzero(req.kind == k)[0], "admitted": None, "head": 0} for k in (COLLIDE, DISTANCE)}
        for Q in queue.values():
            Q["admitted"] = np.zeros(len(Q["rs"]), dtype=bool)
        done_at = np.full(R, np.nan)
        n_launch = n_retry = 0
        max_batch = 0
        t0 = time.perf_counter()
        remaining = R

        def launch(s, gidx, tries):
            """Stage the poses gidx (global indices) in the slot and launch them."""
            n = len(gidx)
            flags = self.first_flags if tries == 0 else self.first_flags & ~NO_SPLIT
            s.hP.numpy()[:n] = req.poses[gidx]
            s.hobj.numpy()[:n] = req.obstacle[req_of[gidx]]
            with torch.cuda.stream(s.stream):
                s.P[:n].copy_(s.hP[:n], non_blocking=True)
                s.obj[:n].copy_(s.hobj[:n], non_blocking=True)
                if s.kind == COLLIDE:
                    cbvh_collide_batch(self.link.handle, self.link.dev, self.obstacles.handle, s.P, s.obj, n,
                                       EARLY_EXIT | flags, s.out, s.status, s.ws, stream=s.stream)
                else:
                    cbvh_distance_batch(self.link.handle, self.link.dev, self.obstacles.handle, s.P, s.obj, n, flags,
                                        s.out, s.status, s.ws, stream=s.stream)
                s.hout[:n].copy_(s.out[:n], non_blocking=True)
                s.hstatus[:n].copy_(s.status[:n], non_blocking=True)
                s.event.record(s.stream)
            s.gidx, s.tries, s.busy = gidx, tries, True

        while remaining:
            now = time.perf_counter() - t0
            progressed = False
            for s in self.slots:
                if s.busy is not None and s.event.query():
                    t_done = time.perf_counter() - t0
                    gidx = s.gidx
                    n_done = len(gidx)
                    out_np, st_np = s.hout.numpy()[:n_done], s.hstatus.numpy()[:n_done]
                    if (st_np == POSE_INCOMPLETE).any():
                        # a wavefront gave up waiting for handed-over work: this
                        # launch's answers cannot be trusted
                        raise RuntimeError("a launch gave up waiting for handed-over work (device wait limit); "
                                           f"results of its {n_done} poses are incomplete")
                    (hit if s.kind == COLLIDE else dist)[gidx] = out_np
                    status[gidx] = st_np
                    # a pose whose traversal state outgrew its wavefront where
                    # nobody could take its pending pairs (its launch's helper
                    # waves had already left, as can happen when launches share
                    # the GPU) is run again in a launch of its own
                    again = (st_np == POSE_STACK_OVERFLOW) & (s.tries < RETRIES)
                    final = gidx[~again]
                    np.subtract.at(pending, req_of[final], 1)
                    for r in np.unique(req_of[final]):
                        if pending[r] == 0:
                            done_at[r] = t_done
                            remaining -= 1
                    s.busy = None
                    progressed = True
                    if again.any():
                        launch(s, gidx[again], s.tries + 1)
                        n_retry += 1
                        continue
                if s.busy is not None:
                    continue
                Q = queue[s.kind]
                rs, adm = Q["rs"], Q["admitted"]
                while Q["head"] < len(rs) and adm[Q["head"]]:
                    Q["head"] += 1
                # admit arrived requests in arrival order while they fit (a
                # small-request slot passes over the large ones)
                arrived_t = now if realtime else np.inf
                chosen, n = [], 0
                for i in range(Q["head"], len(rs)):
                    r = rs[i]
                    if req.arrival[r] > arrived_t:
                        break
                    c = int(req.count[r])
                    if adm[i] or (s.small_max is not None and c > s.small_max):
                        continue
                    if n + c > self.cap[s.kind]:
                        break
                    chosen.append((i, r, n, c))
                    n += c
                if not chosen:
                    continue
                for i, _, _, _ in chosen:
                    adm[i] = True
                launch(s, np.concatenate([np.arange(req.first[r], req.first[r] + c) for _, r, _, c in chosen]), 0)
                n_launch += 1
                max_batch = max(max_batch, n)
                progressed = True
            if not progressed:
                time.sleep(20e-6)
        makespan = time.perf_counter() - t0
        torch.cuda.synchronize()
        lat = done_at - req.arrival
        return {"latency_s": lat, "hit": hit, "dist": dist, "status": status, "makespan_s": makespan,
                "poses_per_sec": N / makespan, "requests_per_sec": R / makespan, "launches": n_launch,
                "retry_launches": n_retry,
                "largest_launch": max_batch, "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3)}
