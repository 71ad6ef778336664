"""GPU tests of the continuous-batching serving loop: every request's result
is the same alone and in the mix (booleans exactly, distances bitwise), and
at the serving workload's scale (requests of up to 4,096 poses, a
200k-triangle obstacle) a margin-filtered sample of every request's poses
matches the oracle."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2012_05348_amd as cb  # noqa: E402
from paper_2012_05348_amd import serve  # noqa: E402
from synth import configs, meshes  # noqa: E402

DEV = "cuda:0"
SMALL = configs.BatchedWorkload(index=4, n_obstacles=6, tri_max=20000, min_poses=0)


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def server():
    w = SMALL
    kw = dict(bv=cb.DOP18, branching=w.branching, leaf_size=w.leaf_size, bits=w.bits)
    link = cb.Model.build(*w.link_mesh(), **kw).to(DEV)
    obs = [cb.Model.build(*w.obstacle_mesh(i), **kw).to(DEV) for i in range(w.n_obstacles)]
    # small launches so that requests really mix across several launches and slots
    srv = serve.Server(link, cb.Obstacles(obs, DEV), DEV, slots_per_kind=2, max_poses=600)
    return link, obs, srv


def _alone(link, obs, req, r):
    P = torch.from_numpy(req.poses[req.first[r]:req.first[r] + req.count[r]]).to(DEV)
    m = obs[int(req.obstacle[r])]
    if req.kind[r] == serve.COLLIDE:
        h, st = cb.collide(link, m, P)
        return h.cpu().numpy(), st.cpu().numpy()
    d, st = cb.distance(link, m, P)
    return d.cpu().numpy(), st.cpu().numpy()


@pytest.mark.parametrize("realtime", [False, True])
def test_results_are_the_same_alone_and_in_the_mix(server, realtime):
    link, obs, srv = server
    rng = np.random.default_rng(11 + realtime)
    # up to 500 poses: some requests are too large for the small-request slot
    req = serve.make_requests(90, 3000.0 if realtime else np.inf, len(obs), rng, batch_max=500)
    res = srv.run(req, realtime=realtime)
    _log(f"serving realtime={realtime}: {res['launches']} launches, largest {res['largest_launch']}, "
         f"p50 {res['p50_ms']:.2f} ms p99 {res['p99_ms']:.2f} ms, {res['poses_per_sec']:.0f} poses/s")
    assert (res["status"] == 0).all()
    assert np.isfinite(res["latency_s"]).all() and (res["latency_s"] >= 0).all()
    assert res["launches"] >= 4
    for r in range(len(req)):
        sl = slice(req.first[r], req.first[r] + req.count[r])
        got = res["hit"][sl] if req.kind[r] == serve.COLLIDE else res["dist"][sl]
        ref, st = _alone(link, obs, req, r)
        assert (st == 0).all()
        if req.kind[r] == serve.COLLIDE:
            assert np.array_equal(got, ref), r
        else:
            assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), r
    assert (req.kind == serve.COLLIDE).any() and (req.kind == serve.DISTANCE).any()


def _merge(a, b):
    return serve.Requests(np.concatenate([a.arrival, b.arrival]), np.concatenate([a.kind, b.kind]),
                          np.concatenate([a.obstacle, b.obstacle]),
                          np.concatenate([a.first, b.first + len(a.poses)]), np.concatenate([a.count, b.count]),
                          np.concatenate([a.poses, b.poses]))


def test_served_results_match_oracle_at_scale():
    """The serving workload's link against a 200k-triangle torus and three of
    its obstacles, behind the default two slots per kind: 40 requests of
    log-uniform size up to 4,096 poses plus a 4,096-pose collision request and
    a 4,096-pose distance request against the 200k-triangle obstacle.  Every
    request's result equals its plain query run alone, and up to 24 poses of
    every request that the margin accepts match the oracle (booleans exactly,
    distances within 1e-5 relative, 0 where the meshes collide)."""
    w = configs.SERVING
    rng = np.random.default_rng(4096)
    link_mesh = w.link_mesh()
    obs_meshes = [meshes.torus(500, 200, 1.0, 0.3, 0.02, rng)] + [w.obstacle_mesh(i) for i in range(3)]
    assert len(obs_meshes[0][1]) == 200000
    kw = dict(bv=cb.DOP18, branching=w.branching, leaf_size=w.leaf_size, bits=w.bits)
    link = cb.Model.build(*link_mesh, **kw).to(DEV)
    obs = [cb.Model.build(V, T, **kw).to(DEV) for V, T in obs_meshes]
    srv = serve.Server(link, cb.Obstacles(obs, DEV), DEV)
    big = serve.make_requests(2, np.inf, 1, rng, batch_min=4096, batch_max=4096)
    big.kind[:] = [serve.COLLIDE, serve.DISTANCE]
    req = _merge(serve.make_requests(40, np.inf, len(obs), rng, batch_max=4096), big)
    _log(f"serving at scale: {len(req)} requests, {len(req.poses)} poses, largest {int(req.count.max())}")
    res = srv.run(req, realtime=False)
    assert (res["status"] == 0).all()
    A = oracle.Mesh(*link_mesh)
    Bs = [oracle.Mesh(V, T) for V, T in obs_meshes]
    checked = {serve.COLLIDE: 0, serve.DISTANCE: 0}
    for r in range(len(req)):
        sl = slice(req.first[r], req.first[r] + req.count[r])
        got = res["hit"][sl] if req.kind[r] == serve.COLLIDE else res["dist"][sl]
        ref, st = _alone(link, obs, req, r)
        assert (st == 0).all()
        assert np.array_equal(np.asarray(got).view(np.uint8 if req.kind[r] == serve.COLLIDE else np.uint32),
                              ref.view(np.uint8 if req.kind[r] == serve.COLLIDE else np.uint32)), r
        k = int(req.obstacle[r])
        idx = np.sort(rng.choice(int(req.count[r]), min(24, int(req.count[r])), replace=False))
        Pq = req.poses[sl][idx]
        m = w.margin_rel * max(meshes.mesh_diameter(link_mesh[0]), meshes.mesh_diameter(obs_meshes[k][0]))
        cls = oracle.classify_batch(A, Bs[k], Pq, m)
        sep, col = cls == oracle.SEPARATED, cls == oracle.COLLIDING
        if req.kind[r] == serve.COLLIDE:
            keep = sep | col
            ref_h, _ = oracle.collide_batch(A, Bs[k], Pq[keep])
            assert np.array_equal(got[idx][keep].astype(bool), ref_h), r
            checked[serve.COLLIDE] += int(keep.sum())
        else:
            ref_d, _ = oracle.distance_batch(A, Bs[k], Pq)
            g = got[idx].astype(np.float64)
            if sep.any():
                assert (np.abs(g[sep] - ref_d[sep]) / ref_d[sep]).max() <= 1e-5, r
            assert (g[col] == 0).all(), r
            checked[serve.DISTANCE] += int((sep | col).sum())
    _log(f"serving at scale: oracle checked {checked}")
    assert checked[serve.COLLIDE] > 200 and checked[serve.DISTANCE] > 60


def test_a_request_larger_than_a_launch_is_rejected(server):
    _, obs, srv = server
    req = serve.make_requests(3, np.inf, len(obs), np.random.default_rng(3), batch_min=700, batch_max=800)
    with pytest.raises(ValueError):
        srv.run(req, realtime=False)


def test_an_incomplete_launch_fails_the_run(server):
    """With a device wait limit of one tick every launch gives up waiting for
    handed-over work and flags its poses incomplete; the loop raises instead
    of returning those answers.  A fresh server (the raise leaves launches
    in flight) runs normally once the default limit is back."""
    link, obs, _ = server
    srv = serve.Server(link, cb.Obstacles(obs, DEV), DEV, slots_per_kind=1, max_poses=600)
    req = serve.make_requests(8, np.inf, len(obs), np.random.default_rng(21), batch_max=300)
    try:
        cb.cbvh_set_wait_limit(1)
        with pytest.raises(RuntimeError, match="wait limit"):
            srv.run(req, realtime=False)
        torch.cuda.synchronize()
    finally:
        cb.cbvh_set_wait_limit(0)
    srv2 = serve.Server(link, cb.Obstacles(obs, DEV), DEV, slots_per_kind=1, max_poses=600)
    res = srv2.run(req, realtime=False)
    assert (res["status"] == 0).all()


def test_poses_that_overflow_their_stack_are_run_again():
    """Small per-wave stacks, and first launches that keep every pose in one
    wavefront (no hand-over), make poses overflow (CBVH_POSE_STACK_OVERFLOW);
    the loop runs those poses again, with hand-over allowed, so every
    request still gets its plain query's answer.  AABB models of branching
    factor 4 (16 child pairs per expansion), so that hand-over with these
    stacks makes progress."""
    w = SMALL
    kw = dict(bv=cb.AABB, branching=4, leaf_size=w.leaf_size, bits=8)
    link = cb.Model.build(*w.link_mesh(), **kw).to(DEV)
    obs = [cb.Model.build(*w.obstacle_mesh(i), **kw).to(DEV) for i in range(w.n_obstacles)]
    srv = serve.Server(link, cb.Obstacles(obs, DEV), DEV, slots_per_kind=1, max_poses=600,
                       first_flags=cb.NO_SPLIT)
    req = serve.make_requests(24, np.inf, len(obs), np.random.default_rng(31), batch_max=300)
    try:
        # 64 records hold about half of a full descent of these trees: poses
        # that reach the leaves overflow without hand-over
        cb.cbvh_set_stack_limits(entries=256, records=64)
        res = srv.run(req, realtime=False)
        alone = [_alone(link, obs, req, r) for r in range(len(req))]
    finally:
        cb.cbvh_set_stack_limits(0, 0)
    _log(f"stack-overflow retries: {res['retry_launches']} retry launches, statuses "
         f"{np.bincount(res['status'], minlength=6).tolist()}")
    assert res["retry_launches"] > 0
    assert (res["status"] == 0).all()
    for r in range(len(req)):
        sl = slice(req.first[r], req.first[r] + req.count[r])
        got = res["hit"][sl] if req.kind[r] == serve.COLLIDE else res["dist"][sl]
        ref, st = alone[r]
        assert (st == 0).all()
        assert np.array_equal(got.view(np.uint32) if got.dtype == np.float32 else got,
                              ref.view(np.uint32) if ref.dtype == np.float32 else ref)
