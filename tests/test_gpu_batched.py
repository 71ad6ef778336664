"""GPU tests of batched queries: one moving link against many obstacles of
uneven size in one launch (reduced size of the batched workload).

The batched answers must equal the plain per-obstacle queries exactly (the
plain kernel is the reference) and match the oracle on a sample of poses."""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
import paper_2012_05348_amd as cb  # noqa: E402
from synth import configs, meshes  # noqa: E402

DEV = "cuda:0"
SMALL = configs.BatchedWorkload(n_obstacles=8, tri_max=20000, min_poses=2000)


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def setup():
    w = SMALL
    kw = dict(bv=cb.DOP18, branching=w.branching, leaf_size=w.leaf_size, bits=w.bits)
    link_mesh = w.link_mesh()
    obs_meshes = [w.obstacle_mesh(i) for i in range(w.n_obstacles)]
    link = cb.Model.build(*link_mesh, **kw).to(DEV)
    obs = [cb.Model.build(V, T, **kw).to(DEV) for V, T in obs_meshes]
    P, obj = w.raw_poses()
    return w, link_mesh, obs_meshes, link, obs, P, obj


def _plain(link, obs, P, obj, query):
    """The plain kernel, one launch per obstacle, results scattered back."""
    n = len(P)
    res = np.zeros(n, dtype=np.float32 if query == "distance" else np.uint8)
    for k, m in enumerate(obs):
        idx = np.nonzero(obj == k)[0]
        if len(idx) == 0:
            continue
        Pd = torch.from_numpy(P[idx]).to(DEV)
        if query == "distance":
            d, st = cb.distance(link, m, Pd)
            r = d
        else:
            r, st = cb.collide(link, m, Pd)
        assert (st == 0).all()
        res[idx] = r.cpu().numpy()
    return res


def test_batched_booleans_equal_plain_per_obstacle_queries(setup):
    w, _, _, link, obs, P, obj = setup
    _log(f"batched collide: {len(obs)} obstacles, {len(P)} poses")
    oset = cb.Obstacles(obs, DEV)
    hit, st = cb.collide_batch(link, oset, torch.from_numpy(P).to(DEV), torch.from_numpy(obj).to(DEV))
    assert (st.cpu().numpy() == 0).all()
    ref = _plain(link, obs, P, obj, "bool")
    assert np.array_equal(hit.cpu().numpy(), ref)
    assert 0 < ref.sum() < len(ref)


def test_batched_distances_equal_plain_per_obstacle_queries(setup):
    w, _, _, link, obs, P, obj = setup
    sel = np.arange(0, len(P), 4)  # a quarter of the poses keeps the test short
    Ps, objs = P[sel], obj[sel]
    _log(f"batched distance: {len(Ps)} poses")
    oset = cb.Obstacles(obs, DEV)
    d, st = cb.distance_batch(link, oset, torch.from_numpy(Ps).to(DEV), torch.from_numpy(objs).to(DEV))
    assert (st.cpu().numpy() == 0).all()
    ref = _plain(link, obs, Ps, objs, "distance")
    assert np.array_equal(d.cpu().numpy().view(np.uint32), ref.view(np.uint32))


def test_batched_booleans_match_oracle_on_sample(setup):
    w, link_mesh, obs_meshes, link, obs, P, obj = setup
    oset = cb.Obstacles(obs, DEV)
    hit, st = cb.collide_batch(link, oset, torch.from_numpy(P).to(DEV), torch.from_numpy(obj).to(DEV))
    hit = hit.cpu().numpy()
    A = oracle.Mesh(*link_mesh)
    rng = np.random.default_rng(5)
    checked = 0
    for k in range(len(obs)):
        idx = np.nonzero(obj == k)[0]
        if len(idx) == 0:
            continue
        idx = rng.choice(idx, min(12, len(idx)), replace=False)
        Vb, Tb = obs_meshes[k]
        B = oracle.Mesh(Vb, Tb)
        m = w.margin_rel * max(meshes.mesh_diameter(link_mesh[0]), meshes.mesh_diameter(Vb))
        cls = oracle.classify_batch(A, B, P[idx], m)
        keep = idx[cls != oracle.MARGINAL]
        ref, _ = oracle.collide_batch(A, B, P[keep])
        assert np.array_equal(hit[keep].astype(bool), ref), k
        checked += len(keep)
    assert checked > 60


def test_bad_obstacle_index_is_flagged_per_pose(setup):
    w, _, _, link, obs, P, obj = setup
    oset = cb.Obstacles(obs, DEV)
    n = 256
    bad = obj[:n].copy()
    bad[7] = len(obs)
    bad[100] = 0xFFFFFFFF
    hit, st = cb.collide_batch(link, oset, torch.from_numpy(P[:n]).to(DEV), torch.from_numpy(bad).to(DEV))
    st = st.cpu().numpy()
    assert st[7] == cb.POSE_BAD_OBSTACLE and st[100] == cb.POSE_BAD_OBSTACLE
    ok = np.ones(n, dtype=bool)
    ok[[7, 100]] = False
    assert (st[ok] == 0).all()
    ref = _plain(link, obs, P[:n][ok], obj[:n][ok], "bool")
    assert np.array_equal(hit.cpu().numpy()[ok], ref)


def test_batched_query_replays_from_a_hip_graph(setup):
    # the query enqueues kernels only (no host copies, no memset nodes): a
    # captured graph replays it; each replay is checked against the eager run
    # with eager work and synchronizations in between
    w, _, _, link, obs, P, obj = setup
    oset = cb.Obstacles(obs, DEV)
    n = 1024
    Pd = torch.from_numpy(P[:n]).to(DEV)
    od = torch.from_numpy(obj[:n]).to(DEV)
    ws = cb.workspace(link, link, n, cb.EARLY_EXIT, 0, DEV)
    hit = torch.empty(n, dtype=torch.uint8, device=DEV)
    st = torch.empty(n, dtype=torch.uint8, device=DEV)
    cb.collide_batch(link, oset, Pd, od, ws=ws, out=(hit, st))
    torch.cuda.synchronize()
    eager = hit.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        cb.cbvh_collide_batch(link.handle, link.dev, oset.handle, Pd, od, n, cb.EARLY_EXIT, hit, st, ws.buf,
                              stream=s)
    for r in range(3):
        hit.fill_(7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(hit, eager), r
        assert (st == 0).all()
        cb.collide_batch(link, oset, Pd, od, ws=ws, out=(hit, st))  # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(hit, eager)


def test_autotuner_keeps_answers_and_picks_a_candidate(setup):
    from paper_2012_05348_amd import autotune
    w, link_mesh, obs_meshes, link, obs, P, obj = setup
    n = 512
    res = autotune.tune(link_mesh, obs_meshes, P[:n], obj[:n], bits=w.bits, leaf_size=w.leaf_size,
                        branchings=(4, 8), treelet_bytes=(8192,), waves_per_cu=(0, 8), steps=2, warmup=1,
                        device=DEV)
    assert len(res["results"]) == 4 and res["all_answers_equal"]
    best = res["best"]
    assert best is not None and best["ms"] == min(r["ms"] for r in res["results"])
    assert "CBVH_WAVES_PER_CU" not in os.environ
