"""GPU tests of batched queries: one moving link against many obstacles of
uneven size in one launch.

At reduced size (8 obstacles) the batched answers must equal the plain
per-obstacle queries exactly (the plain kernel is the reference).  At the
batched workload's full size (the 20k-triangle link against all 64
obstacles, 30,723 poses) the booleans must equal the oracle's on every pose
the margin accepts, and distances against an obstacle set that adds two
200k-triangle obstacles must match the oracle within 1e-5 relative."""
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


def test_autotuner_keeps_answers_and_picks_a_candidate(setup, tmp_path):
    from paper_2012_05348_amd import autotune
    w, link_mesh, obs_meshes, link, obs, P, obj = setup
    n = 512
    res = autotune.tune(link_mesh, obs_meshes, P[:n], obj[:n], bits=w.bits, leaf_size=w.leaf_size,
                        branchings=(4, 8), treelet_bytes=(8192, autotune.WHOLE_TREE), waves_per_cu=(0, 8),
                        waves_per_group=(1, 4), steps=2, warmup=1, device=DEV)
    assert len(res["results"]) == 16 and res["all_answers_equal"]
    best = res["best"]
    assert best is not None and best["ms"] == min(r["ms"] for r in res["results"])
    assert "CBVH_WAVES_PER_CU" not in os.environ and "CBVH_WAVES_PER_GROUP" not in os.environ
    # the pick, stored and applied, answers like the default launch
    path = autotune.save("test workload", best, str(tmp_path / "tune.json"))
    cfg = autotune.load("test workload", path)
    assert cfg == best
    kw = dict(bv=cb.DOP18, leaf_size=w.leaf_size, bits=w.bits, **autotune.build_kwargs(cfg))
    link2 = cb.Model.build(*link_mesh, **kw).to(DEV)
    oset2 = cb.Obstacles([cb.Model.build(V, T, **kw).to(DEV) for V, T in obs_meshes], DEV)
    Pd, od = torch.from_numpy(P[:n]).to(DEV), torch.from_numpy(obj[:n]).to(DEV)
    ref, _ = cb.collide_batch(link, cb.Obstacles(obs, DEV), Pd, od)
    with autotune.launch_env(cfg):
        got, st = cb.collide_batch(link2, oset2, Pd, od)
    assert (st.cpu().numpy() == 0).all() and torch.equal(got, ref)


# ---------------------------------------------------------------- full size
@pytest.fixture(scope="module")
def full():
    w = configs.BATCHED
    kw = dict(bv=cb.DOP18, branching=w.branching, leaf_size=w.leaf_size, bits=w.bits)
    _log(f"full batched workload: building {w.n_obstacles} obstacle models")
    link_mesh = w.link_mesh()
    obs_meshes = [w.obstacle_mesh(i) for i in range(w.n_obstacles)]
    link = cb.Model.build(*link_mesh, **kw).to(DEV)
    obs = [cb.Model.build(V, T, **kw).to(DEV) for V, T in obs_meshes]
    P, obj = w.raw_poses()
    A = oracle.Mesh(*link_mesh)
    return w, link_mesh, obs_meshes, link, obs, P, obj, A


def _margin(w, link_mesh, Vb):
    return w.margin_rel * max(meshes.mesh_diameter(link_mesh[0]), meshes.mesh_diameter(Vb))


def test_full_batched_booleans_match_oracle_on_every_pose(full):
    w, link_mesh, obs_meshes, link, obs, P, obj, A = full
    oset = cb.Obstacles(obs, DEV)
    _log(f"full batched collide: {len(P)} poses")
    hit, st = cb.collide_batch(link, oset, torch.from_numpy(P).to(DEV), torch.from_numpy(obj).to(DEV))
    hit, st = hit.cpu().numpy().astype(bool), st.cpu().numpy()
    assert (st == 0).all()
    checked = 0
    for k, (Vb, Tb) in enumerate(obs_meshes):
        idx = np.nonzero(obj == k)[0]
        if len(idx) == 0:
            continue
        B = oracle.Mesh(Vb, Tb)
        cls = oracle.classify_batch(A, B, P[idx], _margin(w, link_mesh, Vb))
        keep = idx[cls != oracle.MARGINAL]
        ref, _ = oracle.collide_batch(A, B, P[keep])
        bad = np.nonzero(hit[keep] != ref)[0]
        assert len(bad) == 0, (k, keep[bad[:10]])
        checked += len(keep)
    assert checked > len(P) - 64
    assert 0 < hit.sum() < len(P)


def test_batched_distances_with_200k_obstacles_match_oracle(full):
    """The 64 obstacles plus a 200k-triangle torus and a 200k-triangle
    icosphere: per obstacle the first 6 of its poses, and 64 poses each for
    the two large ones; batched distances equal the plain per-obstacle
    queries bitwise and the oracle's within 1e-5 relative (0 where they
    collide)."""
    w, link_mesh, obs_meshes, link, obs, P, obj, A = full
    rng = np.random.default_rng(200000)
    big = [meshes.torus(500, 200, 1.0, 0.3, 0.02, rng), meshes.icosphere(100, 0.1, rng)]
    assert [len(T) for _, T in big] == [200000, 200000]
    kw = dict(bv=cb.DOP18, branching=w.branching, leaf_size=w.leaf_size, bits=w.bits)
    all_meshes = obs_meshes + big
    models = obs + [cb.Model.build(V, T, **kw).to(DEV) for V, T in big]
    sel = np.concatenate([np.nonzero(obj == k)[0][:6] for k in range(len(obs))])
    from synth import poses as sp
    n_big = 64
    Pb = sp.compose(sp.uniform_rotations(2 * n_big, rng), sp.box_translations(2 * n_big, 2.5, rng))
    Pq = np.concatenate([P[sel], Pb])
    oq = np.concatenate([obj[sel], np.repeat(np.arange(len(obs), len(obs) + 2, dtype=np.uint32), n_big)])
    _log(f"batched distances: {len(Pq)} poses over {len(models)} obstacles (two of 200k triangles)")
    oset = cb.Obstacles(models, DEV)
    d, st = cb.distance_batch(link, oset, torch.from_numpy(Pq).to(DEV), torch.from_numpy(oq).to(DEV))
    d, st = d.cpu().numpy(), st.cpu().numpy()
    assert (st == 0).all()
    plain = _plain(link, models, Pq, oq, "distance")
    assert np.array_equal(d.view(np.uint32), plain.view(np.uint32))
    n_sep = 0
    for k, (Vb, Tb) in enumerate(all_meshes):
        idx = np.nonzero(oq == k)[0]
        if len(idx) == 0:
            continue
        B = oracle.Mesh(Vb, Tb)
        cls = oracle.classify_batch(A, B, Pq[idx], _margin(w, link_mesh, Vb))
        ref, _ = oracle.distance_batch(A, B, Pq[idx])
        sep, col = cls == oracle.SEPARATED, cls == oracle.COLLIDING
        got = d[idx].astype(np.float64)
        if sep.any():
            rel = np.abs(got[sep] - ref[sep]) / ref[sep]
            assert rel.max() <= 1e-5, (k, rel.max(), idx[sep][np.argmax(rel)])
        assert (got[col] == 0).all(), k
        n_sep += int(sep.sum())
    assert n_sep > 300
