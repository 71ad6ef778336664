"""GPU parity of oriented-box (OBB) models against the FP64 oracle.

The answers do not depend on the BV type (every BV test is conservative and
every leaf pair is decided exactly), so OBB models must reproduce the
oracle's booleans, pair lists and distances exactly like AABB and 18-DOP
models do:
- decode: every node's decoded descriptor (frame included) bit-identical to
  the oracle's decoder, for FP32 and 8/16-bit codes;
- tiny workload: sorted colliding-pair lists and early-exit booleans on the
  256 margin-filtered poses, 8-bit, 16-bit and FP32 descriptors;
- near-touching icospheres offset along random directions, and pose matrices
  that are not rotations: distances within 1e-5 relative of the oracle, zero
  where they collide;
- small stacks that force work hand-over between waves (items carry the
  frames): pair lists still exact;
- the scaled workload's meshes as OBB models: booleans on all 16,384 poses
  equal the 18-DOP models' and the oracle's on a 512-pose sample;
- the proximity workload's meshes as OBB models: every pose completes, with
  distances bit-identical to the AABB models' on all 4,096 poses;
- batched queries against an obstacle set of OBB models, and the
  allocation-free entry point: equal to the plain queries.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from synth import configs, poses

torch = pytest.importorskip("torch")
cb = pytest.importorskip("paper_2012_05348_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


_cache = {}


def obb_models(cfg, bits, branching=4, leaf_size=1, treelet_bytes=0):
    key = (cfg, bits, branching, leaf_size, treelet_bytes)
    if key not in _cache:
        (va, ta), (vb, tb) = W.meshes(cfg)
        kw = dict(bv=cb.OBB, branching=branching, leaf_size=leaf_size, bits=bits, treelet_bytes=treelet_bytes)
        _cache[key] = cb.Model.build(va, ta, **kw).to(DEV), cb.Model.build(vb, tb, **kw).to(DEV)
    return _cache[key]


@pytest.mark.parametrize("bits", [8, 16, 0])
@pytest.mark.parametrize("cfg,tb", [(0, 0), (0, 1024), (2, 0)])
def test_obb_decode_all_bit_exact(cfg, tb, bits):
    _log(f"obb decode cfg={cfg} treelet={tb} bits={bits}")
    for m in obb_models(cfg, bits, treelet_bytes=tb):
        got = m.decode_all().cpu().numpy()
        ref = oracle.blob_decode(m.blob())
        assert got.shape == ref.shape == (m.info()["n_nodes"], cb.OBB_WORDS)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


@pytest.mark.parametrize("bits", [8, 16, 0])
def test_obb_tiny_pairs_and_booleans_match_oracle(bits):
    P, _ = W.config0_poses()
    A, B = W.oracle_meshes(0)
    ma, mb = obb_models(0, bits)
    Pd = torch.from_numpy(P).to(DEV)
    _log(f"obb tiny pairs bits={bits}")
    hit, st, pairs, offs = cb.collide(ma, mb, Pd, flags=cb.PAIRS, pair_capacity=1 << 18)
    hit2, st2 = cb.collide(ma, mb, Pd, flags=cb.EARLY_EXIT)
    torch.cuda.synchronize()
    hit, st, pairs, offs = (x.cpu().numpy() for x in (hit, st, pairs, offs))
    assert (st == 0).all() and (st2.cpu().numpy() == 0).all()
    for i, p in enumerate(P):
        ref = oracle.collide_pairs(A, B, p)
        seg = pairs[offs[i]:offs[i + 1]]
        assert (seg[:, 0] == i).all()
        assert np.array_equal(seg[:, 1:].astype(np.uint32), ref), f"pose {i}"
        assert bool(hit[i]) == (len(ref) > 0)
    ref, _ = oracle.collide_batch(A, B, P)
    assert np.array_equal(hit2.cpu().numpy().astype(bool), ref)
    assert ref.sum() == 128


def _near_touching(n, seed):
    rng = np.random.default_rng(seed)
    (va, ta), (vb, tb) = W.meshes(0)
    A, B = W.oracle_meshes(0)
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    R = poses.uniform_rotations(n, rng)
    d0, _ = oracle.distance_batch(A, B, poses.compose(R, u * 2.4))
    gap = np.exp(rng.uniform(np.log(1e-3), np.log(0.3), size=n))
    gap[-32:] = -0.02
    return poses.compose(R, u * (2.4 - d0 + gap)[:, None])


def _check_against_oracle(P, d, st, hit=None, hst=None):
    (va, _), (vb, _) = W.meshes(0)
    A, B = W.oracle_meshes(0)
    cls = oracle.classify_batch(A, B, P, configs.WORKLOADS[0].margin(va, vb))
    ref, _ = oracle.distance_batch(A, B, P)
    sep, col = cls == oracle.SEPARATED, cls == oracle.COLLIDING
    assert sep.sum() > 30 and col.sum() > 5
    assert (st.cpu().numpy() == 0).all()
    got = d.cpu().numpy().astype(np.float64)
    rel = np.abs(got[sep] - ref[sep]) / ref[sep]
    assert rel.max() <= 1e-5, (rel.max(), np.nonzero(sep)[0][np.argmax(rel)])
    assert (got[col] == 0).all()
    if hit is not None:
        assert (hst.cpu().numpy() == 0).all()
        h = hit.cpu().numpy().astype(bool)
        assert np.array_equal(h[sep | col], col[sep | col])


@pytest.mark.parametrize("bits", [16, 0])
def test_obb_near_touching_distances_match_oracle(bits):
    _log(f"obb near-touching distances bits={bits}")
    P = _near_touching(256, 2012)
    ma, mb = obb_models(0, bits, branching=4, leaf_size=1, treelet_bytes=1024)
    d, st = cb.distance(ma, mb, torch.from_numpy(P).to(DEV))
    _check_against_oracle(P, d, st)


def test_obb_non_rigid_pose_matrices_match_oracle():
    _log("obb non-rigid poses")
    rng = np.random.default_rng(5150)
    n = 96
    R = poses.uniform_rotations(n, rng)
    D = np.eye(3)[None] + rng.uniform(-2e-3, 2e-3, size=(n, 3, 3))
    P = poses.compose(R @ D, poses.shell_translations(n, 1.6, 3.0, rng))
    ma, mb = obb_models(0, 8)
    Pd = torch.from_numpy(P).to(DEV)
    d, st = cb.distance(ma, mb, Pd)
    hit, hst = cb.collide(ma, mb, Pd, flags=cb.EARLY_EXIT)
    _check_against_oracle(P, d, st, hit, hst)


def test_obb_small_stacks_hand_over_work_and_keep_pairs_exact():
    P, _ = W.config0_poses()
    A, B = W.oracle_meshes(0)
    ma, mb = obb_models(0, 16)
    Pd = torch.from_numpy(P).to(DEV)
    try:
        cb.cbvh_set_stack_limits(entries=128, records=96)
        ws = cb.workspace(ma, mb, len(P), cb.PAIRS, 1 << 18)
        hit, st, pairs, offs = cb.collide(ma, mb, Pd, flags=cb.PAIRS, pair_capacity=1 << 18, ws=ws)
        stats = cb.cbvh_stats(ws.buf)
        d, dst = cb.distance(ma, mb, torch.from_numpy(_near_touching(128, 7)).to(DEV))
    finally:
        cb.cbvh_set_stack_limits(0, 0)
    _log(f"obb small stacks: {stats}")
    assert stats["donated_items"] > 0
    st, pairs, offs = st.cpu().numpy(), pairs.cpu().numpy(), offs.cpu().numpy()
    assert (st == 0).all()
    for i, p in enumerate(P):
        assert np.array_equal(pairs[offs[i]:offs[i + 1], 1:].astype(np.uint32), oracle.collide_pairs(A, B, p))
    _check_against_oracle(_near_touching(128, 7), d, dst)


def test_obb_scaled_booleans_equal_dop18_and_oracle():
    w = configs.WORKLOADS[1]
    P = w.raw_poses()
    Pd = torch.from_numpy(P).to(DEV)
    (va, ta), (vb, tb) = W.meshes(1)
    _log("obb scaled: building models")
    kw = dict(branching=w.branching, leaf_size=w.leaf_size, bits=w.bits)
    mo = [cb.Model.build(v, t, bv=cb.OBB, **kw).to(DEV) for v, t in ((va, ta), (vb, tb))]
    md = [cb.Model.build(v, t, bv=cb.DOP18, **kw).to(DEV) for v, t in ((va, ta), (vb, tb))]
    _log("obb scaled: collide")
    ho, so = cb.collide(mo[0], mo[1], Pd, flags=cb.EARLY_EXIT)
    hd, sd = cb.collide(md[0], md[1], Pd, flags=cb.EARLY_EXIT)
    ho, hd = ho.cpu().numpy().astype(bool), hd.cpu().numpy().astype(bool)
    assert (so.cpu().numpy() == 0).all() and (sd.cpu().numpy() == 0).all()
    assert np.array_equal(ho, hd)
    A, B = W.oracle_meshes(1)
    idx = np.random.default_rng(1).choice(len(P), 512, replace=False)
    cls = oracle.classify_batch(A, B, P[idx], w.margin(va, vb))
    ok = cls != oracle.MARGINAL
    ref, _ = oracle.collide_batch(A, B, P[idx][ok])
    assert ok.sum() > 400
    assert np.array_equal(ho[idx][ok], ref)


def test_obb_proximity_distances_equal_aabb_on_every_pose():
    """The proximity workload (4,096 poses, 50k-triangle meshes, branching 4,
    8-bit codes) as OBB models: every pose completes and its distance is
    bit-identical to the AABB models' (which the oracle checks on every pose
    in the parity suite)."""
    w = configs.WORKLOADS[2]
    P = torch.from_numpy(w.raw_poses()).to(DEV)
    (va, ta), (vb, tb) = W.meshes(2)
    kw = dict(branching=w.branching, leaf_size=w.leaf_size, bits=w.bits)
    mo = [cb.Model.build(v, t, bv=cb.OBB, **kw).to(DEV) for v, t in ((va, ta), (vb, tb))]
    ma = [cb.Model.build(v, t, bv=cb.AABB, **kw).to(DEV) for v, t in ((va, ta), (vb, tb))]
    _log("obb proximity distances")
    do, so = cb.distance(mo[0], mo[1], P)
    da, sa = cb.distance(ma[0], ma[1], P)
    assert (so.cpu().numpy() == 0).all() and (sa.cpu().numpy() == 0).all()
    assert np.array_equal(do.cpu().numpy().view(np.uint32), da.cpu().numpy().view(np.uint32))


def test_obb_batched_queries_equal_plain_queries():
    """A moving OBB model against an obstacle set of OBB models of uneven
    size in one launch (items of other poses carry their own obstacle's
    frames): booleans and distances equal the plain per-obstacle queries,
    and the allocation-free entry point's booleans equal the plain ones."""
    w = configs.BatchedWorkload(n_obstacles=6, tri_max=20000, min_poses=1500)
    kw = dict(bv=cb.OBB, branching=w.branching, leaf_size=w.leaf_size, bits=w.bits)
    link = cb.Model.build(*w.link_mesh(), **kw).to(DEV)
    obs = [cb.Model.build(*w.obstacle_mesh(i), **kw).to(DEV) for i in range(w.n_obstacles)]
    P, obj = w.raw_poses()
    Pd, od = torch.from_numpy(P).to(DEV), torch.from_numpy(obj.astype(np.int32)).to(DEV)
    oset = cb.Obstacles(obs, DEV)
    _log(f"obb batched: {len(obs)} obstacles, {len(P)} poses")
    hit, st = cb.collide_batch(link, oset, Pd, od)
    sel = np.arange(0, len(P), 3)
    d, dst = cb.distance_batch(link, oset, torch.from_numpy(P[sel]).to(DEV),
                               torch.from_numpy(obj[sel].astype(np.int32)).to(DEV))
    assert (st.cpu().numpy() == 0).all() and (dst.cpu().numpy() == 0).all()
    hit, d = hit.cpu().numpy(), d.cpu().numpy()
    assert 0 < hit.sum() < len(hit)
    for k, m in enumerate(obs):
        idx = np.nonzero(obj == k)[0]
        if len(idx) == 0:
            continue
        h, hs = cb.collide(link, m, torch.from_numpy(P[idx]).to(DEV))
        assert (hs.cpu().numpy() == 0).all()
        assert np.array_equal(hit[idx], h.cpu().numpy())
        n = len(idx)
        hst = torch.empty(n, dtype=torch.uint8, device=DEV)
        sst = torch.empty(n, dtype=torch.uint8, device=DEV)
        cb.cbvh_collide_static(link.handle, link.dev, m.handle, m.dev, torch.from_numpy(P[idx]).to(DEV), n,
                               cb.EARLY_EXIT, hst, sst)
        torch.cuda.synchronize()
        assert (sst.cpu().numpy() == 0).all()
        assert np.array_equal(hst.cpu().numpy(), h.cpu().numpy())
        ids = np.nonzero(obj[sel] == k)[0]
        if len(ids):
            dd, ds = cb.distance(link, m, torch.from_numpy(P[sel][ids]).to(DEV))
            assert (ds.cpu().numpy() == 0).all()
            assert np.array_equal(d[ids].view(np.uint32), dd.cpu().numpy().view(np.uint32))
