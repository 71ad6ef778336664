"""GPU parity tests: the HIP path (through the C ABI) against the FP64 oracle.

- decode: every node's decoded bounds bit-identical to the oracle's decoder;
- tiny workload (1,280 vs 1,280 triangles, AABB BF4 leaf 1, 8-bit and FP32):
  booleans and sorted colliding-pair lists equal the oracle's on all 256
  margin-filtered poses;
- scaled workload (100k-triangle tori, 18-DOP BF8 leaf 4, 16-bit and FP32):
  all 16,384 poses in one launch; booleans equal the oracle's on every pose
  the pose-level margin accepts; compressed == uncompressed on all;
- proximity workload (50k icosphere vs 50k torus, AABB BF4 leaf 1, 8-bit and
  FP32): distances within 1e-5 relative of the oracle on every separated
  pose, zero on every colliding one; compressed and uncompressed
  bit-identical on all; the same meshes as 18-DOP models (16-bit, binary16,
  FP32) against the oracle on every pose too;
- near-touching poses offset along random directions (AABB and 18-DOP):
  distances equal the oracle's, so no distance bound overshoots;
- failure paths forced from the host (tiny stack, tiny pair buffer), empty
  and degenerate inputs, determinism.
"""
import sys

import numpy as np
import pytest

import oracle
import workloads as W
from synth import configs, meshes, poses

torch = pytest.importorskip("torch")
cb = pytest.importorskip("paper_2012_05348_amd")

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _models(cfg, compressed=True, **over):
    w = configs.WORKLOADS[cfg]
    (va, ta), (vb, tb) = W.meshes(cfg)
    # compressed: True = corrector codes, False = FP32, "fp16" = half-precision descriptors
    bits = cb.BITS_FP16 if compressed == "fp16" else (w.bits if compressed else 0)
    kw = dict(bv=W.BV[w.bv], branching=w.branching, leaf_size=w.leaf_size, bits=bits)
    kw.update(over)
    return cb.Model.build(va, ta, **kw).to(DEV), cb.Model.build(vb, tb, **kw).to(DEV)


_model_cache = {}


def models(cfg, compressed=True):
    key = (cfg, compressed)
    if key not in _model_cache:
        _model_cache[key] = _models(cfg, compressed)
    return _model_cache[key]


# ---------------------------------------------------------------- decode
@pytest.mark.parametrize("cfg", [0, 1, 2])
@pytest.mark.parametrize("compressed", [True, False, "fp16"])
def test_decode_all_bit_exact(cfg, compressed):
    _log(f"decode cfg={cfg} compressed={compressed}")
    for m in models(cfg, compressed):
        got = m.decode_all().cpu().numpy()
        ref = oracle.blob_decode(m.blob())
        assert got.shape == ref.shape
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))


# ---------------------------------------------------------------- tiny workload
def _pairs_per_pose(pairs, offs, n):
    return [pairs[offs[i]:offs[i + 1]] for i in range(n)]


@pytest.mark.parametrize("compressed", [True, False, "fp16"])
def test_tiny_pairs_match_oracle(compressed):
    P, _ = W.config0_poses()
    A, B = W.oracle_meshes(0)
    ma, mb = models(0, compressed)
    _log(f"tiny pairs compressed={compressed}")
    hit, st, pairs, offs = cb.collide(ma, mb, torch.from_numpy(P).to(DEV), flags=cb.PAIRS, pair_capacity=1 << 18)
    torch.cuda.synchronize()
    hit, st, pairs, offs = (x.cpu().numpy() for x in (hit, st, pairs, offs))
    assert (st == 0).all()
    assert offs[0] == 0 and (np.diff(offs) >= 0).all()
    n_hit = 0
    for i, p in enumerate(P):
        ref = oracle.collide_pairs(A, B, p)
        seg = pairs[offs[i]:offs[i + 1]]
        assert (seg[:, 0] == i).all()
        assert np.array_equal(seg[:, 1:].astype(np.uint32), ref), f"pose {i}"
        assert bool(hit[i]) == (len(ref) > 0)
        n_hit += bool(hit[i])
    assert n_hit == 128


@pytest.mark.parametrize("compressed", [True, False])
def test_tiny_booleans_match_oracle(compressed):
    P, _ = W.config0_poses()
    A, B = W.oracle_meshes(0)
    ma, mb = models(0, compressed)
    hit, st = cb.collide(ma, mb, torch.from_numpy(P).to(DEV), flags=cb.EARLY_EXIT)
    ref, _ = oracle.collide_batch(A, B, P)
    assert (st.cpu().numpy() == 0).all()
    assert np.array_equal(hit.cpu().numpy().astype(bool), ref)


# ---------------------------------------------------------------- scaled workload
@pytest.fixture(scope="module")
def scaled_results():
    w = configs.WORKLOADS[1]
    P = w.raw_poses()
    Pd = torch.from_numpy(P).to(DEV)
    out = {}
    for compressed in (True, False, "fp16"):
        ma, mb = models(1, compressed)
        _log(f"scaled collide compressed={compressed}")
        ws = cb.workspace(ma, mb, len(P))
        hit, st = cb.collide(ma, mb, Pd, flags=cb.EARLY_EXIT, ws=ws)
        stats = cb.cbvh_stats(ws.buf)
        out[compressed] = (hit.cpu().numpy(), st.cpu().numpy(), stats)
    return P, out


def test_scaled_booleans_match_oracle_on_every_pose(scaled_results):
    """Every one of the 16,384 poses that the pose-level margin accepts (all
    but a handful) against the oracle, for the three descriptor formats."""
    P, out = scaled_results
    w = configs.WORKLOADS[1]
    (va, ta), (vb, tb) = W.meshes(1)
    A, B = W.oracle_meshes(1)
    _log("scaled: oracle classification and booleans of every pose")
    cls = oracle.classify_batch(A, B, P, w.margin(va, vb))
    keep = np.nonzero(cls != oracle.MARGINAL)[0]
    assert len(keep) > len(P) - 64
    ref, _ = oracle.collide_batch(A, B, P[keep])
    assert np.array_equal(ref, cls[keep] == oracle.COLLIDING)
    for compressed in (True, False, "fp16"):
        hit, st, _ = out[compressed]
        assert (st == 0).all()
        bad = np.nonzero(hit[keep].astype(bool) != ref)[0]
        assert len(bad) == 0, (compressed, keep[bad[:10]])
    assert 0 < ref.sum() < len(ref)


def test_scaled_compressed_equals_uncompressed(scaled_results):
    _, out = scaled_results
    assert np.array_equal(out[True][0], out[False][0])
    assert np.array_equal(out["fp16"][0], out[False][0])
    sc, su = out[True][2], out[False][2]
    assert sc["bv_tests"] > 0 and su["bv_tests"] > 0
    _log(f"scaled stats compressed={sc} uncompressed={su}")


# ---------------------------------------------------------------- proximity workload
@pytest.fixture(scope="module")
def proximity_results():
    w = configs.WORKLOADS[2]
    P = w.raw_poses()
    Pd = torch.from_numpy(P).to(DEV)
    out = {}
    for compressed in (True, False, "fp16"):
        ma, mb = models(2, compressed)
        _log(f"proximity distance compressed={compressed}")
        ws = cb.workspace(ma, mb, len(P))
        d, st = cb.distance(ma, mb, Pd, ws=ws)
        out[compressed] = (d.cpu().numpy(), st.cpu().numpy(), cb.cbvh_stats(ws.buf))
    return P, out


@pytest.fixture(scope="module")
def proximity_oracle():
    """The oracle's distance and margin class of every proximity pose."""
    w = configs.WORKLOADS[2]
    (va, ta), (vb, tb) = W.meshes(2)
    A, B = W.oracle_meshes(2)
    P = w.raw_poses()
    _log("proximity: oracle distances of every pose")
    cls = oracle.classify_batch(A, B, P, w.margin(va, vb))
    ref, _ = oracle.distance_batch(A, B, P)
    return P, cls, ref


def _check_distances(got, cls, ref, what):
    sep, col = cls == oracle.SEPARATED, cls == oracle.COLLIDING
    got = got.astype(np.float64)
    rel = np.abs(got[sep] - ref[sep]) / ref[sep]
    assert rel.max() <= 1e-5, (what, rel.max(), np.nonzero(sep)[0][np.argmax(rel)])
    assert (got[col] == 0).all(), (what, np.nonzero(col & (got != 0))[0][:10])


def test_proximity_distances_match_oracle_on_every_pose(proximity_results, proximity_oracle):
    P, out = proximity_results
    _, cls, ref = proximity_oracle
    assert (cls == oracle.SEPARATED).sum() > 3500 and (cls == oracle.MARGINAL).sum() < 16
    for compressed in (True, False, "fp16"):
        d, st, _ = out[compressed]
        assert (st == 0).all()
        _check_distances(d, cls, ref, compressed)


def test_proximity_compressed_equals_uncompressed(proximity_results):
    _, out = proximity_results
    assert np.array_equal(out[True][0].view(np.uint32), out[False][0].view(np.uint32))
    assert np.array_equal(out["fp16"][0].view(np.uint32), out[False][0].view(np.uint32))
    _log(f"proximity stats compressed={out[True][2]} uncompressed={out[False][2]}")


def test_proximity_dop18_distances_match_oracle_on_every_pose(proximity_oracle):
    """The proximity meshes as 18-DOP models (BF 8, leaf 4; the slab gaps then
    join the sphere and directional gaps in the distance bound): distances
    within 1e-5 relative of the oracle on every separated pose, zero on
    colliding ones, and the 16-bit, binary16 and FP32 descriptors bit-identical."""
    (va, ta), (vb, tb) = W.meshes(2)
    P, cls, ref = proximity_oracle
    got = {}
    for bits in (16, cb.BITS_FP16, 0):
        _log(f"proximity dop18 distance bits={bits}")
        kw = dict(bv=cb.DOP18, branching=8, leaf_size=4, bits=bits)
        ma, mb = cb.Model.build(va, ta, **kw).to(DEV), cb.Model.build(vb, tb, **kw).to(DEV)
        d, st = cb.distance(ma, mb, torch.from_numpy(P).to(DEV))
        assert (st.cpu().numpy() == 0).all()
        got[bits] = d.cpu().numpy()
        _check_distances(got[bits], cls, ref, bits)
    assert np.array_equal(got[16].view(np.uint32), got[0].view(np.uint32))
    assert np.array_equal(got[cb.BITS_FP16].view(np.uint32), got[0].view(np.uint32))


@pytest.mark.parametrize("bv", ["aabb", "dop18"])
def test_near_touching_poses_in_every_direction_match_oracle(bv):
    """Two 1,280-triangle icospheres placed almost touching, offset along
    uniformly random directions (so the BV pairs near contact are offset
    diagonally, where a distance bound along fixed axes is weakest and a
    bound that overshoots the true distance would prune the closest pair):
    distances within 1e-5 relative of the oracle, zero where they collide."""
    _log(f"near-touching distances bv={bv}")
    rng = np.random.default_rng(2012)
    (va, ta), (vb, tb) = W.meshes(0)
    A, B = W.oracle_meshes(0)
    n = 256
    u = rng.normal(size=(n, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    R = poses.uniform_rotations(n, rng)
    # at an offset of 2.4 the spheres (radii 0.9-1.1) are apart by d0; moving
    # A closer by d0 - gap leaves them at least `gap` apart (the distance is
    # 1-Lipschitz in the offset), near contact for convex-ish shapes; the
    # last 32 poses go 0.02 past that and mostly collide
    d0, _ = oracle.distance_batch(A, B, poses.compose(R, u * 2.4))
    gap = np.exp(rng.uniform(np.log(1e-3), np.log(0.3), size=n))
    gap[-32:] = -0.02
    P = poses.compose(R, u * (2.4 - d0 + gap)[:, None])
    if bv == "aabb":
        kw = dict(bv=cb.AABB, branching=4, leaf_size=1, bits=8)
    else:
        kw = dict(bv=cb.DOP18, branching=8, leaf_size=4, bits=16)
    ma, mb = cb.Model.build(va, ta, **kw).to(DEV), cb.Model.build(vb, tb, **kw).to(DEV)
    d, st = cb.distance(ma, mb, torch.from_numpy(P).to(DEV))
    cls = oracle.classify_batch(A, B, P, configs.WORKLOADS[0].margin(va, vb))
    ref, _ = oracle.distance_batch(A, B, P)
    sep, col = cls == oracle.SEPARATED, cls == oracle.COLLIDING
    assert sep.sum() > 150 and col.sum() > 5 and np.median(ref[sep]) < 0.05
    assert (st.cpu().numpy() == 0).all()
    got = d.cpu().numpy().astype(np.float64)
    rel = np.abs(got[sep] - ref[sep]) / ref[sep]
    assert rel.max() <= 1e-5, (rel.max(), np.nonzero(sep)[0][np.argmax(rel)])
    assert (got[col] == 0).all()


# ---------------------------------------------------------------- edge cases and failure paths
def test_empty_batch_is_a_noop():
    ma, mb = models(0)
    P = torch.zeros((0, 3, 4), dtype=torch.float32, device=DEV)
    hit, st = cb.collide(ma, mb, P)
    assert hit.numel() == 0


def test_single_triangle_meshes():
    a = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], dtype=np.float32)
    t = np.array([[0, 1, 2]], dtype=np.uint32)
    ma = cb.Model.build(a, t, bits=8).to(DEV)
    mb = cb.Model.build(a, t, bits=8).to(DEV)
    # B's triangle pierced by A's triangle turned upright / A lifted clear of B
    up = np.array([[1, 0, 0, 0.2], [0, 0, -1, 0.2], [0, 1, 0, -0.5]], dtype=np.float32)
    lift = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0.25]], dtype=np.float32)
    P = np.stack([up, lift])
    hit, st = cb.collide(ma, mb, torch.from_numpy(P).to(DEV))
    d, dst = cb.distance(ma, mb, torch.from_numpy(P).to(DEV))
    assert hit.cpu().tolist() == [1, 0]
    dd = d.cpu().numpy()
    assert dd[0] == 0.0 and abs(dd[1] - 0.25) <= 1e-6
    A, B = oracle.Mesh(a, t), oracle.Mesh(a, t)
    assert oracle.collide(A, B, up)[0] and not oracle.collide(A, B, lift)[0]


def test_small_stacks_donate_work_and_keep_answers_exact():
    P, _ = W.config0_poses()
    A, B = W.oracle_meshes(0)
    ma, mb = models(0)
    Pd = torch.from_numpy(P).to(DEV)
    try:
        cb.cbvh_set_stack_limits(entries=128, records=96)
        ws = cb.workspace(ma, mb, len(P), cb.PAIRS, 1 << 18)
        hit, st, pairs, offs = cb.collide(ma, mb, Pd, flags=cb.PAIRS, pair_capacity=1 << 18, ws=ws)
        stats = cb.cbvh_stats(ws.buf)
        ws2 = cb.workspace(ma, mb, len(P))
        hit2, st2 = cb.collide(ma, mb, Pd, flags=cb.EARLY_EXIT, ws=ws2)
        hit3, st3 = cb.collide(ma, mb, Pd, flags=cb.EARLY_EXIT | cb.NO_SPLIT)
    finally:
        cb.cbvh_set_stack_limits(0, 0)
    _log(f"small stacks: {stats}")
    assert stats["donated_items"] > 0
    st, pairs, offs = st.cpu().numpy(), pairs.cpu().numpy(), offs.cpu().numpy()
    assert (st == 0).all()
    for i, p in enumerate(P):
        assert np.array_equal(pairs[offs[i]:offs[i + 1], 1:].astype(np.uint32), oracle.collide_pairs(A, B, p))
    ref, _ = oracle.collide_batch(A, B, P)
    assert (st2.cpu().numpy() == 0).all()
    assert np.array_equal(hit2.cpu().numpy().astype(bool), ref)
    # without donation, poses that outgrow the small stacks are flagged; the others stay exact
    st3 = st3.cpu().numpy()
    ok = st3 == 0
    assert np.array_equal(hit3.cpu().numpy()[ok].astype(bool), ref[ok])
    assert set(np.unique(st3)) <= {0, cb.POSE_STACK_OVERFLOW}


def test_split_and_unsplit_runs_agree():
    w = configs.WORKLOADS[2]
    P = torch.from_numpy(w.raw_poses(512)).to(DEV)
    ma, mb = models(2)
    d1, s1 = cb.distance(ma, mb, P)
    d2, s2 = cb.distance(ma, mb, P, flags=cb.NO_SPLIT)
    ok = (s1.cpu().numpy() == 0) & (s2.cpu().numpy() == 0)
    assert ok.mean() > 0.99
    assert np.array_equal(d1.cpu().numpy()[ok].view(np.uint32), d2.cpu().numpy()[ok].view(np.uint32))


def test_pair_buffer_overflow_is_flagged_per_pose():
    P, _ = W.config0_poses()
    A, B = W.oracle_meshes(0)
    ma, mb = models(0)
    cap = 500
    hit, st, pairs, offs = cb.collide(ma, mb, torch.from_numpy(P).to(DEV), flags=cb.PAIRS, pair_capacity=cap)
    st, pairs, offs = st.cpu().numpy(), pairs.cpu().numpy(), offs.cpu().numpy()
    assert (st == cb.POSE_PAIR_OVERFLOW).any()
    assert offs[-1] <= cap
    for i, p in enumerate(P):
        if st[i] == 0:
            assert np.array_equal(pairs[offs[i]:offs[i + 1], 1:].astype(np.uint32), oracle.collide_pairs(A, B, p))


def test_results_do_not_depend_on_batch_composition():
    w = configs.WORKLOADS[1]
    P = w.raw_poses(2048)
    ma, mb = models(1)
    full, _ = cb.collide(ma, mb, torch.from_numpy(P).to(DEV))
    part, _ = cb.collide(ma, mb, torch.from_numpy(P[::7].copy()).to(DEV))
    again, _ = cb.collide(ma, mb, torch.from_numpy(P).to(DEV))
    assert np.array_equal(full.cpu().numpy()[::7], part.cpu().numpy())
    assert np.array_equal(full.cpu().numpy(), again.cpu().numpy())


@pytest.mark.parametrize("bv", ["aabb", "dop18"])
def test_non_rigid_pose_matrices_match_oracle(bv):
    """The BV bounds allow for a pose matrix that is not a rotation (its
    columns' Gram matrix is measured per pose), so distances and booleans
    still match the oracle, which applies the matrix as given."""
    _log(f"non-rigid poses bv={bv}")
    rng = np.random.default_rng(5150)
    (va, ta), (vb, tb) = W.meshes(0)
    n = 96
    R = poses.uniform_rotations(n, rng)
    # stretch and shear: the columns are off orthonormal by up to about 4e-3
    D = np.eye(3)[None] + rng.uniform(-2e-3, 2e-3, size=(n, 3, 3))
    t = poses.shell_translations(n, 1.6, 3.0, rng)
    P = poses.compose(R @ D, t)
    kw = dict(bv=cb.AABB if bv == "aabb" else cb.DOP18, branching=4, leaf_size=1, bits=8)
    ma, mb = cb.Model.build(va, ta, **kw).to(DEV), cb.Model.build(vb, tb, **kw).to(DEV)
    Pd = torch.from_numpy(P).to(DEV)
    d, st = cb.distance(ma, mb, Pd)
    hit, hst = cb.collide(ma, mb, Pd, flags=cb.EARLY_EXIT)
    A, B = W.oracle_meshes(0)
    cls = oracle.classify_batch(A, B, P, configs.WORKLOADS[0].margin(va, vb))
    ref, _ = oracle.distance_batch(A, B, P)
    sep, col = cls == oracle.SEPARATED, cls == oracle.COLLIDING
    assert sep.sum() > 30 and col.sum() > 5
    assert (st.cpu().numpy() == 0).all() and (hst.cpu().numpy() == 0).all()
    got = d.cpu().numpy().astype(np.float64)
    rel = np.abs(got[sep] - ref[sep]) / ref[sep]
    assert rel.max() <= 1e-5, rel.max()
    assert (got[col] == 0).all()
    h = hit.cpu().numpy().astype(bool)
    assert np.array_equal(h[sep | col], col[sep | col])


@pytest.mark.parametrize("bits", [8, 0])
def test_coincident_and_degenerate_geometry_match_oracle(bits):
    """Degenerate inputs the method has to decide exactly: a model against
    itself at the identity pose (every triangle coincides with itself and
    touches its neighbours along shared edges and vertices: coplanar and
    touching pairs, all decided by the FP64 stage), and a mesh with
    zero-area triangles.  Pair lists, booleans and distances equal the
    oracle's."""
    _log(f"coincident geometry bits={bits}")
    (va, ta), _ = W.meshes(0)
    m = cb.Model.build(va, ta, bv=cb.AABB, branching=4, leaf_size=1, bits=bits).to(DEV)
    A = oracle.Mesh(va, ta)
    P = np.eye(3, 4, dtype=np.float32)[None]
    Pd = torch.from_numpy(P).to(DEV)
    cap = 1 << 16
    hit, st, pairs, offs = cb.collide(m, m, Pd, flags=cb.PAIRS, pair_capacity=cap)
    assert st.cpu().numpy()[0] == 0 and hit.cpu().numpy()[0] == 1
    got = pairs.cpu().numpy()[: offs.cpu().numpy()[1], 1:].astype(np.uint32)
    ref = oracle.collide_pairs(A, A, P[0])
    assert len(ref) > len(ta)  # every triangle with itself, plus its neighbours
    assert np.array_equal(got, ref)
    d, dst = cb.distance(m, m, Pd)
    assert dst.cpu().numpy()[0] == 0 and d.cpu().numpy()[0] == 0.0
    # zero-area triangles (a collapsed vertex and a collapsed edge) among ordinary ones
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0], [1, 1, 0], [0.5, 0.5, 0.5]], np.float32)
    T = np.array([[0, 1, 2], [1, 3, 2], [3, 4, 1], [0, 5, 5], [2, 5, 1]], np.uint32)
    md = cb.Model.build(V, T, bv=cb.AABB, branching=4, leaf_size=1, bits=bits).to(DEV)
    D = oracle.Mesh(V, T)
    rng = np.random.default_rng(99)
    Q = poses.compose(poses.uniform_rotations(64, rng), poses.shell_translations(64, 0.0, 1.5, rng))
    Qd = torch.from_numpy(Q).to(DEV)
    hit, st, pairs, offs = cb.collide(md, md, Qd, flags=cb.PAIRS, pair_capacity=cap)
    d, dst = cb.distance(md, md, Qd)
    st, pairs, offs, d = st.cpu().numpy(), pairs.cpu().numpy(), offs.cpu().numpy(), d.cpu().numpy()
    assert (st == 0).all() and (dst.cpu().numpy() == 0).all()
    ref_d, _ = oracle.distance_batch(D, D, Q)
    for i, q in enumerate(Q):
        assert np.array_equal(pairs[offs[i]:offs[i + 1], 1:].astype(np.uint32), oracle.collide_pairs(D, D, q)), i
    pos = ref_d > 0
    assert (d[~pos] == 0).all()
    assert (np.abs(d[pos] - ref_d[pos]) / ref_d[pos]).max() <= 1e-5


def test_large_batch_keeps_every_pose_within_capacity():
    """A batch of 262,144 poses in one launch (sixteen times the scaled
    workload's): no pose overflows a queue or buffer, compressed and FP32
    descriptors agree on every pose, and every pose the margin accepts
    matches the oracle."""
    n = 1 << 18
    rng = np.random.default_rng(262144)
    P = poses.compose(poses.uniform_rotations(n, rng), poses.box_translations(n, 2.5, rng))
    Pd = torch.from_numpy(P).to(DEV)
    _log(f"large batch n={n}")
    out = {}
    for compressed in (True, False):
        ma, mb = models(0, compressed)
        hit, st = cb.collide(ma, mb, Pd, flags=cb.EARLY_EXIT)
        out[compressed] = (hit.cpu().numpy().astype(bool), st.cpu().numpy())
        assert (out[compressed][1] == 0).all()
    assert np.array_equal(out[True][0], out[False][0])
    (va, ta), (vb, tb) = W.meshes(0)
    A, B = W.oracle_meshes(0)
    cls = oracle.classify_batch(A, B, P, configs.WORKLOADS[0].margin(va, vb))
    ok = cls != oracle.MARGINAL
    assert ok.sum() > n - 1024
    ref, _ = oracle.collide_batch(A, B, P[ok])
    assert np.array_equal(ref, cls[ok] == oracle.COLLIDING)
    bad = np.nonzero(out[True][0][ok] != ref)[0]
    assert len(bad) == 0, np.nonzero(ok)[0][bad[:10]]


def test_concurrent_launches_on_several_streams_neither_wait_nor_change_answers():
    """Four queries in flight at once on four streams (two distance, two
    collision launches, each sized to fill the GPU on its own), so a launch's
    waves cannot all be resident: waiting waves must not wait on waves that
    have not started (no wait-limit timeouts), and every answer equals the
    same query run alone."""
    wd, wc = configs.WORKLOADS[2], configs.WORKLOADS[1]
    Pd_ = torch.from_numpy(wd.raw_poses()).to(DEV)
    Pc_ = torch.from_numpy(wc.raw_poses()).to(DEV)
    md, mc = models(2), models(1)
    ref_d, _ = cb.distance(*md, Pd_)
    ref_c, _ = cb.collide(*mc, Pc_)
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in range(4)]
    jobs = []
    for i, s in enumerate(streams):
        kind = "dist" if i % 2 == 0 else "coll"
        m, P = (md, Pd_) if kind == "dist" else (mc, Pc_)
        n = P.shape[0]
        ws = cb.workspace(m[0], m[1], n, 0 if kind == "dist" else cb.EARLY_EXIT, 0, DEV)
        out = torch.empty(n, dtype=torch.float32 if kind == "dist" else torch.uint8, device=DEV)
        st = torch.empty(n, dtype=torch.uint8, device=DEV)
        jobs.append((kind, s, m, P, n, ws, out, st))
    import time
    t0 = time.perf_counter()
    for kind, s, m, P, n, ws, out, st in jobs:
        if kind == "dist":
            cb.cbvh_distance(m[0].handle, m[0].dev, m[1].handle, m[1].dev, P, n, 0, out, st, ws.buf, stream=s)
        else:
            cb.cbvh_collide(m[0].handle, m[0].dev, m[1].handle, m[1].dev, P, n, cb.EARLY_EXIT, out, None, 0, None,
                            st, ws.buf, stream=s)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    _log(f"concurrent launches: {dt * 1e3:.1f} ms")
    assert dt < 2.0
    for kind, s, m, P, n, ws, out, st in jobs:
        stats = cb.cbvh_stats(ws.buf)
        assert stats["wait_timeouts"] == 0
        assert (st.cpu().numpy() == 0).all()
        ref = ref_d if kind == "dist" else ref_c
        assert torch.equal(out.cpu(), ref.cpu())


def test_eight_collision_launches_in_flight_with_few_helpers_keep_answers():
    """The bench's pipelined setting: eight scaled collision launches in
    flight on eight streams, each with 6 waves per CU and 32 helper waves for
    the whole GPU; every launch's booleans equal the lone launch's, with no
    wait-limit timeout."""
    from paper_2012_05348_amd import autotune
    wc = configs.WORKLOADS[1]
    P = torch.from_numpy(wc.raw_poses()).to(DEV)
    mc = models(1)
    ref, _ = cb.collide(*mc, P)
    torch.cuda.synchronize()
    n = P.shape[0]
    streams = [torch.cuda.Stream() for _ in range(8)]
    sets = [(cb.workspace(mc[0], mc[1], n, cb.EARLY_EXIT, 0, DEV), torch.empty(n, dtype=torch.uint8, device=DEV),
             torch.empty(n, dtype=torch.uint8, device=DEV)) for _ in streams]
    with autotune.launch_env({"max_helpers": 32, "waves_per_cu": 6}):
        for r in range(3):
            for s, (ws, out, st) in zip(streams, sets):
                cb.cbvh_collide(mc[0].handle, mc[0].dev, mc[1].handle, mc[1].dev, P, n, cb.EARLY_EXIT, out, None, 0,
                                None, st, ws.buf, stream=s)
        torch.cuda.synchronize()
    for ws, out, st in sets:
        assert cb.cbvh_stats(ws.buf)["wait_timeouts"] == 0
        assert (st.cpu().numpy() == 0).all()
        assert torch.equal(out.cpu(), ref.cpu())


@pytest.mark.parametrize("query", ["collide", "distance"])
def test_wait_limit_timeout_flags_every_pose(query):
    """A waiting wavefront that gives up (forced from the host with a wait
    limit of one device-clock tick, so every kernel still exits at once)
    makes the whole query report CBVH_POSE_INCOMPLETE on every pose and one
    wait timeout in the counters; with the default limit restored the same
    query is clean and matches the oracle."""
    P, _ = W.config0_poses()
    A, B = W.oracle_meshes(0)
    ma, mb = models(0)
    Pd = torch.from_numpy(P).to(DEV)
    n = len(P)
    ws = cb.workspace(ma, mb, n)

    def run():
        if query == "collide":
            return cb.collide(ma, mb, Pd, flags=cb.EARLY_EXIT, ws=ws)
        return cb.distance(ma, mb, Pd, ws=ws)

    _log(f"wait limit of one tick: {query}")
    try:
        cb.cbvh_set_wait_limit(1)
        _, st = run()
        stats = cb.cbvh_stats(ws.buf)
    finally:
        cb.cbvh_set_wait_limit(0)
    assert stats["wait_timeouts"] == 1
    assert (st.cpu().numpy() == cb.POSE_INCOMPLETE).all()
    out, st = run()
    assert cb.cbvh_stats(ws.buf)["wait_timeouts"] == 0
    assert (st.cpu().numpy() == 0).all()
    if query == "collide":
        ref, _ = oracle.collide_batch(A, B, P)
        assert np.array_equal(out.cpu().numpy().astype(bool), ref)
    else:
        ref, _ = oracle.distance_batch(A, B, P)
        got = out.cpu().numpy().astype(np.float64)
        pos = ref > 0
        assert (got[~pos] == 0).all()
        assert (np.abs(got[pos] - ref[pos]) / ref[pos]).max() <= 1e-5


@pytest.mark.parametrize("wpg", ["1", "2", "4"])
def test_workgroup_shape_keeps_answers(wpg, monkeypatch):
    """Independent waves per workgroup (the launch's workgroup shape, a
    tuning knob; the defaults are one for collision and two for distance
    queries) change how waves are placed, never an answer: collision
    booleans of the scaled workload and distances of the proximity workload
    equal the default launch's bitwise."""
    wc, wd = configs.WORKLOADS[1], configs.WORKLOADS[2]
    Pc = torch.from_numpy(wc.raw_poses(4096)).to(DEV)
    Pd = torch.from_numpy(wd.raw_poses(1024)).to(DEV)
    mc, md = models(1), models(2)
    ref_h, _ = cb.collide(*mc, Pc)
    ref_d, _ = cb.distance(*md, Pd)
    monkeypatch.setenv("CBVH_WAVES_PER_GROUP", wpg)
    _log(f"workgroup shape: {wpg} waves per workgroup")
    h, hs = cb.collide(*mc, Pc)
    d, ds = cb.distance(*md, Pd)
    assert (hs.cpu().numpy() == 0).all() and (ds.cpu().numpy() == 0).all()
    assert torch.equal(h, ref_h)
    assert torch.equal(d.view(torch.int32), ref_d.view(torch.int32))
