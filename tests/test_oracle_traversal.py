"""Pins of the oracle's Algorithm-1 traversal, distance branch-and-bound and
margin classification: brute force over all triangle pairs on tiny meshes,
closed-form cube scenes, the pose-inverse symmetry, and the margin
predicate re-derived by brute force."""
import numpy as np
import pytest

import oracle
from synth import meshes, poses


def _ico(freq, seed):
    return meshes.icosphere(freq, 0.1, np.random.default_rng(seed))


def _poses(n, half, seed):
    rng = np.random.default_rng(seed)
    return poses.compose(poses.uniform_rotations(n, rng), poses.box_translations(n, half, rng))


@pytest.mark.parametrize("freq,n_poses", [(2, 40), (4, 24), (8, 6)])
def test_traversal_equals_brute_force_pairs(freq, n_poses):
    A = oracle.Mesh(*_ico(freq, 10 + freq))
    B = oracle.Mesh(*_ico(freq, 20 + freq))
    P = _poses(n_poses, 2.2, freq)
    n_hit = 0
    for p in P:
        got = oracle.collide_pairs(A, B, p)
        ref = oracle.brute_pairs(A, B, p)
        assert np.array_equal(got, ref)
        hit, _ = oracle.collide(A, B, p, early_exit=True)
        assert hit == (len(ref) > 0)
        n_hit += hit
    assert 0 < n_hit < len(P)


@pytest.mark.parametrize("freq,n_poses", [(2, 30), (4, 10)])
def test_distance_equals_brute_force(freq, n_poses):
    A = oracle.Mesh(*_ico(freq, 30 + freq))
    B = oracle.Mesh(*meshes.torus(12, 6, 1.0, 0.3, 0.02, np.random.default_rng(freq)))
    P = _poses(n_poses, 3.0, 100 + freq)
    for p in P:
        d, _ = oracle.distance(A, B, p)
        assert d == oracle.brute_distance(A, B, p)


def _cube(center, half=0.5):
    v, t = meshes.box(center, half)
    return oracle.Mesh(v, t)


IDENT = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 0]], dtype=np.float32)


@pytest.mark.parametrize("g", [0.25, 0.001, 0.0, -0.1])
def test_cube_gap(g):
    A = _cube([0, 0, 0])
    B = _cube([1 + g, 0, 0])
    d, _ = oracle.distance(A, B, IDENT)
    hit, _ = oracle.collide(A, B, IDENT)
    # vertices are float32: B's facing face sits at float32(0.5 + g)
    gap = float(np.float32(1 + g - 0.5)) - 0.5
    if g > 0:
        assert d == pytest.approx(gap, rel=1e-12)
        assert not hit
    else:
        assert d == 0.0
        assert hit


def test_cube_rotated_45():
    c = np.float32(np.cos(np.pi / 4))
    s = np.float32(np.sin(np.pi / 4))
    pose = np.array([[c, -s, 0, 0], [s, c, 0, 0], [0, 0, 1, 0]], dtype=np.float32)
    A = _cube([0, 0, 0])
    B = _cube([1.5, 0, 0])
    d, _ = oracle.distance(A, B, pose)
    expect = 1.5 - 0.5 - 0.5 * (float(c) + float(s))
    assert d == pytest.approx(expect, rel=1e-12)
    # the rotation acts on A's coordinates (x_B = R x_A + t): a 90-degree turn about z
    # maps A's corner (0.5, 0.5, z) to (-0.5, 0.5, z) and keeps the cube in place
    R90 = np.array([[0, -1, 0, -0.1], [1, 0, 0, 0], [0, 0, 1, 0]], dtype=np.float32)
    d90, _ = oracle.distance(A, B, R90)
    assert d90 == pytest.approx(1.0 - 0.5 - float(np.float32(-0.1)), rel=1e-12)


def test_translation_and_rotation_order():
    # a long thin box A along x; rotate by +90 deg about z then translate: it must lie along y
    v, t = meshes.box([0, 0, 0], [2.0, 0.1, 0.1])
    A = oracle.Mesh(v, t)
    B = _cube([0, 3.0, 0], 0.5)
    rot = np.array([[0, -1, 0, 0], [1, 0, 0, 0], [0, 0, 1, 0]], dtype=np.float32)
    d, _ = oracle.distance(A, B, rot)
    assert d == pytest.approx(3.0 - 0.5 - 2.0, rel=1e-9)
    rot_t = rot.copy(); rot_t[0, 3] = 5.0     # translation is applied after the rotation
    d2, _ = oracle.distance(A, B, rot_t)
    assert d2 == pytest.approx(np.hypot(5.0 - 0.5 - 0.1, 0.5), rel=1e-7)


def test_symmetry_under_inverse_pose():
    va, ta = _ico(4, 41)
    vb, tb = _ico(4, 42)
    A, B = oracle.Mesh(va, ta), oracle.Mesh(vb, tb)
    m = 1e-3
    P = _poses(30, 2.0, 7)
    inv = poses.invert(P).astype(np.float32)
    checked = 0
    for p, q in zip(P, inv):
        if oracle.classify(A, B, p, m, pair_level=True) == oracle.MARGINAL:
            continue
        if oracle.classify(B, A, q, m, pair_level=True) == oracle.MARGINAL:
            continue
        ab = oracle.collide_pairs(A, B, p)
        ba = oracle.collide_pairs(B, A, q)[:, ::-1]
        ba = ba[np.lexsort((ba[:, 1], ba[:, 0]))]
        assert np.array_equal(ab, ba)
        checked += 1
    assert checked >= 10


def _brute_signed(A, B, p):
    ta = oracle.transform(p, A.V)[A.T.astype(np.int64)]
    tb = B.V[B.T.astype(np.int64)].astype(np.float64)
    return np.array([[oracle.tt_signed(a, b) for b in tb] for a in ta])


def test_margin_classification_matches_brute_force():
    va, ta = _ico(2, 51)
    vb, tb = _ico(2, 52)
    A, B = oracle.Mesh(va, ta), oracle.Mesh(vb, tb)
    m = 0.02
    P = _poses(60, 2.1, 9)
    seen = set()
    for p in P:
        s = _brute_signed(A, B, p)
        pose_cls = oracle.classify(A, B, p, m, pair_level=False)
        if (s <= -m).any():
            assert pose_cls == oracle.COLLIDING
        elif s.min() >= m:
            assert pose_cls == oracle.SEPARATED
        else:
            assert pose_cls == oracle.MARGINAL
        pair_cls = oracle.classify(A, B, p, m, pair_level=True)
        if ((s > -m) & (s < m)).any():
            assert pair_cls == oracle.MARGINAL
        else:
            assert pair_cls == (oracle.COLLIDING if (s < 0).any() else oracle.SEPARATED)
        seen.add((pose_cls, pair_cls))
    assert len({c for c, _ in seen}) == 3


def test_batches_match_single_calls():
    va, ta = _ico(4, 61)
    vb, tb = _ico(4, 62)
    A, B = oracle.Mesh(va, ta), oracle.Mesh(vb, tb)
    P = _poses(40, 2.5, 11)
    hits, _ = oracle.collide_batch(A, B, P, threads=4)
    dists, _ = oracle.distance_batch(A, B, P, threads=4)
    cls = oracle.classify_batch(A, B, P, 1e-3, threads=4)
    counts, _ = oracle.pair_count_batch(A, B, P, threads=4)
    for i, p in enumerate(P):
        assert counts[i] == len(oracle.brute_pairs(A, B, p))
        assert hits[i] == oracle.collide(A, B, p)[0]
        assert dists[i] == oracle.distance(A, B, p)[0]
        assert cls[i] == oracle.classify(A, B, p, 1e-3)
