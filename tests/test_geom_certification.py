"""The FP32 leaf geometry of the traversal (csrc/geom.h, built for the host)
against the FP64 oracle on adversarial triangle pairs.

The traversal decides most triangle pairs in FP32 and hands the rest to an
FP64 stage.  Its certified FP32 intersection test answers "disjoint" or
"intersecting" only when the error bound proves the answer for the given
float triangles, and its FP32 leaf distance must lie within the bound e of
the exact distance so that branch and bound never drops the closest pair.
Both claims are checked here on pairs built to sit at the edge of those
bounds: near-coplanar pairs, nearly parallel crossing edges, and pairs
offset from touching by 1e-7 to 1e-5, at coordinates up to the workloads'
largest (about 6), placed by random poses as the traversal places them."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import oracle
from synth import poses

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def gh(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("geomhost") / "libgeomhost.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    "-Wno-unknown-pragmas", "-o", out, os.path.join(HERE, "geomhost.cpp")], check=True)
    L = C.CDLL(out)
    P = C.c_void_p
    L.gh_tri_tri_f32.restype, L.gh_tri_tri_f32.argtypes = C.c_int, [P, P]
    L.gh_place_f32.restype, L.gh_place_f32.argtypes = None, [P, P, P]
    L.gh_leaf_dist_f32.restype, L.gh_leaf_dist_f32.argtypes = C.c_float, [P, P, P, P]
    L.gh_dist_err.restype, L.gh_dist_err.argtypes = C.c_float, [P, C.c_float, C.c_float]
    return L


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32).reshape(9))


def _unit(rng, n=None):
    v = rng.normal(size=3 if n is None else (n, 3))
    return v / np.linalg.norm(v, axis=-1, keepdims=True)


def _frame(rng):
    u = _unit(rng)
    v = np.cross(u, _unit(rng))
    v /= np.linalg.norm(v)
    return u, v, np.cross(u, v)


def adversarial_pairs(rng, n):
    """(a, b) float64 triangle pairs near touching; kinds cycle through
    near-coplanar, nearly parallel crossing edges, offset-from-touching, and
    a tiny triangle crossing or grazing a large one far from the large one's
    first vertex (relative coordinates much larger than the small edges)."""
    out = []
    for i in range(n):
        kind = i % 4
        if kind == 3:
            c = rng.uniform(-5.0, 5.0, 3)
            u, v, w = _frame(rng)
            a = c + np.stack([np.zeros(3), 2.0 * u, 2.0 * v])
            p = c + rng.uniform(0.3, 0.9) * u + rng.uniform(0.3, 0.9) * v  # inside A, about 1 from a0
            small = np.exp(rng.uniform(np.log(1e-4), np.log(1e-2)))
            g = np.exp(rng.uniform(np.log(1e-9), np.log(1e-6))) * rng.choice([-1.0, 1.0])
            d = _unit(rng)
            b = np.stack([p + g * w + small * d, p + g * w - small * d + small * w,
                          p + g * w + small * _unit(rng)])
            out.append((a, b))
            continue
        scale = np.exp(rng.uniform(np.log(1e-3), np.log(0.5)))
        c = rng.uniform(-5.0, 5.0, 3)  # up to the largest coordinates of the workloads
        g = np.exp(rng.uniform(np.log(1e-7), np.log(1e-5))) * rng.choice([-1.0, 1.0])
        u, v, w = _frame(rng)
        if kind == 0:
            # B in A's plane, shifted out of it by g (and tilted a little)
            a = c + scale * (rng.uniform(-1, 1, (3, 2)) @ np.stack([u, v]))
            b = c + scale * (rng.uniform(-1, 1, (3, 2)) @ np.stack([u, v]))
            b = b + g * w + rng.uniform(-1, 1, (3, 1)) * (scale * 1e-6) * w
        elif kind == 1:
            # two long thin triangles whose long edges cross at a tiny angle,
            # B's edge offset from A's by g across both
            ang = np.exp(rng.uniform(np.log(1e-6), np.log(1e-2)))
            d1, d2 = u, np.cos(ang) * u + np.sin(ang) * v
            a = np.stack([c - scale * d1, c + scale * d1, c + scale * 0.3 * (v + w)])
            b = np.stack([c - scale * d2 + g * w, c + scale * d2 + g * w, c + scale * 0.3 * (v - w) + g * w])
        else:
            # B touches A at a point of A's face or edge, then moves by g along a random direction
            a = c + scale * rng.normal(size=(3, 3))
            t = rng.dirichlet(np.ones(3)) if rng.random() < 0.5 else np.array([rng.random(), 0.0, 0.0])
            t[2] = 1.0 - t[0] - t[1] if t.sum() != 1.0 else t[2]
            p = t @ a
            b = p + scale * rng.normal(size=(3, 3))
            b[0] = p
            b = b + g * _unit(rng)
        out.append((a, b))
    return out


def test_certified_fp32_intersection_decisions_equal_the_oracle(gh):
    rng = np.random.default_rng(20120534)
    decided = undecided = 0
    for a, b in adversarial_pairs(rng, 6000):
        a32, b32 = _f32(a), _f32(b)
        got = gh.gh_tri_tri_f32(_p(a32), _p(b32))
        ref = oracle.tt_sat(a32.astype(np.float64), b32.astype(np.float64))
        if got == 2:
            undecided += 1
            continue
        decided += 1
        assert got == int(ref), (a32.tolist(), b32.tolist(), got, ref)
    # the bound is not so loose that near-contact pairs are never decided
    assert decided > 2000 and undecided > 100, (decided, undecided)


def test_placed_fp32_leaf_test_and_distance_within_bounds(gh):
    """A's triangle given in its own frame and placed by a random pose in
    FP32, as the traversal does: certified decisions equal the oracle's on
    the placed float triangle, and the FP32 distance of every pair not
    certified intersecting is within e of the oracle's distance of the
    exactly placed triangle."""
    rng = np.random.default_rng(5348)
    pairs = adversarial_pairs(rng, 4000)
    R = poses.uniform_rotations(len(pairs), rng)
    worst = 0.0
    for (a, b), Ri in zip(pairs, R):
        t = rng.uniform(-1.0, 1.0, 3) * rng.uniform(0.0, 4.0)
        P = np.ascontiguousarray(np.concatenate([Ri, t[:, None]], axis=1).astype(np.float32).reshape(12))
        # A in its own frame: the world triangle moved back by the float pose (in FP64)
        Pm = P.reshape(3, 4).astype(np.float64)
        a_local = _f32((a - Pm[:, 3]) @ np.linalg.inv(Pm[:, :3]).T)
        b32 = _f32(b)
        placed = np.zeros(9, dtype=np.float32)
        gh.gh_place_f32(_p(P), _p(a_local), _p(placed))
        res = C.c_int()
        d32 = gh.gh_leaf_dist_f32(_p(P), _p(a_local), _p(b32), C.byref(res))
        if res.value != 2:
            assert res.value == int(oracle.tt_sat(placed.astype(np.float64), b32.astype(np.float64)))
        if res.value == 1:
            continue
        exact = oracle.transform(P, a_local.reshape(3, 3).astype(np.float64))
        d = oracle.tt_dist(exact, b32.astype(np.float64))
        e = gh.gh_dist_err(_p(P), float(np.abs(a_local).max()), float(np.abs(b32).max()))
        assert abs(d32 - d) <= e, (d32, d, e)
        worst = max(worst, abs(d32 - d) / e)
    assert worst > 0.0


def test_fp32_distance_of_separated_pairs_at_workload_scale(gh):
    """Ordinary separated pairs (gaps from 1e-6 to 1) at coordinates up to 6:
    the FP32 distance stays within e of the oracle's."""
    rng = np.random.default_rng(77)
    for _ in range(3000):
        scale = np.exp(rng.uniform(np.log(1e-3), np.log(0.3)))
        c = rng.uniform(-5.0, 5.0, 3)
        a = c + scale * rng.normal(size=(3, 3))
        gap = np.exp(rng.uniform(np.log(1e-6), 0.0))
        b = c + scale * rng.normal(size=(3, 3)) + (2 * scale + gap) * _unit(rng) * 3
        P = np.eye(3, 4, dtype=np.float32).reshape(12).copy()
        a32, b32 = _f32(a), _f32(b)
        res = C.c_int()
        d32 = gh.gh_leaf_dist_f32(_p(P), _p(a32), _p(b32), C.byref(res))
        if res.value == 1:
            continue
        d = oracle.tt_dist(a32.astype(np.float64), b32.astype(np.float64))
        e = gh.gh_dist_err(_p(P), float(np.abs(a32).max()), float(np.abs(b32).max()))
        assert abs(d32 - d) <= e, (d32, d, e)
