"""Oriented-box (OBB) models on the CPU.

- The builder's OBB blobs against the oracle's independent decoder and
  invariant checks (frames whose eps bounds their axes' defect, intervals
  that enclose the frame coordinates of every vertex under each node and nest
  inside the parent's where the frame is shared), over descriptor widths,
  branching factors, leaf sizes and treelet budgets; planted mistakes in a
  blob are caught.
- The traversal's OBB box test (csrc/geom.h built for the host) against exact
  box distances: for random and near-touching box pairs, with frames and pose
  matrices slightly off orthonormal and at coordinates up to 1e3, a positive
  separation never comes from boxes that overlap and the distance lower
  bound never exceeds the exact distance (a bounded least-squares problem
  over the two boxes' frame coordinates, solved in FP64).
"""
import ctypes as C
import os
import struct
import subprocess

import numpy as np
import pytest
from scipy.optimize import lsq_linear

import oracle
import paper_2012_05348_amd as cb
from synth import configs, poses

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def gh(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("geomhost_obb") / "libgeomhost.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    "-Wno-unknown-pragmas", "-o", out, os.path.join(HERE, "geomhost.cpp")], check=True)
    L = C.CDLL(out)
    P = C.c_void_p
    L.gh_obb_test.restype = None
    L.gh_obb_test.argtypes = [P, C.c_float, C.c_float, C.c_float, P, P, P, P]
    return L


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------- builder and checker
@pytest.fixture(scope="module")
def tiny_meshes():
    return configs.WORKLOADS[0].meshes()


@pytest.mark.parametrize("bits", [0, 8, 16])
@pytest.mark.parametrize("bf,leaf,tb", [(4, 1, 0), (8, 4, 0), (2, 2, 1024), (4, 1, 256)])
def test_obb_blobs_pass_the_oracle_checks(tiny_meshes, bits, bf, leaf, tb):
    for V, T in tiny_meshes:
        m = cb.Model.build(V, T, bv=cb.OBB, branching=bf, leaf_size=leaf, bits=bits, treelet_bytes=tb)
        blob = m.blob()
        assert oracle.blob_check(blob, V, T) is None
        dec = oracle.blob_decode(blob)
        assert dec.shape == (m.info()["n_nodes"], cb.OBB_WORDS)
        # frames: near-orthonormal axes with eps bounding the defect
        ax = dec[:, 11:20].astype(np.float64).reshape(-1, 3, 3)
        G = ax @ ax.transpose(0, 2, 1)
        assert (np.abs(G - np.eye(3)).max(axis=(1, 2)) <= dec[:, 7]).all()
        assert dec[:, 7].max() < 1e-5


def test_obb_frames_change_only_at_absolute_nodes(tiny_meshes):
    V, T = tiny_meshes[0]
    m8 = cb.Model.build(V, T, bv=cb.OBB, branching=4, leaf_size=1, bits=8, treelet_bytes=1024)
    m0 = cb.Model.build(V, T, bv=cb.OBB, branching=4, leaf_size=1, bits=0)
    d8, d0 = oracle.blob_decode(m8.blob()), oracle.blob_decode(m0.blob())
    n_frames8 = len({tuple(r) for r in d8[:, 8:20].tolist()})
    n_frames0 = len({tuple(r) for r in d0[:, 8:20].tolist()})
    assert n_frames8 == m8.info()["n_abs"]
    assert n_frames0 > 0.9 * m0.info()["n_nodes"]  # every uncompressed node fits its own frame


def _node_offset(blob, i, word):
    """Byte offset of word `word` of node i's descriptor in a bits = 0 OBB blob."""
    off_codes = struct.unpack_from("<Q", blob, 64)[0]
    stride = struct.unpack_from("<I", blob, 44)[0]
    return off_codes + stride * i + 4 * word


def test_checker_catches_planted_obb_mistakes(tiny_meshes):
    V, T = tiny_meshes[0]
    blob = cb.Model.build(V, T, bv=cb.OBB, branching=4, leaf_size=1, bits=0).blob()
    n = oracle.blob_info(blob)["n_nodes"]
    dec = oracle.blob_decode(blob)
    i = n // 2
    # a bound moved inward by a tenth of the interval
    b = bytearray(blob)
    lo, hi = dec[i, 2], dec[i, 3]
    struct.pack_into("<f", b, _node_offset(blob, i, 2), np.float32(lo + 0.1 * (hi - lo)))
    assert "does not enclose" in oracle.blob_check(bytes(b), V, T)
    # an eps below the axes' defect
    b = bytearray(blob)
    struct.pack_into("<f", b, _node_offset(blob, i, 7), np.float32(0.0))
    assert "eps" in oracle.blob_check(bytes(b), V, T)
    # the root's frame turned by 0.05 rad about its third axis (still
    # orthonormal, eps raised to cover the rounding, but the intervals no
    # longer enclose the vertices)
    b = bytearray(blob)
    a0 = dec[0, 11:14].astype(np.float64)
    a1 = dec[0, 14:17].astype(np.float64)
    c, s_ = np.cos(0.05), np.sin(0.05)
    for k, v in enumerate(np.concatenate([c * a0 + s_ * a1, -s_ * a0 + c * a1])):
        struct.pack_into("<f", b, _node_offset(blob, 0, 11 + k), np.float32(v))
    struct.pack_into("<f", b, _node_offset(blob, 0, 7), np.float32(1e-5))
    assert "does not enclose" in oracle.blob_check(bytes(b), V, T)


def test_obb_needs_float_or_code_descriptors(tiny_meshes):
    V, T = tiny_meshes[0]
    with pytest.raises(cb.CbvhError, match="OBB"):
        cb.Model.build(V, T, bv=cb.OBB, bits=cb.BITS_FP16)
    # an FP16 blob relabelled as OBB fails validation on load
    blob = bytearray(cb.Model.build(V, T, bv=cb.AABB, bits=cb.BITS_FP16).blob())
    struct.pack_into("<I", blob, 8, 2)
    with pytest.raises(cb.CbvhError):
        cb.cbvh_load(bytes(blob))


# ---------------------------------------------------------------- the box test
def _desc(rng, scale, defect):
    """A random OBB descriptor (float32, 20 words): frame from a random
    rotation, axes optionally perturbed off orthonormal, eps bounding the
    defect as the builder computes it."""
    R = poses.uniform_rotations(1, rng)[0]
    ax = R + (rng.uniform(-defect, defect, size=(3, 3)) if defect else 0.0)
    ax = ax.astype(np.float32)
    a64 = ax.astype(np.float64)
    dev = np.abs(a64 @ a64.T - np.eye(3)).max() + 2.0 ** -48
    eps = np.float32(dev)
    if float(eps) < dev:
        eps = np.nextafter(eps, np.float32(np.inf))
    o = rng.uniform(-scale, scale, size=3).astype(np.float32)
    lo = rng.uniform(-0.5 * scale, 0.5 * scale, size=3)
    size = scale * np.exp(rng.uniform(np.log(1e-3), np.log(0.5), size=3))
    d = np.zeros(20, np.float32)
    d[0:6:2] = lo.astype(np.float32)
    d[1:6:2] = (lo + size).astype(np.float32)
    d[7] = eps
    d[8:11] = o
    d[11:20] = ax.reshape(9)
    return d


def _corners(d):
    u = np.array(np.meshgrid(*[[d[2 * k], d[2 * k + 1]] for k in range(3)], indexing="ij")).reshape(3, -1).T
    return d[8:11].astype(np.float64) + u.astype(np.float64) @ d[11:20].astype(np.float64).reshape(3, 3)


def _rot_eps(R):
    R = R.astype(np.float64)
    dev = np.abs(R.T @ R - np.eye(3)).max()
    e = np.float32(dev)
    if float(e) < dev:
        e = np.nextafter(e, np.float32(np.inf))
    return np.float32(e + np.float32(2.0 ** -22))


def _exact_distance(P, dA, dB):
    """Distance of A's box placed by P and B's box: min over the two boxes'
    frame coordinates of |R (oA + MA uA) + t - (oB + MB uB)|, in FP64."""
    R, t = P[:, :3].astype(np.float64), P[:, 3].astype(np.float64)
    MA = dA[11:20].astype(np.float64).reshape(3, 3).T
    MB = dB[11:20].astype(np.float64).reshape(3, 3).T
    A = np.concatenate([R @ MA, -MB], axis=1)
    b = -(R @ dA[8:11].astype(np.float64) + t - dB[8:11].astype(np.float64))
    lo = np.concatenate([dA[0:6:2], dB[0:6:2]]).astype(np.float64)
    hi = np.concatenate([dA[1:6:2], dB[1:6:2]]).astype(np.float64)
    r = lsq_linear(A, b, bounds=(lo, hi), method="bvls", tol=1e-15)
    return float(np.linalg.norm(A @ r.x - b))


def _cases(rng, n, scale, defect, near):
    for _ in range(n):
        dA, dB = _desc(rng, scale, defect), _desc(rng, scale, defect)
        R = poses.uniform_rotations(1, rng)[0]
        if defect:
            R = R @ (np.eye(3) + rng.uniform(-2e-3, 2e-3, size=(3, 3)))
        cA = _corners(dA).mean(axis=0)
        cB = _corners(dB).mean(axis=0)
        # place A's centre near B's: at a random direction and offset
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        reach = 0.5 * (np.ptp(_corners(dA), axis=0).max() + np.ptp(_corners(dB), axis=0).max())
        off = reach * (rng.uniform(0.3, 1.6) if not near else rng.uniform(0.9, 1.1))
        t = cB + u * off - R @ cA
        P = np.concatenate([R, t[:, None]], axis=1).astype(np.float32)
        if near:
            # slide A along u so that the boxes sit at a tiny signed gap
            d0 = _exact_distance(P, dA, dB)
            if d0 == 0.0:
                continue
            gap = scale * rng.choice([-1.0, 1.0]) * np.exp(rng.uniform(np.log(1e-7), np.log(1e-3)))
            t = t - u * (d0 - gap)
            P = np.concatenate([R, t[:, None]], axis=1).astype(np.float32)
        yield P, dA, dB


@pytest.mark.parametrize("scale,defect,near", [(1.0, 0.0, False), (1.0, 1e-4, False), (1e3, 1e-4, False),
                                               (1.0, 0.0, True), (1e3, 1e-4, True)])
def test_obb_box_test_is_conservative(gh, scale, defect, near):
    rng = np.random.default_rng(int(scale) * 7 + int(defect * 1e5) + 3 * near)
    n_sep = n_found = n_lb = n = 0
    for P, dA, dB in _cases(rng, 300, scale, defect, near):
        maxA = np.float32(np.abs(_corners(dA)).max() * (1 + 1e-6))
        maxB = np.float32(np.abs(_corners(dB)).max() * (1 + 1e-6))
        sep, lb = C.c_float(), C.c_float()
        Pc = np.ascontiguousarray(P)
        gh.gh_obb_test(_p(Pc), _rot_eps(P[:, :3]), maxA, maxB, _p(dA), _p(dB), C.byref(sep), C.byref(lb))
        dist = _exact_distance(P, dA, dB)
        tol = 1e-12 * scale
        n += 1
        # the test never separates boxes that touch or overlap
        if sep.value > 0:
            assert dist > tol, (sep.value, dist)
        # the distance bound never overshoots
        assert lb.value <= dist + tol, (lb.value, dist)
        if dist > 0.05 * scale:
            n_sep += 1
            n_found += sep.value > 0
            n_lb += lb.value > 0.5 * dist
    assert n > 100
    if not near:
        # and it is not vacuous: most clearly separated pairs are found
        assert n_sep > 30 and n_found >= 0.6 * n_sep and n_lb >= 0.5 * n_sep, (n_sep, n_found, n_lb)
