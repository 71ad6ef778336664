"""FP64 CPU oracle for compressed-BVH collision detection and proximity queries.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may use it; the product library never does.  It shares no
code with the GPU path.  See oracle.c for what each routine follows.

Python-side helpers here only marshal arrays and sort outputs (a library
sort); every geometric decision is made in oracle.c.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

SEPARATED, COLLIDING, MARGINAL = 0, 1, 2


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build()
        L = C.CDLL(path)
        P, u32, u64, i32, d, sz = C.c_void_p, C.c_uint32, C.c_uint64, C.c_int, C.c_double, C.c_size_t
        sig = {
            "orc_mesh_new": (P, [P, u32, P, u32]),
            "orc_mesh_free": (None, [P]),
            "orc_tt_sat": (i32, [P, P]),
            "orc_tt_segtri": (i32, [P, P]),
            "orc_tt_interval": (i32, [P, P]),
            "orc_tt_dist": (d, [P, P]),
            "orc_tt_pd": (d, [P, P]),
            "orc_tt_signed": (d, [P, P]),
            "orc_pt_tri_dist": (d, [P, P]),
            "orc_seg_seg_dist": (d, [P, P, P, P]),
            "orc_collide": (i32, [P, P, P, i32, P, u64, P, P]),
            "orc_distance": (d, [P, P, P, P]),
            "orc_brute_collide": (u64, [P, P, P, P, u64]),
            "orc_brute_distance": (d, [P, P, P]),
            "orc_classify": (i32, [P, P, P, d, i32]),
            "orc_collide_batch": (None, [P, P, P, u64, i32, P, P]),
            "orc_distance_batch": (None, [P, P, P, u64, i32, P, P]),
            "orc_pair_count_batch": (None, [P, P, P, u64, i32, P, P]),
            "orc_classify_batch": (None, [P, P, P, u64, d, i32, i32, P]),
            "orc_blob_info": (i32, [P, sz, P]),
            "orc_blob_decode": (i32, [P, sz, P, P, sz]),
            "orc_blob_check": (i32, [P, sz, P, u32, P, u32, P, sz]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


def _d9(t):
    t = np.ascontiguousarray(np.asarray(t, dtype=np.float64).reshape(9))
    return t


class Mesh:
    """A triangle mesh with the oracle's own FP64 binary AABB tree."""

    def __init__(self, V, T):
        self.V = np.ascontiguousarray(np.asarray(V, dtype=np.float32))
        self.T = np.ascontiguousarray(np.asarray(T, dtype=np.uint32))
        h = lib().orc_mesh_new(_p(self.V), len(self.V), _p(self.T), len(self.T))
        if not h:
            raise ValueError("invalid mesh")
        self._h = C.c_void_p(h)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.orc_mesh_free(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def tri(self, i):
        return self.V[self.T[i]].astype(np.float64)


def _pose(p):
    p = np.ascontiguousarray(np.asarray(p, dtype=np.float32).reshape(12))
    return p


# ---- primitives -------------------------------------------------------------
def tt_sat(a, b):
    return bool(lib().orc_tt_sat(_p(_d9(a)), _p(_d9(b))))


def tt_segtri(a, b):
    return bool(lib().orc_tt_segtri(_p(_d9(a)), _p(_d9(b))))


def tt_interval(a, b):
    return bool(lib().orc_tt_interval(_p(_d9(a)), _p(_d9(b))))


def tt_dist(a, b):
    return float(lib().orc_tt_dist(_p(_d9(a)), _p(_d9(b))))


def tt_pd(a, b):
    return float(lib().orc_tt_pd(_p(_d9(a)), _p(_d9(b))))


def tt_signed(a, b):
    return float(lib().orc_tt_signed(_p(_d9(a)), _p(_d9(b))))


def pt_tri_dist(p, t):
    p = np.ascontiguousarray(np.asarray(p, dtype=np.float64).reshape(3))
    return float(lib().orc_pt_tri_dist(_p(p), _p(_d9(t))))


def seg_seg_dist(p1, q1, p2, q2):
    a = [np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(3)) for x in (p1, q1, p2, q2)]
    return float(lib().orc_seg_seg_dist(*[_p(x) for x in a]))


def transform(pose, pts):
    """FP64 image of points under a float32 pose [R|t] (helper for tests)."""
    P = np.asarray(pose, dtype=np.float64).reshape(3, 4)
    return np.asarray(pts, dtype=np.float64) @ P[:, :3].T + P[:, 3]


# ---- queries ------------------------------------------------------------------
def collide(A: Mesh, B: Mesh, pose, early_exit=True):
    """Boolean collision by Algorithm 1; returns (hit, counters[bv_tests, tri_tests])."""
    cnt = np.zeros(2, dtype=np.uint64)
    hit = lib().orc_collide(A.handle, B.handle, _p(_pose(pose)), int(early_exit), None, 0, None, _p(cnt))
    return bool(hit), cnt


def collide_pairs(A: Mesh, B: Mesh, pose):
    """All intersecting (triA, triB) input-index pairs, sorted."""
    n = np.zeros(1, dtype=np.uint64)
    lib().orc_collide(A.handle, B.handle, _p(_pose(pose)), 0, None, 0, _p(n), None)
    cap = int(n[0])
    out = np.zeros((max(cap, 1), 2), dtype=np.uint32)
    lib().orc_collide(A.handle, B.handle, _p(_pose(pose)), 0, _p(out), cap, _p(n), None)
    out = out[:cap]
    order = np.lexsort((out[:, 1], out[:, 0]))
    return out[order]


def distance(A: Mesh, B: Mesh, pose):
    cnt = np.zeros(2, dtype=np.uint64)
    d = lib().orc_distance(A.handle, B.handle, _p(_pose(pose)), _p(cnt))
    return float(d), cnt


def brute_pairs(A: Mesh, B: Mesh, pose):
    n = lib().orc_brute_collide(A.handle, B.handle, _p(_pose(pose)), None, 0)
    out = np.zeros((max(int(n), 1), 2), dtype=np.uint32)
    lib().orc_brute_collide(A.handle, B.handle, _p(_pose(pose)), _p(out), n)
    out = out[: int(n)]
    order = np.lexsort((out[:, 1], out[:, 0]))
    return out[order]


def brute_distance(A: Mesh, B: Mesh, pose):
    return float(lib().orc_brute_distance(A.handle, B.handle, _p(_pose(pose))))


def classify(A: Mesh, B: Mesh, pose, margin, pair_level=False):
    return int(lib().orc_classify(A.handle, B.handle, _p(_pose(pose)), float(margin), int(pair_level)))


def _poses(poses):
    return np.ascontiguousarray(np.asarray(poses, dtype=np.float32).reshape(-1, 12))


def collide_batch(A: Mesh, B: Mesh, poses, threads=None):
    P = _poses(poses)
    out = np.zeros(len(P), dtype=np.uint8)
    cnt = np.zeros(2, dtype=np.uint64)
    lib().orc_collide_batch(A.handle, B.handle, _p(P), len(P), int(threads or os.cpu_count() or 1), _p(out), _p(cnt))
    return out.astype(bool), cnt


def distance_batch(A: Mesh, B: Mesh, poses, threads=None):
    P = _poses(poses)
    out = np.zeros(len(P), dtype=np.float64)
    cnt = np.zeros(2, dtype=np.uint64)
    lib().orc_distance_batch(A.handle, B.handle, _p(P), len(P), int(threads or os.cpu_count() or 1), _p(out), _p(cnt))
    return out, cnt


def pair_count_batch(A: Mesh, B: Mesh, poses, threads=None):
    """Number of intersecting triangle pairs per pose (full enumeration, no early exit)."""
    P = _poses(poses)
    out = np.zeros(len(P), dtype=np.uint64)
    cnt = np.zeros(2, dtype=np.uint64)
    lib().orc_pair_count_batch(A.handle, B.handle, _p(P), len(P), int(threads or os.cpu_count() or 1), _p(out),
                               _p(cnt))
    return out, cnt


def classify_batch(A: Mesh, B: Mesh, poses, margin, pair_level=False, threads=None):
    P = _poses(poses)
    out = np.zeros(len(P), dtype=np.uint8)
    lib().orc_classify_batch(A.handle, B.handle, _p(P), len(P), float(margin), int(pair_level),
                             int(threads or os.cpu_count() or 1), _p(out))
    return out


# ---- compressed blob --------------------------------------------------------------
BLOB_INFO_FIELDS = ("bv", "K", "bits", "branching", "leaf_size", "n_nodes", "n_tris", "n_abs",
                    "n_treelets", "code_stride", "depth", "treelet_bytes")


def blob_info(blob: bytes):
    b = np.frombuffer(blob, dtype=np.uint8)
    info = np.zeros(12, dtype=np.uint32)
    if lib().orc_blob_info(_p(b), len(b), _p(info)) != 0:
        raise ValueError("bad blob")
    return dict(zip(BLOB_INFO_FIELDS, (int(x) for x in info)))


def blob_decode(blob: bytes):
    """Decoded float32 bounds of every node, shape (n_nodes, 2K), (lo, hi) per slab;
    OBB blobs (bv 2): shape (n_nodes, 20), each node's descriptor with its frame."""
    info = blob_info(blob)
    b = np.frombuffer(blob, dtype=np.uint8)
    width = 20 if info["bv"] == 2 else 2 * info["K"]
    out = np.zeros((info["n_nodes"], width), dtype=np.float32)
    msg = C.create_string_buffer(256)
    if lib().orc_blob_decode(_p(b), len(b), _p(out), msg, 256) != 0:
        raise ValueError(msg.value.decode())
    return out


def blob_check(blob: bytes, V, T):
    """Check the blob's invariants against the mesh; returns None or the failure message."""
    b = np.frombuffer(blob, dtype=np.uint8)
    V = np.ascontiguousarray(np.asarray(V, dtype=np.float32))
    T = np.ascontiguousarray(np.asarray(T, dtype=np.uint32))
    msg = C.create_string_buffer(256)
    rc = lib().orc_blob_check(_p(b), len(b), _p(V), len(V), _p(T), len(T), msg, 256)
    return None if rc == 0 else msg.value.decode()
