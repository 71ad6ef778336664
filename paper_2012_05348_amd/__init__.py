"""Compressed BVH collision detection and proximity queries on MI355X (gfx950).

Thin Python binding of the C ABI in include/cbvh.h: the functions named
``cbvh_*`` marshal arguments (torch tensors for device memory, the current
torch stream as the HIP stream) into the library ``libcbvh.so``; every step of
the queries runs in the library's HIP kernels.  The convenience layer below
(``Model``, ``collide``, ``distance``) only allocates outputs and calls them.

There is no CPU fallback: importing works without a GPU (model building is
host code), but any device call fails loudly if the HIP library or a GPU is
missing.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcbvh.so")

AABB, DOP18, OBB = 0, 1, 2
# words of an OBB descriptor: lo0 hi0 lo1 hi1 lo2 hi2, 0, eps, origin[3], axes[3][3]
OBB_WORDS = 20
BITS_FP16 = 0x8010  # half-precision absolute descriptors (CBVH_BITS_FP16)
EARLY_EXIT, PAIRS, NO_SPLIT = 0x1, 0x2, 0x4
POSE_OK, POSE_STACK_OVERFLOW, POSE_PAIR_OVERFLOW, POSE_FP64_OVERFLOW, POSE_BAD_OBSTACLE, POSE_INCOMPLETE = range(6)
STATUS_NAMES = {0: "OK", 1: "E_INVALID", 2: "E_NOMEM", 3: "E_DEVICE", 4: "E_CAPACITY", 5: "E_UNSUPPORTED", 6: "E_FORMAT"}


class CbvhError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class BuildParams(C.Structure):
    _fields_ = [("size", C.c_uint32), ("bv", C.c_uint32), ("branching", C.c_uint32), ("leaf_size", C.c_uint32),
                ("bits", C.c_uint32), ("treelet_bytes", C.c_uint32)]


class ModelInfo(C.Structure):
    _fields_ = [(n, C.c_uint32) for n in ("bv", "slabs", "bits", "branching", "leaf_size", "n_nodes", "n_inner",
                                           "n_leaves", "n_tris", "n_abs", "n_treelets", "depth")] + \
               [(n, C.c_uint64) for n in ("blob_bytes", "descriptor_bytes", "topology_bytes", "triangle_bytes")]


class Stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("bv_tests", "tri_tests", "tri_fp64", "expansions", "node_bytes",
                                           "tri_bytes", "donated_items", "max_entries", "max_records",
                                           "t_start", "t_drain", "t_end", "max_pose_steps", "wait_timeouts",
                                           "node_steps", "leaf_steps", "waves")]

    def as_dict(self):
        return {n: int(getattr(self, n)) for n, _ in self._fields_}


_lib = None


def lib():
    """The loaded libcbvh.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python -c 'import __graft_entry__ as g; g.build()'")
        L = C.CDLL(LIB_PATH)
        P, u32, sz, st = C.c_void_p, C.c_uint32, C.c_size_t, C.c_int
        sig = {
            "cbvh_build": (st, [P, u32, P, u32, C.POINTER(BuildParams), C.POINTER(P)]),
            "cbvh_free": (None, [P]),
            "cbvh_blob": (st, [P, C.POINTER(P), C.POINTER(sz)]),
            "cbvh_load": (st, [P, sz, C.POINTER(P)]),
            "cbvh_info": (st, [P, C.POINTER(ModelInfo)]),
            "cbvh_device_bytes": (sz, [P]),
            "cbvh_upload": (st, [P, P, sz, P]),
            "cbvh_workspace_bytes": (sz, [P, P, u32, u32, u32]),
            "cbvh_collide": (st, [P, P, P, P, P, u32, u32, P, P, u32, P, P, P, sz, P]),
            "cbvh_distance": (st, [P, P, P, P, P, u32, u32, P, P, P, sz, P]),
            "cbvh_collide_static": (st, [P, P, P, P, P, u32, u32, P, P, P]),
            "cbvh_obstacles_device_bytes": (sz, [u32]),
            "cbvh_obstacles_create": (st, [C.POINTER(P), C.POINTER(P), u32, P, sz, P, C.POINTER(P)]),
            "cbvh_obstacles_free": (None, [P]),
            "cbvh_collide_batch": (st, [P, P, P, P, P, u32, u32, P, P, P, sz, P]),
            "cbvh_distance_batch": (st, [P, P, P, P, P, u32, u32, P, P, P, sz, P]),
            "cbvh_decode_all": (st, [P, P, P, P]),
            "cbvh_stats": (st, [P, sz, C.POINTER(Stats), P]),
            "cbvh_set_stack_limits": (st, [u32, u32]),
            "cbvh_set_wait_limit": (st, [C.c_uint64]),
            "cbvh_last_error": (C.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(status):
    if status != 0:
        raise CbvhError(status, lib().cbvh_last_error().decode())


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _aligned_empty(nbytes, device, align=256):
    """A uint8 device tensor of nbytes whose storage starts 256-byte aligned."""
    import torch
    buf = torch.empty(nbytes + align, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % align
    return buf[off:off + nbytes]


# ---------------------------------------------------------------------------
# the C ABI, one Python function per entry point (marshalling only)
# ---------------------------------------------------------------------------
def cbvh_build(V: np.ndarray, T: np.ndarray, bv=AABB, branching=4, leaf_size=1, bits=8, treelet_bytes=0):
    V = np.ascontiguousarray(np.asarray(V, dtype=np.float32).reshape(-1, 3))
    T = np.ascontiguousarray(np.asarray(T, dtype=np.uint32).reshape(-1, 3))
    p = BuildParams(C.sizeof(BuildParams), bv, branching, leaf_size, bits, treelet_bytes)
    h = C.c_void_p()
    _check(lib().cbvh_build(V.ctypes.data_as(C.c_void_p), len(V), T.ctypes.data_as(C.c_void_p), len(T), C.byref(p),
                            C.byref(h)))
    return h


def cbvh_free(h):
    if h:
        lib().cbvh_free(h)


def cbvh_blob(h) -> bytes:
    p, n = C.c_void_p(), C.c_size_t()
    _check(lib().cbvh_blob(h, C.byref(p), C.byref(n)))
    return C.string_at(p, n.value)


def cbvh_load(blob: bytes):
    h = C.c_void_p()
    buf = C.create_string_buffer(bytes(blob), len(blob))
    _check(lib().cbvh_load(C.cast(buf, C.c_void_p), len(blob), C.byref(h)))
    return h


def cbvh_info(h) -> dict:
    i = ModelInfo()
    _check(lib().cbvh_info(h, C.byref(i)))
    return {n: int(getattr(i, n)) for n, _ in ModelInfo._fields_}


def cbvh_device_bytes(h) -> int:
    return int(lib().cbvh_device_bytes(h))


def cbvh_upload(h, dev, stream=None):
    _check(lib().cbvh_upload(h, _ptr(dev), dev.numel() * dev.element_size(), _stream(stream)))


def cbvh_workspace_bytes(a, b, n_poses, flags=0, pair_capacity=0) -> int:
    return int(lib().cbvh_workspace_bytes(a, b, n_poses, flags, pair_capacity))


def cbvh_collide(a, a_dev, b, b_dev, poses, n, flags, hit, pairs, pair_capacity, pair_offsets, pose_status, workspace,
                 stream=None):
    _check(lib().cbvh_collide(a, _ptr(a_dev), b, _ptr(b_dev), _ptr(poses), n, flags, _ptr(hit), _ptr(pairs),
                              pair_capacity, _ptr(pair_offsets), _ptr(pose_status), _ptr(workspace),
                              0 if workspace is None else workspace.numel(), _stream(stream)))


def cbvh_distance(a, a_dev, b, b_dev, poses, n, flags, dist, pose_status, workspace, stream=None):
    _check(lib().cbvh_distance(a, _ptr(a_dev), b, _ptr(b_dev), _ptr(poses), n, flags, _ptr(dist), _ptr(pose_status),
                               _ptr(workspace), 0 if workspace is None else workspace.numel(), _stream(stream)))


STATIC_MAX_POSES = 262144  # CBVH_STATIC_MAX_POSES


def cbvh_collide_static(a, a_dev, b, b_dev, poses, n, flags, hit, pose_status, stream=None):
    _check(lib().cbvh_collide_static(a, _ptr(a_dev), b, _ptr(b_dev), _ptr(poses), n, flags, _ptr(hit),
                                     _ptr(pose_status), _stream(stream)))


def cbvh_obstacles_device_bytes(n) -> int:
    return int(lib().cbvh_obstacles_device_bytes(n))


def cbvh_obstacles_create(handles, devs, table, stream=None):
    n = len(handles)
    hs = (C.c_void_p * n)(*[h.value if isinstance(h, C.c_void_p) else h for h in handles])
    ds = (C.c_void_p * n)(*[d.data_ptr() for d in devs])
    out = C.c_void_p()
    _check(lib().cbvh_obstacles_create(C.cast(hs, C.POINTER(C.c_void_p)), C.cast(ds, C.POINTER(C.c_void_p)), n,
                                       _ptr(table), table.numel() * table.element_size(), _stream(stream),
                                       C.byref(out)))
    return out


def cbvh_obstacles_free(h):
    if h:
        lib().cbvh_obstacles_free(h)


def cbvh_collide_batch(a, a_dev, obstacles, poses, pose_obstacle, n, flags, hit, pose_status, workspace, stream=None):
    _check(lib().cbvh_collide_batch(a, _ptr(a_dev), obstacles, _ptr(poses), _ptr(pose_obstacle), n, flags, _ptr(hit),
                                    _ptr(pose_status), _ptr(workspace), 0 if workspace is None else workspace.numel(),
                                    _stream(stream)))


def cbvh_distance_batch(a, a_dev, obstacles, poses, pose_obstacle, n, flags, dist, pose_status, workspace,
                        stream=None):
    _check(lib().cbvh_distance_batch(a, _ptr(a_dev), obstacles, _ptr(poses), _ptr(pose_obstacle), n, flags,
                                     _ptr(dist), _ptr(pose_status), _ptr(workspace),
                                     0 if workspace is None else workspace.numel(), _stream(stream)))


def cbvh_decode_all(h, dev, out, stream=None):
    _check(lib().cbvh_decode_all(h, _ptr(dev), _ptr(out), _stream(stream)))


def cbvh_stats(workspace, stream=None) -> dict:
    s = Stats()
    _check(lib().cbvh_stats(_ptr(workspace), workspace.numel(), C.byref(s), _stream(stream)))
    return s.as_dict()


def cbvh_set_stack_limits(entries=0, records=0):
    _check(lib().cbvh_set_stack_limits(entries, records))


def cbvh_set_wait_limit(ticks=0):
    _check(lib().cbvh_set_wait_limit(ticks))


def cbvh_last_error() -> str:
    return lib().cbvh_last_error().decode()


# ---------------------------------------------------------------------------
# convenience layer
# ---------------------------------------------------------------------------
class Model:
    """A compressed BVH built on the host; ``to(device)`` uploads it once."""

    def __init__(self, handle):
        self._h = handle
        self.dev = None

    @classmethod
    def build(cls, V, T, bv=AABB, branching=4, leaf_size=1, bits=8, treelet_bytes=0):
        return cls(cbvh_build(V, T, bv, branching, leaf_size, bits, treelet_bytes))

    @classmethod
    def load(cls, blob: bytes):
        return cls(cbvh_load(blob))

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.cbvh_free(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def blob(self) -> bytes:
        return cbvh_blob(self._h)

    def info(self) -> dict:
        return cbvh_info(self._h)

    def to(self, device="cuda"):
        self.dev = _aligned_empty(cbvh_device_bytes(self._h), device)
        cbvh_upload(self._h, self.dev)
        return self

    def decode_all(self):
        import torch
        info = self.info()
        width = OBB_WORDS if info["bv"] == OBB else 2 * info["slabs"]
        out = torch.empty((info["n_nodes"], width), dtype=torch.float32, device=self.dev.device)
        cbvh_decode_all(self._h, self.dev, out)
        return out


@dataclass
class Workspace:
    buf: object
    n_poses: int
    flags: int
    pair_capacity: int


def workspace(a: Model, b: Model, n_poses, flags=0, pair_capacity=0, device="cuda"):
    nbytes = cbvh_workspace_bytes(a.handle, b.handle, n_poses, flags, pair_capacity)
    return Workspace(_aligned_empty(nbytes, device), n_poses, flags, pair_capacity)


def collide(a: Model, b: Model, poses, flags=EARLY_EXIT, pair_capacity=0, ws: Workspace | None = None, out=None):
    """Collision query for a batch of device poses (float32 [n, 3, 4]).

    Returns (hit uint8[n], status uint8[n]) or, with PAIRS,
    (hit, status, pairs uint32[m, 3], offsets uint32[n+1]) where m = offsets[n]."""
    import torch
    n = int(poses.shape[0])
    dev = poses.device
    if ws is None:
        ws = workspace(a, b, n, flags, pair_capacity, dev)
    if out is None:
        hit = torch.empty(n, dtype=torch.uint8, device=dev)
        status = torch.empty(n, dtype=torch.uint8, device=dev)
    else:
        hit, status = out
    pairs = offsets = None
    if flags & PAIRS:
        pairs = torch.empty((max(pair_capacity, 1), 3), dtype=torch.int32, device=dev)
        offsets = torch.empty(n + 1, dtype=torch.int32, device=dev)
    cbvh_collide(a.handle, a.dev, b.handle, b.dev, poses, n, flags, hit, pairs, pair_capacity, offsets, status, ws.buf)
    if flags & PAIRS:
        return hit, status, pairs, offsets
    return hit, status


def distance(a: Model, b: Model, poses, flags=0, ws: Workspace | None = None, out=None):
    """Minimum separation distance per pose: (dist float32[n], status uint8[n])."""
    import torch
    n = int(poses.shape[0])
    dev = poses.device
    if ws is None:
        ws = workspace(a, b, n, 0, 0, dev)
    if out is None:
        dist = torch.empty(n, dtype=torch.float32, device=dev)
        status = torch.empty(n, dtype=torch.uint8, device=dev)
    else:
        dist, status = out
    cbvh_distance(a.handle, a.dev, b.handle, b.dev, poses, n, flags, dist, status, ws.buf)
    return dist, status


class Obstacles:
    """A set of uploaded fixed models for batched queries (keeps the models alive)."""

    def __init__(self, models, device="cuda"):
        self.models = list(models)
        self.table = _aligned_empty(max(256, cbvh_obstacles_device_bytes(len(self.models))), device)
        self._h = cbvh_obstacles_create([m.handle for m in self.models], [m.dev for m in self.models], self.table)

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.cbvh_obstacles_free(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def __len__(self):
        return len(self.models)


def collide_batch(a: Model, obstacles: Obstacles, poses, pose_obstacle, flags=EARLY_EXIT, ws: Workspace | None = None,
                  out=None):
    """Batched collision booleans: pose i (float32 [n, 3, 4]) against obstacle pose_obstacle[i] (int32/uint32 [n])."""
    import torch
    n = int(poses.shape[0])
    dev = poses.device
    if ws is None:
        ws = workspace(a, a, n, flags, 0, dev)
    hit, status = out if out is not None else (torch.empty(n, dtype=torch.uint8, device=dev),
                                               torch.empty(n, dtype=torch.uint8, device=dev))
    cbvh_collide_batch(a.handle, a.dev, obstacles.handle, poses, pose_obstacle, n, flags, hit, status, ws.buf)
    return hit, status


def distance_batch(a: Model, obstacles: Obstacles, poses, pose_obstacle, flags=0, ws: Workspace | None = None,
                   out=None):
    """Batched minimum distances: pose i against obstacle pose_obstacle[i]."""
    import torch
    n = int(poses.shape[0])
    dev = poses.device
    if ws is None:
        ws = workspace(a, a, n, 0, 0, dev)
    dist, status = out if out is not None else (torch.empty(n, dtype=torch.float32, device=dev),
                                                torch.empty(n, dtype=torch.uint8, device=dev))
    cbvh_distance_batch(a.handle, a.dev, obstacles.handle, poses, pose_obstacle, n, flags, dist, status, ws.buf)
    return dist, status
