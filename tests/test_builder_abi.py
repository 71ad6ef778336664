"""CPU tests of the host side of the library: the compressed-BVH builder
checked by the oracle's independent decoder and invariant checker, planted
corruptions that the checker must catch, blob validation, argument errors
of the C ABI, and that every function declared in include/cbvh.h is
exported.  No GPU is touched."""
import ctypes as C
import os
import re
import struct

import numpy as np
import pytest

import oracle
import paper_2012_05348_amd as cb
from synth import configs, meshes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BV = {"aabb": cb.AABB, "dop18": cb.DOP18}


@pytest.fixture(scope="module")
def mesh_sets():
    out = {}
    for k, w in configs.WORKLOADS.items():
        out[k] = w.meshes()
    return out


@pytest.mark.parametrize("cfg", [0, 1, 2])
@pytest.mark.parametrize("fmt", ["codes", "fp32", "fp16"])
def test_invariants_on_workload_meshes(cfg, fmt, mesh_sets):
    w = configs.WORKLOADS[cfg]
    bits = {"codes": w.bits, "fp32": 0, "fp16": cb.BITS_FP16}[fmt]
    for V, T in mesh_sets[cfg]:
        h = cb.cbvh_build(V, T, bv=BV[w.bv], branching=w.branching, leaf_size=w.leaf_size, bits=bits)
        blob = cb.cbvh_blob(h)
        assert oracle.blob_check(blob, V, T) is None
        cb.cbvh_free(h)


@pytest.mark.parametrize("bv,bf,leaf,bits,tb", [
    (cb.AABB, 2, 1, 8, 256), (cb.AABB, 8, 8, 16, 0), (cb.DOP18, 4, 2, 8, 1024), (cb.DOP18, 2, 3, 16, 4096),
    (cb.DOP18, 8, 1, 0, 0), (cb.AABB, 4, 5, 0, 512), (cb.DOP18, 8, 4, cb.BITS_FP16, 0),
    (cb.AABB, 2, 1, cb.BITS_FP16, 256)])
def test_invariants_parameter_sweep(bv, bf, leaf, bits, tb):
    V, T = meshes.torus(40, 12, 1.0, 0.3, 0.02, np.random.default_rng(3))
    h = cb.cbvh_build(V, T, bv=bv, branching=bf, leaf_size=leaf, bits=bits, treelet_bytes=tb)
    assert oracle.blob_check(cb.cbvh_blob(h), V, T) is None
    info = cb.cbvh_info(h)
    assert info["n_tris"] == len(T) and info["n_inner"] + info["n_leaves"] == info["n_nodes"]


def test_node_counts_match_the_median_split(mesh_sets):
    # leaf-aligned median split: n_leaves = ceil(n / leaf_size)
    expect = {0: 1877, 1: 29681, 2: 71845}
    for cfg, n in expect.items():
        w = configs.WORKLOADS[cfg]
        V, T = mesh_sets[cfg][1]
        info = cb.cbvh_info(cb.cbvh_build(V, T, bv=BV[w.bv], branching=w.branching, leaf_size=w.leaf_size, bits=w.bits))
        assert info["n_nodes"] == n
        assert info["n_leaves"] == -(-len(T) // w.leaf_size)


def _topo(blob):
    info = oracle.blob_info(blob)
    off = struct.unpack_from("<Q", blob, 56)[0]
    return np.frombuffer(blob, dtype=np.uint32, count=info["n_nodes"], offset=off) & np.uint32(0xBFFFFFFF)


def test_topology_shared_by_all_descriptor_formats():
    V, T = meshes.icosphere(6, 0.1, np.random.default_rng(1))
    ref = None
    for bv in (cb.AABB, cb.DOP18):
        for bits in (0, 8, 16, cb.BITS_FP16):
            h = cb.cbvh_build(V, T, bv=bv, branching=4, leaf_size=2, bits=bits, treelet_bytes=1 << 20)
            t = _topo(cb.cbvh_blob(h))
            if ref is None:
                ref = t
            assert np.array_equal(t, ref)


def test_compressed_descriptors_are_smaller(mesh_sets):
    w = configs.WORKLOADS[1]
    V, T = mesh_sets[1][1]
    c = cb.cbvh_info(cb.cbvh_build(V, T, bv=cb.DOP18, branching=8, leaf_size=4, bits=16))
    u = cb.cbvh_info(cb.cbvh_build(V, T, bv=cb.DOP18, branching=8, leaf_size=4, bits=0))
    assert c["descriptor_bytes"] < 0.7 * u["descriptor_bytes"]
    assert u["descriptor_bytes"] == 72 * u["n_nodes"]


# ---- planted mistakes: the oracle's checker must reject each ---------------------------
def _small_blob(bits=8, bv=cb.AABB):
    V, T = meshes.icosphere(4, 0.1, np.random.default_rng(7))
    h = cb.cbvh_build(V, T, bv=bv, branching=4, leaf_size=1, bits=bits, treelet_bytes=2048)
    return bytearray(cb.cbvh_blob(h)), V, T


def _first_relative_node(blob):
    info = oracle.blob_info(bytes(blob))
    off_topo = struct.unpack_from("<Q", blob, 56)[0]
    topo = np.frombuffer(bytes(blob), dtype=np.uint32, count=info["n_nodes"], offset=off_topo)
    return int(np.nonzero((topo & 0x40000000) == 0)[0][5]), info


@pytest.mark.parametrize("delta", [+1, -1])
def test_checker_catches_a_wrong_code(delta):
    blob, V, T = _small_blob()
    node, info = _first_relative_node(blob)
    off_codes = struct.unpack_from("<Q", blob, 64)[0]
    pos = off_codes + node * info["code_stride"]  # lo code of slab x
    if delta < 0 and blob[pos] == 0:
        pos += 2
    blob[pos] = (blob[pos] + delta) % 256
    msg = oracle.blob_check(bytes(blob), V, T)
    assert msg is not None and ("enclose" in msg or "tight" in msg), msg


def test_checker_catches_a_loose_absolute_bound():
    blob, V, T = _small_blob()
    off_abs = struct.unpack_from("<Q", blob, 72)[0]
    lo = struct.unpack_from("<f", blob, off_abs)[0]
    struct.pack_into("<f", blob, off_abs, np.nextafter(np.float32(lo), np.float32(-np.inf)))
    assert "tight" in oracle.blob_check(bytes(blob), V, T)


def test_checker_catches_swapped_triangles():
    blob, V, T = _small_blob()
    off_perm = struct.unpack_from("<Q", blob, 88)[0]
    a, b = struct.unpack_from("<II", blob, off_perm)
    struct.pack_into("<II", blob, off_perm, b, a)
    assert "differs" in oracle.blob_check(bytes(blob), V, T)


def test_checker_catches_a_wrong_uncompressed_bound():
    blob, V, T = _small_blob(bits=0, bv=cb.DOP18)
    off_codes = struct.unpack_from("<Q", blob, 64)[0]
    stride = oracle.blob_info(bytes(blob))["code_stride"]
    pos = off_codes + 3 * stride + 4 * 7   # node 3, slab 3 (x+y) upper bound
    hi = struct.unpack_from("<f", blob, pos)[0]
    struct.pack_into("<f", blob, pos, np.nextafter(np.float32(hi), np.float32(-np.inf)))
    assert "enclose" in oracle.blob_check(bytes(blob), V, T)


@pytest.mark.parametrize("which", ["lo_inward", "hi_inward", "lo_outward"])
def test_checker_catches_wrong_fp16_bounds(which):
    # FP16 bounds are the tightest halves enclosing the exact slab: one half
    # inward breaks enclosure, one half outward breaks tightness
    blob, V, T = _small_blob(bits=cb.BITS_FP16)
    off_codes = struct.unpack_from("<Q", blob, 64)[0]
    stride = oracle.blob_info(bytes(blob))["code_stride"]
    pos = off_codes + 4 * stride + (2 if which == "hi_inward" else 0)   # node 4, slab x
    h = struct.unpack_from("<H", blob, pos)[0]
    up = which in ("lo_inward",)
    step = lambda x, u: (x + 1 if not (x & 0x8000) else x - 1) if u else (x - 1 if not (x & 0x8000) else x + 1)
    if which == "lo_outward":
        up = False
    if h in (0x0000, 0x8000):
        pytest.skip("zero bound")
    struct.pack_into("<H", blob, pos, step(h, up))
    msg = oracle.blob_check(bytes(blob), V, T)
    assert msg is not None and ("enclose" in msg or "tight" in msg or "parent" in msg), msg


def test_fp16_needs_coordinates_in_half_range():
    V, T = meshes.icosphere(2, 0.1, np.random.default_rng(0))
    cb.cbvh_free(cb.cbvh_build(V * 25000.0, T, bits=cb.BITS_FP16))           # AABB: < 32768
    with pytest.raises(cb.CbvhError):
        cb.cbvh_build(V * 40000.0, T, bits=cb.BITS_FP16)
    with pytest.raises(cb.CbvhError):
        cb.cbvh_build(V * 20000.0, T, bv=cb.DOP18, bits=cb.BITS_FP16)        # 18-DOP: < 16384


# ---- blob validation (cbvh_load) ---------------------------------------------------
def test_load_roundtrip_and_rejects_corruption():
    blob, V, T = _small_blob()
    h = cb.cbvh_load(bytes(blob))
    assert cb.cbvh_blob(h) == bytes(blob)
    with pytest.raises(cb.CbvhError) as e:
        cb.cbvh_load(bytes(blob[:64]))
    assert e.value.status == 6
    bad = bytearray(blob)
    bad[:4] = b"XXXX"
    with pytest.raises(cb.CbvhError):
        cb.cbvh_load(bytes(bad))
    # a child index past the node array
    bad = bytearray(blob)
    off_topo = struct.unpack_from("<Q", bad, 56)[0]
    struct.pack_into("<I", bad, off_topo, (struct.unpack_from("<I", bad, off_topo)[0] & ~0x07FFFFFF) | 0x07FFFFF0)
    with pytest.raises(cb.CbvhError) as e:
        cb.cbvh_load(bytes(bad))
    assert e.value.status == 6
    # a leaf triangle range past the triangle array
    bad = bytearray(blob)
    info = oracle.blob_info(bytes(blob))
    topo = np.frombuffer(bytes(blob), dtype=np.uint32, count=info["n_nodes"], offset=off_topo)
    leaf = int(np.nonzero(topo & 0x80000000)[0][0])
    struct.pack_into("<I", bad, off_topo + 4 * leaf, (int(topo[leaf]) & ~0x07FFFFFF) | (info["n_tris"] & 0x07FFFFFF))
    with pytest.raises(cb.CbvhError):
        cb.cbvh_load(bytes(bad))


# ---- argument errors -----------------------------------------------------------------
def test_build_rejects_bad_inputs():
    V, T = meshes.icosphere(2, 0.1, np.random.default_rng(0))
    for kw in [dict(branching=3), dict(leaf_size=0), dict(leaf_size=9), dict(bits=4), dict(bv=7), dict(treelet_bytes=100)]:
        with pytest.raises(cb.CbvhError) as e:
            cb.cbvh_build(V, T, **kw)
        assert e.value.status == 1
    Tb = T.copy()
    Tb[3, 1] = len(V)
    with pytest.raises(cb.CbvhError):
        cb.cbvh_build(V, Tb)
    Vb = V.copy()
    Vb[5, 2] = np.nan
    with pytest.raises(cb.CbvhError):
        cb.cbvh_build(Vb, T)
    with pytest.raises(cb.CbvhError):
        cb.cbvh_build(V, T[:0])


def test_query_argument_errors_are_reported_before_any_launch():
    L = cb.lib()
    V, T = meshes.icosphere(2, 0.1, np.random.default_rng(0))
    a = cb.cbvh_build(V, T)
    b8 = cb.cbvh_build(V, T, bits=16)
    dop = cb.cbvh_build(V, T, bv=cb.DOP18, bits=8)
    fake = C.c_void_p(1 << 20)   # never dereferenced: validation fails first
    st = L.cbvh_collide(a, fake, dop, fake, fake, 4, 0, fake, None, 0, None, fake, fake, 1 << 30, None)
    assert st == 5  # different BV types
    st = L.cbvh_collide(a, fake, b8, fake, fake, 4, 0, fake, None, 0, None, fake, fake, 1 << 30, None)
    assert st == 5  # different code widths
    st = L.cbvh_collide(a, fake, a, fake, fake, 4, cb.PAIRS | cb.EARLY_EXIT, fake, fake, 8, fake, fake, fake, 1 << 30, None)
    assert st == 1
    st = L.cbvh_collide(a, fake, a, fake, fake, 4, cb.PAIRS, fake, None, 8, None, fake, fake, 1 << 30, None)
    assert st == 1  # pairs requested without buffers
    st = L.cbvh_collide(a, fake, a, fake, fake, 4, 0, fake, None, 0, None, fake, fake, 16, None)
    assert st == 4  # workspace too small
    st = L.cbvh_collide(a, None, a, fake, fake, 4, 0, fake, None, 0, None, fake, fake, 1 << 30, None)
    assert st == 1
    st = L.cbvh_collide(a, C.c_void_p((1 << 20) + 4), a, fake, fake, 4, 0, fake, None, 0, None, fake, fake, 1 << 30, None)
    assert st == 1  # misaligned model
    st = L.cbvh_distance(a, fake, a, fake, fake, 4, 0, None, fake, fake, 1 << 30, None)
    assert st == 1  # no output
    assert L.cbvh_collide(a, fake, a, fake, None, 0, 0, None, None, 0, None, None, None, 0, None) == 0  # n == 0
    assert cb.cbvh_last_error()
    assert cb.cbvh_workspace_bytes(a, a, 1000, cb.PAIRS, 1 << 20) > cb.cbvh_workspace_bytes(a, a, 1000, 0, 0)


def test_every_declared_function_is_exported():
    header = open(os.path.join(ROOT, "include", "cbvh.h")).read()
    names = sorted(set(re.findall(r"\b(cbvh_[a-z_]+)\s*\(", header)))
    assert "cbvh_collide" in names and "cbvh_distance" in names and len(names) >= 14
    L = C.CDLL(cb.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n


def test_wait_limit_argument_is_validated():
    with pytest.raises(cb.CbvhError):
        cb.cbvh_set_wait_limit(10 ** 12)
    cb.cbvh_set_wait_limit(5)
    cb.cbvh_set_wait_limit(0)
