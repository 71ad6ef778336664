"""Hand assembly of compressed-BVH blobs from the byte layout (test helper).

Layout (little endian): 128-byte header, then 256-byte aligned sections
topo[n] u32, codes[n][stride], abs[n_abs][2K] f32, tris[n_tris][9] f32,
perm[n_tris] u32, treelets[n_treelets+1] u32.  Topology word: bit31 leaf,
bit30 absolute, bits27-29 count-1, bits0-26 first child / first triangle.
"""
import struct

import numpy as np


def _align(x, a=256):
    return (x + a - 1) // a * a


def topo_word(first, count, leaf=False, absolute=False):
    return (first & 0x07FFFFFF) | ((count - 1) << 27) | (int(absolute) << 30) | (int(leaf) << 31)


def assemble(bv, bits, branching, leaf_size, topo, codes, abs_bounds, tris, perm, treelets, depth=0,
             treelet_bytes=0, max_abs_coord=0.0):
    K = 3 if bv == 0 else 9
    stride = 8 * K if bits == 0 else 4 * K if bits == 0x8010 else (bits // 8) * 2 * K
    topo = np.asarray(topo, dtype=np.uint32)
    codes = np.asarray(codes, dtype=np.uint8).reshape(len(topo), stride)
    abs_bounds = np.asarray(abs_bounds, dtype=np.float32).reshape(-1, 2 * K)
    tris = np.asarray(tris, dtype=np.float32).reshape(-1, 9)
    perm = np.asarray(perm, dtype=np.uint32)
    treelets = np.asarray(treelets, dtype=np.uint32)
    secs = [topo.tobytes(), codes.tobytes(), abs_bounds.tobytes(), tris.tobytes(), perm.tobytes(), treelets.tobytes()]
    offs, cur = [], 128
    for s in secs:
        cur = _align(cur)
        offs.append(cur)
        cur += len(s)
    total = _align(cur)
    hdr = b"CBVH" + struct.pack("<12I", 1, bv, K, bits, branching, leaf_size, len(topo), len(perm),
                                len(abs_bounds), len(treelets) - 1, stride, depth)
    hdr += struct.pack("<I", treelet_bytes) + struct.pack("<7Q", *offs, total) + struct.pack("<f", max_abs_coord)
    hdr = hdr.ljust(128, b"\0")
    buf = bytearray(total)
    buf[:128] = hdr
    for o, s in zip(offs, secs):
        buf[o:o + len(s)] = s
    return bytes(buf)
