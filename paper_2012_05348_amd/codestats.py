"""How much an integer stream coding of a model's corrector codes could save.

The paper names integer quantization followed by integer stream compression
as future work (section V).  This tool measures, on a built model, what such
codings of the predictor-corrector codes would gain over the fixed-width
codes the library stores, so that the choice not to use one rests on numbers:

* ``node_width``: every node's codes stored with the bit width of its largest
  code (a 5-bit width per node not counted);
* ``var2`` / ``var4``: every code stored in whole 2-bit (4-bit) units, at least
  one, with a per-code unit count (2 or 3 bits) beside it, the byte-aligned
  size per node; the GPU decodes one node per lane, so random access needs a
  per-node start as well, counted separately in ``offset_bytes_per_node``;
* ``ideal``: every code in exactly its bit length with no length information
  (a lower bound for any coding that keeps codes independent).

Only nodes whose bounds are codes relative to the parent count (treelet tops
hold absolute FP32 bounds).  Sizes are bytes; ``plain`` is what the library
stores (one or two bytes per code).

    python -m paper_2012_05348_amd.codestats

reports the library's collision, proximity and tiny workloads.
"""
from __future__ import annotations

import struct
import sys

import numpy as np

_MAGIC = b"CBVH"


def _parse(blob: bytes):
    if blob[:4] != _MAGIC:
        raise ValueError("not a compressed-BVH blob")
    _ver, _bv, K, bits, _bf, _leaf, n, _ntri, _nabs, _ntl, stride, _depth = struct.unpack("<12I", blob[4:52])
    offs = struct.unpack("<7Q", blob[56:112])
    topo = np.frombuffer(blob, np.uint32, n, offs[0])
    codes = np.frombuffer(blob, np.uint8, n * stride, offs[1]).reshape(n, stride)
    return K, bits, n, topo, codes, stride


def _bit_length(c):
    return np.where(c > 0, np.floor(np.log2(np.maximum(c, 1))).astype(np.int64) + 1, 0)


def code_stats(blob: bytes) -> dict:
    """Sizes of the relative nodes' codes under the codings described above."""
    K, bits, n, topo, codes, stride = _parse(blob)
    if bits not in (8, 16):
        raise ValueError("the model stores no integer codes (bits must be 8 or 16)")
    rel = ((topo >> 30) & 1) == 0
    c = (codes.view("<u2") if bits == 16 else codes).reshape(n, 2 * K)[rel].astype(np.int64)
    nb = _bit_length(c)
    out = {"K": int(K), "bits": int(bits), "relative_nodes": int(len(c)), "plain": int(len(c) * stride)}
    wmax = nb.max(axis=1) if len(c) else np.zeros(0, np.int64)
    out["node_width"] = int(((wmax * 2 * K + 7) // 8).sum())
    for gran in (2, 4):
        units = np.maximum((nb + gran - 1) // gran, 1)
        field = 2 if bits // gran <= 4 else 3  # bits of the per-code unit count
        node_bits = units.sum(axis=1) * gran + field * 2 * K
        out[f"var{gran}"] = int(((node_bits + 7) // 8).sum())
    out["ideal"] = int((nb.sum() + 7) // 8)
    out["offset_bytes_per_node"] = 2
    for key in ("node_width", "var2", "var4", "ideal"):
        out[f"{key}_ratio"] = out[key] / out["plain"] if out["plain"] else 1.0
    for gran in (2, 4):
        with_off = out[f"var{gran}"] + out["offset_bytes_per_node"] * len(c)
        out[f"var{gran}_with_offsets_ratio"] = with_off / out["plain"] if out["plain"] else 1.0
    return out


def main(argv=None):
    import os
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from synth import configs

    from . import AABB, DOP18, Model
    for idx, bits in ((1, 16), (1, 8), (2, 8), (0, 8)):
        w = configs.WORKLOADS[idx]
        _, (vb, tb) = w.meshes()
        m = Model.build(vb, tb, bv=AABB if w.bv == "aabb" else DOP18, branching=w.branching,
                        leaf_size=w.leaf_size, bits=bits)
        s = code_stats(m.blob())
        print(f"{w.name.split(':')[0]:10s} K={s['K']} bits={bits:2d}: plain {s['plain']} B; "
              + ", ".join(f"{k} {s[k + '_ratio']:.2f}" for k in ("node_width", "var2", "var4", "ideal"))
              + f"; var2 with 2-byte node offsets {s['var2_with_offsets_ratio']:.2f}")


if __name__ == "__main__":
    main()
