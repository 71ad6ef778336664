"""Pin of the oracle's blob decoder against hand-computed values.

Decode rule of a node relative to its decoded parent [Pl, Ph] (per slab,
b-bit codes ql, qh): E = Ph - Pl in float32, s = E * 2^-b,
lo = fma(ql, s, Pl), hi = fma(-qh, s, Ph), each rounded once to float32.
Expected values below are computed independently: with a power-of-two s the
results are exact dyadic numbers; otherwise the exact product-sum fits in
float64 and is rounded once to float32.
"""
import numpy as np
import pytest

import oracle
from blobfmt import assemble, topo_word


def _tri_blob(bits, root, codes_child, K=3):
    """root (absolute) with two leaf children; child 1 gets `codes_child`, child 2 all-zero codes."""
    stride = (bits // 8) * 2 * K
    codes = np.zeros((3, stride), dtype=np.uint8)
    codes[0, :4] = np.frombuffer(np.uint32(0).tobytes(), np.uint8)    # abs index 0
    codes[1] = np.frombuffer(np.asarray(codes_child, dtype=np.uint8 if bits == 8 else np.uint16).tobytes(), np.uint8)
    topo = [topo_word(1, 2, absolute=True), topo_word(0, 1, leaf=True), topo_word(1, 1, leaf=True)]
    tris = np.zeros((2, 9), dtype=np.float32)
    return assemble(0, bits, 2, 1, topo, codes, np.asarray(root, np.float32), tris, [0, 1], [0, 3])


def test_decode_dyadic_8bit():
    root = [0.0, 1.0, -1.0, 3.0, 2.0, 2.0]        # slabs x, y, z (z degenerate: E = 0)
    blob = _tri_blob(8, root, [64, 32, 3, 255, 7, 9])
    dec = oracle.blob_decode(blob)
    assert dec.shape == (3, 6)
    np.testing.assert_array_equal(dec[0], np.float32(root))
    # x: s = 2^-8: lo = 64/256, hi = 1 - 32/256
    # y: E = 4, s = 2^-6: lo = -1 + 3/64, hi = 3 - 255/64
    # z: E = 0 -> s = 0 -> both bounds equal the parent's
    np.testing.assert_array_equal(dec[1], np.float32([0.25, 0.875, -1 + 3 / 64, 3 - 255 / 64, 2.0, 2.0]))
    # zero codes reproduce the parent exactly
    np.testing.assert_array_equal(dec[2], np.float32(root))


def _fma32(a, b, c):
    """float32 fma with a single rounding: the exact value fits in float64 for these operands."""
    exact = float(np.float32(a)) * float(np.float32(b)) + float(np.float32(c))
    return np.float32(exact)


def test_decode_rounded_16bit():
    Pl, Ph = np.float32(0.1), np.float32(0.7)
    root = [Pl, Ph, np.float32(-0.3), np.float32(1.9), np.float32(0.0), np.float32(1e-3)]
    q = [5, 7, 40000, 65535, 1, 0]
    blob = _tri_blob(16, root, q)
    dec = oracle.blob_decode(blob)
    expect = []
    for k in range(3):
        lo_p, hi_p = np.float32(root[2 * k]), np.float32(root[2 * k + 1])
        E = np.float32(hi_p - lo_p)
        s = np.float32(float(E) * 2.0 ** -16)      # power-of-two scaling: exact
        expect += [_fma32(q[2 * k], s, lo_p), _fma32(-q[2 * k + 1], s, hi_p)]
    np.testing.assert_array_equal(dec[1], np.float32(expect))
    # decoded child stays inside the decoded parent even with the largest code
    assert dec[1][3] >= dec[0][2]


def test_decode_rejects_corrupt_blobs():
    blob = bytearray(_tri_blob(8, [0, 1, 0, 1, 0, 1], [0] * 6))
    with pytest.raises(ValueError):
        oracle.blob_decode(bytes(blob[:100]))
    bad = bytearray(blob)
    bad[0] = ord("X")
    with pytest.raises(ValueError):
        oracle.blob_decode(bytes(bad))


def test_decode_fp16_closed_forms():
    # a root with two leaf children; every bound a binary16 value whose real
    # value is known in closed form
    halves = {0x3C00: 1.0, 0xBC00: -1.0, 0x3555: 0.333251953125, 0x0001: 2.0 ** -24, 0x7BFF: 65504.0,
              0xC400: -4.0, 0x8400: -(2.0 ** -14), 0x3E00: 1.5, 0x0000: 0.0, 0x4248: 3.140625,
              0x03FF: 1023 * 2.0 ** -24, 0xD140: -42.0}
    keys = list(halves)
    root = [0xC400, 0x7BFF, 0xD140, 0x4248, 0x8400, 0x3E00]          # (lo, hi) per axis
    c1 = [0xBC00, 0x3C00, 0x0000, 0x3555, 0x0001, 0x03FF]
    c2 = [0x3555, 0x3E00, 0xBC00, 0x0001, 0x8400, 0x3C00]
    codes = np.zeros((3, 12), dtype=np.uint8)
    for i, row in enumerate((root, c1, c2)):
        codes[i] = np.frombuffer(np.array(row, dtype="<u2").tobytes(), dtype=np.uint8)
    topo = [topo_word(1, 2), topo_word(0, 1, leaf=True), topo_word(1, 1, leaf=True)]
    blob = assemble(0, 0x8010, 2, 1, topo, codes, np.zeros((0, 6)), np.zeros((2, 9)), [0, 1], [0, 3],
                            depth=1)
    out = oracle.blob_decode(blob)
    want = np.array([[halves[h] for h in row] for row in (root, c1, c2)], dtype=np.float64)
    assert np.array_equal(out.astype(np.float64), want)
    assert set(keys) >= set(root + c1 + c2)


def test_decode_fp16_rejects_non_finite_bounds():
    codes = np.zeros((1, 12), dtype=np.uint8)
    codes[0, :2] = np.frombuffer(np.array([0x7C00], dtype="<u2").tobytes(), dtype=np.uint8)  # +inf
    blob = assemble(0, 0x8010, 2, 1, [topo_word(0, 1, leaf=True)], codes, np.zeros((0, 6)),
                            np.zeros((1, 9)), [0], [0, 1])
    with pytest.raises(ValueError):
        oracle.blob_decode(blob)
