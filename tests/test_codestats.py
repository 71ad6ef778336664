"""The code-statistics tool (sizes of integer stream codings of the corrector
codes, the paper's future-work direction) on a hand-assembled blob whose code
bit lengths are known, and its consistency on a built model."""
import numpy as np
import pytest

from blobfmt import assemble, topo_word
from paper_2012_05348_amd.codestats import code_stats


def _blob(codes_rel):
    # node 0: absolute root (code slot = abs index 0); nodes 1, 2: relative leaves
    topo = [topo_word(1, 2, absolute=True), topo_word(0, 1, leaf=True), topo_word(1, 1, leaf=True)]
    codes = np.zeros((3, 6), np.uint8)
    codes[1:] = codes_rel
    tris = np.zeros((2, 9), np.float32)
    return assemble(0, 8, 2, 1, topo, codes, np.zeros((1, 6), np.float32), tris, np.arange(2), [0, 3])


def test_known_code_lengths():
    # bit lengths: node 1 -> 0,1,2,2,8,5 (18 bits); node 2 -> all zero
    s = code_stats(_blob([[0, 1, 2, 3, 255, 16], [0, 0, 0, 0, 0, 0]]))
    assert s["relative_nodes"] == 2 and s["plain"] == 12
    assert s["node_width"] == 6 + 0            # 8 bits x 6 codes, then width 0
    assert s["var2"] == 5 + 3                  # 11 units x 2 + 12 count bits = 34 -> 5 B; 6 x 2 + 12 = 24 -> 3 B
    assert s["var4"] == 6 + 5                  # 8 units x 4 + 12 = 44 -> 6 B; 6 x 4 + 12 = 36 -> 5 B
    assert s["ideal"] == 3                     # 18 bits


def test_rejects_a_non_blob():
    with pytest.raises(ValueError):
        code_stats(b"XXXX" + bytes(124))


@pytest.mark.parametrize("bits", [8, 16])
def test_built_model_orders(bits):
    import paper_2012_05348_amd as cb
    from synth import meshes
    V, T = meshes.icosphere(6, 0.1, np.random.default_rng(7))
    m = cb.Model.build(V, T, bv=cb.DOP18, branching=4, leaf_size=1, bits=bits)
    s = code_stats(m.blob())
    assert s["plain"] == s["relative_nodes"] * 2 * 9 * bits // 8
    assert s["ideal"] <= s["node_width"] <= s["plain"]
    assert s["ideal"] <= s["var2"] and s["ideal"] <= s["var4"]
