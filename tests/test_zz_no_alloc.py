"""GPU test of the allocation-free collision entry point (cbvh_collide_static):
its answers equal cbvh_collide's (with a caller workspace) on two calls in a
row, the second with a smaller batch, and a batch beyond its fixed
workspace is rejected before anything runs."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2012_05348_amd as cb  # noqa: E402
import workloads as W  # noqa: E402
from synth import configs  # noqa: E402

DEV = "cuda:0"


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _models(cfg):
    w = configs.WORKLOADS[cfg]
    (va, ta), (vb, tb) = W.meshes(cfg)
    kw = dict(bv=W.BV[w.bv], branching=w.branching, leaf_size=w.leaf_size, bits=w.bits)
    return cb.Model.build(va, ta, **kw).to(DEV), cb.Model.build(vb, tb, **kw).to(DEV)


def _static(ma, mb, Pd, flags):
    n = int(Pd.shape[0])
    hit = torch.full((n,), 7, dtype=torch.uint8, device=DEV)
    st = torch.full((n,), 9, dtype=torch.uint8, device=DEV)
    cb.cbvh_collide_static(ma.handle, ma.dev, mb.handle, mb.dev, Pd, n, flags, hit, st)
    return hit.cpu().numpy(), st.cpu().numpy()


@pytest.mark.parametrize("cfg", [1, 0])
def test_static_workspace_collide_equals_collide(cfg):
    ma, mb = _models(cfg)
    w = configs.WORKLOADS[cfg]
    P = w.raw_poses(16384)
    for i, (lo, hi) in enumerate(((0, 16384), (5000, 7500))):
        _log(f"static-workspace collide: workload {cfg}, call {i}, poses {lo}:{hi}")
        Pd = torch.from_numpy(P[lo:hi]).to(DEV)
        ref_h, ref_s = cb.collide(ma, mb, Pd, flags=cb.EARLY_EXIT)
        got_h, got_s = _static(ma, mb, Pd, cb.EARLY_EXIT)
        assert (ref_s.cpu().numpy() == 0).all() and (got_s == 0).all()
        assert np.array_equal(got_h, ref_h.cpu().numpy()), (cfg, i)


def test_static_workspace_rejects_batches_beyond_its_size():
    ma, mb = _models(0)
    n = cb.STATIC_MAX_POSES + 1
    Pd = torch.zeros((n, 3, 4), dtype=torch.float32, device=DEV)
    hit = torch.empty(n, dtype=torch.uint8, device=DEV)
    st = torch.empty(n, dtype=torch.uint8, device=DEV)
    with pytest.raises(cb.CbvhError, match="fixed workspace"):
        cb.cbvh_collide_static(ma.handle, ma.dev, mb.handle, mb.dev, Pd, n, cb.EARLY_EXIT, hit, st)
