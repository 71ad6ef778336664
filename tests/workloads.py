"""Test-side preparation of the synthetic workloads: meshes, models and
margin-filtered poses (the filter runs the oracle's margin classification;
the GPU path never sees the oracle)."""
from __future__ import annotations

import functools

import numpy as np

import oracle
from synth import configs

BV = {"aabb": 0, "dop18": 1}


@functools.lru_cache(maxsize=None)
def meshes(cfg):
    return configs.WORKLOADS[cfg].meshes()


@functools.lru_cache(maxsize=None)
def oracle_meshes(cfg):
    (va, ta), (vb, tb) = meshes(cfg)
    return oracle.Mesh(va, ta), oracle.Mesh(vb, tb)


@functools.lru_cache(maxsize=None)
def config0_poses():
    """256 poses of the tiny workload: the first 128 colliding and the first 128
    separated poses of the seeded stream that have no triangle pair within the
    pair-level margin band (-m, m)."""
    w = configs.WORKLOADS[0]
    (va, ta), (vb, tb) = meshes(0)
    A, B = oracle_meshes(0)
    m = w.margin(va, vb)
    raw = w.raw_poses(4096)
    cls = oracle.classify_batch(A, B, raw, m, pair_level=True)
    col = np.nonzero(cls == oracle.COLLIDING)[0][:128]
    sep = np.nonzero(cls == oracle.SEPARATED)[0][:128]
    assert len(col) == 128 and len(sep) == 128
    idx = np.sort(np.concatenate([col, sep]))
    return raw[idx], int(np.count_nonzero(cls[: idx[-1] + 1] == oracle.MARGINAL))

