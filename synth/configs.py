"""The synthetic workloads: meshes, build parameters and raw pose streams.

Seeds: numpy ``Generator(PCG64(SEED_BASE + 1000*config + stream))`` with
stream 0 = mesh A (moving), 1 = mesh B (fixed), 2 = poses.

The raw pose stream of a workload is deterministic; validity filtering
(rejecting poses within the penetration/separation margin) needs exact
geometry and is done by whoever checks results, not here.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import meshes, poses

SEED_BASE = 201205348


def rng_for(config: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(SEED_BASE + 1000 * config + stream))


@dataclass(frozen=True)
class MeshSpec:
    kind: str          # "icosphere" | "torus"
    size: tuple        # (freq,) or (U, V)
    noise: float

    def make(self, rng):
        if self.kind == "icosphere":
            return meshes.icosphere(self.size[0], self.noise, rng)
        if self.kind == "torus":
            return meshes.torus(self.size[0], self.size[1], 1.0, 0.3, self.noise, rng)
        raise ValueError(self.kind)

    @property
    def n_tris(self):
        return 20 * self.size[0] ** 2 if self.kind == "icosphere" else 2 * self.size[0] * self.size[1]


@dataclass(frozen=True)
class Workload:
    index: int
    name: str
    mesh_a: MeshSpec
    mesh_b: MeshSpec
    bv: str            # "aabb" | "dop18"
    branching: int
    leaf_size: int
    bits: int          # compressed code width; the uncompressed twin uses 0
    n_poses: int
    query: str         # "pairs" | "bool" | "distance"
    translation: tuple  # ("box", half) | ("shell", rmin, rmax)
    margin_rel: float = 1e-4

    def meshes(self):
        va, ta = self.mesh_a.make(rng_for(self.index, 0))
        vb, tb = self.mesh_b.make(rng_for(self.index, 1))
        return (va, ta), (vb, tb)

    def raw_poses(self, n: int | None = None) -> np.ndarray:
        """First ``n`` poses (default ``n_poses``) of the workload's seeded pose stream."""
        n = self.n_poses if n is None else n
        rng = rng_for(self.index, 2)
        R = poses.uniform_rotations(n, rng)
        if self.translation[0] == "box":
            t = poses.box_translations(n, self.translation[1], rng)
        else:
            t = poses.shell_translations(n, self.translation[1], self.translation[2], rng)
        return poses.compose(R, t)

    def margin(self, va, vb) -> float:
        """Penetration/separation margin: margin_rel x max(AABB diagonal of A, of B)."""
        return self.margin_rel * max(meshes.mesh_diameter(va), meshes.mesh_diameter(vb))


ICO8 = MeshSpec("icosphere", (8,), 0.1)        # 1,280 triangles
TORUS100K = MeshSpec("torus", (400, 125), 0.02)  # 100,000 triangles
ICO50 = MeshSpec("icosphere", (50,), 0.1)      # 50,000 triangles
TORUS50K = MeshSpec("torus", (250, 100), 0.02)   # 50,000 triangles

WORKLOADS = {
    0: Workload(0, "tiny: icosphere 1,280 vs icosphere 1,280, AABB BF4 leaf1, 8-bit, pair lists",
                ICO8, ICO8, "aabb", 4, 1, 8, 256, "pairs", ("box", 2.5)),
    1: Workload(1, "scaled: torus 100k vs torus 100k, 18-DOP BF8 leaf4, 16-bit, collision booleans",
                TORUS100K, TORUS100K, "dop18", 8, 4, 16, 16384, "bool", ("box", 1.5)),
    2: Workload(2, "proximity: icosphere 50k vs torus 50k, AABB BF4 leaf1, 8-bit, distances",
                ICO50, TORUS50K, "aabb", 4, 1, 8, 4096, "distance", ("shell", 2.0, 4.0)),
}
