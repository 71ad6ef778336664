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


# ---------------------------------------------------------------------------
# Batched workload: one moving link against many obstacles of uneven size
# ---------------------------------------------------------------------------
TORUS20K = MeshSpec("torus", (200, 50), 0.02)  # 20,000 triangles


@dataclass(frozen=True)
class BatchedWorkload:
    """A robot link (20k-triangle torus, moving) queried against ``n_obstacles``
    obstacle meshes whose triangle counts are log-uniform in [tri_min, tri_max]
    (noisy icospheres or tori, each with probability 1/2).  Pose batches cycle
    through the obstacles; each batch has a log-uniform size in
    [batch_min, batch_max]; batches are drawn until ``min_poses`` poses exist.
    Seeds: stream 0 the link, 3 obstacle kinds and sizes, 5 batch sizes,
    2 poses, 100 + i obstacle i."""
    index: int = 3
    n_obstacles: int = 64
    tri_min: int = 1000
    tri_max: int = 200000
    batch_min: int = 1
    batch_max: int = 1024
    min_poses: int = 30000
    link: MeshSpec = TORUS20K
    bv: str = "dop18"
    branching: int = 8
    leaf_size: int = 4
    bits: int = 16
    query: str = "bool"
    translation: tuple = ("box", 2.5)
    margin_rel: float = 1e-4

    @property
    def name(self):
        return (f"batched: torus 20k link vs {self.n_obstacles} obstacles ({self.tri_min}-{self.tri_max} tri), "
                f"18-DOP BF{self.branching} leaf {self.leaf_size}, {self.bits}-bit, booleans")

    def obstacle_specs(self):
        rng = rng_for(self.index, 3)
        kinds = rng.random(self.n_obstacles) < 0.5
        sizes = np.exp(rng.uniform(np.log(self.tri_min), np.log(self.tri_max), self.n_obstacles))
        specs = []
        for is_ico, n in zip(kinds, sizes):
            if is_ico:
                specs.append(MeshSpec("icosphere", (max(1, int(round((n / 20.0) ** 0.5))),), 0.1))
            else:
                specs.append(MeshSpec("torus", meshes.torus_grid_for(int(n)), 0.02))
        return specs

    def obstacle_mesh(self, i: int):
        return self.obstacle_specs()[i].make(rng_for(self.index, 100 + i))

    def link_mesh(self):
        return self.link.make(rng_for(self.index, 0))

    def batches(self):
        """[(obstacle, count)] in launch order."""
        rng = rng_for(self.index, 5)
        out, total, i = [], 0, 0
        while total < self.min_poses:
            c = int(np.floor(np.exp(rng.uniform(np.log(self.batch_min), np.log(self.batch_max + 1)))))
            c = min(max(c, self.batch_min), self.batch_max)
            out.append((i % self.n_obstacles, c))
            total += c
            i += 1
        return out

    def raw_poses(self):
        """(poses float32 [n, 3, 4], obstacle index uint32 [n]), batches contiguous."""
        b = self.batches()
        n = sum(c for _, c in b)
        rng = rng_for(self.index, 2)
        R = poses.uniform_rotations(n, rng)
        t = poses.box_translations(n, self.translation[1], rng)
        obj = np.concatenate([np.full(c, o, dtype=np.uint32) for o, c in b])
        return poses.compose(R, t), obj


BATCHED = BatchedWorkload()

# Serving workload: 32 resident obstacles of 1k-200k triangles and the same
# 20k-triangle link; requests come from paper_2012_05348_amd.serve.make_requests
# with a generator seeded by rng_for(4, 2).
SERVING = BatchedWorkload(index=4, n_obstacles=32, min_poses=0)
