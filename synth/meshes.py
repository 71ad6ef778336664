"""Seeded synthetic triangle meshes.

These meshes stand in for the models of the open collision/proximity benchmark
that the paper times on (Results section); that data set is not available, so
closed, non-self-intersecting meshes of the same kind (curved closed surfaces,
10^3..10^5 triangles) are generated here instead.

Only geometry is produced (vertex and index arrays); nothing in this module
belongs to the collision method itself, so both the oracle and the GPU path
may consume its output.
"""
from __future__ import annotations

import numpy as np

__all__ = ["icosphere", "torus", "torus_grid_for", "box", "mesh_diameter"]


def _icosahedron():
    p = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array(
        [
            [-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
            [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
            [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1],
        ],
        dtype=np.float64,
    )
    f = np.array(
        [
            [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
            [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
            [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
            [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
        ],
        dtype=np.int64,
    )
    return v, f


def icosphere(freq: int, noise: float, rng: np.random.Generator, radius: float = 1.0):
    """Frequency-``freq`` geodesic sphere: 20*freq^2 triangles, 10*freq^2+2 vertices.

    Every face of the icosahedron is split into freq^2 triangles on a
    barycentric grid; grid points on shared edges/corners are shared, the points
    are projected to the sphere and each vertex gets radius
    ``radius * (1 + U(-noise, noise))``.  The surface is star-shaped around the
    origin, hence closed and free of self-intersections.  Faces are wound
    counter-clockwise seen from outside.
    """
    if freq < 1:
        raise ValueError("freq must be >= 1")
    base_v, base_f = _icosahedron()
    key_to_idx: dict = {}
    pts = []

    def vid(a, wa, b, wb, c, wc):
        # canonical key: sorted (corner, weight) pairs with non-zero weight
        key = tuple(sorted((int(x), int(w)) for x, w in ((a, wa), (b, wb), (c, wc)) if w))
        idx = key_to_idx.get(key)
        if idx is None:
            idx = len(pts)
            key_to_idx[key] = idx
            p = sum(w * base_v[x] for x, w in key) / freq
            pts.append(p)
        return idx

    tris = []
    n = freq
    for a, b, c in base_f:
        # grid point (i, j): weight n-i-j on a, i on b, j on c
        grid = {}
        for i in range(n + 1):
            for j in range(n + 1 - i):
                grid[(i, j)] = vid(a, n - i - j, b, i, c, j)
        for i in range(n):
            for j in range(n - i):
                tris.append((grid[(i, j)], grid[(i + 1, j)], grid[(i, j + 1)]))
                if i + j < n - 1:
                    tris.append((grid[(i + 1, j)], grid[(i + 1, j + 1)], grid[(i, j + 1)]))
    v = np.array(pts, dtype=np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    r = radius * (1.0 + rng.uniform(-noise, noise, size=len(v)))
    v *= r[:, None]
    t = np.array(tris, dtype=np.uint32)
    assert len(t) == 20 * n * n and len(v) == 10 * n * n + 2
    return v.astype(np.float32), t


def torus(U: int, V: int, R: float, r: float, noise: float, rng: np.random.Generator):
    """Closed torus on a U x V (theta, phi) grid: 2*U*V triangles, U*V vertices.

    Major radius ``R`` about the z axis; each vertex gets its own tube radius
    ``r + U(-noise, noise)``.  Every grid quad is split along the same
    diagonal; indices wrap so the surface is closed.
    """
    if U < 3 or V < 3:
        raise ValueError("U, V must be >= 3")
    th = 2.0 * np.pi * np.arange(U) / U
    ph = 2.0 * np.pi * np.arange(V) / V
    T, P = np.meshgrid(th, ph, indexing="ij")
    rr = r + rng.uniform(-noise, noise, size=(U, V))
    x = (R + rr * np.cos(P)) * np.cos(T)
    y = (R + rr * np.cos(P)) * np.sin(T)
    z = rr * np.sin(P)
    v = np.stack([x, y, z], axis=-1).reshape(-1, 3)
    iu = np.arange(U)[:, None]
    iv = np.arange(V)[None, :]
    a = iu * V + iv
    b = ((iu + 1) % U) * V + iv
    c = ((iu + 1) % U) * V + (iv + 1) % V
    d = iu * V + (iv + 1) % V
    t1 = np.stack([a, b, c], axis=-1).reshape(-1, 3)
    t2 = np.stack([a, c, d], axis=-1).reshape(-1, 3)
    t = np.empty((2 * U * V, 3), dtype=np.uint32)
    t[0::2] = t1
    t[1::2] = t2
    return v.astype(np.float32), t


def torus_grid_for(n_tris: int, R: float = 1.0, r: float = 0.3):
    """Grid (U, V) of a torus with about ``n_tris`` triangles, V/U ~ r/R."""
    V = max(3, int(round((n_tris / 2.0 * r / R) ** 0.5)))
    U = max(3, int(round(n_tris / (2.0 * V))))
    return U, V


def box(center, half):
    """Axis-aligned box as 12 outward-wound triangles (8 vertices)."""
    c = np.asarray(center, dtype=np.float64)
    h = np.asarray(half, dtype=np.float64) * np.ones(3)
    s = np.array([[x, y, z] for x in (-1, 1) for y in (-1, 1) for z in (-1, 1)], dtype=np.float64)
    v = c + s * h
    # vertex index = 4*(x>0) + 2*(y>0) + (z>0)
    f = [
        (0, 1, 3), (0, 3, 2),  # x-
        (4, 6, 7), (4, 7, 5),  # x+
        (0, 4, 5), (0, 5, 1),  # y-
        (2, 3, 7), (2, 7, 6),  # y+
        (0, 2, 6), (0, 6, 4),  # z-
        (1, 5, 7), (1, 7, 3),  # z+
    ]
    return v.astype(np.float32), np.array(f, dtype=np.uint32)


def mesh_diameter(v: np.ndarray) -> float:
    """Diagonal of the axis-aligned bounding box of the vertices (FP64)."""
    v = np.asarray(v, dtype=np.float64)
    return float(np.linalg.norm(v.max(axis=0) - v.min(axis=0)))
