"""Seeded rigid poses.

A pose is a float32 [3, 4] matrix [R | t]; a point x of the moving mesh A is
placed in the frame of the fixed mesh B as R @ x + t.  The float32 matrix is
the canonical pose: every consumer promotes exactly these values.
"""
from __future__ import annotations

import numpy as np

__all__ = ["uniform_rotations", "quat_to_matrix", "compose", "box_translations", "shell_translations", "invert"]


def quat_to_matrix(q: np.ndarray) -> np.ndarray:
    """Unit quaternions (..., 4) as (x, y, z, w) -> float64 rotation matrices (..., 3, 3)."""
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    x, y, z, w = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    m = np.empty(q.shape[:-1] + (3, 3))
    m[..., 0, 0] = 1 - 2 * (y * y + z * z)
    m[..., 0, 1] = 2 * (x * y - z * w)
    m[..., 0, 2] = 2 * (x * z + y * w)
    m[..., 1, 0] = 2 * (x * y + z * w)
    m[..., 1, 1] = 1 - 2 * (x * x + z * z)
    m[..., 1, 2] = 2 * (y * z - x * w)
    m[..., 2, 0] = 2 * (x * z - y * w)
    m[..., 2, 1] = 2 * (y * z + x * w)
    m[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return m


def uniform_rotations(n: int, rng: np.random.Generator) -> np.ndarray:
    """n uniformly distributed rotations (Shoemake's subgroup algorithm), float64 (n, 3, 3)."""
    u1, u2, u3 = rng.random(n), rng.random(n), rng.random(n)
    a, b = np.sqrt(1.0 - u1), np.sqrt(u1)
    q = np.stack(
        [a * np.sin(2 * np.pi * u2), a * np.cos(2 * np.pi * u2), b * np.sin(2 * np.pi * u3), b * np.cos(2 * np.pi * u3)],
        axis=-1,
    )
    return quat_to_matrix(q)


def box_translations(n: int, half: float, rng: np.random.Generator) -> np.ndarray:
    return rng.uniform(-half, half, size=(n, 3))


def shell_translations(n: int, rmin: float, rmax: float, rng: np.random.Generator) -> np.ndarray:
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    return d * rng.uniform(rmin, rmax, size=(n, 1))


def compose(R: np.ndarray, t: np.ndarray) -> np.ndarray:
    """(n,3,3) rotations + (n,3) translations -> canonical float32 poses (n, 3, 4)."""
    P = np.concatenate([np.asarray(R, np.float64), np.asarray(t, np.float64)[:, :, None]], axis=2)
    return np.ascontiguousarray(P.astype(np.float32))


def invert(poses: np.ndarray) -> np.ndarray:
    """Inverse rigid motions in float64 (n, 3, 4): x_A = R^T (x_B - t)."""
    P = np.asarray(poses, dtype=np.float64)
    Rt = np.transpose(P[:, :, :3], (0, 2, 1))
    t = -np.einsum("nij,nj->ni", Rt, P[:, :, 3])
    return np.concatenate([Rt, t[:, :, None]], axis=2)
