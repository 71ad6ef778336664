"""Seeded synthetic inputs (meshes and rigid poses) shared by the oracle and the GPU path."""
from . import configs, meshes, poses  # noqa: F401
