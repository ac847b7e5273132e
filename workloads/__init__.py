"""Seeded synthetic inputs (meshes and flow maps) for the FTLE hot path.

Input generation only: shared by the oracle-side tests and by the GPU side,
it computes no part of the FTLE method.
"""
from . import configs, flows, meshes  # noqa: F401
