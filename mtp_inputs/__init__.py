"""Seeded synthetic inputs shared by the GPU library's tests/bench and the CPU oracle.

This package holds problem data only: meshes, material layouts, initial fields and
exact solutions of Maxwell's equations.  It contains none of the tent-pitching,
DG or time-stepping arithmetic; both sides implement that on their own.
"""
from . import meshes, fields  # noqa: F401
