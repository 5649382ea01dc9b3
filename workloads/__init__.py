"""Seeded synthetic inputs for the AMG eigensolver: meshes, P1 matrices, random blocks.

Shared by the oracle, the tests and the benchmark; contains none of the
eigensolver's arithmetic.
"""
from . import prng, fem, configs  # noqa: F401
