"""Seeded synthetic inputs for the HDG hot path: meshes and element blocks.

This package is the input generator shared by the oracle and the GPU path. It
produces the element matrices of one Newton linearisation (the inputs of the
condensation step); it contains no condensation, assembly, Krylov or
preconditioner arithmetic.
"""
from . import basis, quadrature, mesh, physics, blocks, configs  # noqa: F401
