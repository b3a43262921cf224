"""Seeded synthetic inputs for the laplacianFoam assembly + PCG path.

This package only *generates inputs*: box meshes in OpenFOAM face-addressing
form (owner/neighbour, volumes, centres, face area vectors, boundary patches),
renumberings of those meshes, initial temperature fields and request streams.
It contains none of the method's arithmetic (no coefficients, no matrix, no
solver), so both the oracle and the GPU library can consume it without sharing
any part of the computation they are compared on.
"""
from .rng import splitmix64, uniform01
from .mesh import (BoxMesh, box_mesh, from_arrays, box_aggregation, graded_nodes, renumber, random_permutation, affine, SKEW, STEEP,
                   red_black_numbering, initial_field, fixed_x_bcs, all_zero_gradient,
                   ZERO_GRADIENT, FIXED_VALUE, PATCH_NAMES)
from .configs import CONFIGS, TOL, REL_TOL, MAX_ITER, build_config, request_stream

__all__ = [
    "splitmix64", "uniform01", "BoxMesh", "box_mesh", "from_arrays", "box_aggregation", "graded_nodes", "renumber",
    "random_permutation", "affine", "SKEW", "STEEP", "red_black_numbering", "initial_field", "fixed_x_bcs",
    "all_zero_gradient", "ZERO_GRADIENT", "FIXED_VALUE", "PATCH_NAMES", "CONFIGS", "TOL",
    "REL_TOL", "MAX_ITER", "build_config", "request_stream",
]
