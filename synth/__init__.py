"""Seeded synthetic inputs for the CSRC sparse matrix-vector product.

This package only *generates inputs*: sparsity patterns shaped like finite
element matrices (2D/3D stencils, tetrahedral meshes with 3x3 blocks, banded
and power-law graphs), node orderings, matrix values and source vectors.  It
holds none of the product's arithmetic and none of the CSRC format logic: its
output is an ordinary CSR matrix ``(n, rowptr, col, val)``.  Both the CPU
oracle and the GPU path consume the same generated arrays.

Randomness is counter based (SplitMix64 keyed by seed and position) so that a
value depends only on the seed and on the *original* node pair, never on the
numbering or on the order of generation.
"""

from .rng import splitmix64, uniform_pm1, uniform01, randint_pm
from .patterns import (
    CSR,
    stencil_offsets_2d,
    stencil_offsets_3d,
    grid_stencil,
    q1_quad,
    q1_hex,
    kuhn_tet,
    block_expand,
    banded,
    power_law,
    permute,
    random_order,
    rcm_order,
    reorder,
)
from .values import fill_values, vector, block_vector
from . import workloads

__all__ = [
    "splitmix64", "uniform_pm1", "uniform01", "randint_pm",
    "CSR", "stencil_offsets_2d", "stencil_offsets_3d", "grid_stencil",
    "q1_quad", "q1_hex", "kuhn_tet", "block_expand", "banded", "power_law",
    "permute", "random_order", "rcm_order", "reorder",
    "fill_values", "vector", "block_vector", "workloads",
]
