"""Seeded synthetic inputs for the SpGEMM hot path.

This module only builds input matrices (and random draws handed to the
method as inputs).  It contains none of the product arithmetic, so both the
CPU oracle and the GPU path can take their inputs from here without sharing
any code of the method itself.
"""

from .gen import (  # noqa: F401
    CSR,
    canonical_from_coo,
    er_uniform_columns,
    rmat,
    poisson7,
    aggregation_2x2x2,
    identity,
    permutation_matrix,
    permute_symmetric,
    random_csr,
    with_values,
    layer_bounds,
    submatrix,
    process_share,
    galerkin_batch,
    G500,
    SSCA,
    ER,
)
