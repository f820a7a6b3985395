"""Seeded synthetic inputs shared by the HIP path, the oracle, the tests and the benchmark.

This package holds problem *descriptions* only: lattices (site list), term lists with couplings,
parameter vectors and random state vectors.  It contains none of the matrix-free method's arithmetic
(no index decoding, no ladder coefficients, no matvec), so the oracle and the GPU path can both consume
its output without sharing any of the computation they are compared on.
"""
from .model import (SPIN, BOSON, OP_Z, OP_Z2, OP_RAISE, OP_LOWER, OP_RAISE2, OP_LOWER2, OP_LOCAL_BASE, LocalOp, Site, Term,
                    Model,
                    spin_site, boson_site, dim_of, xxz_bond_terms)
from .configs import (heisenberg_chain, ferrimagnetic_ring, square_lattice_spin1, batched_chains,
                      tavis_cummings, random_model, xx_chain_in_field, random_state, config,
                      staggered_xxz_ring, paper_c1, paper_c2, zero_field_splitting,
                      spin_matrices, band_op, bilinear_biquadratic_chain, adjoint_op,
                      random_general_model, truncated_spin_ops)

__all__ = [
    "SPIN", "BOSON", "OP_Z", "OP_Z2", "OP_RAISE", "OP_LOWER", "OP_RAISE2", "OP_LOWER2", "OP_LOCAL_BASE", "LocalOp", "Site", "Term",
    "Model",
    "spin_site", "boson_site", "dim_of", "xxz_bond_terms", "heisenberg_chain", "ferrimagnetic_ring",
    "square_lattice_spin1", "batched_chains", "tavis_cummings", "random_model", "xx_chain_in_field",
    "random_state", "config", "staggered_xxz_ring", "paper_c1", "paper_c2", "zero_field_splitting",
    "spin_matrices", "band_op", "bilinear_biquadratic_chain", "adjoint_op", "random_general_model",
    "truncated_spin_ops",
]
