"""Seeded input generators for the GPU decoder and its FP64 oracle (codes, noise)."""
from .codes import (StabilizerCode, planar, toric, xzzx, trapping_ring, make, gf2_rank,
                    gf2_nullspace, symplectic_product, logical_basis, depolarizing_probs,
                    biased_probs, thresholds, config_seed, hypergraph_product, bivariate_bicycle,
                    bb, BB_CODES, chamon)
