"""Seeded synthetic inputs shared by the tests, the bench and the reference checker.

This module only *builds inputs*: matrices with an exactly known singular spectrum, Gaussian test
matrices and serving-load draws.  It holds none of the single-pass PCA arithmetic, and it imports
neither the reference implementation under ``oracle/`` nor the HIP library.

Spectra follow the paper's accuracy study (Sec. 4.1, Types 1-5) and the workload recipes written
down in the design notes (exp, 1/j, j^-2 decays with a noise term on sigma).
"""
from .spectra import (paper_type_spectrum, noisy_spectrum, exp_spectrum, inv_spectrum,
                      inv_floor_spectrum, inv_square_spectrum)
from .matrices import (orthonormal_factor, small_matrix, KronMatrix, StackedPool,
                       gaussian_omega, low_rank_matrix)
from .serving import ServingDraws, draw_serving_streams, serving_pool_torch

__all__ = [
    "paper_type_spectrum", "noisy_spectrum", "exp_spectrum", "inv_spectrum", "inv_floor_spectrum",
    "inv_square_spectrum", "orthonormal_factor", "small_matrix", "KronMatrix", "StackedPool",
    "gaussian_omega", "low_rank_matrix", "ServingDraws", "draw_serving_streams", "serving_pool_torch",
]
