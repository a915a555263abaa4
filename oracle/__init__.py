"""Reference implementation of single-pass PCA (Yu et al., "Single-Pass PCA of Large
High-Dimensional Data", IJCAI 2017), in plain FP64 NumPy.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links this package: only
the tests, the package smoke check and the CPU-baseline leg of the benchmark use it.  It shares no
code, constants or helpers with the HIP library; both sides receive their inputs from ``synth``.

Modules
  pca       Algorithm 4 (single pass, re-orthogonalised column-block loop, SVD of B),
            Algorithm 1 (two-pass basic randomised SVD) as a cross-check, the power scheme with
            P = 1 (Sec. 3.3, 4.2) and implicit column centring (Sec. 2.1).
  alg2      Algorithm 2, the earlier single-pass algorithm of the accuracy study (Sec. 4.1).
  philox    Philox-4x64-10 counter-based generator and the Box-Muller Gaussian test matrix.
  rounding  Round-to-nearest-even conversions to FP32, BF16 and FP8 E4M3 used to build the exact
            quantised operands a reduced-precision kernel consumes.
  jacobi    Brute-force one-sided Jacobi SVD for tiny matrices.
  metrics   Relative singular-value error, subspace angles, sign convention.

Every function cites the passage of the paper it follows.  All pins live in ``tests/``.
Parity-unpinned items: the paper's printed accuracy figures for its 3000x3000 Type-1 matrix
(Sec. 4.1), Algorithm 2's errors there and the power scheme's max_err figures (Sec. 4.2) depend on
its undisclosed random draws and matrices, so they are checked to order of magnitude only.
"""
from .pca import (sketch_pass, qb_from_sketch, svd_from_qb, single_pass_pca, basic_randqb_svd,
                  apply_sign_convention, PCAResult, power_omega, single_pass_pca_power,
                  sketch_pass_centred, centre_sketch, single_pass_pca_centred)
from .alg2 import alg2_single_pass
from .philox import philox4x64_10, philox_words, gaussian_omega_philox
from .rounding import (round_fp32, round_bf16, split_bf16x2, round_fp8_e4m3, fp8_block_exponent,
                       quantize_block, quantize_omega)
from .jacobi import jacobi_svd
from .metrics import rel_sigma_error, sin_theta_max, column_cosines

__all__ = [
    "sketch_pass", "qb_from_sketch", "svd_from_qb", "single_pass_pca", "basic_randqb_svd",
    "apply_sign_convention", "PCAResult", "philox4x64_10", "philox_words", "gaussian_omega_philox",
    "round_fp32", "round_bf16", "split_bf16x2", "round_fp8_e4m3", "fp8_block_exponent",
    "quantize_block", "quantize_omega", "jacobi_svd", "rel_sigma_error", "sin_theta_max",
    "column_cosines", "power_omega", "single_pass_pca_power", "sketch_pass_centred",
    "centre_sketch", "single_pass_pca_centred", "alg2_single_pass",
]
