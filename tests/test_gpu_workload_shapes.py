"""Parity at the block shapes of the host-streamed workloads, through the pinned-host staging ring.

The 40 GB precision workload streams 8192-row blocks of 10000 FP32 columns and the 150 GB one
16384-row blocks of 25000 columns (FP32 or BF16 rows); there the planner picks other split and
row-split counts than at the resident workload's shapes, and the staging slots hold 0.3-1.6 GB.
Three (two) such blocks are ingested from pinned host memory and G and H are compared element by
element with the reference on the same rounded rows A' and Omega', within the rigorous bounds of
the FP32-accumulating products (Eq. 10).  Also: FP8 end to end on the slowly decaying 1/j
spectrum of the resident workload (not only on a fast-decaying one).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import g_bound, h_bound, quantized_blocks, run_gpu

pytestmark = pytest.mark.gpu


def _kron_rows(K, count):
    import torch
    return K.rows_torch(0, count, "cuda").to(torch.float32).cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def c3_rows():
    n = 10000
    sig = synth.noisy_spectrum(synth.inv_square_spectrum(n), 1e-5, 1003)
    K = synth.KronMatrix(100, 250, 100, 100, sig, 1003)      # 25000 rows >= the 24576 used
    return _kron_rows(K, 3 * 8192)


@pytest.mark.parametrize("mode", ["f32", "bf16", "bf16x2", "fp8"])
def test_precision_workload_blocks(gpu_lib, c3_rows, mode):
    A = c3_rows
    n, l, k = A.shape[1], 100, 50
    blocks = [8192, 8192, 8192]
    Om = synth.gaussian_omega(n, l, 2003)
    out = run_gpu(A, Om, k, 10, mode, blocks, src="f32", want_u=False, host=True, host_slots=3)
    Omq = oracle.quantize_omega(Om, mode)
    assert np.array_equal(out["Om"], Omq)
    Aq = quantized_blocks(A, blocks, mode, "f32")
    G_ref, H_ref = oracle.sketch_pass(Aq, Omq)
    gb = g_bound(Aq, Omq)
    hb = h_bound(Aq, Omq, G_ref, gb, 8192, split_g=(mode != "f32"))
    assert np.all(np.abs(out["G"] - G_ref) <= gb + 1e-300)
    assert np.all(np.abs(out["H"] - H_ref) <= hb + 1e-300)


@pytest.mark.parametrize("mode,src", [("bf16", "bf16"), ("f32", "f32")])
def test_paper_scale_workload_blocks(gpu_lib, mode, src):
    n, l, k = 25000, 100, 50
    sig = synth.noisy_spectrum(synth.inv_spectrum(n), 1e-4, 1005) / np.sqrt(48)
    K = synth.KronMatrix(125, 300, 125, 200, sig, 1005)      # 37500 rows >= the 32768 used
    A = _kron_rows(K, 2 * 16384)
    blocks = [16384, 16384]
    Om = synth.gaussian_omega(n, l, 2005)
    out = run_gpu(A, Om, k, 10, mode, blocks, src=src, want_u=False, host=True, host_slots=2)
    Omq = oracle.quantize_omega(Om, mode)
    Aq = quantized_blocks(A, blocks, mode, src)
    G_ref, H_ref = oracle.sketch_pass(Aq, Omq)
    gb = g_bound(Aq, Omq)
    hb = h_bound(Aq, Omq, G_ref, gb, 16384, split_g=(mode != "f32"))
    assert np.all(np.abs(out["G"] - G_ref) <= gb + 1e-300)
    assert np.all(np.abs(out["H"] - H_ref) <= hb + 1e-300)


def test_fp8_end_to_end_slow_decay(gpu_lib):
    """FP8 on sigma_j = 1/j (the resident workload's spectrum, at 4000 x 1500, l = 40): the
    finalize on the device's sketch equals the reference's, and the result against the reference
    on A' (the same FP8 rows) stays within the reduced-mode tolerance."""
    m, n, k, l = 4000, 1500, 20, 40
    sig = synth.noisy_spectrum(synth.inv_spectrum(n), 1e-4, 77)
    A, _, s, _ = synth.small_matrix(m, n, sig, 77)
    Om = synth.gaussian_omega(n, l, 78)
    blocks = [1500, 1500, 1000]
    out = run_gpu(A, Om, k, 10, "fp8", blocks, src="f32")
    Q, B, rank, _ = oracle.qb_from_sketch(out["G"], out["H"], out["Om"], 10)
    S, U, V = oracle.svd_from_qb(Q, B, k)
    assert np.max(oracle.rel_sigma_error(out["S"], S)) < 1e-10
    ref = oracle.single_pass_pca(quantized_blocks(A, blocks, "fp8", "f32"), out["Om"], k, 10)
    assert out["rank"] == ref.rank
    assert np.max(oracle.rel_sigma_error(out["S"], ref.S)) < 2e-4
    assert oracle.sin_theta_max(ref.V, out["V"]) < 2e-3
