"""Parity of the HIP path (through the C ABI) with the FP64 reference on the same inputs.

Reference operands: every reduced-precision mode is compared with the oracle run on A' and Omega',
the exact operands the kernels consume, rebuilt by the oracle's own rounding (RNE to FP32/BF16,
BF16 hi+lo, OCP E4M3 with the per-block power-of-two scale).  Omega is supplied by the caller (a
seeded Gaussian) so both sides see identical bits; the device generator is pinned separately.

Tolerances:
  G (m x l): |G - G_ref| <= (n + 66) u32 (|A'| |Omega'|) elementwise in the FP32-accumulating
             modes (a rigorous FP32 summation bound over n terms plus the split partials);
             FP64 mode: the same with u64.
  H (n x l): |A'|^T (G error bound + (2^-17 [BF16 hi/lo of G] + (rows+8) u32) |G_ref|).
  S, V, U:   FP64 mode 1e-10 relative on sigma and 1e-8 on subspace sines; reduced modes against
             oracle(A', Omega') at 2e-4 relative on sigma_1..k (the finalize is FP64; the residual
             is the FP32-level error of G and H amplified by the (sigma_1/sigma_k)^2 cancellation in
             Eq. 9, which is below 10 on these spectra).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import (U32, U64, g_bound, h_bound, quantized_blocks, run_gpu, split_blocks)

pytestmark = pytest.mark.gpu

MODES = [("f64", "f64"), ("f32", "f32"), ("bf16", "f32"), ("bf16", "bf16"), ("bf16x2", "f32"),
         ("fp8", "f32")]


@pytest.fixture(scope="module")
def ragged():
    """777 columns (not a multiple of 16 or of the 512-column k-chunks), 1531 rows in ragged
    blocks, l = 40 (48 padded), b = 10, spectrum exp(-j/8)."""
    m, n, l, k, b = 1531, 777, 40, 20, 10
    sig = synth.noisy_spectrum(synth.exp_spectrum(n, 8.0), 1e-6, 11)
    A, _, s, _ = synth.small_matrix(m, n, sig, 11)
    Om = synth.gaussian_omega(n, l, 12)
    blocks = [1, 17, 300, 513, 700]
    return dict(A=A, Om=Om, k=k, b=b, blocks=blocks, s=s)


@pytest.mark.parametrize("mode,src", MODES)
def test_sketch_state_parity(gpu_lib, ragged, mode, src):
    """G and H after the pass, elementwise against the reference on A', Omega' (Eq. 10)."""
    A, Om, blocks = ragged["A"], ragged["Om"], ragged["blocks"]
    out = run_gpu(A, Om, ragged["k"], ragged["b"], mode, blocks, src=src)
    Omq = oracle.quantize_omega(Om, mode)
    assert np.array_equal(out["Om"], Omq)          # Omega' identical bits
    Aq = quantized_blocks(A, blocks, mode, src)
    G_ref, H_ref = oracle.sketch_pass(Aq, Omq)
    if mode == "f64":
        gb = (A.shape[1] + 4) * U64 * (np.abs(np.vstack(Aq)) @ np.abs(Omq))
        hb = np.abs(np.vstack(Aq)).T @ (gb + (max(blocks) + 8) * U64 * np.abs(G_ref))
    else:
        gb = g_bound(Aq, Omq)
        hb = h_bound(Aq, Omq, G_ref, gb, max(blocks), split_g=(mode != "f32"))
    assert np.all(np.abs(out["G"] - G_ref) <= gb + 1e-300)
    assert np.all(np.abs(out["H"] - H_ref) <= hb + 1e-300)


@pytest.mark.parametrize("mode,src", MODES)
def test_end_to_end_parity(gpu_lib, ragged, mode, src):
    """S, V, U against Algorithm 4 run by the reference on A', Omega'."""
    A, Om, blocks, k, b = ragged["A"], ragged["Om"], ragged["blocks"], ragged["k"], ragged["b"]
    out = run_gpu(A, Om, k, b, mode, blocks, src=src, keep_state=False)
    Omq = oracle.quantize_omega(Om, mode)
    ref = oracle.single_pass_pca(quantized_blocks(A, blocks, mode, src), Omq, k, b)
    assert out["rank"] == ref.rank
    tol_s, tol_v = (1e-10, 1e-8) if mode == "f64" else (2e-4, 2e-3)
    assert np.max(oracle.rel_sigma_error(out["S"], ref.S)) < tol_s
    assert oracle.sin_theta_max(ref.V, out["V"]) < tol_v
    assert oracle.sin_theta_max(ref.U, out["U"]) < tol_v
    # orthonormal outputs
    assert np.linalg.norm(out["V"].T @ out["V"] - np.eye(k)) < 1e-10
    assert np.linalg.norm(out["U"].T @ out["U"] - np.eye(k)) < 1e-8
    # sign convention: the largest-magnitude entry of each v_j is positive
    idx = np.argmax(np.abs(out["V"]), axis=0)
    assert np.all(out["V"][idx, np.arange(k)] > 0)


def test_plain_fp64_workload(gpu_lib):
    """2000 x 1000, sigma_j = exp(-j/10) + N(0,1e-6), k = 10, l = 20, ten 200-row blocks, FP64:
    identical to the reference up to FP64 round-off, and to Algorithm 1 with the same Omega."""
    m, n, k, l, b = 2000, 1000, 10, 20, 10
    sig = synth.noisy_spectrum(synth.exp_spectrum(n, 10.0), 1e-6, 1001)
    A, _, s, V = synth.small_matrix(m, n, sig, 1001)
    Om = synth.gaussian_omega(n, l, 2001)
    out = run_gpu(A, Om, k, b, "f64", [200] * 10, src="f64")
    ref = oracle.single_pass_pca(split_blocks(A, [200] * 10), Om, k, b)
    alg1 = oracle.basic_randqb_svd(A, Om, k)
    assert out["rank"] == l
    assert np.max(oracle.rel_sigma_error(out["S"], ref.S)) < 1e-12
    assert np.max(oracle.rel_sigma_error(out["S"], alg1.S)) < 1e-11
    assert np.max(np.abs(out["V"] - ref.V)) < 1e-10          # same signs by the convention
    assert np.max(np.abs(out["U"] - ref.U)) < 1e-10


@pytest.mark.parametrize("l,b,k", [(100, 10, 50), (100, 20, 50), (32, 32, 32), (30, 5, 30),
                                   (16, 1, 8), (16, 2, 8), (32, 8, 16), (30, 15, 30), (60, 5, 30),
                                   (24, 6, 24), (128, 16, 64)])
def test_widths_and_block_sizes(gpu_lib, l, b, k):
    """Sketch widths across 1..8 padded column tiles, b from 1 to 32, k = l.  The b values make
    the earlier-basis width p = i*b hit 16 exactly (a single 16-row tile of the FP64 row
    reductions, whose accumulator read-back needs the explicit drain)."""
    m, n = 2100, 1500
    sig = synth.noisy_spectrum(synth.inv_floor_spectrum(n, knee=200, floor=1e-4), 1e-4, l)
    A, _, s, _ = synth.small_matrix(m, n, sig, l + b)
    Om = synth.gaussian_omega(n, l, 7 + b)
    blocks = [1024, 1024, 52]
    out = run_gpu(A, Om, k, b, "f64", blocks, src="f64", keep_state=False)
    ref = oracle.single_pass_pca(split_blocks(A, blocks), Om, k, b)
    assert out["rank"] == ref.rank == l
    assert np.max(oracle.rel_sigma_error(out["S"], ref.S)) < 1e-9
    assert oracle.sin_theta_max(ref.V, out["V"]) < 1e-7


@pytest.mark.parametrize("rank", [7, 25, 30])
def test_rank_guard(gpu_lib, rank):
    """rank(A) < l: the guard stops the loop at the rank (also when not a multiple of b) and the
    rank's singular values are exact; trailing outputs are zero."""
    m, n, l, b, k = 800, 500, 40, 10, 20
    sig = np.linspace(2.0, 0.05, rank)
    A, _, s, V = synth.low_rank_matrix(m, n, sig, 30 + rank)
    Om = synth.gaussian_omega(n, l, 40 + rank)
    out = run_gpu(A, Om, k, b, "f64", [300, 300, 200], src="f64", keep_state=False)
    kk = min(k, rank)
    assert out["rank"] == rank
    assert np.max(oracle.rel_sigma_error(out["S"][:kk], s[:kk])) < 1e-10
    assert np.all(out["S"][kk:] == 0) and np.all(out["V"][:, kk:] == 0)
    assert np.all(out["U"][:, kk:] == 0)
    assert oracle.sin_theta_max(V[:, :kk], out["V"][:, :kk]) < 1e-8


@pytest.mark.parametrize("force", [(0, 0), (1, 0), (0, 1), (0, 2), (1, 1), (0, 3)])
def test_finalize_paths_agree(gpu_lib, ragged, force):
    """Cholesky QR, shifted Cholesky QR3 for R_B and the Householder fallbacks (forced through the
    test hook) all match the reference on the same sketch; without forcing, a well-conditioned
    sketch takes Cholesky QR (QR2 for R_B).  Mode 3 treats QR2 as not accepted after the SVD and
    the outputs were formed from it: they are formed again from shifted QR3 (reported as 2)."""
    A, Om, blocks, k, b = ragged["A"], ragged["Om"], ragged["blocks"], ragged["k"], ragged["b"]
    out = run_gpu(A, Om, k, b, "f64", blocks, src="f64", keep_state=False, force=force)
    ref = oracle.single_pass_pca(split_blocks(A, blocks), Om, k, b)
    assert out["paths"] == ((force[0], 2) if force[1] == 3 else force)
    assert out["rank"] == ref.rank
    assert np.max(oracle.rel_sigma_error(out["S"], ref.S)) < 1e-10
    assert oracle.sin_theta_max(ref.V, out["V"]) < 1e-8
    assert oracle.sin_theta_max(ref.U, out["U"]) < 1e-8


def test_cholqr_flags_ill_conditioned_block(gpu_lib):
    """Two sketch columns nearly parallel (Omega columns equal up to 1e-6): the first block's Gram
    matrix has a pivot far below 1e-10 of its diagonal, so the loop falls back to Householder
    TSQR; the rank guard keeps every column (the pair still differs by far more than 1e-10 of
    R's first diagonal) and the result matches the reference.  The near-dependence amplifies
    rounding by about 1e6, hence the looser bounds."""
    m, n, l, k, b = 1200, 600, 20, 8, 10
    sig = synth.noisy_spectrum(synth.exp_spectrum(n, 8.0), 1e-6, 5)
    A, _, _, _ = synth.small_matrix(m, n, sig, 5)
    Om = synth.gaussian_omega(n, l, 6)
    Om[:, 1] = Om[:, 0] + 1e-6 * Om[:, 1]
    blocks = [500, 500, 200]
    out = run_gpu(A, Om, k, b, "f64", blocks, src="f64", keep_state=False)
    ref = oracle.single_pass_pca(split_blocks(A, blocks), Om, k, b)
    assert out["paths"][0] == 1
    assert out["rank"] == ref.rank == l
    assert np.max(oracle.rel_sigma_error(out["S"], ref.S)) < 1e-8
    assert oracle.sin_theta_max(ref.V, out["V"]) < 1e-6


def test_zero_matrix(gpu_lib):
    A = np.zeros((300, 200))
    out = run_gpu(A, synth.gaussian_omega(200, 20, 1), 10, 10, "f32", [300], keep_state=False)
    assert out["rank"] == 0 and np.all(out["S"] == 0) and np.all(out["V"] == 0)


@pytest.mark.parametrize("mode,src", [("f32", "f32"), ("bf16", "bf16"), ("f64", "f64")])
def test_host_staged_ingest(gpu_lib, ragged, mode, src):
    """Pinned-host blocks through the staging ring give the same G and H as device blocks."""
    A, Om, blocks = ragged["A"], ragged["Om"], ragged["blocks"]
    d = run_gpu(A, Om, ragged["k"], ragged["b"], mode, blocks, src=src)
    h = run_gpu(A, Om, ragged["k"], ragged["b"], mode, blocks, src=src, host=True, host_slots=2)
    assert np.array_equal(d["G"], h["G"]) and np.array_equal(d["H"], h["H"])
    assert np.array_equal(d["S"], h["S"])
    for t in h["tickets"]:
        assert h["sketch"].poll(t)


@pytest.mark.parametrize("mode,src", [("f32", "f32"), ("bf16", "bf16"), ("fp8", "f32")])
def test_host_staged_linear_copy(gpu_lib, mode, src):
    """Host rows whose length keeps 16-byte alignment (n = 1024) are copied linearly into the
    staging ring; the result equals device ingest bit for bit."""
    m, n, l, k, b = 1000, 1024, 32, 16, 8
    sig = synth.noisy_spectrum(synth.exp_spectrum(min(m, n), 8.0), 1e-6, 31)
    A, _, _, _ = synth.small_matrix(m, n, sig, 31)
    Om = synth.gaussian_omega(n, l, 32)
    blocks = [300, 300, 255, 145]
    d = run_gpu(A, Om, k, b, mode, blocks, src=src)
    h = run_gpu(A, Om, k, b, mode, blocks, src=src, host=True, host_slots=3)
    assert np.array_equal(d["G"], h["G"]) and np.array_equal(d["H"], h["H"])
    assert np.array_equal(d["S"], h["S"]) and np.array_equal(d["V"], h["V"])


def test_deterministic(gpu_lib, ragged):
    """No atomics on the result path: repeated runs are bitwise identical."""
    A, Om, blocks = ragged["A"], ragged["Om"], ragged["blocks"]
    r1 = run_gpu(A, Om, ragged["k"], ragged["b"], "bf16", blocks)
    r2 = run_gpu(A, Om, ragged["k"], ragged["b"], "bf16", blocks)
    for key in ("G", "H", "S", "V", "U"):
        assert np.array_equal(r1[key], r2[key]), key


def test_device_omega_generator(gpu_lib):
    """Omega from a seed (Philox-4x64-10 + Box-Muller) against the reference generator."""
    import torch
    import paper_1704_07669_amd as sk
    words = torch.empty(4096, dtype=torch.int64, device="cuda")
    sk.sketch_philox_words(777, 12, 4096, words)
    ref = oracle.philox_words(777, 12, 4096)
    assert np.array_equal(words.cpu().numpy().view(np.uint64), ref)
    n, l = 3001, 37
    s = sk.Sketch(n, 64, 64, 5, l, 1, compute="f64", seed=4242)
    Om = s.omega().cpu().numpy()
    Z = oracle.gaussian_omega_philox(n, l, 4242)
    assert np.max(np.abs(Om - Z)) < 1e-13
    s.close()


def test_error_paths(gpu_lib):
    import torch
    import paper_1704_07669_amd as sk
    n = 256
    s = sk.Sketch(n, 100, 50, 4, 8, 4, compute="f32", seed=1)
    A = torch.randn(60, n, device="cuda")
    with pytest.raises(sk.SketchError) as e:
        s.ingest(A)                                   # 60 > max_block_rows
    assert e.value.status == 4
    with pytest.raises(sk.SketchError) as e:
        s.ingest(A[:10].cpu())                        # host memory without staging slots
    assert e.value.status == 1
    s.ingest(A[:50])
    s.ingest(A[:50])
    with pytest.raises(sk.SketchError) as e:
        s.ingest(A[:1])                               # m_capacity 100 exceeded
    assert e.value.status == 4
    S, V, U, rank = s.finalize()
    assert rank == 8
    with pytest.raises(sk.SketchError) as e:
        s.ingest(A[:10])                              # ingest after finalize
    assert e.value.status == 2
    s.reset(5)                                        # a new pass on the same workspace
    s.ingest(A[:50])
    S2, _, _, _ = s.finalize()
    assert np.all(np.isfinite(S2.cpu().numpy()))
    s.close()


def test_pageable_host_rows_rejected(gpu_lib):
    import torch
    import paper_1704_07669_amd as sk
    s = sk.Sketch(128, 64, 64, 4, 8, 4, compute="f32", seed=1, host_slots=2)
    with pytest.raises(sk.SketchError) as e:
        s.ingest(torch.randn(16, 128))                # pageable: must be pinned
    assert e.value.status == 1 and "pinned" in str(e.value)
    s.ingest(torch.randn(16, 128).pin_memory())
    s.close()


def test_nonfinite_block_is_sticky(gpu_lib):
    import torch
    import paper_1704_07669_amd as sk
    s = sk.Sketch(128, 64, 64, 4, 8, 4, compute="bf16", seed=1)
    A = torch.randn(32, 128, device="cuda")
    A[3, 7] = float("nan")
    s.ingest(A)
    with pytest.raises(sk.SketchError) as e:
        s.finalize()
    assert e.value.status == 5
    with pytest.raises(sk.SketchError) as e:
        s.ingest(A)
    assert e.value.status == 5
    s.close()


@pytest.mark.parametrize("mode", ["f32", "bf16"])
def test_accuracy_gate_vs_fp64(gpu_lib, mode):
    """Against the FP64 reference on the stored A with the same Omega': relative sigma_k error <= 1e-3
    on a 1/j spectrum with a 1e-4 floor (the FP32-resident workload's spectrum, smaller)."""
    m, n, l, k, b = 6000, 3000, 100, 50, 10
    sig = synth.noisy_spectrum(synth.inv_floor_spectrum(n, knee=200, floor=1e-4), 1e-4, 5)
    A, _, s, _ = synth.small_matrix(m, n, sig, 5)
    A = oracle.round_fp32(A)                      # the matrix as stored (FP32)
    Om = synth.gaussian_omega(n, l, 6)
    blocks = [4096, 1904]
    out = run_gpu(A, Om, k, b, mode, blocks, keep_state=False)
    ref = oracle.single_pass_pca(split_blocks(A, blocks), oracle.quantize_omega(Om, mode), k, b)
    err = oracle.rel_sigma_error(out["S"], ref.S)
    assert err[k - 1] <= 1e-3 and np.max(err) <= 1e-3
