"""The finalize with one column block (b = l): Alg. 4 steps 9-15 with t = 1.

Y_1 = G, [Q, R] = qr(G) by Cholesky QR applied twice, B = R^{-T} H^T (Eq. 9 with Q and B still
empty), the rank guard on R's diagonal.  Theorem 1 holds for every b and the result does not
depend on b in exact arithmetic (pin P9), so the device's b = l result is checked against the
reference run with b = l and with the paper's b = 10.  When Cholesky QR2 rejects G (ill
conditioned or rank deficient), the blocked loop takes over with the widest block width up to 32
that divides l; those cases are checked too.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import quantized_blocks, run_gpu, split_blocks

pytestmark = pytest.mark.gpu

MODES = [("f64", "f64"), ("f32", "f32"), ("bf16", "f32"), ("bf16x2", "f32"), ("fp8", "f32")]


@pytest.fixture(scope="module")
def ragged():
    m, n, l, k = 1531, 777, 40, 20
    sig = synth.noisy_spectrum(synth.exp_spectrum(n, 8.0), 1e-6, 11)
    A, _, s, _ = synth.small_matrix(m, n, sig, 11)
    Om = synth.gaussian_omega(n, l, 12)
    return dict(A=A, Om=Om, k=k, l=l, blocks=[1, 17, 300, 513, 700])


def test_plain_fp64_workload_one_block(gpu_lib):
    """2000 x 1000, exp(-j/10) spectrum, k = 10, l = b = 20: the reference with b = 20 and with
    b = 10, and Algorithm 1."""
    m, n, k, l = 2000, 1000, 10, 20
    sig = synth.noisy_spectrum(synth.exp_spectrum(n, 10.0), 1e-6, 1001)
    A, _, s, V = synth.small_matrix(m, n, sig, 1001)
    Om = synth.gaussian_omega(n, l, 2001)
    out = run_gpu(A, Om, k, l, "f64", [200] * 10, src="f64")
    assert out["paths"][0] == 2
    assert out["rank"] == l
    for b in (l, 10):
        ref = oracle.single_pass_pca(split_blocks(A, [200] * 10), Om, k, b)
        assert np.max(oracle.rel_sigma_error(out["S"], ref.S)) < 1e-12
        assert np.max(np.abs(out["V"] - ref.V)) < 1e-10
        assert np.max(np.abs(out["U"] - ref.U)) < 1e-10
    alg1 = oracle.basic_randqb_svd(A, Om, k)
    assert np.max(oracle.rel_sigma_error(out["S"], alg1.S)) < 1e-11


@pytest.mark.parametrize("mode,src", MODES)
def test_one_block_parity(gpu_lib, ragged, mode, src):
    A, Om, k, l, blocks = ragged["A"], ragged["Om"], ragged["k"], ragged["l"], ragged["blocks"]
    out = run_gpu(A, Om, k, l, mode, blocks, src=src)
    assert out["paths"][0] == 2
    # finalize-only: the reference's loop (b = l) on the device's own sketch
    Q, B, rank, _ = oracle.qb_from_sketch(out["G"], out["H"], out["Om"], l)
    S, U, V = oracle.svd_from_qb(Q, B, k)
    assert out["rank"] == rank
    assert np.max(oracle.rel_sigma_error(out["S"], S)) < 1e-10
    assert oracle.sin_theta_max(V, out["V"]) < 1e-8
    assert oracle.sin_theta_max(U, out["U"]) < 1e-8
    assert np.max(np.abs(out["V"] - V)) < 1e-7
    # end to end against the reference on A', Omega' with the paper's b = 10
    ref = oracle.single_pass_pca(quantized_blocks(A, blocks, mode, src), out["Om"], k, 10)
    tol_s, tol_v = (1e-10, 1e-8) if mode == "f64" else (2e-4, 2e-3)
    assert np.max(oracle.rel_sigma_error(out["S"], ref.S)) < tol_s
    assert oracle.sin_theta_max(ref.V, out["V"]) < tol_v
    assert np.linalg.norm(out["U"].T @ out["U"] - np.eye(k)) < 1e-8


@pytest.mark.parametrize("l,k", [(100, 50), (128, 64), (48, 48)])
def test_one_block_widths(gpu_lib, l, k):
    m, n = 2500, 1300
    sig = synth.noisy_spectrum(synth.inv_spectrum(n), 1e-7, l)
    A, _, s, _ = synth.small_matrix(m, n, sig, l)
    Om = synth.gaussian_omega(n, l, l + 1)
    out = run_gpu(A, Om, k, l, "f64", [1000, 1000, 500], src="f64", keep_state=False)
    ref = oracle.single_pass_pca(split_blocks(A, [1000, 1000, 500]), Om, k, l)
    assert out["paths"][0] == 2 and out["rank"] == ref.rank == l
    amp = (ref.S[0] / ref.S) ** 2
    assert np.all(oracle.rel_sigma_error(out["S"], ref.S) <= 1e-12 * amp + 1e-12)
    assert oracle.sin_theta_max(ref.V[:, :10], out["V"][:, :10]) < 1e-9


@pytest.mark.parametrize("rank", [7, 25, 30])
def test_one_block_rank_guard(gpu_lib, rank):
    """Exact rank r < l: Cholesky QR2 rejects the singular Gram matrix of G and the blocked loop
    (b = 20 here) recovers exactly r triplets."""
    m, n, l, k = 900, 400, 40, 35
    s = np.linspace(2.0, 0.5, rank)
    A, _, _, V = synth.low_rank_matrix(m, n, s, 100 + rank)
    Om = synth.gaussian_omega(n, l, 200 + rank)
    out = run_gpu(A, Om, k, l, "f64", [450, 450], src="f64", keep_state=False)
    assert out["rank"] == rank
    assert np.allclose(out["S"][:rank], s, rtol=1e-11)
    assert np.all(out["S"][rank:] == 0)
    assert oracle.sin_theta_max(V, out["V"][:, :rank]) < 1e-9


def test_one_block_rank_guard_cuts_an_accepted_basis(gpu_lib):
    """The last column of Omega scaled by 1e-11: G's last column is tiny but independent of the
    others, so Cholesky QR2 accepts G (Cholesky QR is unaffected by column scaling), while the
    rank guard (R_jj > 1e-10 R_00) drops that column.  The finalize, which went ahead with all l
    columns before reading R's diagonal, forms the SVD again from the leading l - 1, and must
    match the reference run with the same Omega (b = l)."""
    m, n, k, l = 900, 400, 10, 24
    sig = synth.noisy_spectrum(synth.exp_spectrum(n, 10.0), 1e-6, 31)
    A, _, s, _ = synth.small_matrix(m, n, sig, 31)
    Om = synth.gaussian_omega(n, l, 32)
    Om[:, -1] *= 1e-11
    out = run_gpu(A, Om, k, l, "f64", [450, 450], src="f64")
    assert out["paths"][0] == 2                  # the one-block path kept G
    ref = oracle.single_pass_pca(split_blocks(A, [450, 450]), Om, k, l)
    assert ref.rank == l - 1
    assert out["rank"] == ref.rank
    assert np.max(oracle.rel_sigma_error(out["S"], ref.S)) < 1e-10
    assert oracle.sin_theta_max(ref.V, out["V"]) < 1e-8
    assert oracle.sin_theta_max(ref.U, out["U"]) < 1e-8


def test_one_block_ill_conditioned_falls_back(gpu_lib):
    """Type 5 spectrum, l = 60: G's Gram matrix is too ill conditioned for unshifted Cholesky QR
    (cond(G) ~ 1e6), so the blocked loop runs, and matches the reference."""
    m, n, k, l = 1500, 700, 10, 60
    sig = synth.paper_type_spectrum(5, n)
    A, _, s, _ = synth.small_matrix(m, n, sig, 110)
    Om = synth.gaussian_omega(n, l, 120)
    out = run_gpu(A, Om, k, l, "f64", [700, 700, 100], src="f64", keep_state=False)
    assert out["paths"][0] in (0, 1)
    ref = oracle.single_pass_pca(split_blocks(A, [700, 700, 100]), Om, k, l)
    tol = 1e4 * 2.0 ** -53 * s[0] ** 2 / (s[l - 1] * s[:k])
    assert np.all(oracle.rel_sigma_error(out["S"], ref.S) <= tol)
    assert np.max(oracle.rel_sigma_error(out["S"][:5], s[:5])) < 1e-6


def test_one_block_forced_householder_loop(gpu_lib, ragged):
    """The test hook sends b = l through the blocked Householder loop (blocks of 20 for l = 40):
    the same triplets as the one-block path."""
    A, Om, k, l, blocks = ragged["A"], ragged["Om"], ragged["k"], ragged["l"], ragged["blocks"]
    a = run_gpu(A, Om, k, l, "f64", blocks, src="f64", keep_state=False)
    b = run_gpu(A, Om, k, l, "f64", blocks, src="f64", keep_state=False, force=(1, 0))
    assert a["paths"][0] == 2 and b["paths"][0] == 1
    assert np.max(oracle.rel_sigma_error(a["S"], b["S"])) < 1e-11
    assert oracle.sin_theta_max(a["V"], b["V"]) < 1e-9
