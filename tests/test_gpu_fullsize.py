"""Parity at the full size of the FP32-resident workload, in the launch configuration the
benchmark times: A is 100000 x 20000 FP32 resident on the GPU (Kronecker SVD, sigma_j = 1/j for
j <= 200 then 1e-4, N(0, 1e-4) noise on sigma), k = 50, l = 100, b = 10, 25 blocks of 4096 rows
(the last 1696).

Every element of G and H is checked against the FP64 reference run on the exact operands the
kernels consume (A' and Omega'), block by block, with the same rigorous bounds as the small-size
tests; S and V are checked end to end against the reference's Algorithm 4 on the same G and H
arithmetic."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import U32

pytestmark = pytest.mark.gpu

M, N, K, L, B, BLK = 100000, 20000, 50, 100, 10, 4096


@pytest.fixture(scope="module")
def workload():
    import torch
    sig = synth.noisy_spectrum(synth.inv_floor_spectrum(N, knee=200, floor=1e-4), 1e-4, 1002)
    Km = synth.KronMatrix(500, 200, 100, 200, sig, 1002)
    A = torch.empty(M, N, dtype=torch.float32, device="cuda")
    for r0 in range(0, M, 2048):
        c = min(2048, M - r0)
        Km.rows_torch(r0, c, "cuda", out=A[r0:r0 + c])
    torch.cuda.synchronize()
    yield A, A.cpu().numpy()
    del A
    torch.cuda.empty_cache()


@pytest.mark.parametrize("mode", ["bf16", "f32"])
def test_full_size_parity(gpu_lib, workload, mode):
    import torch
    A, A_host = workload
    h = gpu_lib.Sketch(N, M, BLK, K, L, B, compute=mode, seed=2002)
    for r0 in range(0, M, BLK):
        h.ingest(A[r0:r0 + BLK])
    G, H = h.state()
    G, H = G.cpu().numpy(), H.cpu().numpy()
    Om = h.omega().cpu().numpy()
    S, V, _, rank = h.finalize()
    S, V = S.cpu().numpy(), V.cpu().numpy()
    h.close()
    torch.cuda.synchronize()
    assert np.array_equal(oracle.quantize_omega(Om, mode), Om)    # Omega' is a fixed point
    absOm = np.abs(Om)
    H_ref = np.zeros((N, L))
    H_bnd = np.zeros((N, L))
    G_ref = np.empty((M, L))
    worst_g = 0.0
    for r0 in range(0, M, BLK):
        a = oracle.quantize_block(A_host[r0:r0 + BLK].astype(np.float64), mode)
        g = a @ Om
        gb = (N + 66) * U32 * (np.abs(a) @ absOm)
        err = np.abs(G[r0:r0 + a.shape[0]] - g)
        assert np.all(err <= gb + 1e-300), f"G rows {r0}.."
        worst_g = max(worst_g, float(np.max(err / (gb + 1e-300))))
        G_ref[r0:r0 + a.shape[0]] = g
        H_ref += a.T @ g
        split = 2.0 ** -17 if mode != "f32" else 0.0
        H_bnd += np.abs(a).T @ (gb + (split + (a.shape[0] + 8) * U32) * np.abs(g))
    assert np.all(np.abs(H - H_ref) <= H_bnd + 1e-300)
    Q, Bm, r, _ = oracle.qb_from_sketch(G_ref, H_ref, Om, B)
    S_ref, _, V_ref = oracle.svd_from_qb(Q, Bm, K, want_u=False)
    assert rank == r == L
    assert np.max(oracle.rel_sigma_error(S, S_ref)) < 2e-4
    assert oracle.sin_theta_max(V_ref, V) < 2e-3
    assert worst_g <= 1.0
