"""sketch_pca_static: the whole method in one call with the library's fixed device scratch.

It runs the same kernels as sketch_init + sketch_ingest_block (blocks of max_block_rows rows) +
sketch_finalize on a caller workspace, so its outputs must equal that path's bit for bit.  Two
calls in a row, the second on a smaller input, check that nothing of the first call's scratch
contents leaks into the second.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def _cfg(sk, n, m, block, k, l, b, mode, seed, want_u=1):
    return sk.sketch_config(n=n, m_capacity=m, max_block_rows=block, k=k, l=l, b=b,
                            compute=sk.DTYPES[mode], host_slots=0, host_src=sk.F32,
                            want_u=want_u, omega_from_seed=1, seed=seed)


def _handle_path(sk, A, cfg):
    import torch
    s = sk.Sketch(cfg.n, cfg.m_capacity, cfg.max_block_rows, cfg.k, cfg.l, cfg.b,
                  compute={v: k for k, v in sk.DTYPES.items()}[cfg.compute],
                  want_u=bool(cfg.want_u), seed=cfg.seed)
    for r0 in range(0, A.shape[0], cfg.max_block_rows):
        s.ingest(A[r0:r0 + cfg.max_block_rows])
    S, V, U, rank = s.finalize()
    torch.cuda.synchronize()
    s.close()
    return S.cpu().numpy(), V.cpu().numpy(), None if U is None else U.cpu().numpy(), rank


def _static_path(sk, A, cfg):
    import torch
    S = torch.full((cfg.k,), float("nan"), dtype=torch.float64, device="cuda")
    V = torch.full((cfg.n, cfg.k), float("nan"), dtype=torch.float64, device="cuda")
    U = (torch.full((A.shape[0], cfg.k), float("nan"), dtype=torch.float64, device="cuda")
         if cfg.want_u else None)
    rank = sk.sketch_pca_static(cfg, A, S, U, V)
    torch.cuda.synchronize()
    return S.cpu().numpy(), V.cpu().numpy(), None if U is None else U.cpu().numpy(), rank


@pytest.mark.parametrize("mode,src", [("f64", "f64"), ("f32", "f32"), ("bf16", "f32"),
                                      ("fp8", "f32")])
def test_static_entry_matches_handle_path(gpu_lib, mode, src):
    import torch
    sk = gpu_lib
    dt = {"f64": torch.float64, "f32": torch.float32}[src]
    # call 1: 2000 x 1000, l = 20, 200-row blocks; call 2: a smaller 1111 x 640, l = 30, ragged
    cases = [(2000, 1000, 10, 20, 10, 200, 31), (1111, 640, 12, 30, 10, 256, 32)]
    for (m, n, k, l, b, block, seed) in cases:
        sig = synth.noisy_spectrum(synth.exp_spectrum(n, 10.0), 1e-6, seed)
        A, _, _, _ = synth.small_matrix(m, n, sig, seed)
        At = torch.from_numpy(A).to(dt).cuda()
        cfg = _cfg(sk, n, m, block, k, l, b, mode, seed + 100)
        S0, V0, U0, r0 = _handle_path(sk, At, cfg)
        S1, V1, U1, r1 = _static_path(sk, At, cfg)
        assert r1 == r0 == l
        assert np.array_equal(S0, S1)
        assert np.array_equal(V0, V1)
        assert np.array_equal(U0, U1)
        # and the result is the method's: the oracle on the same (rounded) Omega and rows
        if mode == "f64":
            Om = oracle.gaussian_omega_philox(n, l, seed + 100)
            ref = oracle.single_pass_pca([A], Om, k, b)
            assert np.max(oracle.rel_sigma_error(S1, ref.S)) < 1e-9


def test_static_entry_without_u(gpu_lib):
    import torch
    sk = gpu_lib
    m, n = 700, 300
    A = torch.randn(m, n, dtype=torch.float32, device="cuda")
    cfg = _cfg(sk, n, m, 128, 5, 10, 5, "f32", 9, want_u=0)
    S0, V0, _, r0 = _handle_path(sk, A, cfg)
    S1, V1, U1, r1 = _static_path(sk, A, cfg)
    assert U1 is None and r0 == r1
    assert np.array_equal(S0, S1) and np.array_equal(V0, V1)


def test_static_entry_rejects_oversize_and_bad_arguments(gpu_lib):
    import torch
    sk = gpu_lib
    A = torch.zeros(16, 64, dtype=torch.float32, device="cuda")
    S = torch.empty(4, dtype=torch.float64, device="cuda")
    V = torch.empty(64, 4, dtype=torch.float64, device="cuda")
    big = _cfg(sk, 20000, 100000, 4096, 4, 100, 10, "f32", 1, want_u=0)
    Abig = torch.zeros(16, 20000, dtype=torch.float32, device="cuda")
    Vbig = torch.empty(20000, 4, dtype=torch.float64, device="cuda")
    with pytest.raises(sk.SketchError) as e:
        sk.sketch_pca_static(big, Abig, S, None, Vbig)
    assert e.value.status == 4 and "static scratch" in str(e.value)
    cfg = _cfg(sk, 64, 8, 8, 4, 8, 4, "f32", 1, want_u=0)
    with pytest.raises(sk.SketchError) as e:                 # m > m_capacity
        sk.sketch_pca_static(cfg, A, S, None, V)
    assert e.value.status == 4
    cfg = _cfg(sk, 64, 16, 8, 4, 8, 4, "f32", 1, want_u=0)
    with pytest.raises(sk.SketchError) as e:                 # host rows are refused
        sk.sketch_pca_static(cfg, A.cpu(), S, None, V)
    assert e.value.status == 1
