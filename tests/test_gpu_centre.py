"""Implicit column centring on the GPU (PCA of A - 1 mu^T, the method assuming centred data,
Sec. 2.1), still in one pass.

The pass also sums the columns of A (an all-ones operand column of g in a^T g); sketch_finalize
centres G and H before the column-block loop.  Checked against the reference's
single_pass_pca_centred on the same rounded rows A' and Omega' (end-to-end tolerances as for the
uncentred parity), the means against numpy, a checkpoint round trip, the power scheme on centred
data, and the one-call entry point.

Round-off of the reduced modes is relative to the uncentred sketch: a mean m_c times the spread
of the data inflates the error of the centred result by about m_c.  The matrices here have means
of a few times the spread, as image rows do before normalisation (Sec. 4.3).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import quantized_blocks, split_blocks

pytestmark = pytest.mark.gpu

MODES = [("f64", "f64"), ("f32", "f32"), ("bf16", "f32"), ("bf16x2", "f32"), ("fp8", "f32")]


@pytest.fixture(scope="module")
def case():
    m, n, l, k, b = 1531, 777, 40, 20, 10
    sig = synth.noisy_spectrum(synth.exp_spectrum(n, 8.0), 1e-6, 51)
    A0, _, _, _ = synth.small_matrix(m, n, sig, 51)
    rng = np.random.default_rng(52)
    spread = np.std(A0)
    A = A0 + (3.0 * spread) * rng.standard_normal(n)[None, :]
    return dict(A=A, k=k, l=l, b=b, blocks=[1, 17, 300, 513, 700])


def _tensor(A, src):
    import torch
    dt = {"f64": torch.float64, "f32": torch.float32}[src]
    return torch.from_numpy(np.ascontiguousarray(A)).to(dt).cuda()


def _run(sk, At, case, mode, seed=7, power=False):
    import torch
    m, n = At.shape
    s = sk.Sketch(n, m, max(case["blocks"]), case["k"], case["l"], case["b"], compute=mode,
                  want_u=True, seed=seed, centre=True)

    def one_pass():
        r0 = 0
        for cnt in case["blocks"]:
            s.ingest(At[r0:r0 + cnt])
            r0 += cnt

    one_pass()
    if power:
        s.power_restart()
        one_pass()
    mu_before = s.column_mean().cpu().numpy()
    Om = s.omega().cpu().numpy()
    S, V, U, rank = s.finalize()
    mu_after = s.column_mean().cpu().numpy()
    torch.cuda.synchronize()
    s.close()
    return dict(S=S.cpu().numpy(), V=V.cpu().numpy(), U=U.cpu().numpy(), rank=rank, Om=Om,
                mu=mu_before, mu_after=mu_after)


@pytest.mark.parametrize("mode,src", MODES)
def test_centred_parity(gpu_lib, case, mode, src):
    A, k, b, blocks = case["A"], case["k"], case["b"], case["blocks"]
    out = _run(gpu_lib, _tensor(A, src), case, mode)
    Aq = quantized_blocks(A, blocks, mode, src)
    ref = oracle.single_pass_pca_centred(Aq, out["Om"], k, b)
    assert out["rank"] == ref.rank
    tol_s, tol_v = (1e-10, 1e-8) if mode == "f64" else (2e-4, 2e-3)
    assert np.max(oracle.rel_sigma_error(out["S"], ref.S)) < tol_s
    assert oracle.sin_theta_max(ref.V, out["V"]) < tol_v
    assert oracle.sin_theta_max(ref.U, out["U"]) < tol_v
    # the means: column sums accumulated like H (FP32 within a block, FP64 across blocks)
    mu_ref = np.vstack(Aq).mean(axis=0)
    scale = np.abs(np.vstack(Aq)).mean(axis=0)
    mtol = 1e-13 if mode == "f64" else 1e-5
    assert np.all(np.abs(out["mu"] - mu_ref) <= mtol * scale)
    assert np.array_equal(out["mu"], out["mu_after"])
    # U is centred: the reference's columns are orthogonal to the ones vector, and the device's
    # are within the subspace tolerance of them (|1^T u_j| <= tol_v sqrt(m))
    m = A.shape[0]
    assert np.max(np.abs(ref.U.sum(axis=0))) < 1e-10
    assert np.max(np.abs(out["U"].sum(axis=0))) < tol_v * np.sqrt(m)


def test_centred_matches_pca_of_explicitly_centred_matrix(gpu_lib, case):
    """FP64: the same triplets as the uncentred path run on A - mean(A) (Sec. 2.1's assumption
    made explicit), and the means equal numpy's."""
    A, k, b, blocks = case["A"], case["k"], case["b"], case["blocks"]
    out = _run(gpu_lib, _tensor(A, "f64"), case, "f64")
    Ac = A - A.mean(axis=0)
    ref = oracle.single_pass_pca(split_blocks(Ac, blocks), out["Om"], k, b)
    assert np.max(oracle.rel_sigma_error(out["S"], ref.S)) < 1e-9
    assert oracle.sin_theta_max(ref.V, out["V"]) < 1e-8
    assert np.max(np.abs(out["mu"] - A.mean(axis=0))) < 1e-13 * np.max(np.abs(A))


@pytest.mark.parametrize("mode,src", [("f64", "f64"), ("bf16", "f32")])
def test_centred_power_scheme(gpu_lib, case, mode, src):
    """P = 1 on centred data: Omega_2 from the centred first-pass H; the second pass against the
    reference's centred Algorithm 4 on the device's Omega_2'."""
    A, k, b, blocks = case["A"], case["k"], case["b"], case["blocks"]
    out = _run(gpu_lib, _tensor(A, src), case, mode, power=True)
    ref = oracle.single_pass_pca_centred(quantized_blocks(A, blocks, mode, src), out["Om"], k, b)
    tol_s, tol_v = (1e-10, 1e-8) if mode == "f64" else (2e-4, 2e-3)
    assert np.max(oracle.rel_sigma_error(out["S"], ref.S)) < tol_s
    assert oracle.sin_theta_max(ref.V, out["V"]) < tol_v
    # and Omega_2 spans the centred power direction of the reference's first pass (FP64 only)
    if mode == "f64":
        G1, H1, sA, sG, m = oracle.sketch_pass_centred(split_blocks(A, blocks),
                                                       oracle.gaussian_omega_philox(A.shape[1],
                                                                                    case["l"], 7))
        _, Hc, _ = oracle.centre_sketch(G1, H1, oracle.gaussian_omega_philox(A.shape[1],
                                                                             case["l"], 7),
                                        sA, sG, m)
        W = oracle.power_omega(Hc) / np.sqrt(A.shape[1])
        assert oracle.sin_theta_max(W, np.linalg.qr(out["Om"])[0]) < 1e-6


def test_centred_checkpoint_round_trip(gpu_lib, case):
    import torch
    sk = gpu_lib
    A, blocks = case["A"], case["blocks"]
    At = _tensor(A, "f32")
    m, n = A.shape
    ref = _run(sk, At, case, "f32", seed=9)
    s = sk.Sketch(n, m, max(blocks), case["k"], case["l"], case["b"], compute="f32", want_u=True,
                  seed=9, centre=True)
    r0 = 0
    for cnt in blocks[:3]:
        s.ingest(At[r0:r0 + cnt])
        r0 += cnt
    buf = s.checkpoint()
    s.close()
    t = sk.Sketch(n, m, max(blocks), case["k"], case["l"], case["b"], compute="f32", want_u=True,
                  seed=1, centre=True)
    t.restore(buf)
    for cnt in blocks[3:]:
        t.ingest(At[r0:r0 + cnt])
        r0 += cnt
    S, V, U, rank = t.finalize()
    torch.cuda.synchronize()
    t.close()
    assert np.array_equal(S.cpu().numpy(), ref["S"]) and np.array_equal(V.cpu().numpy(), ref["V"])
    # an uncentred handle does not take a centred checkpoint
    u = sk.Sketch(n, m, max(blocks), case["k"], case["l"], case["b"], compute="f32", seed=9)
    with pytest.raises(sk.SketchError) as e:
        u.restore(buf)
    assert e.value.status == 1
    with pytest.raises(sk.SketchError) as e:
        u.column_mean()
    assert e.value.status == 2
    u.close()


def test_centred_static_entry(gpu_lib, case):
    """The one-call entry point centres the same way, with the same bits as a handle."""
    import torch
    sk = gpu_lib
    A = case["A"][:1200]
    At = _tensor(A, "f32")
    m, n = A.shape
    cfg = sk.sketch_config(n=n, m_capacity=m, max_block_rows=256, k=10, l=30, b=10,
                           compute=sk.F32, host_slots=0, host_src=sk.F32, want_u=0,
                           omega_from_seed=1, centre=1, seed=11)
    h = sk.Sketch(n, m, 256, 10, 30, 10, compute="f32", seed=11, centre=True)
    for r0 in range(0, m, 256):
        h.ingest(At[r0:r0 + 256])
    S0, V0, _, _ = h.finalize()
    h.close()
    S1 = torch.empty(10, dtype=torch.float64, device="cuda")
    V1 = torch.empty(n, 10, dtype=torch.float64, device="cuda")
    sk.sketch_pca_static(cfg, At, S1, None, V1)
    torch.cuda.synchronize()
    assert torch.equal(S0, S1) and torch.equal(V0, V1)
