"""The accuracy study of Sec. 4.1 on the GPU: spectra Type 1-5, 3000 x 3000, k = 50, l = 60, b = 10,
every compute mode.

Per (type, mode): kernel parity (the pass against the reference on the same rounded rows A' and
Omega', the finalize against the reference on the device's own sketch), and against the known
spectrum:
  * FP64: the paper's observations, to order of magnitude (parity unpinned: its draws are
    unknown): on Type 1 the largest singular-value error is of order 1e-4 (printed 1.3e-4), the
    first principal component differs by about 1e-5 in the infinity norm (printed 2.8e-5), the
    first ten principal components correlate at >= 0.999 (printed 0.9993 at worst), and Types
    2-5 decay faster and come out more accurate than Type 1;
  * Algorithm 2 (reference only) is much less accurate than Algorithm 4 on Type 1 (Fig. 4).
The reduced modes' errors against the known spectrum are recorded, not gated: rounding A to BF16
or FP8 adds noise of about 2^-9 or 2^-4 of A's norm, above the whole tail of Types 1 and 2.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import U64, g_bound, h_bound, quantized_blocks

pytestmark = pytest.mark.gpu

N, K, L, B = 3000, 50, 60, 10
BLOCKS = [1000, 1000, 1000]
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def factors():
    rng = np.random.default_rng(4100)
    U = synth.orthonormal_factor(N, N, rng)
    V = synth.orthonormal_factor(N, N, rng)
    Om = synth.gaussian_omega(N, L, 4101)
    return U, V, Om


def _matrix(factors, kind):
    U, V, _ = factors
    s = synth.paper_type_spectrum(kind, N)
    return (U * s) @ V.T, s


def _gpu(A, Om, mode, src):
    import torch
    import paper_1704_07669_amd as sk
    dt = {"f64": torch.float64, "f32": torch.float32}[src]
    At = torch.from_numpy(A).to(dt).cuda()
    h = sk.Sketch(N, N, max(BLOCKS), K, L, B, compute=mode, omega=Om)
    r0 = 0
    for cnt in BLOCKS:
        h.ingest(At[r0:r0 + cnt])
        r0 += cnt
    Omq = h.omega().cpu().numpy()
    S, V, _, rank = h.finalize()
    torch.cuda.synchronize()
    h.close()
    return S.cpu().numpy(), V.cpu().numpy(), rank, Omq


@pytest.mark.parametrize("kind", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("mode,src", [("f64", "f64"), ("f32", "f32"), ("bf16", "f32"),
                                      ("bf16x2", "f32"), ("fp8", "f32")])
def test_type_spectra_parity(gpu_lib, factors, kind, mode, src):
    """Kernel parity on every spectrum: the pass within its rigorous elementwise bounds, and the
    FP64 finalize on the device's own sketch equal to the reference's on that sketch.  In FP64 the
    end result is also gated against the reference on A: the literal Algorithm 4 amplifies a
    relative sketch perturbation e by (sigma_1 / sigma_j)^2 through the Eq. 9 numerator, so the
    gate is 100 sqrt(n) u64 (sigma_1 / sigma_j)^2 per index.  In the FP32-accumulating modes e is
    about 1e-7, which that amplification turns into O(1) errors on Types 3 and 5 (and even moves
    sigma_1 when garbage rows of B outgrow it): the method's conditioning, measured and reported
    by the benchmark rather than gated here."""
    import torch
    import paper_1704_07669_amd as sk
    A, s = _matrix(factors, kind)
    dt = {"f64": torch.float64, "f32": torch.float32}[src]
    At = torch.from_numpy(A).to(dt).cuda()
    h = sk.Sketch(N, N, max(BLOCKS), K, L, B, compute=mode, omega=factors[2])
    r0 = 0
    for cnt in BLOCKS:
        h.ingest(At[r0:r0 + cnt])
        r0 += cnt
    Omq = h.omega().cpu().numpy()
    G, H = (x.cpu().numpy() for x in h.state())
    S, V, _, rank = h.finalize()
    torch.cuda.synchronize()
    h.close()
    S, V = S.cpu().numpy(), V.cpu().numpy()
    Aq = quantized_blocks(A, BLOCKS, mode, src)
    Gr, Hr = oracle.sketch_pass(Aq, Omq)
    if mode == "f64":
        gb = (N + 4) * U64 * (np.abs(np.vstack(Aq)) @ np.abs(Omq))
        hb = np.abs(np.vstack(Aq)).T @ (gb + (max(BLOCKS) + 8) * U64 * np.abs(Gr))
    else:
        gb = g_bound(Aq, Omq)
        hb = h_bound(Aq, Omq, Gr, gb, max(BLOCKS), split_g=(mode != "f32"))
    assert np.all(np.abs(G - Gr) <= gb + 1e-300)
    assert np.all(np.abs(H - Hr) <= hb + 1e-300)
    Q2, B2, r2, _ = oracle.qb_from_sketch(G, H, Omq, B)
    S2, _, V2 = oracle.svd_from_qb(Q2, B2, K)
    assert rank == r2
    # both finalizes are FP64 but factor differently (Cholesky QR against Householder QR); their
    # round-off meets the (sigma_1 / sigma_j)^2 amplification of the spectrum
    amp = (s[0] / s[:K]) ** 2
    assert np.all(oracle.rel_sigma_error(S, S2) <= 1e-9 + 100 * U64 * amp)
    if mode == "f64":
        ref = oracle.single_pass_pca(Aq, Omq, K, B)
        amp = (ref.S[0] / ref.S) ** 2
        assert np.all(oracle.rel_sigma_error(S, ref.S) <= 100 * np.sqrt(N) * U64 * amp)


def test_paper_observations_fp64(gpu_lib, factors):
    with open(os.path.join(GOLDEN, "paper_type1_accuracy.json")) as f:
        g = json.load(f)["printed"]
    Vt = factors[1]
    errs = {}
    for kind in range(1, 6):
        A, s = _matrix(factors, kind)
        S, V, rank, Omq = _gpu(A, factors[2], "f64", "f64")
        errs[kind] = float(np.max(np.abs(S - s[:K])))
        if kind == 1:
            assert g["alg4_max_abs_sigma_error"] / 10 <= errs[1] <= g["alg4_max_abs_sigma_error"] * 10
            _, Vs = oracle.apply_sign_convention(None, Vt[:, :1])
            assert np.max(np.abs(V[:, 0] - Vs[:, 0])) <= g["v1_inf_norm_difference"] * 10
            corr = [abs(np.corrcoef(V[:, j], Vt[:, j])[0, 1]) for j in range(10)]
            assert min(corr) >= 1 - (1 - g["lowest_pc_correlation_first10"]) * 10
            # Algorithm 2 on the same matrix and Omega (reference only) is far less accurate
            S2, _, _ = oracle.alg2_single_pass(A, Omq, synth.gaussian_omega(N, L, 4102), K)
            assert np.max(np.abs(S2 - s[:K])) > 10 * errs[1]
    for kind in range(2, 6):
        assert errs[kind] < errs[1], errs
