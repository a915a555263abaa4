"""The power scheme with P = 1 on the GPU (Sec. 2.2; the remark closing Sec. 3.3; Sec. 4.2).

After the first pass the library replaces Omega by Omega_2 = sqrt(n) orth(H) and the rows are
ingested again.  Checked against the reference:
  * orth: the device's Omega_2 (before rounding to the operand format only the FP64 route matters)
    spans the same space as the reference's power_omega of the device's own H;
  * the second pass and finalize: Algorithm 4 of the reference on A' and the device's Omega_2'
    (the same comparison, and tolerances, as the single-pass end-to-end parity);
  * every orthonormalisation route gives the same result;
  * accuracy against the known spectrum improves by orders of magnitude on the slowly decaying
    Type 2 spectrum (Sec. 4.2).
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
    sig = synth.noisy_spectrum(synth.exp_spectrum(n, 8.0), 1e-6, 41)
    A, _, s, _ = synth.small_matrix(m, n, sig, 41)
    return dict(A=A, s=s, k=k, l=l, b=b, blocks=[1, 17, 300, 513, 700])


def _tensor(A, src):
    import torch
    dt = {"f64": torch.float64, "f32": torch.float32}[src]
    return torch.from_numpy(np.ascontiguousarray(A)).to(dt).cuda()


def _two_passes(sk, At, case, mode, route=0, seed=5):
    import torch
    m, n = At.shape
    s = sk.Sketch(n, m, max(case["blocks"]), case["k"], case["l"], case["b"], compute=mode,
                  want_u=True, seed=seed)

    def one_pass():
        r0 = 0
        for cnt in case["blocks"]:
            s.ingest(At[r0:r0 + cnt])
            r0 += cnt

    one_pass()
    _, H1 = s.state()
    H1 = H1.cpu().numpy()
    used = s.power_restart(route)
    Om2 = s.omega().cpu().numpy()
    one_pass()
    S, V, U, rank = s.finalize()
    torch.cuda.synchronize()
    s.close()
    return dict(H1=H1, Om2=Om2, route=used, S=S.cpu().numpy(), V=V.cpu().numpy(),
                U=U.cpu().numpy(), rank=rank)


@pytest.mark.parametrize("mode,src", MODES)
def test_power_scheme_parity(gpu_lib, case, mode, src):
    A, k, b, blocks = case["A"], case["k"], case["b"], case["blocks"]
    out = _two_passes(gpu_lib, _tensor(A, src), case, mode)
    n = A.shape[1]
    # Omega_2 spans orth(H) of the device's own first-pass H (rounding to the operand format
    # moves the span by at most the format's relative precision, times the conditioning of H)
    ref_om = oracle.power_omega(out["H1"])
    ang_tol = {"f64": 1e-8, "f32": 1e-5, "bf16": 3e-2, "bf16x2": 3e-2, "fp8": 0.3}[mode]
    assert oracle.sin_theta_max(ref_om / np.sqrt(n), np.linalg.qr(out["Om2"])[0]) < ang_tol
    # the second pass and finalize against the reference on the same A' and Omega_2'
    ref = oracle.single_pass_pca(quantized_blocks(A, blocks, mode, src), out["Om2"], k, b)
    assert out["rank"] == ref.rank
    tol_s, tol_v = (1e-10, 1e-8) if mode == "f64" else (2e-4, 2e-3)
    assert np.max(oracle.rel_sigma_error(out["S"], ref.S)) < tol_s
    assert oracle.sin_theta_max(ref.V, out["V"]) < tol_v
    assert oracle.sin_theta_max(ref.U, out["U"]) < tol_v


@pytest.mark.parametrize("route", [1, 2])
def test_power_routes_agree(gpu_lib, case, route):
    """Shifted Cholesky QR3 and Gram-Schmidt + TSQR give the same orth(H) as the automatic route
    (the span, and so the final triplets, to FP64 round-off)."""
    At = _tensor(case["A"], "f64")
    auto = _two_passes(gpu_lib, At, case, "f64", route=0)
    forced = _two_passes(gpu_lib, At, case, "f64", route=route)
    assert forced["route"] == route
    n = case["A"].shape[1]
    assert np.linalg.norm(forced["Om2"].T @ forced["Om2"] / n - np.eye(case["l"])) < 1e-10
    assert oracle.sin_theta_max(np.linalg.qr(auto["Om2"])[0], np.linalg.qr(forced["Om2"])[0]) < 1e-8
    assert np.max(oracle.rel_sigma_error(forced["S"], auto["S"])) < 1e-10
    assert oracle.sin_theta_max(auto["V"], forced["V"]) < 1e-8


@pytest.mark.parametrize("mode,src", [("f64", "f64"), ("f32", "f32"), ("bf16", "f32")])
def test_power_scheme_improves_accuracy(gpu_lib, mode, src):
    """Type 2 spectrum, 3000 x 1500, k = 16, l = 30: P = 1 brings max |sigma_j - sigma_j(A)| down
    by more than an order of magnitude, as the reference does (Sec. 4.2)."""
    import torch
    sk = gpu_lib
    m, n, k, l, b = 3000, 1500, 16, 30, 10
    sig = synth.paper_type_spectrum(2, n)
    A, _, s, _ = synth.small_matrix(m, n, sig, 61)
    At = _tensor(A, src)
    h = sk.Sketch(n, m, 1000, k, l, b, compute=mode, seed=62)
    for r0 in range(0, m, 1000):
        h.ingest(At[r0:r0 + 1000])
    S0, _, _, _ = h.finalize()
    h.reset(62)
    for r0 in range(0, m, 1000):
        h.ingest(At[r0:r0 + 1000])
    h.power_restart()
    for r0 in range(0, m, 1000):
        h.ingest(At[r0:r0 + 1000])
    S1, _, _, _ = h.finalize()
    torch.cuda.synchronize()
    h.close()
    e0 = np.max(np.abs(S0.cpu().numpy() - s[:k]))
    e1 = np.max(np.abs(S1.cpu().numpy() - s[:k]))
    Om = oracle.gaussian_omega_philox(n, l, 62)
    r1 = oracle.single_pass_pca_power(split_blocks(A, [1000] * 3), Om, k, b)
    e_ref = np.max(np.abs(r1.S - s[:k]))
    assert e1 * 10 < e0, (e0, e1)
    assert e1 < 10 * e_ref + (1e-6 if mode == "bf16" else 1e-9), (e1, e_ref)


def test_power_restart_states(gpu_lib, case):
    sk = gpu_lib
    At = _tensor(case["A"], "f32")
    s = sk.Sketch(case["A"].shape[1], case["A"].shape[0], 700, 20, 40, 10, compute="f32", seed=3)
    with pytest.raises(sk.SketchError) as e:      # no first pass yet
        s.power_restart()
    assert e.value.status == 2
    s.ingest(At[:700])
    with pytest.raises(sk.SketchError) as e:
        s.power_restart(7)
    assert e.value.status == 1
    s.power_restart()
    # a checkpoint now carries Omega_2 itself, and a restore continues with it
    s.ingest(At[:300])
    buf = s.checkpoint()
    t = sk.Sketch(case["A"].shape[1], case["A"].shape[0], 700, 20, 40, 10, compute="f32", seed=3)
    t.restore(buf)
    assert np.array_equal(t.omega().cpu().numpy(), s.omega().cpu().numpy())
    t.close()
    s.finalize()
    with pytest.raises(sk.SketchError) as e:      # after finalize
        s.power_restart()
    assert e.value.status == 2
    s.close()
