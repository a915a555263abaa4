"""Checkpoint, restore and merge of the pass state through the C ABI.

The state after any prefix of the row blocks is G (rows so far), H and Omega' (Alg. 4 steps 3-8).
A pass checkpointed mid-stream, restored into a fresh handle and continued must give the same bits
as the uninterrupted pass.  Eq. 10 makes the state mergeable: merging the sketch of a second row
shard into the first gives G = [G_1; G_2] (bit for bit, the blocks being the same) and
H = H_1 + H_2 (the FP64 sums in another order: within the FP64 round-off of the sums).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import U64

pytestmark = pytest.mark.gpu

MODES = [("f64", "f64"), ("f32", "f32"), ("bf16", "f32"), ("bf16x2", "f32"), ("fp8", "f32")]


@pytest.fixture(scope="module")
def case():
    m, n, l, k, b = 1531, 777, 40, 20, 10
    sig = synth.noisy_spectrum(synth.exp_spectrum(n, 8.0), 1e-6, 21)
    A, _, s, _ = synth.small_matrix(m, n, sig, 21)
    Om = synth.gaussian_omega(n, l, 22)
    return dict(A=A, Om=Om, k=k, l=l, b=b, blocks=[300, 1, 430, 513, 287])


def _tensor(A, src):
    import torch
    dt = {"f64": torch.float64, "f32": torch.float32}[src]
    return torch.from_numpy(np.ascontiguousarray(A)).to(dt).cuda()


def _sketch(sk, case, mode, seeded, m_capacity=None):
    A = case["A"]
    m, n = A.shape
    return sk.Sketch(n, m_capacity or m, max(case["blocks"]), case["k"], case["l"], case["b"],
                     compute=mode, want_u=True, seed=77 if seeded else 0,
                     omega=None if seeded else case["Om"])


def _ingest(s, At, blocks, start=0):
    r0 = start
    for cnt in blocks:
        s.ingest(At[r0:r0 + cnt])
        r0 += cnt
    return r0


def _result(s):
    import torch
    S, V, U, rank = s.finalize()
    torch.cuda.synchronize()
    return S.cpu().numpy(), V.cpu().numpy(), U.cpu().numpy(), rank


@pytest.mark.parametrize("seeded", [True, False])
@pytest.mark.parametrize("mode,src", MODES)
def test_restore_continues_bit_for_bit(gpu_lib, case, mode, src, seeded):
    sk = gpu_lib
    At = _tensor(case["A"], src)
    blocks = case["blocks"]
    ref = _sketch(sk, case, mode, seeded)
    _ingest(ref, At, blocks)
    S0, V0, U0, r0 = _result(ref)
    ref.close()

    first = _sketch(sk, case, mode, seeded)
    done = _ingest(first, At, blocks[:3])
    buf = first.checkpoint()
    first.close()
    # the fresh handle draws another Omega (or none): the restore replaces it by the checkpoint's
    second = _sketch(sk, case, mode, seeded)
    if seeded:
        second.reset(12345)
    second.restore(buf)
    _ingest(second, At, blocks[3:], start=done)
    S1, V1, U1, r1 = _result(second)
    second.close()
    assert r1 == r0
    assert np.array_equal(S0, S1) and np.array_equal(V0, V1) and np.array_equal(U0, U1)


@pytest.mark.parametrize("mode,src", MODES)
def test_merge_of_row_shards(gpu_lib, case, mode, src):
    sk = gpu_lib
    At = _tensor(case["A"], src)
    blocks = case["blocks"]
    whole = _sketch(sk, case, mode, True)
    _ingest(whole, At, blocks)
    G0, H0 = (x.cpu().numpy() for x in whole.state())
    S0, V0, _, _ = _result(whole)
    whole.close()

    a = _sketch(sk, case, mode, True)
    split = _ingest(a, At, blocks[:2])
    b = _sketch(sk, case, mode, True, m_capacity=case["A"].shape[0])
    _ingest(b, At, blocks[2:], start=split)
    a.merge(b.checkpoint())
    b.close()
    G1, H1 = (x.cpu().numpy() for x in a.state())
    assert np.array_equal(G0, G1)
    # H_1 + H_2 against one running sum: each entry differs by at most a few FP64 roundings of
    # the partial sums' sizes
    Ga = np.abs(G0)
    Aabs = np.abs(case["A"])
    bound = 8 * U64 * (Aabs.T @ Ga) + 1e-300
    assert np.all(np.abs(H1 - H0) <= bound)
    S1, V1, _, _ = _result(a)
    a.close()
    assert np.max(oracle.rel_sigma_error(S1, S0)) < 1e-9
    assert oracle.sin_theta_max(V0, V1) < 1e-7


def test_checkpoint_errors(gpu_lib, case):
    sk = gpu_lib
    At = _tensor(case["A"], "f32")
    s = _sketch(sk, case, "f32", True)
    _ingest(s, At, case["blocks"][:2])
    buf = s.checkpoint()
    # wrong compute mode, wrong n, too few rows of capacity
    other = sk.Sketch(case["A"].shape[1], case["A"].shape[0], 600, 20, 40, 10, compute="bf16", seed=77)
    with pytest.raises(sk.SketchError) as e:
        other.restore(buf)
    assert e.value.status == 1
    other.close()
    small = sk.Sketch(case["A"].shape[1], 100, 100, 20, 40, 10, compute="f32", seed=77)
    with pytest.raises(sk.SketchError) as e:
        small.restore(buf)
    assert e.value.status == 4
    small.close()
    # truncated and corrupted buffers
    with pytest.raises(sk.SketchError) as e:
        s.restore(buf[:-8])
    assert e.value.status == 1
    bad = buf.copy()
    bad[0] ^= 0xFF
    with pytest.raises(sk.SketchError) as e:
        s.restore(bad)
    assert e.value.status == 1
    # a sketch with another Omega cannot be merged
    t = _sketch(sk, case, "f32", True)
    t.reset(78)
    _ingest(t, At, case["blocks"][:1])
    with pytest.raises(sk.SketchError) as e:
        s.merge(t.checkpoint())
    assert e.value.status == 1
    t.close()
    # after finalize there is no state to save or merge into
    s.finalize()
    with pytest.raises(sk.SketchError) as e:
        s.checkpoint()
    with pytest.raises(sk.SketchError) as e:
        s.merge(buf)
    assert e.value.status == 2
    s.close()


def test_empty_checkpoint_round_trip(gpu_lib, case):
    sk = gpu_lib
    At = _tensor(case["A"], "f32")
    s = _sketch(sk, case, "f32", False)
    buf = s.checkpoint()
    s.close()
    t = _sketch(sk, case, "f32", False)
    t.restore(buf)
    _ingest(t, At, case["blocks"])
    S1, _, _, _ = _result(t)
    t.close()
    ref = oracle.single_pass_pca([case["A"]], case["Om"], case["k"], case["b"])
    assert np.max(oracle.rel_sigma_error(S1, ref.S)) < 1e-4
