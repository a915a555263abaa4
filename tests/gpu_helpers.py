"""Shared helpers of the GPU tests: run the HIP path through the C ABI, and build the reference
operands (A', Omega') with the oracle's own rounding."""
import numpy as np

import oracle

U32 = 2.0 ** -24
U64 = 2.0 ** -53


def run_gpu(A, Omega, k, b, mode, blocks, src="f32", want_u=True, host=False, host_slots=3,
            seed=None, keep_state=True, force=(0, 0)):
    """Run the library on A (numpy) split into row blocks of the given sizes; `force` takes the
    Householder paths of the finalize directly (loop, R_B).

    Returns dict(S, V, U, rank, G, H, Om, paths) as numpy float64 (G, H before finalize); paths =
    the finalize's (loop, R_B) methods, 0 Cholesky QR, 1 Householder."""
    import torch
    import paper_1704_07669_amd as sk
    m, n = A.shape
    l = Omega.shape[1] if Omega is not None else None
    tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[src]
    sketch = sk.Sketch(n, m, max(blocks), k, l, b, compute=mode, want_u=want_u,
                       host_slots=host_slots if host else 0, host_src=src,
                       omega=Omega, seed=seed or 0)
    At = torch.from_numpy(np.ascontiguousarray(A)).to(tdt)
    if host:
        At = At.pin_memory()
    else:
        At = At.cuda()
    r0 = 0
    tickets = []
    for cnt in blocks:
        tickets.append(sketch.ingest(At[r0:r0 + cnt]))
        r0 += cnt
    assert r0 == m
    out = {}
    if keep_state:
        G, H = sketch.state()
        out["G"], out["H"] = G.cpu().numpy(), H.cpu().numpy()
    out["Om"] = sketch.omega().cpu().numpy()
    if any(force):
        sketch.force_paths(*force)
    S, V, U, rank = sketch.finalize()
    torch.cuda.synchronize()
    out.update(S=S.cpu().numpy(), V=V.cpu().numpy(), U=None if U is None else U.cpu().numpy(),
               rank=rank, tickets=tickets, sketch=sketch, paths=sketch.finalize_paths())
    return out


def split_blocks(A, blocks):
    out, r0 = [], 0
    for cnt in blocks:
        out.append(A[r0:r0 + cnt])
        r0 += cnt
    return out


def quantized_blocks(A, blocks, mode, src="f32"):
    """The exact row blocks A' the kernels consume in `mode` (per-block FP8 scales)."""
    base = np.asarray(A, dtype=np.float64)
    if src == "f32":
        base = oracle.round_fp32(base)
    elif src == "bf16":
        base = oracle.round_bf16(base)
    return [oracle.quantize_block(a, mode) for a in split_blocks(base, blocks)]


def g_bound(Ablocks, Om, splits=64):
    """Elementwise rigorous bound (K + splits + 2) u32 (|A'| |Omega'|) for FP32 accumulation."""
    K = Om.shape[0]
    absA = np.abs(np.vstack(Ablocks))
    return (K + splits + 2) * U32 * (absA @ np.abs(Om))


def h_bound(Ablocks, Om, G_ref, gb, block_rows, split_g):
    """Bound on |H_gpu - A'^T G_ref| from the G error, the BF16 hi/lo split of G (2^-17 relative)
    and FP32 accumulation over a block's rows."""
    absA = np.abs(np.vstack(Ablocks))
    per = gb + ((2.0 ** -17 if split_g else 0.0) + (block_rows + 8) * U32) * np.abs(G_ref)
    return absA.T @ per
