"""Seeded draws for the many-stream serving workload.

64 streams; n uniform over the 32 multiples of 1024 up to 32768; m uniform in [10000, 200000]
rounded to a multiple of 1024; row blocks uniform in [256, 4096]; per-stream Poisson arrivals.
"""
from dataclasses import dataclass, field
import numpy as np


@dataclass
class ServingDraws:
    n: np.ndarray              # per stream
    m: np.ndarray              # per stream
    blocks: list = field(default_factory=list)    # per stream: array of block row counts
    arrivals: list = field(default_factory=list)  # per stream: arrival times (s), same length


def draw_serving_streams(num_streams: int = 64, n_choices=None, m_lo: int = 10000,
                         m_hi: int = 200000, blk_lo: int = 256, blk_hi: int = 4096,
                         rate_blocks_per_s: float = 100.0, seed: int = 30000,
                         m_scale: float = 1.0) -> ServingDraws:
    """Draw stream shapes, block sizes and Poisson arrival times.

    ``m_scale`` shrinks every m (for quick runs); block sizes are clipped to the stream length.
    """
    if n_choices is None:
        n_choices = 1024 * np.arange(1, 33)
    rs_shape = np.random.default_rng(seed)
    rs_arr = np.random.default_rng(seed + 1)
    rs_blk = np.random.default_rng(seed + 2)
    n = rs_shape.choice(np.asarray(n_choices), size=num_streams)
    m = rs_shape.integers(m_lo, m_hi + 1, size=num_streams)
    m = np.maximum(1024, (np.round(m * m_scale / 1024) * 1024).astype(np.int64))
    blocks, arrivals = [], []
    for s in range(num_streams):
        rows_left, sizes = int(m[s]), []
        while rows_left > 0:
            b = int(rs_blk.integers(blk_lo, blk_hi + 1))
            b = min(b, rows_left)
            sizes.append(b)
            rows_left -= b
        sizes = np.asarray(sizes, dtype=np.int64)
        gaps = rs_arr.exponential(1.0 / rate_blocks_per_s, size=len(sizes))
        blocks.append(sizes)
        arrivals.append(np.cumsum(gaps))
    return ServingDraws(n=n.astype(np.int64), m=m.astype(np.int64), blocks=blocks,
                        arrivals=arrivals)


def serving_pool_torch(n: int, sigma: np.ndarray, copies: int, seed: int, device, m0: int = 1024,
                       ext: int = 4096):
    """Stacking pool of one serving stream, as a float32 tensor of (m0 + ext) x n rows on `device`.

    A = [A0; ...; A0] (``copies`` copies) with A0 = U0 diag(sigma / sqrt(copies)) V0^T, U0 (m0 x r)
    and V0 (n x r) orthonormal from the QR of seeded Gaussians (r = number of nonzero sigma), so
    sigma(A) = sigma exactly.  The pool is A0 followed by its first ``ext`` rows again: a block of
    at most ``ext`` rows starting at row r0 of A is pool[r0 % m0 : r0 % m0 + rows].
    """
    import torch
    sig = np.asarray(sigma, dtype=np.float64)
    r = int(np.count_nonzero(sig))
    gen = torch.Generator(device="cpu").manual_seed(int(seed))
    U = torch.linalg.qr(torch.randn(m0, r, generator=gen, dtype=torch.float64).to(device))[0]
    V = torch.linalg.qr(torch.randn(n, r, generator=gen, dtype=torch.float64).to(device))[0]
    s = torch.as_tensor(sig[:r] / np.sqrt(copies), dtype=torch.float64, device=device)
    A0 = (U * s[None, :]) @ V.t()
    pool = torch.empty(m0 + ext, n, dtype=torch.float32, device=device)
    pool[:m0] = A0.to(torch.float32)
    reps = 0
    while m0 + reps < m0 + ext:
        cnt = min(m0, ext - reps)
        pool[m0 + reps:m0 + reps + cnt] = pool[:cnt]
        reps += cnt
    return pool
