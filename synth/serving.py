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
