"""Philox-4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11) and the Box-Muller Gaussian test matrix built from it.

Test infrastructure only.  The paper draws Omega = randn(n, l) (Algorithm 4, step 3) without naming
a generator; the reading used here is: entry (r, c) of Omega, with linear index q = r*l + c, takes
the 64-bit words 2q and 2q+1 of the Philox stream with key (seed, 0), where word w is lane w % 4 of
the block at counter (w // 4, 0, 0, 0); u1 = (w0 >> 11) 2^-53, u2 = (w1 >> 11) 2^-53 and
z = sqrt(-2 ln(1 - u1)) cos(2 pi u2).
"""
import numpy as np

_M = (0xD2E7470EE14C6C93, 0xCA5A826395121157)     # Philox-4x64 round multipliers (SC'11)
_W = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)     # key schedule (Weyl) increments (SC'11)
_MASK32 = np.uint64(0xFFFFFFFF)


def _mulhilo(a, b):
    """Full 64x64 -> 128-bit product of uint64 arrays, as (hi, lo)."""
    a = a.astype(np.uint64)
    b = np.uint64(b)
    s32 = np.uint64(32)
    al, ah = a & _MASK32, a >> s32
    bl, bh = b & _MASK32, b >> s32
    ll = al * bl
    lh = al * bh
    hl = ah * bl
    hh = ah * bh
    mid = (ll >> s32) + (lh & _MASK32) + (hl & _MASK32)
    hi = hh + (lh >> s32) + (hl >> s32) + (mid >> s32)
    lo = a * b
    return hi, lo


def philox4x64_10(counters, key0: int, key1: int = 0):
    """Philox-4x64 with 10 rounds on an array of counters (N x 4 uint64); returns N x 4 uint64."""
    x = np.array(counters, dtype=np.uint64).reshape(-1, 4).copy()
    k0, k1 = np.uint64(key0 & 0xFFFFFFFFFFFFFFFF), np.uint64(key1 & 0xFFFFFFFFFFFFFFFF)
    with np.errstate(over="ignore"):
        for _ in range(10):
            hi0, lo0 = _mulhilo(x[:, 0], _M[0])
            hi1, lo1 = _mulhilo(x[:, 2], _M[1])
            x = np.stack([hi1 ^ x[:, 1] ^ k0, lo1, hi0 ^ x[:, 3] ^ k1, lo0], axis=1)
            k0 = k0 + np.uint64(_W[0])
            k1 = k1 + np.uint64(_W[1])
    return x


def philox_words(seed: int, first_word: int, count: int):
    """Words first_word .. first_word+count-1 of the stream with key (seed, 0)."""
    w = np.arange(first_word, first_word + count, dtype=np.uint64)
    blocks = w // np.uint64(4)
    ub = np.unique(blocks)
    ctr = np.zeros((len(ub), 4), dtype=np.uint64)
    ctr[:, 0] = ub
    out = philox4x64_10(ctr, seed)
    idx = np.searchsorted(ub, blocks)
    return out[idx, (w % np.uint64(4)).astype(np.int64)]


def gaussian_omega_philox(n: int, l: int, seed: int) -> np.ndarray:
    """Omega (n x l) under the reading in the module docstring, in FP64."""
    q = np.arange(n * l, dtype=np.uint64)
    w0 = philox_words(seed, 0, 2 * n * l)
    u1 = (w0[0::2] >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    u2 = (w0[1::2] >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    z = np.sqrt(-2.0 * np.log1p(-u1)) * np.cos(2.0 * np.pi * u2)
    del q
    return z.reshape(n, l)
