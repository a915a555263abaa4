"""Round-to-nearest-even conversions that define the exact operands of the reduced-precision modes.

Test infrastructure only.  The paper computes in FP64 after reading FP32 files (Sec. 4.2); the
reduced-precision modes are not in the paper.  Their reading: the kernel consumes A' (and Omega'),
the input rounded once to the compute format, and the reference is then run on A' and Omega'
exactly.  These functions build A' and Omega' from their definitions:

* FP32: IEEE round-to-nearest-even of the FP64 value.
* BF16: round-to-nearest-even of the value itself to 8 significant bits (the BF16 grid), taken
  from its FP64 representation; for FP32 inputs this is the usual RNE of the FP32 value.  Values
  below 2^-126 in magnitude (BF16's subnormal range) go through FP32 first.
* BF16X2: hi = bf16(x), lo = bf16(x - hi) (x - hi is exact in FP32); the operand is hi + lo.
* FP8 E4M3 (OCP, bias 7, largest finite 448): round-to-nearest-even with a power-of-two block
  scale 2^e chosen as the largest with amax * 2^e <= 448, so scaling itself is exact.
* Omega' for BF16/BF16X2 is bf16(Omega), rounded once from FP64; for FP8 it is
  fp8(32 * fp32(Omega)) / 32.
"""
import numpy as np


def round_fp32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def _round_bf16_from_fp32(f):
    u = np.ascontiguousarray(f, dtype=np.float32).view(np.uint32).astype(np.uint64)
    bias = np.uint64(0x7FFF) + ((u >> np.uint64(16)) & np.uint64(1))
    r = ((u + bias) & np.uint64(0xFFFF0000)).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def round_bf16(x):
    """bf16 RNE of x (one rounding from its FP64 value), returned as float64: the FP64 bit pattern
    rounded to nearest even at 45 bits below its significand's top, i.e. to 8 significant bits."""
    d = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    u = d.view(np.uint64)
    bias = np.uint64((1 << 44) - 1) + ((u >> np.uint64(45)) & np.uint64(1))
    r = ((u + bias) & ~np.uint64((1 << 45) - 1)).view(np.float64)
    small = ~(np.abs(d) >= 2.0 ** -126)
    if np.any(small):
        r = np.where(small, _round_bf16_from_fp32(d.astype(np.float32)), r)
    return r


def split_bf16x2(x):
    """(hi, lo) with hi = bf16(x), lo = bf16(x - hi), x taken as fp32."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)
    hi = round_bf16(f)
    lo = round_bf16((f - hi).astype(np.float32))
    return hi, lo


def round_fp8_e4m3(x):
    """RNE to the OCP E4M3 grid (3 mantissa bits, min normal 2^-6, subnormal step 2^-9), saturating
    at +-448.  Input is rounded to fp32 first."""
    v = np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)
    a = np.abs(v)
    with np.errstate(divide="ignore"):
        e = np.floor(np.log2(np.where(a > 0, a, 1.0)))
    # guard the floor(log2) against representation error at exact powers of two
    e = np.where(2.0 ** (e + 1) <= a, e + 1, e)
    e = np.where(2.0 ** e > a, e - 1, e)
    e = np.maximum(e, -6.0)
    quantum = 2.0 ** (e - 3.0)
    r = np.rint(a / quantum) * quantum          # np.rint rounds half to even
    r = np.minimum(r, 448.0)
    return np.copysign(r, v)


def fp8_block_exponent(amax: float) -> int:
    """Largest integer e with amax * 2^e <= 448 (0 for an all-zero block)."""
    amax = float(np.float32(amax))
    if amax == 0.0 or not np.isfinite(amax):
        return 0
    f, ex = np.frexp(amax)            # amax = f * 2^ex, f in [0.5, 1)
    return int((9 - ex) if f <= 0.875 else (8 - ex))


def quantize_block(a, mode: str):
    """The exact operand A' a kernel of the given mode consumes for this row block (FP64 array)."""
    a = np.asarray(a, dtype=np.float64)
    if mode == "f64":
        return a.copy()
    if mode == "f32":
        return round_fp32(a)
    if mode == "bf16":
        return round_bf16(a)
    if mode == "bf16x2":
        hi, lo = split_bf16x2(a)
        return hi + lo
    if mode == "fp8":
        f = round_fp32(a)
        e = fp8_block_exponent(np.max(np.abs(f)) if f.size else 0.0)
        return round_fp8_e4m3(f * 2.0 ** e) * 2.0 ** (-e)
    raise ValueError(mode)


def quantize_omega(Omega, mode: str):
    """Omega' as used by every step of the given mode (FP64 array)."""
    Omega = np.asarray(Omega, dtype=np.float64)
    if mode == "f64":
        return Omega.copy()
    if mode == "f32":
        return round_fp32(Omega)
    if mode in ("bf16", "bf16x2"):
        return round_bf16(Omega)
    if mode == "fp8":
        return round_fp8_e4m3(round_fp32(Omega) * 32.0) / 32.0
    raise ValueError(mode)
