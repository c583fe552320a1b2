"""Round-to-format emulation.

The paper (section "Floating-Point Arithmetic in Modern Technology") describes a
binary floating-point number as  x = +-m * 2^(e - t + 1)  with integer
significand 0 <= m <= 2^t - 1, precision t and exponent e in [emin, emax], and
gives the FP64 / FP32 / FP16 field widths (1/11/52, 1/8/23, 1/5/10).  BF16
(1/8/7) and FP8-E4M3FN (1/4/3, OCP "fn" variant: no infinities, one NaN code
per sign, largest finite 448) are the two further formats the mixed path uses.

Rounding is round-to-nearest, ties-to-even, applied ONCE to the exact float64
input (no intermediate FP32 step).  IEEE formats overflow to +-inf; FP8-E4M3FN
saturates to +-448 (the saturating conversion).  Subnormals are kept.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Format:
    name: str
    t: int          # precision in bits, including the implicit leading bit
    emin: int       # smallest normal exponent
    emax: int       # largest exponent
    ebits: int      # exponent field width
    mbits: int      # stored significand field width (t - 1)
    max_finite: float
    saturate: bool  # True: out-of-range values clamp to +-max_finite
    has_inf: bool

    @property
    def unit_roundoff(self) -> float:
        return 2.0 ** (-self.t)


FP64 = Format("fp64", 53, -1022, 1023, 11, 52, float(np.finfo(np.float64).max), False, True)
FP32 = Format("fp32", 24, -126, 127, 8, 23, (2 - 2.0 ** -23) * 2.0 ** 127, False, True)
FP16 = Format("fp16", 11, -14, 15, 5, 10, (2 - 2.0 ** -10) * 2.0 ** 15, False, True)
BF16 = Format("bf16", 8, -126, 127, 8, 7, (2 - 2.0 ** -7) * 2.0 ** 127, False, True)
# E4M3FN: bias 7, exponent field 1111 is an ordinary binade except that the
# all-ones significand is NaN, so the largest finite value is 1.75 * 2^8 = 448.
FP8_E4M3 = Format("fp8_e4m3", 4, -6, 8, 4, 3, 448.0, True, False)

FORMATS = {f.name: f for f in (FP64, FP32, FP16, BF16, FP8_E4M3)}
# Integer codes used by the C interface (mpcr_prec_t).
CODE = {"fp64": 0, "fp32": 1, "fp16": 2, "bf16": 3, "fp8_e4m3": 4}
BY_CODE = {v: FORMATS[k] for k, v in CODE.items()}


def fmt_of(f) -> Format:
    if isinstance(f, Format):
        return f
    if isinstance(f, (int, np.integer)):
        return BY_CODE[int(f)]
    return FORMATS[{"fp8": "fp8_e4m3"}.get(f, f)]


def round_to(x, f) -> np.ndarray:
    """Round float64 values to the nearest value of format ``f`` (ties to even),
    returned as float64.  One rounding step, from the exact input."""
    f = fmt_of(f)
    x = np.asarray(x, dtype=np.float64)
    if f is FP64:
        return x.copy()
    a = np.abs(x)
    finite_nz = np.isfinite(x) & (a > 0)
    safe = np.where(finite_nz, a, 1.0)
    _, E = np.frexp(safe)              # safe = mant * 2^E, mant in [0.5, 1)
    e = np.maximum(E - 1, f.emin)      # exponent of the binade (clamped: subnormals)
    q = np.ldexp(1.0, e - (f.t - 1))   # spacing of format values in that binade
    r = np.rint(x / q) * q             # x/q and *q are exact (power-of-two scaling)
    r = np.where(finite_nz, r, x)      # zeros, infs and NaNs pass through
    over = np.abs(r) > f.max_finite
    if f.saturate:
        r = np.where(over | np.isinf(x), np.copysign(f.max_finite, x), r)
    else:
        r = np.where(over, np.copysign(np.inf, x), r)
    return r


def decode(code, f) -> np.ndarray:
    """Value of each bit pattern ``code`` (unsigned integers of the format's
    width) read with the sign / exponent / significand layout of ``f``."""
    f = fmt_of(f)
    c = np.asarray(code, dtype=np.uint64)
    width = 1 + f.ebits + f.mbits
    sign = (c >> np.uint64(width - 1)) & np.uint64(1)
    ef = ((c >> np.uint64(f.mbits)) & np.uint64((1 << f.ebits) - 1)).astype(np.int64)
    mf = (c & np.uint64((1 << f.mbits) - 1)).astype(np.float64)
    bias = (1 << (f.ebits - 1)) - 1
    normal = np.ldexp(1.0 + mf / 2.0 ** f.mbits, ef - bias)
    sub = np.ldexp(mf / 2.0 ** f.mbits, 1 - bias)
    v = np.where(ef == 0, sub, normal)
    allones = (1 << f.ebits) - 1
    if f.has_inf:
        v = np.where((ef == allones) & (mf == 0), np.inf, v)
        v = np.where((ef == allones) & (mf != 0), np.nan, v)
    else:
        v = np.where((ef == allones) & (mf == (1 << f.mbits) - 1), np.nan, v)
    return np.where(sign == 1, -v, v)


def encode(x, f) -> np.ndarray:
    """Bit pattern of values that are already exactly representable in ``f``
    (finite, or +-inf for IEEE formats).  Inverse of ``decode`` on those."""
    f = fmt_of(f)
    x = np.asarray(x, dtype=np.float64)
    width = 1 + f.ebits + f.mbits
    bias = (1 << (f.ebits - 1)) - 1
    sign = np.signbit(x).astype(np.uint64)
    a = np.abs(x)
    out = np.zeros(x.shape, dtype=np.uint64)
    nz = (a > 0) & np.isfinite(a)
    safe = np.where(nz, a, 1.0)
    _, E = np.frexp(safe)
    e = E - 1
    is_sub = e < f.emin
    ef = np.where(is_sub, 0, e + bias).astype(np.int64)
    mant = np.where(is_sub, safe / 2.0 ** (f.emin - f.mbits), safe / np.ldexp(1.0, e) * 2.0 ** f.mbits - 2.0 ** f.mbits)
    mant = np.rint(mant).astype(np.uint64)
    bits = (ef.astype(np.uint64) << np.uint64(f.mbits)) | mant
    out = np.where(nz, bits, out)
    if f.has_inf:
        out = np.where(np.isinf(a), np.uint64(((1 << f.ebits) - 1) << f.mbits), out)
    return out | (sign << np.uint64(width - 1))


def pow2_scale_exponent(amax) -> np.ndarray:
    """Exponent s of the power-of-two scale 2^s that maps a block with largest
    magnitude ``amax`` into FP8-E4M3FN range: the largest integer s with
    amax * 2^s <= 448 (that is floor(log2(448 / amax)) evaluated exactly), and
    s = 0 for an all-zero block.  The exponent is stored as a signed byte, so it
    is clamped to [-128, 127]."""
    amax = np.asarray(amax, dtype=np.float64)
    pos = amax > 0
    m, E = np.frexp(np.where(pos, amax, 1.0))   # amax = m 2^E, m in [0.5, 1); 448 = 0.875 2^9
    s = np.where(m <= 0.875, 9 - E, 8 - E)
    return np.clip(np.where(pos, s, 0), -128, 127).astype(np.int64)
