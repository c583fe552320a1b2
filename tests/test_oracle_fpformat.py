"""Pins for the round-to-format emulation (oracle/fpformat.py).

* every bit pattern of FP16, BF16 and FP8-E4M3FN decodes to a value that the
  rounding leaves unchanged, and encodes back to the same pattern;
* FP16 and FP32 rounding agree with numpy's own (correctly rounded) float64 ->
  float16 / float32 conversions;
* BF16 and FP8 rounding agree with torch's conversions on inputs that are
  already float32 (where torch's float32 -> target rounding is a single one);
* ties go to the even neighbour, overflow goes to inf (IEEE) or saturates at
  448 (E4M3FN), the largest finite values match the section on floating-point
  formats in the paper: (2 - 2^-23) 2^127 for FP32 and (2 - 2^-10) 2^15 for FP16.
"""
import numpy as np
import pytest
import torch

from oracle import fpformat as ff


def _finite_codes(f):
    width = 1 + f.ebits + f.mbits
    codes = np.arange(2 ** width, dtype=np.uint64)
    vals = ff.decode(codes, f)
    ok = np.isfinite(vals)
    return codes[ok], vals[ok]


@pytest.mark.parametrize("name", ["fp16", "bf16", "fp8_e4m3"])
def test_all_codes_round_trip(name):
    f = ff.FORMATS[name]
    codes, vals = _finite_codes(f)
    assert np.array_equal(ff.round_to(vals, f), vals)
    enc = ff.encode(vals, f)
    # -0 and +0 both decode to zero; compare through the value
    assert np.array_equal(ff.decode(enc, f), vals)
    nz = vals != 0
    assert np.array_equal(enc[nz], codes[nz])


def test_paper_max_finite_values():
    assert ff.FP32.max_finite == float(np.finfo(np.float32).max)
    assert ff.FP16.max_finite == float(np.finfo(np.float16).max)
    assert ff.FP32.max_finite == (2 - 2.0 ** -23) * 2.0 ** 127
    assert ff.FP16.max_finite == (2 - 2.0 ** -10) * 2.0 ** 15
    codes, vals = _finite_codes(ff.FP8_E4M3)
    assert vals.max() == 448.0 and np.min(np.abs(vals[vals != 0])) == 2.0 ** -9


def _wide_sample(n, seed):
    g = np.random.default_rng(seed)
    mant = g.uniform(1.0, 2.0, n)
    exps = g.integers(-160, 140, n)
    sign = g.choice([-1.0, 1.0], n)
    return sign * np.ldexp(mant, exps)


def test_fp16_matches_numpy():
    x = _wide_sample(200000, 1)
    x = np.concatenate([x, _wide_sample(20000, 2) * 2.0 ** -120])  # into fp16 subnormals / zero
    with np.errstate(over="ignore"):
        ref = x.astype(np.float16).astype(np.float64)
    assert np.array_equal(ff.round_to(x, "fp16"), ref)


def test_fp32_matches_numpy():
    x = _wide_sample(200000, 3)
    with np.errstate(over="ignore"):
        ref = x.astype(np.float32).astype(np.float64)
    assert np.array_equal(ff.round_to(x, "fp32"), ref)


def test_bf16_matches_torch_on_fp32_inputs():
    x = _wide_sample(200000, 4).astype(np.float32).astype(np.float64)
    x = x[np.isfinite(x)]
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(ff.round_to(x, "bf16"), ref)


def test_fp8_matches_torch_in_range():
    g = np.random.default_rng(5)
    x = g.uniform(-448, 448, 100000) * np.ldexp(1.0, g.integers(-12, 1, 100000))
    x = x.astype(np.float32).astype(np.float64)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.float8_e4m3fn).to(torch.float64).numpy()
    assert np.array_equal(ff.round_to(x, "fp8_e4m3"), ref)


def test_ties_to_even_and_single_rounding():
    # 1 + 2^-11 is the midpoint of 1 and 1 + 2^-10 in FP16: ties to 1 (even)
    assert ff.round_to(1.0 + 2.0 ** -11, "fp16") == 1.0
    # 1 + 3 * 2^-11 is the midpoint of 1+2^-10 and 1+2^-9: ties to 1 + 2^-9
    assert ff.round_to(1.0 + 3 * 2.0 ** -11, "fp16") == 1.0 + 2.0 ** -9
    # just above a midpoint goes up, even when FP32 would have landed on it
    assert ff.round_to(1.0 + 2.0 ** -11 + 2.0 ** -40, "fp16") == 1.0 + 2.0 ** -10
    assert ff.round_to(1.0 + 2.0 ** -8 + 2.0 ** -40, "bf16") == 1.0 + 2.0 ** -7
    assert ff.round_to(1.0 + 2.0 ** -8, "bf16") == 1.0
    assert ff.round_to(1.0 + 2.0 ** -4, "fp8_e4m3") == 1.0
    assert ff.round_to(1.0 + 3 * 2.0 ** -4, "fp8_e4m3") == 1.25


def test_overflow_and_saturation():
    assert ff.round_to(65520.0, "fp16") == np.inf        # midpoint above max -> inf
    assert ff.round_to(65519.99, "fp16") == 65504.0
    assert ff.round_to(-1e6, "fp16") == -np.inf
    for v in (449.0, 464.0, 480.0, 1e9, np.inf):
        assert ff.round_to(v, "fp8_e4m3") == 448.0
        assert ff.round_to(-v, "fp8_e4m3") == -448.0
    assert np.isnan(ff.round_to(np.nan, "bf16"))


def test_subnormals_kept():
    assert ff.round_to(2.0 ** -24, "fp16") == 2.0 ** -24
    assert ff.round_to(2.0 ** -25, "fp16") == 0.0                  # tie -> even (zero)
    assert ff.round_to(1.5 * 2.0 ** -25, "fp16") == 2.0 ** -24
    assert ff.round_to(2.0 ** -9, "fp8_e4m3") == 2.0 ** -9
    assert ff.round_to(3 * 2.0 ** -11, "fp8_e4m3") == 2.0 ** -9    # 0.75 ulp -> 1 ulp


def test_pow2_scale_exponent():
    assert int(ff.pow2_scale_exponent(448.0)) == 0
    assert int(ff.pow2_scale_exponent(1.0)) == 8        # 448 / 1 -> 2^8 = 256 <= 448 < 512
    assert int(ff.pow2_scale_exponent(4.0)) == 6
    assert int(ff.pow2_scale_exponent(449.0)) == -1
    assert int(ff.pow2_scale_exponent(0.0)) == 0
    g = np.random.default_rng(6)
    amax = np.abs(g.standard_normal(1000)) * 10.0 ** g.integers(-5, 5, 1000)
    s = ff.pow2_scale_exponent(amax)
    assert np.all(amax * 2.0 ** s <= 448.0) and np.all(amax * 2.0 ** (s + 1) > 448.0)
