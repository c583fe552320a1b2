"""Pins for the multi-format GEMM emulation (oracle/gemm.py).

P8(i)  Integer entries in [-4, 4] with k = 8192 keep every partial sum an
       integer below 2^24, so every format (FP8 after its 2^6 block scale too)
       must give the FP64 product exactly.
P8(ii) For U(-1, 1) entries rounded to nearest, the relative Frobenius error of
       the product is about u / sqrt(3) (u the unit roundoff), the measure the
       paper's section "Linear Algebra Functions Performance" reports.
FP8 block scales follow s = floor(log2(448 / amax)) per 128 x 128 block and
dequantise exactly.
"""
import math

import numpy as np
import pytest

import synth
from oracle import dense, fpformat as ff, gemm


@pytest.mark.parametrize("fmt", ["fp64", "fp32", "fp16", "bf16", "fp8_e4m3"])
def test_integer_inputs_exact_in_every_format(fmt):
    A = synth.integer_matrix(64, 8192, 50)
    B = synth.integer_matrix(8192, 48, 51)
    C = gemm.gemm_emulated(A, B, fmt, c_fmt="fp32" if fmt != "fp64" else "fp64")
    assert np.array_equal(C, A @ B)
    assert np.all(np.abs(A @ B) < 2 ** 24)


@pytest.mark.parametrize("fmt,lo,hi", [("fp32", 0.5, 1.6), ("fp16", 0.5, 1.6), ("bf16", 0.5, 1.6), ("fp8_e4m3", 0.4, 2.0)])
def test_uniform_inputs_error_near_u_over_sqrt3(fmt, lo, hi):
    A = synth.uniform_matrix(256, 1024, 52)
    B = synth.uniform_matrix(1024, 256, 53)
    ref = dense.gemm(A, B)
    C = gemm.gemm_emulated(A, B, fmt, c_fmt="fp64")
    u = ff.fmt_of(fmt).unit_roundoff
    ratio = gemm.rel_frobenius(C, ref) / (u / math.sqrt(3))
    assert lo < ratio < hi, ratio


def test_fp8_block_scaling():
    A = synth.uniform_matrix(300, 260, 54) * np.logspace(-3, 2, 260)[None, :]
    Q, S = gemm.fp8_block_quantize(A)
    assert S.shape == (3, 3)
    assert np.all(np.abs(Q) <= 448.0)
    for bi in range(3):
        for bj in range(3):
            blk = A[bi * 128:(bi + 1) * 128, bj * 128:(bj + 1) * 128]
            assert S[bi, bj] == ff.pow2_scale_exponent(np.abs(blk).max())
    D = gemm.fp8_block_dequantize(Q, S)
    assert np.array_equal(gemm.fp8_block_dequantize(*gemm.fp8_block_quantize(D)), D)
    assert gemm.rel_max(D, A) < 2 * ff.FP8_E4M3.unit_roundoff * 4


def test_transposes_alpha_beta():
    A = synth.uniform_matrix(40, 30, 55)
    B = synth.uniform_matrix(50, 40, 56)
    C = synth.uniform_matrix(30, 50, 57)
    out = gemm.gemm_emulated(A, B, "fp64", transA=True, transB=True, alpha=0.5, beta=2.0, C=C)
    np.testing.assert_allclose(out, 0.5 * A.T @ B.T + 2.0 * C, rtol=1e-14)
