"""Multi-format GEMM emulation (oracle side).

The paper's section "Linear Algebra Functions Performance" multiplies the same
matrices in double, single and half precision and reports the relative
Frobenius error ||C - C_ref||_F / ||C_ref||_F against the double-precision
product.  Emulation model used as the parity target for the GPU GEMM:

* both operands are rounded once from FP64 to the input format (FP8-E4M3FN
  after scaling each 128 x 128 block of the stored matrix by its power-of-two
  factor 2^s, s = floor(log2(448 / amax)); the block is dequantised by 2^-s,
  which is exact);
* the product of the rounded operands is accumulated exactly (FP64 model);
* alpha, beta are applied in FP64 and the result is rounded once to the output
  format.
"""
from __future__ import annotations

import numpy as np

from .fpformat import FP8_E4M3, fmt_of, pow2_scale_exponent, round_to

BLOCK = 128


def fp8_block_quantize(A: np.ndarray, block: int = BLOCK):
    """Returns (Q, s): Q holds the FP8 values (as float64) of A * 2^s_blk and
    s[bi, bj] the exponent of block (bi, bj) of the stored matrix."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    bm, bn = (m + block - 1) // block, (n + block - 1) // block
    Q = np.empty_like(A)
    S = np.zeros((bm, bn), dtype=np.int64)
    for bi in range(bm):
        for bj in range(bn):
            sl = (slice(bi * block, (bi + 1) * block), slice(bj * block, (bj + 1) * block))
            s = int(pow2_scale_exponent(np.max(np.abs(A[sl])) if A[sl].size else 0.0))
            S[bi, bj] = s
            Q[sl] = round_to(np.ldexp(A[sl], s), FP8_E4M3)
    return Q, S


def fp8_block_dequantize(Q: np.ndarray, S: np.ndarray, block: int = BLOCK) -> np.ndarray:
    out = np.empty_like(Q)
    for bi in range(S.shape[0]):
        for bj in range(S.shape[1]):
            sl = (slice(bi * block, (bi + 1) * block), slice(bj * block, (bj + 1) * block))
            out[sl] = np.ldexp(Q[sl], -int(S[bi, bj]))
    return out


def input_rounded(A: np.ndarray, fmt) -> np.ndarray:
    """Operand as the GEMM sees it, widened back to float64."""
    f = fmt_of(fmt)
    if f is FP8_E4M3:
        Q, S = fp8_block_quantize(A)
        return fp8_block_dequantize(Q, S)
    return round_to(A, f)


def gemm_emulated(A, B, fmt, transA=False, transB=False, alpha=1.0, beta=0.0, C=None, c_fmt="fp64"):
    Ar = input_rounded(A, fmt)
    Br = input_rounded(B, fmt)
    opA = Ar.T if transA else Ar
    opB = Br.T if transB else Br
    P = alpha * np.matmul(opA, opB)
    if C is not None and beta != 0.0:
        P = P + beta * np.asarray(C, np.float64)
    return round_to(P, c_fmt)


def rel_frobenius(C, C_ref) -> float:
    return float(np.linalg.norm(C - C_ref) / np.linalg.norm(C_ref))


def rel_max(C, C_ref) -> float:
    return float(np.max(np.abs(C - C_ref)) / np.max(np.abs(C_ref)))
