"""Emulated mixed-precision tile Cholesky (oracle side).

The paper's "Discussion and Future Work" section names the method: tiled
matrix algorithms in which tiles of one matrix are held at different
precisions (16, 32 and 64 bit).  This module writes that method out with the
textbook right-looking tile Cholesky (POTRF on the diagonal tile, TRSM on the
panel below it, SYRK/GEMM on the trailing tiles) and these readings:

* the tile map p(i, j) gives each lower tile its storage format; the diagonal
  tiles are FP64 (the diagonal POTRF, the log-determinant and the SYRK into the
  diagonal stay in FP64);
* Sigma's tiles are rounded ONCE from FP64 to their format before step 0;
* POTRF of A_kk in FP64; TRSM  A_ik <- round_{p(i,k)}(A_ik L_kk^{-T}) with the
  solve done in FP64 on the widened operands and one rounding at the end;
* SYRK  A_jj <- A_jj - L_jk L_jk^T in FP64;
* GEMM  A_ij <- round_p(A_ij - round_p(L_ik) round_p(L_jk)^T), p = p(i,j): the
  update runs in the output tile's format (operands converted to it on load),
  the product is accumulated exactly (FP64 model) and the result is rounded
  once to p;
* an FP8-E4M3 tile carries one power-of-two scale 2^s per tile, s from the
  largest magnitude of the values being rounded (the rule of the FP8 block
  scales of the GEMM); every rounding to FP8 above, of a tile or of an operand
  converted on load, chooses the scale from the tile it rounds;
* n that is not a multiple of nb is padded with an identity block, which
  leaves the log-determinant and the solution of the leading block unchanged.
"""
from __future__ import annotations

import numpy as np

from .dense import NotPositiveDefinite, cholesky_lower, forward_substitution
from .fpformat import CODE, FP8_E4M3, fmt_of, pow2_scale_exponent, round_to

FP64_CODE = CODE["fp64"]
FP8_CODE = CODE["fp8_e4m3"]
UNUSED = 255


def tile_scale_exponent(X: np.ndarray) -> int:
    """Exponent s of an FP8 tile's scale 2^s (the largest s with max|X| 2^s <= 448)."""
    return int(pow2_scale_exponent(np.max(np.abs(X)) if X.size else 0.0))


def round_tile(X: np.ndarray, code: int) -> np.ndarray:
    """A whole tile rounded to format `code`; FP8 tiles are decode(RNE(X 2^s)) 2^-s
    with their own scale exponent s."""
    if int(code) != FP8_CODE:
        return round_to(X, code)
    s = tile_scale_exponent(X)
    return np.ldexp(round_to(np.ldexp(X, s), FP8_E4M3), -s)


def num_tiles(n: int, nb: int) -> int:
    return (n + nb - 1) // nb


def tilemap_uniform(n: int, nb: int, fmt="fp64") -> np.ndarray:
    nt = num_tiles(n, nb)
    m = np.full((nt, nt), UNUSED, dtype=np.uint8)
    code = CODE[fmt_of(fmt).name]
    for i in range(nt):
        for j in range(i + 1):
            m[i, j] = FP64_CODE if i == j else code
    return m


def tilemap_banded(n: int, nb: int, bands) -> np.ndarray:
    """Map from bands [(d_max, fmt), ..., (None, fmt)]: tile (i, j), i >= j,
    with distance d = i - j gets the format of the first band whose d_max >= d.
    The diagonal (d = 0) must fall in an FP64 band."""
    nt = num_tiles(n, nb)
    m = np.full((nt, nt), UNUSED, dtype=np.uint8)
    for i in range(nt):
        for j in range(i + 1):
            d = i - j
            for dmax, f in bands:
                if dmax is None or d <= dmax:
                    m[i, j] = CODE[fmt_of(f).name]
                    break
    if any(m[i, i] != FP64_CODE for i in range(nt)):
        raise ValueError("diagonal tiles must be FP64")
    return m


def pad_identity(A: np.ndarray, N: int) -> np.ndarray:
    n = A.shape[0]
    P = np.eye(N)
    P[:n, :n] = A
    return P


def flops_by_format(nt: int, nb: int, tmap: np.ndarray) -> dict:
    """Algorithmic flops of the tile factorisation split by the format the
    step computes in: POTRF nb^3/3, TRSM nb^3, SYRK nb^3 (all FP64), GEMM
    2 nb^3 in the output tile's format."""
    out = {}
    def add(code, v):
        out[code] = out.get(code, 0.0) + v
    for k in range(nt):
        add(FP64_CODE, nb ** 3 / 3.0)
        for i in range(k + 1, nt):
            add(FP64_CODE, float(nb) ** 3)        # TRSM
            add(FP64_CODE, float(nb) ** 3)        # SYRK into (i, i)
            for j in range(k + 1, i):
                add(int(tmap[i, j]), 2.0 * nb ** 3)
    return out


def tile_cholesky_emulated(Sigma: np.ndarray, nb: int, tmap: np.ndarray):
    """Returns dict(L, info, N) where L is the N x N lower factor (padded size)
    holding the stored tile values widened to float64; info is 0 or the 1-based
    global column of the first non-positive pivot."""
    n = Sigma.shape[0]
    nt = num_tiles(n, nb)
    N = nt * nb
    A = pad_identity(np.asarray(Sigma, dtype=np.float64), N)
    T = lambda i, j: (slice(i * nb, (i + 1) * nb), slice(j * nb, (j + 1) * nb))
    p = lambda i, j: int(tmap[i, j])
    for i in range(nt):
        if p(i, i) != FP64_CODE:
            raise ValueError("diagonal tiles must be FP64")
        for j in range(i):
            A[T(i, j)] = round_tile(A[T(i, j)], p(i, j))
    for k in range(nt):
        try:
            Lkk = cholesky_lower(A[T(k, k)])
        except NotPositiveDefinite as e:
            return dict(L=np.tril(A), info=k * nb + e.info, N=N)
        A[T(k, k)] = Lkk
        for i in range(k + 1, nt):
            # X L_kk^T = A_ik  <=>  L_kk X^T = A_ik^T
            X = forward_substitution(Lkk, A[T(i, k)].T).T
            A[T(i, k)] = round_tile(X, p(i, k))
        for j in range(k + 1, nt):
            Ljk = A[T(j, k)]
            A[T(j, j)] = A[T(j, j)] - Ljk @ Ljk.T
            for i in range(j + 1, nt):
                f = p(i, j)
                upd = round_tile(A[T(i, k)], f) @ round_tile(Ljk, f).T
                A[T(i, j)] = round_tile(A[T(i, j)] - upd, f)
    return dict(L=np.tril(A), info=0, N=N)


# ---------------------------------------------------------------------------
# Norm-guarded tile map and promotion after a breakdown (readings of the
# Discussion section's tiled multi-precision method together with the MLE
# section's warning that low precision fails on ill-conditioned covariances).
# ---------------------------------------------------------------------------

# Each format's next finer format when a tile has to be promoted.
PROMOTE_TO = {CODE["fp8_e4m3"]: CODE["fp16"], CODE["fp16"]: CODE["fp32"], CODE["bf16"]: CODE["fp32"],
              CODE["fp32"]: FP64_CODE, FP64_CODE: FP64_CODE}


def tile_amax(Sigma: np.ndarray, nb: int) -> np.ndarray:
    """nt x nt array: the largest |Sigma_ij| of every lower tile (i >= j, the
    last tile row/column cut at n); 0 above the diagonal."""
    n = Sigma.shape[0]
    nt = num_tiles(n, nb)
    out = np.zeros((nt, nt))
    for i in range(nt):
        for j in range(i + 1):
            out[i, j] = np.max(np.abs(Sigma[i * nb:min((i + 1) * nb, n), j * nb:min((j + 1) * nb, n)]))
    return out


def rounding_bound(code: int, amax: float) -> float:
    """Largest absolute error of rounding values of magnitude <= amax to the
    format: max(u amax, half the smallest subnormal).  An FP8 tile carries its
    own power-of-two scale, so only the relative term applies to it."""
    f = fmt_of(int(code))
    if f.name == "fp64":
        return f.unit_roundoff * amax
    rel = f.unit_roundoff * amax
    if f.name == "fp8_e4m3":
        return rel
    return max(rel, 2.0 ** (f.emin - f.mbits - 1))


def tilemap_guarded(banded: np.ndarray, amax: np.ndarray, guard: float) -> np.ndarray:
    """Each off-diagonal tile keeps its banded format p if rounding_bound(p,
    max|tile|) <= guard; otherwise it climbs PROMOTE_TO until the bound holds
    (FP64 always does)."""
    nt = banded.shape[0]
    out = np.full((nt, nt), UNUSED, dtype=np.uint8)
    for i in range(nt):
        for j in range(i + 1):
            p = int(banded[i, j])
            while p != FP64_CODE and rounding_bound(p, float(amax[i, j])) > guard:
                p = PROMOTE_TO[p]
            out[i, j] = p
    return out


def promote_after_breakdown(tmap: np.ndarray, nb: int, info: int) -> np.ndarray:
    """The map to refactor with after a breakdown at global column `info`
    (1-based).  The pivot of tile step k = (info-1)//nb depends on the leading
    (k+1) x (k+1) tiles; let p be the coarsest format among them and d_fail
    the smallest tile distance i - j at which p occurs there.  Every tile of
    the whole map with format p and distance >= d_fail moves one format up
    (PROMOTE_TO).  Returns the map unchanged when the leading block is all
    FP64 (nothing left to promote)."""
    nt = tmap.shape[0]
    k = (int(info) - 1) // nb
    rank = {CODE["fp8_e4m3"]: 0, CODE["fp16"]: 1, CODE["bf16"]: 1, CODE["fp32"]: 2, FP64_CODE: 3}
    lead = [(i, j, int(tmap[i, j])) for i in range(k + 1) for j in range(i)]
    low = [t for t in lead if t[2] != FP64_CODE]
    out = tmap.copy()
    if not low:
        return out
    r = min(rank[p] for _, _, p in low)
    coarse = {p for _, _, p in low if rank[p] == r}
    d_fail = min(i - j for i, j, p in low if p in coarse)
    for i in range(nt):
        for j in range(i):
            if int(tmap[i, j]) in coarse and i - j >= d_fail:
                out[i, j] = PROMOTE_TO[int(tmap[i, j])]
    return out
