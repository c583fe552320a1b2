// Tile triangular solves, FP64 residuals and the refinement vector kernels.
//
// Forward solve L W = B and backward solve L^T X = W over the tile factor (the
// paper's forwardsolve / backsolve pair of the MLE section), with the inverted
// FP64 diagonal tiles (each stored by rows, i.e. Linv_kk^T in column-major order):
//   forward,  k = 0 .. nt-1:  W_k = Linv_kk R_k ;  R_i -= L_ik W_k   (i > k)
//   backward, k = nt-1 .. 0:  X_k = Linv_kk^T V_k ; V_i -= L_ki^T X_k (i < k)
// Off-diagonal tiles are read in their storage format and widened to FP64.
// All right-hand-side blocks are column-major with leading dimension ld >= the
// padded order nt*nb; padded rows are kept at zero.
#include "mpcr_internal.h"

namespace mpcr {

constexpr int RHS_CHUNK = 16;

typedef double d4 __attribute__((ext_vector_type(4)));

template <int F>
__device__ __forceinline__ double ldw(const void* p, int64_t i) {
  if constexpr (F == F64) return ((const double*)p)[i];
  else if constexpr (F == F32) return (double)((const float*)p)[i];
  else if constexpr (F == F16) return (double)f16_to_f32(((const uint16_t*)p)[i]);
  else if constexpr (F == BF16) return (double)bf16_to_f32(((const uint16_t*)p)[i]);
  else return (double)e4m3_to_f32(((const uint8_t*)p)[i]);
}

// The tile products of the solves and residuals are small GEMMs (nb x nb times
// nb x 16 right-hand sides) done with FP64 MFMA 16x16x4.  They sit on the
// sequential chain of the sweeps, so they are organised for latency: one
// workgroup owns 16 output rows, its SW waves split the contraction into
// equal parts and add their 16 x 16 partial products through LDS in a fixed
// order.  Both operands are read straight from memory (the tile widened to
// FP64 on load), eight k4 steps per batch with the next batch's loads issued
// before the current batch's MFMAs.  Lane l supplies A[row = l % 16][k = l / 16]
// and B[k = l / 16][c = l % 16]; the result lane l, register r is
// D[l / 16 + 4 r][l % 16].
constexpr int MB = 8;  // k4 steps per batch
constexpr int SW = 8;  // waves per workgroup of the tile products (each nb / SW of the contraction)
constexpr int STHREADS = 64 * SW;
constexpr int SW4 = 8;  // waves per workgroup of the wide update products

// Raw storage element of a tile format and its widening to FP64: the wide
// update loop holds its prefetched tile values in the storage width and widens
// them at the MFMA, which keeps the narrow formats' register footprint small.
template <int F> struct RawOf { using T = double; };
template <> struct RawOf<F32> { using T = float; };
template <> struct RawOf<F16> { using T = uint16_t; };
template <> struct RawOf<BF16> { using T = uint16_t; };
template <> struct RawOf<F8> { using T = uint8_t; };
template <int F>
__device__ __forceinline__ typename RawOf<F>::T ldraw(const void* p, int64_t i) {
  return ((const typename RawOf<F>::T*)p)[i];
}
template <int F>
__device__ __forceinline__ double widen(typename RawOf<F>::T v, double mul) {
  if constexpr (F == F64) return v;
  else if constexpr (F == F32) return (double)v;
  else if constexpr (F == F16) return (double)f16_to_f32(v);
  else if constexpr (F == BF16) return (double)bf16_to_f32(v);
  else return (double)e4m3_to_f32(v) * mul;  // FP8 tiles hold codes of v 2^s
}

// N consecutive stored elements M[idx .. idx+N) with one vector load (idx a
// multiple of N).
template <int F, int N>
__device__ __forceinline__ void ldrow(const void* M, int64_t idx, typename RawOf<F>::T (&out)[N]) {
  using RT = typename RawOf<F>::T;
  typedef RT VT __attribute__((ext_vector_type(N)));
  const VT v = *(const VT*)((const RT*)M + idx);
#pragma unroll
  for (int i = 0; i < N; ++i) out[i] = v[i];
}

// acc0/acc1 += op(M)[row, k0 .. k1) * V[k0 .. k1, c], op(M)[row][k] = M[k * ldm + row]
// (TRANS false) or M[row * ldm + k] (TRANS true); V is this lane's column of
// the right-hand side (element k at V[k * vsk]; NULL: zero).  k0 and k1 are
// multiples of 16; the k4 steps of a batch past k1 read nothing and multiply
// zeros.  Which k a lane group supplies at which k4 step is free (A and B
// agree): TRANS false, group q takes k = kk + 4u + q at step u (the 16 lanes
// of a group read 16 consecutive rows of a column); TRANS true with FP64
// tiles (the inverted diagonal tiles), group q takes the runs of four k from
// kk + 4q and kk + 16 + 4q (each lane reads a run of its row with one vector
// load); the other formats of the short update launches keep the first order,
// which holds their loop within 128 VGPRs.
template <int F, bool TRANS>
__device__ __forceinline__ void mfma_span(const void* M, int64_t ldm, int64_t row, int k0, int k1, const double* V,
                                          int64_t vsk, int lane, d4& acc0, d4& acc1, double mul = 1.0) {
  const int q = lane >> 4;
  double a[MB], b[MB], an[MB], bn[MB];
  auto load = [&](int kk, double* da, double* db) {
    if constexpr (TRANS && F == F64) {
#pragma unroll
      for (int g = 0; g < MB / 4; ++g) {
        const int64_t kb = kk + 16 * g + 4 * q;
        const bool in = kk + 16 * g < k1;
        typename RawOf<F>::T raw[4];
        if (in) ldrow<F, 4>(M, row * ldm + kb, raw);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          da[4 * g + u] = in ? widen<F>(raw[u], mul) : 0.0;
          db[4 * g + u] = (V && in) ? V[(kb + u) * vsk] : 0.0;
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < MB; ++u) {
        const int64_t k = kk + 4 * u + q;
        const bool in = kk + 4 * u < k1;
        da[u] = !in ? 0.0 : TRANS ? ldw<F>(M, row * ldm + k) : ldw<F>(M, k * ldm + row);
        if constexpr (F == F8) da[u] *= mul;  // FP8 tiles hold codes of v 2^s
        db[u] = (V && in) ? V[k * vsk] : 0.0;
      }
    }
  };
  load(k0, a, b);
  for (int kk = k0; kk < k1; kk += 4 * MB) {
    const bool more = kk + 4 * MB < k1;
    if (more) load(kk + 4 * MB, an, bn);
#pragma unroll
    for (int u = 0; u < MB; u += 2) {
      acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u + 1], b[u + 1], acc1, 0, 0, 0);
    }
    if (more) {
#pragma unroll
      for (int u = 0; u < MB; ++u) {
        a[u] = an[u];
        b[u] = bn[u];
      }
    }
  }
}

// out[r0 .. r0+15][c] (op)= sum_k op(M)[r0 + .., k] V[k][c] over one nb x nb tile M
// (format F, column-major); V[k][c] at V[k * vsk + c * vsc]; mode 0:
// out = product, mode 1: out -= product.  With copy (mode 0), the result is
// also written by rows: copy[row * nrhs + c].
template <int F, bool TRANS>
__device__ void tile_mfma(const void* M, int nb, int r0, const double* V, int64_t vsc, int64_t vsk, double* out,
                          int64_t ldo, int nrhs, int mode, double (*red)[16][17], double mul = 1.0,
                          double* copy = nullptr) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int q = lane >> 4, c = lane & 15;
  const int kw = nb / SW;
  // one 16-column chunk of right-hand sides per workgroup row of the grid
  for (int c0 = blockIdx.y * RHS_CHUNK; c0 < nrhs && c0 < (int)(blockIdx.y + 1) * RHS_CHUNK; c0 += RHS_CHUNK) {
    const int nc = (nrhs - c0) < RHS_CHUNK ? (nrhs - c0) : RHS_CHUNK;
    d4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    mfma_span<F, TRANS>(M, nb, r0 + c, w * kw, (w + 1) * kw, c < nc ? V + (int64_t)(c0 + c) * vsc : nullptr, vsk,
                        lane, acc0, acc1, mul);
#pragma unroll
    for (int r = 0; r < 4; ++r) red[w][q + 4 * r][c] = acc0[r] + acc1[r];
    __syncthreads();
    if (w == 0 && c < nc) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = q + 4 * r;
        double v = red[0][rr][c];
#pragma unroll
        for (int x = 1; x < SW; ++x) v += red[x][rr][c];
        double* o = out + (int64_t)(c0 + c) * ldo + r0 + rr;
        *o = mode == 0 ? v : *o - v;
        if (copy) copy[(int64_t)(r0 + rr) * nrhs + c0 + c] = v;
      }
    }
    __syncthreads();
  }
}

template <bool TRANS>
__device__ void tile_mfma_any(const void* M, int f, double mul, int nb, int r0, const double* V, int64_t vsc,
                              int64_t vsk, double* out, int64_t ldo, int nrhs, int mode, double (*red)[16][17]) {
  switch (f) {
    case F64: tile_mfma<F64, TRANS>(M, nb, r0, V, vsc, vsk, out, ldo, nrhs, mode, red); break;
    case F32: tile_mfma<F32, TRANS>(M, nb, r0, V, vsc, vsk, out, ldo, nrhs, mode, red); break;
    case F16: tile_mfma<F16, TRANS>(M, nb, r0, V, vsc, vsk, out, ldo, nrhs, mode, red); break;
    case BF16: tile_mfma<BF16, TRANS>(M, nb, r0, V, vsc, vsk, out, ldo, nrhs, mode, red); break;
    default: tile_mfma<F8, TRANS>(M, nb, r0, V, vsc, vsk, out, ldo, nrhs, mode, red, mul); break;
  }
}

// Wide variant for the update launches with many tiles: one workgroup owns 64
// output rows (four 16-row blocks that share each right-hand-side value it
// loads), its SW4 waves split the contraction into equal parts.
template <int F, bool TRANS>
__device__ __forceinline__ void mfma_span4(const void* M, int64_t ldm, int64_t row0, int k0, int k1, const double* V,
                                           int64_t vsk, int lane, d4 (&acc)[4], double mul) {
  // k4 steps per batch; the transposed loads take runs of U (one vector per
  // row: 16 bytes for FP64, 8 for FP32 and the 16-bit formats, 4 for FP8)
  constexpr int U = (F == F64 || (TRANS && F == F32)) ? 2 : 4;
  using RT = typename RawOf<F>::T;
  const int q = lane >> 4;
  RT a[4][U], an[4][U];
  double b[U], bn[U];
  auto load = [&](int kk, RT (*da)[U], double* db) {
    if constexpr (TRANS) {
      // group q takes the U consecutive k from kk + U q (k0, k1 multiples of 16)
      const int64_t kb = kk + U * q;
      const bool in = kb < k1;
#pragma unroll
      for (int h = 0; h < 4; ++h) {
        if (in) ldrow<F, U>(M, (row0 + 16 * h) * ldm + kb, da[h]);
        else {
#pragma unroll
          for (int u = 0; u < U; ++u) da[h][u] = RT(0);
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) db[u] = (V && in) ? V[(kb + u) * vsk] : 0.0;
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t k = kk + 4 * u + q;
        const bool in = kk + 4 * u < k1;
#pragma unroll
        for (int h = 0; h < 4; ++h) da[h][u] = !in ? RT(0) : ldraw<F>(M, k * ldm + row0 + 16 * h);
        db[u] = (V && in) ? V[k * vsk] : 0.0;
      }
    }
  };
  load(k0, a, b);
  for (int kk = k0; kk < k1; kk += 4 * U) {
    const bool more = kk + 4 * U < k1;
    if (more) load(kk + 4 * U, an, bn);
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int h = 0; h < 4; ++h)
        acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(widen<F>(a[h][u], mul), b[u], acc[h], 0, 0, 0);
    if (more) {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        b[u] = bn[u];
#pragma unroll
        for (int h = 0; h < 4; ++h) a[h][u] = an[h][u];
      }
    }
  }
}

// out[r0 .. r0+63][c] -= sum_k op(M)[r0 + .., k] V[k][c]; V[k][c] at V[k * vsk + c * vsc];
// the waves' partial products are added in a fixed order
template <int F, bool TRANS>
__device__ void tile_mfma4(const void* M, int nb, int r0, const double* V, int64_t vsc, int64_t vsk, double* out,
                           int64_t ldo, int nrhs, double (*red)[64][17], double mul) {
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int q = lane >> 4, c = lane & 15;
  const int kw = nb / SW4;
  for (int c0 = blockIdx.y * RHS_CHUNK; c0 < nrhs && c0 < (int)(blockIdx.y + 1) * RHS_CHUNK; c0 += RHS_CHUNK) {
    const int nc = (nrhs - c0) < RHS_CHUNK ? (nrhs - c0) : RHS_CHUNK;
    d4 acc[4];
#pragma unroll
    for (int h = 0; h < 4; ++h) acc[h] = d4{0, 0, 0, 0};
    mfma_span4<F, TRANS>(M, nb, r0 + c, w * kw, (w + 1) * kw, c < nc ? V + (int64_t)(c0 + c) * vsc : nullptr, vsk,
                         lane, acc, mul);
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[w][16 * h + q + 4 * r][c] = acc[h][r];
    __syncthreads();
    for (int e = tid; e < 64 * RHS_CHUNK; e += 64 * SW4) {
      const int rr = e % 64, cc = e / 64;
      if (cc < nc) {
        double v = red[0][rr][cc];
#pragma unroll
        for (int x = 1; x < SW4; ++x) v += red[x][rr][cc];
        out[(int64_t)(c0 + cc) * ldo + r0 + rr] -= v;
      }
    }
    __syncthreads();
  }
}

template <bool TRANS>
__device__ void tile_mfma4_any(const void* M, int f, double mul, int nb, int r0, const double* V, int64_t vsc,
                               int64_t vsk, double* out, int64_t ldo, int nrhs, double (*red)[64][17]) {
  switch (f) {
    case F64: tile_mfma4<F64, TRANS>(M, nb, r0, V, vsc, vsk, out, ldo, nrhs, red, mul); break;
    case F32: tile_mfma4<F32, TRANS>(M, nb, r0, V, vsc, vsk, out, ldo, nrhs, red, mul); break;
    case F16: tile_mfma4<F16, TRANS>(M, nb, r0, V, vsc, vsk, out, ldo, nrhs, red, mul); break;
    case BF16: tile_mfma4<BF16, TRANS>(M, nb, r0, V, vsc, vsk, out, ldo, nrhs, red, mul); break;
    default: tile_mfma4<F8, TRANS>(M, nb, r0, V, vsc, vsk, out, ldo, nrhs, red, mul); break;
  }
}

// Each step solves one block (diag kernel) and then updates the rest (update
// kernel).  The update kernels hold every tile format's loop; they are held to
// 128 VGPRs so that two 512-thread workgroups fit on a CU (with 156 VGPRs only
// one did, which halved their bandwidth).  The diag kernel also writes the solved block by rows into stage
// (nb x nrhs, row stride nrhs), which the update kernel reads as its
// right-hand side: lanes then read whole rows of 16 values.

// one workgroup per 16 output rows
__global__ __launch_bounds__(STHREADS) void k_fwd_diag(int nb, const double* Linv, int k, const double* R, double* W,
                                                       int64_t ld, int nrhs, const int* info, double* stage) {
  if (*info) return;
  __shared__ double red[SW][16][17];
  const int64_t off = (int64_t)k * nb;
  tile_mfma<F64, true>(Linv + (int64_t)k * nb * nb, nb, blockIdx.x * 16, R + off, ld, 1, W + off, ld, nrhs, 0, red, 1.0,
                       stage);
}

__global__ __launch_bounds__(STHREADS) __attribute__((amdgpu_waves_per_eu(4))) void k_fwd_update(TileView tv, int k, double* R, const double* stage,
                                                         int64_t ld, int nrhs) {
  if (*tv.info) return;
  __shared__ double red[SW][16][17];
  const int nb = tv.nb, rb = nb / 16;
  const int i = k + 1 + blockIdx.x / rb;
  tile_mfma_any<false>(tv.tile(i, k), tv.tfmt(i, k), tv.tmul(i, k), nb, (blockIdx.x % rb) * 16, stage, 1, nrhs,
                       R + (int64_t)i * nb, ld, nrhs, 1, red);
}

// X_k = Linv_kk^T V_k: the stored (row-major) inverse read as column-major
__global__ __launch_bounds__(STHREADS) void k_bwd_diag(int nb, const double* Linv, int k, const double* V, double* X,
                                                       int64_t ld, int nrhs, const int* info, double* stage) {
  if (*info) return;
  __shared__ double red[SW][16][17];
  const int64_t off = (int64_t)k * nb;
  tile_mfma<F64, false>(Linv + (int64_t)k * nb * nb, nb, blockIdx.x * 16, V + off, ld, 1, X + off, ld, nrhs, 0, red,
                        1.0, stage);
}

__global__ __launch_bounds__(STHREADS) __attribute__((amdgpu_waves_per_eu(4))) void k_bwd_update(TileView tv, int k, double* V, const double* stage,
                                                         int64_t ld, int nrhs) {
  if (*tv.info) return;
  __shared__ double red[SW][16][17];
  const int nb = tv.nb, rb = nb / 16;
  const int i = blockIdx.x / rb;  // i < k
  tile_mfma_any<true>(tv.tile(k, i), tv.tfmt(k, i), tv.tmul(k, i), nb, (blockIdx.x % rb) * 16, stage, 1, nrhs,
                      V + (int64_t)i * nb, ld, nrhs, 1, red);
}

__global__ __launch_bounds__(64 * SW4) __attribute__((amdgpu_waves_per_eu(4))) void k_fwd_update4(TileView tv, int k, double* R, const double* stage, int64_t ld,
                                                     int nrhs) {
  if (*tv.info) return;
  __shared__ double red[SW4][64][17];
  const int nb = tv.nb, rb = nb / 64;
  const int i = k + 1 + blockIdx.x / rb;
  tile_mfma4_any<false>(tv.tile(i, k), tv.tfmt(i, k), tv.tmul(i, k), nb, (blockIdx.x % rb) * 64, stage, 1, nrhs,
                        R + (int64_t)i * nb, ld, nrhs, red);
}

__global__ __launch_bounds__(64 * SW4) __attribute__((amdgpu_waves_per_eu(4))) void k_bwd_update4(TileView tv, int k, double* V, const double* stage, int64_t ld,
                                                     int nrhs) {
  if (*tv.info) return;
  __shared__ double red[SW4][64][17];
  const int nb = tv.nb, rb = nb / 64;
  const int i = blockIdx.x / rb;  // i < k
  tile_mfma4_any<true>(tv.tile(k, i), tv.tfmt(k, i), tv.tmul(k, i), nb, (blockIdx.x % rb) * 64, stage, 1, nrhs,
                       V + (int64_t)i * nb, ld, nrhs, red);
}

constexpr int WIDE_MIN_TILES = 16;  // update launches over at least this many tiles use 64-row workgroups
static unsigned nchunk(int nrhs) { return (unsigned)((nrhs + RHS_CHUNK - 1) / RHS_CHUNK); }

hipError_t launch_fwd_diag(const TileView& tv, const double* Linv, int k, double* R, double* W, int64_t ld,
                           int nrhs, double* stage, hipStream_t s) {
  k_fwd_diag<<<dim3(tv.nb / 16, nchunk(nrhs)), STHREADS, 0, s>>>(tv.nb, Linv, k, R, W, ld, nrhs, tv.info, stage);
  return hipGetLastError();
}
hipError_t launch_fwd_update(const TileView& tv, int k, double* R, const double* stage, int64_t ld, int nrhs,
                             hipStream_t s) {
  int nt = tv.nt - k - 1;
  if (nt <= 0) return hipSuccess;
  if (nt >= WIDE_MIN_TILES)
    k_fwd_update4<<<dim3(nt * (tv.nb / 64), nchunk(nrhs)), 64 * SW4, 0, s>>>(tv, k, R, stage, ld, nrhs);
  else
    k_fwd_update<<<dim3(nt * (tv.nb / 16), nchunk(nrhs)), STHREADS, 0, s>>>(tv, k, R, stage, ld, nrhs);
  return hipGetLastError();
}
hipError_t launch_bwd_diag(const TileView& tv, const double* Linv, int k, double* V, double* X, int64_t ld,
                           int nrhs, double* stage, hipStream_t s) {
  k_bwd_diag<<<dim3(tv.nb / 16, nchunk(nrhs)), STHREADS, 0, s>>>(tv.nb, Linv, k, V, X, ld, nrhs, tv.info, stage);
  return hipGetLastError();
}
hipError_t launch_bwd_update(const TileView& tv, int k, double* V, const double* stage, int64_t ld, int nrhs,
                             hipStream_t s) {
  if (k <= 0) return hipSuccess;
  if (k >= WIDE_MIN_TILES)
    k_bwd_update4<<<dim3(k * (tv.nb / 64), nchunk(nrhs)), 64 * SW4, 0, s>>>(tv, k, V, stage, ld, nrhs);
  else
    k_bwd_update<<<dim3(k * (tv.nb / 16), nchunk(nrhs)), STHREADS, 0, s>>>(tv, k, V, stage, ld, nrhs);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 residual R = B - Sigma X over the first n rows (matrix-free: Sigma's
// entries regenerated from the sites), and ||Sigma||_inf row sums.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double matern_corr_s(double x, int nuc) {
  double e = exp(-x);
  if (nuc == 0) return e;
  if (nuc == 1) return (1.0 + x) * e;
  return (1.0 + x + x * x / 3.0) * e;
}

static int nu_code_s(double nu) { return nu == 0.5 ? 0 : (nu == 1.5 ? 1 : 2); }

// One workgroup per 64 rows; thread (r, q) sums columns q, q+4, ... of each
// 256-column chunk; the four partials are combined in a fixed order.
// MODE 0: R = B - Sigma X (B == NULL: R = -Sigma X) ; MODE 1: R[:,0] = sum_c |Sigma_rc|.
// DENSE: Sigma read from the FP64 matrix A instead of regenerated from the sites.
template <int MODE, bool DENSE>
__global__ __launch_bounds__(256) void k_sigma_apply(int n, const double* locs, double s2, double range, int nuc,
                                                     double nugget, const double* A, int64_t lda, const double* B,
                                                     const double* X, double* R, int64_t ld, int nrhs,
                                                     double* rowsum) {
  constexpr int CC = 256;
  __shared__ double Ls[2][CC];
  __shared__ double Xs[CC * RHS_CHUNK];
  __shared__ double part[4][64][RHS_CHUNK + 1];  // [.][.][RHS_CHUNK]: |Sigma| row sums
  const int tid = threadIdx.x, r = tid & 63, q = tid >> 6;
  const int row = blockIdx.x * 64 + r;
  const bool live = row < n;
  double px = 0, py = 0;
  if (!DENSE && live) { px = locs[row]; py = locs[n + row]; }
  const int ncol = MODE == 1 ? 1 : nrhs;
  for (int c0 = 0; c0 < ncol; c0 += RHS_CHUNK) {
    double acc[RHS_CHUNK];
    double asum = 0.0;  // sum_c |Sigma_rc| when rowsum is requested (first chunk only)
#pragma unroll
    for (int j = 0; j < RHS_CHUNK; ++j) acc[j] = 0.0;
    for (int k0 = 0; k0 < n; k0 += CC) {
      __syncthreads();
      for (int e = tid; e < CC; e += 256) {
        int c = k0 + e;
        if (!DENSE) {
          Ls[0][e] = c < n ? locs[c] : 0.0;
          Ls[1][e] = c < n ? locs[n + c] : 0.0;
        }
      }
      if (MODE == 0)
        for (int e = tid; e < CC * RHS_CHUNK; e += 256) {
          int kk = e % CC, j = e / CC;
          Xs[kk * RHS_CHUNK + j] = (k0 + kk < n && c0 + j < nrhs) ? X[(int64_t)(c0 + j) * ld + k0 + kk] : 0.0;
        }
      __syncthreads();
      if (live) {
        const int kend = (n - k0) < CC ? (n - k0) : CC;
        for (int kk = q; kk < kend; kk += 4) {
          const int col = k0 + kk;
          double sv;
          if (DENSE) {
            sv = A[(int64_t)col * lda + row];
          } else {
            double dx = px - Ls[0][kk], dy = py - Ls[1][kk];
            sv = s2 * matern_corr_s(sqrt(dx * dx + dy * dy) / range, nuc);
            if (col == row) sv += nugget;
          }
          if (MODE == 1) {
            acc[0] += fabs(sv);
          } else {
            asum += fabs(sv);
#pragma unroll
            for (int j = 0; j < RHS_CHUNK; ++j) acc[j] += sv * Xs[kk * RHS_CHUNK + j];
          }
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < RHS_CHUNK; ++j) part[q][r][j] = acc[j];
    part[q][r][RHS_CHUNK] = asum;
    __syncthreads();
    if (MODE == 0 && rowsum && c0 == 0 && tid < 64 && blockIdx.x * 64 + tid < n)
      rowsum[blockIdx.x * 64 + tid] = ((part[0][tid][RHS_CHUNK] + part[1][tid][RHS_CHUNK]) + part[2][tid][RHS_CHUNK]) +
                                      part[3][tid][RHS_CHUNK];
    for (int e = tid; e < 64 * RHS_CHUNK; e += 256) {
      int rr = e % 64, j = e / 64;
      int grow = blockIdx.x * 64 + rr, c = c0 + j;
      if (grow < n && c < ncol) {
        double s = ((part[0][rr][j] + part[1][rr][j]) + part[2][rr][j]) + part[3][rr][j];
        if (MODE == 1)
          R[grow] = s;
        else
          R[(int64_t)c * ld + grow] = (B ? B[(int64_t)c * ld + grow] : 0.0) - s;
      }
    }
  }
}

hipError_t launch_residual_cov(int n, const double* locs, const mpcr_theta_t& th, const double* B, const double* X,
                               double* R, int64_t ld, int nrhs, hipStream_t s, double* rowsum) {
  if (n == 0) return hipSuccess;
  k_sigma_apply<0, false><<<(n + 63) / 64, 256, 0, s>>>(n, locs, th.sigma2, th.range, nu_code_s(th.nu), th.nugget,
                                                        nullptr, 0, B, X, R, ld, nrhs, rowsum);
  return hipGetLastError();
}
hipError_t launch_residual_dense(int n, const double* A, int64_t lda, const double* B, const double* X, double* R,
                                 int64_t ld, int nrhs, hipStream_t s, double* rowsum) {
  if (n == 0) return hipSuccess;
  k_sigma_apply<0, true><<<(n + 63) / 64, 256, 0, s>>>(n, nullptr, 0, 1, 0, 0, A, lda, B, X, R, ld, nrhs, rowsum);
  return hipGetLastError();
}
hipError_t launch_rowsum_abs_cov(int n, const double* locs, const mpcr_theta_t& th, double* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_sigma_apply<1, false><<<(n + 63) / 64, 256, 0, s>>>(n, locs, th.sigma2, th.range, nu_code_s(th.nu), th.nugget,
                                                        nullptr, 0, nullptr, nullptr, out, 0, 1, nullptr);
  return hipGetLastError();
}
hipError_t launch_rowsum_abs_dense(int n, const double* A, int64_t lda, double* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_sigma_apply<1, true><<<(n + 63) / 64, 256, 0, s>>>(n, nullptr, 0, 1, 0, 0, A, lda, nullptr, nullptr, out, 0, 1,
                                                       nullptr);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 residual from the stored lower tiles of Sigma, R = B - Sigma X.
// Streaming pass: one workgroup per stored tile (i, j), j <= i, reads the tile
// once (64 x 64 pieces staged through LDS, double-buffered, row of pieces by
// row of pieces) and forms both of its products with FP64 MFMA, 16
// right-hand sides per pass:
//   P[i][j] = S_ij X_j     wave w contracts over columns 16 w .. 16 w + 15 of
//                          each piece (4 values of X_j per lane and piece) for
//                          all 64 rows, accumulates along the row of pieces in
//                          registers and the four waves' sums are added in a
//                          fixed order at its end;
//   P[j][i] = S_ij^T X_i   (off the diagonal) wave w owns rows 16 w .. of the
//                          piece's columns, contracts over all 64 piece rows
//                          (X_i fixed along the row of pieces) and adds into
//                          the partial block in order of the piece rows; each
//                          element has one owner lane.
// With rowsum it also forms the |S| row and column sums.  A second kernel
// adds, for every row block a, B_a - sum_b P[a][b] in the order
// b = 0, 1, ..., nt-1 (and the row sums likewise), so results do not depend on
// scheduling.  Partials: nt x nt blocks of nb x 16 doubles, then nt x nt
// blocks of nb doubles for the row sums.
// ---------------------------------------------------------------------------
constexpr int RP = 64;        // rows / columns of a staged piece
constexpr int RPLD = RP + 2;  // LDS leading dimension (doubles) of a piece, [column][row]

__global__ __launch_bounds__(256) void k_residual_stream(int nb, int nt, const double* sig, const double* X, int64_t ld,
                                                         int c0, int nc, double* part, int want_sum) {
  __shared__ __attribute__((aligned(16))) double Sp[2][RP * RPLD];
  __shared__ double rn[RP][RHS_CHUNK + 1];  // the waves' P[i][j] sums of a row of pieces
  __shared__ double red[4][RP];
  int i = 0, rem = blockIdx.x;  // tile (i, j) from the packed lower index
  while (rem > i) { rem -= i + 1; ++i; }
  const int j = rem;
  const bool diag = i == j;
  const double* T = sig + (int64_t)blockIdx.x * nb * nb;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, q = lane >> 4, col = lane & 15;
  const int np = nb / RP;  // pieces per dimension (>= 2)
  const int64_t blk = (int64_t)nb * RHS_CHUNK;
  double* Pij = part + ((int64_t)i * nt + j) * blk;
  double* Pji = part + ((int64_t)j * nt + i) * blk;
  double* RSij = part + (int64_t)nt * nt * blk + ((int64_t)i * nt + j) * nb;
  double* RSji = part + (int64_t)nt * nt * blk + ((int64_t)j * nt + i) * nb;
  const bool cv = col < nc;
  const double* Xj = X + (int64_t)(c0 + (cv ? col : 0)) * ld + (int64_t)j * nb;
  const double* Xi = X + (int64_t)(c0 + (cv ? col : 0)) * ld + (int64_t)i * nb;

  // Requested one piece ahead: the piece itself (thread t: column t / 16 + 16 h,
  // rows 4 (t % 16) .. +3), this lane's X_j values for the piece's columns
  // 16 w .., the running transposed partial it adds to, and at the start of a
  // row of pieces that row's X_i values.
  double4 ld4[4];
  double xn[4], pold[4], xtn[RP / 4];
  auto prefetch = [&](int pr, int pc) {
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int c = tid / 16 + 16 * h, r = 4 * (tid % 16);
      ld4[h] = *(const double4*)(T + (int64_t)(RP * pc + c) * nb + RP * pr + r);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) xn[u] = cv ? Xj[RP * pc + 16 * w + 4 * u + q] : 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      pold[r] = (!diag && cv && pr > 0) ? Pji[(int64_t)col * nb + RP * pc + 16 * w + q + 4 * r] : 0.0;
    if (pc == 0) {
#pragma unroll
      for (int u = 0; u < RP / 4; ++u) xtn[u] = cv ? Xi[RP * pr + 4 * u + q] : 0.0;
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int c = tid / 16 + 16 * h, r = 4 * (tid % 16);
      double* d = &Sp[buf][c * RPLD + r];
      d[0] = ld4[h].x;
      d[1] = ld4[h].y;
      d[2] = ld4[h].z;
      d[3] = ld4[h].w;
    }
  };
  auto sum4 = [&](int r) { return ((red[0][r] + red[1][r]) + red[2][r]) + red[3][r]; };

  prefetch(0, 0);
  sstore(0);
  double cxn[4], cpold[4], cxt[RP / 4];
#pragma unroll
  for (int u = 0; u < 4; ++u) cxn[u] = xn[u];
#pragma unroll
  for (int u = 0; u < RP / 4; ++u) cxt[u] = xtn[u];
#pragma unroll
  for (int r = 0; r < 4; ++r) cpold[r] = pold[r];
  __syncthreads();
  int cur = 0;
#pragma unroll 1
  for (int pr = 0; pr < np; ++pr) {
    d4 accN[4];  // rows 64 pr + 16 a + .. of block i, this wave's quarter of the columns
#pragma unroll
    for (int a = 0; a < 4; ++a) accN[a] = d4{0, 0, 0, 0};
    double rs = 0.0;  // |S| row sums of row 64 pr + tid % 64 (columns tid / 64 + 4 m of each piece)
#pragma unroll 1
    for (int pc = 0; pc < np; ++pc) {
      const int nxt = pr * np + pc + 1;
      const bool more = nxt < np * np;
      if (more) prefetch(nxt / np, nxt % np);
      const double* S = Sp[cur];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int a = 0; a < 4; ++a)
          accN[a] = __builtin_amdgcn_mfma_f64_16x16x4f64(S[(16 * w + 4 * u + q) * RPLD + 16 * a + col], cxn[u], accN[a],
                                                         0, 0, 0);
      if (!diag) {  // rows 64 pc + 16 w + col of block j over the piece's rows, added to P[j][i] in order of pr
        d4 accT = {cpold[0], cpold[1], cpold[2], cpold[3]};
#pragma unroll
        for (int u = 0; u < RP / 4; ++u)
          accT = __builtin_amdgcn_mfma_f64_16x16x4f64(S[(16 * w + col) * RPLD + 4 * u + q], cxt[u], accT, 0, 0, 0);
        if (cv) {
#pragma unroll
          for (int r = 0; r < 4; ++r) Pji[(int64_t)col * nb + RP * pc + 16 * w + q + 4 * r] = accT[r];
        }
      }
      if (want_sum) {
        const int rr = tid % 64, g = tid / 64;
        double cs = 0.0;
        for (int m = g; m < RP; m += 4) {
          rs += fabs(S[m * RPLD + rr]);
          cs += fabs(S[rr * RPLD + m]);
        }
        if (!diag) {
          red[g][rr] = cs;
          __syncthreads();
          if (tid < RP) RSji[RP * pc + tid] = pr == 0 ? sum4(tid) : RSji[RP * pc + tid] + sum4(tid);
        }
      }
      if (more) {
        sstore(cur ^ 1);
#pragma unroll
        for (int u = 0; u < 4; ++u) cxn[u] = xn[u];
#pragma unroll
        for (int r = 0; r < 4; ++r) cpold[r] = pold[r];
        if (nxt % np == 0) {
#pragma unroll
          for (int u = 0; u < RP / 4; ++u) cxt[u] = xtn[u];
        }
      }
      __syncthreads();
      cur ^= 1;
    }
    // P[i][j] rows of this row of pieces: ((p3 + p2) + p1) + p0 through rn
#pragma unroll 1
    for (int s = 3; s >= 0; --s) {
      if (w == s) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int rr = 16 * a + q + 4 * r;
            const double v = s == 3 ? accN[a][r] : accN[a][r] + rn[rr][col];
            if (s > 0)
              rn[rr][col] = v;
            else if (cv)
              Pij[(int64_t)col * nb + RP * pr + rr] = v;
          }
      }
      __syncthreads();
    }
    if (want_sum) {
      red[tid / 64][tid % 64] = rs;
      __syncthreads();
      if (tid < RP) RSij[RP * pr + tid] = sum4(tid);
      __syncthreads();
    }
  }
}

// R[row, c0 + c] = B - sum_b P[a][b][row, c] (b in order); rowsum[row] = sum_b RS[a][b][row]
__global__ __launch_bounds__(256) void k_residual_reduce(int n, int nb, int nt, const double* part, const double* B,
                                                         double* R, int64_t ld, int c0, int nc, double* rowsum) {
  const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int row = (int)(g % n), c = (int)(g / n);
  if (c >= nc) return;
  const int a = row / nb, r = row % nb;
  const int64_t blk = (int64_t)nb * RHS_CHUNK;
  double v = 0.0;
  for (int b = 0; b < nt; ++b) v += part[((int64_t)a * nt + b) * blk + (int64_t)c * nb + r];
  const int64_t o = (int64_t)(c0 + c) * ld + row;
  R[o] = (B ? B[o] : 0.0) - v;
  if (rowsum && c == 0) {
    double t = 0.0;
    for (int b = 0; b < nt; ++b) t += part[(int64_t)nt * nt * blk + ((int64_t)a * nt + b) * nb + r];
    rowsum[row] = t;
  }
}

size_t residual_part_bytes(int nb, int nt) {
  return ((size_t)nt * nt * nb * RHS_CHUNK + (size_t)nt * nt * nb) * sizeof(double);
}

hipError_t launch_residual_tiles(int n, int nb, int nt, const double* sig64, const double* B, const double* X,
                                 double* R, int64_t ld, int nrhs, hipStream_t s, double* rowsum, double* part) {
  if (n == 0) return hipSuccess;
  if (nb % RP != 0 || nb < 2 * RP || part == nullptr) return hipErrorInvalidValue;
  const int ntiles = nt * (nt + 1) / 2;
  for (int c0 = 0; c0 < nrhs; c0 += RHS_CHUNK) {
    const int nc = (nrhs - c0) < RHS_CHUNK ? (nrhs - c0) : RHS_CHUNK;
    const int want = rowsum != nullptr && c0 == 0;
    k_residual_stream<<<ntiles, 256, 0, s>>>(nb, nt, sig64, X, ld, c0, nc, part, want);
    const int64_t total = (int64_t)n * nc;
    k_residual_reduce<<<(unsigned)((total + 255) / 256), 256, 0, s>>>(n, nb, nt, part, B, R, ld, c0, nc,
                                                                        want ? rowsum : nullptr);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// deterministic column reductions: stage 1 over fixed 1024-row slabs, stage 2
// sums the slabs in order
// ---------------------------------------------------------------------------
constexpr int SLAB = 1024;

__device__ __forceinline__ double block_sum(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  double s = red[0];
  __syncthreads();
  return s;
}
__device__ __forceinline__ double block_max(double v, double* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  double s = red[0];
  __syncthreads();
  return s;
}

// partial[slab][c] = sum over the slab of A[:,c] * B[:,c]
__global__ __launch_bounds__(256) void k_col_dot_1(int n, const double* A, const double* B, int64_t ld,
                                                   double* partial, int nslab) {
  __shared__ double red[256];
  const int slab = blockIdx.x, c = blockIdx.y;
  double s = 0.0;
  for (int r = slab * SLAB + threadIdx.x; r < n && r < (slab + 1) * SLAB; r += 256)
    s += A[(int64_t)c * ld + r] * B[(int64_t)c * ld + r];
  s = block_sum(s, red);
  if (threadIdx.x == 0) partial[(int64_t)c * nslab + slab] = s;
}
__global__ void k_col_sum_2(int nslab, int ncol, const double* partial, double* out) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  double s = 0.0;
  for (int i = 0; i < nslab; ++i) s += partial[(int64_t)c * nslab + i];
  out[c] = s;
}

hipError_t launch_col_dot(int n, int nrhs, const double* A, const double* B, int64_t ld, double* partial,
                          double* out, hipStream_t s) {
  int nslab = (n + SLAB - 1) / SLAB;
  if (nslab == 0) nslab = 1;
  k_col_dot_1<<<dim3(nslab, nrhs), 256, 0, s>>>(n, A, B, ld, partial, nslab);
  k_col_sum_2<<<(nrhs + 63) / 64, 64, 0, s>>>(nslab, nrhs, partial, out);
  return hipGetLastError();
}

// Per column: stats[c] = { ||R||_2^2, ||B||_2^2, max|R|, max|X|, max|B| } (5 x nrhs),
// then eta = max|R| / (sig_inf max|X| + max|B|), rel2 = ||R|| / ||B|| in stats[5 nrhs + 2c .. ].
__global__ __launch_bounds__(256) void k_col_stats_1(int n, const double* R, const double* X, const double* B,
                                                     int64_t ld, double* partial, int nslab) {
  __shared__ double red[256];
  const int slab = blockIdx.x, c = blockIdx.y;
  double rr = 0, bb = 0, mr = 0, mx = 0, mb = 0;
  for (int r = slab * SLAB + threadIdx.x; r < n && r < (slab + 1) * SLAB; r += 256) {
    double a = R[(int64_t)c * ld + r], x = X[(int64_t)c * ld + r], b = B[(int64_t)c * ld + r];
    rr += a * a;
    bb += b * b;
    mr = fmax(mr, fabs(a));
    mx = fmax(mx, fabs(x));
    mb = fmax(mb, fabs(b));
  }
  rr = block_sum(rr, red);
  bb = block_sum(bb, red);
  mr = block_max(mr, red);
  mx = block_max(mx, red);
  mb = block_max(mb, red);
  if (threadIdx.x == 0) {
    double* p = partial + ((int64_t)c * nslab + slab) * 5;
    p[0] = rr; p[1] = bb; p[2] = mr; p[3] = mx; p[4] = mb;
  }
}
__global__ void k_col_stats_2(int nslab, int ncol, const double* partial, const double* sig_inf, double* stats) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  double rr = 0, bb = 0, mr = 0, mx = 0, mb = 0;
  for (int i = 0; i < nslab; ++i) {
    const double* p = partial + ((int64_t)c * nslab + i) * 5;
    rr += p[0]; bb += p[1];
    mr = fmax(mr, p[2]); mx = fmax(mx, p[3]); mb = fmax(mb, p[4]);
  }
  double den = (*sig_inf) * mx + mb;
  stats[2 * c] = den > 0 ? mr / den : 0.0;               // eta
  stats[2 * c + 1] = bb > 0 ? sqrt(rr) / sqrt(bb) : 0.0;  // ||r||_2 / ||b||_2
}

hipError_t launch_col_stats(int n, int nrhs, const double* R, const double* X, const double* B, int64_t ld,
                            const double* sig_inf, double* partial, double* stats, hipStream_t s) {
  int nslab = (n + SLAB - 1) / SLAB;
  if (nslab == 0) nslab = 1;
  k_col_stats_1<<<dim3(nslab, nrhs), 256, 0, s>>>(n, R, X, B, ld, partial, nslab);
  k_col_stats_2<<<(nrhs + 63) / 64, 64, 0, s>>>(nslab, nrhs, partial, sig_inf, stats);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_max_1(int n, const double* v, double* partial) {
  __shared__ double red[256];
  double m = 0.0;
  for (int r = blockIdx.x * SLAB + threadIdx.x; r < n && r < (int)(blockIdx.x + 1) * SLAB; r += 256)
    m = fmax(m, v[r]);
  m = block_max(m, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = m;
}
__global__ void k_max_2(int nslab, const double* partial, double* out) {
  if (threadIdx.x != 0) return;
  double m = 0.0;
  for (int i = 0; i < nslab; ++i) m = fmax(m, partial[i]);
  *out = m;
}
hipError_t launch_max_reduce(int n, const double* v, double* partial, double* out, hipStream_t s) {
  int nslab = (n + SLAB - 1) / SLAB;
  if (nslab == 0) nslab = 1;
  k_max_1<<<nslab, 256, 0, s>>>(n, v, partial);
  k_max_2<<<1, 64, 0, s>>>(nslab, partial, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// elementwise helpers (columns of n x nrhs blocks, leading dimension ld)
// ---------------------------------------------------------------------------
__global__ void k_fill(double* p, int64_t count, double v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}
hipError_t launch_fill(double* p, int64_t count, double v, hipStream_t s) {
  if (count == 0) return hipSuccess;
  int64_t g = (count + 255) / 256;
  k_fill<<<(unsigned)(g < 4096 ? g : 4096), 256, 0, s>>>(p, count, v);
  return hipGetLastError();
}

__global__ void k_copy_cols(int n, const double* src, int64_t lds, double* dst, int64_t ldd) {
  const int c = blockIdx.y;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
    dst[(int64_t)c * ldd + r] = src[(int64_t)c * lds + r];
}
hipError_t launch_copy_cols(int n, int nrhs, const double* src, int64_t lds, double* dst, int64_t ldd,
                            hipStream_t s) {
  if (n == 0 || nrhs == 0) return hipSuccess;
  int g = (n + 255) / 256;
  k_copy_cols<<<dim3(g < 256 ? g : 256, nrhs), 256, 0, s>>>(n, src, lds, dst, ldd);
  return hipGetLastError();
}

// Y[:,c] += sign * alpha[c] * X[:,c]
__global__ void k_axpy_cols(int n, const double* alpha, double sign, const double* X, double* Y, int64_t ld) {
  const int c = blockIdx.y;
  const double a = sign * alpha[c];
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
    Y[(int64_t)c * ld + r] += a * X[(int64_t)c * ld + r];
}
hipError_t launch_axpy_cols(int n, int nrhs, const double* alpha, double sign, const double* X, double* Y,
                            int64_t ld, hipStream_t s) {
  if (n == 0 || nrhs == 0) return hipSuccess;
  int g = (n + 255) / 256;
  k_axpy_cols<<<dim3(g < 256 ? g : 256, nrhs), 256, 0, s>>>(n, alpha, sign, X, Y, ld);
  return hipGetLastError();
}

// Y[:,c] = X[:,c] + beta[c] * Y[:,c]
__global__ void k_xpby_cols(int n, const double* X, const double* beta, double* Y, int64_t ld) {
  const int c = blockIdx.y;
  const double b = beta[c];
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
    Y[(int64_t)c * ld + r] = X[(int64_t)c * ld + r] + b * Y[(int64_t)c * ld + r];
}
hipError_t launch_xpby_cols(int n, int nrhs, const double* X, const double* beta, double* Y, int64_t ld,
                            hipStream_t s) {
  if (n == 0 || nrhs == 0) return hipSuccess;
  int g = (n + 255) / 256;
  k_xpby_cols<<<dim3(g < 256 ? g : 256, nrhs), 256, 0, s>>>(n, X, beta, Y, ld);
  return hipGetLastError();
}

// PCG step sizes; columns that are not active get 0 (they stay frozen).
__global__ void k_pcg_alpha(int nrhs, const double* rz, const double* pq, const int* active, double* alpha) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  alpha[c] = (active[c] && pq[c] != 0.0) ? rz[c] / pq[c] : 0.0;
}
__global__ void k_pcg_beta(int nrhs, const double* rz_new, double* rz, const int* active, double* beta) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  double b = (active[c] && rz[c] != 0.0) ? rz_new[c] / rz[c] : 0.0;
  beta[c] = b;
  if (active[c]) rz[c] = rz_new[c];
}
hipError_t launch_pcg_alpha(int nrhs, const double* rz, const double* pq, const int* active, double* alpha,
                            hipStream_t s) {
  k_pcg_alpha<<<(nrhs + 63) / 64, 64, 0, s>>>(nrhs, rz, pq, active, alpha);
  return hipGetLastError();
}
hipError_t launch_pcg_beta(int nrhs, const double* rz_new, double* rz, const int* active, double* beta,
                           hipStream_t s) {
  k_pcg_beta<<<(nrhs + 63) / 64, 64, 0, s>>>(nrhs, rz_new, rz, active, beta);
  return hipGetLastError();
}

// l = -(n/2) log(2 pi) - logdet/2 - quad_c/2  (MLE section of the paper)
__global__ void k_loglik(int n, int nrhs, const double* logdet, const double* quad, double* out) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  out[c] = -0.5 * (double)n * log(2.0 * M_PI) - 0.5 * (*logdet) - 0.5 * quad[c];
}
hipError_t launch_loglik(int n, int nrhs, const double* logdet, const double* quad, double* out, hipStream_t s) {
  k_loglik<<<(nrhs + 63) / 64, 64, 0, s>>>(n, nrhs, logdet, quad, out);
  return hipGetLastError();
}

// quad_c = z_c^T x_c + x_c^T r_c
__global__ __launch_bounds__(256) void k_quad_1(int n, const double* Z, const double* X, const double* R, int64_t ld,
                                                double* partial, int nslab) {
  __shared__ double red[256];
  const int slab = blockIdx.x, c = blockIdx.y;
  double s = 0.0;
  for (int r = slab * SLAB + threadIdx.x; r < n && r < (slab + 1) * SLAB; r += 256) {
    double x = X[(int64_t)c * ld + r];
    s += Z[(int64_t)c * ld + r] * x + x * R[(int64_t)c * ld + r];
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) partial[(int64_t)c * nslab + slab] = s;
}
hipError_t launch_quad_refined(int n, int nrhs, const double* Z, const double* X, const double* R, int64_t ld,
                               double* partial, double* quad, hipStream_t s) {
  int nslab = (n + SLAB - 1) / SLAB;
  if (nslab == 0) nslab = 1;
  k_quad_1<<<dim3(nslab, nrhs), 256, 0, s>>>(n, Z, X, R, ld, partial, nslab);
  k_col_sum_2<<<(nrhs + 63) / 64, 64, 0, s>>>(nslab, nrhs, partial, quad);
  return hipGetLastError();
}

}  // namespace mpcr
