// Covariance generation and format conversion into the tile store.
//
// Matern covariance (MLE section of the paper, read with M_nu(x) = x^nu K_nu(x)):
//   Sigma_ij = sigma2 * m_nu(||s_i - s_j|| / range) + nugget [i == j]
// with the half-integer closed forms
//   nu = 1/2: exp(-x),  nu = 3/2: (1 + x) exp(-x),  nu = 5/2: (1 + x + x^2/3) exp(-x).
// Tiles past the true order n are padded with an identity block.
#include "mpcr_internal.h"

namespace mpcr {

__device__ __forceinline__ double matern_corr(double x, int nuc) {
  double e = exp(-x);
  if (nuc == 0) return e;
  if (nuc == 1) return (1.0 + x) * e;
  return (1.0 + x + x * x / 3.0) * e;
}

__device__ __forceinline__ double cov_entry(const double* locs, int n, int r, int c, double s2, double range,
                                            int nuc, double nugget) {
  double dx = locs[r] - locs[c];
  double dy = locs[n + r] - locs[n + c];
  double d = sqrt(dx * dx + dy * dy);
  double v = s2 * matern_corr(d / range, nuc);
  if (r == c) v += nugget;
  return v;
}

static int nu_code(double nu) { return nu == 0.5 ? 0 : (nu == 1.5 ? 1 : 2); }

// Row/column of packed lower-triangular index t = i (i + 1) / 2 + j.
__device__ __forceinline__ void tri_unpack(int t, int& i, int& j) {
  int ii = (int)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((ii + 1) * (ii + 2) / 2 <= t) ++ii;
  while (ii * (ii + 1) / 2 > t) --ii;
  i = ii;
  j = t - ii * (ii + 1) / 2;
}

// One workgroup per (lower tile, 16-column slab); each thread owns rows r of
// the tile (consecutive across threads, so stores are coalesced) and walks the
// 16 columns; a column's coordinates are the same for the whole workgroup.
// The tile's format is resolved once per workgroup.
// MODE 0: Sigma from the sites; 1: from a dense FP64 lower triangle;
// 2: I + diag(w) Sigma diag(w) from the sites and per-site weights w.
template <int MODE, int F>
__device__ __forceinline__ void fill_slab(void* tile, int sc, int ti, int tj, int c0, int nb, int n,
                                          const double* src, int64_t lds, double s2, double range, int nuc,
                                          double nugget, double* sig, const double* wsc) {
  for (int r = threadIdx.x; r < nb; r += blockDim.x) {
    const int R = ti * nb + r;
    const bool rin = R < n;
    double xr = 0.0, yr = 0.0, wr = 0.0;
    if (MODE != 1 && rin) {
      xr = src[R];
      yr = src[n + R];
      if (MODE == 2) wr = wsc[R];
    }
#pragma unroll 4
    for (int cc = 0; cc < 16; ++cc) {
      const int c = c0 + cc, C = tj * nb + c;
      double v;
      if (!rin || C >= n) {
        v = (R == C) ? 1.0 : 0.0;
      } else if (MODE != 1) {
        const double dx = xr - src[C];
        const double dy = yr - src[n + C];
        const double d = sqrt(dx * dx + dy * dy);
        v = s2 * matern_corr(d / range, nuc);
        if (R == C) v += nugget;
        if (MODE == 2) v = wr * v * wsc[C] + (R == C ? 1.0 : 0.0);
      } else {
        const int hi = R > C ? R : C, lo = R > C ? C : R;
        v = src[(int64_t)lo * lds + hi];
      }
      const int64_t idx = (int64_t)c * nb + r;
      store_round(tile, F, idx, F == F8 ? ldexp(v, sc) : v);
      if (sig) sig[idx] = v;
    }
  }
}

template <int MODE>  // 0: from covariance, 1: from dense FP64 lower triangle, 2: I + W Sigma W
__global__ __launch_bounds__(256) void k_fill_tiles(TileView tv, const double* src, int64_t lds, double s2,
                                                   double range, int nuc, double nugget, double* sig64,
                                                   const double* wsc) {
  int ti, tj;
  tri_unpack(blockIdx.x, ti, tj);
  const int nb = tv.nb, n = tv.n;
  void* tile = tv.tile(ti, tj);
  const int f = tv.tfmt(ti, tj);
  const int sc = f == F8 ? tv.tscale(ti, tj) : 0;  // FP8 tiles hold codes of v 2^sc
  const int c0 = blockIdx.y * 16;
  double* sig = sig64 ? sig64 + (int64_t)blockIdx.x * nb * nb : nullptr;  // FP64 copy, packed tile order
  switch (f) {
    case F64: fill_slab<MODE, F64>(tile, sc, ti, tj, c0, nb, n, src, lds, s2, range, nuc, nugget, sig, wsc); break;
    case F32: fill_slab<MODE, F32>(tile, sc, ti, tj, c0, nb, n, src, lds, s2, range, nuc, nugget, sig, wsc); break;
    case F16: fill_slab<MODE, F16>(tile, sc, ti, tj, c0, nb, n, src, lds, s2, range, nuc, nugget, sig, wsc); break;
    case BF16: fill_slab<MODE, BF16>(tile, sc, ti, tj, c0, nb, n, src, lds, s2, range, nuc, nugget, sig, wsc); break;
    default: fill_slab<MODE, F8>(tile, sc, ti, tj, c0, nb, n, src, lds, s2, range, nuc, nugget, sig, wsc); break;
  }
}

hipError_t launch_tiles_from_covariance(const TileView& tv, const double* locs, const mpcr_theta_t& th,
                                        hipStream_t s, double* sig64) {
  dim3 grid(tv.nt * (tv.nt + 1) / 2, tv.nb / 16);
  k_fill_tiles<0><<<grid, 256, 0, s>>>(tv, locs, 0, th.sigma2, th.range, nu_code(th.nu), th.nugget, sig64, nullptr);
  return hipGetLastError();
}

hipError_t launch_tiles_from_weighted_covariance(const TileView& tv, const double* locs, const mpcr_theta_t& th,
                                                 const double* w, hipStream_t s) {
  dim3 grid(tv.nt * (tv.nt + 1) / 2, tv.nb / 16);
  k_fill_tiles<2><<<grid, 256, 0, s>>>(tv, locs, 0, th.sigma2, th.range, nu_code(th.nu), th.nugget, nullptr, w);
  return hipGetLastError();
}

hipError_t launch_tiles_from_dense(const TileView& tv, const double* A, int64_t lda, hipStream_t s) {
  dim3 grid(tv.nt * (tv.nt + 1) / 2, tv.nb / 16);
  k_fill_tiles<1><<<grid, 256, 0, s>>>(tv, A, lda, 0, 1, 0, 0, nullptr, nullptr);
  return hipGetLastError();
}

// Dense lower factor (widened to FP64) from the tile store; strictly upper part 0.
__global__ __launch_bounds__(256) void k_tiles_to_dense(TileView tv, double* L, int64_t ldl) {
  const int C = blockIdx.x;
  const int n = tv.n, nb = tv.nb;
  const int tj = C / nb, c = C % nb;
  for (int R = threadIdx.x; R < n; R += blockDim.x) {
    double v = 0.0;
    if (R >= C) {
      int ti = R / nb, r = R % nb;
      v = load_wide(tv.tile(ti, tj), tv.tfmt(ti, tj), (int64_t)c * nb + r) * tv.tmul(ti, tj);
    }
    L[(int64_t)C * ldl + R] = v;
  }
}

hipError_t launch_tiles_to_dense(const TileView& tv, double* L, int64_t ldl, hipStream_t s) {
  if (tv.n == 0) return hipSuccess;
  k_tiles_to_dense<<<tv.n, 256, 0, s>>>(tv, L, ldl);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_cov_dense(int n, const double* locs, double s2, double range, int nuc,
                                                   double nugget, double* A, int64_t lda) {
  const int C = blockIdx.x;
  for (int R = threadIdx.x; R < n; R += blockDim.x)
    A[(int64_t)C * lda + R] = cov_entry(locs, n, R, C, s2, range, nuc, nugget);
}

hipError_t launch_covariance_dense(int n, const double* locs, const mpcr_theta_t& th, double* A, int64_t lda,
                                   hipStream_t s) {
  if (n == 0) return hipSuccess;
  k_cov_dense<<<n, 256, 0, s>>>(n, locs, th.sigma2, th.range, nu_code(th.nu), th.nugget, A, lda);
  return hipGetLastError();
}

// Largest |Sigma_rc| over the true entries of each lower tile.
__global__ __launch_bounds__(256) void k_cov_tile_amax(int n, int nb, int nt, const double* locs, double s2,
                                                       double range, int nuc, double nugget, double* amax) {
  int ti, tj;
  tri_unpack(blockIdx.x, ti, tj);
  __shared__ double red[256];
  double m = 0.0;
  for (int64_t e = threadIdx.x; e < (int64_t)nb * nb; e += blockDim.x) {
    int c = (int)(e / nb), r = (int)(e % nb);
    int R = ti * nb + r, C = tj * nb + c;
    if (R < n && C < n) m = fmax(m, fabs(cov_entry(locs, n, R, C, s2, range, nuc, nugget)));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) amax[(int64_t)ti * nt + tj] = red[0];
}

// Largest |A_rc| over the true entries of each lower tile of a dense FP64 matrix
// (lower triangle read).
__global__ __launch_bounds__(256) void k_dense_tile_amax(int n, int nb, int nt, const double* A, int64_t lda,
                                                         double* amax) {
  int ti, tj;
  tri_unpack(blockIdx.x, ti, tj);
  __shared__ double red[256];
  double m = 0.0;
  for (int64_t e = threadIdx.x; e < (int64_t)nb * nb; e += blockDim.x) {
    int c = (int)(e / nb), r = (int)(e % nb);
    int R = ti * nb + r, C = tj * nb + c;
    if (R < n && C < n) {
      const int hi = R > C ? R : C, lo = R > C ? C : R;
      m = fmax(m, fabs(A[(int64_t)lo * lda + hi]));
    }
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) amax[(int64_t)ti * nt + tj] = red[0];
}

hipError_t launch_dense_tile_amax(int n, int nb, const double* A, int64_t lda, double* amax, hipStream_t s) {
  int nt = (n + nb - 1) / nb;
  if (nt == 0) return hipSuccess;
  k_dense_tile_amax<<<nt * (nt + 1) / 2, 256, 0, s>>>(n, nb, nt, A, lda, amax);
  return hipGetLastError();
}

// scale exponent of every FP8 tile from its largest magnitude (0 for the others)
__global__ void k_fp8_scales(TileView tv, const double* amax) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= tv.nt * (tv.nt + 1) / 2) return;
  int ti, tj;
  tri_unpack(t, ti, tj);
  tv.sc[t] = (int8_t)(tv.fmt[t] == F8 ? fp8_scale_exp(amax[(int64_t)ti * tv.nt + tj]) : 0);
}

hipError_t launch_fp8_scales(const TileView& tv, const double* amax, hipStream_t s) {
  const int ntiles = tv.nt * (tv.nt + 1) / 2;
  k_fp8_scales<<<(ntiles + 255) / 256, 256, 0, s>>>(tv, amax);
  return hipGetLastError();
}

hipError_t launch_covariance_tile_amax(int n, int nb, const double* locs, const mpcr_theta_t& th, double* amax,
                                       hipStream_t s) {
  int nt = (n + nb - 1) / nb;
  if (nt == 0) return hipSuccess;
  k_cov_tile_amax<<<nt * (nt + 1) / 2, 256, 0, s>>>(n, nb, nt, locs, th.sigma2, th.range, nu_code(th.nu),
                                                     th.nugget, amax);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// dense conversion for the matrix product (FP8: power-of-two scale per 128 x 128
// block, the largest s with max|block| * 2^s <= 448)
// ---------------------------------------------------------------------------


__global__ __launch_bounds__(256) void k_block_scale(int64_t m, int64_t n, const double* src, int64_t lds,
                                                     int8_t* sexp, int64_t bm) {
  const int64_t bi = blockIdx.x, bj = blockIdx.y;
  __shared__ double red[256];
  double a = 0.0;
  for (int e = threadIdx.x; e < 128 * 128; e += blockDim.x) {
    int64_t r = bi * 128 + (e % 128), c = bj * 128 + (e / 128);
    if (r < m && c < n) a = fmax(a, fabs(src[c * lds + r]));
  }
  red[threadIdx.x] = a;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) sexp[bj * bm + bi] = (int8_t)fp8_scale_exp(red[0]);
}

__global__ __launch_bounds__(256) void k_convert(int prec, int64_t m, int64_t n, const double* src, int64_t lds,
                                                 void* dst, int64_t ldd, const int8_t* sexp, int64_t bm) {
  for (int64_t c = blockIdx.y; c < n; c += gridDim.y) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < m; r += (int64_t)gridDim.x * blockDim.x) {
      double v = src[c * lds + r];
      if (prec == F8) v = ldexp(v, (int)sexp[(c / 128) * bm + r / 128]);
      store_round(dst, prec, c * ldd + r, v);
    }
  }
}

hipError_t launch_convert(int prec, int64_t m, int64_t n, const double* src, int64_t lds, void* dst, int64_t ldd,
                          int8_t* scale_exp, hipStream_t s) {
  if (m == 0 || n == 0) return hipSuccess;
  int64_t bm = (m + 127) / 128, bn = (n + 127) / 128;
  if (prec == F8) {
    k_block_scale<<<dim3((unsigned)bm, (unsigned)bn), 256, 0, s>>>(m, n, src, lds, scale_exp, bm);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  unsigned gx = (unsigned)((m + 255) / 256 < 64 ? (m + 255) / 256 : 64);
  k_convert<<<dim3(gx, (unsigned)(n < 65535 ? n : 65535)), 256, 0, s>>>(prec, m, n, src, lds, dst, ldd, scale_exp, bm);
  return hipGetLastError();
}

}  // namespace mpcr
