// Kernels of the Metropolis-adjusted Langevin sampler (the paper's
// "Metropolis-Hastings Algorithm in High Dimensions" section) that the tile
// solves and covariance products do not already cover: the product of the
// lower tile factor with a vector (the proposal noise L eps) and the
// element-wise combinations of the proposal.
#include "mpcr_internal.h"

namespace mpcr {

// y = L x over the lower tiles (L widened to FP64; the padded tail of x is 0).
// Workgroup (i, slab): rows 64 slab .. 64 slab + 63 of tile row i; four groups
// of 64 threads take every fourth column (one row per thread, so a column of a
// column-major tile is read contiguously), then add their sums through LDS.
__global__ __launch_bounds__(256) void k_trmv_lower(TileView tv, const double* x, double* y) {
  __shared__ double part[4][64];
  const int i = blockIdx.x, nb = tv.nb;
  const int r = blockIdx.y * 64 + (threadIdx.x & 63);
  const int cg = threadIdx.x >> 6;
  double acc = 0.0;
  if (r < nb) {
    for (int j = 0; j <= i; ++j) {
      const void* t = tv.tile(i, j);
      const int f = tv.tfmt(i, j);
      const double mul = tv.tmul(i, j);
      const double* xj = x + (int64_t)j * nb;
      const int cend = (j == i) ? r + 1 : nb;
      double a = 0.0;
      for (int c = cg; c < cend; c += 4) a += load_wide(t, f, (int64_t)c * nb + r) * xj[c];
      acc += a * mul;
    }
  }
  part[cg][threadIdx.x & 63] = acc;
  __syncthreads();
  if (cg == 0 && r < nb) {
    const int lr = threadIdx.x;
    y[(int64_t)i * nb + r] = ((part[0][lr] + part[1][lr]) + part[2][lr]) + part[3][lr];
  }
}

hipError_t launch_trmv_lower(const TileView& tv, const double* x, double* y, hipStream_t s) {
  dim3 grid((unsigned)tv.nt, (unsigned)((tv.nb + 63) / 64));
  k_trmv_lower<<<grid, 256, 0, s>>>(tv, x, y);
  return hipGetLastError();
}

// out = a + alpha * b (element-wise, n entries)
__global__ void k_axpby(int n, const double* a, double alpha, const double* b, double* out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) out[i] = a[i] + alpha * b[i];
}

hipError_t launch_axpby(int n, const double* a, double alpha, const double* b, double* out, hipStream_t s) {
  int g = (n + 255) / 256;
  k_axpby<<<g < 1024 ? (g > 0 ? g : 1) : 1024, 256, 0, s>>>(n, a, alpha, b, out);
  return hipGetLastError();
}

}  // namespace mpcr
