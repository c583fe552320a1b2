// Kernels of the Krylov refinement variants: block PCG over groups of
// right-hand sides (O'Leary's block conjugate gradients) and GMRES on the
// left-preconditioned correction equation (GMRES-based iterative
// refinement).  The introduction of the paper defines multi-precision
// refinement: the low-precision tile factor preconditions, every vector and
// residual is FP64.
//
// Right-hand sides are n x nrhs column-major blocks (leading dimension ld).
// Block PCG splits the columns into groups of `bs` consecutive columns (the
// last group may be narrower); every small matrix of a group is bs x bs,
// column-major, at offset g * bs * bs.
#include "mpcr_internal.h"

namespace mpcr {

namespace {
constexpr int GRAM_SLAB = 1024;  // rows per first-stage workgroup (fixed: the sum order does not depend on n)
constexpr int GRAM_ROWS = 64;    // rows staged in LDS at a time

__device__ __forceinline__ int group_width(int g, int bs, int nrhs) {
  const int w = nrhs - g * bs;
  return w < bs ? w : bs;
}
}  // namespace

// partial[(g * nslab + slab) * bs * bs + i + bs * j] = sum over the slab's rows of A[r, g bs + i] * B[r, g bs + j]
__global__ __launch_bounds__(256) void k_gram_1(int n, int nrhs, int bs, const double* A, const double* B,
                                                int64_t ld, double* partial, int nslab) {
  __shared__ double sa[GRAM_ROWS][KRYLOV_MAX_BLOCK + 1];
  __shared__ double sb[GRAM_ROWS][KRYLOV_MAX_BLOCK + 1];
  const int slab = blockIdx.x, g = blockIdx.y;
  const int w = group_width(g, bs, nrhs);
  const int c0 = g * bs;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};  // outputs tid, tid + 256, ... (w * w <= 1024)
  const int r_end = min(n, (slab + 1) * GRAM_SLAB);
  for (int r0 = slab * GRAM_SLAB; r0 < r_end; r0 += GRAM_ROWS) {
    const int rows = min(GRAM_ROWS, r_end - r0);
    for (int e = threadIdx.x; e < GRAM_ROWS * w; e += 256) {
      const int rr = e % GRAM_ROWS, c = e / GRAM_ROWS;
      const bool in = rr < rows;
      sa[rr][c] = in ? A[(int64_t)(c0 + c) * ld + r0 + rr] : 0.0;
      sb[rr][c] = in ? B[(int64_t)(c0 + c) * ld + r0 + rr] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int o = threadIdx.x + 256 * q;
      if (o < w * w) {
        const int i = o % w, j = o / w;
        double s = acc[q];
        for (int rr = 0; rr < rows; ++rr) s = fma(sa[rr][i], sb[rr][j], s);
        acc[q] = s;
      }
    }
    __syncthreads();
  }
  double* out = partial + ((int64_t)g * nslab + slab) * bs * bs;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int o = threadIdx.x + 256 * q;
    if (o < w * w) out[(o % w) + bs * (o / w)] = acc[q];
  }
}

// G[g] = sign * (sum of the slabs in order); entries outside the group's width are 0
__global__ void k_gram_2(int nrhs, int bs, int nslab, const double* partial, double* G, double sign) {
  const int g = blockIdx.x;
  const int w = group_width(g, bs, nrhs);
  for (int o = threadIdx.x; o < bs * bs; o += blockDim.x) {
    const int i = o % bs, j = o / bs;
    double s = 0.0;
    if (i < w && j < w)
      for (int sl = 0; sl < nslab; ++sl) s += partial[((int64_t)g * nslab + sl) * bs * bs + o];
    G[(int64_t)g * bs * bs + o] = sign * s;
  }
}

size_t gram_partial_bytes(int n, int nrhs, int bs) {
  const int nslab = n > 0 ? (n + GRAM_SLAB - 1) / GRAM_SLAB : 1;
  const int ng = (nrhs + bs - 1) / bs;
  return (size_t)nslab * ng * bs * bs * sizeof(double);
}

hipError_t launch_group_gram(int n, int nrhs, int bs, const double* A, const double* B, int64_t ld,
                             double* partial, double* G, double sign, hipStream_t s) {
  if (bs < 1 || bs > KRYLOV_MAX_BLOCK || nrhs < 1) return hipErrorInvalidValue;
  const int nslab = n > 0 ? (n + GRAM_SLAB - 1) / GRAM_SLAB : 1;
  const int ng = (nrhs + bs - 1) / bs;
  k_gram_1<<<dim3(nslab, ng), 256, 0, s>>>(n, nrhs, bs, A, B, ld, partial, nslab);
  k_gram_2<<<ng, 256, 0, s>>>(nrhs, bs, nslab, partial, G, sign);
  return hipGetLastError();
}

// C[g] = G[g]^{-1} F[g] for active groups (else 0).  G is scaled to unit
// diagonal, D G D with D = diag(G)^{-1/2}, and factored by Cholesky; a
// non-positive diagonal or a pivot of the scaled matrix below 1e-12 marks the
// group as broken down (flag[g] = 1, C[g] = 0).  One wave per group.
__global__ __launch_bounds__(64) void k_group_spd_solve(int nrhs, int bs, const double* G, const double* F,
                                                        const int* active, double* C, int* flag) {
  __shared__ double L[KRYLOV_MAX_BLOCK][KRYLOV_MAX_BLOCK + 1];
  __shared__ double Y[KRYLOV_MAX_BLOCK][KRYLOV_MAX_BLOCK + 1];
  __shared__ double D[KRYLOV_MAX_BLOCK];
  __shared__ int bad;
  const int g = blockIdx.x, t = threadIdx.x;
  const int w = group_width(g, bs, nrhs);
  const double* Gg = G + (int64_t)g * bs * bs;
  const double* Fg = F + (int64_t)g * bs * bs;
  double* Cg = C + (int64_t)g * bs * bs;
  if (t == 0) bad = active[g] ? 0 : 2;
  __syncthreads();
  if (bad == 0) {
    if (t < w) {
      const double d = Gg[t + bs * t];
      if (!(d > 0.0)) atomicOr(&bad, 1);
      D[t] = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
    }
    __syncthreads();
    for (int e = t; e < w * w; e += 64) {
      const int i = e % w, j = e / w;
      L[i][j] = D[i] * Gg[i + bs * j] * D[j];
      Y[i][j] = D[i] * Fg[i + bs * j];
    }
    __syncthreads();
    // right-looking Cholesky of the scaled matrix (lower triangle of L)
    for (int j = 0; j < w && bad == 0; ++j) {
      if (t == 0) {
        const double v = L[j][j];
        if (!(v > 1e-12)) bad = 1;
        L[j][j] = sqrt(v > 0.0 ? v : 0.0);
      }
      __syncthreads();
      if (bad) break;
      const double piv = L[j][j];
      for (int i = j + 1 + t; i < w; i += 64) L[i][j] /= piv;
      __syncthreads();
      for (int e = t; e < (w - j - 1) * (w - j - 1); e += 64) {
        const int i = j + 1 + e % (w - j - 1), k = j + 1 + e / (w - j - 1);
        if (k <= i) L[i][k] -= L[i][j] * L[k][j];
      }
      __syncthreads();
    }
    // forward and backward substitution, one right-hand side column per lane
    if (bad == 0 && t < w) {
      for (int i = 0; i < w; ++i) {
        double v = Y[i][t];
        for (int k = 0; k < i; ++k) v -= L[i][k] * Y[k][t];
        Y[i][t] = v / L[i][i];
      }
      for (int i = w - 1; i >= 0; --i) {
        double v = Y[i][t];
        for (int k = i + 1; k < w; ++k) v -= L[k][i] * Y[k][t];
        Y[i][t] = v / L[i][i];
      }
    }
    __syncthreads();
  }
  for (int e = t; e < bs * bs; e += 64) {
    const int i = e % bs, j = e / bs;
    Cg[e] = (bad == 0 && i < w && j < w) ? D[i] * Y[i][j] : 0.0;
  }
  if (t == 0) flag[g] = bad == 1 ? 1 : 0;
}

hipError_t launch_group_spd_solve(int nrhs, int bs, const double* G, const double* F, const int* active, double* C,
                                  int* flag, hipStream_t s) {
  if (bs < 1 || bs > KRYLOV_MAX_BLOCK || nrhs < 1) return hipErrorInvalidValue;
  k_group_spd_solve<<<(nrhs + bs - 1) / bs, 64, 0, s>>>(nrhs, bs, G, F, active, C, flag);
  return hipGetLastError();
}

// mode 0: Y[:, group] += sign * X[:, group] C[g]
// mode 1: Y[:, group] = X[:, group] + Y[:, group] C[g]   (in place on Y, row by row)
template <int MODE>
__global__ __launch_bounds__(256) void k_group_update(int n, int nrhs, int bs, const double* X, const double* C,
                                                      double sign, double* Y, int64_t ld) {
  __shared__ double sc[KRYLOV_MAX_BLOCK * KRYLOV_MAX_BLOCK];
  const int g = blockIdx.y;
  const int w = group_width(g, bs, nrhs);
  const int c0 = g * bs;
  for (int e = threadIdx.x; e < bs * bs; e += 256) sc[e] = C[(int64_t)g * bs * bs + e];
  __syncthreads();
  for (int r = blockIdx.x * 256 + threadIdx.x; r < n; r += gridDim.x * 256) {
    double v[KRYLOV_MAX_BLOCK];
    const double* src = MODE == 0 ? X : Y;
#pragma unroll
    for (int i = 0; i < KRYLOV_MAX_BLOCK; ++i) v[i] = i < w ? src[(int64_t)(c0 + i) * ld + r] : 0.0;
    for (int j = 0; j < w; ++j) {
      double a = 0.0;
#pragma unroll
      for (int i = 0; i < KRYLOV_MAX_BLOCK; ++i)
        if (i < w) a = fma(v[i], sc[i + bs * j], a);
      double* y = Y + (int64_t)(c0 + j) * ld + r;
      if (MODE == 0)
        *y += sign * a;
      else
        *y = X[(int64_t)(c0 + j) * ld + r] + a;
    }
  }
}

hipError_t launch_group_axpy(int n, int nrhs, int bs, const double* X, const double* C, double sign, double* Y,
                             int64_t ld, hipStream_t s) {
  if (bs < 1 || bs > KRYLOV_MAX_BLOCK || nrhs < 1) return hipErrorInvalidValue;
  if (n == 0) return hipSuccess;
  const int gx = min((n + 255) / 256, 512);
  k_group_update<0><<<dim3(gx, (nrhs + bs - 1) / bs), 256, 0, s>>>(n, nrhs, bs, X, C, sign, Y, ld);
  return hipGetLastError();
}

hipError_t launch_group_xpyc(int n, int nrhs, int bs, const double* X, const double* C, double* Y, int64_t ld,
                             hipStream_t s) {
  if (bs < 1 || bs > KRYLOV_MAX_BLOCK || nrhs < 1) return hipErrorInvalidValue;
  if (n == 0) return hipSuccess;
  const int gx = min((n + 255) / 256, 512);
  k_group_update<1><<<dim3(gx, (nrhs + bs - 1) / bs), 256, 0, s>>>(n, nrhs, bs, X, C, 0.0, Y, ld);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// GMRES (one Hessenberg matrix per column; H[c] is (m+1) x m column-major at
// c * (m+1) * m; cs, sn, g per column at c * (m+1))
// ---------------------------------------------------------------------------

// out[c * stride] = sum of the column reduction partials (see launch_col_dot)
__global__ __launch_bounds__(256) void k_dot_1(int n, const double* A, const double* B, int64_t ld, double* partial,
                                               int nslab) {
  __shared__ double red[256];
  const int slab = blockIdx.x, c = blockIdx.y;
  double s = 0.0;
  for (int r = slab * GRAM_SLAB + threadIdx.x; r < n && r < (slab + 1) * GRAM_SLAB; r += 256)
    s += A[(int64_t)c * ld + r] * B[(int64_t)c * ld + r];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(int64_t)c * nslab + slab] = red[0];
}
__global__ void k_dot_2(int nslab, int ncol, const double* partial, double* out, int64_t stride) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncol) return;
  double s = 0.0;
  for (int i = 0; i < nslab; ++i) s += partial[(int64_t)c * nslab + i];
  out[(int64_t)c * stride] = s;
}
hipError_t launch_col_dot_strided(int n, int nrhs, const double* A, const double* B, int64_t ld, double* partial,
                                  double* out, int64_t stride, hipStream_t s) {
  const int nslab = n > 0 ? (n + GRAM_SLAB - 1) / GRAM_SLAB : 1;
  k_dot_1<<<dim3(nslab, nrhs), 256, 0, s>>>(n, A, B, ld, partial, nslab);
  k_dot_2<<<(nrhs + 63) / 64, 64, 0, s>>>(nslab, nrhs, partial, out, stride);
  return hipGetLastError();
}

// Y[:, c] += sign * a[c * stride] * X[:, c]
__global__ void k_axpy_strided(int n, const double* a, int64_t stride, double sign, const double* X, double* Y,
                               int64_t ld) {
  const int c = blockIdx.y;
  const double f = sign * a[(int64_t)c * stride];
  if (f == 0.0) return;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
    Y[(int64_t)c * ld + r] += f * X[(int64_t)c * ld + r];
}
hipError_t launch_axpy_strided(int n, int nrhs, const double* a, int64_t stride, double sign, const double* X,
                               double* Y, int64_t ld, hipStream_t s) {
  if (n == 0 || nrhs == 0) return hipSuccess;
  const int g = (n + 255) / 256;
  k_axpy_strided<<<dim3(g < 256 ? g : 256, nrhs), 256, 0, s>>>(n, a, stride, sign, X, Y, ld);
  return hipGetLastError();
}

// Y[:, c] = f[c] * X[:, c], with f[c] = 0 giving exact zeros
__global__ void k_scale_cols(int n, const double* f, const double* X, double* Y, int64_t ld) {
  const int c = blockIdx.y;
  const double a = f[c];
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
    Y[(int64_t)c * ld + r] = a == 0.0 ? 0.0 : a * X[(int64_t)c * ld + r];
}
hipError_t launch_scale_cols(int n, int nrhs, const double* f, const double* X, double* Y, int64_t ld,
                             hipStream_t s) {
  if (n == 0 || nrhs == 0) return hipSuccess;
  const int g = (n + 255) / 256;
  k_scale_cols<<<dim3(g < 256 ? g : 256, nrhs), 256, 0, s>>>(n, f, X, Y, ld);
  return hipGetLastError();
}

// Start of a GMRES cycle: beta[c] = sqrt(dot[c]); g[c] = (beta, 0, ...);
// inv[c] = 1 / beta for active columns with beta > 0, else 0.
__global__ void k_gmres_start(int nrhs, int m, const double* dot, const int* active, double* beta, double* g,
                              double* inv) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  const double b = sqrt(fmax(dot[c], 0.0));
  beta[c] = b;
  for (int i = 0; i <= m; ++i) g[(int64_t)c * (m + 1) + i] = i == 0 ? b : 0.0;
  inv[c] = (active[c] && b > 0.0) ? 1.0 / b : 0.0;
}
hipError_t launch_gmres_start(int nrhs, int m, const double* dot, const int* active, double* beta, double* g,
                              double* inv, hipStream_t s) {
  k_gmres_start<<<(nrhs + 63) / 64, 64, 0, s>>>(nrhs, m, dot, active, beta, g, inv);
  return hipGetLastError();
}

// Step j of every column that is still running (run[c] != 0): H[j+1, j] =
// sqrt(dot[c]); the earlier rotations are applied to column j of H, a new
// rotation zeroes H[j+1, j], and g is rotated.  out[2c] = |g[j+1]| (the
// residual estimate), out[2c+1] = the norm before rotation (0: the Krylov
// space is invariant and the column's GMRES solution is exact).
__global__ void k_gmres_rotate(int nrhs, int m, int j, const double* dot, const int* run, double* H, double* cs,
                               double* sn, double* g, double* out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  if (!run[c]) {
    out[2 * c] = 0.0;
    out[2 * c + 1] = 0.0;
    return;
  }
  double* h = H + (int64_t)c * (m + 1) * m + (int64_t)(m + 1) * j;
  double* cc = cs + (int64_t)c * (m + 1);
  double* ss = sn + (int64_t)c * (m + 1);
  double* gg = g + (int64_t)c * (m + 1);
  const double hn = sqrt(fmax(dot[c], 0.0));
  h[j + 1] = hn;
  for (int i = 0; i < j; ++i) {
    const double t = cc[i] * h[i] + ss[i] * h[i + 1];
    h[i + 1] = -ss[i] * h[i] + cc[i] * h[i + 1];
    h[i] = t;
  }
  const double a = h[j], b = h[j + 1];
  const double r = hypot(a, b);
  const double cj = r != 0.0 ? a / r : 1.0, sj = r != 0.0 ? b / r : 0.0;
  cc[j] = cj;
  ss[j] = sj;
  h[j] = r;
  h[j + 1] = 0.0;
  gg[j + 1] = -sj * gg[j];
  gg[j] = cj * gg[j];
  out[2 * c] = fabs(gg[j + 1]);
  out[2 * c + 1] = hn;
}
hipError_t launch_gmres_rotate(int nrhs, int m, int j, const double* dot, const int* run, double* H, double* cs,
                               double* sn, double* g, double* out, hipStream_t s) {
  k_gmres_rotate<<<(nrhs + 63) / 64, 64, 0, s>>>(nrhs, m, j, dot, run, H, cs, sn, g, out);
  return hipGetLastError();
}

// inv[c] = 1 / norm[2c+1] for columns that continue (cont[c] != 0) with a
// non-zero norm, else 0 (the next basis vector of that column is zero)
__global__ void k_gmres_inv(int nrhs, const double* norm, const int* cont, double* inv) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  const double h = norm[2 * c + 1];
  inv[c] = (cont[c] && h != 0.0) ? 1.0 / h : 0.0;
}
hipError_t launch_gmres_inv(int nrhs, const double* norm, const int* cont, double* inv, hipStream_t s) {
  k_gmres_inv<<<(nrhs + 63) / 64, 64, 0, s>>>(nrhs, norm, cont, inv);
  return hipGetLastError();
}

// y[c] = R_k^{-1} g[c][0..k) with k = steps[c] (the rotated Hessenberg is
// upper triangular); y[c][i] = 0 for i >= k.  y[c] is at c * m.
__global__ void k_gmres_backsolve(int nrhs, int m, const double* H, const double* g, const int* steps, double* y) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nrhs) return;
  const double* h = H + (int64_t)c * (m + 1) * m;
  const double* gg = g + (int64_t)c * (m + 1);
  double* yy = y + (int64_t)c * m;
  const int k = steps[c];
  for (int i = m - 1; i >= 0; --i) {
    if (i >= k) {
      yy[i] = 0.0;
      continue;
    }
    double v = gg[i];
    for (int q = i + 1; q < k; ++q) v -= h[(int64_t)(m + 1) * q + i] * yy[q];
    yy[i] = v / h[(int64_t)(m + 1) * i + i];
  }
}
hipError_t launch_gmres_backsolve(int nrhs, int m, const double* H, const double* g, const int* steps, double* y,
                                  hipStream_t s) {
  k_gmres_backsolve<<<(nrhs + 63) / 64, 64, 0, s>>>(nrhs, m, H, g, steps, y);
  return hipGetLastError();
}

}  // namespace mpcr
