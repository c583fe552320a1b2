// Element-wise steps of the Laplace approximation of a latent Gaussian model
// with Bernoulli observations and a logit link (the paper's "Integrated Nested
// Multi-Precision Arithmetic Laplace Approximation" section): for the latent
// field x, success probability pi = 1 / (1 + exp(-beta x)),
//   log p(y | x)       = sum_i beta x_i y_i - log(1 + exp(beta x_i)),
//   gradient            g_i = beta (y_i - pi_i),
//   minus the Hessian   W_i = beta^2 pi_i (1 - pi_i)   (diagonal, > 0).
// The dense algebra (Sigma products, the factor of I + W^1/2 Sigma W^1/2 and its
// solves) runs in the tile kernels; these kernels only combine vectors.
#include "mpcr_internal.h"

namespace mpcr {

__device__ __forceinline__ double log1pexp(double z) {  // log(1 + e^z) without overflow
  return z > 0.0 ? z + log1p(exp(-z)) : log1p(exp(z));
}

// g = grad log p(y|x), s = sqrt(W), lik_i = beta x_i y_i - log(1 + exp(beta x_i)),
// b = W x + g (the right-hand side of the Newton step)
__global__ void k_laplace_terms(int n, double beta, const double* x, const double* y, double* g, double* s,
                                double* lik, double* b) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double z = beta * x[i];
    const double pi = 1.0 / (1.0 + exp(-z));
    const double w = beta * beta * pi * (1.0 - pi);
    const double gi = beta * (y[i] - pi);
    g[i] = gi;
    s[i] = sqrt(w);
    lik[i] = z * y[i] - log1pexp(z);
    b[i] = w * x[i] + gi;
  }
}

// out = sign * s .* u
__global__ void k_scale(int n, const double* s, const double* u, double sign, double* out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) out[i] = sign * s[i] * u[i];
}

// a = b - s .* v
__global__ void k_laplace_a(int n, const double* b, const double* s, const double* v, double* a) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) a[i] = b[i] - s[i] * v[i];
}

// d = x_new - x_old, x_old = x_new
__global__ void k_step_diff(int n, const double* xnew, double* xold, double* d) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    d[i] = xnew[i] - xold[i];
    xold[i] = xnew[i];
  }
}

static unsigned grid_of(int n) {
  const int g = (n + 255) / 256;
  return (unsigned)(g < 1024 ? (g > 0 ? g : 1) : 1024);
}

hipError_t launch_laplace_terms(int n, double beta, const double* x, const double* y, double* g, double* s,
                                double* lik, double* b, hipStream_t st) {
  k_laplace_terms<<<grid_of(n), 256, 0, st>>>(n, beta, x, y, g, s, lik, b);
  return hipGetLastError();
}
hipError_t launch_scale(int n, const double* s, const double* u, double sign, double* out, hipStream_t st) {
  k_scale<<<grid_of(n), 256, 0, st>>>(n, s, u, sign, out);
  return hipGetLastError();
}
hipError_t launch_laplace_a(int n, const double* b, const double* s, const double* v, double* a, hipStream_t st) {
  k_laplace_a<<<grid_of(n), 256, 0, st>>>(n, b, s, v, a);
  return hipGetLastError();
}
hipError_t launch_step_diff(int n, const double* xnew, double* xold, double* d, hipStream_t st) {
  k_step_diff<<<grid_of(n), 256, 0, st>>>(n, xnew, xold, d);
  return hipGetLastError();
}

}  // namespace mpcr
