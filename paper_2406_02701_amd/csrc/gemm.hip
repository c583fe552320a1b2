// Multi-format matrix product C = alpha op(A) op(B) + beta C.
//
// The paper's section "Linear Algebra Functions Performance" multiplies the
// same matrices in double, single and half precision; here each input format
// has its own MFMA path on gfx950:
//   FP64  v_mfma_f64_16x16x4f64      (FP64 accumulation)
//   FP32  v_mfma_f32_16x16x4f32      (FP32 accumulation)
//   BF16  v_mfma_f32_16x16x32_bf16   (FP32 accumulation)
//   FP16  v_mfma_f32_16x16x32_f16    (FP32 accumulation)
//   FP8   v_mfma_f32_16x16x32_fp8_fp8 (FP32 accumulation); each 128-wide k block
//         is accumulated separately and added with its factor 2^-(sA + sB)
// One workgroup computes a 128 x 128 block of C with four waves (2 x 2), each
// 64 x 64 = 4 x 4 MFMA tiles; operands are staged through LDS, k-major for the
// FP64/FP32 paths and row-major (k contiguous per row) for the 16/8-bit paths.
#include "mpcr_internal.h"

namespace mpcr {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

constexpr int GB = 128;  // block of C per workgroup

template <int P> struct GTraits;
template <> struct GTraits<F64> { using S = double; static constexpr int BK = 16; static constexpr bool KM = true; };
template <> struct GTraits<F32> { using S = float; static constexpr int BK = 32; static constexpr bool KM = true; };
template <> struct GTraits<BF16> { using S = uint16_t; static constexpr int BK = 64; static constexpr bool KM = false; };
template <> struct GTraits<F16> { using S = uint16_t; static constexpr int BK = 64; static constexpr bool KM = false; };
template <> struct GTraits<F8> { using S = uint8_t; static constexpr int BK = 64; static constexpr bool KM = false; };

template <int P>
__global__ __launch_bounds__(256) void k_gemm(int transA, int transB, int64_t M, int64_t N, int64_t K, double alpha,
                                              const void* Av, int64_t lda, const int8_t* sA, const void* Bv,
                                              int64_t ldb, const int8_t* sB, double beta, void* Cv, int64_t ldc,
                                              int cprec) {
  using S = typename GTraits<P>::S;
  constexpr int BK = GTraits<P>::BK;
  constexpr bool KM = GTraits<P>::KM;
  constexpr int PADK = (sizeof(S) >= 4) ? (16 / (int)sizeof(S)) : 16 / (int)sizeof(S);
  // k-major: [BK][GB + pad]; row-major: [GB][BK + pad]
  constexpr int D0 = KM ? BK : GB;
  constexpr int D1 = KM ? GB + PADK : BK + PADK;
  __shared__ __attribute__((aligned(16))) S As[D0][D1];
  __shared__ __attribute__((aligned(16))) S Bs[D0][D1];

  const S* A = (const S*)Av;
  const S* B = (const S*)Bv;
  // XCD-aware order: each XCD sweeps a contiguous run of blocks, grouped 8 block
  // rows high so that the blocks in flight on one XCD share A and B panels
  const int gm = gridDim.x, gn = gridDim.y;
  const int lb = xcd_remap(blockIdx.y * gm + blockIdx.x, gm * gn);
  constexpr int GROUP = 8;
  const int group = lb / (GROUP * gn), first = group * GROUP;
  const int rows = (gm - first) < GROUP ? (gm - first) : GROUP;
  const int bi = first + (lb % (GROUP * gn)) % rows, bj = (lb % (GROUP * gn)) / rows;
  const int64_t r0 = (int64_t)bi * GB, c0 = (int64_t)bj * GB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int64_t mbA = transA ? (K + 127) / 128 : (M + 127) / 128;  // rows of A's scale grid
  const int64_t mbB = transB ? (N + 127) / 128 : (K + 127) / 128;

  constexpr int PER = GB * BK / 256;  // elements per thread per operand
  S ra[PER], rb[PER];
  // element e of a 128 x BK slab: index order chosen so that consecutive threads
  // read consecutive addresses of the stored matrix
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + 256 * q;
      int r, kk;
      if (!transA) { r = e % GB; kk = e / GB; } else { kk = e % BK; r = e / BK; }
      const int64_t gr = r0 + r, gk = k0 + kk;
      ra[q] = (gr < M && gk < K) ? A[transA ? gr * lda + gk : gk * lda + gr] : (S)0;
      int c, kb;
      if (transB) { c = e % GB; kb = e / GB; } else { kb = e % BK; c = e / BK; }
      const int64_t gc = c0 + c, gkb = k0 + kb;
      rb[q] = (gc < N && gkb < K) ? B[transB ? gkb * ldb + gc : gc * ldb + gkb] : (S)0;
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + 256 * q;
      int r, kk;
      if (!transA) { r = e % GB; kk = e / GB; } else { kk = e % BK; r = e / BK; }
      if (KM) As[kk][r] = ra[q]; else As[r][kk] = ra[q];
      int c, kb;
      if (transB) { c = e % GB; kb = e / GB; } else { kb = e % BK; c = e / BK; }
      if (KM) Bs[kb][c] = rb[q]; else Bs[c][kb] = rb[q];
    }
  };

  using Acc = typename std::conditional<P == F64, d4, f4>::type;
  Acc acc[4][4];
  f4 part[4][4];  // FP8 only: sums of the current 128-wide k block
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = Acc{0, 0, 0, 0};

  if (K > 0) gload(0);
  for (int64_t k0 = 0; k0 < K; k0 += BK) {
    __syncthreads();
    sstore();
    __syncthreads();
    if (k0 + BK < K) gload(k0 + BK);
    if constexpr (P == F64 || P == F32) {
#pragma unroll
      for (int k4 = 0; k4 < BK; k4 += 4) {
        S av[4], bv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) av[a] = As[k4 + (lane >> 4)][wm * 64 + a * 16 + (lane & 15)];
#pragma unroll
        for (int b = 0; b < 4; ++b) bv[b] = Bs[k4 + (lane >> 4)][wn * 64 + b * 16 + (lane & 15)];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            if constexpr (P == F64)
              acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
            else
              acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
          }
      }
    } else if constexpr (P == BF16 || P == F16) {
#pragma unroll
      for (int k32 = 0; k32 < BK; k32 += 32) {
        u16x8 av[4], bv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) av[a] = *(const u16x8*)&As[wm * 64 + a * 16 + (lane & 15)][k32 + 8 * (lane >> 4)];
#pragma unroll
        for (int b = 0; b < 4; ++b) bv[b] = *(const u16x8*)&Bs[wn * 64 + b * 16 + (lane & 15)][k32 + 8 * (lane >> 4)];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            if constexpr (P == BF16)
              acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av[a]),
                                                                   __builtin_bit_cast(bf16x8, bv[b]), acc[a][b], 0, 0, 0);
            else
              acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, av[a]),
                                                                  __builtin_bit_cast(f16x8, bv[b]), acc[a][b], 0, 0, 0);
          }
      }
    } else {  // FP8: the two 64-wide slabs of each 128-wide k block share one scale
      if (k0 % 128 == 0) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) part[a][b] = f4{0, 0, 0, 0};
      }
#pragma unroll
      for (int k32 = 0; k32 < BK; k32 += 32) {
        long av[4], bv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) av[a] = *(const long*)&As[wm * 64 + a * 16 + (lane & 15)][k32 + 8 * (lane >> 4)];
#pragma unroll
        for (int b = 0; b < 4; ++b) bv[b] = *(const long*)&Bs[wn * 64 + b * 16 + (lane & 15)][k32 + 8 * (lane >> 4)];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b)
            part[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av[a], bv[b], part[a][b], 0, 0, 0);
      }
      if (k0 % 128 == 64 || k0 + BK >= K) {
        const int64_t kb = k0 / 128, ib = r0 / 128, jb = c0 / 128;
        const int ea = transA ? sA[ib * mbA + kb] : sA[kb * mbA + ib];
        const int eb = transB ? sB[kb * mbB + jb] : sB[jb * mbB + kb];
        const float sc = ldexpf(1.0f, -(ea + eb));
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] += sc * part[a][b];
      }
    }
  }

#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = (P == F64) ? ((lane >> 4) + 4 * r) : (4 * (lane >> 4) + r);
        const int64_t R = r0 + wm * 64 + a * 16 + row;
        const int64_t C = c0 + wn * 64 + b * 16 + (lane & 15);
        if (R >= M || C >= N) continue;
        const int64_t idx = C * ldc + R;
        double v = alpha * (double)acc[a][b][r];
        if (cprec == F64) {
          double* Cp = (double*)Cv;
          if (beta != 0.0) v += beta * Cp[idx];
          Cp[idx] = v;
        } else {
          float* Cp = (float*)Cv;
          if (beta != 0.0) v += beta * (double)Cp[idx];
          Cp[idx] = (float)v;
        }
      }
}

hipError_t launch_gemm(int prec, int transA, int transB, int64_t m, int64_t n, int64_t k, double alpha, const void* A,
                       int64_t lda, const int8_t* sA, const void* B, int64_t ldb, const int8_t* sB, double beta,
                       void* C, int64_t ldc, int cprec, hipStream_t s) {
  dim3 grid((unsigned)((m + GB - 1) / GB), (unsigned)((n + GB - 1) / GB));
  switch (prec) {
    case F64: k_gemm<F64><<<grid, 256, 0, s>>>(transA, transB, m, n, k, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, cprec); break;
    case F32: k_gemm<F32><<<grid, 256, 0, s>>>(transA, transB, m, n, k, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, cprec); break;
    case BF16: k_gemm<BF16><<<grid, 256, 0, s>>>(transA, transB, m, n, k, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, cprec); break;
    case F16: k_gemm<F16><<<grid, 256, 0, s>>>(transA, transB, m, n, k, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, cprec); break;
    case F8: k_gemm<F8><<<grid, 256, 0, s>>>(transA, transB, m, n, k, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, cprec); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mpcr
