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
// The FP8 k blocks of 128 are those of the block scaling (one exponent per
// 128 x 128 block of each operand).
#include "mpcr_internal.h"

namespace mpcr {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

constexpr int GB = 128;  // block of C per workgroup

// FP64 uses 8 waves of 64 x 32 (more waves per CU hide the staging of the
// slow FP64 MFMA better than more work per wave), FP32 4 waves of 64 x 64;
// both stage 16 k per chunk, double-buffered with one barrier per chunk (the
// shapes of the factorisation's tile-update loop).
template <int P> struct GTraits;
template <> struct GTraits<F64> { using S = double; static constexpr int BK = 16, NW = 8, WPE = 2; };
template <> struct GTraits<F32> { using S = float; static constexpr int BK = 16, NW = 4, WPE = 2; };

// FP64 / FP32 path: operands staged k-major ([BK][GB + pad]) through LDS.
template <int P>
__global__ __launch_bounds__(GTraits<P>::NW * 64) __attribute__((amdgpu_waves_per_eu(GTraits<P>::WPE))) void
k_gemm(int transA, int transB, int64_t M, int64_t N, int64_t K, double alpha, const void* Av, int64_t lda,
       const void* Bv, int64_t ldb, double beta, void* Cv, int64_t ldc, int cprec) {
  using S = typename GTraits<P>::S;
  constexpr int BK = GTraits<P>::BK, NW = GTraits<P>::NW, NT = NW * 64;
  constexpr int WM = 2, WN = NW / WM, TM = GB / WM, TN = GB / WN, FM = TM / 16, FN = TN / 16;
  constexpr int PADK = 16;  // rows k, k+1 (FP64) or k .. k+3 (FP32) of a fragment on disjoint banks
  __shared__ __attribute__((aligned(16))) S As[2][BK][GB + PADK];
  __shared__ __attribute__((aligned(16))) S Bs[2][BK][GB + PADK];

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
  const int wm = wave % WM, wn = wave / WM;

  constexpr int PER = GB * BK / NT;  // elements per thread per operand
  constexpr int V = 16 / sizeof(S);  // elements per 16-byte vector
  constexpr int PV = PER / V;        // vectors per thread per operand
  S ra[PER], rb[PER];
  // Whole blocks with 16-byte aligned columns move 16-byte vectors (V
  // consecutive elements of the stored matrix: rows of a column, or k values
  // of a transposed operand's column); other blocks move single elements with
  // bounds checks.  Consecutive threads read consecutive addresses.
  const bool vec = (r0 + GB <= M) && (c0 + GB <= N) && (K % BK == 0) && ((lda * (int64_t)sizeof(S)) % 16 == 0) &&
                   ((ldb * (int64_t)sizeof(S)) % 16 == 0) && ((uintptr_t)A % 16 == 0) && ((uintptr_t)B % 16 == 0);
  // vector v of a thread: (row-or-column index, k index) of its first element
  auto avec = [&](int v, int& r, int& kk) {
    const int e = tid + NT * v;
    if (!transA) { r = (e % (GB / V)) * V; kk = e / (GB / V); } else { kk = (e % (BK / V)) * V; r = e / (BK / V); }
  };
  auto bvec = [&](int v, int& c, int& kb) {
    const int e = tid + NT * v;
    if (transB) { c = (e % (GB / V)) * V; kb = e / (GB / V); } else { kb = (e % (BK / V)) * V; c = e / (BK / V); }
  };
  auto gload = [&](int64_t k0) {
    if (vec) {
#pragma unroll
      for (int v = 0; v < PV; ++v) {
        int r, kk, c, kb;
        avec(v, r, kk);
        bvec(v, c, kb);
        const S* pa = A + (transA ? (r0 + r) * lda + k0 + kk : (k0 + kk) * lda + r0 + r);
        const S* pb = B + (transB ? (k0 + kb) * ldb + c0 + c : (c0 + c) * ldb + k0 + kb);
        *(uint4*)&ra[V * v] = *(const uint4*)pa;
        *(uint4*)&rb[V * v] = *(const uint4*)pb;
      }
      return;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + NT * q;
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
  auto sstore = [&](int buf) {
    if (vec) {
#pragma unroll
      for (int v = 0; v < PV; ++v) {
        int r, kk, c, kb;
        avec(v, r, kk);
        bvec(v, c, kb);
#pragma unroll
        for (int u = 0; u < V; ++u) {
          if (!transA) As[buf][kk][r + u] = ra[V * v + u]; else As[buf][kk + u][r] = ra[V * v + u];
          if (transB) Bs[buf][kb][c + u] = rb[V * v + u]; else Bs[buf][kb + u][c] = rb[V * v + u];
        }
      }
      return;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + NT * q;
      int r, kk;
      if (!transA) { r = e % GB; kk = e / GB; } else { kk = e % BK; r = e / BK; }
      As[buf][kk][r] = ra[q];
      int c, kb;
      if (transB) { c = e % GB; kb = e / GB; } else { kb = e % BK; c = e / BK; }
      Bs[buf][kb][c] = rb[q];
    }
  };

  using Acc = typename std::conditional<P == F64, d4, f4>::type;
  Acc acc[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) acc[a][b] = Acc{0, 0, 0, 0};

  if (K > 0) {
    gload(0);
    sstore(0);
  }
  __syncthreads();
  int cur = 0;
  for (int64_t k0 = 0; k0 < K; k0 += BK) {
    const bool more = k0 + BK < K;
    if (more) gload(k0 + BK);
#pragma unroll
    for (int k4 = 0; k4 < BK; k4 += 4) {
      S av[FM], bv[FN];
#pragma unroll
      for (int a = 0; a < FM; ++a) av[a] = As[cur][k4 + (lane >> 4)][wm * TM + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < FN; ++b) bv[b] = Bs[cur][k4 + (lane >> 4)][wn * TN + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < FM; ++a)
#pragma unroll
        for (int b = 0; b < FN; ++b) {
          if constexpr (P == F64)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
          else
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
    }
    if (more) sstore(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }

#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = (P == F64) ? ((lane >> 4) + 4 * r) : (4 * (lane >> 4) + r);
        const int64_t R = r0 + wm * TM + a * 16 + row;
        const int64_t C = c0 + wn * TN + b * 16 + (lane & 15);
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

// ---------------------------------------------------------------------------
// 16- and 8-bit path.  Both operands are read "k-contiguous": A as an m x k
// row-major array (AT, leading dimension ldat) and B as the usual k x n
// column-major array.  Every thread moves 16-byte vectors global -> LDS, rows
// are padded by 16 bytes (conflict-free 16-byte fragment reads), LDS is
// double-buffered.  Operands in another layout, or whose rows are not 16-byte
// aligned, are first packed (k_pack).  FP8 takes one 128-wide k block per
// chunk, so each chunk's sums are scaled by 2^-(sA + sB) once.
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void k_gemm_lowp(int64_t M, int64_t N, int64_t K, double alpha, const void* ATv,
                                                   int64_t ldat, const int8_t* sA, int64_t mbA, const void* Bv,
                                                   int64_t ldb, const int8_t* sB, int64_t mbB, int sa_kmajor,
                                                   int sb_kmajor, double beta, void* Cv, int64_t ldc, int cprec) {
  constexpr int ES = (P == F8) ? 1 : 2;       // element bytes
  constexpr int BK = (P == F8) ? 128 : 64;    // k per chunk (one FP8 scale block)
  constexpr int VE = 16 / ES;                 // elements per 16-byte vector
  constexpr int LDR = BK * ES + 16;           // padded LDS row in bytes
  constexpr int VPR = BK / VE;                // vectors per row per chunk (8)
  __shared__ __attribute__((aligned(16))) uint8_t As[2][GB * LDR];
  __shared__ __attribute__((aligned(16))) uint8_t Bs[2][GB * LDR];

  const uint8_t* AT = (const uint8_t*)ATv;
  const uint8_t* B = (const uint8_t*)Bv;
  const int gm = gridDim.x, gn = gridDim.y;
  const int lb = xcd_remap(blockIdx.y * gm + blockIdx.x, gm * gn);
  constexpr int GROUP = 8;
  const int group = lb / (GROUP * gn), first = group * GROUP;
  const int rows = (gm - first) < GROUP ? (gm - first) : GROUP;
  const int bi = first + (lb % (GROUP * gn)) % rows, bj = (lb % (GROUP * gn)) / rows;
  const int64_t r0 = (int64_t)bi * GB, c0 = (int64_t)bj * GB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const bool full = (r0 + GB <= M) && (c0 + GB <= N) && (K % BK == 0);

  // loader: thread t moves vectors (row = t / VPR + 32 v, chunk t % VPR), v = 0..3
  uint4 ra[4], rb[4];
  auto gload = [&](int64_t k0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = tid / VPR + 32 * v, kc = tid % VPR;
      const int64_t gk = k0 + kc * VE;
      const int64_t ga = r0 + row, gb = c0 + row;
      if (full || (ga < M && gk + VE <= K)) {
        ra[v] = *(const uint4*)(AT + (ga * ldat + gk) * ES);
      } else {
        uint8_t tmp[16] = {0};
        for (int e = 0; e < VE; ++e)
          if (ga < M && gk + e < K)
            for (int b = 0; b < ES; ++b) tmp[e * ES + b] = AT[(ga * ldat + gk + e) * ES + b];
        ra[v] = *(uint4*)tmp;
      }
      if (full || (gb < N && gk + VE <= K)) {
        rb[v] = *(const uint4*)(B + (gb * ldb + gk) * ES);
      } else {
        uint8_t tmp[16] = {0};
        for (int e = 0; e < VE; ++e)
          if (gb < N && gk + e < K)
            for (int b = 0; b < ES; ++b) tmp[e * ES + b] = B[(gb * ldb + gk + e) * ES + b];
        rb[v] = *(uint4*)tmp;
      }
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = tid / VPR + 32 * v, kc = tid % VPR;
      *(uint4*)&As[buf][row * LDR + kc * 16] = ra[v];
      *(uint4*)&Bs[buf][row * LDR + kc * 16] = rb[v];
    }
  };

  f4 acc[4][4], part[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f4{0, 0, 0, 0};

  if (K > 0) {
    gload(0);
    sstore(0);
  }
  __syncthreads();
  int cur = 0;
  for (int64_t k0 = 0; k0 < K; k0 += BK) {
    const bool more = k0 + BK < K;
    if (more) gload(k0 + BK);
    if constexpr (P == F8) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) part[a][b] = f4{0, 0, 0, 0};
    }
#pragma unroll
    for (int k32 = 0; k32 < BK; k32 += 32) {
      const int kb = (k32 + 8 * (lane >> 4)) * ES;  // byte offset of this lane's 8 k values
      if constexpr (P == F8) {
        long av[4], bv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) av[a] = *(const long*)&As[cur][(wm * 64 + a * 16 + (lane & 15)) * LDR + kb];
#pragma unroll
        for (int b = 0; b < 4; ++b) bv[b] = *(const long*)&Bs[cur][(wn * 64 + b * 16 + (lane & 15)) * LDR + kb];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b)
            part[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av[a], bv[b], part[a][b], 0, 0, 0);
      } else {
        u16x8 av[4], bv[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) av[a] = *(const u16x8*)&As[cur][(wm * 64 + a * 16 + (lane & 15)) * LDR + kb];
#pragma unroll
        for (int b = 0; b < 4; ++b) bv[b] = *(const u16x8*)&Bs[cur][(wn * 64 + b * 16 + (lane & 15)) * LDR + kb];
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
    }
    if constexpr (P == F8) {
      const int64_t kb = k0 / 128, ib = r0 / 128, jb = c0 / 128;
      const int ea = sa_kmajor ? sA[ib * mbA + kb] : sA[kb * mbA + ib];
      const int eb = sb_kmajor ? sB[kb * mbB + jb] : sB[jb * mbB + kb];
      const float sc = ldexpf(1.0f, -(ea + eb));
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] += sc * part[a][b];
    }
    if (more) sstore(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }

#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t R = r0 + wm * 64 + a * 16 + 4 * (lane >> 4) + r;
        const int64_t Cc = c0 + wn * 64 + b * 16 + (lane & 15);
        if (R >= M || Cc >= N) continue;
        const int64_t idx = Cc * ldc + R;
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

// ---------------------------------------------------------------------------
// Large 16-bit products (m, n multiples of 256, k a multiple of 64): one
// workgroup of eight waves (two per SIMD) computes a 256 x 256 block of C;
// wave (wm, wn), wm < 2, wn < 4, owns rows 128 wm .. +127 and columns
// 64 wn .. +63 as 8 x 4 tiles of 16 x 16 (measured: 8 waves of 128 x 64 run
// 1.27x faster than 4 waves of 128 x 128, whose accumulators fill every
// accumulation register and force copies).  Stages of 64 k: both operands' 256 rows of 128
// bytes are moved global -> registers -> LDS (rows padded to 144 bytes, so
// the 16-byte fragment reads of 16 consecutive rows hit disjoint banks),
// double-buffered with one barrier per stage; the next stage's global loads
// are in flight during the current stage's MFMAs.  The MFMA takes the B
// fragment as its first operand, so a lane's four results are four columns of
// one row of C: for each register the 16 lanes of a group store 16
// consecutive rows (64 contiguous bytes) of a column.
// ---------------------------------------------------------------------------
constexpr int BG = 256;  // block of C per workgroup of the large kernel

template <int P, int WN>  // WN waves along n (2: 128 x 128 per wave, 4: 128 x 64 per wave)
__global__ __launch_bounds__(128 * WN) void k_gemm_lowp_big(int64_t M, int64_t N, int64_t K, double alpha,
                                                            const void* ATv, int64_t ldat, const void* Bv,
                                                            int64_t ldb, double beta, void* Cv, int64_t ldc,
                                                            int cprec) {
  static_assert(P == BF16 || P == F16, "16-bit formats");
  constexpr int NT = 128 * WN;           // threads
  constexpr int TN = BG / WN / 16;       // 16-column tiles per wave
  constexpr int RPL = NT / 8;            // rows per load instruction
  constexpr int NV = BG / RPL;           // 16-byte vectors per thread and operand
  // LDS rows of 128 bytes padded to 160 (measured at 8192^3: 32-byte pad 1027 TF/s BF16, 16-byte 984, an
  // XOR swizzle of the 16-byte granules 1016, 8-byte 364); the two buffers of both operands fill the 160 KB
  constexpr int ES = 2, BK = 64, ROWB = BK * ES, LDR = ROWB + 32;
  __shared__ __attribute__((aligned(16))) uint8_t As[2][BG * LDR];
  __shared__ __attribute__((aligned(16))) uint8_t Bs[2][BG * LDR];
  const uint8_t* AT = (const uint8_t*)ATv;
  const uint8_t* B = (const uint8_t*)Bv;
  // XCD-aware order, grouped 8 block rows high (blocks in flight on one XCD share panels)
  const int gm = gridDim.x, gn = gridDim.y;
  const int lb = xcd_remap(blockIdx.y * gm + blockIdx.x, gm * gn);
  constexpr int GROUP = 8;
  const int group = lb / (GROUP * gn), first = group * GROUP;
  const int rows = (gm - first) < GROUP ? (gm - first) : GROUP;
  const int bi = first + (lb % (GROUP * gn)) % rows, bj = (lb % (GROUP * gn)) / rows;
  const int64_t r0 = (int64_t)bi * BG, c0 = (int64_t)bj * BG;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int g16 = lane & 15, q = lane >> 4;

  // loader: thread t moves 16-byte vectors (row t / 8 + RPL v, chunk t % 8),
  // v < NV, of both operands.  The last stage reloads itself (no branch around
  // the staging, so the staged vectors stay in registers); its copies are
  // never read.
  const int lrow = tid >> 3, lchunk = tid & 7;
  const uint8_t* ga = AT + ((r0 + lrow) * ldat) * ES + lchunk * 16;
  const uint8_t* gb = B + ((c0 + lrow) * ldb) * ES + lchunk * 16;
  const int64_t stepa = RPL * ldat * ES, stepb = RPL * ldb * ES;
  auto lds_at = [](int row, int gran) { return row * LDR + gran * 16; };
  const int soff = lds_at(lrow, lchunk);

  f4 acc[8][TN];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = f4{0, 0, 0, 0};

  static_assert(NV == 4, "four 16-byte vectors per thread and operand");
  uint4 ga0, ga1, ga2, ga3, gb0, gb1, gb2, gb3;
#define MPCR_GLOAD(KB)                                                                                \
  ga0 = *(const uint4*)(ga + 0 * stepa + KB); ga1 = *(const uint4*)(ga + 1 * stepa + KB);            \
  ga2 = *(const uint4*)(ga + 2 * stepa + KB); ga3 = *(const uint4*)(ga + 3 * stepa + KB);            \
  gb0 = *(const uint4*)(gb + 0 * stepb + KB); gb1 = *(const uint4*)(gb + 1 * stepb + KB);            \
  gb2 = *(const uint4*)(gb + 2 * stepb + KB); gb3 = *(const uint4*)(gb + 3 * stepb + KB);
#define MPCR_SSTORE(BUF)                                                                              \
  *(uint4*)&As[BUF][soff + 0 * RPL * LDR] = ga0; *(uint4*)&As[BUF][soff + 1 * RPL * LDR] = ga1;      \
  *(uint4*)&As[BUF][soff + 2 * RPL * LDR] = ga2; *(uint4*)&As[BUF][soff + 3 * RPL * LDR] = ga3;      \
  *(uint4*)&Bs[BUF][soff + 0 * RPL * LDR] = gb0; *(uint4*)&Bs[BUF][soff + 1 * RPL * LDR] = gb1;      \
  *(uint4*)&Bs[BUF][soff + 2 * RPL * LDR] = gb2; *(uint4*)&Bs[BUF][soff + 3 * RPL * LDR] = gb3;

  // fragments of one 32-wide k step: A rows 16 a + g16, B columns 16 b + g16,
  // k values 8 q .. 8 q + 7 of the step
  u16x8 fa0[8], fb0[TN], fa1[8], fb1[TN];
  auto frag = [&](int buf, int k32, u16x8* fa, u16x8* fb) {
    const int gran = (k32 + 8 * q) * ES / 16;
    const uint8_t* Ab = &As[buf][lds_at(wm * 128 + g16, gran)];
    const uint8_t* Bb = &Bs[buf][lds_at(wn * TN * 16 + g16, gran)];
#pragma unroll
    for (int b = 0; b < TN; ++b) fb[b] = *(const u16x8*)(Bb + b * 16 * LDR);
#pragma unroll
    for (int a = 0; a < 8; ++a) fa[a] = *(const u16x8*)(Ab + a * 16 * LDR);
  };
  auto mma = [&](const u16x8* fa, const u16x8* fb) {
#pragma unroll
    for (int a = 0; a < 8; ++a)
#pragma unroll
      for (int b = 0; b < TN; ++b) {
        if constexpr (P == BF16)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, fb[b]),
                                                               __builtin_bit_cast(bf16x8, fa[a]), acc[a][b], 0, 0, 0);
        else
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, fb[b]),
                                                              __builtin_bit_cast(f16x8, fa[a]), acc[a][b], 0, 0, 0);
      }
  };
  MPCR_GLOAD(0)
  MPCR_SSTORE(0)
  __syncthreads();
  int cur = 0;
  frag(0, 0, fa0, fb0);
  // per stage: the next stage's A and B are requested at its start and stored
  // to the other LDS buffer at its end; the second step's fragments are read
  // while the first step's MFMAs run; after the barrier the next stage's first
  // fragments are read
  for (int64_t k0 = 0; k0 < K; k0 += BK) {
    const int64_t kn = (k0 + BK < K ? k0 + BK : k0) * ES;  // the next stage (the last one reloads itself)
    MPCR_GLOAD(kn)
    frag(cur, 32, fa1, fb1);
    mma(fa0, fb0);
    mma(fa1, fb1);
    MPCR_SSTORE(cur ^ 1)
    __syncthreads();
    cur ^= 1;
    frag(cur, 0, fa0, fb0);
  }
#undef MPCR_GLOAD
#undef MPCR_SSTORE

  // lane (g16, q), register r of tile (a, b): C[r0 + 128 wm + 16 a + g16][c0 + 16 TN wn + 16 b + 4 q + r]
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t R = r0 + wm * 128 + a * 16 + g16;
        const int64_t Cc = c0 + wn * TN * 16 + b * 16 + 4 * q + r;
        const int64_t idx = Cc * ldc + R;
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

// ---------------------------------------------------------------------------
// Large FP8 products (m, n multiples of 256, k a multiple of 128): the same
// 256 x 256 blocking, eight waves of 128 x 64 and operand staging as the
// 16-bit kernel, with stages of 128 k = one block of the power-of-two
// scaling.  Each 16 x 16 tile of a stage is one gfx950 block-scaled MFMA
// (v_mfma_scale_f32_16x16x128_f8f6f4, E4M3 operands): its E8M0 scales
// 2^(127 - e) undo the operands' block exponents inside the instruction
// (exact powers of two), so the stages accumulate straight into the FP32
// results.  A lane supplies 32 consecutive k of one row or column; the same
// lane-to-k assignment for both operands makes the sum correct for any
// internal order of the 128 products.
// ---------------------------------------------------------------------------
typedef int i32x8 __attribute__((ext_vector_type(8)));

__global__ __launch_bounds__(512) void k_gemm_fp8_big(int64_t M, int64_t N, int64_t K, double alpha,
                                                     const void* ATv, int64_t ldat, const int8_t* sA, int64_t mbA,
                                                     int sa_kmajor, const void* Bv, int64_t ldb, const int8_t* sB,
                                                     int64_t mbB, int sb_kmajor, double beta, void* Cv,
                                                     int64_t ldc, int cprec) {
  constexpr int WN = 4, NT = 512, TN = 4;  // waves along n, threads, 16-column tiles per wave
  constexpr int BK = 128, ROWB = BK, LDR = ROWB + 16;
  constexpr int RPL = NT / 8;              // rows per load instruction
  __shared__ __attribute__((aligned(16))) uint8_t As[2][BG * LDR];
  __shared__ __attribute__((aligned(16))) uint8_t Bs[2][BG * LDR];
  const uint8_t* AT = (const uint8_t*)ATv;
  const uint8_t* B = (const uint8_t*)Bv;
  const int gm = gridDim.x, gn = gridDim.y;
  const int lb = xcd_remap(blockIdx.y * gm + blockIdx.x, gm * gn);
  constexpr int GROUP = 8;
  const int group = lb / (GROUP * gn), first = group * GROUP;
  const int rows = (gm - first) < GROUP ? (gm - first) : GROUP;
  const int bi = first + (lb % (GROUP * gn)) % rows, bj = (lb % (GROUP * gn)) / rows;
  const int64_t r0 = (int64_t)bi * BG, c0 = (int64_t)bj * BG;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int g16 = lane & 15, q = lane >> 4;
  // the scale blocks of this wave's rows and columns
  const int64_t ib = (r0 + 128 * wm) / 128, jb = (c0 + 64 * wn) / 128;

  const int lrow = tid >> 3, lchunk = tid & 7;
  const uint8_t* ga = AT + (r0 + lrow) * ldat + lchunk * 16;
  const uint8_t* gb = B + (c0 + lrow) * ldb + lchunk * 16;
  const int64_t stepa = RPL * ldat, stepb = RPL * ldb;
  auto lds_at = [](int row, int gran) { return row * LDR + gran * 16; };
  const int soff = lds_at(lrow, lchunk);

  f4 acc[8][TN];
#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b) acc[a][b] = f4{0, 0, 0, 0};

  uint4 ga0, ga1, ga2, ga3, gb0, gb1, gb2, gb3;
#define MPCR_GLOAD(KB)                                                                                \
  ga0 = *(const uint4*)(ga + 0 * stepa + KB); ga1 = *(const uint4*)(ga + 1 * stepa + KB);            \
  ga2 = *(const uint4*)(ga + 2 * stepa + KB); ga3 = *(const uint4*)(ga + 3 * stepa + KB);            \
  gb0 = *(const uint4*)(gb + 0 * stepb + KB); gb1 = *(const uint4*)(gb + 1 * stepb + KB);            \
  gb2 = *(const uint4*)(gb + 2 * stepb + KB); gb3 = *(const uint4*)(gb + 3 * stepb + KB);
#define MPCR_SSTORE(BUF)                                                                              \
  *(uint4*)&As[BUF][soff + 0 * RPL * LDR] = ga0; *(uint4*)&As[BUF][soff + 1 * RPL * LDR] = ga1;      \
  *(uint4*)&As[BUF][soff + 2 * RPL * LDR] = ga2; *(uint4*)&As[BUF][soff + 3 * RPL * LDR] = ga3;      \
  *(uint4*)&Bs[BUF][soff + 0 * RPL * LDR] = gb0; *(uint4*)&Bs[BUF][soff + 1 * RPL * LDR] = gb1;      \
  *(uint4*)&Bs[BUF][soff + 2 * RPL * LDR] = gb2; *(uint4*)&Bs[BUF][soff + 3 * RPL * LDR] = gb3;

  auto frag = [&](const uint8_t* p) {  // 32 consecutive bytes
    const uint4 lo = *(const uint4*)p, hi = *(const uint4*)(p + 16);
    return i32x8{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
  };
  MPCR_GLOAD(0)
  MPCR_SSTORE(0)
  __syncthreads();
  int cur = 0;
  for (int64_t k0 = 0; k0 < K; k0 += BK) {
    const int64_t kn = k0 + BK < K ? k0 + BK : k0;  // the next stage (the last one reloads itself)
    MPCR_GLOAD(kn)
    const int64_t kb = k0 / 128;
    const int ea = sa_kmajor ? sA[ib * mbA + kb] : sA[kb * mbA + ib];
    const int eb = sb_kmajor ? sB[kb * mbB + jb] : sB[jb * mbB + kb];
    // E8M0 scale bytes 2^(127 - e) (exponents below -127 are outside E8M0's range: clamped)
    const int sca = 127 - ea < 0 ? 0 : (127 - ea > 254 ? 254 : 127 - ea);
    const int scb = 127 - eb < 0 ? 0 : (127 - eb > 254 ? 254 : 127 - eb);
    const uint8_t* Ab = &As[cur][(wm * 128 + g16) * LDR + 32 * q];
    const uint8_t* Bb = &Bs[cur][(wn * TN * 16 + g16) * LDR + 32 * q];
    i32x8 fb[TN];
#pragma unroll
    for (int b = 0; b < TN; ++b) fb[b] = frag(Bb + b * 16 * LDR);
    i32x8 fa = frag(Ab);
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const i32x8 fan = frag(Ab + ((a + 1) & 7) * 16 * LDR);  // the next row block's fragment
#pragma unroll
      for (int b = 0; b < TN; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(fb[b], fa, acc[a][b], 0, 0, 0, scb, 0, sca);
      fa = fan;
    }
    MPCR_SSTORE(cur ^ 1)
    __syncthreads();
    cur ^= 1;
  }
#undef MPCR_GLOAD
#undef MPCR_SSTORE

#pragma unroll
  for (int a = 0; a < 8; ++a)
#pragma unroll
    for (int b = 0; b < TN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t R = r0 + wm * 128 + a * 16 + g16;
        const int64_t Cc = c0 + wn * TN * 16 + b * 16 + 4 * q + r;
        const int64_t idx = Cc * ldc + R;
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

// Packs a rows x cols operand into a k-contiguous array: out[r * ldo + c] =
// element (r, c), read from in[c * ldi + r] (TR) or in[r * ldi + c] (!TR).
// 64 x 64 pieces go through LDS so that both the reads and the writes are
// coalesced.
template <typename T, bool TR>
__global__ __launch_bounds__(256) void k_pack(int64_t rows, int64_t cols, const T* in, int64_t ldi, T* out,
                                              int64_t ldo) {
  __shared__ T t[64][65];
  const int64_t rb = (int64_t)blockIdx.x * 64, cb = (int64_t)blockIdx.y * 64;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int fast = e % 64, slow = e / 64;
    const int r = TR ? fast : slow, c = TR ? slow : fast;
    if (rb + r < rows && cb + c < cols) t[r][c] = TR ? in[(cb + c) * ldi + rb + r] : in[(rb + r) * ldi + cb + c];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int c = e % 64, r = e / 64;
    if (rb + r < rows && cb + c < cols) out[(rb + r) * ldo + cb + c] = t[r][c];
  }
}

hipError_t launch_pack(int es, int trans, int64_t rows, int64_t cols, const void* in, int64_t ldi, void* out,
                       int64_t ldo, hipStream_t s) {
  if (rows == 0 || cols == 0) return hipSuccess;
  dim3 grid((unsigned)((rows + 63) / 64), (unsigned)((cols + 63) / 64));
  if (es == 1) {
    if (trans) k_pack<uint8_t, true><<<grid, 256, 0, s>>>(rows, cols, (const uint8_t*)in, ldi, (uint8_t*)out, ldo);
    else k_pack<uint8_t, false><<<grid, 256, 0, s>>>(rows, cols, (const uint8_t*)in, ldi, (uint8_t*)out, ldo);
  } else {
    if (trans) k_pack<uint16_t, true><<<grid, 256, 0, s>>>(rows, cols, (const uint16_t*)in, ldi, (uint16_t*)out, ldo);
    else k_pack<uint16_t, false><<<grid, 256, 0, s>>>(rows, cols, (const uint16_t*)in, ldi, (uint16_t*)out, ldo);
  }
  return hipGetLastError();
}

hipError_t launch_gemm_lowp(int prec, int64_t m, int64_t n, int64_t k, double alpha, const void* AT, int64_t ldat,
                            const int8_t* sA, int64_t mbA, int sa_kmajor, const void* B, int64_t ldb,
                            const int8_t* sB, int64_t mbB, int sb_kmajor, double beta, void* C, int64_t ldc, int cprec,
                            hipStream_t s) {
  // whole 256 x 256 blocks and 64-wide k stages with 16-byte aligned rows: the large kernel
  if ((prec == BF16 || prec == F16) && m % BG == 0 && n % BG == 0 && k % 64 == 0 && k > 0 && (ldat * 2) % 16 == 0 &&
      (ldb * 2) % 16 == 0 && (uintptr_t)AT % 16 == 0 && (uintptr_t)B % 16 == 0) {
    dim3 g2((unsigned)(m / BG), (unsigned)(n / BG));
    if (prec == BF16) k_gemm_lowp_big<BF16, 4><<<g2, 512, 0, s>>>(m, n, k, alpha, AT, ldat, B, ldb, beta, C, ldc, cprec);
    else k_gemm_lowp_big<F16, 4><<<g2, 512, 0, s>>>(m, n, k, alpha, AT, ldat, B, ldb, beta, C, ldc, cprec);
    return hipGetLastError();
  }
  if (prec == F8 && m % BG == 0 && n % BG == 0 && k % 128 == 0 && k >= 128 && ldat % 16 == 0 && ldb % 16 == 0 &&
      (uintptr_t)AT % 16 == 0 && (uintptr_t)B % 16 == 0) {
    dim3 g2((unsigned)(m / BG), (unsigned)(n / BG));
    k_gemm_fp8_big<<<g2, 512, 0, s>>>(m, n, k, alpha, AT, ldat, sA, mbA, sa_kmajor, B, ldb, sB, mbB, sb_kmajor, beta,
                                      C, ldc, cprec);
    return hipGetLastError();
  }
  dim3 grid((unsigned)((m + GB - 1) / GB), (unsigned)((n + GB - 1) / GB));
  switch (prec) {
    case BF16: k_gemm_lowp<BF16><<<grid, 256, 0, s>>>(m, n, k, alpha, AT, ldat, sA, mbA, B, ldb, sB, mbB, sa_kmajor, sb_kmajor, beta, C, ldc, cprec); break;
    case F16: k_gemm_lowp<F16><<<grid, 256, 0, s>>>(m, n, k, alpha, AT, ldat, sA, mbA, B, ldb, sB, mbB, sa_kmajor, sb_kmajor, beta, C, ldc, cprec); break;
    case F8: k_gemm_lowp<F8><<<grid, 256, 0, s>>>(m, n, k, alpha, AT, ldat, sA, mbA, B, ldb, sB, mbB, sa_kmajor, sb_kmajor, beta, C, ldc, cprec); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_gemm(int prec, int transA, int transB, int64_t m, int64_t n, int64_t k, double alpha, const void* A,
                       int64_t lda, const void* B, int64_t ldb, double beta, void* C, int64_t ldc, int cprec,
                       hipStream_t s) {
  dim3 grid((unsigned)((m + GB - 1) / GB), (unsigned)((n + GB - 1) / GB));
  switch (prec) {
    case F64: k_gemm<F64><<<grid, GTraits<F64>::NW * 64, 0, s>>>(transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, cprec); break;
    case F32: k_gemm<F32><<<grid, GTraits<F32>::NW * 64, 0, s>>>(transA, transB, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, cprec); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace mpcr
