// Tile Cholesky kernels (gfx950).
//
// Right-looking tile Cholesky over nb x nb tiles held in per-tile formats
// (the tiled multi-precision algorithm named in the paper's "Discussion and
// Future Work" section; the factor feeds the log-determinant and the solves
// of the MLE section):
//   POTRF  L_kk = chol(A_kk)                          FP64, one workgroup
//   TRSM   L_ik = A_ik L_kk^{-T}                      FP64 compute, rounded once to p(i,k)
//   SYRK   A_jj -= L_jk L_jk^T                        FP64 MFMA
//   GEMM   A_ij -= L_ik L_jk^T (i > j)                MFMA in the format of tile (i,j)
// Every kernel first checks the device info word and does nothing once a
// pivot has failed, so a whole factorisation can be queued without host syncs.
#include <type_traits>

#include "mpcr_internal.h"

namespace mpcr {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

// MFMA 16x16 lane layouts on gfx950 (checked with an in-bounds probe):
//   operands (f64 16x16x4, f32 16x16x4): lane l holds A[l%16][l/16], B[l/16][l%16]
//   operands (bf16/f16 16x16x32): lane l holds A[l%16][8(l/16) .. 8(l/16)+7], B likewise
//   result f32: lane l, register r -> D[4(l/16) + r][l%16]
//   result f64: lane l, register r -> D[l/16 + 4r][l%16]

// ---------------------------------------------------------------------------
// operand conversion on load (A7a: the update runs in the output tile's format)
// ---------------------------------------------------------------------------
template <int CF> struct CTraits;
template <> struct CTraits<F64> { using T = double; };
template <> struct CTraits<F32> { using T = float; };
template <> struct CTraits<BF16> { using T = uint16_t; };
template <> struct CTraits<F16> { using T = uint16_t; };

template <int CF>
__device__ __forceinline__ typename CTraits<CF>::T load_as(const void* p, int f, int64_t idx) {
  if constexpr (CF == F64) {
    return load_wide(p, f, idx);
  } else if constexpr (CF == F32) {
    if (f == F32) return ((const float*)p)[idx];
    return to_f32(load_wide(p, f, idx));
  } else if constexpr (CF == BF16) {
    if (f == BF16) return ((const uint16_t*)p)[idx];
    if (f == F32) return f32_to_bf16_rne(((const float*)p)[idx]);
    return to_bf16(load_wide(p, f, idx));
  } else {
    if (f == F16) return ((const uint16_t*)p)[idx];
    if (f == F32) return __builtin_bit_cast(uint16_t, (_Float16)((const float*)p)[idx]);
    return to_f16(load_wide(p, f, idx));
  }
}

// ---------------------------------------------------------------------------
// batched tile update  C(i,j) -= A(i,k) B(j,k)^T, one 128 x 128 block of C per
// workgroup (4 waves, 2 x 2, each 64 x 64 = 4 x 4 MFMA tiles of 16 x 16)
// ---------------------------------------------------------------------------
constexpr int UBM = 128;

// Four consecutive elements (idx % 4 == 0) of a tile stored in format SF,
// converted to the compute type of CF with one vector load.
template <int CF, int SF>
__device__ __forceinline__ void load4(const void* p, int64_t idx, typename CTraits<CF>::T out[4]) {
  using T = typename CTraits<CF>::T;
  if constexpr (SF == F64) {
    const double4 v = *(const double4*)((const double*)p + idx);
    const double w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int r = 0; r < 4; ++r) out[r] = (CF == F64) ? (T)w[r] : (T)to_f32(w[r]);
  } else if constexpr (SF == F32) {
    const float4 v = *(const float4*)((const float*)p + idx);
    out[0] = (T)v.x; out[1] = (T)v.y; out[2] = (T)v.z; out[3] = (T)v.w;
  } else if constexpr (SF == F16 || SF == BF16) {
    const ushort4 v = *(const ushort4*)((const uint16_t*)p + idx);
    const uint16_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int r = 0; r < 4; ++r) out[r] = (T)(SF == F16 ? f16_to_f32(w[r]) : bf16_to_f32(w[r]));
  } else {
    const uchar4 v = *(const uchar4*)((const uint8_t*)p + idx);
    const uint8_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int r = 0; r < 4; ++r) out[r] = (T)e4m3_to_f32(w[r]);
  }
}

// C[idx] <- round_f(C[idx] - acc) for the epilogue, with a static format.
template <int F>
__device__ __forceinline__ void rmw_sub(void* Cp, int64_t idx, double acc) {
  if constexpr (F == F64) { double* c = (double*)Cp; c[idx] = c[idx] - acc; }
  else if constexpr (F == F32) { float* c = (float*)Cp; c[idx] = to_f32((double)c[idx] - acc); }
  else if constexpr (F == F16) { uint16_t* c = (uint16_t*)Cp; c[idx] = to_f16((double)f16_to_f32(c[idx]) - acc); }
  else if constexpr (F == BF16) { uint16_t* c = (uint16_t*)Cp; c[idx] = to_bf16((double)bf16_to_f32(c[idx]) - acc); }
  else { uint8_t* c = (uint8_t*)Cp; c[idx] = to_e4m3((double)e4m3_to_f32(c[idx]) - acc); }
}

// FP64 / FP32: operands staged k-major in LDS ([k][m]), double-buffered;
// fragments are contiguous across lanes.  The main loop is instantiated per
// pair of operand formats (one branch per workgroup), so each variant holds
// only its own staging registers.  Shapes (measured on a full-size batch of
// 2016 tile updates): FP64 uses 8 waves of 64 x 32 (the FP64 MFMA is slow
// enough that more waves per CU, not more work per wave, hides the staging),
// FP32 4 waves of 64 x 64 with 16-wide k chunks (four workgroups per CU).
template <int CF> struct KMajor {
  using T = typename CTraits<CF>::T;
  static constexpr int NW = (CF == F64) ? 8 : 4;   // waves per workgroup
  static constexpr int WM = 2;                      // waves along m
  static constexpr int WN = NW / WM;
  static constexpr int TM = UBM / WM, TN = UBM / WN;  // per-wave block
  static constexpr int FM = TM / 16, FN = TN / 16;    // MFMA tiles per wave
  static constexpr int NT = NW * 64;
  static constexpr int BK = 16;
  // row padding: a fragment read covers 4 consecutive k rows of 16 elements;
  // the padding puts those rows on disjoint LDS banks
  static constexpr int PAD = 16;
  static constexpr int LD = UBM * BK / 4 / NT;  // 4-element loads per thread per operand
  using Acc = typename std::conditional<CF == F64, d4, f4>::type;
  using Buf = T[2][BK][UBM + PAD];
};

template <int CF, int FA, int FB>
__device__ __forceinline__ void kmajor_mainloop(const void* Ap, const void* Bp, double ma, double mb, int nb,
                                                int64_t arow0, int64_t brow0,
                                                typename KMajor<CF>::Buf& As, typename KMajor<CF>::Buf& Bs,
                                                typename KMajor<CF>::Acc (&acc)[KMajor<CF>::FM][KMajor<CF>::FN]) {
  using K = KMajor<CF>;
  using T = typename K::T;
  constexpr int BK = K::BK, LD = K::LD, NT = K::NT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave % K::WM, wn = wave / K::WM;
  T ra[LD][4], rb[LD][4];
  // load e = tid + NT g: rows 4 (e % 32) .. +3 of column e / 32 of the chunk
  auto gload = [&](int kk) {
#pragma unroll
    for (int g = 0; g < LD; ++g) {
      const int e = tid + NT * g, r = (e % (UBM / 4)) * 4, k = e / (UBM / 4);
      load4<CF, FA>(Ap, (int64_t)(kk + k) * nb + arow0 + r, ra[g]);
      load4<CF, FB>(Bp, (int64_t)(kk + k) * nb + brow0 + r, rb[g]);
      if constexpr (FA == F8) {  // FP8 tiles hold codes of v 2^s: scale back (exact)
#pragma unroll
        for (int u = 0; u < 4; ++u) ra[g][u] = (T)((double)ra[g][u] * ma);
      }
      if constexpr (FB == F8) {
#pragma unroll
        for (int u = 0; u < 4; ++u) rb[g][u] = (T)((double)rb[g][u] * mb);
      }
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int g = 0; g < LD; ++g) {
      const int e = tid + NT * g, r = (e % (UBM / 4)) * 4, k = e / (UBM / 4);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        As[buf][k][r + u] = ra[g][u];
        Bs[buf][k][r + u] = rb[g][u];
      }
    }
  };
  gload(0);
  sstore(0);
  __syncthreads();
  int cur = 0;
  for (int kk = 0; kk < nb; kk += BK) {
    const bool more = kk + BK < nb;
    if (more) gload(kk + BK);
#pragma unroll
    for (int k4 = 0; k4 < BK; k4 += 4) {
      T av[K::FM], bv[K::FN];
#pragma unroll
      for (int a = 0; a < K::FM; ++a) av[a] = As[cur][k4 + (lane >> 4)][wm * K::TM + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < K::FN; ++b) bv[b] = Bs[cur][k4 + (lane >> 4)][wn * K::TN + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < K::FM; ++a)
#pragma unroll
        for (int b = 0; b < K::FN; ++b) {
          if constexpr (CF == F64)
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
          else
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[b], acc[a][b], 0, 0, 0);
        }
    }
    if (more) sstore(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
}

template <int CF>
__global__ __launch_bounds__(KMajor<CF>::NT) __attribute__((amdgpu_waves_per_eu(CF == F64 ? 2 : 4))) void
k_update_kmajor(TileView tv, int k, const GemmTask* tasks) {
  using K = KMajor<CF>;
  __shared__ __attribute__((aligned(16))) typename K::Buf As;
  __shared__ __attribute__((aligned(16))) typename K::Buf Bs;

  const int nb = tv.nb;
  const int sub = nb / UBM;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int task = lb / (sub * sub);
  const int blk = lb % (sub * sub);
  const int bm = blk % sub, bn = blk / sub;
  const GemmTask t = tasks[task];
  if (t.i == t.j && bn > bm) return;
  if (*tv.info) return;

  const void* Ap = tv.tile(t.i, k);
  const void* Bp = tv.tile(t.j, k);
  const int fa = tv.tfmt(t.i, k), fb = tv.tfmt(t.j, k);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave % K::WM, wn = wave / K::WM;
  const int64_t arow0 = (int64_t)bm * UBM, brow0 = (int64_t)bn * UBM;

  typename K::Acc acc[K::FM][K::FN];
#pragma unroll
  for (int a = 0; a < K::FM; ++a)
#pragma unroll
    for (int b = 0; b < K::FN; ++b) acc[a][b] = typename K::Acc{0, 0, 0, 0};

  // operand tiles in any format (codes 0..4; FP8 operands carry their scale)
  const double ma = tv.tmul(t.i, k), mb = tv.tmul(t.j, k);
#define MPCR_PAIR(FA, FB) \
  case FA * 5 + FB: kmajor_mainloop<CF, FA, FB>(Ap, Bp, ma, mb, nb, arow0, brow0, As, Bs, acc); break;
#define MPCR_ROW(FA) MPCR_PAIR(FA, F64) MPCR_PAIR(FA, F32) MPCR_PAIR(FA, F16) MPCR_PAIR(FA, BF16) MPCR_PAIR(FA, F8)
  switch (fa * 5 + fb) {
    MPCR_ROW(F64)
    MPCR_ROW(F32)
    MPCR_ROW(F16)
    MPCR_ROW(BF16)
    MPCR_ROW(F8)
    default: break;
  }
#undef MPCR_ROW
#undef MPCR_PAIR

  void* Cp = tv.tile(t.i, t.j);
  const int fc = tv.tfmt(t.i, t.j);
  const bool diag = (t.i == t.j);
  auto epilogue = [&](auto fmt_tag) {
    constexpr int FC = decltype(fmt_tag)::value;
#pragma unroll
    for (int a = 0; a < K::FM; ++a)
#pragma unroll
      for (int b = 0; b < K::FN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          int row = (CF == F64) ? ((lane >> 4) + 4 * r) : (4 * (lane >> 4) + r);
          int64_t R = arow0 + wm * K::TM + a * 16 + row;
          int64_t C = brow0 + wn * K::TN + b * 16 + (lane & 15);
          if (diag && C > R) continue;
          rmw_sub<FC>(Cp, C * nb + R, (double)acc[a][b][r]);
        }
  };
  switch (fc) {
    case F64: epilogue(std::integral_constant<int, F64>{}); break;
    case F32: epilogue(std::integral_constant<int, F32>{}); break;
    case F16: epilogue(std::integral_constant<int, F16>{}); break;
    case BF16: epilogue(std::integral_constant<int, BF16>{}); break;
    default: epilogue(std::integral_constant<int, F8>{}); break;
  }
}

// BF16 / FP16: operands staged m-major in LDS ([m][k]) so that each lane reads
// its 8 consecutive k values with one 16-byte load.  The column-major tiles
// are read 8 rows at a time (one vector load per column), converted to the
// compute format and scattered into 8 LDS rows; LDS is double-buffered and
// the main loop is instantiated per pair of operand formats.
template <int CF, int SF>
__device__ __forceinline__ void load8_16(const void* p, int64_t idx, uint16_t out[8], double mul) {
  auto cvt = [](double x) -> uint16_t { return CF == BF16 ? to_bf16(x) : to_f16(x); };
  if constexpr (SF == CF) {
    const u16x8 v = *(const u16x8*)((const uint16_t*)p + idx);
#pragma unroll
    for (int e = 0; e < 8; ++e) out[e] = v[e];
  } else if constexpr (SF == F64) {
    const double4 v0 = *(const double4*)((const double*)p + idx), v1 = *(const double4*)((const double*)p + idx + 4);
    const double w[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
    for (int e = 0; e < 8; ++e) out[e] = cvt(w[e]);
  } else if constexpr (SF == F32) {
    const float4 v0 = *(const float4*)((const float*)p + idx), v1 = *(const float4*)((const float*)p + idx + 4);
    const float w[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
    for (int e = 0; e < 8; ++e) out[e] = CF == BF16 ? f32_to_bf16_rne(w[e]) : __builtin_bit_cast(uint16_t, (_Float16)w[e]);
  } else if constexpr (SF == F8) {  // codes of v 2^s: widen, scale back (mul = 2^-s), round once
    const uint2 v = *(const uint2*)((const uint8_t*)p + idx);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const uint8_t c = (uint8_t)(((e < 4 ? v.x : v.y) >> (8 * (e & 3))) & 0xffu);
      out[e] = cvt((double)e4m3_to_f32(c) * mul);
    }
  } else {  // the other 16-bit format: widen exactly, round once
    const u16x8 v = *(const u16x8*)((const uint16_t*)p + idx);
#pragma unroll
    for (int e = 0; e < 8; ++e) out[e] = cvt((double)(SF == F16 ? f16_to_f32(v[e]) : bf16_to_f32(v[e])));
  }
}

constexpr int MBK = 64;        // k per chunk
constexpr int MLDK = MBK + 8;  // LDS row (halfwords)

template <int CF, int FA, int FB>
__device__ __forceinline__ void mmajor_mainloop(const void* Ap, const void* Bp, double ma, double mb, int nb,
                                                int64_t arow0, int64_t brow0,
                                                uint16_t (&As)[2][UBM][MLDK], uint16_t (&Bs)[2][UBM][MLDK],
                                                f4 (&acc)[4][4]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int rg = tid & 15;  // rows 8 rg .. 8 rg + 7
  const int kq = tid >> 4;  // k = kq + 16 g
  uint16_t ra[4][8], rb[4][8];
  auto gload = [&](int kk) {
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int64_t col = kk + kq + 16 * g;
      load8_16<CF, FA>(Ap, col * nb + arow0 + 8 * rg, ra[g], ma);
      load8_16<CF, FB>(Bp, col * nb + brow0 + 8 * rg, rb[g], mb);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int g = 0; g < 4; ++g)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        As[buf][8 * rg + e][kq + 16 * g] = ra[g][e];
        Bs[buf][8 * rg + e][kq + 16 * g] = rb[g][e];
      }
  };
  gload(0);
  sstore(0);
  __syncthreads();
  int cur = 0;
  for (int kk = 0; kk < nb; kk += MBK) {
    const bool more = kk + MBK < nb;
    if (more) gload(kk + MBK);
#pragma unroll
    for (int k32 = 0; k32 < MBK; k32 += 32) {
      u16x8 av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = *(const u16x8*)&As[cur][wm * 64 + a * 16 + (lane & 15)][k32 + 8 * (lane >> 4)];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = *(const u16x8*)&Bs[cur][wn * 64 + b * 16 + (lane & 15)][k32 + 8 * (lane >> 4)];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          if constexpr (CF == BF16)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, av[a]),
                                                                 __builtin_bit_cast(bf16x8, bv[b]), acc[a][b], 0, 0, 0);
          else
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, av[a]),
                                                                __builtin_bit_cast(f16x8, bv[b]), acc[a][b], 0, 0, 0);
        }
    }
    if (more) sstore(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
}

template <int CF>
__global__ __launch_bounds__(256) void k_update_mmajor(TileView tv, int k, const GemmTask* tasks) {
  __shared__ __attribute__((aligned(16))) uint16_t As[2][UBM][MLDK];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[2][UBM][MLDK];

  const int nb = tv.nb;
  const int sub = nb / UBM;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int task = lb / (sub * sub);
  const int blk = lb % (sub * sub);
  const int bm = blk % sub, bn = blk / sub;
  const GemmTask t = tasks[task];
  if (t.i == t.j && bn > bm) return;
  if (*tv.info) return;

  const void* Ap = tv.tile(t.i, k);
  const void* Bp = tv.tile(t.j, k);
  const int fa = tv.tfmt(t.i, k), fb = tv.tfmt(t.j, k);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int64_t arow0 = (int64_t)bm * UBM, brow0 = (int64_t)bn * UBM;

  f4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f4{0, 0, 0, 0};

  const double ma = tv.tmul(t.i, k), mb = tv.tmul(t.j, k);
#define MPCR_PAIR(FA, FB) \
  case FA * 5 + FB: mmajor_mainloop<CF, FA, FB>(Ap, Bp, ma, mb, nb, arow0, brow0, As, Bs, acc); break;
#define MPCR_ROW(FA) MPCR_PAIR(FA, F64) MPCR_PAIR(FA, F32) MPCR_PAIR(FA, F16) MPCR_PAIR(FA, BF16) MPCR_PAIR(FA, F8)
  switch (fa * 5 + fb) {
    MPCR_ROW(F64)
    MPCR_ROW(F32)
    MPCR_ROW(F16)
    MPCR_ROW(BF16)
    MPCR_ROW(F8)
    default: break;
  }
#undef MPCR_ROW
#undef MPCR_PAIR

  void* Cp = tv.tile(t.i, t.j);  // in format CF (the update runs in the output tile's format)
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int64_t R = arow0 + wm * 64 + a * 16 + 4 * (lane >> 4) + r;
        int64_t C = brow0 + wn * 64 + b * 16 + (lane & 15);
        rmw_sub<CF>(Cp, C * nb + R, (double)acc[a][b][r]);
      }
}

// ---------------------------------------------------------------------------
// FP32 output tiles through the BF16 MFMA.  gfx950's dense BF16 rate is 16
// times its FP32 rate, so an FP32 product can be formed from BF16 pieces:
// each operand, converted to FP32 as in the FP32 update, is split exactly
// into three BF16 numbers x = h + m + l (h = bf16(x), m = bf16(x - h),
// l = x - h - m; every difference is exact by Sterbenz's lemma and l needs at
// most 8 significant bits), and a b is accumulated as
//   ah bh + ah bm + am bh + ah bl + al bh + am bm
// in FP32 on v_mfma_f32_16x16x32_bf16 (which returns the exact FP32-rounded
// sums).  The three dropped products am bl + al bm + al bl are below
// 2^-23 |a b|, so every update keeps FP32-level accuracy; the output tile is
// rounded to FP32 as in the FP32 update.  One 128 x 128 block of C per
// workgroup, 8 waves of 64 x 32, k chunks of 32; the three planes of both
// operands (61 KB) sit in one LDS buffer so that two workgroups share a CU.
// ---------------------------------------------------------------------------
constexpr int SBK = 32;          // k per chunk
constexpr int SLDK = SBK + 8;    // LDS row (halfwords): 80-byte rows put the 16 rows of a fragment read on disjoint banks

__device__ __forceinline__ void split3_bf16(float x, uint16_t& h, uint16_t& m, uint16_t& l) {
  // finite inputs: round to nearest even by adding half an ulp (ties to even)
  uint32_t u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  h = (uint16_t)(u >> 16);
  const float r1 = x - __uint_as_float((uint32_t)h << 16);
  uint32_t v = __float_as_uint(r1);
  v += 0x7fffu + ((v >> 16) & 1u);
  m = (uint16_t)(v >> 16);
  const float r2 = r1 - __uint_as_float((uint32_t)m << 16);
  l = (uint16_t)(__float_as_uint(r2) >> 16);  // r2 has at most 8 significant bits: exact
}

// element idx of a tile (format SF) converted to FP32 (FP8 codes scaled back
// by mul = 2^-s)
template <int SF>
__device__ __forceinline__ float load1_f32(const void* p, int64_t idx, double mul) {
  if constexpr (SF == F64) return to_f32(((const double*)p)[idx]);
  else if constexpr (SF == F32) return ((const float*)p)[idx];
  else if constexpr (SF == F16) return f16_to_f32(((const uint16_t*)p)[idx]);
  else if constexpr (SF == BF16) return bf16_to_f32(((const uint16_t*)p)[idx]);
  else return to_f32((double)e4m3_to_f32(((const uint8_t*)p)[idx]) * mul);
}

using SplitBuf = uint16_t[3][UBM][SLDK];

template <int FA, int FB>
__device__ __forceinline__ void split_mainloop(const void* Ap, const void* Bp, double ma, double mb, int nb,
                                               int64_t arow0, int64_t brow0, SplitBuf& As, SplitBuf& Bs,
                                               f4 (&acc)[4][2]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  // staging: thread = one row (m) and 8 consecutive k of the chunk; a load
  // instruction covers 64 consecutive rows of one k column (coalesced), and
  // the split values go to LDS as one 16-byte vector per plane
  const int mr = tid & (UBM - 1);
  const int k0 = 8 * (tid / UBM);
  float ra[8], rb[8];
  auto gload = [&](int kk) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t col = kk + k0 + e;
      ra[e] = load1_f32<FA>(Ap, col * nb + arow0 + mr, ma);
      rb[e] = load1_f32<FB>(Bp, col * nb + brow0 + mr, mb);
    }
  };
  auto sstore = [&]() {
    u16x8 ah, am, al, bh, bm, bl;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      uint16_t h, m, l;
      split3_bf16(ra[e], h, m, l);
      ah[e] = h;
      am[e] = m;
      al[e] = l;
      split3_bf16(rb[e], h, m, l);
      bh[e] = h;
      bm[e] = m;
      bl[e] = l;
    }
    *(u16x8*)&As[0][mr][k0] = ah;
    *(u16x8*)&As[1][mr][k0] = am;
    *(u16x8*)&As[2][mr][k0] = al;
    *(u16x8*)&Bs[0][mr][k0] = bh;
    *(u16x8*)&Bs[1][mr][k0] = bm;
    *(u16x8*)&Bs[2][mr][k0] = bl;
  };
  gload(0);
  sstore();
  __syncthreads();
  const int kq8 = 8 * (lane >> 4);
  // one LDS buffer (two workgroups per CU): the next chunk is loaded into
  // registers during this chunk's products and stored after a barrier
  for (int kk = 0; kk < nb; kk += SBK) {
    const bool more = kk + SBK < nb;
    if (more) gload(kk + SBK);
    u16x8 a[3][4], b[3][2];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
#pragma unroll
      for (int x = 0; x < 4; ++x) a[p][x] = *(const u16x8*)&As[p][wm * 64 + x * 16 + (lane & 15)][kq8];
#pragma unroll
      for (int y = 0; y < 2; ++y) b[p][y] = *(const u16x8*)&Bs[p][wn * 32 + y * 16 + (lane & 15)][kq8];
    }
#define MPCR_MF(PA, PB)                                                                                   \
  acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[PA][x]),              \
                                                      __builtin_bit_cast(bf16x8, b[PB][y]), acc[x][y], 0, 0, 0)
    // the small products first, the leading one last
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < 2; ++y) {
        MPCR_MF(1, 1);
        MPCR_MF(0, 2);
        MPCR_MF(2, 0);
        MPCR_MF(0, 1);
        MPCR_MF(1, 0);
        MPCR_MF(0, 0);
      }
#undef MPCR_MF
    if (more) {
      __syncthreads();
      sstore();
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(512) void k_update_f32_split(TileView tv, int k, const GemmTask* tasks) {
  __shared__ __attribute__((aligned(16))) SplitBuf As;
  __shared__ __attribute__((aligned(16))) SplitBuf Bs;

  const int nb = tv.nb;
  const int sub = nb / UBM;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int task = lb / (sub * sub);
  const int blk = lb % (sub * sub);
  const int bm = blk % sub, bn = blk / sub;
  const GemmTask t = tasks[task];
  if (t.i == t.j && bn > bm) return;
  if (*tv.info) return;

  const void* Ap = tv.tile(t.i, k);
  const void* Bp = tv.tile(t.j, k);
  const int fa = tv.tfmt(t.i, k), fb = tv.tfmt(t.j, k);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int64_t arow0 = (int64_t)bm * UBM, brow0 = (int64_t)bn * UBM;

  f4 acc[4][2];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) acc[x][y] = f4{0, 0, 0, 0};

  const double ma = tv.tmul(t.i, k), mb = tv.tmul(t.j, k);
#define MPCR_PAIR(FA, FB) \
  case FA * 5 + FB: split_mainloop<FA, FB>(Ap, Bp, ma, mb, nb, arow0, brow0, As, Bs, acc); break;
#define MPCR_ROW(FA) MPCR_PAIR(FA, F64) MPCR_PAIR(FA, F32) MPCR_PAIR(FA, F16) MPCR_PAIR(FA, BF16) MPCR_PAIR(FA, F8)
  switch (fa * 5 + fb) {
    MPCR_ROW(F64)
    MPCR_ROW(F32)
    MPCR_ROW(F16)
    MPCR_ROW(BF16)
    MPCR_ROW(F8)
    default: break;
  }
#undef MPCR_ROW
#undef MPCR_PAIR

  void* Cp = tv.tile(t.i, t.j);  // FP32 (the update runs in the output tile's format)
  const bool diag = (t.i == t.j);
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t R = arow0 + wm * 64 + x * 16 + 4 * (lane >> 4) + r;
        const int64_t C = brow0 + wn * 32 + y * 16 + (lane & 15);
        if (diag && C > R) continue;
        rmw_sub<F32>(Cp, C * nb + R, (double)acc[x][y][r]);
      }
}

// Split panels: after the TRSM of step k, every panel tile (i, k) is converted
// to FP32 and split once into its three BF16 planes, stored for the update
// kernel in chunks of 32 k: plane p of panel tile q = i - k - 1 at
//   out3[(q * 3 + p) * nb^2 + (c * nb + row) * 32 + kk]   (k = 32 c + kk),
// so a 128-row block of one chunk is 8 contiguous KB.  The FP32 updates of the
// step then copy planes instead of splitting every operand in every block.
// outb (when not NULL) receives, in the same layout, each element rounded once
// to BF16 from its stored format: the operands of the step's BF16 updates.
template <int SF>
__device__ __forceinline__ uint16_t load1_bf16(const void* p, int64_t idx, double mul) {
  if constexpr (SF == BF16) return ((const uint16_t*)p)[idx];
  else if constexpr (SF == F32) return f32_to_bf16_rne(((const float*)p)[idx]);
  else if constexpr (SF == F64) return to_bf16(((const double*)p)[idx]);
  else if constexpr (SF == F16) return to_bf16((double)f16_to_f32(((const uint16_t*)p)[idx]));
  else return to_bf16((double)e4m3_to_f32(((const uint8_t*)p)[idx]) * mul);
}

__global__ __launch_bounds__(512) void k_pack_split(TileView tv, int k, uint16_t* out3, uint16_t* outb) {
  const int nb = tv.nb, nch = nb / SBK, nrb = nb / UBM;
  const int b = blockIdx.x;
  const int q = b / (nch * nrb), c = (b / nrb) % nch, rb = b % nrb;
  const int i = k + 1 + q;
  const void* P = tv.tile(i, k);
  const int f = tv.tfmt(i, k);
  const double mul = tv.tmul(i, k);
  const int mr = threadIdx.x & (UBM - 1), k0 = 8 * (threadIdx.x / UBM);
  const int64_t row = (int64_t)rb * UBM + mr;
  const int64_t nb2 = (int64_t)nb * nb;
  const int64_t at = ((int64_t)c * nb + row) * SBK + k0;
  float v[8];
  u16x8 bv;
  auto load = [&](auto tag) {
    constexpr int SF = decltype(tag)::value;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t idx = (int64_t)(SBK * c + k0 + e) * nb + row;
      if (out3) v[e] = load1_f32<SF>(P, idx, mul);
      if (outb) bv[e] = load1_bf16<SF>(P, idx, mul);
    }
  };
  switch (f) {
    case F64: load(std::integral_constant<int, F64>{}); break;
    case F32: load(std::integral_constant<int, F32>{}); break;
    case F16: load(std::integral_constant<int, F16>{}); break;
    case BF16: load(std::integral_constant<int, BF16>{}); break;
    default: load(std::integral_constant<int, F8>{}); break;
  }
  if (outb) *(u16x8*)(outb + (int64_t)q * nb2 + at) = bv;
  if (out3) {
    u16x8 h, m, l;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      uint16_t a, bb, cc;
      split3_bf16(v[e], a, bb, cc);
      h[e] = a;
      m[e] = bb;
      l[e] = cc;
    }
    uint16_t* o = out3 + (int64_t)q * 3 * nb2 + at;
    *(u16x8*)o = h;
    *(u16x8*)(o + nb2) = m;
    *(u16x8*)(o + 2 * nb2) = l;
  }
}

hipError_t launch_pack_split(const TileView& tv, int k, uint16_t* out3, uint16_t* outb, hipStream_t s) {
  const int cnt = tv.nt - k - 1;
  if (cnt <= 0 || (!out3 && !outb)) return hipSuccess;
  k_pack_split<<<cnt * (tv.nb / SBK) * (tv.nb / UBM), 512, 0, s>>>(tv, k, out3, outb);
  return hipGetLastError();
}

// Updates from the packed panels of step k (see k_pack_split), planes copied
// with 16-byte loads (four per row of a chunk).  NPL = 3: FP32 output tiles,
// the six split products of k_update_f32_split; NPL = 1: BF16 output tiles,
// one BF16 product per fragment pair on operands rounded once to BF16 (the
// same k order of MFMAs as k_update_mmajor<BF16>, so the same results).  NW waves per 128 x 128 block: 8 waves of 64 x 32 or
// 4 waves of 64 x 64; both run at the same rate in the factorisation (about
// 112 TF/s FP32-equivalent at n = 32768), where the three planes (6 bytes per
// operand element) make the operand stream, not the LDS or the MFMA, the limit.
constexpr int SPLIT_WAVES = 8;

template <int NW, int NPL>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW == 8 ? 4 : 2))) void
k_update_packed(TileView tv, int k, const GemmTask* tasks, const uint16_t* split) {
  constexpr int NT = 64 * NW;
  constexpr int WN = NW / 2;             // waves along n (2 along m)
  constexpr int FY = (UBM / WN) / 16;    // 16-column MFMA tiles per wave along n
  constexpr int G = NPL * UBM * 4 / NT;  // 16-byte vectors per thread per operand and chunk
  constexpr int CF = NPL == 3 ? F32 : BF16;
  __shared__ __attribute__((aligned(16))) uint16_t As[NPL][UBM][SLDK];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[NPL][UBM][SLDK];

  const int nb = tv.nb;
  const int sub = nb / UBM;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int task = lb / (sub * sub);
  const int blk = lb % (sub * sub);
  const int bm = blk % sub, bn = blk / sub;
  const GemmTask t = tasks[task];
  if (t.i == t.j && bn > bm) return;
  if (*tv.info) return;

  const int64_t nb2 = (int64_t)nb * nb;
  const uint16_t* Ap = split + (int64_t)(t.i - k - 1) * NPL * nb2;
  const uint16_t* Bp = split + (int64_t)(t.j - k - 1) * NPL * nb2;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int64_t arow0 = (int64_t)bm * UBM, brow0 = (int64_t)bn * UBM;

  f4 acc[4][FY];
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < FY; ++y) acc[x][y] = f4{0, 0, 0, 0};

  // vector v = tid + NT g: plane v / 512, row (v % 512) / 4, k offset 8 (v % 4)
  u16x8 ra[G], rb[G];
  auto gload = [&](int kk) {
    const int64_t c = kk / SBK;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int v = tid + NT * g, p = v / (UBM * 4), r = (v % (UBM * 4)) >> 2, k0 = 8 * (v & 3);
      ra[g] = *(const u16x8*)(Ap + p * nb2 + (c * nb + arow0 + r) * SBK + k0);
      rb[g] = *(const u16x8*)(Bp + p * nb2 + (c * nb + brow0 + r) * SBK + k0);
    }
  };
  auto sstore = [&]() {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int v = tid + NT * g, p = v / (UBM * 4), r = (v % (UBM * 4)) >> 2, k0 = 8 * (v & 3);
      *(u16x8*)&As[p][r][k0] = ra[g];
      *(u16x8*)&Bs[p][r][k0] = rb[g];
    }
  };
  gload(0);
  sstore();
  __syncthreads();
  const int kq8 = 8 * (lane >> 4);
  for (int kk = 0; kk < nb; kk += SBK) {
    const bool more = kk + SBK < nb;
    if (more) gload(kk + SBK);
    u16x8 a[NPL][4], b[NPL][FY];
#pragma unroll
    for (int p = 0; p < NPL; ++p) {
#pragma unroll
      for (int x = 0; x < 4; ++x) a[p][x] = *(const u16x8*)&As[p][wm * 64 + x * 16 + (lane & 15)][kq8];
#pragma unroll
      for (int y = 0; y < FY; ++y) b[p][y] = *(const u16x8*)&Bs[p][wn * (16 * FY) + y * 16 + (lane & 15)][kq8];
    }
#define MPCR_MF(PA, PB)                                                                                   \
  acc[x][y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a[PA][x]),              \
                                                      __builtin_bit_cast(bf16x8, b[PB][y]), acc[x][y], 0, 0, 0)
#pragma unroll
    for (int x = 0; x < 4; ++x)
#pragma unroll
      for (int y = 0; y < FY; ++y) {
        if constexpr (NPL == 3) {
          MPCR_MF(1, 1);
          MPCR_MF(0, 2);
          MPCR_MF(2, 0);
          MPCR_MF(0, 1);
          MPCR_MF(1, 0);
        }
        MPCR_MF(0, 0);
      }
#undef MPCR_MF
    if (more) {
      __syncthreads();
      sstore();
      __syncthreads();
    }
  }

  void* Cp = tv.tile(t.i, t.j);
  const bool diag = (t.i == t.j);
#pragma unroll
  for (int x = 0; x < 4; ++x)
#pragma unroll
    for (int y = 0; y < FY; ++y)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t R = arow0 + wm * 64 + x * 16 + 4 * (lane >> 4) + r;
        const int64_t C = brow0 + wn * (16 * FY) + y * 16 + (lane & 15);
        if (diag && C > R) continue;
        rmw_sub<CF>(Cp, C * nb + R, (double)acc[x][y][r]);
      }
}

hipError_t launch_tile_update_packed(const TileView& tv, int k, int cfmt, const GemmTask* tasks, int ntasks,
                                     const uint16_t* planes, hipStream_t s) {
  if (ntasks == 0) return hipSuccess;
  const int sub = tv.nb / UBM;
  if (cfmt == F32)
    k_update_packed<SPLIT_WAVES, 3><<<ntasks * sub * sub, 64 * SPLIT_WAVES, 0, s>>>(tv, k, tasks, planes);
  else if (cfmt == BF16)
    k_update_packed<8, 1><<<ntasks * sub * sub, 512, 0, s>>>(tv, k, tasks, planes);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Updates of FP8 output tiles (the update runs in the output tile's format):
// both operands are converted to FP8 on load with the scale of their own tile
// (a stored FP8 tile keeps its codes; any other operand tile (i, k) is
// quantised with the scale that its largest magnitude pamax[i] gives), the
// products accumulate in FP32 through v_mfma_f32_16x16x32_fp8_fp8, and the new
// tile C - 2^-(sA+sB) acc is formed in FP64 and staged in FP32 by round-to-odd
// with its largest magnitude; k_requant_f8 then rounds it once to FP8 with the
// scale of that maximum (the two roundings equal one: FP32 keeps two more bits
// than E4M3 needs).
// ---------------------------------------------------------------------------
constexpr int FBK = 128;           // k per chunk
constexpr int FLDK = FBK + 16;     // LDS row (bytes)

template <int SF>
__device__ __forceinline__ void load8_f8(const void* p, int64_t idx, uint8_t out[8], double qs) {
  if constexpr (SF == F8) {
    const uint2 v = *(const uint2*)((const uint8_t*)p + idx);
#pragma unroll
    for (int e = 0; e < 8; ++e) out[e] = (uint8_t)(((e < 4 ? v.x : v.y) >> (8 * (e & 3))) & 0xffu);
  } else if constexpr (SF == F64) {
    const double4 v0 = *(const double4*)((const double*)p + idx), v1 = *(const double4*)((const double*)p + idx + 4);
    const double w[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
    for (int e = 0; e < 8; ++e) out[e] = to_e4m3(w[e] * qs);
  } else if constexpr (SF == F32) {
    const float4 v0 = *(const float4*)((const float*)p + idx), v1 = *(const float4*)((const float*)p + idx + 4);
    const float w[8] = {v0.x, v0.y, v0.z, v0.w, v1.x, v1.y, v1.z, v1.w};
#pragma unroll
    for (int e = 0; e < 8; ++e) out[e] = to_e4m3((double)w[e] * qs);
  } else {
    const u16x8 v = *(const u16x8*)((const uint16_t*)p + idx);
#pragma unroll
    for (int e = 0; e < 8; ++e) out[e] = to_e4m3((double)(SF == F16 ? f16_to_f32(v[e]) : bf16_to_f32(v[e])) * qs);
  }
}

template <int FA, int FB>
__device__ __forceinline__ void f8_mainloop(const void* Ap, const void* Bp, double qa, double qb, int nb, int64_t arow0,
                                            int64_t brow0, uint8_t (&As)[2][UBM][FLDK], uint8_t (&Bs)[2][UBM][FLDK],
                                            f4 (&acc)[4][4]) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int rg = tid & 15;  // rows 8 rg .. 8 rg + 7
  const int kq = tid >> 4;  // k = kq + 16 g, g = 0 .. 7
  uint8_t ra[8][8], rb[8][8];
  auto gload = [&](int kk) {
#pragma unroll
    for (int g = 0; g < FBK / 16; ++g) {
      const int64_t col = kk + kq + 16 * g;
      load8_f8<FA>(Ap, col * nb + arow0 + 8 * rg, ra[g], qa);
      load8_f8<FB>(Bp, col * nb + brow0 + 8 * rg, rb[g], qb);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int g = 0; g < FBK / 16; ++g)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        As[buf][8 * rg + e][kq + 16 * g] = ra[g][e];
        Bs[buf][8 * rg + e][kq + 16 * g] = rb[g][e];
      }
  };
  gload(0);
  sstore(0);
  __syncthreads();
  int cur = 0;
  for (int kk = 0; kk < nb; kk += FBK) {
    const bool more = kk + FBK < nb;
    if (more) gload(kk + FBK);
#pragma unroll
    for (int k32 = 0; k32 < FBK; k32 += 32) {
      long av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = *(const long*)&As[cur][wm * 64 + a * 16 + (lane & 15)][k32 + 8 * (lane >> 4)];
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = *(const long*)&Bs[cur][wn * 64 + b * 16 + (lane & 15)][k32 + 8 * (lane >> 4)];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    if (more) sstore(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
}

// scale exponent of operand tile (i, k) as an FP8 operand
__device__ __forceinline__ int operand_f8_scale(const TileView& tv, int i, int k, const double* pamax) {
  return tv.tfmt(i, k) == F8 ? tv.tscale(i, k) : fp8_scale_exp(pamax[i]);
}

__global__ __launch_bounds__(256) void k_update_f8(TileView tv, int k, const GemmTask* tasks, const double* pamax,
                                                   float* ws32, unsigned* amax32) {
  __shared__ __attribute__((aligned(16))) uint8_t As[2][UBM][FLDK];
  __shared__ __attribute__((aligned(16))) uint8_t Bs[2][UBM][FLDK];
  __shared__ float red[256];
  const int nb = tv.nb;
  const int sub = nb / UBM;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int task = lb / (sub * sub);
  const int blk = lb % (sub * sub);
  const int bm = blk % sub, bn = blk / sub;
  const GemmTask t = tasks[task];
  if (*tv.info) return;

  const void* Ap = tv.tile(t.i, k);
  const void* Bp = tv.tile(t.j, k);
  const int fa = tv.tfmt(t.i, k), fb = tv.tfmt(t.j, k);
  const int sa = operand_f8_scale(tv, t.i, k, pamax), sb = operand_f8_scale(tv, t.j, k, pamax);
  const double qa = ldexp(1.0, sa), qb = ldexp(1.0, sb);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int64_t arow0 = (int64_t)bm * UBM, brow0 = (int64_t)bn * UBM;

  f4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f4{0, 0, 0, 0};
#define MPCR_PAIR(FA, FB) \
  case FA * 5 + FB: f8_mainloop<FA, FB>(Ap, Bp, qa, qb, nb, arow0, brow0, As, Bs, acc); break;
#define MPCR_ROW(FA) MPCR_PAIR(FA, F64) MPCR_PAIR(FA, F32) MPCR_PAIR(FA, F16) MPCR_PAIR(FA, BF16) MPCR_PAIR(FA, F8)
  switch (fa * 5 + fb) {
    MPCR_ROW(F64)
    MPCR_ROW(F32)
    MPCR_ROW(F16)
    MPCR_ROW(BF16)
    MPCR_ROW(F8)
    default: break;
  }
#undef MPCR_ROW
#undef MPCR_PAIR

  const uint8_t* Cp = (const uint8_t*)tv.tile(t.i, t.j);
  const double mc = ldexp(1.0, -tv.tscale(t.i, t.j)), mp = ldexp(1.0, -(sa + sb));
  float* W = ws32 + (int64_t)task * nb * nb;
  float m = 0.0f;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t R = arow0 + wm * 64 + a * 16 + 4 * (lane >> 4) + r;
        const int64_t C = brow0 + wn * 64 + b * 16 + (lane & 15);
        const int64_t idx = C * nb + R;
        const float v = round_odd_f32((double)e4m3_to_f32(Cp[idx]) * mc - (double)acc[a][b][r] * mp);
        W[idx] = v;
        m = fmaxf(m, fabsf(v));
      }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicMax(&amax32[task], __float_as_uint(red[0]));  // non-negative floats order as integers
}

// one workgroup per (FP8 task, 16-column slab): round the staged tile once to FP8
__global__ __launch_bounds__(256) void k_requant_f8(TileView tv, const GemmTask* tasks, const float* ws32,
                                                    const unsigned* amax32) {
  if (*tv.info) return;
  const int nb = tv.nb, slabs = nb / 16;
  const int task = blockIdx.x / slabs, c0 = (blockIdx.x % slabs) * 16;
  const GemmTask t = tasks[task];
  const int s = fp8_scale_exp((double)__uint_as_float(amax32[task]));
  uint8_t* Cp = (uint8_t*)tv.tile(t.i, t.j);
  const float* W = ws32 + (int64_t)task * nb * nb;
  for (int e = threadIdx.x; e < 16 * nb; e += 256) {
    const int64_t idx = (int64_t)(c0 + e / nb) * nb + e % nb;
    Cp[idx] = to_e4m3(ldexp((double)W[idx], s));
  }
  if (blockIdx.x % slabs == 0 && threadIdx.x == 0) tv.sc[tri_index(t.i, t.j)] = (int8_t)s;
}

__global__ void k_zero_u32(unsigned* p, int n) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) p[i] = 0u;
}

hipError_t launch_tile_update_fp8(const TileView& tv, int k, const GemmTask* tasks, int ntasks, const double* pamax,
                                  float* ws32, unsigned* amax32, hipStream_t s) {
  if (ntasks == 0) return hipSuccess;
  const int sub = tv.nb / UBM;
  k_zero_u32<<<(ntasks + 255) / 256, 256, 0, s>>>(amax32, ntasks);
  k_update_f8<<<ntasks * sub * sub, 256, 0, s>>>(tv, k, tasks, pamax, ws32, amax32);
  k_requant_f8<<<ntasks * (tv.nb / 16), 256, 0, s>>>(tv, tasks, ws32, amax32);
  return hipGetLastError();
}

// largest magnitude of each panel tile (i, k), i > k (widened values)
__global__ __launch_bounds__(256) void k_panel_amax(TileView tv, int k, double* pamax) {
  const int i = k + 1 + blockIdx.x;
  const int nb = tv.nb;
  const void* P = tv.tile(i, k);
  const int f = tv.tfmt(i, k);
  __shared__ double red[256];
  double m = 0.0;
  for (int64_t e = threadIdx.x; e < (int64_t)nb * nb; e += 256) m = fmax(m, fabs(load_wide(P, f, e)));
  red[threadIdx.x] = m * tv.tmul(i, k);
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) pamax[i] = red[0];
}

hipError_t launch_panel_amax(const TileView& tv, int k, double* pamax, hipStream_t s) {
  const int cnt = tv.nt - k - 1;
  if (cnt <= 0) return hipSuccess;
  k_panel_amax<<<cnt, 256, 0, s>>>(tv, k, pamax);
  return hipGetLastError();
}

hipError_t launch_tile_update(const TileView& tv, int k, int cfmt, const GemmTask* tasks, int ntasks,
                              hipStream_t s, bool fp32_split) {
  if (ntasks == 0) return hipSuccess;
  const int sub = tv.nb / UBM;
  dim3 grid(ntasks * sub * sub);
  switch (cfmt) {
    case F64: k_update_kmajor<F64><<<grid, KMajor<F64>::NT, 0, s>>>(tv, k, tasks); break;
    case F32:
      if (fp32_split)
        k_update_f32_split<<<grid, 512, 0, s>>>(tv, k, tasks);
      else
        k_update_kmajor<F32><<<grid, KMajor<F32>::NT, 0, s>>>(tv, k, tasks);
      break;
    case BF16: k_update_mmajor<BF16><<<grid, 256, 0, s>>>(tv, k, tasks); break;
    case F16: k_update_mmajor<F16><<<grid, 256, 0, s>>>(tv, k, tasks); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Shared pieces of the diagonal-tile POTRF and the panel TRSM.
// ---------------------------------------------------------------------------
constexpr int PW = 32;

// acc0/acc1 (16 x 16 each) += A[R0.., K0:K1] * B[C0.., K0:K1]^T, operands read
// straight from column-major FP64 storage (lda = ldb = ld).  Software
// pipelined: the twelve loads of the next 16-wide k batch are issued before the
// eight MFMAs of the current one.  K1 - K0 is a multiple of 4.
__device__ __forceinline__ void mfma_rows16x32(const double* A, const double* B, int64_t ld, int R0, int C0, int K0,
                                               int K1, int lane, d4& acc0, d4& acc1) {
  const int r = lane & 15, q = lane >> 4;
  auto ld12 = [&](int kk, double* a, double* b0, double* b1) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t col = kk + 4 * u + q;
      a[u] = A[col * ld + R0 + r];
      b0[u] = B[col * ld + C0 + r];
      b1[u] = B[col * ld + C0 + 16 + r];
    }
  };
  int kk = K0;
  const int full_end = K0 + ((K1 - K0) / 16) * 16;
  if (kk < full_end) {
    double a[4], b0[4], b1[4];
    ld12(kk, a, b0, b1);
    for (; kk < full_end; kk += 16) {
      double na[4], nb0[4], nb1[4];
      const bool more = kk + 16 < full_end;
      if (more) ld12(kk + 16, na, nb0, nb1);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b0[u], acc0, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b1[u], acc1, 0, 0, 0);
      }
      if (more) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          a[u] = na[u];
          b0[u] = nb0[u];
          b1[u] = nb1[u];
        }
      }
    }
  }
  for (; kk < K1; kk += 4) {
    const int64_t col = kk + q;
    double a = A[col * ld + R0 + r], b0 = B[col * ld + C0 + r], b1 = B[col * ld + C0 + 16 + r];
    acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b0, acc0, 0, 0, 0);
    acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b1, acc1, 0, 0, 0);
  }
}

// ---------------------------------------------------------------------------
// Triangular solves by one wave with inverted 32 x 32 diagonal blocks.
//
// invert_lower32: the inverse of a 32 x 32 lower-triangular block (column-major,
// leading dimension ld) into out (32 x 32, column-major); lane c < 32 computes
// column c by forward substitution on the unit vector e_c (fixed order).
//
// trsm_rows16_inv solves X L^T = A for 16 rows r0 .. r0+15 over the columns
// [c0, c1), left-looking over 32-column chunks J:
//   T   = A[rows, J] - X[rows, c0:J] L[J, c0:J]^T     (FP64 MFMA)
//   X_J = T D_J^{-T}                                 (FP64 MFMA, D_J^{-1} given)
// X (ld ldx) holds the solved columns of these rows, L the factor (ld ldl);
// load_a(idx) and store_x(idx, v) read A and write X_J at a column-major index
// of the rows' storage.  Each wave works alone (no barriers): the chunk goes
// from the MFMA result layout to the operand layout through Ts (16 x 33
// doubles of LDS per wave), and X is re-read by the same wave after a
// workgroup-scope fence.
// ---------------------------------------------------------------------------
// rdiag (optional) holds 1 / L[r][r]; the substitution then multiplies instead
// of dividing.
__device__ __forceinline__ void invert_lower32(const double* L, int64_t ld, double* out, double (*W)[PW + 1],
                                               int lane, const double* rdiag = nullptr) {
  for (int e = lane; e < PW * PW; e += 64) {
    const int r = e % PW, c = e / PW;
    W[r][c] = r >= c ? L[(int64_t)c * ld + r] : 0.0;
  }
  __builtin_amdgcn_wave_barrier();
  if (lane < PW) {
    double y[PW];
#pragma unroll
    for (int r = 0; r < PW; ++r) {
      double v = (r == lane) ? 1.0 : 0.0;
#pragma unroll
      for (int m = 0; m < r; ++m) v = fma(-W[r][m], y[m], v);
      y[r] = rdiag ? v * rdiag[r] : v / W[r][r];
    }
#pragma unroll
    for (int r = 0; r < PW; ++r) out[lane * PW + r] = y[r];
  }
}

template <class LoadA, class StoreX>
__device__ __forceinline__ void trsm_rows16_inv(const double* X, const double* L, int64_t ld, const double* dinv,
                                                int c0, int c1, int r0, double (*Ts)[PW + 1], int lane, LoadA load_a,
                                                StoreX store_x) {
  const int q = lane >> 4, c = lane & 15;
  // A and D_J^{-1} of the next chunk are requested before the current chunk's
  // product, so their latency hides behind it
  double av[8], dv[PW / 2];
  auto fetch = [&](int J0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int R = q + 4 * r;
      av[2 * r] = load_a((int64_t)(J0 + c) * ld + r0 + R);
      av[2 * r + 1] = load_a((int64_t)(J0 + c + 16) * ld + r0 + R);
    }
    const double* Di = dinv + (int64_t)(J0 / PW) * PW * PW;  // Di[kk * 32 + n] = D_J^{-1}[n][kk]
#pragma unroll
    for (int u = 0; u < PW / 4; ++u) {
      dv[2 * u] = Di[(4 * u + q) * PW + c];
      dv[2 * u + 1] = Di[(4 * u + q) * PW + 16 + c];
    }
  };
  fetch(c0);
#pragma unroll 1
  for (int J0 = c0; J0 < c1; J0 += PW) {
    double ca[8], cd[PW / 2];
#pragma unroll
    for (int e = 0; e < 8; ++e) ca[e] = av[e];
#pragma unroll
    for (int e = 0; e < PW / 2; ++e) cd[e] = dv[e];
    if (J0 + PW < c1) fetch(J0 + PW);
    d4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    mfma_rows16x32(X, L, ld, r0, J0, c0, J0, lane, acc0, acc1);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int R = q + 4 * r;
      Ts[R][c] = ca[2 * r] - acc0[r];
      Ts[R][c + 16] = ca[2 * r + 1] - acc1[r];
    }
    __builtin_amdgcn_wave_barrier();
    d4 x0 = {0, 0, 0, 0}, x1 = {0, 0, 0, 0};
#pragma unroll
    for (int u = 0; u < PW / 4; ++u) {
      const int kk = 4 * u + q;
      const double a = Ts[c][kk];
      x0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, cd[2 * u], x0, 0, 0, 0);
      x1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, cd[2 * u + 1], x1, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t i0 = (int64_t)(J0 + c) * ld + r0 + q + 4 * r;
      store_x(i0, x0[r]);
      store_x(i0 + 16 * ld, x1[r]);
    }
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
  }
}

// ---------------------------------------------------------------------------
// Blocked POTRF of the FP64 diagonal tile k, spread over several workgroups:
// the tile is split into SB x SB blocks and, for each block column j,
//   (a) k_potrf_block  one workgroup factors the diagonal block D_jj, held
//                      in registers (right-looking over 16-column panels,
//                      FP64 MFMA for the panel and trailing blocks, the
//                      16 x 16 diagonal blocks by one wave with lane
//                      broadcasts); it also inverts the four 32 x 32
//                      diagonal blocks of D_jj into dinv for the solves below,
//   (b) k_potrf_panel  the rows below solve X D_jj^T = A, one wave per 16
//                      rows (trsm_rows16_inv),
//   (c) k_potrf_syrk   the lower trailing part loses L_{:,j} L_{:,j}^T
//                      (64 x 64 output blocks, FP64 MFMA).
// ---------------------------------------------------------------------------
constexpr int SB = 128;

// 64-bit lane broadcast: the value v of lane src, read as a wave-uniform scalar.
__device__ __forceinline__ double readlane_f64(double v, int src) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, src);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), src);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// 1 / sqrt(d) for d > 0 (normal): the hardware estimate refined by two
// Newton steps y <- y + (y / 2)(1 - d y^2), each of which squares the relative
// error (about 3/2 e^2), so an estimate good to 2^-14 or better ends within a
// few units in the last place.
__device__ __forceinline__ double rsqrt_f64(double d) {
  double y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-d * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// Unblocked Cholesky of an N x N block held one row per lane (lane r < N:
// x[c] = D[r][c], c <= r), by one wave with lane broadcasts and no barriers.
// The pivot's reciprocal square root r_c gives both L[c][c] = d_c r_c and the
// column below as multiplications (no divide on the column-to-column chain);
// rdiag[c] receives r_c = 1 / L[c][c].  Returns the first column whose pivot
// is not positive, or -1.
template <int N>
__device__ __forceinline__ int chol_wave(double (&x)[N], int lane, double* rdiag) {
#pragma unroll
  for (int c = 0; c < N; ++c) {
    const double d = readlane_f64(x[c], c);
    if (!(d > 0.0)) return c;
    const double rs = rsqrt_f64(d);
    if (lane == 0) rdiag[c] = rs;
    const double lc = (lane == c) ? d * rs : x[c] * rs;
    x[c] = lc;
#pragma unroll
    for (int q = c + 1; q < N; ++q) {
      const double lq = readlane_f64(lc, q);
      if (lane >= q) x[q] = fma(-lc, lq, x[q]);
    }
  }
  return -1;
}

// acc[h] += A[R0 .. R0+15, K0:K1] * B[C0 + 16h .. C0 + 16h + 15, K0:K1]^T, h < 4,
// straight from column-major FP64 storage (leading dimension ld), 16 k per
// batch with the next batch's loads in flight.  K1 - K0 is a multiple of 16.
__device__ __forceinline__ void mfma_rows16x64(const double* A, const double* B, int64_t ld, int R0, int C0, int K0,
                                               int K1, int lane, d4 (&acc)[4]) {
  const int r = lane & 15, q = lane >> 4;
  auto ld20 = [&](int kk, double* a, double (*b)[4]) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t col = kk + 4 * u + q;
      a[u] = A[col * ld + R0 + r];
#pragma unroll
      for (int h = 0; h < 4; ++h) b[h][u] = B[col * ld + C0 + 16 * h + r];
    }
  };
  double a[4], b[4][4];
  ld20(K0, a, b);
  for (int kk = K0; kk < K1; kk += 16) {
    double na[4], nbv[4][4];
    const bool more = kk + 16 < K1;
    if (more) ld20(kk + 16, na, nbv);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int h = 0; h < 4; ++h) acc[h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[h][u], acc[h], 0, 0, 0);
    if (more) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        a[u] = na[u];
#pragma unroll
        for (int h = 0; h < 4; ++h) b[h][u] = nbv[h][u];
      }
    }
  }
}

constexpr int PB = 16;  // panel width inside the diagonal block

// The 36 lower 16 x 16 blocks (bi >= bj) of a 128 x 128 diagonal block, by
// columns; block b belongs to wave b % 4 (its slot b / 4 of nine).
constexpr int NBLK = (SB / PB) * (SB / PB + 1) / 2;
__device__ __forceinline__ void blk_ij(int b, int& bi, int& bj) {
  bj = 0;
  int rem = b, len = SB / PB;
  while (rem >= len) { rem -= len; ++bj; --len; }
  bi = bj + rem;
}

// Register-resident right-looking factorisation of the diagonal block: every
// wave holds its nine 16 x 16 blocks in the MFMA result layout for the whole
// kernel (loaded once, stored once).  Per 16-column panel p:
//   (1) the owner of block (p, p) factors it by one wave with lane broadcasts
//       and inverts the 16 x 16 factor (forward substitution on unit vectors);
//   (2) the owners of the blocks (i, p) below form L_ip = A_ip L_pp^{-T} (FP64
//       MFMA, the block brought into the operand layout through LDS) and put
//       L_ip in LDS;
//   (3) every trailing block (i, j), p < j <= i, loses L_ip L_jp^T (FP64 MFMA
//       from LDS).
// Two barriers per panel; the panel's blocks pass through 16 x 17 LDS slots.
__global__ __launch_bounds__(256) void k_potrf_block(TileView tv, int k, int j, double* dinv) {
  if (*tv.info) return;
  const int nb = tv.nb, c0 = j * SB, c1 = c0 + SB;
  double* A = (double*)tv.tile(k, k);
  __shared__ double Dg[PB][PB + 1];  // the diagonal block, then its factor
  __shared__ double Di[PB][PB + 1];  // the factor's inverse
  __shared__ double Dr[SB];          // 1 / L[c][c] of the block's columns
  // panel blocks P[i] (16 x 17 each), later the waves' store slots and 32 x 32
  // inversion space
  constexpr int PSZ = (SB / PB) * PB * (PB + 1);
  constexpr int WSZ = 4 * PW * (PW + 1);
  __shared__ double pool[PSZ > WSZ ? PSZ : WSZ];
  double (*P)[PB][PB + 1] = (double (*)[PB][PB + 1])pool;
  __shared__ int fail;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lr = lane >> 4, lc = lane & 15;  // result layout: rows lr + 4 r, column lc
  if (tid == 0) fail = 0;

  d4 acc[9];
#pragma unroll
  for (int sl = 0; sl < 9; ++sl) {
    const int b = 4 * sl + wave;
    acc[sl] = d4{0, 0, 0, 0};
    if (b < NBLK) {
      int bi, bj;
      blk_ij(b, bi, bj);
#pragma unroll
      for (int r = 0; r < 4; ++r)
        acc[sl][r] = A[(int64_t)(c0 + PB * bj + lc) * nb + c0 + PB * bi + lr + 4 * r];
    }
  }
  __syncthreads();

#pragma unroll 1
  for (int p = 0; p < SB / PB; ++p) {
    // (1) diagonal block (p, p), block index 8p - p(p-1)/2; the factorisation
    // code is outside the slot loop so that it exists once in the kernel
    const int bpp = (SB / PB) * p - p * (p - 1) / 2;
#pragma unroll
    for (int sl = 0; sl < 9; ++sl)
      if (4 * sl + wave == bpp) {
#pragma unroll
        for (int r = 0; r < 4; ++r) Dg[lr + 4 * r][lc] = acc[sl][r];
      }
    if (wave == bpp % 4) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      double x[PB];
#pragma unroll
      for (int c = 0; c < PB; ++c) x[c] = (lane < PB && c <= lane) ? Dg[lane][c] : 0.0;
      const int bad = chol_wave<PB>(x, lane, Dr + PB * p);
      if (bad >= 0) {
        if (lane == 0) {
          fail = 1;
          if (*tv.info == 0) *tv.info = k * nb + c0 + PB * p + bad + 1;
        }
      } else {
        if (lane < PB) {
#pragma unroll
          for (int c = 0; c < PB; ++c) Dg[lane][c] = c <= lane ? x[c] : 0.0;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (lane < PB) {  // column lane of the inverse
          double y[PB];
#pragma unroll
          for (int r = 0; r < PB; ++r) {
            double v = (r == lane) ? 1.0 : 0.0;
#pragma unroll
            for (int m = 0; m < r; ++m) v = fma(-Dg[r][m], y[m], v);
            y[r] = v * Dr[PB * p + r];
          }
#pragma unroll
          for (int r = 0; r < PB; ++r) Di[r][lane] = y[r];
        }
#pragma unroll
        for (int sl = 0; sl < 9; ++sl)
          if (4 * sl + wave == bpp) {
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[sl][r] = Dg[lr + 4 * r][lc];
          }
      }
    }
    __syncthreads();
    if (fail) return;
    // (2) panel blocks (i, p), i > p
#pragma unroll
    for (int sl = 0; sl < 9; ++sl) {
      const int b = 4 * sl + wave;
      if (b >= NBLK) continue;
      int bi, bj;
      blk_ij(b, bi, bj);
      if (bj != p || bi == p) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) P[bi][lr + 4 * r][lc] = acc[sl][r];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      d4 xv = {0, 0, 0, 0};
#pragma unroll
      for (int u = 0; u < 4; ++u)
        xv = __builtin_amdgcn_mfma_f64_16x16x4f64(P[bi][lc][4 * u + lr], Di[lc][4 * u + lr], xv, 0, 0, 0);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      acc[sl] = xv;
#pragma unroll
      for (int r = 0; r < 4; ++r) P[bi][lr + 4 * r][lc] = xv[r];
    }
    __syncthreads();
    // (3) trailing blocks (i, j), p < j <= i
#pragma unroll
    for (int sl = 0; sl < 9; ++sl) {
      const int b = 4 * sl + wave;
      if (b >= NBLK) continue;
      int bi, bj;
      blk_ij(b, bi, bj);
      if (bj <= p) continue;
#pragma unroll
      for (int u = 0; u < 4; ++u)
        acc[sl] = __builtin_amdgcn_mfma_f64_16x16x4f64(-P[bi][lc][4 * u + lr], P[bj][lc][4 * u + lr], acc[sl], 0,
                                                       0, 0);
    }
  }

  // the factor's lower blocks, each turned through a 16 x 17 LDS slot of its
  // wave so that a lane stores four consecutive rows of one column (a store
  // instruction then covers whole 128-byte pieces of 16 columns), then zeros
  // above the diagonal in columns c0 .. c1
  __syncthreads();  // the panel slots are free once every wave has left (3)
  {
    double (*T)[PB + 1] = (double (*)[PB + 1])(pool + wave * PB * (PB + 1));
    const int tc = lane >> 2, tr = 4 * (lane & 3);
#pragma unroll
    for (int sl = 0; sl < 9; ++sl) {
      const int b = 4 * sl + wave;
      if (b >= NBLK) continue;
      int bi, bj;
      blk_ij(b, bi, bj);
#pragma unroll
      for (int r = 0; r < 4; ++r) T[lr + 4 * r][lc] = acc[sl][r];
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      double v[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = T[tr + e][tc];
      double* o = A + (int64_t)(c0 + PB * bj + tc) * nb + c0 + PB * bi + tr;
      if (bi > bj) {
        *(double2*)o = double2{v[0], v[1]};
        *(double2*)(o + 2) = double2{v[2], v[3]};
      } else {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (tr + e >= tc) o[e] = v[e];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  // (one wave per column, two rows per lane and store)
  for (int c = c0 + wave; c < c1; c += 4)
    for (int r = 2 * lane; r < c; r += 128) {
      double* o = A + (int64_t)c * nb + r;
      if (r + 1 < c) *(double2*)o = double2{0.0, 0.0};
      else *o = 0.0;
    }
  __syncthreads();
  // inverses of the four 32 x 32 diagonal blocks, one per wave
  double (*W)[PW][PW + 1] = (double (*)[PW][PW + 1])pool;
  const int d0 = c0 + wave * PW;
  invert_lower32(A + (int64_t)d0 * nb + d0, nb, dinv + (int64_t)d0 * PW, W[wave], lane, Dr + wave * PW);
}

// rows c1 .. nb of block column j: X D_jj^T = A in place, one wave per 16 rows
__global__ __launch_bounds__(64) void k_potrf_panel(TileView tv, int k, int j, const double* dinv) {
  if (*tv.info) return;
  const int nb = tv.nb, c0 = j * SB, c1 = c0 + SB;
  double* A = (double*)tv.tile(k, k);
  __shared__ double Ts[16][PW + 1];
  trsm_rows16_inv(A, A, nb, dinv, c0, c1, c1 + blockIdx.x * 16, Ts, threadIdx.x, [&](int64_t i) { return A[i]; },
                  [&](int64_t i, double v) { A[i] = v; });
}

// A[R, C] -= L[R, c0:c1] L[C, c0:c1]^T for c1 <= C <= R < nb; one workgroup per
// lower 64 x 64 block (bi >= bj), eight waves: wave w takes rows 16 (w % 4) ..
// of the block over one half of the 128 columns, and the second half's partial
// products are added to the first's through LDS (half the chain of dependent
// loads and MFMAs per wave on this critical-path step)
__global__ __launch_bounds__(512) void k_potrf_syrk(TileView tv, int k, int j) {
  if (*tv.info) return;
  const int nb = tv.nb, c0 = j * SB, c1 = c0 + SB;
  double* A = (double*)tv.tile(k, k);
  int bi = 0, rem = blockIdx.x;
  while (rem > bi) { rem -= bi + 1; ++bi; }
  const int bj = rem;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rg = wave & 3, kh = wave >> 2, kw = SB / 2;
  const int R0 = c1 + bi * 64 + rg * 16, C0 = c1 + bj * 64;
  __shared__ double red[4][16][65];
  d4 acc[4];
#pragma unroll
  for (int h = 0; h < 4; ++h) acc[h] = d4{0, 0, 0, 0};
  mfma_rows16x64(A, A, nb, R0, C0, c0 + kh * kw, c0 + (kh + 1) * kw, lane, acc);
  if (kh == 1) {
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[rg][(lane >> 4) + 4 * r][16 * h + (lane & 15)] = acc[h][r];
  }
  __syncthreads();
  if (kh == 0) {
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int R = R0 + (lane >> 4) + 4 * r, C = C0 + 16 * h + (lane & 15);
        if (R >= C) A[(int64_t)C * nb + R] -= acc[h][r] + red[rg][(lane >> 4) + 4 * r][16 * h + (lane & 15)];
      }
  }
}

// A_jj -= L_jk L_jk^T for one diagonal tile with an FP64 panel tile (the SYRK
// on the factorisation's critical path): one workgroup per lower 64 x 64 block,
// eight waves: wave w takes rows 16 (w % 4) .. of the block over one half of
// the contraction (FP64 MFMA straight from the tiles); the second half's
// partial products are added to the first's through LDS.  Halving each wave's
// chain of dependent MFMAs halves the kernel's latency, which is what counts
// here: the 36 workgroups of a 512-tile occupy few CUs.
__global__ __launch_bounds__(512) void k_syrk_tile(TileView tv, int k, int j) {
  if (*tv.info) return;
  const int nb = tv.nb;
  int bi = 0, rem = blockIdx.x;
  while (rem > bi) { rem -= bi + 1; ++bi; }
  const int bj = rem;
  const double* L = (const double*)tv.tile(j, k);
  double* A = (double*)tv.tile(j, j);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rg = wave & 3, kh = wave >> 2, kw = nb / 2;
  const int R0 = bi * 64 + rg * 16, C0 = bj * 64;
  __shared__ double red[4][16][65];
  d4 acc[4];
#pragma unroll
  for (int h = 0; h < 4; ++h) acc[h] = d4{0, 0, 0, 0};
  mfma_rows16x64(L, L, nb, R0, C0, kh * kw, (kh + 1) * kw, lane, acc);
  if (kh == 1) {
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[rg][(lane >> 4) + 4 * r][16 * h + (lane & 15)] = acc[h][r];
  }
  __syncthreads();
  if (kh == 0) {
#pragma unroll
    for (int h = 0; h < 4; ++h)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int R = R0 + (lane >> 4) + 4 * r, C = C0 + 16 * h + (lane & 15);
        if (R >= C) A[(int64_t)C * nb + R] -= acc[h][r] + red[rg][(lane >> 4) + 4 * r][16 * h + (lane & 15)];
      }
  }
}

hipError_t launch_syrk_tile(const TileView& tv, int k, int j, hipStream_t s) {
  const int nbk = tv.nb / 64;
  k_syrk_tile<<<nbk * (nbk + 1) / 2, 512, 0, s>>>(tv, k, j);
  return hipGetLastError();
}

hipError_t launch_potrf_tile(const TileView& tv, int k, double* dinv, hipStream_t s) {
  const int nsb = tv.nb / SB;
  for (int j = 0; j < nsb; ++j) {
    k_potrf_block<<<1, 256, 0, s>>>(tv, k, j, dinv);
    const int rest = (tv.nb - (j + 1) * SB) / 64;  // 64-row blocks below block j
    if (rest > 0) {
      k_potrf_panel<<<rest * 4, 64, 0, s>>>(tv, k, j, dinv);
      k_potrf_syrk<<<rest * (rest + 1) / 2, 512, 0, s>>>(tv, k, j);
    }
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Panel TRSM: for i > k, X = A_ik L_kk^{-T} in FP64, rounded once to p(i,k).
// One wave per 16 rows of a panel tile (trsm_rows16_inv with the inverted
// diagonal blocks of L_kk from its POTRF); the FP64 X goes to the workspace ws
// ((nt-k-1) tiles of nb x nb) and the tile receives one rounding of it.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_trsm(TileView tv, int k, double* ws, const double* dinv) {
  if (*tv.info) return;
  const int nb = tv.nb, rblocks = nb / 16;
  const int ti = k + 1 + blockIdx.x / rblocks;
  const int r0 = (blockIdx.x % rblocks) * 16;
  void* Ap = tv.tile(ti, k);
  const int fa = tv.tfmt(ti, k);
  const double ma = tv.tmul(ti, k);
  double* X = ws + (int64_t)(ti - k - 1) * nb * nb;
  __shared__ double Ts[16][PW + 1];
  // FP8 tiles are rounded by k_quant_panel_f8 once the whole tile's largest magnitude is known
  trsm_rows16_inv(X, (const double*)tv.tile(k, k), nb, dinv, 0, nb, r0, Ts, threadIdx.x,
                  [&](int64_t i) { return load_wide(Ap, fa, i) * ma; },
                  [&](int64_t i, double v) {
                    X[i] = v;
                    if (fa != F8) store_round(Ap, fa, i, v);
                  });
}

// FP8 panel tiles after k_trsm: scale from the solved tile's largest magnitude,
// then one rounding of every value (one workgroup per panel tile)
__global__ __launch_bounds__(256) void k_quant_panel_f8(TileView tv, int k, const double* ws) {
  const int ti = k + 1 + blockIdx.x;
  if (*tv.info || tv.tfmt(ti, k) != F8) return;
  const int nb = tv.nb;
  const double* X = ws + (int64_t)blockIdx.x * nb * nb;
  __shared__ double red[256];
  double m = 0.0;
  for (int64_t e = threadIdx.x; e < (int64_t)nb * nb; e += 256) m = fmax(m, fabs(X[e]));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  const int sc = fp8_scale_exp(red[0]);
  uint8_t* P = (uint8_t*)tv.tile(ti, k);
  for (int64_t e = threadIdx.x; e < (int64_t)nb * nb; e += 256) P[e] = to_e4m3(ldexp(X[e], sc));
  if (threadIdx.x == 0) tv.sc[tri_index(ti, k)] = (int8_t)sc;
}

// The same panel solve with four waves per 16 rows, for steps with few panel
// tiles, where the solve sits alone on the critical path: the update of every
// 32-column chunk is split over the waves by quarters of its contraction
// (their partial products added in wave order through LDS), and wave 0 forms
// the chunk's columns with the inverted diagonal block.  Two barriers per
// chunk; the chunk's columns reach the other waves through global memory
// after a workgroup-scope fence.
constexpr int TRSM_SPLIT_MAX = 32;  // panel tiles up to which the split solve is used

__global__ __launch_bounds__(256) void k_trsm4(TileView tv, int k, double* ws, const double* dinv) {
  if (*tv.info) return;
  const int nb = tv.nb, rblocks = nb / 16;
  const int ti = k + 1 + blockIdx.x / rblocks;
  const int r0 = (blockIdx.x % rblocks) * 16;
  void* Ap = tv.tile(ti, k);
  const int fa = tv.tfmt(ti, k);
  const double ma = tv.tmul(ti, k);
  double* X = ws + (int64_t)(ti - k - 1) * nb * nb;
  const double* L = (const double*)tv.tile(k, k);
  __shared__ double red[4][16][PW + 1];
  __shared__ double Ts[16][PW + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int q = lane >> 4, c = lane & 15;
#pragma unroll 1
  for (int J0 = 0; J0 < nb; J0 += PW) {
    const int part = J0 / 4;  // a multiple of 8
    d4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    mfma_rows16x32(X, L, nb, r0, J0, w * part, (w + 1) * part, lane, acc0, acc1);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      red[w][q + 4 * r][c] = acc0[r];
      red[w][q + 4 * r][c + 16] = acc1[r];
    }
    __syncthreads();
    if (w == 0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int R = q + 4 * r;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int cc = c + 16 * h;
          const double a = load_wide(Ap, fa, (int64_t)(J0 + cc) * nb + r0 + R) * ma;
          Ts[R][cc] = a - (((red[0][R][cc] + red[1][R][cc]) + red[2][R][cc]) + red[3][R][cc]);
        }
      }
      __builtin_amdgcn_wave_barrier();
      const double* Di = dinv + (int64_t)(J0 / PW) * PW * PW;  // Di[kk * 32 + n] = D_J^{-1}[n][kk]
      d4 x0 = {0, 0, 0, 0}, x1 = {0, 0, 0, 0};
#pragma unroll
      for (int u = 0; u < PW / 4; ++u) {
        const int kk = 4 * u + q;
        const double a = Ts[c][kk];
        x0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Di[kk * PW + c], x0, 0, 0, 0);
        x1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Di[kk * PW + 16 + c], x1, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i0 = (int64_t)(J0 + c) * nb + r0 + q + 4 * r;
        X[i0] = x0[r];
        X[i0 + 16 * nb] = x1[r];
        // FP8 tiles are rounded by k_quant_panel_f8 once the whole tile's largest magnitude is known
        if (fa != F8) {
          store_round(Ap, fa, i0, x0[r]);
          store_round(Ap, fa, i0 + 16 * nb, x1[r]);
        }
      }
      __threadfence_block();
    }
    __syncthreads();
  }
}

hipError_t launch_trsm_panel(const TileView& tv, int k, double* ws, const double* dinv, bool fp8_panel,
                             hipStream_t s) {
  int ntile = tv.nt - k - 1;
  if (ntile <= 0) return hipSuccess;
  if (ntile <= TRSM_SPLIT_MAX)
    k_trsm4<<<ntile * (tv.nb / 16), 256, 0, s>>>(tv, k, ws, dinv);
  else
    k_trsm<<<ntile * (tv.nb / 16), 64, 0, s>>>(tv, k, ws, dinv);
  if (fp8_panel) k_quant_panel_f8<<<ntile, 256, 0, s>>>(tv, k, ws);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// log|Sigma| = 2 sum_i log L_ii over the first n diagonal entries; fixed
// summation order (strided per thread, then a fixed tree).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_logdet(TileView tv, double* out) {
  __shared__ double red[256];
  const int nb = tv.nb;
  double s = 0.0;
  if (*tv.info == 0) {
    for (int g = threadIdx.x; g < tv.n; g += 256) {
      int t = g / nb, l = g % nb;
      s += log(((const double*)tv.tile(t, t))[(int64_t)l * nb + l]);
    }
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = 2.0 * red[0];
}

hipError_t launch_logdet(const TileView& tv, double* out, hipStream_t s) {
  k_logdet<<<1, 256, 0, s>>>(tv, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Inverted diagonal tiles for the solves.  Row r of X = L_kk^{-T} (X L^T = I) is
// column r of L_kk^{-1}, so trsm_rows16_inv applied to the identity, one wave
// per 16 rows, gives L_kk^{-1} stored by rows (its transpose in column-major
// order) from the 32 x 32 block inverses that the tile's POTRF left in dinv;
// entries left of the rows' own 32-column chunk are zero.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_trtri(TileView tv, double* Linv, const double* dinv) {
  if (*tv.info) return;
  const int nb = tv.nb, rb = nb / 16;
  const int kt = blockIdx.x / rb, r0 = (blockIdx.x % rb) * 16;
  const int c0 = (r0 / PW) * PW;
  double* X = Linv + (int64_t)kt * nb * nb;
  __shared__ double Ts[16][PW + 1];
  const int lane = threadIdx.x;
  for (int e = lane; e < 16 * c0; e += 64) X[(int64_t)(e / 16) * nb + r0 + e % 16] = 0.0;
  trsm_rows16_inv(X, (const double*)tv.tile(kt, kt), nb, dinv + (int64_t)kt * nb * PW, c0, nb, r0, Ts, lane,
                  [&](int64_t i) { return (i % nb) == (i / nb) ? 1.0 : 0.0; }, [&](int64_t i, double v) { X[i] = v; });
}

hipError_t launch_trtri_diag(const TileView& tv, double* Linv, const double* dinv, hipStream_t s) {
  k_trtri<<<tv.nt * (tv.nb / 16), 64, 0, s>>>(tv, Linv, dinv);
  return hipGetLastError();
}

}  // namespace mpcr
