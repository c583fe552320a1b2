// Internal declarations of the mpcr HIP library (gfx950 only).
//
// Formats: the device rounding functions take an FP64 value and round it ONCE
// to the target with round-to-nearest-even.  FP64 -> FP32 is the hardware
// conversion (v_cvt_f32_f64, RNE).  For the narrower formats the value is
// first rounded to FP32 by round-to-odd (truncate, then set the last bit when
// inexact) and then rounded to nearest-even to the target; because every
// target keeps at most 11 significand bits and FP32 keeps 24 >= 11 + 2, the
// two steps give the correctly rounded result (Boldo & Melquiond, "When double
// rounding is odd", 2005).  FP8-E4M3FN conversions saturate at +-448.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mpcr.h"
#include <rocprofiler-sdk-roctx/roctx.h>

namespace mpcr {

// Host-side trace range (rocprofv3 --marker-trace): spans the queueing of a
// call or phase; with a synchronisation inside the phase it also spans its GPU
// work.  The kernels themselves appear in the kernel trace.
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};


enum Fmt : int { F64 = 0, F32 = 1, F16 = 2, BF16 = 3, F8 = 4 };

__host__ __device__ inline int fmt_bytes(int f) {
  return f == F64 ? 8 : (f == F32 ? 4 : (f == F8 ? 1 : 2));
}

// Unit roundoff 2^-t of each format (t = significand bits incl. implicit bit).
__host__ __device__ inline double fmt_unit_roundoff(int f) {
  return f == F64 ? 0x1p-53 : f == F32 ? 0x1p-24 : f == F16 ? 0x1p-11 : f == BF16 ? 0x1p-8 : 0x1p-4;
}
// Half the smallest subnormal: the absolute rounding error of values below the
// normal range (FP8 is scaled per block or tile, so its floor is relative;
// FP64's, 2^-1075, is not representable and lies far below every guard).
__host__ __device__ inline double fmt_abs_floor(int f) {
  return f == F32 ? 0x1p-150 : f == F16 ? 0x1p-25 : f == BF16 ? 0x1p-134 : 0.0;
}

// ---------------------------------------------------------------------------
// device rounding / widening
// ---------------------------------------------------------------------------

__device__ __forceinline__ float round_odd_f32(double x) {
  float t = __double2float_rz(x);
  if ((double)t != x) t = __uint_as_float(__float_as_uint(t) | 1u);
  return t;
}

__device__ __forceinline__ float to_f32(double x) { return (float)x; }

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ uint16_t to_bf16(double x) { return f32_to_bf16_rne(round_odd_f32(x)); }

__device__ __forceinline__ uint16_t to_f16(double x) {
  _Float16 h = (_Float16)round_odd_f32(x);  // v_cvt_f16_f32, round-to-nearest-even
  return __builtin_bit_cast(uint16_t, h);
}

// FP32 -> FP8-E4M3FN (bias 7, 3 stored significand bits, subnormal quantum
// 2^-9, largest finite 448 = 0x7e), nearest-even, saturating.
__device__ __forceinline__ uint8_t f32_to_e4m3_sat(float f) {
  uint32_t u = __float_as_uint(f);
  uint8_t sign = (uint8_t)((u >> 24) & 0x80u);
  uint32_t a = u & 0x7fffffffu;
  if (a > 0x7f800000u) return 0x7f;                   // NaN
  if (a >= 0x43e00000u) return sign | 0x7e;           // |f| >= 448 (incl. inf): saturate
  if (a < 0x3c800000u) {                              // |f| < 2^-6: subnormal range
    float q = __uint_as_float(a) * 512.0f;            // in units of 2^-9, exact
    float r = __builtin_rintf(q);                     // ties to even, 0..8
    return sign | (uint8_t)r;                         // r == 8 is the smallest normal 0x08
  }
  uint32_t e = (a >> 23) - 127u + 7u;                 // biased FP8 exponent, 1..15
  uint32_t m = a & 0x7fffffu;
  uint32_t r = m + 0x7ffffu + ((m >> 20) & 1u);       // round 23 -> 3 bits, ties to even
  if (r & 0x800000u) { e += 1; r = 0; }
  uint32_t code = (e << 3) | ((r >> 20) & 7u);
  if (code > 0x7e) code = 0x7e;
  return sign | (uint8_t)code;
}

__device__ __forceinline__ uint8_t to_e4m3(double x) { return f32_to_e4m3_sat(round_odd_f32(x)); }

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ float f16_to_f32(uint16_t b) { return (float)__builtin_bit_cast(_Float16, b); }
__device__ __forceinline__ float e4m3_to_f32(uint8_t c) {
  uint32_t s = (c & 0x80u) << 24;
  uint32_t e = (c >> 3) & 15u, m = c & 7u;
  if (e == 15u && m == 7u) return __uint_as_float(0x7fc00000u | s);
  float v = e == 0 ? (float)m * 0x1p-9f : __uint_as_float(((e + 120u) << 23) | (m << 20));
  return __uint_as_float(__float_as_uint(v) | s);
}

// Load element `idx` of a buffer of format f, widened to double (exact).
__device__ __forceinline__ double load_wide(const void* p, int f, int64_t idx) {
  switch (f) {
    case F64: return ((const double*)p)[idx];
    case F32: return (double)((const float*)p)[idx];
    case F16: return (double)f16_to_f32(((const uint16_t*)p)[idx]);
    case BF16: return (double)bf16_to_f32(((const uint16_t*)p)[idx]);
    default: return (double)e4m3_to_f32(((const uint8_t*)p)[idx]);
  }
}

// Store x rounded once to format f.
__device__ __forceinline__ void store_round(void* p, int f, int64_t idx, double x) {
  switch (f) {
    case F64: ((double*)p)[idx] = x; break;
    case F32: ((float*)p)[idx] = to_f32(x); break;
    case F16: ((uint16_t*)p)[idx] = to_f16(x); break;
    case BF16: ((uint16_t*)p)[idx] = to_bf16(x); break;
    default: ((uint8_t*)p)[idx] = to_e4m3(x); break;
  }
}

// ---------------------------------------------------------------------------
// tile store: lower tiles (i >= j) of an nt x nt tiling, each tile nb x nb
// column-major and contiguous in its own format; packed index
// t(i, j) = i (i + 1) / 2 + j.
// ---------------------------------------------------------------------------

__host__ __device__ inline int64_t tri_index(int64_t i, int64_t j) { return i * (i + 1) / 2 + j; }

struct TileView {
  uint8_t* base;          // device base address of all tiles
  const int64_t* off;     // device: byte offset of tile t(i, j)
  const uint8_t* fmt;     // device: format of tile t(i, j)
  int nb;
  int nt;
  int n;                  // true (unpadded) order
  int* info;              // device: 0, or 1-based global column of a failed pivot
  int8_t* sc;             // device: scale exponent s of each FP8 tile (values = codes * 2^-s)

  __device__ __forceinline__ void* tile(int i, int j) const { return base + off[tri_index(i, j)]; }
  __device__ __forceinline__ int tfmt(int i, int j) const { return fmt[tri_index(i, j)]; }
  __device__ __forceinline__ int tscale(int i, int j) const { return sc[tri_index(i, j)]; }
  // widening multiplier of tile (i, j): 2^-s for an FP8 tile, 1 otherwise
  __device__ __forceinline__ double tmul(int i, int j) const {
    return tfmt(i, j) == F8 ? ldexp(1.0, -tscale(i, j)) : 1.0;
  }
};

// FP8 scale exponent of a tile or block with largest magnitude amax: the
// largest s with amax * 2^s <= 448 (from the binary exponent, exact), 0 for an
// all-zero block, clamped to a signed byte.
__host__ __device__ inline int fp8_scale_exp(double amax) {
  if (!(amax > 0.0)) return 0;
  int E;
  const double m = frexp(amax, &E);  // amax = m 2^E, m in [0.5, 1); 448 = 0.875 2^9
  const int s = (m <= 0.875) ? 9 - E : 8 - E;
  return s < -128 ? -128 : (s > 127 ? 127 : s);
}

// Workgroups are dispatched round-robin over the 8 XCDs of an MI355X (workgroup
// b runs on XCD b % 8), each with its own L2.  This remaps the launch index so
// that every XCD works through one contiguous range of logical blocks:
// neighbouring blocks, which share operand panels, then share an L2.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
  constexpr int NXCD = 8;
  const int xcd = bid % NXCD, idx = bid / NXCD;
  const int per = nblocks / NXCD, rem = nblocks % NXCD;
  return xcd * per + (xcd < rem ? xcd : rem) + idx;
}

struct GemmTask {
  int i, j;  // output tile (i, j); operands are tiles (i, k) and (j, k)
};

}  // namespace mpcr

#include <map>
#include <mutex>
#include <unordered_map>
namespace mpcr {
// Device memory arena (host-side bookkeeping; see api.cpp).
class Arena {
 public:
  Arena() = default;
  Arena(const Arena&) = delete;
  Arena& operator=(const Arena&) = delete;
  ~Arena();
  hipError_t init(size_t bytes);
  void* alloc(size_t bytes);  // NULL when no free block is large enough
  void free(void* p);
  size_t capacity() const { return capacity_; }
  size_t in_use();

 private:
  std::mutex mu_;
  char* base_ = nullptr;
  size_t capacity_ = 0, in_use_ = 0;
  std::map<size_t, size_t> free_;            // offset -> length
  std::unordered_map<size_t, size_t> used_;  // offset -> length
};

// Internal context helpers for the serving engine (not part of the C ABI).
int ctx_create_with_arena(int device, Arena* arena, mpcr_ctx** out);  // owns a new stream
void ctx_release_workspace(mpcr_ctx* ctx);                            // returns cached buffers
hipStream_t ctx_stream(mpcr_ctx* ctx);
// Device bytes one log-likelihood evaluation of order n (tile size nb, nrhs) may hold
// at once, for an all-FP64 map (an upper bound for any map).
size_t loglik_footprint(int64_t n, int64_t nb, int64_t nrhs);
}  // namespace mpcr

// ---------------------------------------------------------------------------
// kernel launchers (defined in the .hip files, called by the host driver)
// ---------------------------------------------------------------------------
namespace mpcr {

hipError_t launch_tiles_from_dense(const TileView& tv, const double* A, int64_t lda, hipStream_t s);
// sig64 != NULL: also write each tile's FP64 values (packed tile order, nb^2 doubles per tile)
hipError_t launch_tiles_from_covariance(const TileView& tv, const double* locs, const mpcr_theta_t& th,
                                        hipStream_t s, double* sig64 = nullptr);
hipError_t launch_tiles_to_dense(const TileView& tv, double* L, int64_t ldl, hipStream_t s);
hipError_t launch_covariance_dense(int n, const double* locs, const mpcr_theta_t& th, double* A,
                                   int64_t lda, hipStream_t s);
hipError_t launch_covariance_tile_amax(int n, int nb, const double* locs, const mpcr_theta_t& th,
                                       double* amax /* device nt*nt */, hipStream_t s);
hipError_t launch_convert(int prec, int64_t m, int64_t n, const double* src, int64_t lds, void* dst,
                          int64_t ldd, int8_t* scale_exp, hipStream_t s);

hipError_t launch_potrf_tile(const TileView& tv, int k, double* dinv, hipStream_t s);
// A_jj -= L_jk L_jk^T for an FP64 panel tile (j, k)
hipError_t launch_syrk_tile(const TileView& tv, int k, int j, hipStream_t s);
// FP8 tiles: per-tile scales from the tile maxima (amax: nt x nt, row-major)
hipError_t launch_fp8_scales(const TileView& tv, const double* amax, hipStream_t s);
hipError_t launch_dense_tile_amax(int n, int nb, const double* A, int64_t lda, double* amax, hipStream_t s);
// largest magnitude of each panel tile (i, k), i > k -> pamax[i]
hipError_t launch_panel_amax(const TileView& tv, int k, double* pamax, hipStream_t s);
// updates with FP8 output tiles: FP8 MFMA (operands quantised per tile), the new
// values staged in FP32 (ws32: cnt nb^2 floats, amax32: cnt words), then requantised
hipError_t launch_tile_update_fp8(const TileView& tv, int k, const GemmTask* tasks, int ntasks, const double* pamax,
                                  float* ws32, unsigned* amax32, hipStream_t s);
hipError_t launch_trsm_panel(const TileView& tv, int k, double* ws, const double* dinv, bool fp8_panel,
                             hipStream_t s);
// packed panels of step k: every panel tile (i, k), i > k, converted to FP32
// and split into three BF16 planes (out3: 3 (nt-k-1) nb^2 halfwords) and/or
// rounded once to BF16 (outb: (nt-k-1) nb^2 halfwords); either may be NULL
hipError_t launch_pack_split(const TileView& tv, int k, uint16_t* out3, uint16_t* outb, hipStream_t s);
// tile updates of step k from those planes: cfmt F32 (three planes, six BF16
// products) or BF16 (one plane)
hipError_t launch_tile_update_packed(const TileView& tv, int k, int cfmt, const GemmTask* tasks, int ntasks,
                                     const uint16_t* planes, hipStream_t s);
// fp32_split: FP32 output tiles through the BF16 MFMA with operands split
// into three BF16 parts (FP32-level accuracy); else the FP32 MFMA
hipError_t launch_tile_update(const TileView& tv, int k, int cfmt, const GemmTask* tasks, int ntasks,
                              hipStream_t s, bool fp32_split = false);
hipError_t launch_logdet(const TileView& tv, double* out, hipStream_t s);
hipError_t launch_trtri_diag(const TileView& tv, double* Linv, const double* dinv, hipStream_t s);

// One step of the tile sweeps: the diag launch solves block k (and writes it
// by rows into stage, nb x nrhs), the update launch subtracts its product from
// the remaining blocks, reading the right-hand side from stage.
hipError_t launch_fwd_diag(const TileView& tv, const double* Linv, int k, double* R, double* W,
                           int64_t ld, int nrhs, double* stage, hipStream_t s);
hipError_t launch_fwd_update(const TileView& tv, int k, double* R, const double* stage, int64_t ld, int nrhs,
                             hipStream_t s);
hipError_t launch_bwd_diag(const TileView& tv, const double* Linv, int k, double* R, double* X,
                           int64_t ld, int nrhs, double* stage, hipStream_t s);
hipError_t launch_bwd_update(const TileView& tv, int k, double* R, const double* stage, int64_t ld, int nrhs,
                             hipStream_t s);

// R = B - Sigma X (B == NULL: R = -Sigma X); rowsum != NULL also receives sum_c |Sigma_rc|
hipError_t launch_residual_cov(int n, const double* locs, const mpcr_theta_t& th, const double* B,
                               const double* X, double* R, int64_t ld, int nrhs, hipStream_t s,
                               double* rowsum = nullptr);
hipError_t launch_residual_dense(int n, const double* A, int64_t lda, const double* B, const double* X,
                                 double* R, int64_t ld, int nrhs, hipStream_t s, double* rowsum = nullptr);
// R = B - Sigma X from the FP64 copy of Sigma's lower tiles (B == NULL: R = -Sigma X);
// rowsum != NULL also receives sum_c |Sigma_rc|
size_t residual_part_bytes(int nb, int nt);
hipError_t launch_residual_tiles(int n, int nb, int nt, const double* sig64, const double* B, const double* X,
                                 double* R, int64_t ld, int nrhs, hipStream_t s, double* rowsum, double* part);
hipError_t launch_rowsum_abs_cov(int n, const double* locs, const mpcr_theta_t& th, double* out,
                                 hipStream_t s);
hipError_t launch_rowsum_abs_dense(int n, const double* A, int64_t lda, double* out, hipStream_t s);

// column reductions over the first n rows of n x nrhs blocks (ld), deterministic
hipError_t launch_col_dot(int n, int nrhs, const double* A, const double* B, int64_t ld, double* partial,
                          double* out, hipStream_t s);
hipError_t launch_col_stats(int n, int nrhs, const double* R, const double* X, const double* B, int64_t ld,
                            const double* sig_inf, double* partial, double* stats, hipStream_t s);
hipError_t launch_max_reduce(int n, const double* v, double* partial, double* out, hipStream_t s);

hipError_t launch_fill(double* p, int64_t count, double v, hipStream_t s);
hipError_t launch_copy_cols(int n, int nrhs, const double* src, int64_t lds, double* dst, int64_t ldd,
                            hipStream_t s);
hipError_t launch_axpy_cols(int n, int nrhs, const double* alpha, double sign, const double* X, double* Y,
                            int64_t ld, hipStream_t s);
hipError_t launch_xpby_cols(int n, int nrhs, const double* X, const double* beta, double* Y, int64_t ld,
                            hipStream_t s);
hipError_t launch_pcg_alpha(int nrhs, const double* rz, const double* pq, const int* active, double* alpha,
                            hipStream_t s);
hipError_t launch_pcg_beta(int nrhs, const double* rz_new, double* rz, const int* active, double* beta,
                           hipStream_t s);
hipError_t launch_loglik(int n, int nrhs, const double* logdet, const double* quad, double* out,
                         hipStream_t s);
hipError_t launch_quad_refined(int n, int nrhs, const double* Z, const double* X, const double* R, int64_t ld,
                               double* partial, double* quad, hipStream_t s);

// Krylov refinement variants (krylov.hip).  Block PCG works on groups of at
// most KRYLOV_MAX_BLOCK consecutive right-hand sides.
constexpr int KRYLOV_MAX_BLOCK = 32;
size_t gram_partial_bytes(int n, int nrhs, int bs);
// G[g] = sign * A_g^T B_g for every group g of bs consecutive columns (bs x bs, column-major)
hipError_t launch_group_gram(int n, int nrhs, int bs, const double* A, const double* B, int64_t ld,
                             double* partial, double* G, double sign, hipStream_t s);
hipError_t launch_group_spd_solve(int nrhs, int bs, const double* G, const double* F, const int* active, double* C,
                                  int* flag, hipStream_t s);
hipError_t launch_group_axpy(int n, int nrhs, int bs, const double* X, const double* C, double sign, double* Y,
                             int64_t ld, hipStream_t s);
hipError_t launch_group_xpyc(int n, int nrhs, int bs, const double* X, const double* C, double* Y, int64_t ld,
                             hipStream_t s);
hipError_t launch_col_dot_strided(int n, int nrhs, const double* A, const double* B, int64_t ld, double* partial,
                                  double* out, int64_t stride, hipStream_t s);
hipError_t launch_axpy_strided(int n, int nrhs, const double* a, int64_t stride, double sign, const double* X,
                               double* Y, int64_t ld, hipStream_t s);
hipError_t launch_scale_cols(int n, int nrhs, const double* f, const double* X, double* Y, int64_t ld,
                             hipStream_t s);
hipError_t launch_gmres_start(int nrhs, int m, const double* dot, const int* active, double* beta, double* g,
                              double* inv, hipStream_t s);
hipError_t launch_gmres_rotate(int nrhs, int m, int j, const double* dot, const int* run, double* H, double* cs,
                               double* sn, double* g, double* out, hipStream_t s);
hipError_t launch_gmres_inv(int nrhs, const double* norm, const int* cont, double* inv, hipStream_t s);
hipError_t launch_gmres_backsolve(int nrhs, int m, const double* H, const double* g, const int* steps, double* y,
                                  hipStream_t s);

// I + diag(w) Sigma diag(w) into the tile store (Sigma from the sites)
hipError_t launch_tiles_from_weighted_covariance(const TileView& tv, const double* locs, const mpcr_theta_t& th,
                                                 const double* w, hipStream_t s);
// Laplace approximation, Bernoulli-logit observations: element-wise steps
hipError_t launch_laplace_terms(int n, double beta, const double* x, const double* y, double* g, double* s,
                                double* lik, double* b, hipStream_t st);
hipError_t launch_scale(int n, const double* s, const double* u, double sign, double* out, hipStream_t st);
hipError_t launch_laplace_a(int n, const double* b, const double* s, const double* v, double* a, hipStream_t st);
hipError_t launch_step_diff(int n, const double* xnew, double* xold, double* d, hipStream_t st);

// y = L x with the lower tile factor (MALA proposal noise); out = a + alpha b
hipError_t launch_trmv_lower(const TileView& tv, const double* x, double* y, hipStream_t s);
hipError_t launch_axpby(int n, const double* a, double alpha, const double* b, double* out, hipStream_t s);

// Allocation-free ordering: the sort keys live in a static device array of
// MORTON_NOALLOC_MAX_KEYS entries (8 MiB per GPU).
constexpr int MORTON_NOALLOC_MAX_KEYS = 1 << 20;
constexpr int MAX_DEVICES = 64;
hipError_t morton_noalloc_keys(int device, uint64_t** out);
hipError_t launch_morton_codes(int n, const double* locs, uint64_t* keys, int npow2, hipStream_t s);
hipError_t launch_bitonic_sort(uint64_t* keys, int npow2, hipStream_t s);
hipError_t launch_keys_to_perm(int n, const uint64_t* keys, int64_t* perm, hipStream_t s);
hipError_t launch_gather_rows(int n, int ncols, const double* src, int64_t lds, const int64_t* perm,
                              double* dst, int64_t ldd, hipStream_t s);

hipError_t launch_gemm(int prec, int transA, int transB, int64_t m, int64_t n, int64_t k, double alpha,
                       const void* A, int64_t lda, const void* B, int64_t ldb, double beta, void* C, int64_t ldc,
                       int cprec, hipStream_t s);
hipError_t launch_pack(int es, int trans, int64_t rows, int64_t cols, const void* in, int64_t ldi, void* out,
                       int64_t ldo, hipStream_t s);
hipError_t launch_gemm_lowp(int prec, int64_t m, int64_t n, int64_t k, double alpha, const void* AT, int64_t ldat,
                            const int8_t* sA, int64_t mbA, int sa_kmajor, const void* B, int64_t ldb,
                            const int8_t* sB, int64_t mbB, int sb_kmajor, double beta, void* C, int64_t ldc, int cprec,
                            hipStream_t s);

}  // namespace mpcr
