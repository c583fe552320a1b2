// C interface of the mpcr library: argument checking, device memory, and the
// stream-ordered schedule of the tile kernels.  Every numerical step runs in
// the HIP kernels of this library; the host only validates, allocates, queues
// launches and reads back small result arrays.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "mpcr_internal.h"

using namespace mpcr;

namespace mpcr {
// First-fit sub-allocator over one device allocation, 256-byte granules.  Used
// by the serving engine so that admitting and retiring requests never calls
// hipMalloc / hipFree (which would serialise the device).
hipError_t Arena::init(size_t bytes) {
  bytes = (bytes + 255) / 256 * 256;
  hipError_t e = hipMalloc((void**)&base_, bytes);
  if (e != hipSuccess) return e;
  capacity_ = bytes;
  free_[0] = bytes;
  return hipSuccess;
}
Arena::~Arena() {
  if (base_) (void)hipFree(base_);
}
void* Arena::alloc(size_t bytes) {
  bytes = (std::max<size_t>(bytes, 1) + 255) / 256 * 256;
  std::lock_guard<std::mutex> g(mu_);
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second < bytes) continue;
    size_t off = it->first, len = it->second;
    free_.erase(it);
    if (len > bytes) free_[off + bytes] = len - bytes;
    used_[off] = bytes;
    in_use_ += bytes;
    return base_ + off;
  }
  return nullptr;
}
void Arena::free(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> g(mu_);
  size_t off = (size_t)((char*)p - base_);
  auto u = used_.find(off);
  if (u == used_.end()) return;
  size_t len = u->second;
  used_.erase(u);
  in_use_ -= len;
  auto next = free_.lower_bound(off);
  if (next != free_.end() && off + len == next->first) {  // merge with the following block
    len += next->second;
    free_.erase(next);
  }
  auto it = free_.lower_bound(off);
  if (it != free_.begin()) {  // merge with the preceding block
    auto prev = std::prev(it);
    if (prev->first + prev->second == off) {
      prev->second += len;
      return;
    }
  }
  free_[off] = len;
}
size_t Arena::in_use() {
  std::lock_guard<std::mutex> g(mu_);
  return in_use_;
}
}  // namespace mpcr

constexpr int NKIND = 11;  // kernel kinds timed by the context (see mpcr_ctx_kernel_stats)

struct mpcr_ctx {
  int device = 0;
  Arena* arena = nullptr;  // device allocations come from here when set (serving workers)
  bool own_stream = false;
  hipStream_t stream = nullptr;
  std::string err;
  // workspace reused across mpcr_gauss_loglik calls of the same shape
  mpcr_factor* ws_factor = nullptr;
  std::vector<uint8_t> ws_map;
  int64_t ws_n = -1, ws_nb = -1;
  double* ws_locs = nullptr;      // n x 2 sorted sites
  double* ws_vec = nullptr;       // vector workspace
  int64_t ws_vec_bytes = 0;
  void* ws_kry = nullptr;         // Krylov workspace of the GMRES and block PCG solvers
  int64_t ws_kry_bytes = 0;
  uint8_t* ws_gemm = nullptr;     // packed 16/8-bit GEMM operands
  uint64_t* noalloc_keys = nullptr;  // device address of the static sort-key array on this device
  int64_t ws_gemm_bytes = 0;
  hipEvent_t ev[6] = {};
  // kernel timing (see mpcr_ctx_set_profiling)
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  struct Pending { hipEvent_t a, b; int kind; double flops; };
  std::vector<Pending> pending;
  double k_ms[NKIND] = {0}, k_flops[NKIND] = {0};
  int64_t k_launches[NKIND] = {0};
  int fp32_split = 1;              // FP32 tile updates through the BF16 MFMA (three-way split)
  // lookahead: a second stream for the bulk of each trailing update
  hipStream_t upd = nullptr;        // trailing updates of the factorisation
  hipStream_t col = nullptr;        // updates of the next panel column
  hipStream_t upd2 = nullptr;       // trailing updates of the tiles below FP64 (FP32, 16-bit, FP8)
  std::vector<hipEvent_t> sync_ev;  // timing-disabled events, 3 per step
};

namespace {
hipEvent_t take_event(mpcr_ctx* ctx) {
  if (!ctx->ev_pool.empty()) {
    hipEvent_t e = ctx->ev_pool.back();
    ctx->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
// Accumulates the elapsed times of recorded launches (the stream must have been synchronised).
void drain_timing(mpcr_ctx* ctx) {
  for (auto& p : ctx->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      ctx->k_ms[p.kind] += ms;
      ctx->k_launches[p.kind] += 1;
      ctx->k_flops[p.kind] += p.flops;
    }
    ctx->ev_pool.push_back(p.a);
    ctx->ev_pool.push_back(p.b);
  }
  ctx->pending.clear();
}
// Runs `launch` (queued on stream s) between two events when profiling is on.
template <class F>
hipError_t timed(mpcr_ctx* ctx, hipStream_t s, int kind, double flops, F&& launch) {
  if (!ctx->profiling) return launch();
  hipEvent_t a = take_event(ctx), b = take_event(ctx);
  if (!a || !b) return launch();
  hipError_t e = hipEventRecord(a, s);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(b, s);
  ctx->pending.push_back({a, b, kind, flops});
  return e;
}

hipError_t ensure_lookahead(mpcr_ctx* ctx, size_t nev, bool need_col) {
  for (hipStream_t* st : {&ctx->upd, &ctx->col, &ctx->upd2})
    if (!*st && (st == &ctx->upd || need_col)) {
      hipError_t e = hipStreamCreateWithFlags(st, hipStreamNonBlocking);
      if (e != hipSuccess) return e;
    }
  while (ctx->sync_ev.size() < nev) {
    hipEvent_t ev;
    hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return e;
    ctx->sync_ev.push_back(ev);
  }
  return hipSuccess;
}
}  // namespace

struct mpcr_factor {
  int64_t n = 0, nb = 0, nt = 0, N = 0;
  int device = 0;
  std::vector<uint8_t> map;        // nt x nt, row-major, host
  std::vector<uint8_t> fmt_packed; // per lower tile
  std::vector<int64_t> off_packed; // byte offsets
  uint8_t* d_base = nullptr;
  int64_t* d_off = nullptr;
  uint8_t* d_fmt = nullptr;
  int* d_info = nullptr;
  double* d_trsm_ws = nullptr;     // (nt-1) nb^2 doubles (the panel TRSM's FP64 workspace)
  double* d_dinv = nullptr;        // nt x nb x 32 doubles: inverted 32 x 32 diagonal blocks of every L_kk
  uint16_t* d_split = nullptr;     // 2 x 3 (nt-1) nb^2 halfwords: split panels of the FP32 updates (step parity)
  uint16_t* d_b16 = nullptr;       // 2 x (nt-1) nb^2 halfwords: BF16 panels of the BF16 updates (step parity)
  double* d_Linv = nullptr;        // nt nb^2 doubles: the inverted diagonal tiles, each stored by rows
  double* d_sig = nullptr;         // optional FP64 copy of Sigma's lower tiles (stored residual)
  double* d_rpart = nullptr;       // partial products of the stored residual
  bool linv_ready = false;
  // FP8 tiles: per-tile scale exponents, and for FP8 output updates the panel
  // maxima (two step-parity buffers of nt) and the FP32 staging of the new tiles
  int8_t* d_sc = nullptr;
  bool has_f8 = false;
  double* d_pamax = nullptr;
  double* d_tamax = nullptr;       // nt x nt tile maxima for the FP8 scales at generation
  float* d_ws8 = nullptr;
  unsigned* d_amax8 = nullptr;
  int f8_maxP = 0, f8_maxU = 0;    // FP8 output tasks per step: next column / the columns after it
  GemmTask* d_tasks = nullptr;
  std::vector<int64_t> task_off;   // [(k * 5 + f)] offset into d_tasks
  std::vector<int> task_cnt;
  std::vector<int> task_cnt_next;  // leading tasks of each list that update column k+1
  double flops[5] = {0, 0, 0, 0, 0};
  int64_t info = 0;
  Arena* arena = nullptr;  // allocator the device buffers came from (NULL: hipMalloc)

  TileView view() const {
    TileView tv;
    tv.base = d_base;
    tv.off = d_off;
    tv.fmt = d_fmt;
    tv.nb = (int)nb;
    tv.nt = (int)nt;
    tv.n = (int)n;
    tv.info = d_info;
    tv.sc = d_sc;
    return tv;
  }
};

static const char* kVersion = "mpcr 0.1 gfx950";
static thread_local std::string g_err;  // last error of calls made without a context

static int set_err(mpcr_ctx* ctx, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  (ctx ? ctx->err : g_err) = buf;
  return code;
}

#define HIP_TRY(ctx, expr)                                                                      \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess)                                                                       \
      return set_err(ctx, e_ == hipErrorOutOfMemory ? MPCR_ERR_NOMEM : MPCR_ERR_DEVICE,        \
                     "%s failed: %s", #expr, hipGetErrorString(e_));                            \
  } while (0)

#define CHECK_ARG(ctx, cond, ...)                                 \
  do {                                                            \
    if (!(cond)) return set_err(ctx, MPCR_ERR_ARG, __VA_ARGS__);  \
  } while (0)

namespace {

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// Device allocation from the arena when one is given, else hipMalloc.
template <class T>
hipError_t dmalloc(Arena* a, T** p, size_t bytes) {
  if (bytes == 0) bytes = 16;
  if (a) {
    *p = (T*)a->alloc(bytes);
    return *p ? hipSuccess : hipErrorOutOfMemory;
  }
  return hipMalloc((void**)p, bytes);
}
void dfree(Arena* a, void* p) {
  if (!p) return;
  if (a) a->free(p);
  else (void)hipFree(p);
}

void free_factor(mpcr_factor* f) {
  if (!f) return;
  DeviceGuard g(f->device);
  for (void* p : {(void*)f->d_base, (void*)f->d_off, (void*)f->d_fmt, (void*)f->d_info, (void*)f->d_trsm_ws,
                  (void*)f->d_Linv, (void*)f->d_tasks, (void*)f->d_sig, (void*)f->d_rpart, (void*)f->d_sc,
                  (void*)f->d_pamax, (void*)f->d_tamax, (void*)f->d_ws8, (void*)f->d_amax8, (void*)f->d_dinv,
                  (void*)f->d_split, (void*)f->d_b16})
    dfree(f->arena, p);
  delete f;
}

bool valid_prec(int p) { return p >= 0 && p <= 4; }

// Checks a tile map and copies it (nt x nt) into out.
int check_map(mpcr_ctx* ctx, int64_t n, const mpcr_tilemap_t* map, std::vector<uint8_t>& out, int64_t& nb) {
  CHECK_ARG(ctx, map != nullptr, "map is NULL");
  CHECK_ARG(ctx, map->n == n, "map->n (%lld) != n (%lld)", (long long)map->n, (long long)n);
  nb = map->nb;
  CHECK_ARG(ctx, nb >= 128 && nb % 128 == 0 && nb <= 4096, "nb must be a positive multiple of 128 (<= 4096)");
  int64_t nt = (n + nb - 1) / nb;
  CHECK_ARG(ctx, map->nt == nt, "map->nt must be ceil(n / nb) = %lld", (long long)nt);
  CHECK_ARG(ctx, map->h_map != nullptr, "map->h_map is NULL");
  out.assign(map->h_map, map->h_map + nt * nt);
  for (int64_t i = 0; i < nt; ++i)
    for (int64_t j = 0; j <= i; ++j) {
      int p = out[i * nt + j];
      CHECK_ARG(ctx, valid_prec(p), "map(%lld,%lld) = %d is not a format", (long long)i, (long long)j, p);
      if (i == j) CHECK_ARG(ctx, p == F64, "diagonal tile %lld must be FP64", (long long)i);
    }
  return MPCR_OK;
}

// The map to factor again with after a breakdown at global column `info`
// (1-based): the pivot of tile step k = (info-1)/nb depends on the leading
// (k+1) x (k+1) tiles; p is the coarsest format among their off-diagonal tiles
// and d_fail the smallest distance i - j at which p occurs there.  Every tile
// of format p (FP16 and BF16 count as one level) with distance >= d_fail moves
// one format up.  Returns false when the leading tiles are all FP64.
bool promote_map(std::vector<uint8_t>& map, int64_t nt, int64_t nb, int64_t info) {
  auto rank = [](int p) { return p == F64 ? 3 : p == F32 ? 2 : p == F8 ? 0 : 1; };
  auto up = [](int p) { return p == F8 ? F16 : (p == F16 || p == BF16) ? F32 : F64; };
  const int64_t k = std::min<int64_t>((info - 1) / nb, nt - 1);
  int rmin = 3;
  for (int64_t i = 0; i <= k; ++i)
    for (int64_t j = 0; j < i; ++j) rmin = std::min(rmin, rank(map[i * nt + j]));
  if (rmin == 3) return false;
  int64_t dfail = nt;
  for (int64_t i = 0; i <= k; ++i)
    for (int64_t j = 0; j < i; ++j)
      if (rank(map[i * nt + j]) == rmin) dfail = std::min(dfail, i - j);
  for (int64_t i = 0; i < nt; ++i)
    for (int64_t j = 0; j < i; ++j) {
      uint8_t& p = map[i * nt + j];
      if (rank(p) == rmin && i - j >= dfail) p = (uint8_t)up(p);
    }
  return true;
}

// Allocates a factor for the map and fills its task lists.
int make_factor(mpcr_ctx* ctx, int64_t n, int64_t nb, const std::vector<uint8_t>& map, mpcr_factor** out) {
  DeviceGuard g(ctx->device);
  auto* f = new mpcr_factor();
  f->device = ctx->device;
  f->arena = ctx->arena;
  f->n = n;
  f->nb = nb;
  f->nt = (n + nb - 1) / nb;
  f->N = f->nt * nb;
  f->map = map;
  const int64_t nt = f->nt;
  const int64_t ntiles = nt * (nt + 1) / 2;
  f->fmt_packed.resize(ntiles);
  f->off_packed.resize(ntiles);
  int64_t off = 0;
  for (int64_t i = 0; i < nt; ++i)
    for (int64_t j = 0; j <= i; ++j) {
      int p = map[i * nt + j];
      int64_t t = tri_index(i, j);
      f->fmt_packed[t] = (uint8_t)p;
      f->off_packed[t] = off;
      off += ((nb * nb * fmt_bytes(p)) + 255) / 256 * 256;
    }
  // task lists: for each step k and compute format, the trailing tiles (i, j), j > k
  std::vector<GemmTask> tasks;
  f->task_off.assign(nt * 5, 0);
  f->task_cnt.assign(nt * 5, 0);
  f->task_cnt_next.assign(nt * 5, 0);
  for (int64_t k = 0; k < nt; ++k) {
    f->flops[F64] += (double)nb * nb * nb / 3.0;
    for (int64_t i = k + 1; i < nt; ++i) f->flops[F64] += 2.0 * (double)nb * nb * nb;  // TRSM + SYRK
    for (int p = 0; p < 5; ++p) {
      f->task_off[k * 5 + p] = (int64_t)tasks.size();
      for (int64_t j = k + 1; j < nt; ++j)
        for (int64_t i = j; i < nt; ++i)
          if (map[i * nt + j] == p) {
            tasks.push_back(GemmTask{(int)i, (int)j});
            if (i != j) f->flops[p] += 2.0 * (double)nb * nb * nb;
          }
      f->task_cnt[k * 5 + p] = (int)((int64_t)tasks.size() - f->task_off[k * 5 + p]);
      int nx = 0;
      for (int64_t t = f->task_off[k * 5 + p]; t < (int64_t)tasks.size(); ++t) nx += (tasks[t].j == k + 1);
      f->task_cnt_next[k * 5 + p] = nx;
    }
  }
  for (int64_t k = 0; k < nt; ++k) {
    const int all = f->task_cnt[k * 5 + F8], nx = f->task_cnt_next[k * 5 + F8];
    f->f8_maxP = std::max(f->f8_maxP, nx);
    f->f8_maxU = std::max(f->f8_maxU, all - nx);
  }
  for (uint8_t p : f->fmt_packed) f->has_f8 |= (p == F8);
  hipError_t e;
  Arena* A = f->arena;
  if (f->has_f8) {
    const size_t nf8 = (size_t)(f->f8_maxP + f->f8_maxU);
    if ((e = dmalloc(A, &f->d_pamax, (size_t)2 * nt * 8)) != hipSuccess ||
        (e = dmalloc(A, &f->d_tamax, (size_t)nt * nt * 8)) != hipSuccess ||
        (e = dmalloc(A, &f->d_ws8, std::max<size_t>(nf8, 1) * nb * nb * 4)) != hipSuccess ||
        (e = dmalloc(A, &f->d_amax8, std::max<size_t>(nf8, 1) * 4)) != hipSuccess) {
      free_factor(f);
      return set_err(ctx, MPCR_ERR_NOMEM, "device allocation failed: %s", hipGetErrorString(e));
    }
  }
  if ((e = dmalloc(A, &f->d_sc, std::max<int64_t>(ntiles, 1))) != hipSuccess ||
      (e = dmalloc(A, &f->d_base, (size_t)off)) != hipSuccess || (e = dmalloc(A, &f->d_off, ntiles * 8)) != hipSuccess ||
      (e = dmalloc(A, &f->d_fmt, ntiles)) != hipSuccess || (e = dmalloc(A, &f->d_info, sizeof(int))) != hipSuccess ||
      (e = dmalloc(A, &f->d_trsm_ws, (size_t)std::max<int64_t>(nt - 1, 1) * nb * nb * 8)) != hipSuccess ||
      (e = dmalloc(A, &f->d_dinv, (size_t)nt * nb * 32 * 8)) != hipSuccess ||
      (e = dmalloc(A, &f->d_tasks, std::max<size_t>(tasks.size(), 1) * sizeof(GemmTask))) != hipSuccess) {
    free_factor(f);
    return set_err(ctx, MPCR_ERR_NOMEM, "device allocation failed: %s", hipGetErrorString(e));
  }
  hipStream_t s = ctx->stream;
  if ((e = hipMemsetAsync(f->d_sc, 0, std::max<int64_t>(ntiles, 1), s)) != hipSuccess ||
      (e = hipMemcpyAsync(f->d_off, f->off_packed.data(), ntiles * 8, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (e = hipMemcpyAsync(f->d_fmt, f->fmt_packed.data(), ntiles, hipMemcpyHostToDevice, s)) != hipSuccess ||
      (tasks.size() &&
       (e = hipMemcpyAsync(f->d_tasks, tasks.data(), tasks.size() * sizeof(GemmTask), hipMemcpyHostToDevice, s)) !=
           hipSuccess) ||
      (e = hipStreamSynchronize(s)) != hipSuccess) {
    free_factor(f);
    return set_err(ctx, MPCR_ERR_DEVICE, "upload failed: %s", hipGetErrorString(e));
  }
  *out = f;
  return MPCR_OK;
}

// Queues the right-looking factorisation of an already filled tile store with
// a depth-1 lookahead over three streams.  The context's stream P carries the
// critical path: POTRF(k), TRSM(k), then the SYRK of the next diagonal tile
// (k+1, k+1), so POTRF(k+1) can start at once.  Stream C updates the rest of
// column k+1 (the next panel) from panel k while POTRF(k+1) runs; P waits for
// it before TRSM(k+1).  Stream U carries the rest of step k's trailing update
// (columns k+2 ..).  U and C wait for TRSM(k); P and C wait for U's step k-1
// before they touch column k+1, which that step also updates.
constexpr int64_t COL_STREAM_MIN_NT = 32;  // more tiles per dimension than this: next column on its own stream

int run_factorisation(mpcr_ctx* ctx, mpcr_factor* f) {
  hipStream_t P = ctx->stream;
  TileView tv = f->view();
  f->linv_ready = false;
  const double nb3 = (double)f->nb * f->nb * f->nb;
  const int64_t nt = f->nt;
  // the column stream pays off once the trailing updates are long enough to
  // hide POTRF(k+1) behind; small factorisations (serving) keep the next
  // column on P, which then runs POTRF(k), TRSM(k) and the whole column k+1
  const bool use_col = nt > COL_STREAM_MIN_NT;
  HIP_TRY(ctx, ensure_lookahead(ctx, (size_t)(4 * nt + 2), use_col));
  // the trailing updates of step k go to U (FP64 tiles) and U2 (the other
  // formats): a tile has one format, so the two streams never write the same
  // tile, and their launches fill each other's tails
  hipStream_t U = ctx->upd, C = use_col ? ctx->col : P, U2 = use_col ? ctx->upd2 : ctx->upd;
  auto ev = [&](int64_t i) { return ctx->sync_ev[i]; };      // 2k: TRSM(k) done (P), 2k+1: U's step k done
  auto evc = [&](int64_t k) { return ctx->sync_ev[2 * nt + 2 + k]; };  // C's column k+1 done
  auto ev2 = [&](int64_t k) { return ctx->sync_ev[3 * nt + 2 + k]; };  // U2's step k done
  // U, U2 and C start after everything queued on P so far (the tile fill)
  HIP_TRY(ctx, hipEventRecord(ev(2 * nt), P));
  HIP_TRY(ctx, hipStreamWaitEvent(U, ev(2 * nt), 0));
  HIP_TRY(ctx, hipStreamWaitEvent(C, ev(2 * nt), 0));
  if (U2 != U) HIP_TRY(ctx, hipStreamWaitEvent(U2, ev(2 * nt), 0));
  static const int order[5] = {F64, F32, BF16, F16, F8};
  const int64_t nb2 = f->nb * f->nb;
  // FP32 updates through the BF16 MFMA read split panels (two step parities)
  bool any32 = false;
  for (int64_t k = 0; k < nt; ++k) any32 |= f->task_cnt[k * 5 + F32] > 0;
  const bool split32 = ctx->fp32_split && any32 && nt > 1;
  const int64_t split_stride = 3 * (nt - 1) * nb2;
  if (split32 && !f->d_split)
    HIP_TRY(ctx, dmalloc(f->arena, &f->d_split, (size_t)(2 * split_stride) * sizeof(uint16_t)));
  // BF16 updates read their operands from BF16 panels packed the same way
  bool any16 = false;
  for (int64_t k = 0; k < nt; ++k) any16 |= f->task_cnt[k * 5 + BF16] > 0;
  const bool pack16 = any16 && nt > 1;
  const int64_t b16_stride = (nt - 1) * nb2;
  if (pack16 && !f->d_b16)
    HIP_TRY(ctx, dmalloc(f->arena, &f->d_b16, (size_t)(2 * b16_stride) * sizeof(uint16_t)));
  // which: 0 = the SYRK of the next diagonal tile, 1 = the rest of the next
  // column, 2 = the columns after it
  auto launch_updates = [&](int64_t k, hipStream_t s0, int which) -> int {
    for (int p : order) {
      const hipStream_t s = (which == 2 && p != F64) ? U2 : s0;
      const int all = f->task_cnt[k * 5 + p], nx = f->task_cnt_next[k * 5 + p];
      // the next column's tasks come first, its diagonal tile (FP64) first among them
      const int nd = (p == F64 && nx > 0) ? 1 : 0;
      const int off = which == 0 ? 0 : which == 1 ? nd : nx;
      const int cnt = which == 0 ? nd : which == 1 ? nx - nd : all - nx;
      if (cnt <= 0) continue;
      const GemmTask* t = f->d_tasks + f->task_off[k * 5 + p] + off;
      // GEMM tiles count 2 nb^3, the SYRK (diagonal) tiles nb^3
      const double ndiag = (p == F64) ? (which == 0 ? 1.0 : which == 1 ? 0.0 : (double)(nt - k - 2)) : 0.0;
      const double fl = nb3 * (2.0 * cnt - ndiag);
      if (p == F8) {  // each stream stages in its own part of the FP8 workspace
        const int base = which == 2 ? f->f8_maxP : 0;
        const double* pamax = f->d_pamax + (k & 1) * nt;
        HIP_TRY(ctx, timed(ctx, s, p, fl, [&] {
          return launch_tile_update_fp8(tv, (int)k, t, cnt, pamax, f->d_ws8 + (int64_t)base * nb2, f->d_amax8 + base, s);
        }));
      } else if (which == 0 && f->map[(k + 1) * nt + k] == F64) {
        HIP_TRY(ctx, timed(ctx, s, 10, fl, [&] { return launch_syrk_tile(tv, (int)k, (int)k + 1, s); }));
      } else if ((p == F32 && split32) || (p == BF16 && pack16)) {
        const uint16_t* sp = p == F32 ? f->d_split + (k & 1) * split_stride : f->d_b16 + (k & 1) * b16_stride;
        HIP_TRY(ctx, timed(ctx, s, p, fl, [&] { return launch_tile_update_packed(tv, (int)k, p, t, cnt, sp, s); }));
      } else {
        HIP_TRY(ctx, timed(ctx, s, p, fl, [&] { return launch_tile_update(tv, (int)k, p, t, cnt, s, ctx->fp32_split); }));
      }
    }
    return MPCR_OK;
  };
  int rc;
  for (int64_t k = 0; k < nt; ++k) {
    TraceRange step("tile step");
    bool fp8_panel = false;
    for (int64_t i = k + 1; i < nt; ++i) fp8_panel |= (f->map[i * nt + k] == F8);
    HIP_TRY(ctx, timed(ctx, P, 5, nb3 / 3.0, [&] { return launch_potrf_tile(tv, (int)k, f->d_dinv + k * f->nb * 32, P); }));
    if (k > 0) HIP_TRY(ctx, hipStreamWaitEvent(P, evc(k - 1), 0));  // column k updated by C
    HIP_TRY(ctx, timed(ctx, P, 6, nb3 * (double)(nt - k - 1),
                       [&] { return launch_trsm_panel(tv, (int)k, f->d_trsm_ws, f->d_dinv + k * f->nb * 32, fp8_panel, P); }));
    if (f->task_cnt[k * 5 + F8] > 0)  // operand scales of the FP8 updates (buffer of this step's parity)
      HIP_TRY(ctx, launch_panel_amax(tv, (int)k, f->d_pamax + (k & 1) * nt, P));
    // split panel of the FP32 updates (this step's parity: the buffer was last
    // read by step k-2, whose updates P and C have waited for)
    {
      uint16_t* o3 = (split32 && f->task_cnt[k * 5 + F32] > 0) ? f->d_split + (k & 1) * split_stride : nullptr;
      uint16_t* ob = (pack16 && f->task_cnt[k * 5 + BF16] > 0) ? f->d_b16 + (k & 1) * b16_stride : nullptr;
      HIP_TRY(ctx, launch_pack_split(tv, (int)k, o3, ob, P));
    }
    HIP_TRY(ctx, hipEventRecord(ev(2 * k), P));
    // P next updates the diagonal tile (k+1, k+1), last written by U in step
    // k-1 (diagonal tiles are FP64).  It does not wait for U2: the FP32 and
    // lower tiles of step k-1 matter to P only from TRSM(k+1) on (the panel
    // tiles, and the split-panel buffer that pack(k+1) rewrites), and C, which
    // P waits for before TRSM(k+1), has waited for U2.  POTRF(k+1) thus
    // overlaps the tail of step k-1's lower-format update.
    if (k > 0) HIP_TRY(ctx, hipStreamWaitEvent(P, ev(2 * (k - 1) + 1), 0));
    if ((rc = launch_updates(k, P, 0)) != MPCR_OK) return rc;
    HIP_TRY(ctx, hipStreamWaitEvent(C, ev(2 * k), 0));
    if (k > 0) {
      HIP_TRY(ctx, hipStreamWaitEvent(C, ev(2 * (k - 1) + 1), 0));
      HIP_TRY(ctx, hipStreamWaitEvent(C, ev2(k - 1), 0));
    }
    if ((rc = launch_updates(k, C, 1)) != MPCR_OK) return rc;
    HIP_TRY(ctx, hipEventRecord(evc(k), C));
    HIP_TRY(ctx, hipStreamWaitEvent(U, ev(2 * k), 0));
    if (U2 != U) HIP_TRY(ctx, hipStreamWaitEvent(U2, ev(2 * k), 0));
    if ((rc = launch_updates(k, U, 2)) != MPCR_OK) return rc;
    HIP_TRY(ctx, hipEventRecord(ev(2 * k + 1), U));
    HIP_TRY(ctx, hipEventRecord(ev2(k), U2));
  }
  HIP_TRY(ctx, hipStreamWaitEvent(P, ev(2 * nt - 1), 0));  // join
  HIP_TRY(ctx, hipStreamWaitEvent(P, ev2(nt - 1), 0));
  HIP_TRY(ctx, hipStreamWaitEvent(P, evc(nt - 1), 0));
  return MPCR_OK;
}

int read_info(mpcr_ctx* ctx, mpcr_factor* f, int64_t* h_info) {
  int info = 0;
  HIP_TRY(ctx, hipMemcpyAsync(&info, f->d_info, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  drain_timing(ctx);
  f->info = info;
  if (h_info) *h_info = info;
  if (info) return set_err(ctx, MPCR_ERR_NOT_SPD, "leading minor of order %d is not positive definite", info);
  return MPCR_OK;
}

int ensure_linv(mpcr_ctx* ctx, mpcr_factor* f) {
  if (f->linv_ready) return MPCR_OK;
  if (!f->d_Linv) HIP_TRY(ctx, dmalloc(f->arena, &f->d_Linv, (size_t)f->nt * f->nb * f->nb * 8));
  const double nb3 = (double)f->nb * f->nb * f->nb;
  HIP_TRY(ctx, timed(ctx, ctx->stream, 7, nb3 / 3.0 * (double)f->nt,
                     [&] { return launch_trtri_diag(f->view(), f->d_Linv, f->d_dinv, ctx->stream); }));
  f->linv_ready = true;
  return MPCR_OK;
}

// Padded-order FP64 work blocks for the solves.
struct SolveBufs {
  int64_t N = 0, nrhs = 0;
  double *B = nullptr, *X = nullptr, *W = nullptr, *R = nullptr, *V = nullptr;  // N x nrhs each
  double *P = nullptr, *Q = nullptr, *Z = nullptr;
  double* S = nullptr;  // one solved block by rows (N x nrhs reserved)
  double *scal = nullptr;  // small per-column scalars
  double *partial = nullptr;
  int* active = nullptr;
};

int64_t solve_bytes(int64_t N, int64_t nrhs, int64_t n) {
  int64_t blk = N * nrhs * 8;
  int64_t nslab = (n + 1023) / 1024 + 1;
  return 9 * blk + 16 * nrhs * 8 + nslab * nrhs * 5 * 8 + nrhs * 4 + 4096;
}

int carve(mpcr_ctx* ctx, int64_t N, int64_t nrhs, int64_t n, SolveBufs& b) {
  int64_t need = solve_bytes(N, nrhs, n);
  if (ctx->ws_vec_bytes < need) {
    dfree(ctx->arena, ctx->ws_vec);
    ctx->ws_vec = nullptr;
    ctx->ws_vec_bytes = 0;
    HIP_TRY(ctx, dmalloc(ctx->arena, &ctx->ws_vec, (size_t)need));
    ctx->ws_vec_bytes = need;
  }
  char* p = (char*)ctx->ws_vec;
  int64_t blk = N * nrhs * 8;
  b.N = N;
  b.nrhs = nrhs;
  double** blocks[9] = {&b.B, &b.X, &b.W, &b.R, &b.V, &b.P, &b.Q, &b.Z, &b.S};
  for (auto bp : blocks) {
    *bp = (double*)p;
    p += blk;
  }
  b.scal = (double*)p;
  p += 16 * nrhs * 8;
  int64_t nslab = (n + 1023) / 1024 + 1;
  b.partial = (double*)p;
  p += nslab * nrhs * 5 * 8;
  b.active = (int*)p;
  HIP_TRY(ctx, launch_fill(ctx->ws_vec, 9 * N * nrhs, 0.0, ctx->stream));
  return MPCR_OK;
}

// X = M^{-1} B with M = L L^T over the tiles; also leaves W = L^{-1} B.
int tile_solve(mpcr_ctx* ctx, mpcr_factor* f, SolveBufs& b, const double* Bsrc, double* Xdst, double* Wdst,
               bool backward = true) {
  hipStream_t s = ctx->stream;
  TileView tv = f->view();
  const int nrhs = (int)b.nrhs;
  const int64_t ld = b.N;
  // algorithmic flops: 2 N^2 nrhs per triangular sweep
  const double fl = 2.0 * (double)f->N * (double)f->N * nrhs * (backward ? 2.0 : 1.0);
  hipError_t e = timed(ctx, s, 8, fl, [&]() -> hipError_t {
    // b.V is the working copy of both sweeps, so Bsrc may be any other block
    hipError_t r = launch_copy_cols((int)f->N, nrhs, Bsrc, ld, b.V, ld, s);
    for (int64_t k = 0; k < f->nt && r == hipSuccess; ++k) {
      r = launch_fwd_diag(tv, f->d_Linv, (int)k, b.V, Wdst, ld, nrhs, b.S, s);
      if (r == hipSuccess) r = launch_fwd_update(tv, (int)k, b.V, b.S, ld, nrhs, s);
    }
    if (!backward || r != hipSuccess) return r;
    r = launch_copy_cols((int)f->N, nrhs, Wdst, ld, b.V, ld, s);
    for (int64_t k = f->nt - 1; k >= 0 && r == hipSuccess; --k) {
      r = launch_bwd_diag(tv, f->d_Linv, (int)k, b.V, Xdst, ld, nrhs, b.S, s);
      if (r == hipSuccess) r = launch_bwd_update(tv, (int)k, b.V, b.S, ld, nrhs, s);
    }
    return r;
  });
  HIP_TRY(ctx, e);
  return MPCR_OK;
}

// Sigma application for refinement: either matrix-free from sites or a dense FP64 matrix.
struct SigmaOp {
  mpcr_ctx* ctx = nullptr;  // for kernel timing
  const double* sig = nullptr;  // stored FP64 lower tiles (preferred when set)
  double* part = nullptr;       // their partial-product workspace
  int nb = 0, nt = 0;
  const double* locs = nullptr;
  mpcr_theta_t th{};
  const double* A = nullptr;
  int64_t lda = 0;
  int n = 0;
  hipError_t residual(const double* B, const double* X, double* R, int64_t ld, int nrhs, hipStream_t s,
                      double* rowsum = nullptr) const {
    auto go = [&] {
      if (sig) return launch_residual_tiles(n, nb, nt, sig, B, X, R, ld, nrhs, s, rowsum, part);
      return A ? launch_residual_dense(n, A, lda, B, X, R, ld, nrhs, s, rowsum)
               : launch_residual_cov(n, locs, th, B, X, R, ld, nrhs, s, rowsum);
    };
    return ctx ? timed(ctx, s, 9, 2.0 * (double)n * n * nrhs, go) : go();
  }
  hipError_t rowsum(double* out, hipStream_t s) const {
    return A ? launch_rowsum_abs_dense(n, A, lda, out, s) : launch_rowsum_abs_cov(n, locs, th, out, s);
  }
};

// Solver options common to mpcr_potrs and mpcr_gauss_loglik.
bool refine_opts_ok(const mpcr_refine_opts_t& o) {
  return o.tol > 0 && o.max_iter >= 0 && o.solver >= 0 && o.solver <= 3 && o.recompute >= 0 && o.gmres_m >= 0 &&
         o.gmres_m <= 64 && o.gmres_inner_tol >= 0 && o.gmres_inner_tol < 1 && o.block_size >= 0 &&
         o.block_size <= KRYLOV_MAX_BLOCK;
}

// Krylov workspace of at least `bytes` bytes (kept by the context).
int krylov_ws(mpcr_ctx* ctx, int64_t bytes, char** out) {
  if (ctx->ws_kry_bytes < bytes) {
    dfree(ctx->arena, ctx->ws_kry);
    ctx->ws_kry = nullptr;
    ctx->ws_kry_bytes = 0;
    HIP_TRY(ctx, dmalloc(ctx->arena, &ctx->ws_kry, (size_t)bytes));
    ctx->ws_kry_bytes = bytes;
  }
  *out = (char*)ctx->ws_kry;
  return MPCR_OK;
}

// Refined solve of Sigma X = B (PCG, IR, GMRES-IR or block PCG); B, X in
// b.B / b.X (padded N x nrhs).
int refine(mpcr_ctx* ctx, mpcr_factor* f, SolveBufs& b, const SigmaOp& op, const mpcr_refine_opts_t& o,
           mpcr_diag_t* diag, bool* converged_out) {
  TraceRange tr("refinement");
  hipStream_t s = ctx->stream;
  const int n = (int)f->n, nrhs = (int)b.nrhs;
  const int64_t ld = b.N;
  double* sig_inf = b.scal;                // [0]
  double* rz = b.scal + nrhs;              // nrhs
  double* pq = b.scal + 2 * nrhs;
  double* alpha = b.scal + 3 * nrhs;
  double* beta = b.scal + 4 * nrhs;
  double* rzn = b.scal + 5 * nrhs;
  double* stats = b.scal + 6 * nrhs;       // 2 nrhs
  double* rowsum = b.Z;                    // temporary use before Z is needed

  std::vector<double> hst(2 * nrhs);
  std::vector<int> act(nrhs, 1);
  auto col_converged = [&](int c) { return hst[2 * c] <= o.tol; };
  auto fetch_stats = [&](const double* R) -> int {
    HIP_TRY(ctx, launch_col_stats(n, nrhs, R, b.X, b.B, ld, sig_inf, b.partial, stats, s));
    HIP_TRY(ctx, hipMemcpyAsync(hst.data(), stats, 2 * nrhs * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    return MPCR_OK;
  };
  auto push_active = [&]() -> int {
    HIP_TRY(ctx, hipMemcpyAsync(b.active, act.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, s));
    return MPCR_OK;
  };

  int rc;
  // x0 = M^{-1} b, r0 = b - Sigma x0 (the same pass gives ||Sigma||_inf)
  if ((rc = tile_solve(ctx, f, b, b.B, b.X, b.W)) != MPCR_OK) return rc;
  HIP_TRY(ctx, op.residual(b.B, b.X, b.R, ld, nrhs, s, rowsum));
  HIP_TRY(ctx, launch_max_reduce(n, rowsum, b.partial, sig_inf, s));
  if ((rc = fetch_stats(b.R)) != MPCR_OK) return rc;
  int nact = 0;
  for (int c = 0; c < nrhs; ++c) {
    act[c] = col_converged(c) ? 0 : 1;
    nact += act[c];
  }
  if ((rc = push_active()) != MPCR_OK) return rc;
  int it = 0;
  bool r_true = true;  // R (and the fetched statistics) hold the true residual of the current X

  // PCG from the current X, whose true residual is in R, on the active columns
  auto pcg_loop = [&]() -> int {
    int rc2;
    if ((rc2 = tile_solve(ctx, f, b, b.R, b.Z, b.W)) != MPCR_OK) return rc2;  // z = M^{-1} r
    HIP_TRY(ctx, launch_copy_cols((int)b.N, nrhs, b.Z, ld, b.P, ld, s));
    HIP_TRY(ctx, launch_col_dot(n, nrhs, b.R, b.Z, ld, b.partial, rz, s));
    while (nact > 0 && it < o.max_iter) {
      ++it;
      // q = Sigma p  (as -(0 - Sigma p) through the residual kernel with a zero right-hand side)
      HIP_TRY(ctx, op.residual(nullptr, b.P, b.Q, ld, nrhs, s));  // Q = -Sigma P
      HIP_TRY(ctx, launch_col_dot(n, nrhs, b.P, b.Q, ld, b.partial, pq, s));  // = -p^T Sigma p
      HIP_TRY(ctx, launch_pcg_alpha(nrhs, rz, pq, b.active, alpha, s));      // = -alpha
      HIP_TRY(ctx, launch_axpy_cols(n, nrhs, alpha, -1.0, b.P, b.X, ld, s)); // x += alpha p
      if (o.recompute > 0 && it % o.recompute == 0) {
        HIP_TRY(ctx, op.residual(b.B, b.X, b.R, ld, nrhs, s));
        r_true = true;
      } else {
        HIP_TRY(ctx, launch_axpy_cols(n, nrhs, alpha, -1.0, b.Q, b.R, ld, s)); // r -= alpha Sigma p
        r_true = false;
      }
      if ((rc2 = fetch_stats(b.R)) != MPCR_OK) return rc2;
      bool any = false;
      for (int c = 0; c < nrhs; ++c) any |= act[c] && col_converged(c);
      if (any) {  // confirm with the true residual
        HIP_TRY(ctx, op.residual(b.B, b.X, b.W, ld, nrhs, s));
        if ((rc2 = fetch_stats(b.W)) != MPCR_OK) return rc2;
        HIP_TRY(ctx, launch_copy_cols(n, nrhs, b.W, ld, b.R, ld, s));
        r_true = true;
        for (int c = 0; c < nrhs; ++c)
          if (act[c] && col_converged(c)) {
            act[c] = 0;
            --nact;
          }
        if ((rc2 = push_active()) != MPCR_OK) return rc2;
      }
      if (nact == 0 || it >= o.max_iter) break;
      if ((rc2 = tile_solve(ctx, f, b, b.R, b.Z, b.W)) != MPCR_OK) return rc2;
      HIP_TRY(ctx, launch_col_dot(n, nrhs, b.R, b.Z, ld, b.partial, rzn, s));
      HIP_TRY(ctx, launch_pcg_beta(nrhs, rzn, rz, b.active, beta, s));
      HIP_TRY(ctx, launch_xpby_cols(n, nrhs, b.Z, beta, b.P, ld, s));
    }
    return MPCR_OK;
  };

  if (o.solver == 0 && nact > 0) {
    if ((rc = pcg_loop()) != MPCR_OK) return rc;
  } else if (o.solver == 1) {
    while (nact > 0 && it < o.max_iter) {
      ++it;
      if ((rc = tile_solve(ctx, f, b, b.R, b.Z, b.W)) != MPCR_OK) return rc;
      // x += d for active columns (alpha = active ? 1 : 0)
      std::vector<double> ones(nrhs);
      for (int c = 0; c < nrhs; ++c) ones[c] = act[c] ? 1.0 : 0.0;
      HIP_TRY(ctx, hipMemcpyAsync(alpha, ones.data(), nrhs * 8, hipMemcpyHostToDevice, s));
      HIP_TRY(ctx, launch_axpy_cols(n, nrhs, alpha, 1.0, b.Z, b.X, ld, s));
      HIP_TRY(ctx, op.residual(b.B, b.X, b.R, ld, nrhs, s));
      if ((rc = fetch_stats(b.R)) != MPCR_OK) return rc;
      for (int c = 0; c < nrhs; ++c)
        if (act[c] && col_converged(c)) {
          act[c] = 0;
          --nact;
        }
    }
  } else if (o.solver == 2 && nact > 0) {
    // GMRES-IR: per refinement step, GMRES on M^-1 Sigma d = M^-1 r for every
    // active column (one Hessenberg matrix per column), then x += d and the
    // true residual.
    const int m = o.gmres_m > 0 ? o.gmres_m : 20;
    const double itol = o.gmres_inner_tol > 0 ? o.gmres_inner_tol : 1e-6;
    const int64_t blk = ld * nrhs;
    const int64_t need = 8 * ((int64_t)(m + 1) * blk + (int64_t)nrhs * ((m + 1) * m + 3 * (m + 1) + m + 8)) +
                         4 * 3 * nrhs + 1024;
    char* w;
    if ((rc = krylov_ws(ctx, need, &w)) != MPCR_OK) return rc;
    double* V = (double*)w;                                   // m + 1 blocks
    double* H = V + (int64_t)(m + 1) * blk;                   // nrhs x (m+1) x m
    double* cs = H + (int64_t)nrhs * (m + 1) * m;             // nrhs x (m+1)
    double* sn = cs + (int64_t)nrhs * (m + 1);
    double* g = sn + (int64_t)nrhs * (m + 1);
    double* y = g + (int64_t)nrhs * (m + 1);                  // nrhs x m
    double* bet = y + (int64_t)nrhs * m;                      // nrhs
    double* inv = bet + nrhs;
    double* dotv = inv + nrhs;
    double* out = dotv + nrhs;                                // 2 nrhs
    double* neg1 = out + 2 * nrhs;                            // nrhs
    int* run_d = (int*)(neg1 + nrhs);
    int* steps_d = run_d + nrhs;
    HIP_TRY(ctx, launch_fill(neg1, nrhs, -1.0, s));
    HIP_TRY(ctx, launch_fill(V, (int64_t)(m + 1) * blk, 0.0, s));
    std::vector<double> hbeta(nrhs), hout(2 * nrhs);
    std::vector<int> run(nrhs), steps(nrhs);
    while (nact > 0 && it < o.max_iter) {
      ++it;
      if ((rc = push_active()) != MPCR_OK) return rc;
      // v0 = M^-1 r / |M^-1 r|
      if ((rc = tile_solve(ctx, f, b, b.R, V, b.W)) != MPCR_OK) return rc;
      HIP_TRY(ctx, launch_col_dot(n, nrhs, V, V, ld, b.partial, dotv, s));
      HIP_TRY(ctx, launch_gmres_start(nrhs, m, dotv, b.active, bet, g, inv, s));
      HIP_TRY(ctx, launch_scale_cols(n, nrhs, inv, V, V, ld, s));
      HIP_TRY(ctx, hipMemcpyAsync(hbeta.data(), bet, nrhs * 8, hipMemcpyDeviceToHost, s));
      HIP_TRY(ctx, hipStreamSynchronize(s));
      int nrun = 0;
      for (int c = 0; c < nrhs; ++c) {
        run[c] = act[c] && hbeta[c] > 0.0;
        steps[c] = 0;
        nrun += run[c];
      }
      int jmax = 0;
      for (int j = 0; j < m && nrun > 0; ++j) {
        HIP_TRY(ctx, hipMemcpyAsync(run_d, run.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, s));
        const double* vj = V + (int64_t)j * blk;
        // w = M^-1 Sigma v_j (the residual kernel gives -Sigma v_j)
        HIP_TRY(ctx, op.residual(nullptr, vj, b.Q, ld, nrhs, s));
        if ((rc = tile_solve(ctx, f, b, b.Q, b.Z, b.W)) != MPCR_OK) return rc;
        HIP_TRY(ctx, launch_scale_cols(n, nrhs, neg1, b.Z, b.Z, ld, s));
        // modified Gram-Schmidt against v_0 .. v_j
        const int64_t hs = (int64_t)(m + 1) * m;
        for (int i = 0; i <= j; ++i) {
          double* hij = H + (int64_t)(m + 1) * j + i;
          HIP_TRY(ctx, launch_col_dot_strided(n, nrhs, V + (int64_t)i * blk, b.Z, ld, b.partial, hij, hs, s));
          HIP_TRY(ctx, launch_axpy_strided(n, nrhs, hij, hs, -1.0, V + (int64_t)i * blk, b.Z, ld, s));
        }
        HIP_TRY(ctx, launch_col_dot(n, nrhs, b.Z, b.Z, ld, b.partial, dotv, s));
        HIP_TRY(ctx, launch_gmres_rotate(nrhs, m, j, dotv, run_d, H, cs, sn, g, out, s));
        HIP_TRY(ctx, hipMemcpyAsync(hout.data(), out, 2 * nrhs * 8, hipMemcpyDeviceToHost, s));
        HIP_TRY(ctx, hipStreamSynchronize(s));
        jmax = j + 1;
        for (int c = 0; c < nrhs; ++c) {
          if (!run[c]) continue;
          steps[c] = j + 1;
          if (hout[2 * c] <= itol * hbeta[c] || hout[2 * c + 1] == 0.0) {
            run[c] = 0;
            --nrun;
          }
        }
        if (nrun == 0 || j + 1 == m) break;
        // v_{j+1} = w / |w| for the columns that continue (0 for the others)
        HIP_TRY(ctx, hipMemcpyAsync(run_d, run.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, s));
        HIP_TRY(ctx, launch_gmres_inv(nrhs, out, run_d, inv, s));
        HIP_TRY(ctx, launch_scale_cols(n, nrhs, inv, b.Z, V + (int64_t)(j + 1) * blk, ld, s));
      }
      // x += V_k y, y from the rotated Hessenberg system
      HIP_TRY(ctx, hipMemcpyAsync(steps_d, steps.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, s));
      HIP_TRY(ctx, launch_gmres_backsolve(nrhs, m, H, g, steps_d, y, s));
      for (int i = 0; i < jmax; ++i)
        HIP_TRY(ctx, launch_axpy_strided(n, nrhs, y + i, m, 1.0, V + (int64_t)i * blk, b.X, ld, s));
      HIP_TRY(ctx, op.residual(b.B, b.X, b.R, ld, nrhs, s));
      if ((rc = fetch_stats(b.R)) != MPCR_OK) return rc;
      for (int c = 0; c < nrhs; ++c)
        if (act[c] && col_converged(c)) {
          act[c] = 0;
          --nact;
        }
    }
    r_true = true;
  } else if (o.solver == 3 && nact > 0) {
    // block PCG on groups of bs consecutive columns, all groups in lockstep
    const int bs = o.block_size > 0 ? std::min(o.block_size, nrhs) : std::min(nrhs, KRYLOV_MAX_BLOCK);
    const int ng = (nrhs + bs - 1) / bs;
    const int64_t sq = (int64_t)ng * bs * bs;
    const int64_t need = 8 * 5 * sq + (int64_t)gram_partial_bytes(n, nrhs, bs) + 4 * 2 * ng + 1024;
    char* w;
    if ((rc = krylov_ws(ctx, need, &w)) != MPCR_OK) return rc;
    double* PQ = (double*)w;   // P^T Sigma P
    double* ZR = PQ + sq;      // Z^T R (current)
    double* ZRn = ZR + sq;     // Z^T R (next)
    double* CA = ZRn + sq;     // alpha
    double* CB = CA + sq;      // beta
    double* part = CB + sq;    // Gram partials
    int* gact_d = (int*)((char*)part + gram_partial_bytes(n, nrhs, bs));
    int* flag_d = gact_d + ng;
    std::vector<int> gact(ng), flag(ng), broken(ng, 0);
    auto group_state = [&]() {
      int na = 0;
      for (int g = 0; g < ng; ++g) {
        bool any = false;
        for (int c = g * bs; c < std::min(nrhs, (g + 1) * bs); ++c) any |= !col_converged(c);
        gact[g] = any && !broken[g];
        na += gact[g];
      }
      return na;
    };
    auto push_groups = [&]() -> int {
      HIP_TRY(ctx, hipMemcpyAsync(gact_d, gact.data(), ng * sizeof(int), hipMemcpyHostToDevice, s));
      return MPCR_OK;
    };
    auto take_flags = [&]() -> int {  // groups whose s x s system broke down leave the block iteration
      HIP_TRY(ctx, hipMemcpyAsync(flag.data(), flag_d, ng * sizeof(int), hipMemcpyDeviceToHost, s));
      HIP_TRY(ctx, hipStreamSynchronize(s));
      for (int g = 0; g < ng; ++g)
        if (flag[g]) broken[g] = 1;
      return MPCR_OK;
    };
    int nga = group_state();
    if ((rc = push_groups()) != MPCR_OK) return rc;
    if (nga > 0) {
      if ((rc = tile_solve(ctx, f, b, b.R, b.Z, b.W)) != MPCR_OK) return rc;  // Z = M^-1 R
      HIP_TRY(ctx, launch_copy_cols((int)b.N, nrhs, b.Z, ld, b.P, ld, s));
      HIP_TRY(ctx, launch_group_gram(n, nrhs, bs, b.Z, b.R, ld, part, ZR, 1.0, s));
    }
    while (nga > 0 && it < o.max_iter) {
      // Q = -Sigma P; PQ = P^T Sigma P; alpha = PQ^-1 ZR
      HIP_TRY(ctx, op.residual(nullptr, b.P, b.Q, ld, nrhs, s));
      HIP_TRY(ctx, launch_group_gram(n, nrhs, bs, b.P, b.Q, ld, part, PQ, -1.0, s));
      HIP_TRY(ctx, launch_group_spd_solve(nrhs, bs, PQ, ZR, gact_d, CA, flag_d, s));
      if ((rc = take_flags()) != MPCR_OK) return rc;
      ++it;
      HIP_TRY(ctx, launch_group_axpy(n, nrhs, bs, b.P, CA, 1.0, b.X, ld, s));    // X += P alpha
      if (o.recompute > 0 && it % o.recompute == 0) {
        HIP_TRY(ctx, op.residual(b.B, b.X, b.R, ld, nrhs, s));
        r_true = true;
      } else {
        HIP_TRY(ctx, launch_group_axpy(n, nrhs, bs, b.Q, CA, 1.0, b.R, ld, s));  // R -= Sigma P alpha
        r_true = false;
      }
      if ((rc = fetch_stats(b.R)) != MPCR_OK) return rc;
      bool check = false;  // a group whose columns all meet the tolerance is confirmed with the true residual
      for (int g = 0; g < ng; ++g) {
        if (!gact[g]) continue;
        bool all = true;
        for (int c = g * bs; c < std::min(nrhs, (g + 1) * bs); ++c) all &= col_converged(c);
        check |= all;
      }
      if (check) {
        HIP_TRY(ctx, op.residual(b.B, b.X, b.W, ld, nrhs, s));
        if ((rc = fetch_stats(b.W)) != MPCR_OK) return rc;
        HIP_TRY(ctx, launch_copy_cols(n, nrhs, b.W, ld, b.R, ld, s));
        r_true = true;
      }
      nga = group_state();
      if ((rc = push_groups()) != MPCR_OK) return rc;
      if (nga == 0 || it >= o.max_iter) break;
      // Z = M^-1 R; beta = ZR^-1 ZRn; P = Z + P beta
      if ((rc = tile_solve(ctx, f, b, b.R, b.Z, b.W)) != MPCR_OK) return rc;
      HIP_TRY(ctx, launch_group_gram(n, nrhs, bs, b.Z, b.R, ld, part, ZRn, 1.0, s));
      HIP_TRY(ctx, launch_group_spd_solve(nrhs, bs, ZR, ZRn, gact_d, CB, flag_d, s));
      if ((rc = take_flags()) != MPCR_OK) return rc;
      HIP_TRY(ctx, hipMemcpyAsync(ZR, ZRn, sq * 8, hipMemcpyDeviceToDevice, s));
      HIP_TRY(ctx, launch_group_xpyc(n, nrhs, bs, b.Z, CB, b.P, ld, s));
      nga = group_state();
      if ((rc = push_groups()) != MPCR_OK) return rc;
    }
    // groups that broke down finish with PCG from their current iterate
    bool any_broken = false;
    for (int g = 0; g < ng; ++g) any_broken |= broken[g] != 0;
    if (any_broken && it < o.max_iter) {
      if (!r_true) {
        HIP_TRY(ctx, op.residual(b.B, b.X, b.R, ld, nrhs, s));
        if ((rc = fetch_stats(b.R)) != MPCR_OK) return rc;
        r_true = true;
      }
      nact = 0;
      for (int c = 0; c < nrhs; ++c) {
        act[c] = broken[c / bs] && !col_converged(c);
        nact += act[c];
      }
      if ((rc = push_active()) != MPCR_OK) return rc;
      if (nact > 0 && (rc = pcg_loop()) != MPCR_OK) return rc;
    }
  }
  // final true residual and statistics (already current when the last step
  // confirmed convergence with the true residual)
  if (!r_true) {
    HIP_TRY(ctx, op.residual(b.B, b.X, b.R, ld, nrhs, s));
    if ((rc = fetch_stats(b.R)) != MPCR_OK) return rc;
  }
  bool conv = true;
  double eta = 0, rel = 0;
  for (int c = 0; c < nrhs; ++c) {
    conv &= col_converged(c);
    eta = std::max(eta, hst[2 * c]);
    rel = std::max(rel, hst[2 * c + 1]);
  }
  if (diag) {
    diag->iters = it;
    diag->converged = conv ? 1 : 0;
    diag->eta = eta;
    diag->rel_resid2 = rel;
  }
  *converged_out = conv;
  return MPCR_OK;
}

float ev_ms(hipEvent_t a, hipEvent_t b) {
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, a, b) != hipSuccess) ms = 0.f;
  return ms;
}

}  // namespace

// ===========================================================================
// internal helpers for the serving engine
// ===========================================================================
namespace mpcr {
int ctx_create_with_arena(int device, Arena* arena, mpcr_ctx** out) {
  DeviceGuard g(device);
  hipStream_t s = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);  // default priority
  if (e != hipSuccess) return set_err(nullptr, MPCR_ERR_DEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
  int rc = mpcr_ctx_create(device, (void*)s, out);
  if (rc != MPCR_OK) {
    (void)hipStreamDestroy(s);
    return rc;
  }
  (*out)->arena = arena;
  (*out)->own_stream = true;
  return MPCR_OK;
}

void ctx_release_workspace(mpcr_ctx* ctx) {
  DeviceGuard g(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  free_factor(ctx->ws_factor);
  ctx->ws_factor = nullptr;
  ctx->ws_map.clear();
  ctx->ws_n = ctx->ws_nb = -1;
  dfree(ctx->arena, ctx->ws_locs);
  ctx->ws_locs = nullptr;
  dfree(ctx->arena, ctx->ws_vec);
  ctx->ws_vec = nullptr;
  ctx->ws_vec_bytes = 0;
  dfree(ctx->arena, ctx->ws_kry);
  ctx->ws_kry = nullptr;
  ctx->ws_kry_bytes = 0;
  dfree(ctx->arena, ctx->ws_gemm);
  ctx->ws_gemm = nullptr;
  ctx->ws_gemm_bytes = 0;
}

hipStream_t ctx_stream(mpcr_ctx* ctx) { return ctx->stream; }

size_t loglik_footprint(int64_t n, int64_t nb, int64_t nrhs) {
  const int64_t nt = (n + nb - 1) / nb, N = nt * nb;
  const int64_t tile = nb * nb * 8;
  size_t bytes = 0;
  bytes += (size_t)(nt * (nt + 1) / 2) * tile;            // tiles (FP64 bound)
  bytes += (size_t)std::max<int64_t>(nt - 1, 1) * tile;     // TRSM workspace
  bytes += (size_t)nt * nb * 32 * 8;                        // inverted 32 x 32 diagonal blocks
  bytes += (size_t)nt * tile;                               // inverted diagonal tiles
  bytes += (size_t)std::max<int64_t>(nt - 1, 1) * nb * nb * 16;  // split FP32 and BF16 panels of the updates
  bytes += (size_t)solve_bytes(N, nrhs, n);                 // vectors
  bytes += (size_t)n * 24 + (size_t)nt * nt * 16 + 65536;   // sites, permutation, tables
  size_t npow2 = 1;
  while ((int64_t)npow2 < n) npow2 <<= 1;
  bytes += npow2 * 8;                                       // ordering keys
  return bytes + (bytes >> 5);                              // allocator granules
}
}  // namespace mpcr

namespace {
// One Laplace evaluation at theta (see mpcr_inla_posterior): Newton iterations
// for the mode of p(x | y) with B = I + W^1/2 Sigma W^1/2 factored in the tile
// store, then l(theta) = log p(y | x) - x^T Sigma^-1 x / 2 - log|B| / 2.
int laplace_one(mpcr_ctx* ctx, int64_t n, int64_t nb, const std::vector<uint8_t>& m, const double* d_locs,
                const double* d_y, const mpcr_theta_t& th, double beta, double tol, int max_newton, double* vec,
                double* h_lpost, int* h_iters) {
  hipStream_t s = ctx->stream;
  if (!ctx->ws_factor || ctx->ws_factor->n != n || ctx->ws_nb != nb || ctx->ws_map != m) {
    free_factor(ctx->ws_factor);
    ctx->ws_factor = nullptr;
    ctx->ws_map.clear();
    int r = make_factor(ctx, n, nb, m, &ctx->ws_factor);
    if (r != MPCR_OK) return r;
    ctx->ws_nb = nb;
    ctx->ws_map = m;
  }
  mpcr_factor* f = ctx->ws_factor;
  SolveBufs b;
  int rc = carve(ctx, f->N, 1, n, b);
  if (rc) return rc;
  double *x = vec, *g = vec + n, *sw = vec + 2 * n, *lik = vec + 3 * n, *rhs = vec + 4 * n, *t = vec + 5 * n,
         *a = vec + 6 * n, *xn = vec + 7 * n, *d = vec + 8 * n, *ones = vec + 9 * n, *red = vec + 10 * n;
  double* partial = b.partial;
  HIP_TRY(ctx, launch_fill(x, n, 0.0, s));
  HIP_TRY(ctx, launch_fill(ones, n, 1.0, s));
  SigmaOp op;
  op.ctx = nullptr;
  op.locs = d_locs;
  op.th = th;
  op.n = (int)n;
  auto factor_B = [&]() -> int {
    HIP_TRY(ctx, hipMemsetAsync(f->d_info, 0, sizeof(int), s));
    HIP_TRY(ctx, launch_tiles_from_weighted_covariance(f->view(), d_locs, th, sw, s));
    int r = run_factorisation(ctx, f);
    if (r) return r;
    int64_t info = 0;
    return read_info(ctx, f, &info);
  };
  int it = 0;
  for (;;) {
    ++it;
    HIP_TRY(ctx, launch_laplace_terms((int)n, beta, x, d_y, g, sw, lik, rhs, s));
    if ((rc = factor_B()) != MPCR_OK) return rc;
    if ((rc = ensure_linv(ctx, f)) != MPCR_OK) return rc;
    HIP_TRY(ctx, op.residual(nullptr, rhs, t, n, 1, s));               // t = -Sigma rhs
    HIP_TRY(ctx, launch_scale((int)n, sw, t, -1.0, b.B, s));            // W^1/2 Sigma rhs
    if ((rc = tile_solve(ctx, f, b, b.B, b.X, b.W)) != MPCR_OK) return rc;  // B^-1 (...)
    HIP_TRY(ctx, launch_laplace_a((int)n, rhs, sw, b.X, a, s));          // a = rhs - W^1/2 B^-1 W^1/2 Sigma rhs
    HIP_TRY(ctx, op.residual(nullptr, a, t, n, 1, s));                  // t = -Sigma a
    HIP_TRY(ctx, launch_scale((int)n, ones, t, -1.0, xn, s));           // x_new = Sigma a
    HIP_TRY(ctx, launch_step_diff((int)n, xn, x, d, s));                 // d = x_new - x, x = x_new
    HIP_TRY(ctx, launch_col_dot((int)n, 1, d, d, n, partial, red, s));
    double ss = 0;
    HIP_TRY(ctx, hipMemcpyAsync(&ss, red, 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    if (!std::isfinite(ss)) return set_err(ctx, MPCR_ERR_NOT_CONVERGED, "Newton iteration diverged");
    if (ss / (double)n < tol) break;
    if (it >= max_newton) return set_err(ctx, MPCR_ERR_NOT_CONVERGED, "Newton iteration reached max_newton");
  }
  // at the mode: W, B and log|B|; x^T Sigma^-1 x = a^T x since x = Sigma a
  HIP_TRY(ctx, launch_laplace_terms((int)n, beta, x, d_y, g, sw, lik, rhs, s));
  if ((rc = factor_B()) != MPCR_OK) return rc;
  HIP_TRY(ctx, launch_logdet(f->view(), red, s));
  HIP_TRY(ctx, launch_col_dot((int)n, 1, a, x, n, partial, red + 1, s));
  HIP_TRY(ctx, launch_col_dot((int)n, 1, lik, ones, n, partial, red + 2, s));
  double h[3];
  HIP_TRY(ctx, hipMemcpyAsync(h, red, 24, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  *h_lpost = h[2] - 0.5 * h[1] - 0.5 * h[0];
  if (h_iters) *h_iters = it;
  return MPCR_OK;
}
}  // namespace

// ===========================================================================
// exported entry points
// ===========================================================================
extern "C" {

const char* mpcr_version(void) { return kVersion; }

int mpcr_ctx_create(int device, void* hip_stream, mpcr_ctx** out) {
  if (!out) return set_err(nullptr, MPCR_ERR_ARG, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev == 0)
    return set_err(nullptr, MPCR_ERR_DEVICE, "hipGetDeviceCount: %s (%d devices)", hipGetErrorString(e), ndev);
  if (device < 0 || device >= ndev) return set_err(nullptr, MPCR_ERR_ARG, "device %d out of range", device);
  auto* c = new mpcr_ctx();
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  DeviceGuard g(device);
  if ((e = morton_noalloc_keys(device, &c->noalloc_keys)) != hipSuccess) {
    delete c;
    return set_err(nullptr, MPCR_ERR_DEVICE, "hipGetSymbolAddress: %s", hipGetErrorString(e));
  }
  for (auto& ev : c->ev)
    if ((e = hipEventCreate(&ev)) != hipSuccess) {
      delete c;
      return set_err(nullptr, MPCR_ERR_DEVICE, "hipEventCreate: %s", hipGetErrorString(e));
    }
  *out = c;
  return MPCR_OK;
}

int mpcr_ctx_destroy(mpcr_ctx* ctx) {
  if (!ctx) return MPCR_ERR_ARG;
  {
    DeviceGuard g(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    free_factor(ctx->ws_factor);
    dfree(ctx->arena, ctx->ws_locs);
    dfree(ctx->arena, ctx->ws_vec);
    dfree(ctx->arena, ctx->ws_kry);
    dfree(ctx->arena, ctx->ws_gemm);
    for (auto& e : ctx->ev) (void)hipEventDestroy(e);
    drain_timing(ctx);
    for (auto& e : ctx->ev_pool) (void)hipEventDestroy(e);
    for (auto& e : ctx->sync_ev) (void)hipEventDestroy(e);
    if (ctx->upd) (void)hipStreamDestroy(ctx->upd);
    if (ctx->col) (void)hipStreamDestroy(ctx->col);
    if (ctx->upd2) (void)hipStreamDestroy(ctx->upd2);
    if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  }
  delete ctx;
  return MPCR_OK;
}

const char* mpcr_last_error(const mpcr_ctx* ctx) { return ctx ? ctx->err.c_str() : g_err.c_str(); }

int mpcr_ctx_set_profiling(mpcr_ctx* ctx, int on) {
  if (!ctx) return MPCR_ERR_ARG;
  ctx->profiling = on != 0;
  return MPCR_OK;
}

int mpcr_ctx_set_fp32_split(mpcr_ctx* ctx, int on) {
  if (!ctx || (on != 0 && on != 1)) return set_err(ctx, MPCR_ERR_ARG, "mpcr_ctx_set_fp32_split: bad arguments");
  ctx->fp32_split = on;
  return MPCR_OK;
}

int mpcr_ctx_reset_stats(mpcr_ctx* ctx) {
  if (!ctx) return MPCR_ERR_ARG;
  for (int k = 0; k < NKIND; ++k) {
    ctx->k_ms[k] = 0;
    ctx->k_flops[k] = 0;
    ctx->k_launches[k] = 0;
  }
  return MPCR_OK;
}

int mpcr_ctx_kernel_stats(const mpcr_ctx* ctx, int kind, double* h_total_ms, int64_t* h_launches, double* h_flops) {
  if (!ctx || kind < 0 || kind >= NKIND) return MPCR_ERR_ARG;
  if (h_total_ms) *h_total_ms = ctx->k_ms[kind];
  if (h_launches) *h_launches = ctx->k_launches[kind];
  if (h_flops) *h_flops = ctx->k_flops[kind];
  return MPCR_OK;
}

int mpcr_tilemap_banded(int64_t n, int64_t nb, const int* band_dmax, const int* precs, int nbands,
                        uint8_t* h_map_out) {
  if (n < 0 || nb <= 0 || !band_dmax || !precs || nbands <= 0 || !h_map_out) return MPCR_ERR_ARG;
  int64_t nt = (n + nb - 1) / nb;
  for (int b = 0; b < nbands; ++b)
    if (!valid_prec(precs[b])) return MPCR_ERR_ARG;
  for (int64_t i = 0; i < nt; ++i)
    for (int64_t j = 0; j < nt; ++j) {
      if (j > i) {
        h_map_out[i * nt + j] = 255;
        continue;
      }
      int64_t d = i - j;
      int p = -1;
      for (int b = 0; b < nbands; ++b)
        if (band_dmax[b] < 0 || d <= band_dmax[b]) {
          p = precs[b];
          break;
        }
      if (p < 0) return MPCR_ERR_ARG;
      if (d == 0 && p != F64) return MPCR_ERR_ARG;
      h_map_out[i * nt + j] = (uint8_t)p;
    }
  return MPCR_OK;
}

int mpcr_tilemap_guarded(int64_t n, int64_t nb, const uint8_t* h_banded_map, const double* h_tile_amax,
                         double guard, uint8_t* h_map_out) {
  if (n < 0 || nb <= 0 || !h_banded_map || !h_tile_amax || !h_map_out || !(guard > 0)) return MPCR_ERR_ARG;
  int64_t nt = (n + nb - 1) / nb;
  // precision rank: FP8 0, FP16/BF16 1, FP32 2, FP64 3
  auto rank = [](int p) { return p == F64 ? 3 : p == F32 ? 2 : p == F8 ? 0 : 1; };
  for (int64_t i = 0; i < nt; ++i)
    for (int64_t j = 0; j < nt; ++j) {
      int64_t t = i * nt + j;
      if (j > i) {
        h_map_out[t] = 255;
        continue;
      }
      int p = h_banded_map[t];
      if (!valid_prec(p)) return MPCR_ERR_ARG;
      if (i == j && p != F64) return MPCR_ERR_ARG;
      // promote until the rounding error bound max(u_p amax, floor_p) <= guard
      auto too_coarse = [&](int f) {
        return std::max(fmt_unit_roundoff(f) * h_tile_amax[t], fmt_abs_floor(f)) > guard;
      };
      while (p != F64 && too_coarse(p)) {
        int r = rank(p);
        p = r == 0 ? F16 : (r == 1 ? F32 : F64);
        if (rank(p) == 1 && h_banded_map[t] == BF16) p = BF16;  // stay in the map's 16-bit flavour
        if (p == BF16 && too_coarse(BF16)) p = F32;
      }
      h_map_out[t] = (uint8_t)p;
    }
  return MPCR_OK;
}

int mpcr_morton_order(mpcr_ctx* ctx, int64_t n, const double* d_locs, int64_t* d_perm_out) {
  CHECK_ARG(ctx, ctx != nullptr, "NULL context");
  CHECK_ARG(ctx, n >= 0 && n < (1ll << 31), "n out of range");
  CHECK_ARG(ctx, n == 0 || (d_locs && d_perm_out), "NULL pointer");
  if (n == 0) return MPCR_OK;
  DeviceGuard g(ctx->device);
  int npow2 = 1;
  while (npow2 < n) npow2 <<= 1;
  uint64_t* keys = nullptr;
  HIP_TRY(ctx, dmalloc(ctx->arena, &keys, (size_t)npow2 * 8));
  hipStream_t s = ctx->stream;
  hipError_t e = launch_morton_codes((int)n, d_locs, keys, npow2, s);
  if (e == hipSuccess) e = launch_bitonic_sort(keys, npow2, s);
  if (e == hipSuccess) e = launch_keys_to_perm((int)n, keys, d_perm_out, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dfree(ctx->arena, keys);
  HIP_TRY(ctx, e);
  return MPCR_OK;
}

int mpcr_morton_order_noalloc(mpcr_ctx* ctx, int64_t n, const double* d_locs, int64_t* d_perm_out) {
  CHECK_ARG(ctx, ctx != nullptr, "NULL context");
  CHECK_ARG(ctx, n >= 0 && n <= MORTON_NOALLOC_MAX_KEYS, "n must be <= %d for the allocation-free ordering",
            MORTON_NOALLOC_MAX_KEYS);
  CHECK_ARG(ctx, n == 0 || (d_locs && d_perm_out), "NULL pointer");
  if (n == 0) return MPCR_OK;
  CHECK_ARG(ctx, ctx->noalloc_keys != nullptr, "sort-key array not set up");
  DeviceGuard g(ctx->device);
  int npow2 = 1;
  while (npow2 < n) npow2 <<= 1;
  // every key slot below npow2 is written by the key kernel: nothing to clear
  hipStream_t s = ctx->stream;
  hipError_t e = launch_morton_codes((int)n, d_locs, ctx->noalloc_keys, npow2, s);
  if (e == hipSuccess) e = launch_bitonic_sort(ctx->noalloc_keys, npow2, s);
  if (e == hipSuccess) e = launch_keys_to_perm((int)n, ctx->noalloc_keys, d_perm_out, s);
  HIP_TRY(ctx, e);
  return MPCR_OK;
}

static int check_theta(mpcr_ctx* ctx, const mpcr_theta_t* th) {
  CHECK_ARG(ctx, th != nullptr, "theta is NULL");
  CHECK_ARG(ctx, th->nu == 0.5 || th->nu == 1.5 || th->nu == 2.5, "nu must be 0.5, 1.5 or 2.5");
  CHECK_ARG(ctx, th->sigma2 > 0 && th->range > 0 && th->nugget >= 0 && std::isfinite(th->sigma2) &&
                     std::isfinite(th->range) && std::isfinite(th->nugget),
            "need sigma2 > 0, range > 0, nugget >= 0");
  return MPCR_OK;
}

int mpcr_covariance(mpcr_ctx* ctx, int64_t n, const double* d_locs, const mpcr_theta_t* theta, double* d_A,
                    int64_t lda) {
  CHECK_ARG(ctx, ctx != nullptr, "NULL context");
  int rc = check_theta(ctx, theta);
  if (rc) return rc;
  CHECK_ARG(ctx, n >= 0 && n < (1ll << 31) && lda >= std::max<int64_t>(n, 1), "bad n / lda");
  CHECK_ARG(ctx, n == 0 || (d_locs && d_A), "NULL pointer");
  DeviceGuard g(ctx->device);
  HIP_TRY(ctx, launch_covariance_dense((int)n, d_locs, *theta, d_A, lda, ctx->stream));
  return MPCR_OK;
}

int mpcr_covariance_tile_amax(mpcr_ctx* ctx, int64_t n, int64_t nb, const double* d_locs, const mpcr_theta_t* theta,
                              double* h_amax_out) {
  CHECK_ARG(ctx, ctx != nullptr, "NULL context");
  int rc = check_theta(ctx, theta);
  if (rc) return rc;
  CHECK_ARG(ctx, n > 0 && n < (1ll << 31) && nb > 0 && d_locs && h_amax_out, "bad arguments");
  DeviceGuard g(ctx->device);
  int64_t nt = (n + nb - 1) / nb;
  double* d = nullptr;
  HIP_TRY(ctx, dmalloc(ctx->arena, &d, (size_t)nt * nt * 8));
  hipError_t e = hipMemsetAsync(d, 0, nt * nt * 8, ctx->stream);
  if (e == hipSuccess) e = launch_covariance_tile_amax((int)n, (int)nb, d_locs, *theta, d, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(h_amax_out, d, nt * nt * 8, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  dfree(ctx->arena, d);
  HIP_TRY(ctx, e);
  return MPCR_OK;
}

int mpcr_potrf_tiled(mpcr_ctx* ctx, int64_t n, const double* d_A, int64_t lda, const mpcr_tilemap_t* map,
                     mpcr_factor** out, int64_t* h_info) {
  TraceRange tr("mpcr_potrf_tiled");
  CHECK_ARG(ctx, ctx != nullptr, "NULL context");
  CHECK_ARG(ctx, out != nullptr, "out is NULL");
  *out = nullptr;
  CHECK_ARG(ctx, n > 0 && n < (1ll << 31) && lda >= n && d_A, "bad n / lda / A");
  std::vector<uint8_t> m;
  int64_t nb;
  int rc = check_map(ctx, n, map, m, nb);
  if (rc) return rc;
  DeviceGuard g(ctx->device);
  mpcr_factor* f = nullptr;
  if ((rc = make_factor(ctx, n, nb, m, &f)) != MPCR_OK) return rc;
  *out = f;
  HIP_TRY(ctx, hipMemsetAsync(f->d_info, 0, sizeof(int), ctx->stream));
  if (f->has_f8) {  // FP8 tile scales from the tile maxima of the input
    HIP_TRY(ctx, launch_dense_tile_amax((int)n, (int)nb, d_A, lda, f->d_tamax, ctx->stream));
    HIP_TRY(ctx, launch_fp8_scales(f->view(), f->d_tamax, ctx->stream));
  }
  HIP_TRY(ctx, launch_tiles_from_dense(f->view(), d_A, lda, ctx->stream));
  if ((rc = run_factorisation(ctx, f)) != MPCR_OK) return rc;
  return read_info(ctx, f, h_info);
}

int mpcr_potrf_tiled_covariance(mpcr_ctx* ctx, int64_t n, const double* d_locs, const mpcr_theta_t* theta,
                                const mpcr_tilemap_t* map, mpcr_factor** out, int64_t* h_info) {
  TraceRange tr("mpcr_potrf_tiled_covariance");
  CHECK_ARG(ctx, ctx != nullptr, "NULL context");
  CHECK_ARG(ctx, out != nullptr, "out is NULL");
  *out = nullptr;
  int rc = check_theta(ctx, theta);
  if (rc) return rc;
  CHECK_ARG(ctx, n > 0 && n < (1ll << 31) && d_locs, "bad n / locs");
  std::vector<uint8_t> m;
  int64_t nb;
  if ((rc = check_map(ctx, n, map, m, nb)) != MPCR_OK) return rc;
  DeviceGuard g(ctx->device);
  mpcr_factor* f = nullptr;
  if ((rc = make_factor(ctx, n, nb, m, &f)) != MPCR_OK) return rc;
  *out = f;
  HIP_TRY(ctx, hipMemsetAsync(f->d_info, 0, sizeof(int), ctx->stream));
  if (f->has_f8) {
    HIP_TRY(ctx, launch_covariance_tile_amax((int)n, (int)nb, d_locs, *theta, f->d_tamax, ctx->stream));
    HIP_TRY(ctx, launch_fp8_scales(f->view(), f->d_tamax, ctx->stream));
  }
  HIP_TRY(ctx, launch_tiles_from_covariance(f->view(), d_locs, *theta, ctx->stream));
  if ((rc = run_factorisation(ctx, f)) != MPCR_OK) return rc;
  return read_info(ctx, f, h_info);
}

int mpcr_factor_destroy(mpcr_factor* f) {
  if (!f) return MPCR_ERR_ARG;
  free_factor(f);
  return MPCR_OK;
}

int mpcr_factor_logdet(mpcr_ctx* ctx, const mpcr_factor* fc, double* h_logdet) {
  CHECK_ARG(ctx, ctx != nullptr, "NULL context");
  CHECK_ARG(ctx, fc && h_logdet, "NULL argument");
  CHECK_ARG(ctx, fc->info == 0, "factor is not positive definite (info %lld)", (long long)fc->info);
  DeviceGuard g(ctx->device);
  double* d = nullptr;
  HIP_TRY(ctx, dmalloc(ctx->arena, &d, 8));
  hipError_t e = launch_logdet(fc->view(), d, ctx->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(h_logdet, d, 8, hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  dfree(ctx->arena, d);
  HIP_TRY(ctx, e);
  return MPCR_OK;
}

int mpcr_factor_to_dense(mpcr_ctx* ctx, const mpcr_factor* fc, double* d_L, int64_t ldl) {
  CHECK_ARG(ctx, ctx != nullptr, "NULL context");
  CHECK_ARG(ctx, fc && d_L && ldl >= fc->n, "bad arguments");
  DeviceGuard g(ctx->device);
  HIP_TRY(ctx, launch_tiles_to_dense(fc->view(), d_L, ldl, ctx->stream));
  return MPCR_OK;
}

int mpcr_factor_flops(const mpcr_factor* f, double* h_flops5) {
  if (!f || !h_flops5) return MPCR_ERR_ARG;
  for (int p = 0; p < 5; ++p) h_flops5[p] = f->flops[p];
  return MPCR_OK;
}

int mpcr_trsm_forward(mpcr_ctx* ctx, const mpcr_factor* fc, int64_t nrhs, const double* d_B, int64_t ldb,
                      double* d_W, int64_t ldw) {
  CHECK_ARG(ctx, ctx != nullptr, "NULL context");
  CHECK_ARG(ctx, fc != nullptr, "factor is NULL");
  CHECK_ARG(ctx, fc->info == 0, "factor is not positive definite");
  CHECK_ARG(ctx, nrhs >= 0 && ldb >= fc->n && ldw >= fc->n, "bad nrhs / ld");
  if (nrhs == 0) return MPCR_OK;
  CHECK_ARG(ctx, d_B && d_W, "NULL pointer");
  auto* f = const_cast<mpcr_factor*>(fc);
  DeviceGuard g(ctx->device);
  int rc = ensure_linv(ctx, f);
  if (rc) return rc;
  SolveBufs b;
  if ((rc = carve(ctx, f->N, nrhs, f->n, b)) != MPCR_OK) return rc;
  HIP_TRY(ctx, launch_copy_cols((int)f->n, (int)nrhs, d_B, ldb, b.B, b.N, ctx->stream));
  if ((rc = tile_solve(ctx, f, b, b.B, b.X, b.W, false)) != MPCR_OK) return rc;
  HIP_TRY(ctx, launch_copy_cols((int)f->n, (int)nrhs, b.W, b.N, d_W, ldw, ctx->stream));
  HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
  return MPCR_OK;
}

int mpcr_potrs(mpcr_ctx* ctx, const mpcr_factor* fc, int64_t nrhs, const double* d_B, int64_t ldb, double* d_X,
               int64_t ldx, const double* d_A_fp64, int64_t lda, const mpcr_refine_opts_t* opts, mpcr_diag_t* diag) {
  TraceRange tr("mpcr_potrs");
  CHECK_ARG(ctx, ctx != nullptr, "NULL context");
  CHECK_ARG(ctx, fc != nullptr, "factor is NULL");
  CHECK_ARG(ctx, fc->info == 0, "factor is not positive definite");
  CHECK_ARG(ctx, nrhs >= 0 && ldb >= fc->n && ldx >= fc->n, "bad nrhs / ld");
  if (nrhs == 0) return MPCR_OK;
  CHECK_ARG(ctx, d_B && d_X, "NULL pointer");
  const bool do_ref = d_A_fp64 && opts && opts->max_iter > 0;
  if (do_ref) {
    CHECK_ARG(ctx, lda >= fc->n, "lda < n");
    CHECK_ARG(ctx, refine_opts_ok(*opts), "bad opts");
  }
  auto* f = const_cast<mpcr_factor*>(fc);
  DeviceGuard g(ctx->device);
  hipStream_t s = ctx->stream;
  int rc = ensure_linv(ctx, f);
  if (rc) return rc;
  SolveBufs b;
  if ((rc = carve(ctx, f->N, nrhs, f->n, b)) != MPCR_OK) return rc;
  HIP_TRY(ctx, launch_copy_cols((int)f->n, (int)nrhs, d_B, ldb, b.B, b.N, s));
  bool conv = true;
  if (do_ref) {
    SigmaOp op;
    op.ctx = ctx;
    op.A = d_A_fp64;
    op.lda = lda;
    op.n = (int)f->n;
    if ((rc = refine(ctx, f, b, op, *opts, diag, &conv)) != MPCR_OK) return rc;
  } else {
    if ((rc = tile_solve(ctx, f, b, b.B, b.X, b.W)) != MPCR_OK) return rc;
    if (diag) diag->iters = 0;
  }
  HIP_TRY(ctx, launch_copy_cols((int)f->n, (int)nrhs, b.X, b.N, d_X, ldx, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  drain_timing(ctx);
  if (diag) diag->info = 0;
  if (!conv) return set_err(ctx, MPCR_ERR_NOT_CONVERGED, "refinement did not reach the tolerance");
  return MPCR_OK;
}

int mpcr_gauss_loglik(mpcr_ctx* ctx, int64_t n, const double* d_locs, const double* d_Z, int64_t nrhs,
                      const mpcr_theta_t* theta, const mpcr_tilemap_t* map, int order, const mpcr_refine_opts_t* opts,
                      double* h_loglik, mpcr_diag_t* diag) {
  TraceRange tr("mpcr_gauss_loglik");
  CHECK_ARG(ctx, ctx != nullptr, "NULL context");
  int rc = check_theta(ctx, theta);
  if (rc) return rc;
  CHECK_ARG(ctx, n > 0 && n < (1ll << 31) && nrhs >= 1 && nrhs <= 4096, "need n > 0 and 1 <= nrhs <= 4096");
  CHECK_ARG(ctx, d_locs && d_Z && h_loglik, "NULL pointer");
  std::vector<uint8_t> m;
  int64_t nb = 256;
  if (map) {
    if ((rc = check_map(ctx, n, map, m, nb)) != MPCR_OK) return rc;
  } else {
    int64_t nt = (n + nb - 1) / nb;
    m.assign(nt * nt, 255);
    for (int64_t i = 0; i < nt; ++i)
      for (int64_t j = 0; j <= i; ++j) m[i * nt + j] = F64;
  }
  const int64_t nt = (n + nb - 1) / nb;
  if (opts) CHECK_ARG(ctx, refine_opts_ok(*opts) && (opts->residual == 0 || opts->residual == 1) &&
                               (opts->promote_on_breakdown == 0 || opts->promote_on_breakdown == 1) &&
                               (opts->direct_eta == 0 || opts->direct_eta == 1),
                      "bad refinement options");
  const bool promote = opts && opts->promote_on_breakdown;
  const bool refine_on = opts && opts->max_iter > 0;
  const bool stored_residual = refine_on && opts->residual == 1;
  DeviceGuard g(ctx->device);
  hipStream_t s = ctx->stream;

  // workspace: the sorted sites (per n) and the factor (per n, nb and map)
  if (ctx->ws_n != n) {
    free_factor(ctx->ws_factor);
    ctx->ws_factor = nullptr;
    dfree(ctx->arena, ctx->ws_locs);
    ctx->ws_locs = nullptr;
    ctx->ws_n = -1;
    HIP_TRY(ctx, dmalloc(ctx->arena, &ctx->ws_locs, (size_t)n * 2 * 8 + (size_t)n * 8));
    ctx->ws_n = n;
  }
  auto ensure_factor = [&](const std::vector<uint8_t>& mm) -> int {
    if (ctx->ws_factor && ctx->ws_factor->n == n && ctx->ws_nb == nb && ctx->ws_map == mm) return MPCR_OK;
    free_factor(ctx->ws_factor);
    ctx->ws_factor = nullptr;
    ctx->ws_map.clear();
    int r = make_factor(ctx, n, nb, mm, &ctx->ws_factor);
    if (r != MPCR_OK) return r;
    ctx->ws_nb = nb;
    ctx->ws_map = mm;
    return MPCR_OK;
  };
  if ((rc = ensure_factor(m)) != MPCR_OK) return rc;
  SolveBufs b;
  if ((rc = carve(ctx, ctx->ws_factor->N, nrhs, n, b)) != MPCR_OK) return rc;
  double* locs = ctx->ws_locs;
  int64_t* perm = (int64_t*)(ctx->ws_locs + 2 * n);

  HIP_TRY(ctx, hipEventRecord(ctx->ev[0], s));
  if (order) {
    int npow2 = 1;
    while (npow2 < n) npow2 <<= 1;
    // the sort keys use the P, Q, Z blocks when they are large enough
    uint64_t* keys = nullptr;
    bool own = false;
    if ((int64_t)npow2 * 8 <= 3 * b.N * nrhs * 8) {
      keys = (uint64_t*)b.P;
    } else {
      HIP_TRY(ctx, dmalloc(ctx->arena, &keys, (size_t)npow2 * 8));
      own = true;
    }
    hipError_t e = launch_morton_codes((int)n, d_locs, keys, npow2, s);
    if (e == hipSuccess) e = launch_bitonic_sort(keys, npow2, s);
    if (e == hipSuccess) e = launch_keys_to_perm((int)n, keys, perm, s);
    if (e == hipSuccess) e = launch_gather_rows((int)n, 2, d_locs, n, perm, locs, n, s);
    if (e == hipSuccess) e = launch_gather_rows((int)n, (int)nrhs, d_Z, n, perm, b.B, b.N, s);
    if (own) {
      (void)hipStreamSynchronize(s);
      dfree(ctx->arena, keys);
    }
    HIP_TRY(ctx, e);
    HIP_TRY(ctx, launch_fill(b.P, 3 * b.N * nrhs, 0.0, s));
  } else {
    HIP_TRY(ctx, launch_copy_cols((int)n, 2, d_locs, n, locs, n, s));
    HIP_TRY(ctx, launch_copy_cols((int)n, (int)nrhs, d_Z, n, b.B, b.N, s));
  }

  // tiles and factorisation; after a breakdown, optionally promote and again
  int promotions = 0;
  int64_t info = 0;
  for (;;) {
    mpcr_factor* f = ctx->ws_factor;
    HIP_TRY(ctx, hipMemsetAsync(f->d_info, 0, sizeof(int), s));
    if (stored_residual && !f->d_sig) {
      HIP_TRY(ctx, dmalloc(f->arena, &f->d_sig, (size_t)(f->nt * (f->nt + 1) / 2) * f->nb * f->nb * 8));
      HIP_TRY(ctx, dmalloc(f->arena, &f->d_rpart, residual_part_bytes((int)f->nb, (int)f->nt)));
    }
    if (f->has_f8) {
      HIP_TRY(ctx, launch_covariance_tile_amax((int)n, (int)f->nb, locs, *theta, f->d_tamax, s));
      HIP_TRY(ctx, launch_fp8_scales(f->view(), f->d_tamax, s));
    }
    HIP_TRY(ctx, launch_tiles_from_covariance(f->view(), locs, *theta, s, stored_residual ? f->d_sig : nullptr));
    if (promotions == 0) HIP_TRY(ctx, hipEventRecord(ctx->ev[1], s));
    {
      TraceRange tr("factorisation");
      if ((rc = run_factorisation(ctx, f)) != MPCR_OK) return rc;
      HIP_TRY(ctx, hipEventRecord(ctx->ev[2], s));
      rc = read_info(ctx, f, &info);  // synchronises: the range spans the factorisation's GPU work
    }
    if (rc != MPCR_ERR_NOT_SPD || !promote || promotions >= 8) break;
    std::vector<uint8_t> m2 = ctx->ws_map;
    if (!promote_map(m2, nt, nb, info)) break;
    ++promotions;
    if ((rc = ensure_factor(m2)) != MPCR_OK) return rc;
  }
  mpcr_factor* f = ctx->ws_factor;
  bool all64 = true;
  for (int64_t i = 0; i < nt; ++i)
    for (int64_t j = 0; j <= i; ++j) all64 &= (ctx->ws_map[i * nt + j] == F64);
  if (diag) {
    memset(diag, 0, sizeof *diag);
    diag->info = info;
    diag->promotions = promotions;
    for (int p = 0; p < 5; ++p) diag->flops_by_prec[p] = f->flops[p];
  }
  if (rc) return rc;

  double* d_logdet = b.scal + 8 * nrhs;
  double* d_quad = b.scal + 9 * nrhs;
  double* d_ll = b.scal + 10 * nrhs;
  HIP_TRY(ctx, launch_logdet(f->view(), d_logdet, s));
  if ((rc = ensure_linv(ctx, f)) != MPCR_OK) return rc;
  bool conv = true;
  HIP_TRY(ctx, hipEventRecord(ctx->ev[3], s));
  if (all64 && !refine_on) {
    // the paper's path: w = L^{-1} z, quad = ||w||^2, and x = L^{-T} w
    if ((rc = tile_solve(ctx, f, b, b.B, b.X, b.W)) != MPCR_OK) return rc;
    HIP_TRY(ctx, launch_col_dot((int)n, (int)nrhs, b.W, b.W, b.N, b.partial, d_quad, s));
    HIP_TRY(ctx, hipEventRecord(ctx->ev[4], s));
    if (diag && (!opts || opts->direct_eta)) {  // backward error of the direct solve
      SigmaOp op;
      op.ctx = ctx;
      op.locs = locs;
      op.th = *theta;
      op.n = (int)n;
      double* sig_inf = b.scal;
      double* stats = b.scal + 6 * nrhs;
      HIP_TRY(ctx, op.residual(b.B, b.X, b.R, b.N, (int)nrhs, s, b.Z));
      HIP_TRY(ctx, launch_max_reduce((int)n, b.Z, b.partial, sig_inf, s));
      HIP_TRY(ctx, launch_col_stats((int)n, (int)nrhs, b.R, b.X, b.B, b.N, sig_inf, b.partial, stats, s));
      std::vector<double> hst(2 * nrhs);
      HIP_TRY(ctx, hipMemcpyAsync(hst.data(), stats, 2 * nrhs * 8, hipMemcpyDeviceToHost, s));
      HIP_TRY(ctx, hipStreamSynchronize(s));
      for (int64_t c = 0; c < nrhs; ++c) {
        diag->eta = std::max(diag->eta, hst[2 * c]);
        diag->rel_resid2 = std::max(diag->rel_resid2, hst[2 * c + 1]);
      }
    }
    if (diag) diag->converged = 1;
  } else {
    mpcr_refine_opts_t o = opts ? *opts : mpcr_refine_opts_t{1e-9, 0, 0, 20, 0, 0, 0, 0, 0.0, 0};
    SigmaOp op;
    op.ctx = ctx;
    if (stored_residual) {
      op.sig = f->d_sig;
      op.part = f->d_rpart;
      op.nb = (int)f->nb;
      op.nt = (int)f->nt;
    }
    op.locs = locs;
    op.th = *theta;
    op.n = (int)n;
    if (o.max_iter > 0) {
      if ((rc = refine(ctx, f, b, op, o, diag, &conv)) != MPCR_OK) return rc;
    } else {
      if ((rc = tile_solve(ctx, f, b, b.B, b.X, b.W)) != MPCR_OK) return rc;
      HIP_TRY(ctx, op.residual(b.B, b.X, b.R, b.N, (int)nrhs, s));
    }
    HIP_TRY(ctx, hipEventRecord(ctx->ev[4], s));
    HIP_TRY(ctx, launch_quad_refined((int)n, (int)nrhs, b.B, b.X, b.R, b.N, b.partial, d_quad, s));
  }
  HIP_TRY(ctx, launch_loglik((int)n, (int)nrhs, d_logdet, d_quad, d_ll, s));
  HIP_TRY(ctx, hipEventRecord(ctx->ev[5], s));
  HIP_TRY(ctx, hipMemcpyAsync(h_loglik, d_ll, nrhs * 8, hipMemcpyDeviceToHost, s));
  double host_ld = 0, host_q0 = 0;
  HIP_TRY(ctx, hipMemcpyAsync(&host_ld, d_logdet, 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipMemcpyAsync(&host_q0, d_quad, 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(ctx, hipStreamSynchronize(s));
  drain_timing(ctx);
  if (diag) {
    diag->logdet = host_ld;
    diag->quad0 = host_q0;
    diag->t_gen_ms = ev_ms(ctx->ev[0], ctx->ev[1]);
    diag->t_factor_ms = ev_ms(ctx->ev[1], ctx->ev[2]);
    diag->t_solve_ms = ev_ms(ctx->ev[3], ctx->ev[4]);
    diag->t_refine_ms = ev_ms(ctx->ev[4], ctx->ev[5]);
  }
  if (!conv) return set_err(ctx, MPCR_ERR_NOT_CONVERGED, "refinement did not reach the tolerance");
  return MPCR_OK;
}

int mpcr_mle_fit(mpcr_ctx* ctx, int64_t n, const double* d_locs, const double* d_z, double nu, double nugget,
                 const mpcr_tilemap_t* map, const mpcr_refine_opts_t* refine, const double* h_x0, int max_iter,
                 double reltol, double* h_x_out, double* h_nll_out, int* h_iters, int* h_evals) {
  TraceRange tr("mpcr_mle_fit");
  CHECK_ARG(ctx, ctx != nullptr, "NULL context");
  CHECK_ARG(ctx, n > 0 && n < (1ll << 31) && d_locs && d_z && h_x0 && h_x_out && h_nll_out, "bad arguments");
  CHECK_ARG(ctx, nu == 0.5 || nu == 1.5 || nu == 2.5, "nu must be 0.5, 1.5 or 2.5");
  CHECK_ARG(ctx, nugget >= 0 && std::isfinite(nugget) && max_iter >= 0 && reltol >= 0, "bad nugget / options");
  CHECK_ARG(ctx, std::isfinite(h_x0[0]) && std::isfinite(h_x0[1]), "x0 must be finite");
  DeviceGuard g(ctx->device);
  hipStream_t s = ctx->stream;
  // the sites and observations in Morton order, once for the whole fit
  double* dsorted = nullptr;
  int64_t* perm = nullptr;
  HIP_TRY(ctx, dmalloc(ctx->arena, &dsorted, (size_t)n * 3 * 8));
  auto release = [&] {
    (void)hipStreamSynchronize(s);
    dfree(ctx->arena, dsorted);
    dfree(ctx->arena, perm);
  };
  hipError_t e = dmalloc(ctx->arena, &perm, (size_t)n * 8);
  if (e != hipSuccess) {
    release();
    HIP_TRY(ctx, e);
  }
  int rc = mpcr_morton_order(ctx, n, d_locs, perm);
  if (rc) {
    release();
    return rc;
  }
  e = launch_gather_rows((int)n, 2, d_locs, n, perm, dsorted, n, s);
  if (e == hipSuccess) e = launch_gather_rows((int)n, 1, d_z, n, perm, dsorted + 2 * n, n, s);
  if (e != hipSuccess) {
    release();
    HIP_TRY(ctx, e);
  }
  // f(p) = -l(range = e^p0, variance = e^p1); a breakdown of the factor is +inf
  int fail = MPCR_OK;
  int evals = 0;
  auto nll = [&](const double* p) -> double {
    if (fail) return INFINITY;
    mpcr_theta_t th{std::exp(p[1]), std::exp(p[0]), nu, nugget};
    if (!(th.sigma2 > 0) || !(th.range > 0) || !std::isfinite(th.sigma2) || !std::isfinite(th.range))
      return INFINITY;
    double ll = 0;
    ++evals;
    int r = mpcr_gauss_loglik(ctx, n, dsorted, dsorted + 2 * n, 1, &th, map, 0, refine, &ll, nullptr);
    if (r == MPCR_ERR_NOT_SPD) return INFINITY;
    if (r != MPCR_OK) {
      fail = r;
      return INFINITY;
    }
    return -ll;
  };
  // Nelder-Mead (reflection 1, expansion 2, contraction 1/2, shrink 1/2),
  // first simplex x0 + s e_i with s = 0.1 max|x0_i| (0.1 for x0 = 0)
  const double s0 = std::max(std::fabs(h_x0[0]), std::fabs(h_x0[1]));
  const double step = s0 > 0 ? 0.1 * s0 : 0.1;
  double pts[3][2] = {{h_x0[0], h_x0[1]}, {h_x0[0] + step, h_x0[1]}, {h_x0[0], h_x0[1] + step}};
  double val[3];
  for (int i = 0; i < 3; ++i) val[i] = nll(pts[i]);
  int it = 0;
  for (;;) {
    int idx[3] = {0, 1, 2};
    std::stable_sort(idx, idx + 3, [&](int a, int b) { return val[a] < val[b]; });
    double sp[3][2], sv[3];
    for (int i = 0; i < 3; ++i) {
      sp[i][0] = pts[idx[i]][0];
      sp[i][1] = pts[idx[i]][1];
      sv[i] = val[idx[i]];
    }
    memcpy(pts, sp, sizeof pts);
    memcpy(val, sv, sizeof val);
    if (fail || val[2] - val[0] <= reltol * (std::fabs(val[0]) + reltol) || it >= max_iter) break;
    ++it;
    const double c[2] = {0.5 * (pts[0][0] + pts[1][0]), 0.5 * (pts[0][1] + pts[1][1])};
    const double xr[2] = {c[0] + (c[0] - pts[2][0]), c[1] + (c[1] - pts[2][1])};
    const double fr = nll(xr);
    auto take = [&](const double* x, double fx) {
      pts[2][0] = x[0];
      pts[2][1] = x[1];
      val[2] = fx;
    };
    if (val[0] <= fr && fr < val[1]) {
      take(xr, fr);
      continue;
    }
    if (fr < val[0]) {
      const double xe[2] = {c[0] + 2.0 * (xr[0] - c[0]), c[1] + 2.0 * (xr[1] - c[1])};
      const double fe = nll(xe);
      if (fe < fr) take(xe, fe);
      else take(xr, fr);
      continue;
    }
    if (fr < val[2]) {
      const double xc[2] = {c[0] + 0.5 * (xr[0] - c[0]), c[1] + 0.5 * (xr[1] - c[1])};
      const double fc = nll(xc);
      if (fc <= fr) {
        take(xc, fc);
        continue;
      }
    } else {
      const double xcc[2] = {c[0] - 0.5 * (c[0] - pts[2][0]), c[1] - 0.5 * (c[1] - pts[2][1])};
      const double fcc = nll(xcc);
      if (fcc < val[2]) {
        take(xcc, fcc);
        continue;
      }
    }
    for (int i = 1; i < 3; ++i) {
      pts[i][0] = pts[0][0] + 0.5 * (pts[i][0] - pts[0][0]);
      pts[i][1] = pts[0][1] + 0.5 * (pts[i][1] - pts[0][1]);
      val[i] = nll(pts[i]);
    }
  }
  release();
  if (fail) return fail;
  h_x_out[0] = pts[0][0];
  h_x_out[1] = pts[0][1];
  *h_nll_out = val[0];
  if (h_iters) *h_iters = it;
  if (h_evals) *h_evals = evals;
  return MPCR_OK;
}


int mpcr_inla_posterior(mpcr_ctx* ctx, int64_t n, const double* d_locs, const double* d_y, double sigma2, double nu,
                        double beta, const double* h_range, int nrange, double newton_tol, int max_newton,
                        const mpcr_tilemap_t* map, double* h_lpost, double* h_posterior, int* h_newton_iters,
                        double* d_mode_out) {
  TraceRange tr("mpcr_inla_posterior");
  CHECK_ARG(ctx, ctx != nullptr, "NULL context");
  CHECK_ARG(ctx, n > 0 && n < (1ll << 31) && d_locs && d_y && h_range && h_lpost, "bad arguments");
  CHECK_ARG(ctx, nu == 0.5 || nu == 1.5 || nu == 2.5, "nu must be 0.5, 1.5 or 2.5");
  CHECK_ARG(ctx, sigma2 > 0 && std::isfinite(sigma2) && std::isfinite(beta) && newton_tol > 0 && max_newton >= 1,
            "bad sigma2 / beta / Newton options");
  CHECK_ARG(ctx, nrange >= 1, "need at least one range value");
  for (int i = 0; i < nrange; ++i) CHECK_ARG(ctx, h_range[i] > 0 && std::isfinite(h_range[i]), "ranges must be > 0");
  if (h_posterior) {
    CHECK_ARG(ctx, nrange >= 3 && nrange % 2 == 1, "the Simpson posterior needs an odd number (>= 3) of ranges");
    const double hstep = h_range[1] - h_range[0];
    for (int i = 1; i < nrange; ++i)
      CHECK_ARG(ctx, hstep > 0 && std::fabs(h_range[i] - h_range[i - 1] - hstep) <= 1e-9 * hstep,
                "the Simpson posterior needs equally spaced increasing ranges");
  }
  std::vector<uint8_t> m;
  int64_t nb = 256;
  int rc;
  if (map) {
    if ((rc = check_map(ctx, n, map, m, nb)) != MPCR_OK) return rc;
  } else {
    const int64_t nt = (n + nb - 1) / nb;
    m.assign(nt * nt, 255);
    for (int64_t i = 0; i < nt; ++i)
      for (int64_t j = 0; j <= i; ++j) m[i * nt + j] = F64;
  }
  DeviceGuard g(ctx->device);
  double* vec = nullptr;
  HIP_TRY(ctx, dmalloc(ctx->arena, &vec, (size_t)(10 * n + 8) * 8));
  rc = MPCR_OK;
  for (int i = 0; i < nrange && rc == MPCR_OK; ++i) {
    mpcr_theta_t th{sigma2, h_range[i], nu, 0.0};
    rc = laplace_one(ctx, n, nb, m, d_locs, d_y, th, beta, newton_tol, max_newton, vec, &h_lpost[i],
                     h_newton_iters ? &h_newton_iters[i] : nullptr);
    if (rc == MPCR_OK && d_mode_out && i == nrange - 1)
      rc = hipMemcpyAsync(d_mode_out, vec, n * 8, hipMemcpyDeviceToDevice, ctx->stream) == hipSuccess
               ? MPCR_OK
               : set_err(ctx, MPCR_ERR_DEVICE, "mode copy failed");
  }
  (void)hipStreamSynchronize(ctx->stream);
  dfree(ctx->arena, vec);
  if (rc) return rc;
  if (h_posterior) {
    // the paper's normalisation: centre the log values, Simpson's rule over the grid
    double mean = 0;
    for (int i = 0; i < nrange; ++i) mean += h_lpost[i];
    mean /= nrange;
    const double hstep = h_range[1] - h_range[0];
    double z = 0;
    for (int i = 0; i < nrange; ++i) {
      const double w = (i == 0 || i == nrange - 1) ? 1.0 : (i % 2 == 1 ? 4.0 : 2.0);
      z += w * std::exp(h_lpost[i] - mean);
    }
    z *= hstep / 3.0;
    for (int i = 0; i < nrange; ++i) h_posterior[i] = std::exp(h_lpost[i] - mean) / z;
  }
  return MPCR_OK;
}

int mpcr_mala_run(mpcr_ctx* ctx, int64_t n, const double* d_locs, const mpcr_theta_t* target,
                  const mpcr_theta_t* precond, double h, const double* d_z0, int iters, const double* d_eps,
                  const double* h_unif, const mpcr_tilemap_t* map, double* d_z_out, double* d_trace,
                  int* h_accepted, double* h_log_ratio) {
  TraceRange tr("mpcr_mala_run");
  CHECK_ARG(ctx, ctx != nullptr, "NULL context");
  int rc = check_theta(ctx, target);
  if (rc) return rc;
  if ((rc = check_theta(ctx, precond)) != MPCR_OK) return rc;
  CHECK_ARG(ctx, n > 0 && n < (1ll << 31) && d_locs && d_z0 && d_z_out && iters >= 0, "bad arguments");
  CHECK_ARG(ctx, iters == 0 || (d_eps && h_unif), "need the noise and the uniforms");
  CHECK_ARG(ctx, h > 0 && std::isfinite(h), "need h > 0");
  std::vector<uint8_t> m;
  int64_t nb = 256;
  if (map) {
    if ((rc = check_map(ctx, n, map, m, nb)) != MPCR_OK) return rc;
  } else {
    const int64_t nt = (n + nb - 1) / nb;
    m.assign(nt * nt, 255);
    for (int64_t i = 0; i < nt; ++i)
      for (int64_t j = 0; j <= i; ++j) m[i * nt + j] = F64;
  }
  DeviceGuard g(ctx->device);
  hipStream_t s = ctx->stream;
  // factors of the target covariance Sigma and of h M (M the preconditioner)
  mpcr_factor *fs = nullptr, *fm = nullptr;
  double* vec = nullptr;
  auto release = [&] {
    (void)hipStreamSynchronize(s);
    free_factor(fs);
    free_factor(fm);
    dfree(ctx->arena, vec);
  };
  const mpcr_theta_t thm{h * precond->sigma2, precond->range, precond->nu, h * precond->nugget};
  auto factor = [&](mpcr_factor** f, const mpcr_theta_t& th) -> int {
    int r = make_factor(ctx, n, nb, m, f);
    if (r) return r;
    HIP_TRY(ctx, hipMemsetAsync((*f)->d_info, 0, sizeof(int), s));
    if ((*f)->has_f8) {
      HIP_TRY(ctx, launch_covariance_tile_amax((int)n, (int)nb, d_locs, th, (*f)->d_tamax, s));
      HIP_TRY(ctx, launch_fp8_scales((*f)->view(), (*f)->d_tamax, s));
    }
    HIP_TRY(ctx, launch_tiles_from_covariance((*f)->view(), d_locs, th, s));
    if ((r = run_factorisation(ctx, *f)) != MPCR_OK) return r;
    int64_t info = 0;
    if ((r = read_info(ctx, *f, &info)) != MPCR_OK) return r;
    return ensure_linv(ctx, *f);
  };
  if ((rc = factor(&fs, *target)) != MPCR_OK || (rc = factor(&fm, thm)) != MPCR_OK) {
    release();
    return rc;
  }
  const int64_t N = fs->N;
  SolveBufs b;
  if ((rc = carve(ctx, N, 1, n, b)) != MPCR_OK) {
    release();
    return rc;
  }
  // state and work vectors (padded order N, tails zero)
  if (dmalloc(ctx->arena, &vec, (size_t)(10 * N + 8) * 8) != hipSuccess) {
    release();
    return set_err(ctx, MPCR_ERR_NOMEM, "device allocation failed");
  }
  double *z = vec, *gz = vec + N, *stz = vec + 2 * N, *zp = vec + 3 * N, *gzp = vec + 4 * N, *stzp = vec + 5 * N,
         *t = vec + 6 * N, *dq = vec + 7 * N, *le = vec + 8 * N, *ones = vec + 9 * N, *red = vec + 10 * N;
  SigmaOp opm;  // products with M (unscaled) from the sites
  opm.locs = d_locs;
  opm.th = *precond;
  opm.n = (int)n;
  auto fail = [&](hipError_t e) {
    release();
    return set_err(ctx, e == hipErrorOutOfMemory ? MPCR_ERR_NOMEM : MPCR_ERR_DEVICE, "%s", hipGetErrorString(e));
  };
  hipError_t e = launch_fill(vec, 10 * N, 0.0, s);
  if (e == hipSuccess) e = launch_fill(ones, n, 1.0, s);
  if (e == hipSuccess) e = launch_copy_cols((int)n, 1, d_z0, n, z, N, s);
  if (e != hipSuccess) return fail(e);
  // grad-related quantities of a state x: g = Sigma^-1 x, st = x - (h/2) M g
  auto drift = [&](const double* x, double* gx, double* stx) -> int {
    int r = tile_solve(ctx, fs, b, x, gx, b.W);
    if (r) return r;
    hipError_t e2 = opm.residual(nullptr, gx, t, N, 1, s);  // t = -M g
    if (e2 == hipSuccess) e2 = launch_axpby((int)n, x, 0.5 * h, t, stx, s);
    return e2 == hipSuccess ? MPCR_OK : set_err(ctx, MPCR_ERR_DEVICE, "%s", hipGetErrorString(e2));
  };
  // -(1/2) v^T (h M)^-1 v = -(1/2) ||L_hM^-1 v||^2 into red[slot]
  auto qform = [&](const double* v, int slot) -> int {
    int r = tile_solve(ctx, fm, b, v, b.X, b.W, false);
    if (r) return r;
    hipError_t e2 = launch_col_dot((int)n, 1, b.W, b.W, N, b.partial, red + slot, s);
    return e2 == hipSuccess ? MPCR_OK : set_err(ctx, MPCR_ERR_DEVICE, "%s", hipGetErrorString(e2));
  };
  if ((rc = drift(z, gz, stz)) != MPCR_OK) {
    release();
    return rc;
  }
  for (int it = 0; it < iters; ++it) {
    // proposal z' = z - (h/2) M Sigma^-1 z + L_hM eps
    e = launch_copy_cols((int)n, 1, d_eps + (int64_t)it * n, n, dq, N, s);
    if (e == hipSuccess) e = launch_trmv_lower(fm->view(), dq, le, s);
    if (e == hipSuccess) e = launch_axpby((int)n, stz, 1.0, le, zp, s);
    if (e != hipSuccess) return fail(e);
    if ((rc = drift(zp, gzp, stzp)) != MPCR_OK) {
      release();
      return rc;
    }
    // log target ratio and the two proposal densities
    e = launch_col_dot((int)n, 1, zp, gzp, N, b.partial, red + 0, s);
    if (e == hipSuccess) e = launch_col_dot((int)n, 1, z, gz, N, b.partial, red + 1, s);
    if (e == hipSuccess) e = launch_axpby((int)n, z, -1.0, stzp, dq, s);  // z - st(z')
    if (e != hipSuccess) return fail(e);
    if ((rc = qform(dq, 2)) != MPCR_OK) {
      release();
      return rc;
    }
    if ((e = launch_axpby((int)n, zp, -1.0, stz, dq, s)) != hipSuccess) return fail(e);  // z' - st(z)
    if ((rc = qform(dq, 3)) != MPCR_OK) {
      release();
      return rc;
    }
    double hv[4];
    if ((e = hipMemcpyAsync(hv, red, 32, hipMemcpyDeviceToHost, s)) != hipSuccess ||
        (e = hipStreamSynchronize(s)) != hipSuccess)
      return fail(e);
    const double logr = -0.5 * hv[0] + 0.5 * hv[1] - 0.5 * hv[2] + 0.5 * hv[3];
    const bool acc = h_unif[it] < std::exp(std::min(0.0, logr));
    if (h_log_ratio) h_log_ratio[it] = logr;
    if (h_accepted) h_accepted[it] = acc ? 1 : 0;
    if (acc) {
      std::swap(z, zp);
      std::swap(gz, gzp);
      std::swap(stz, stzp);
    }
    if (d_trace && (e = launch_copy_cols((int)n, 1, z, N, d_trace + (int64_t)it * n, n, s)) != hipSuccess)
      return fail(e);
  }
  e = launch_copy_cols((int)n, 1, z, N, d_z_out, n, s);
  if (e != hipSuccess) return fail(e);
  release();
  return MPCR_OK;
}

int mpcr_loglik_map(const mpcr_ctx* ctx, int64_t* h_nt, uint8_t* h_map_out, int64_t capacity) {
  if (!ctx || !h_nt) return MPCR_ERR_ARG;
  if (!ctx->ws_factor || ctx->ws_map.empty()) return MPCR_ERR_ARG;
  const int64_t nt = ctx->ws_factor->nt;
  *h_nt = nt;
  if (!h_map_out || capacity < nt * nt) return MPCR_ERR_ARG;
  memcpy(h_map_out, ctx->ws_map.data(), (size_t)(nt * nt));
  return MPCR_OK;
}

int mpcr_convert(mpcr_ctx* ctx, mpcr_prec_t prec, int64_t m, int64_t n, const double* d_src, int64_t lds, void* d_dst,
                 int64_t ldd, int8_t* d_scale_exp) {
  CHECK_ARG(ctx, ctx != nullptr, "NULL context");
  CHECK_ARG(ctx, valid_prec(prec), "bad format");
  CHECK_ARG(ctx, m >= 0 && n >= 0 && lds >= std::max<int64_t>(m, 1) && ldd >= std::max<int64_t>(m, 1), "bad shape");
  CHECK_ARG(ctx, (m == 0 || n == 0) || (d_src && d_dst), "NULL pointer");
  CHECK_ARG(ctx, ((int)prec == F8) == (d_scale_exp != nullptr), "scale exponents go with (and only with) FP8");
  DeviceGuard g(ctx->device);
  HIP_TRY(ctx, launch_convert(prec, m, n, d_src, lds, d_dst, ldd, d_scale_exp, ctx->stream));
  return MPCR_OK;
}

int mpcr_gemm(mpcr_ctx* ctx, mpcr_prec_t prec, int transA, int transB, int64_t m, int64_t n, int64_t k, double alpha,
              const void* d_A, int64_t lda, const int8_t* d_scaleA_exp, const void* d_B, int64_t ldb,
              const int8_t* d_scaleB_exp, double beta, void* d_C, int64_t ldc, mpcr_prec_t c_prec) {
  TraceRange tr("mpcr_gemm");
  CHECK_ARG(ctx, ctx != nullptr, "NULL context");
  const int p = (int)prec, cp = (int)c_prec;
  CHECK_ARG(ctx, valid_prec(p) && (cp == F64 || cp == F32), "bad formats");
  CHECK_ARG(ctx, !(p == F64 && cp != F64), "FP64 products are written in FP64");
  CHECK_ARG(ctx, m >= 0 && n >= 0 && k >= 0, "negative size");
  const int64_t arows = transA ? k : m, brows = transB ? n : k;
  CHECK_ARG(ctx, lda >= std::max<int64_t>(arows, 1) && ldb >= std::max<int64_t>(brows, 1) &&
                     ldc >= std::max<int64_t>(m, 1),
            "leading dimension too small");
  if (m == 0 || n == 0) return MPCR_OK;
  CHECK_ARG(ctx, d_C && (k == 0 || (d_A && d_B)), "NULL pointer");
  CHECK_ARG(ctx, (p == F8) == (d_scaleA_exp != nullptr && d_scaleB_exp != nullptr) || k == 0,
            "FP8 operands need their scale exponents (and only FP8 takes them)");
  DeviceGuard g(ctx->device);
  hipStream_t s = ctx->stream;
  if (p == F64 || p == F32) {
    HIP_TRY(ctx, launch_gemm(p, transA, transB, m, n, k, alpha, d_A, lda, d_B, ldb, beta, d_C, ldc, cp, s));
    return MPCR_OK;
  }
  // 16/8-bit: the kernel reads op(A) as m x k and op(B) as n x k arrays with k
  // contiguous and 16-byte aligned rows; operands in another layout are packed
  // into a workspace first (one pass over each, small next to the product).
  const int es = (p == F8) ? 1 : 2;
  auto usable = [&](const void* ptr, int64_t ld, bool kcontig) {
    return kcontig && ((uintptr_t)ptr % 16 == 0) && ((ld * es) % 16 == 0);
  };
  const bool a_ok = usable(d_A, lda, transA != 0), b_ok = usable(d_B, ldb, transB == 0);
  const int64_t ldk = (k + 15) / 16 * 16;  // packed leading dimension (elements)
  const int64_t a_bytes = a_ok ? 0 : (m * ldk * es + 255) / 256 * 256, b_bytes = b_ok ? 0 : n * ldk * es;
  if (ctx->ws_gemm_bytes < a_bytes + b_bytes) {
    HIP_TRY(ctx, hipStreamSynchronize(s));
    dfree(ctx->arena, ctx->ws_gemm);
    ctx->ws_gemm = nullptr;
    ctx->ws_gemm_bytes = 0;
    HIP_TRY(ctx, dmalloc(ctx->arena, &ctx->ws_gemm, (size_t)(a_bytes + b_bytes)));
    ctx->ws_gemm_bytes = a_bytes + b_bytes;
  }
  const void* A = d_A;
  int64_t ldat = lda;
  if (!a_ok) {
    A = ctx->ws_gemm;
    ldat = ldk;
    HIP_TRY(ctx, launch_pack(es, transA == 0, m, k, d_A, lda, ctx->ws_gemm, ldk, s));
  }
  const void* B = d_B;
  int64_t ldbk = ldb;
  if (!b_ok) {
    B = ctx->ws_gemm + a_bytes;
    ldbk = ldk;
    HIP_TRY(ctx, launch_pack(es, transB != 0, n, k, d_B, ldb, ctx->ws_gemm + a_bytes, ldk, s));
  }
  // FP8 scale grids belong to the stored matrices (column-major over 128 x 128 blocks)
  const int64_t mbA = transA ? (k + 127) / 128 : (m + 127) / 128;
  const int64_t mbB = transB ? (n + 127) / 128 : (k + 127) / 128;
  HIP_TRY(ctx, launch_gemm_lowp(p, m, n, k, alpha, A, ldat, d_scaleA_exp, mbA, transA != 0, B, ldbk, d_scaleB_exp,
                                mbB, transB != 0, beta, d_C, ldc, cp, s));
  return MPCR_OK;
}

}  // extern "C"
