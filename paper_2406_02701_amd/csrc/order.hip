// Morton (Z-order) ordering of the sites on the device.
//
// A band map of the tile factor only makes sense when sites that are close in
// space get close indices.  Each coordinate in [0,1) is quantised to 16 bits,
// q = min(floor(65536 x), 65535), and the bits are interleaved (x in the even
// positions, y in the odd ones).  Keys (code << 32 | index) are unique, so a
// bitonic sort of the keys gives the stable order by code.
#include <mutex>

#include "mpcr_internal.h"

namespace mpcr {

// Sort keys of the allocation-free ordering entry point: a library-owned
// device array (one copy per GPU, alive until the process ends) holding up
// to MORTON_NOALLOC_MAX_KEYS keys, i.e. orders of up to that many sites.
static __device__ __align__(256) uint64_t scratch[MORTON_NOALLOC_MAX_KEYS];

// Device address of `scratch` on `device`, looked up once per device with that
// device current (the host-side name of the array is not a device address).
hipError_t morton_noalloc_keys(int device, uint64_t** out) {
  static std::mutex mu;
  static uint64_t* addr[MAX_DEVICES] = {};
  if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(mu);
  if (!addr[device]) {
    int prev = -1;
    hipError_t e = hipGetDevice(&prev);
    if (e != hipSuccess) return e;
    if (prev != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (prev != device) (void)hipSetDevice(prev);
    if (e != hipSuccess) return e;
    addr[device] = (uint64_t*)p;
  }
  *out = addr[device];
  return hipSuccess;
}

__device__ __forceinline__ uint32_t spread_bits16(uint32_t v) {
  v &= 0xffffu;
  v = (v | (v << 8)) & 0x00ff00ffu;
  v = (v | (v << 4)) & 0x0f0f0f0fu;
  v = (v | (v << 2)) & 0x33333333u;
  v = (v | (v << 1)) & 0x55555555u;
  return v;
}

__device__ __forceinline__ uint32_t quant16(double x) {
  double q = floor((x > 0.0 ? x : 0.0) * 65536.0);
  return q > 65535.0 ? 65535u : (uint32_t)q;
}

__global__ void k_morton_keys(int n, const double* locs, uint64_t* keys, int npow2) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < npow2; i += gridDim.x * blockDim.x) {
    if (i < n) {
      uint32_t code = spread_bits16(quant16(locs[i])) | (spread_bits16(quant16(locs[n + i])) << 1);
      keys[i] = ((uint64_t)code << 32) | (uint32_t)i;
    } else {
      keys[i] = ~0ull;
    }
  }
}

hipError_t launch_morton_codes(int n, const double* locs, uint64_t* keys, int npow2, hipStream_t s) {
  int g = (npow2 + 255) / 256;
  k_morton_keys<<<g < 1024 ? g : 1024, 256, 0, s>>>(n, locs, keys, npow2);
  return hipGetLastError();
}

constexpr int LBLK = 2048;  // elements sorted in LDS per workgroup

__device__ __forceinline__ void cmp_swap(uint64_t& a, uint64_t& b, bool up) {
  if ((a > b) == up) {
    uint64_t t = a;
    a = b;
    b = t;
  }
}

// All stages with k <= kmax_local inside blocks of `blk` elements (blk = min(N, 2048)),
// or (merge_k > 0) the tail j < blk of stage merge_k.
__global__ __launch_bounds__(1024) void k_bitonic_local(uint64_t* keys, int N, int blk, int merge_k) {
  __shared__ uint64_t s[LBLK];
  const int base = blockIdx.x * blk;
  for (int e = threadIdx.x; e < blk; e += blockDim.x) s[e] = keys[base + e];
  __syncthreads();
  const int kfirst = merge_k > 0 ? merge_k : 2;
  const int klast = merge_k > 0 ? merge_k : blk;
  for (int k = kfirst; k <= klast; k <<= 1) {
    for (int j = (merge_k > 0 ? blk / 2 : k / 2); j > 0; j >>= 1) {
      for (int e = threadIdx.x; e < blk; e += blockDim.x) {
        int l = e ^ j;
        if (l > e) {
          bool up = (((base + e) & k) == 0);
          uint64_t a = s[e], b = s[l];
          cmp_swap(a, b, up);
          s[e] = a;
          s[l] = b;
        }
      }
      __syncthreads();
    }
  }
  for (int e = threadIdx.x; e < blk; e += blockDim.x) keys[base + e] = s[e];
}

__global__ void k_bitonic_global(uint64_t* keys, int N, int k, int j) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < N; e += gridDim.x * blockDim.x) {
    int l = e ^ j;
    if (l > e) {
      bool up = ((e & k) == 0);
      uint64_t a = keys[e], b = keys[l];
      if ((a > b) == up) {
        keys[e] = b;
        keys[l] = a;
      }
    }
  }
}

hipError_t launch_bitonic_sort(uint64_t* keys, int N, hipStream_t s) {
  if (N <= 1) return hipSuccess;
  const int blk = N < LBLK ? N : LBLK;
  const int nblk = N / blk;
  const int thr = blk / 2 < 1024 ? (blk / 2 < 64 ? 64 : blk / 2) : 1024;
  k_bitonic_local<<<nblk, thr, 0, s>>>(keys, N, blk, 0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  for (int k = 2 * blk; k <= N; k <<= 1) {
    for (int j = k / 2; j >= blk; j >>= 1) {
      int g = (N + 255) / 256;
      k_bitonic_global<<<g < 2048 ? g : 2048, 256, 0, s>>>(keys, N, k, j);
    }
    k_bitonic_local<<<nblk, thr, 0, s>>>(keys, N, blk, k);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

__global__ void k_keys_to_perm(int n, const uint64_t* keys, int64_t* perm) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    perm[i] = (int64_t)(keys[i] & 0xffffffffull);
}
hipError_t launch_keys_to_perm(int n, const uint64_t* keys, int64_t* perm, hipStream_t s) {
  if (n == 0) return hipSuccess;
  int g = (n + 255) / 256;
  k_keys_to_perm<<<g < 1024 ? g : 1024, 256, 0, s>>>(n, keys, perm);
  return hipGetLastError();
}

// dst[r][c] = src[perm[r]][c] for r < n, c < ncols (column-major blocks)
__global__ void k_gather_rows(int n, const double* src, int64_t lds, const int64_t* perm, double* dst, int64_t ldd) {
  const int c = blockIdx.y;
  for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < n; r += gridDim.x * blockDim.x)
    dst[(int64_t)c * ldd + r] = src[(int64_t)c * lds + perm[r]];
}
hipError_t launch_gather_rows(int n, int ncols, const double* src, int64_t lds, const int64_t* perm, double* dst,
                              int64_t ldd, hipStream_t s) {
  if (n == 0 || ncols == 0) return hipSuccess;
  int g = (n + 255) / 256;
  k_gather_rows<<<dim3(g < 256 ? g : 256, ncols), 256, 0, s>>>(n, src, lds, perm, dst, ldd);
  return hipGetLastError();
}

}  // namespace mpcr
