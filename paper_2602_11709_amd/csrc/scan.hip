// Device-wide exclusive scan (int32 -> int64) and fill kernels.
//
// Reduce-then-scan in three launches: per-block sums, a single-block scan of
// those sums, then a per-block scan seeded with its prefix.  Integer sums are
// exact, so the result does not depend on scheduling.  The element count may
// live on the device (``n_dev``) so that a captured graph can scan a
// data-dependent prefix of a capacity-sized array.
#include "xrd_internal.h"

namespace xrd {

namespace {

constexpr int kThreads = 256;
constexpr int kPer = kScanBlock / kThreads;  // 8

__device__ __forceinline__ int64_t wave_incl_scan(int64_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int64_t o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

// Exclusive block scan of one value per thread; returns the block total in *total.
__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t *total) {
  __shared__ int64_t wsum[kThreads / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int64_t inc = wave_incl_scan(v);
  if (lane == 63) wsum[wid] = inc;
  __syncthreads();
  int64_t base = 0, tot = 0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) {
    if (w < wid) base += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  *total = tot;
  return base + inc - v;
}

__global__ __launch_bounds__(kThreads) void k_scan_reduce(const int32_t *__restrict__ in, int64_t n,
                                                          const int64_t *__restrict__ n_dev,
                                                          int64_t *__restrict__ part) {
  const int64_t lim = n_dev ? min(n, *n_dev) : n;
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  int64_t s = 0;
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    int64_t i = base + (int64_t)u * kThreads + threadIdx.x;
    if (i < lim) s += in[i];
  }
  int64_t tot;
  block_excl_scan(s, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Single block: exclusive scan of nb partial sums, in place; part[nb] = total.
__global__ __launch_bounds__(kThreads) void k_scan_partials(int64_t *__restrict__ part, int64_t nb) {
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += kThreads) {
    int64_t i = b0 + threadIdx.x;
    int64_t v = i < nb ? part[i] : 0;
    int64_t tot;
    int64_t ex = block_excl_scan(v, &tot);
    if (i < nb) part[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) part[nb] = carry;
}

__global__ __launch_bounds__(kThreads) void k_scan_apply(const int32_t *__restrict__ in, int64_t n,
                                                         const int64_t *__restrict__ n_dev,
                                                         const int64_t *__restrict__ part,
                                                         int64_t *__restrict__ out, int64_t nb) {
  const int64_t lim = n_dev ? min(n, *n_dev) : n;
  const int64_t base = (int64_t)blockIdx.x * kScanBlock;
  // each thread owns kPer consecutive elements: coalescing is traded for a
  // sequential in-thread scan; the array is read once more here.
  const int64_t t0 = base + (int64_t)threadIdx.x * kPer;
  int32_t v[kPer];
  int64_t s = 0;
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    int64_t i = t0 + u;
    v[u] = i < lim ? in[i] : 0;
    s += v[u];
  }
  int64_t tot;
  int64_t ex = block_excl_scan(s, &tot) + part[blockIdx.x];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    int64_t i = t0 + u;
    if (i <= lim && i < n) out[i] = ex;
    ex += v[u];
  }
  if (blockIdx.x == nb - 1 && threadIdx.x == 0) out[n] = part[nb];
}

__global__ void k_fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += st) p[i] = v;
}

__global__ void k_fill_u64(uint64_t *__restrict__ p, int64_t n, uint64_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += st) p[i] = v;
}

int fill_grid(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  return (int)(g < 1 ? 1 : g);
}

}  // namespace

void launch_scan_i32(const int32_t *in, int64_t n, const int64_t *n_dev, int64_t *out, int64_t *part,
                     hipStream_t s) {
  int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb == 0) nb = 1;  // n == 0: one block writes out[0] = 0
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kThreads), 0, s, in, n, n_dev, part);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kThreads), 0, s, part, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)nb), dim3(kThreads), 0, s, in, n, n_dev, part, out, nb);
}

void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_i32, dim3(fill_grid(n)), dim3(256), 0, s, p, n, v);
}

void launch_fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_u64, dim3(fill_grid(n)), dim3(256), 0, s, p, n, v);
}

}  // namespace xrd
