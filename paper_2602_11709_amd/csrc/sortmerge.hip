// Sort of each crystal's reflections by (2theta, h, k, l) and the merge into
// peaks (paper, Section 2: merging of reflections within specified angular
// tolerances; grouping of reflections into peaks).
//
// Sort: crystals of up to 4096 reflections are sorted by one block each in
// LDS; larger crystals use the same bucket sort through global memory.  The
// buckets are exactly monotone.  The bucket of a
// reflection is floor((2theta - tmin) * bins_per_degree), clamped; a
// subtraction, a product with a positive constant and floor are each monotone
// in IEEE arithmetic, so bucket order never contradicts key order and equal
// keys share a bucket.  Count (atomics), scan, scatter (atomics), then a
// per-bucket insertion sort on the full key (2theta, h, k, l), which removes
// the scatter's order dependence.  About 40 bytes of traffic per reflection
// instead of the ~170 of an 8-pass radix sort on 64-bit keys.
//
// Merge (anchor rule): walking the sorted order, a reflection joins the open
// peak while 2theta - 2theta(peak's first member) < tol.  A gap >= tol between
// neighbours always opens a peak, so the sorted list splits at such gaps into
// independent components; one thread walks each component with the anchor
// rule and flags peak starts.  A scan of the flags numbers the peaks; one
// thread per peak then sums its members' intensities in sorted order.
#include <math.h>

#include "xrd_internal.h"

namespace xrd {

namespace {

constexpr int kThreads = 256;
constexpr int kPer = kSortChunk / kThreads;  // 4
constexpr int kSmallSort = 4096;              // reflections sorted by one block in LDS
static_assert(kSortChunk / kBinDiv == kThreads, "one bucket per thread of a sort chunk");

__device__ __forceinline__ int bin_of(const CrystalPlan &P, double tt) {
#pragma clang fp contract(off)
  const double x = floor((tt - P.tmin) * P.bin_scale);
  int b = x < 0.0 ? 0 : (x >= (double)(P.n_bins - 1) ? P.n_bins - 1 : (int)x);
  return b;
}

__device__ __forceinline__ int64_t hkl_key(const int16_t *h, const int16_t *k, const int16_t *l, int32_t i) {
  return ((int64_t)(h[i] + 32768) << 32) | ((int64_t)(k[i] + 32768) << 16) | (int64_t)(l[i] + 32768);
}

// Reflection range of sort chunk ``blockIdx.x``: positions base + u * 256 + tid
// for u < kPer that are below r1 hold real reflections of crystal ``cry``.
struct ChunkRange {
  int32_t cry;
  int64_t r0, r1, base;
};

__device__ __forceinline__ ChunkRange chunk_range(const CrystalPlan *__restrict__ plan,
                                                  const int32_t *__restrict__ chunk_crystal,
                                                  const int64_t *__restrict__ refl_offset) {
  ChunkRange c;
  c.cry = chunk_crystal[blockIdx.x];
  c.r0 = refl_offset[c.cry];
  c.r1 = refl_offset[c.cry + 1];
  c.base = c.r0 + (int64_t)(blockIdx.x - plan[c.cry].sort_chunk_begin) * kSortChunk;
  return c;
}

// Crystals with at most kSmallSort reflections: one block sorts the whole
// crystal in LDS with the same monotone buckets as the large-crystal path
// (R/2 of them): count with LDS atomics, scan, scatter with LDS atomics, then
// an insertion sort of each bucket on (2theta bits, position).  The input is
// in lexicographic (h, k, l) order, so ordering ties by position orders them
// by (h, k, l); positive doubles order like their bit patterns.
__global__ __launch_bounds__(kThreads) void k_sort_small(const CrystalPlan *__restrict__ plan,
                                                         const int64_t *__restrict__ refl_offset,
                                                         const double *__restrict__ tt, double *__restrict__ skey,
                                                         int32_t *__restrict__ sidx) {
  __shared__ uint64_t key[kSmallSort];
  __shared__ uint32_t pos[kSmallSort];
  __shared__ int32_t cnt[kSmallSort / 2];
  __shared__ int32_t wsum[kThreads / 64];
  const CrystalPlan &P = plan[blockIdx.x];
  const int64_t r0 = refl_offset[blockIdx.x], r1 = refl_offset[blockIdx.x + 1];
  if (r1 - r0 > kSmallSort || r1 <= r0) return;
  const int R = (int)(r1 - r0);
  const int B = R / 2 > 1 ? R / 2 : 1;
  const double scale = (double)B / (P.tmax - P.tmin);
  for (int b = threadIdx.x; b < B; b += kThreads) cnt[b] = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < R; i += kThreads) {
#pragma clang fp contract(off)
    const double x = floor((tt[r0 + i] - P.tmin) * scale);
    const int b = x < 0.0 ? 0 : (x >= (double)(B - 1) ? B - 1 : (int)x);
    atomicAdd(&cnt[b], 1);
  }
  __syncthreads();
  // exclusive scan of the bucket counts: each thread owns a contiguous run
  {
    constexpr int per = (kSmallSort / 2 + kThreads - 1) / kThreads;
    const int b0 = threadIdx.x * per;
    int v[per], sum = 0;
#pragma unroll
    for (int u = 0; u < per; ++u) {
      v[u] = b0 + u < B ? cnt[b0 + u] : 0;
      sum += v[u];
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int inc = sum;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int o = __shfl_up(inc, d, 64);
      if (lane >= d) inc += o;
    }
    if (lane == 63) wsum[wid] = inc;
    __syncthreads();
    int ex = inc - sum;
    for (int w = 0; w < wid; ++w) ex += wsum[w];
#pragma unroll
    for (int u = 0; u < per; ++u) {
      if (b0 + u < B) cnt[b0 + u] = ex;
      ex += v[u];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < R; i += kThreads) {
#pragma clang fp contract(off)
    const double t = tt[r0 + i];
    const double x = floor((t - P.tmin) * scale);
    const int b = x < 0.0 ? 0 : (x >= (double)(B - 1) ? B - 1 : (int)x);
    const int slot = atomicAdd(&cnt[b], 1);
    key[slot] = (uint64_t)__double_as_longlong(t);
    pos[slot] = (uint32_t)i;
  }
  __syncthreads();
  // cnt[b] is now the end of bucket b, and its start is the end of bucket b - 1
  for (int b = threadIdx.x; b < B; b += kThreads) {
    const int s = b ? cnt[b - 1] : 0, e = cnt[b];
    for (int i = s + 1; i < e; ++i) {
      const uint64_t k = key[i];
      const uint32_t p = pos[i];
      int j = i - 1;
      while (j >= s && (key[j] > k || (key[j] == k && pos[j] > p))) {
        key[j + 1] = key[j];
        pos[j + 1] = pos[j];
        --j;
      }
      key[j + 1] = k;
      pos[j + 1] = p;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < R; i += kThreads) {
    skey[r0 + i] = __longlong_as_double((long long)key[i]);
    sidx[r0 + i] = (int32_t)(r0 + pos[i]);
  }
}

__global__ __launch_bounds__(kThreads) void k_bin_count(const CrystalPlan *__restrict__ plan,
                                                        const int32_t *__restrict__ chunk_crystal,
                                                        const int64_t *__restrict__ refl_offset,
                                                        const double *__restrict__ tt, int32_t *__restrict__ count) {
  const ChunkRange cr = chunk_range(plan, chunk_crystal, refl_offset);
  if (cr.r1 - cr.r0 <= kSmallSort) return;  // sorted in LDS by k_sort_small
  const CrystalPlan &P = plan[cr.cry];
  for (int u = 0; u < kPer; ++u) {
    const int64_t i = cr.base + u * kThreads + threadIdx.x;
    if (i >= cr.r1) break;
    atomicAdd(&count[P.bin_begin + bin_of(P, tt[i])], 1);
  }
}

__global__ __launch_bounds__(kThreads) void k_bin_scatter(const CrystalPlan *__restrict__ plan,
                                                          const int32_t *__restrict__ chunk_crystal,
                                                          const int64_t *__restrict__ refl_offset,
                                                          const double *__restrict__ tt,
                                                          const int64_t *__restrict__ start,
                                                          int32_t *__restrict__ count, double *__restrict__ skey,
                                                          int32_t *__restrict__ sidx) {
  const ChunkRange cr = chunk_range(plan, chunk_crystal, refl_offset);
  if (cr.r1 - cr.r0 <= kSmallSort) return;
  const CrystalPlan &P = plan[cr.cry];
  for (int u = 0; u < kPer; ++u) {
    const int64_t i = cr.base + u * kThreads + threadIdx.x;
    if (i >= cr.r1) break;
    const double t = tt[i];
    const int64_t gb = P.bin_begin + bin_of(P, t);
    // bucket ranges are relative to the crystal's first bucket: crystals
    // sorted in LDS leave their buckets empty, so the global prefix is not
    // the crystal's reflection offset
    const int64_t slot = cr.r0 + (start[gb] - start[P.bin_begin]) + atomicSub(&count[gb], 1) - 1;
    skey[slot] = t;
    sidx[slot] = (int32_t)i;
  }
}

// One thread per bucket of a large crystal (blocks follow the sort chunks:
// 256 buckets per chunk, and a crystal has at most 256 buckets per chunk):
// insertion sort on (2theta, h, k, l).  Buckets hold a few reflections on
// average (at most a few tens for high-symmetry cells).
__global__ __launch_bounds__(kThreads) void k_bin_sort(const CrystalPlan *__restrict__ plan,
                                                       const int32_t *__restrict__ chunk_crystal,
                                                       const int64_t *__restrict__ refl_offset,
                                                       const int64_t *__restrict__ start, double *__restrict__ skey,
                                                       int32_t *__restrict__ sidx, const int16_t *__restrict__ h,
                                                       const int16_t *__restrict__ k,
                                                       const int16_t *__restrict__ l) {
  const int32_t cry = chunk_crystal[blockIdx.x];
  const CrystalPlan &P = plan[cry];
  const int64_t r0 = refl_offset[cry], r1 = refl_offset[cry + 1];
  if (r1 - r0 <= kSmallSort) return;
  const int64_t bl = (int64_t)(blockIdx.x - P.sort_chunk_begin) * kThreads + threadIdx.x;
  if (bl >= P.n_bins) return;
  const int64_t b = P.bin_begin + bl;
  const int64_t s = r0 + (start[b] - start[P.bin_begin]), e = r0 + (start[b + 1] - start[P.bin_begin]);
  for (int64_t i = s + 1; i < e; ++i) {
    const double key = skey[i];
    const int32_t id = sidx[i];
    const int64_t hk = hkl_key(h, k, l, id);
    int64_t j = i - 1;
    while (j >= s) {
      const double kj = skey[j];
      const int32_t ij = sidx[j];
      const bool gt = kj > key || (kj == key && hkl_key(h, k, l, ij) > hk);
      if (!gt) break;
      skey[j + 1] = kj;
      sidx[j + 1] = ij;
      --j;
    }
    skey[j + 1] = key;
    sidx[j + 1] = id;
  }
}

// Component walk: a thread whose position starts a component (crystal start or
// a gap >= tol) applies the anchor rule up to the next such gap and writes the
// peak-start flag of every position in it.
__global__ __launch_bounds__(kThreads) void k_merge_flags(const CrystalPlan *__restrict__ plan,
                                                          const int32_t *__restrict__ chunk_crystal,
                                                          const int64_t *__restrict__ refl_offset,
                                                          const double *__restrict__ skey, double tol,
                                                          int32_t *__restrict__ flags) {
#pragma clang fp contract(off)
  const ChunkRange cr = chunk_range(plan, chunk_crystal, refl_offset);
  const int64_t r0 = cr.r0, r1 = cr.r1;
  for (int u = 0; u < kPer; ++u) {
    const int64_t i = cr.base + u * kThreads + threadIdx.x;
    if (i >= r1) break;
    const double ti = skey[i];
    const bool start = (i == r0) || (ti - skey[i - 1] >= tol);
    if (start) {
      flags[i] = 1;
      double anchor = ti, prev = ti;
      for (int64_t j = i + 1; j < r1; ++j) {
        const double tj = skey[j];
        if (tj - prev >= tol) break;
        const bool open = (tj - anchor) >= tol;
        flags[j] = open ? 1 : 0;
        if (open) anchor = tj;
        prev = tj;
      }
    }
  }
}

// Peak offsets per crystal from the flag scan; also the total peak count.
__global__ void k_peak_offsets(const int64_t *__restrict__ refl_offset, int64_t n_c,
                               const int64_t *__restrict__ pscan, int64_t *__restrict__ peak_offset,
                               int64_t *__restrict__ n_peaks) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c <= n_c) {
    const int64_t v = pscan[refl_offset[c]];
    peak_offset[c] = v;
    if (c == n_c) *n_peaks = v;
  }
}

// One thread per peak start: member count and intensity sum in sorted order.
__global__ __launch_bounds__(kThreads) void k_merge_reduce(
    const CrystalPlan *__restrict__ plan, const int32_t *__restrict__ chunk_crystal,
    const int64_t *__restrict__ refl_offset, const double *__restrict__ skey, const int32_t *__restrict__ sidx,
    const int32_t *__restrict__ flags, const int64_t *__restrict__ pscan, const double *__restrict__ inten,
    double *__restrict__ pk_tt, double *__restrict__ pk_i, int32_t *__restrict__ pk_mult,
    int64_t *__restrict__ pk_first, int64_t *__restrict__ perm, uint64_t *__restrict__ cmax) {
  const ChunkRange cr = chunk_range(plan, chunk_crystal, refl_offset);
  const int64_t r1 = cr.r1;
  for (int u = 0; u < kPer; ++u) {
    const int64_t i = cr.base + u * kThreads + threadIdx.x;
    if (i >= r1) break;
    perm[i] = sidx[i];
    if (flags[i]) {
      const int64_t p = pscan[i];
      double s = inten[sidx[i]];
      int m = 1;
      for (int64_t j = i + 1; j < r1 && !flags[j]; ++j) {
        s += inten[sidx[j]];
        ++m;
      }
      pk_tt[p] = skey[i];
      pk_i[p] = s;
      pk_mult[p] = m;
      pk_first[p] = i;
      atomicMax((unsigned long long *)&cmax[cr.cry], (unsigned long long)__double_as_longlong(s));
    }
  }
}

// Scaled intensity 100 I / max I of the crystal; with a threshold, also the
// keep flag of each peak.
__global__ __launch_bounds__(kThreads) void k_merge_scale(
    const CrystalPlan *__restrict__ plan, const int32_t *__restrict__ chunk_crystal,
    const int64_t *__restrict__ refl_offset, const int32_t *__restrict__ flags, const int64_t *__restrict__ pscan,
    const double *__restrict__ pk_i, double *__restrict__ pk_y, const uint64_t *__restrict__ cmax, double thr,
    int32_t *__restrict__ keep) {
  const ChunkRange cr = chunk_range(plan, chunk_crystal, refl_offset);
  for (int u = 0; u < kPer; ++u) {
    const int64_t i = cr.base + u * kThreads + threadIdx.x;
    if (i >= cr.r1) break;
    if (flags[i]) {
      const int64_t p = pscan[i];
      const double mx = __longlong_as_double((long long)cmax[cr.cry]);
      const double v = pk_i[p];
      pk_y[p] = mx > 0.0 ? 100.0 * v / mx : 0.0;
      if (keep) keep[p] = (v >= thr * mx) ? 1 : 0;
    }
  }
}

// Compaction of the kept peaks (threshold > 0).
__global__ void k_peak_compact(const int64_t *__restrict__ n_peaks, int64_t cap, const int32_t *__restrict__ keep,
                               const int64_t *__restrict__ kscan, const double *__restrict__ t_tt,
                               const double *__restrict__ t_i, const double *__restrict__ t_y,
                               const int32_t *__restrict__ t_m, const int64_t *__restrict__ t_f,
                               double *__restrict__ o_tt, double *__restrict__ o_i, double *__restrict__ o_y,
                               int32_t *__restrict__ o_m, int64_t *__restrict__ o_f) {
  const int64_t np = *n_peaks;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np && p < cap;
       p += (int64_t)gridDim.x * blockDim.x) {
    if (keep[p]) {
      const int64_t d = kscan[p];
      o_tt[d] = t_tt[p];
      o_i[d] = t_i[p];
      o_y[d] = t_y[p];
      o_m[d] = t_m[p];
      o_f[d] = t_f[p];
    }
  }
}

__global__ void k_peak_offsets_compact(int64_t n_c, const int64_t *__restrict__ raw, const int64_t *__restrict__ kscan,
                                       int64_t *__restrict__ peak_offset) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c <= n_c) peak_offset[c] = kscan[raw[c]];
}

}  // namespace

void launch_sort(const SortArgs &a, hipStream_t s) {
  if (a.n_c > 0)
    hipLaunchKernelGGL(k_sort_small, dim3((unsigned)a.n_c), dim3(kThreads), 0, s, a.plan, a.refl_offset, a.tt,
                       a.skey, a.sidx);
  launch_fill_i32(a.bin_count, a.n_bins, 0, s);
  if (a.n_chunks > 0)
    hipLaunchKernelGGL(k_bin_count, dim3((unsigned)a.n_chunks), dim3(kThreads), 0, s, a.plan, a.chunk_crystal,
                       a.refl_offset, a.tt, a.bin_count);
  launch_scan_i32(a.bin_count, a.n_bins, nullptr, a.bin_start, a.scan_part, s);
  if (a.n_chunks > 0)
    hipLaunchKernelGGL(k_bin_scatter, dim3((unsigned)a.n_chunks), dim3(kThreads), 0, s, a.plan, a.chunk_crystal,
                       a.refl_offset, a.tt, a.bin_start, a.bin_count, a.skey, a.sidx);
  if (a.n_chunks > 0)
    hipLaunchKernelGGL(k_bin_sort, dim3((unsigned)a.n_chunks), dim3(kThreads), 0, s, a.plan, a.chunk_crystal,
                       a.refl_offset, a.bin_start, a.skey, a.sidx, a.h, a.k, a.l);
}

void launch_merge(const MergeArgs &a, hipStream_t s) {
  const SortArgs &o = a.sort;  // sorted by the caller
  launch_fill_u64(a.cmax, a.n_c, 0, s);
  const dim3 cg((unsigned)(o.n_chunks > 0 ? o.n_chunks : 1)), cb(kThreads);
  if (o.n_chunks > 0)
    hipLaunchKernelGGL(k_merge_flags, cg, cb, 0, s, o.plan, o.chunk_crystal, o.refl_offset, o.skey, a.tol, a.flags);
  launch_scan_i32(a.flags, a.refl_cap, o.refl_offset + a.n_c, a.pscan, o.scan_part, s);
  const bool thr = a.thr > 0.0;
  int64_t *poff = thr ? a.raw_peak_offset : a.peak_offset;
  hipLaunchKernelGGL(k_peak_offsets, dim3((unsigned)((a.n_c + 1 + 255) / 256)), dim3(256), 0, s, o.refl_offset, a.n_c,
                     a.pscan, poff, a.n_peaks);
  double *d_tt = thr ? a.tmp_tt : a.pk_tt;
  double *d_i = thr ? a.tmp_i : a.pk_i;
  int32_t *d_m = thr ? a.tmp_mult : a.pk_mult;
  int64_t *d_f = thr ? a.tmp_first : a.pk_first;
  if (o.n_chunks > 0) {
    hipLaunchKernelGGL(k_merge_reduce, cg, cb, 0, s, o.plan, o.chunk_crystal, o.refl_offset, o.skey, o.sidx, a.flags,
                       a.pscan, a.inten, d_tt, d_i, d_m, d_f, a.perm, a.cmax);
    hipLaunchKernelGGL(k_merge_scale, cg, cb, 0, s, o.plan, o.chunk_crystal, o.refl_offset, a.flags, a.pscan, d_i,
                       thr ? a.tmp_y : a.pk_y, a.cmax, a.thr, thr ? a.keep : nullptr);
  }
  if (thr) {
    launch_scan_i32(a.keep, a.refl_cap, a.n_peaks, a.kscan, o.scan_part, s);
    hipLaunchKernelGGL(k_peak_compact, dim3(1024), dim3(256), 0, s, a.n_peaks, a.refl_cap, a.keep, a.kscan, a.tmp_tt,
                       a.tmp_i, a.tmp_y, a.tmp_mult, a.tmp_first, a.pk_tt, a.pk_i, a.pk_y, a.pk_mult,
                       a.pk_first);
    hipLaunchKernelGGL(k_peak_offsets_compact, dim3((unsigned)((a.n_c + 1 + 255) / 256)), dim3(256), 0, s, a.n_c,
                       a.raw_peak_offset, a.kscan, a.peak_offset);
  }
}

}  // namespace xrd
