// Sort of each crystal's reflections by (2theta, h, k, l) and the merge into
// peaks (paper, Section 2: merging of reflections within specified angular
// tolerances; grouping of reflections into peaks).
//
// Sort: crystals of up to 4096 reflections are sorted by one block each in
// LDS; larger crystals use the same bucket sort through global memory, by
// kernels that walk a device-built list of those crystals.  The buckets are
// exactly monotone.  The bucket of a
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
constexpr int kSmallSort = 4096;              // reflections sorted by one 256-thread block in LDS
constexpr int kMidSort = 12288;               // reflections sorted by one 1024-thread block in LDS
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

// Crystals of at most CAP reflections: one block of T threads sorts the
// whole crystal in LDS with the same kind of monotone buckets as the global
// path (R/2 of them): count with LDS atomics, scan, scatter with LDS atomics,
// then an insertion sort of each bucket on (2theta bits, position).  The input
// is in lexicographic (h, k, l) order, so ordering ties by position orders them
// by (h, k, l); positive doubles order like their bit patterns.  Two sizes
// are launched: CAP 4096 (256 threads, ~48 KB of LDS) takes the crystals up to
// 4096 reflections, CAP 12288 (1024 threads, 144 KB of LDS, which gfx950
// provides per workgroup) the ones up to 12288.  The larger one zeroes the
// buckets of still larger crystals and registers their chunks for the
// bucket kernels.
template <int CAP, int T, bool LARGE>
__global__ __launch_bounds__(T) void k_sort_lds(const CrystalPlan *__restrict__ plan,
                                                const int64_t *__restrict__ refl_offset,
                                                const double *__restrict__ tt, double *__restrict__ skey,
                                                int32_t *__restrict__ sidx, int32_t *__restrict__ bin_count,
                                                int32_t *__restrict__ big_list, int2 *__restrict__ big_chunks,
                                                int32_t *__restrict__ counters) {
  __shared__ uint64_t key[CAP];
  __shared__ uint16_t pos[CAP];
  __shared__ int32_t cnt[CAP / 2];
  __shared__ int32_t wsum[T / 64];
  const CrystalPlan &P = plan[blockIdx.x];
  const int64_t r0 = refl_offset[blockIdx.x], r1 = refl_offset[blockIdx.x + 1];
  if (LARGE && r1 - r0 > CAP) {
    // too large for LDS: zero the crystal's buckets and register its chunks
    // for the bucket kernels (their order in the list does not matter)
    for (int64_t b = threadIdx.x; b < P.n_bins; b += T) bin_count[P.bin_begin + b] = 0;
    const int nch = (int)((r1 - r0 + kSortChunk - 1) / kSortChunk);
    if (threadIdx.x == 0) {
      big_list[atomicAdd(&counters[0], 1)] = blockIdx.x;
      wsum[0] = atomicAdd(&counters[1], nch);
    }
    __syncthreads();
    const int base = wsum[0];
    for (int k = threadIdx.x; k < nch; k += T) big_chunks[base + k] = make_int2((int)blockIdx.x, k);
    return;
  }
  if (r1 - r0 > CAP || r1 - r0 <= (LARGE ? kSmallSort : 0)) return;
  const int R = (int)(r1 - r0);
  const int B = R / 2 > 1 ? R / 2 : 1;
  const double scale = (double)B / (P.tmax - P.tmin);
  for (int b = threadIdx.x; b < B; b += T) cnt[b] = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < R; i += T) {
#pragma clang fp contract(off)
    const double x = floor((tt[r0 + i] - P.tmin) * scale);
    const int b = x < 0.0 ? 0 : (x >= (double)(B - 1) ? B - 1 : (int)x);
    atomicAdd(&cnt[b], 1);
  }
  __syncthreads();
  // exclusive scan of the bucket counts: each thread owns a contiguous run
  {
    constexpr int per = (CAP / 2 + T - 1) / T;
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
  for (int i = threadIdx.x; i < R; i += T) {
#pragma clang fp contract(off)
    const double t = tt[r0 + i];
    const double x = floor((t - P.tmin) * scale);
    const int b = x < 0.0 ? 0 : (x >= (double)(B - 1) ? B - 1 : (int)x);
    const int slot = atomicAdd(&cnt[b], 1);
    key[slot] = (uint64_t)__double_as_longlong(t);
    pos[slot] = (uint16_t)i;
  }
  __syncthreads();
  // cnt[b] is now the end of bucket b, and its start is the end of bucket b - 1
  for (int b = threadIdx.x; b < B; b += T) {
    const int s = b ? cnt[b - 1] : 0, e = cnt[b];
    for (int i = s + 1; i < e; ++i) {
      const uint64_t k = key[i];
      const uint16_t p = pos[i];
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
  for (int i = threadIdx.x; i < R; i += T) {
    skey[r0 + i] = __longlong_as_double((long long)key[i]);
    sidx[r0 + i] = (int32_t)(r0 + pos[i]);
  }
}

// Bucket path for the crystals registered by k_sort_lds: each kernel walks
// the device-built list of their sort chunks with a grid-stride loop, so the
// launch size does not depend on how many crystals are small.
__global__ __launch_bounds__(kThreads) void k_bin_count(const CrystalPlan *__restrict__ plan,
                                                        const int2 *__restrict__ big_chunks,
                                                        const int32_t *__restrict__ counters,
                                                        const int64_t *__restrict__ refl_offset,
                                                        const double *__restrict__ tt, int32_t *__restrict__ count) {
  const int n = counters[1];
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const int2 ck = big_chunks[i];
    const CrystalPlan &P = plan[ck.x];
    const int64_t r1 = refl_offset[ck.x + 1];
    const int64_t base = refl_offset[ck.x] + (int64_t)ck.y * kSortChunk;
    for (int u = 0; u < kPer; ++u) {
      const int64_t j = base + u * kThreads + threadIdx.x;
      if (j >= r1) break;
      atomicAdd(&count[P.bin_begin + bin_of(P, tt[j])], 1);
    }
  }
}

// Exclusive scan of one registered crystal's bucket counts per block
// (crystal-relative starts).
__global__ __launch_bounds__(kThreads) void k_bin_scan(const CrystalPlan *__restrict__ plan,
                                                       const int32_t *__restrict__ big_list,
                                                       const int32_t *__restrict__ counters,
                                                       const int32_t *__restrict__ count,
                                                       int64_t *__restrict__ start) {
  __shared__ int64_t wsum[kThreads / 64];
  const int n = counters[0];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const CrystalPlan &P = plan[big_list[i]];
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < P.n_bins; b0 += kThreads) {
      const int64_t b = b0 + threadIdx.x;
      const int64_t v = b < P.n_bins ? count[P.bin_begin + b] : 0;
      int64_t inc = v;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int64_t o = __shfl_up(inc, d, 64);
        if (lane >= d) inc += o;
      }
      if (lane == 63) wsum[wid] = inc;
      __syncthreads();
      int64_t before = 0, total = 0;
      for (int w = 0; w < kThreads / 64; ++w) {
        before += w < wid ? wsum[w] : 0;
        total += wsum[w];
      }
      if (b < P.n_bins) start[P.bin_begin + b] = carry + before + inc - v;
      carry += total;
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(kThreads) void k_bin_scatter(const CrystalPlan *__restrict__ plan,
                                                          const int2 *__restrict__ big_chunks,
                                                          const int32_t *__restrict__ counters,
                                                          const int64_t *__restrict__ refl_offset,
                                                          const double *__restrict__ tt,
                                                          const int64_t *__restrict__ start,
                                                          int32_t *__restrict__ count, double *__restrict__ skey,
                                                          int32_t *__restrict__ sidx) {
  const int n = counters[1];
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const int2 ck = big_chunks[i];
    const CrystalPlan &P = plan[ck.x];
    const int64_t r0 = refl_offset[ck.x], r1 = refl_offset[ck.x + 1];
    const int64_t base = r0 + (int64_t)ck.y * kSortChunk;
    for (int u = 0; u < kPer; ++u) {
      const int64_t j = base + u * kThreads + threadIdx.x;
      if (j >= r1) break;
      const double t = tt[j];
      const int64_t gb = P.bin_begin + bin_of(P, t);
      const int64_t slot = r0 + start[gb] + atomicSub(&count[gb], 1) - 1;
      skey[slot] = t;
      sidx[slot] = (int32_t)j;
    }
  }
}

// One thread per bucket: insertion sort on (2theta, h, k, l).  Buckets hold a
// few reflections on average (a few tens at most for high-symmetry cells).
__global__ __launch_bounds__(kThreads) void k_bin_sort(const CrystalPlan *__restrict__ plan,
                                                       const int2 *__restrict__ big_chunks,
                                                       const int32_t *__restrict__ counters,
                                                       const int64_t *__restrict__ refl_offset,
                                                       const int64_t *__restrict__ start, double *__restrict__ skey,
                                                       int32_t *__restrict__ sidx, const int16_t *__restrict__ h,
                                                       const int16_t *__restrict__ k,
                                                       const int16_t *__restrict__ l) {
  const int n = counters[1];
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const int2 ck = big_chunks[i];
    const CrystalPlan &P = plan[ck.x];
    const int64_t r0 = refl_offset[ck.x], r1 = refl_offset[ck.x + 1];
    // the crystal's chunks follow its reflection count and its buckets its
    // capacity (more of them): chunk ck.y takes every nch-th group of 256
    const int64_t nch = (r1 - r0 + kSortChunk - 1) / kSortChunk;
    for (int64_t bl = (int64_t)ck.y * kThreads + threadIdx.x; bl < P.n_bins; bl += nch * kThreads) {
      const int64_t b = P.bin_begin + bl;
      const int64_t s = r0 + start[b], e = bl + 1 < P.n_bins ? r0 + start[b + 1] : r1;
      for (int64_t x = s + 1; x < e; ++x) {
        const double key = skey[x];
        const int32_t id = sidx[x];
        const int64_t hk = hkl_key(h, k, l, id);
        int64_t j = x - 1;
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
  if (a.n_c <= 0) return;
  launch_fill_i32(a.counters, 2, 0, s);
  hipLaunchKernelGGL((k_sort_lds<kSmallSort, 256, false>), dim3((unsigned)a.n_c), dim3(256), 0, s, a.plan,
                     a.refl_offset, a.tt, a.skey, a.sidx, a.bin_count, a.big_list, a.big_chunks, a.counters);
  hipLaunchKernelGGL((k_sort_lds<kMidSort, 1024, true>), dim3((unsigned)a.n_c), dim3(1024), 0, s, a.plan,
                     a.refl_offset, a.tt, a.skey, a.sidx, a.bin_count, a.big_list, a.big_chunks, a.counters);
  if (a.n_chunks <= 0) return;
  const unsigned g = (unsigned)(a.n_chunks < 2048 ? a.n_chunks : 2048);
  const unsigned gc = (unsigned)(a.n_c < 1024 ? a.n_c : 1024);
  hipLaunchKernelGGL(k_bin_count, dim3(g), dim3(kThreads), 0, s, a.plan, a.big_chunks, a.counters, a.refl_offset, a.tt,
                     a.bin_count);
  hipLaunchKernelGGL(k_bin_scan, dim3(gc), dim3(kThreads), 0, s, a.plan, a.big_list, a.counters, a.bin_count,
                     a.bin_start);
  hipLaunchKernelGGL(k_bin_scatter, dim3(g), dim3(kThreads), 0, s, a.plan, a.big_chunks, a.counters, a.refl_offset,
                     a.tt, a.bin_start, a.bin_count, a.skey, a.sidx);
  hipLaunchKernelGGL(k_bin_sort, dim3(g), dim3(kThreads), 0, s, a.plan, a.big_chunks, a.counters, a.refl_offset,
                     a.bin_start, a.skey, a.sidx, a.h, a.k, a.l);
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
